"""Pins of the oracle's lab-frame output (section 2: each boosted-frame
particle mapped back to the lab by the inverse of Eq. Lor1, Lor2) and of its
grouping by boosted slices (Eq. DT).

The beam is defined in the lab at lab time 0 (seeded normals) and then
transformed; with no plasma, no undulator and negligible charge it moves
ballistically in the lab.  So every particle's lab output, at any boosted
step, must give back the lab momentum it was defined with and lie on its
lab straight line through its initial lab position: a wrong sign or a
dropped term in the inverse transform, or a wrong offset, fails these."""
import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po
from test_oracle_labprobe import _ballistic_case

pytestmark = pytest.mark.usefixtures("oracle_built")


def _lab_defined(w, nrm, sim):
    b, g, dx = w["beam"], w["grid"], w["grid"]["dx_m"]
    sx, sy = b["sigma_cells"][0], b["sigma_cells"][1]
    ux = b["emit_n_m"][0] / (sx * dx) * nrm[3]
    uy = b["emit_n_m"][1] / (sy * dx) * nrm[4]
    gam = b["gamma_lab"] * (1.0 + b["rel_energy_spread_rms"] * nrm[5])
    uz = np.sqrt(gam * gam - 1.0 - ux * ux - uy * uy)
    return {"x": 0.5 * g["nx"] + sx * nrm[0], "y": 0.5 * g["ny"] + sy * nrm[1], "z": sim.info().sig_zlab * nrm[2],
            "ux": ux, "uy": uy, "uz": uz, "gamma": gam}


@pytest.mark.parametrize("nsteps", [0, 40])
def test_lab_output_is_the_ballistic_lab_beam(nsteps):
    w = _ballistic_case(2048)
    nrm = pin.beam_normals(w["beam"]["n_macro"], 6)
    s = po.Sim(w, nrm)
    s.step(nsteps)
    L = po.lab_beam(s)
    d = _lab_defined(w, nrm, s)
    assert (L["alive"] == 1).all()
    # the 1e-18 C beam's own fields change momenta by ~1e-10 over the steps; a transform error is O(gamma_R)
    for k in ("ux", "uy", "uz", "gamma"):
        np.testing.assert_allclose(L[k], d[k], rtol=1e-12, atol=1e-8, err_msg=k)
    # the mass shell in the lab
    np.testing.assert_allclose(L["gamma"] ** 2 - L["ux"] ** 2 - L["uy"] ** 2 - L["uz"] ** 2, 1.0, rtol=0, atol=1e-8)
    # on the lab straight line: z_lab - v_z t_lab = z_lab(0), x - v_x t_lab = x(0) (mod nx)
    t = L["t"]
    np.testing.assert_allclose(L["z"] - d["uz"] / d["gamma"] * t, d["z"], rtol=0, atol=1e-9 * np.abs(t).max())
    nx = w["grid"]["nx"]
    dxp = (L["x"] - d["ux"] / d["gamma"] * t - d["x"] + nx / 2) % nx - nx / 2
    np.testing.assert_allclose(dxp, 0.0, rtol=0, atol=1e-9 * np.abs(t).max())
    # lab times at one boosted instant differ by gR bR (z'_1 - z'_2) (Eq. DT)
    i = s.info()
    zb = L["z_boost"]
    np.testing.assert_allclose(t - t[0], i.gR * i.bR * (zb - zb[0]), rtol=0, atol=1e-9 * np.abs(t).max())


def test_lab_groups_span_partition_and_sums():
    w = _ballistic_case(4096)
    nrm = pin.beam_normals(w["beam"]["n_macro"], 7)
    s = po.Sim(w, nrm)
    s.step(10)
    i = s.info()
    L = po.lab_beam(s)
    zb, ub = L["z_boost"], L["uz_boost"]
    dz, nzg = 1.7, 24
    z_lo = zb.mean() - 0.5 * dz * nzg
    u_lo, du, nug = ub.min() - 1e-9, (ub.max() - ub.min()) / 3.0 + 1e-9, 3  # u slices cover every particle
    T = po.lab_groups(s, z_lo, dz, nzg, u_lo, du, nug)
    inside = (zb >= z_lo) & (zb < z_lo + dz * nzg)
    # partition: counts add up to the particles in the covered z range; each particle counted once
    assert T[:, 0].sum() == inside.sum()
    assert T[:, 1].sum() == pytest.approx(L["w"][inside].sum(), rel=1e-14)
    # brute force on one group: the particles in slice 7, u slice 1
    m = inside & (np.floor((zb - z_lo) / dz) == 7) & (np.floor((ub - u_lo) / du) == 1)
    row = T[7 * nug + 1]
    assert row[0] == m.sum() > 0
    assert row[3] == L["t"][m].min() and row[4] == L["t"][m].max()
    assert row[5] == pytest.approx((L["w"] * L["z"])[m].sum(), rel=1e-13)
    # a group spans at most gR bR dz of lab time (Eq. DT), the whole beam much more
    nonempty = T[:, 0] > 0
    span = T[nonempty, 4] - T[nonempty, 3]
    assert (span <= i.gR * i.bR * dz * (1 + 1e-12)).all()
    assert L["t"].max() - L["t"].min() > 5 * i.gR * i.bR * dz
    # the summed lab gamma of all groups equals the total lab energy of the covered particles
    assert T[:, 15].sum() == pytest.approx((L["w"] * L["gamma"])[inside].sum(), rel=1e-13)
    # empty groups keep their +inf / -inf extrema
    assert (T[~nonempty, 3] == np.inf).all() and (T[~nonempty, 4] == -np.inf).all()
