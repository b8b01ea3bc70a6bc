"""Pins of the oracle's lab-frame probe (section 2 frame relations between the
boosted run and the lab).

A low-charge beam with no plasma or undulator moves ballistically in the lab:
x(T) = x(0) + v_x T, z(T) = z(0) + v_z T, with the lab positions and
velocities the beam was defined by (the seeded normals).  The probe, which
only sees the boosted-frame run, must return exactly these, every particle
sampled once."""
import math

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po

pytestmark = pytest.mark.usefixtures("oracle_built")


def _ballistic_case(n=2048):
    w = pin.scaled(pin.workload(0), n_beam=n, nz=192)  # long enough that no particle leaves the band
    w["undulator"]["kind"] = 0
    w["beam"]["charge_C"] = 1e-18  # self-fields far below the probe's round-off
    w["beam"]["rel_energy_spread_rms"] = 0.02
    w["beam"]["gamma_lab"] = 30.0
    return w


def _lab_initial(w, nrm, sim):
    """Lab positions at lab time 0 and lab velocities, as the beam is defined (pic.h / oracle init)."""
    b = w["beam"]
    g = w["grid"]
    dx = g["dx_m"]
    sx, sy = b["sigma_cells"][0], b["sigma_cells"][1]
    szl = sim.info().sig_zlab
    ux = b["emit_n_m"][0] / (sx * dx) * nrm[3]
    uy = b["emit_n_m"][1] / (sy * dx) * nrm[4]
    gam = b["gamma_lab"] * (1.0 + b["rel_energy_spread_rms"] * nrm[5])
    uz = np.sqrt(gam * gam - 1.0 - ux * ux - uy * uy)
    x = 0.5 * g["nx"] + sx * nrm[0]
    z = szl * nrm[2]
    return x, z, ux / gam, uz / gam


def _steps_to(i, zp, T):
    """Steps after which every particle's lab time has passed T: a step advances a
    particle's lab time by gR dt (1 + bR v'_z) >= gR dt / 2 here (v'_z > -1/2)."""
    return int(math.ceil((T - i.gR * i.bR * (zp.min() - i.zoff)) / (0.5 * i.gR * i.dt))) + 2


def test_probe_returns_ballistic_lab_positions():
    w = _ballistic_case()
    nrm = pin.beam_normals(w["beam"]["n_macro"], 4)
    s = po.Sim(w, nrm)
    x0, z0, vx, vz = _lab_initial(w, nrm, s)
    i = s.info()
    # lab time of the beam at t' = 0 spans gR bR (z' - z0); probe beyond its latest particle
    zp = np.real(s.particles(0)["z"])
    T = i.gR * i.bR * (zp.max() - i.zoff) + 5.0
    r = po.lab_probe(s, _steps_to(i, zp, T), T, 2 * math.pi / 20.0)
    assert not np.isnan(r["z_lab"]).any()  # every particle sampled once
    np.testing.assert_allclose(r["z_lab"], z0 + vz * T, rtol=0, atol=1e-9 * T)
    np.testing.assert_allclose(r["x_lab"], x0 + vx * T, rtol=0, atol=1e-9 * T)
    wsum = np.real(s.particles(0)["w"]).sum()
    assert r["w"] == pytest.approx(wsum, rel=1e-15)


def test_probe_bunching_of_a_lab_lattice_decays_with_the_energy_spread():
    """Lab positions on a lattice of period lambda (b = 1 at lab time 0) spread by
    the velocity spread: |b(T)| = |<exp(i k v_z T)>| (computed from the same
    particles' lab velocities), well below 1 at the probed time."""
    n = 4096
    w = _ballistic_case(n)
    w["beam"]["rel_energy_spread_rms"] = 0.05
    w["beam"]["gamma_lab"] = 6.0
    w["frame"]["gamma_boost"] = 2.0
    nrm = pin.beam_normals(n, 5)
    s0 = po.Sim(w, nrm)
    szl = s0.info().sig_zlab
    lam = 2.0
    nrm[2] = np.round(nrm[2] * szl / lam) * lam / szl  # lab z of every particle on a lattice of period lam
    s = po.Sim(w, nrm)
    x0, z0, vx, vz = _lab_initial(w, nrm, s)
    i = s.info()
    k = 2 * math.pi / lam
    assert abs(np.exp(1j * k * z0).mean()) == pytest.approx(1.0, abs=1e-9)
    zp = np.real(s.particles(0)["z"])
    T = i.gR * i.bR * (zp.max() - i.zoff) + 200.0
    r = po.lab_probe(s, _steps_to(i, zp, T), T, k)
    assert not np.isnan(r["z_lab"]).any()
    b = math.hypot(r["c"], r["s"]) / r["w"]
    expect = abs(np.exp(1j * k * (z0 + vz * T)).mean())
    assert b == pytest.approx(expect, abs=1e-8)
    assert b < 0.9
