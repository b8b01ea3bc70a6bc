"""Oracle pins: frame helpers, beam transform and external field against the
paper's printed numbers and closed forms (section 1, Eq. Lor1-Belon, M1-M4,
Vprime, Nnormi; Table 1; section 3 and 4 run times)."""
import json
import math
import os

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_numbers.json")))

C = 299792458.0
QE = 1.602176634e-19
ME = 9.1093837015e-31

pytestmark = pytest.mark.usefixtures("oracle_built")


def test_elongation_worked_example():
    g = GOLD["elongation"]
    L = po.lib()
    F = L.orc_elongation(g["gamma_beam"], g["gamma_frame"])
    assert abs(g["length_lab_m"] * F - g["length_boosted_m"]) <= g["rel_tol"] * g["length_boosted_m"]


def test_fel_wavelength_and_doppler():
    g = GOLD["fel_wavelength"]
    K = QE * g["B_peak_T"] * g["period_m"] / (2 * math.pi * ME * C)  # deflection parameter of the undulator
    lam = po.lib().orc_fel_wavelength(g["period_m"], K, g["gamma_beam"])
    assert abs(lam - g["lambda_m"]) <= g["rel_tol"] * g["lambda_m"]
    d = GOLD["doppler"]
    lamb = po.lib().orc_doppler(lam, d["gamma_frame"])
    assert abs(lamb - d["lambda_boosted_m"]) <= d["rel_tol"] * d["lambda_boosted_m"]


def test_beta_closed_form():
    L = po.lib()
    for g in (1.0, 1.5, 10.0, 40.0, 1e4):
        b = L.orc_beta(g)
        assert abs(g * g * (1 - b * b) - 1.0) < 1e-12 * g * g


def test_lab_distance_vs_boosted_time():
    """z_lab ~ gamma_R beta_R c t' for the frame origin: Lorentz-transform the lab event."""
    g = GOLD["lab_distance_vs_boosted_time"]
    L = po.lib()
    for p in g["pairs"]:
        gR = p["gamma_frame"]
        bR = L.orc_beta(gR)
        z = p["z_lab_m"]
        lab = np.array([0.0, 0.0, z, z / bR])  # (x, y, z, ct): frame origin passes z at c t = z / beta_R
        out = np.zeros(4)
        uout = np.zeros(3)
        L.orc_lab_to_boosted(gR, lab.ctypes.data, np.zeros(3).ctypes.data, out.ctypes.data, uout.ctypes.data)
        assert abs(out[2]) < 1e-12 * z  # stays at the frame origin
        t_ps = out[3] / C * 1e12
        assert abs(t_ps - p["t_boosted_ps"]) <= g["rel_tol"] * p["t_boosted_ps"], p


def test_lorentz_round_trip_and_invariants():
    L = po.lib()
    rng = np.random.default_rng(1)
    for _ in range(50):
        gR = 1 + 50 * rng.random()
        lab = rng.normal(size=4)
        u = rng.normal(size=3) * 5
        out = np.zeros(4)
        uo = np.zeros(3)
        L.orc_lab_to_boosted(gR, lab.ctypes.data, u.ctypes.data, out.ctypes.data, uo.ctypes.data)
        # interval invariance: t^2 - z^2 (c = 1 in these units)
        assert abs((lab[3] ** 2 - lab[2] ** 2) - (out[3] ** 2 - out[2] ** 2)) < 1e-9 * (1 + gR * gR)
        # mass shell: gamma'^2 - u'^2 = 1 with gamma' = gR (gamma - bR u_z)
        bR = L.orc_beta(gR)
        g = math.sqrt(1 + u @ u)
        gp = gR * (g - bR * u[2])
        assert abs(gp * gp - uo @ uo - 1.0) < 1e-10 * gp * gp


def _small(w=None, n=2048, **kw):
    w = w or pin.workload(0)
    return pin.scaled(w, n_beam=n, **kw)


def test_monoenergetic_beam_maps_by_elongation():
    """Per-particle transform + drift of a cold beam reproduces Eq. Belon exactly:
    z'_j - z'_c = F z_j with F = gamma_B / (gamma_B gamma_R - u_B u_R)."""
    w = _small()
    w["beam"]["rel_energy_spread_rms"] = 0.0
    w["beam"]["emit_n_m"] = [0.0, 0.0]
    nrm = pin.beam_normals(w["beam"]["n_macro"], 3)
    s = po.Sim(w, nrm)
    i = s.info()
    p = s.particles(0)
    zlab = i.sig_zlab * nrm[2]
    F = po.lib().orc_elongation(w["beam"]["gamma_lab"], w["frame"]["gamma_boost"])
    alive = p["alive"] == 1
    np.testing.assert_allclose(p["z"][alive] - i.zoff, F * zlab[alive], rtol=1e-12, atol=1e-12)
    gB, gR = w["beam"]["gamma_lab"], w["frame"]["gamma_boost"]
    gp = gR * gB * (1 - math.sqrt(1 - 1 / gB ** 2) * math.sqrt(1 - 1 / gR ** 2))
    np.testing.assert_allclose(p["uz"][alive], math.sqrt(gp * gp - 1), rtol=1e-12)


def test_beam_sample_moments():
    w = _small(n=65536)
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    s = po.Sim(w, nrm)
    d = s.diag(2 * math.pi / 20)
    N = d["n_beam_alive"]
    sig = w["beam"]["sigma_cells"]
    for k in range(3):
        assert abs(d["sigma"][k] - sig[k]) < 4 * sig[k] / math.sqrt(2 * N), (k, d["sigma"][k])
    # normalised emittance: sigma_x sigma_ux in cells -> metres
    for k in range(2):
        eps = d["emit"][k] * w["grid"]["dx_m"]
        assert abs(eps - w["beam"]["emit_n_m"][k]) < 4 * 1e-6 * math.sqrt(2.0 / N) * 2


def test_beam_sampling_reproducible():
    w = _small(n=1000)
    a = po.Sim(w, pin.beam_normals(1000, 7)).particles(0)
    b = po.Sim(w, pin.beam_normals(1000, 7)).particles(0)
    for k in ("x", "y", "z", "ux", "uy", "uz"):
        assert np.array_equal(a[k], b[k])


def _ext(s, z, t):
    E = np.zeros(3)
    B = np.zeros(3)
    s.L.orc_ext_field.argtypes = [po.C.c_void_p, po.C.c_double, po.C.c_double, po.C.c_void_p, po.C.c_void_p]
    s.L.orc_ext_field(s.h, z, t, E.ctypes.data, B.ctypes.data)
    return E, B


def test_external_field_invariants_and_period():
    """Eq. M1-M4: E'.B' = 0 and |B'|^2 - |E'|^2 = |B_lab|^2; spatial period lambda_u / gamma_R
    (Table 1: 2 cm at gamma_R = 50 -> 0.4 mm); pattern drifts at -beta_R (Eq. Vprime)."""
    w = _small(n=16)
    gR = 50.0
    w["frame"]["gamma_boost"] = gR
    w["undulator"].update(kind=1, K=1.3, period_lab_m=0.02, z_start_lab_m=-1.0, length_lab_m=10.0,
                          entrance_ramp_periods=0.0)
    s = po.Sim(w, pin.beam_normals(16, 0))
    i = s.info()
    dx = w["grid"]["dx_m"]
    per_cells = 0.4e-3 / dx
    B0 = i.B0
    for z in np.linspace(10, 40, 7):
        for t in (0.0, 3.7, 100.0):
            E, B = _ext(s, z, t)
            assert abs(E @ B) < 1e-12 * (B @ B)
            assert abs((B @ B - E @ E) - B0 ** 2) < 1e-10 * B0 ** 2
            E2, B2 = _ext(s, z + per_cells, t)
            np.testing.assert_allclose(B2, B, atol=1e-9 * B0)
            dt = 1.234
            E3, B3 = _ext(s, z - i.bR * dt, t + dt)
            np.testing.assert_allclose(B3, B, atol=1e-9 * B0)
    # normalised amplitude: |B_lab| = K k_u D
    assert abs(B0 - 1.3 * 2 * math.pi * dx / 0.02) < 1e-14


def test_planar_external_field_structure():
    """Planar lab field B = (0, B0 sin phi, 0) through Eq. M1-M4: B' = (0, gR B_y, 0),
    E' = (-bR B'_y, 0, 0), peak |B'_y| = gR B0, spatial period lambda_u / gR, pattern
    drifting at -beta_R (Eq. Vprime)."""
    w = _small(n=16)
    gR = 50.0
    w["frame"]["gamma_boost"] = gR
    w["undulator"].update(kind=2, K=1.3, period_lab_m=0.02, z_start_lab_m=-1.0, length_lab_m=10.0,
                          entrance_ramp_periods=0.0)
    s = po.Sim(w, pin.beam_normals(16, 0))
    i = s.info()
    dx = w["grid"]["dx_m"]
    per_cells = 0.4e-3 / dx
    peak = 0.0
    for z in np.linspace(10, 10 + per_cells, 41):
        for t in (0.0, 3.7):
            E, B = _ext(s, z, t)
            assert B[0] == 0.0 and B[2] == 0.0 and E[1] == 0.0 and E[2] == 0.0
            assert abs(E[0] + i.bR * B[1]) < 1e-12 * i.B0 * gR
            peak = max(peak, abs(B[1]))
            E2, B2 = _ext(s, z + per_cells, t)
            np.testing.assert_allclose(B2, B, atol=1e-9 * i.B0 * gR)
            dt = 1.234
            E3, B3 = _ext(s, z - i.bR * dt, t + dt)
            np.testing.assert_allclose(B3, B, atol=1e-9 * i.B0 * gR)
    assert abs(peak - gR * i.B0) < 2e-3 * gR * i.B0  # 41 samples per period: cos(pi/40) = 0.9969


def test_lab_static_particle_is_force_free_under_vay():
    """A particle at rest in the lab has u' = -gR bR z; with E' + v' x B' = 0 the Vay pusher
    keeps it exactly (Vay 2008); Boris does not."""
    w = _small(n=16)
    w["frame"]["gamma_boost"] = 20.0
    s = po.Sim(w, pin.beam_normals(16, 0))
    i = s.info()
    u = np.array([0.0, 0.0, -i.uR])
    worst_boris = 0.0
    for z in np.linspace(20, 60, 11):
        E, B = _ext(s, z, 5.0)
        if B @ B == 0:
            continue
        out = po.push(1, -1.0, i.dt, u, E, B)
        np.testing.assert_allclose(out, u, atol=1e-13 * i.uR)
        ob = po.push(0, -1.0, i.dt, u, E, B)
        worst_boris = max(worst_boris, np.abs(ob - u).max())
    assert worst_boris > 1e-9


def _undulator_invariants(kind, dt, t_end=60.0):
    """Deviation of the two closed-form invariants of an electron in the flat part
    of an ideal undulator, carried into the boosted frame: the transverse
    canonical momentum u_perp - A_perp, A_perp = -K (cos k_u a, sin k_u a) for the
    helical field (-K cos k_u a, 0) for the planar one (a: lab distance into the
    undulator; the transverse vector potential is the same in both frames), and
    the lab energy gamma_R (gamma' + beta_R u'_z) (the lab field is purely
    magnetic).  Self-fields are switched off by a vanishing charge; the
    undulator starts well behind the beam, so it sits in the flat part."""
    w = pin.scaled(pin.workload(0), n_beam=64)
    w["beam"]["charge_C"] = 1e-30
    w["beam"]["rel_energy_spread_rms"] = 0.0
    w["beam"]["emit_n_m"] = [1e-12, 1e-12]
    u = w["undulator"]
    lu = u["period_lab_m"]
    u.update(kind=kind, z_start_lab_m=-5 * lu, length_lab_m=200 * lu, entrance_ramp_periods=2.0)
    s = po.Sim(w, pin.beam_normals(64, 0), dt_override=dt)
    i = s.info()
    K, z0 = u["K"], u["z_start_lab_m"] / w["grid"]["dx_m"]
    inv, glab = [], []
    p0 = s.particles(0)
    for n in range(int(round(t_end / dt))):
        s.step(1)
        p1 = s.particles(0)
        # u^(n+1/2) belongs to the middle of the move x^n -> x^(n+1)
        a = i.gR * (0.5 * (p0["z"] + p1["z"]) - i.zoff + i.bR * (n + 0.5) * i.dt) - z0
        ax = -K * np.cos(i.ku * a)
        ay = -K * np.sin(i.ku * a) if kind == 1 else 0.0 * a
        inv.append(np.stack([p1["ux"] - ax, p1["uy"] - ay]))
        g = np.sqrt(1 + p1["ux"] ** 2 + p1["uy"] ** 2 + p1["uz"] ** 2)
        glab.append(i.gR * (g + i.bR * p1["uz"]))
        p0 = p1
    assert (p1["alive"] == 1).all()
    inv, glab = np.array(inv), np.array(glab)
    # the electrons pass several undulator periods
    assert i.ku * i.gR * (1 + i.bw) * t_end > 4 * 2 * math.pi
    return np.abs(inv - inv[0]).max() / K, np.abs(glab / glab[0] - 1).max()


@pytest.mark.parametrize("kind", [1, 2])
def test_undulator_trajectory_invariants(kind):
    """The leap-frog orbit keeps both invariants to second order in dt: their
    deviation is below 5e-4 of K (lab energy 1e-7) at dt = 0.1 and grows by
    4x when dt doubles.  A wrong sign or boost factor of the transformed
    field, or a phase that does not drift at -beta_R, breaks both at order one."""
    d1, g1 = _undulator_invariants(kind, 0.1)
    d2, g2 = _undulator_invariants(kind, 0.2)
    assert d1 < 5e-4 and g1 < 1e-7, (d1, g1)
    assert 3.5 < d2 / d1 < 4.5, (d1, d2)
    assert 3.5 < g2 / g1 < 4.5, (g1, g2)
