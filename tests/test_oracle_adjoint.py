"""Oracle pins for the discrete adjoint of the step (gradient of the final
bunching factor w.r.t. undulator K and plasma density).

* complex-step derivatives of the whole forward run (Squire & Trapp 1998)
  give dL/dK and dL/dn0 to round-off, independently of the adjoint code;
* the one-step dot-product test <lam_in, J v> = <J^T lam_in, v> with J v
  from the complex-step tangent of one step;
* central finite differences at h = 1e-6 relative (1e-4 bar).
"""
import math

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po

pytestmark = pytest.mark.usefixtures("oracle_built")

KB = 2 * math.pi / 20.0


def _case(n_beam=256, nz=32, charge=3e-9, pusher=None):
    w = pin.scaled(pin.adjoint_subcase(), nx=8, ny=8, nz=nz, n_beam=n_beam, sigma=(2, 2, 4))
    w["beam"]["charge_C"] = charge
    # the undulator reaches the beam within a few steps
    w["undulator"]["z_start_lab_m"] = w["frame"]["gamma_boost"] * 10 * w["grid"]["dx_m"]
    w["undulator"]["entrance_ramp_periods"] = 0.5
    return w


@pytest.mark.parametrize("pusher", [1, 0])
def test_adjoint_matches_complex_step(pusher):
    w = _case()
    nrm = pin.beam_normals(w["beam"]["n_macro"], 2)
    N = 14
    L, gK, gn = po.grad_bunching(w, nrm, N, KB, pusher=pusher)
    K, n0 = w["undulator"]["K"], w["plasma"]["n0_lab_cm3"]
    h = 1e-30
    lk = po.loss_bunching(w, nrm, N, KB, complex_step=True, pusher=pusher, hK=h * K)
    ln = po.loss_bunching(w, nrm, N, KB, complex_step=True, pusher=pusher, hn0=h * n0)
    assert abs(lk[0] - L) < 1e-13 * L and abs(ln[0] - L) < 1e-13 * L
    cs_gK = lk[1] / h  # = K dL/dK
    cs_gn = ln[1] / h  # = n0 dL/dn0
    assert abs(cs_gK) > 1e-8 and abs(cs_gn) > 1e-8, (cs_gK, cs_gn)
    assert abs(gK - cs_gK) < 1e-9 * abs(cs_gK), (gK, cs_gK)
    assert abs(gn - cs_gn) < 1e-9 * abs(cs_gn), (gn, cs_gn)


def _alive_mask_for_state(s_info, alive_b, alive_p, nc):
    nb, npl = s_info.n_beam, s_info.n_plasma
    m = np.ones(6 * (nb + npl) + 6 * nc, bool)
    o = 0
    for n, al in ((nb, alive_b), (npl, alive_p)):
        for _ in range(6):
            m[o:o + n] = al[:n] == 1
            o += n
    return m


@pytest.mark.parametrize("n_before", [3, 6])
def test_one_step_dot_product(n_before):
    w = _case(n_beam=128)
    nrm = pin.beam_normals(w["beam"]["n_macro"], 4)
    sr = po.Sim(w, nrm)
    sc = po.Sim(w, nrm, complex_step=True)
    sr.step(n_before)
    sc.step(n_before)
    x_n = sr.state()
    info_n = sr.info()
    pb, pp = sr.particles(0), sr.particles(1)
    mask_n = _alive_mask_for_state(info_n, pb["alive"].copy(), pp["alive"].copy(), sr.nc)
    rng = np.random.default_rng(n_before)
    v = rng.normal(size=x_n.size) * mask_n
    # scale perturbation per block so every part of the state matters
    h = 1e-25
    xc = sc.state()
    np.testing.assert_allclose(xc.real, x_n, rtol=1e-13, atol=1e-13)
    sc.set_state(xc.real + 1j * h * v)
    sc.step(1)
    Jv = sc.state().imag / h
    # forward real step to learn the layout and the alive flags of state n+1
    sr2 = po.Sim(w, nrm)
    sr2.step(n_before + 1)
    info_1 = sr2.info()
    mask_1 = _alive_mask_for_state(info_1, sr2.particles(0)["alive"].copy(), sr2.particles(1)["alive"].copy(), sr.nc)
    lam = rng.normal(size=Jv.size) * mask_1
    lam_out, gK, gn = sr.adjoint_step(lam, x_n.size)
    lhs = lam @ Jv
    rhs = lam_out @ v
    assert abs(lhs - rhs) < 1e-10 * (abs(lam) @ abs(Jv) + abs(lam_out) @ abs(v)), (lhs, rhs)
    # the adjoint leaves the forward state untouched
    np.testing.assert_array_equal(sr.state(), x_n)


def test_adjoint_matches_central_differences():
    w = _case()
    nrm = pin.beam_normals(w["beam"]["n_macro"], 5)
    N = 14
    L, gK, gn = po.grad_bunching(w, nrm, N, KB)
    for key, sub, g in (("K", "undulator", gK), ("n0_lab_cm3", "plasma", gn)):
        p0 = w[sub][key]
        h = 1e-6
        vals = []
        for sgn in (+1, -1):
            ww = pin.scaled(w)
            ww[sub][key] = p0 * (1 + sgn * h)
            vals.append(po.loss_bunching(ww, nrm, N, KB)[0])
        fd = (vals[0] - vals[1]) / (2 * h)  # = p0 dL/dp0
        assert abs(fd - g) < 1e-4 * abs(g), (key, fd, g)


def test_stored_500_step_adjoint_agrees_with_complex_step():
    """The oracle's 500-step adjoint of the 16x16x64 subcase (checkpointed every step, the
    reference for the GPU's checkpointed adjoint) agrees with the complex-step derivative of
    the oracle's forward run, computed by the same script, to 1e-11 relative."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_subcase_500.json")
    g = json.load(open(path))
    assert g["nsteps"] == 500
    for a, b in (("K_dL_dK", "complex_step_K_dL_dK"), ("n0_dL_dn0", "complex_step_n0_dL_dn0")):
        assert abs(g[a]) > 1e-2 * g["L"]
        assert abs(g[a] - g[b]) <= 1e-11 * abs(g[b]), (a, g[a], g[b])
