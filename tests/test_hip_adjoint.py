"""GPU adjoint (FP64 record mode, checkpoint and recompute) against central
finite differences of the GPU forward, h = 1e-6 relative, bar 1e-4 relative:
on the 16x16x64 subcase at both ends of the parameter ranges (K in [0.5, 2],
n0 in [1e15, 1e17] cm^-3; there also at h/10, with the perturbed runs' discrete
events equal to the unperturbed run's), and on the 64x64x256 adjoint workload
(1,048,576 beam particles plus 2 ppc plasma, 500 steps, checkpoint every 50)."""
import copy

import numpy as np
import pytest
import torch

import picinputs as pin
from oracle import pyoracle as po

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_built")]

H = 1e-6


def _loss(w, nrm, nsteps, every, K, n0):
    from paper_2411_04703_amd.autograd import bunching_loss
    with torch.no_grad():
        return float(bunching_loss(torch.tensor(K, dtype=torch.float64), torch.tensor(n0, dtype=torch.float64),
                                   w, nrm, nsteps, every))


def _check(w, nrm, nsteps, every):
    from paper_2411_04703_amd.autograd import bunching_grad
    K, n0 = w["undulator"]["K"], w["plasma"]["n0_lab_cm3"]
    L, gK, gn = bunching_grad(w, nrm, nsteps, every=every)
    fK = (_loss(w, nrm, nsteps, every, K * (1 + H), n0) - _loss(w, nrm, nsteps, every, K * (1 - H), n0)) / (2 * H)
    fn = (_loss(w, nrm, nsteps, every, K, n0 * (1 + H)) - _loss(w, nrm, nsteps, every, K, n0 * (1 - H))) / (2 * H)
    assert abs(gK) > 1e-4 * L and abs(gn) > 1e-4 * L, (L, gK, gn)  # both gradients are nontrivial
    assert gK == pytest.approx(fK, rel=1e-4), (gK, fK)
    assert gn == pytest.approx(fn, rel=1e-4), (gn, fn)
    return L, gK, gn


def _events(w, nrm, nsteps, K, n0):
    """The discrete events of a forward run: window shifts, plasma entering and leaving, beam losses."""
    from paper_2411_04703_amd.sim import Sim
    w2 = copy.deepcopy(w)
    w2["undulator"]["K"] = K
    w2["plasma"]["n0_lab_cm3"] = n0
    s = Sim(w2, nrm, precision=0, max_steps=nsteps + 2)
    s.step(nsteps)
    d = s.diag()
    return d["k0"], d["n_beam"], d["n_plasma"], d["beam_lost"]


@pytest.mark.parametrize("K,n0", [(0.5, 1e15), (2.0, 1e17)])
def test_adjoint_subcase_matches_central_differences(K, n0):
    """Also: the central differences at h and h/10 agree (neither step size is truncation- or
    rounding-limited at the bar), and the perturbed forward runs see the same discrete events as the
    unperturbed one (the loss is differentiable along the differences)."""
    w = pin.adjoint_subcase()
    w["undulator"]["K"] = K
    w["plasma"]["n0_lab_cm3"] = n0
    w["beam"]["charge_C"] = 3e-9
    nrm = pin.beam_normals(w["beam"]["n_macro"], 7)
    w["frame"]["window_beta"] = po.Sim(w, nrm).info().bw
    nsteps, every = 48, 12
    L, gK, gn = _check(w, nrm, nsteps, every)
    h = H / 10
    fK = (_loss(w, nrm, nsteps, every, K * (1 + h), n0) - _loss(w, nrm, nsteps, every, K * (1 - h), n0)) / (2 * h)
    fn = (_loss(w, nrm, nsteps, every, K, n0 * (1 + h)) - _loss(w, nrm, nsteps, every, K, n0 * (1 - h))) / (2 * h)
    assert gK == pytest.approx(fK, rel=1e-4), (gK, fK)
    assert gn == pytest.approx(fn, rel=1e-4), (gn, fn)
    base = _events(w, nrm, nsteps, K, n0)
    assert base[0] > 0 and base[2] > 0, base
    for KK, nn in ((K * (1 + H), n0), (K * (1 - H), n0), (K, n0 * (1 + H)), (K, n0 * (1 - H))):
        assert _events(w, nrm, nsteps, KK, nn) == base, (KK, nn)


def test_adjoint_workload3_matches_central_differences():
    w = copy.deepcopy(pin.workload(3))
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    _check(w, nrm, w["steps"], w["checkpoint_every"])


def test_fp32_mode_adjoint_workload3_matches_fp64_mode_and_differences(progress):
    """FP32 mode on the 64x64x256 adjoint workload (500 steps, checkpoint every 50): the adjoint
    linearised about the FP32 trajectory against the FP64-mode adjoint and central differences of
    the FP64 forward, 1e-3 relative -- the FP32 trajectory departs from the FP64 one by per-step
    FP32 rounding that the beam-plasma dynamics amplifies (1e-5..1e-4 in the beam moments over
    this many steps), far above the FP64 gradient's own 1e-9 agreement with its differences."""
    from paper_2411_04703_amd import abi
    from paper_2411_04703_amd.autograd import bunching_grad
    w = copy.deepcopy(pin.workload(3))
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    n, every = w["steps"], w["checkpoint_every"]
    K, n0 = w["undulator"]["K"], w["plasma"]["n0_lab_cm3"]
    L64, gK64, gn64 = bunching_grad(w, nrm, n, every=every)
    progress("workload 3: fp64-mode gradient done")
    L32, gK32, gn32 = bunching_grad(w, nrm, n, every=every, precision=abi.PIC_FP32_SPLIT)
    progress("workload 3: fp32-mode gradient done")
    fK = (_loss(w, nrm, n, every, K * (1 + H), n0) - _loss(w, nrm, n, every, K * (1 - H), n0)) / (2 * H)
    fn = (_loss(w, nrm, n, every, K, n0 * (1 + H)) - _loss(w, nrm, n, every, K, n0 * (1 - H))) / (2 * H)
    print("workload 3 FP32-mode adjoint", L32 / L64 - 1, gK32 / gK64 - 1, gn32 / gn64 - 1, gK32 / fK - 1,
          gn32 / fn - 1, flush=True)
    assert L32 == pytest.approx(L64, rel=1e-3)
    for g32, g64, fd in ((gK32, gK64, fK), (gn32, gn64, fn)):
        assert g32 == pytest.approx(g64, rel=1e-3), (g32, g64)
        assert g32 == pytest.approx(fd, rel=1e-3), (g32, fd)


def test_fp32_record_ids_leave_the_forward_unchanged():
    """Carrying particle ids (FP32 record mode) does not change a single bit."""
    from paper_2411_04703_amd.sim import Sim
    w = pin.adjoint_subcase()
    w["beam"]["charge_C"] = 3e-9
    nrm = pin.beam_normals(w["beam"]["n_macro"], 3)
    a = Sim(w, nrm, precision=1)
    b = Sim(w, nrm, precision=1, record=1, max_steps=40)
    a.step(17)
    b.step(17)
    for f in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        assert np.array_equal(a.field(f), b.field(f)), f


@pytest.mark.parametrize("ions", [1, 2])
def test_fp32_state_export_matches_the_fp64_record_layout(ions):
    """An FP32 state exported to an FP64 record context puts every particle in
    the slot the FP64 run gives it: positions agree to FP32 offsets, alive
    flags exactly (up to a lattice sheet at the band edge); with mobile ions
    as well, which follow their sheet's electrons in both layouts."""
    from paper_2411_04703_amd.sim import Sim
    w = pin.adjoint_subcase()
    w["beam"]["charge_C"] = 3e-9
    w["plasma"].update(ions=ions, ion_mass=4.0)
    nrm = pin.beam_normals(w["beam"]["n_macro"], 4)
    w["frame"]["window_beta"] = po.Sim(w, nrm).info().bw
    s32 = Sim(w, nrm, precision=1, record=1, max_steps=30)
    s64 = Sim(w, nrm, precision=0, record=1, max_steps=30)
    ref = Sim(w, nrm, precision=0, record=1, max_steps=30)
    s32.step(12)
    ref.step(12)
    s32.export_to(s64)
    assert s64.diag()["step"] == 12 and s64.diag()["k0"] == ref.diag()["k0"]
    for sp in (0, 1):
        p, q = s64.particles(sp), ref.particles(sp)
        assert len(p["x"]) == len(q["x"])
        # a lattice sheet exactly at the band edge may be removed by one precision and not the other
        assert (p["alive"] != q["alive"]).sum() <= 2 * 16 * 16 * 2 * (2 if ions == 2 else 1), sp
        if sp == 1:
            assert ((p["w"] < 0) == (q["w"] < 0)).all() and ((q["w"] < 0).sum() > 0) == (ions == 2)
        al = (q["alive"] == 1) & (p["alive"] == 1)
        assert al.sum() > 0.99 * (q["alive"] == 1).sum()
        for k in ("x", "y", "z"):
            np.testing.assert_allclose(p[k][al], q[k][al], atol=1e-4, err_msg=(sp, k))
        for k in ("ux", "uy", "uz"):
            np.testing.assert_allclose(p[k][al], q[k][al], rtol=1e-4, atol=1e-6, err_msg=(sp, k))
    for f in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        assert np.allclose(s64.field(f), s32.field(f), rtol=0, atol=0), f


@pytest.mark.parametrize("K,n0", [(1.0, 1e16)])
def test_fp32_mode_adjoint_matches_fp64_mode_and_differences(K, n0):
    """FP32 mode: the adjoint linearised about the FP32 trajectory.  It agrees
    with the FP64-mode adjoint and with central differences of the FP64 forward
    to 1e-3 relative (the two trajectories differ at FP32 rounding; central
    differences of the FP32 forward itself at h = 1e-6 would measure its
    rounding, not its derivative)."""
    from paper_2411_04703_amd import abi
    from paper_2411_04703_amd.autograd import bunching_grad
    w = pin.adjoint_subcase()
    w["undulator"]["K"] = K
    w["plasma"]["n0_lab_cm3"] = n0
    w["beam"]["charge_C"] = 3e-9
    nrm = pin.beam_normals(w["beam"]["n_macro"], 7)
    w["frame"]["window_beta"] = po.Sim(w, nrm).info().bw
    L64, gK64, gn64 = bunching_grad(w, nrm, 48, every=12)
    L32, gK32, gn32 = bunching_grad(w, nrm, 48, every=12, precision=abi.PIC_FP32_SPLIT)
    assert L32 == pytest.approx(L64, rel=1e-4)
    assert gK32 == pytest.approx(gK64, rel=1e-3), (gK32, gK64)
    assert gn32 == pytest.approx(gn64, rel=1e-3), (gn32, gn64)
    fK = (_loss(w, nrm, 48, 12, K * (1 + H), n0) - _loss(w, nrm, 48, 12, K * (1 - H), n0)) / (2 * H)
    assert gK32 == pytest.approx(fK, rel=1e-3)


def _golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_subcase_500.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("precision,bar", [(0, 1e-9), (1, 1e-3)])
def test_adjoint_subcase_500_steps_against_oracle(precision, bar):
    """The 16x16x64 subcase of the adjoint workload over 500 steps with a checkpoint every 50
    (ten recomputed segments), against the oracle's stored-state adjoint of the same run
    (tests/golden/adjoint_subcase_500.json, written by the oracle alone; there the oracle's
    adjoint agrees with its complex-step derivatives to 3e-12).  FP64 mode: 1e-9 relative.
    FP32 mode (the adjoint linearised about the FP32 trajectory): 1e-3 relative, the FP32
    path's stated bar."""
    from paper_2411_04703_amd.autograd import bunching_grad
    g = _golden()
    w = pin.adjoint_subcase()
    w["frame"]["window_beta"] = g["window_beta"]
    nrm = pin.beam_normals(w["beam"]["n_macro"], g["seed"])
    L, gK, gn = bunching_grad(w, nrm, g["nsteps"], every=50, bunch_period=g["bunch_period_cells"],
                              precision=precision)
    print("adjoint 500", precision, L, gK, gn, g["L"], g["K_dL_dK"], g["n0_dL_dn0"], flush=True)
    assert L == pytest.approx(g["L"], rel=bar)
    assert gK == pytest.approx(g["K_dL_dK"], rel=bar)
    assert gn == pytest.approx(g["n0_dL_dn0"], rel=bar)
