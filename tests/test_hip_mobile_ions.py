"""GPU tests of mobile plasma ions (ions = 2) beyond the shared FP64 parity and
FP32 tracking cases: plasma diagnostics against the oracle, the ions' own
phase space in FP32 against FP64, and the adjoint's refusal.

Bars: FP64 counts exact, plasma kinetic energy 1e-12 relative (sums of the
same terms in another order); FP32 ion momenta 1e-4 of the momentum
magnitude after 20 steps (FP32 rounding of fields and offsets, as the FP32
tracking bar), positions 2e-5 cells."""
import math

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po
from test_hip_fp64 import _case, _pair

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_built")]


def _oracle_plasma(ref):
    n = sum(int((ref.particles(sp)["alive"] == 1).sum()) for sp in (1, 2))
    return n, ref.diag(1.0)["kin_plasma"]


@pytest.mark.parametrize("case", ["mobile_ions", "light_ions"])
def test_fp64_plasma_diagnostics_match_oracle(case):
    ref, gpu = _pair(_case(case))
    for n in (0, 10):
        ref.step(n - ref.info().step)
        gpu.step(n - int(gpu.diag()["step"]))
        d = gpu.diag()
        cnt, kin = _oracle_plasma(ref)
        assert d["n_plasma"] == cnt, n
        assert d["kin_plasma"] == pytest.approx(kin, rel=1e-12), n
    i = ref.info()
    assert i.n_ions > 0 and i.ion_mass == (1836.15267343 if case == "mobile_ions" else 4.0)


def test_fp32_ion_phase_space_tracks_fp64():
    from paper_2411_04703_amd.sim import Sim
    w = _case("light_ions")
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    w = pin.scaled(w)
    i = po.Sim(w, nrm).info()
    w["frame"]["window_beta"] = i.bw
    s32 = Sim(w, nrm, precision=1)
    s64 = Sim(w, nrm, precision=0, max_steps=64)
    nsteps = 20
    s32.step(nsteps)
    s64.step(nsteps)
    ppz = w["plasma"]["ppc"][2]

    def ions(p):
        """ions ordered by their lattice site (sheet, row, column): they stay within a
        small fraction of a cell of the site, so the integer keys match exactly"""
        al = (p["alive"] == 1) & (p["w"] < 0)
        a = np.stack([p[k][al] for k in ("z", "y", "x", "uz", "uy", "ux", "w")], axis=1)
        sheet = np.rint((a[:, 0] + i.bR * nsteps * i.dt) * ppz - 0.5)
        keys = (np.rint(a[:, 2] - 0.5), np.rint(a[:, 1] - 0.5), sheet)
        return a[np.lexsort(keys)]

    a, b = ions(s32.particles(1)), ions(s64.particles(1))
    assert a.shape == b.shape and a.shape[0] > 0
    np.testing.assert_allclose(a[:, :3], b[:, :3], atol=2e-5)
    umag = np.linalg.norm(b[:, 3:6])
    assert np.linalg.norm(a[:, 3:6] - b[:, 3:6]) <= 1e-4 * umag
    # the ions did respond: transverse momenta well above the FP32 noise
    assert np.abs(b[:, 4:6]).max() > 1e-6
    assert s32.diag()["kin_plasma"] == pytest.approx(s64.diag()["kin_plasma"], rel=1e-5)


def test_adjoint_refuses_mobile_ions():
    import torch

    from paper_2411_04703_amd import abi
    from paper_2411_04703_amd.sim import Sim
    w = _case("mobile_ions")
    s = Sim(pin.scaled(w), pin.beam_normals(w["beam"]["n_macro"], 0), precision=0, record=1, max_steps=8)
    lam = torch.zeros(s.lambda_len(), dtype=torch.float64, device="cuda")
    with pytest.raises(abi.PicError) as e:
        s.adjoint_seed(lam)
    assert e.value.status == abi.PIC_EINVAL
    with pytest.raises(abi.PicError) as e:
        s.adjoint_step(lam, np.zeros(2))
    assert e.value.status == abi.PIC_EINVAL
    assert not math.isnan(s.diag()["kin_plasma"])
