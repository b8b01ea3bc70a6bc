"""GPU parity of the initial beam self-field (options.init_fields = 1): the
FP64 relativistic Poisson solve of k_initfield.hip against the oracle's
(FFT + tridiagonal in numpy), then the step from that field.

Bars: FP64 fields 1e-11 of the field's norm at t' = 0 (two exact solvers in
FP64 with different summation orders: O(n) line DFTs against FFTs); the
following FP64 steps 1e-12 per step as the other FP64 parity tests; FP32
fields 1e-6 (FP32 storage and the split positions' rounding of the charge);
Gauss's law at t' = 0 to 1e-13 of the gross charge density (FP64)."""
import math

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po
from test_hip_fp64 import FIELDS, _case, _compare, _pair

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_built")]

CASES = ["undulator_beam", "beam_plasma_ions", "ragged"]


def _field_err(gpu, ref):
    out = {}
    for f in FIELDS:
        a, b = gpu.field(f).astype(np.float64), ref.field(f)
        nb = np.linalg.norm(b)
        out[f] = np.linalg.norm(a - b) / nb if nb > 0 else np.abs(a).max()
    return out


@pytest.mark.parametrize("case", CASES)
def test_fp64_initial_field_matches_oracle(case):
    ref, gpu = _pair(_case(case), init_fields=1)
    po.init_beam_fields(ref)
    err = _field_err(gpu, ref)
    assert np.linalg.norm(ref.field("Ex")) > 0
    for f, e in err.items():
        assert e <= 1e-11, (f, err)


@pytest.mark.parametrize("case", ["beam_plasma_ions", "undulator_beam"])
def test_fp64_steps_from_initial_field_match_oracle(case):
    ref, gpu = _pair(_case(case), init_fields=1)
    po.init_beam_fields(ref)
    for n in (1, 4, 10):
        k = n - ref.info().step
        ref.step(k)
        gpu.step(k)
        _compare(ref, gpu, 1e-11 + 1e-12 * n, f"step {n}")


def test_fp64_initial_field_satisfies_gauss_law():
    """div E - rho at t' = 0, against the gross density (plasma electrons and
    ions cancel to round-off of gamma_R n0) or the net one, whichever is larger."""
    from paper_2411_04703_amd import abi
    from paper_2411_04703_amd.sim import derive
    w = _case("beam_plasma_ions")
    _, gpu = _pair(w, init_fields=1)
    d = gpu.diag(abi.PIC_DIAG_GAUSS)
    dv = derive(pin.scaled(w))
    scale = max(d["rho_max"], dv["gamma_R"] * dv["n0_norm"])
    assert d["rho_max"] > 0
    assert d["gauss_max"] <= 1e-13 * scale, (d["gauss_max"], d["rho_max"], scale)


@pytest.mark.parametrize("case", CASES)
def test_fp32_initial_field_matches_oracle(case):
    from paper_2411_04703_amd.sim import Sim
    w = _case(case)
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    ref = po.Sim(w, nrm)
    po.init_beam_fields(ref)
    w = pin.scaled(w)
    w["frame"]["window_beta"] = ref.info().bw
    s32 = Sim(w, nrm, precision=1, init_fields=1)
    err = _field_err(s32, ref)
    for f, e in err.items():
        assert e <= 1e-6, (f, err)


def test_fp32_tracks_fp64_from_initial_field():
    from paper_2411_04703_amd.sim import Sim
    w = _case("beam_plasma_ions")
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    w = pin.scaled(w)
    w["frame"]["window_beta"] = po.Sim(w, nrm).info().bw
    s32 = Sim(w, nrm, precision=1, init_fields=1)
    s64 = Sim(w, nrm, precision=0, init_fields=1, max_steps=64)
    s32.step(20)
    s64.step(20)
    # as for the zero-field start: FP32 rounds each step's field change relative to the gross
    # (cancelling) plasma and ion currents
    i = po.Sim(w, nrm).info()
    gross = i.dt * i.gR * i.n0n * i.bR * math.sqrt(w["grid"]["nx"] * w["grid"]["ny"] * w["grid"]["nz"])
    total = math.sqrt(sum(np.linalg.norm(s64.field(f)) ** 2 for f in FIELDS))
    for f in FIELDS:
        err = np.linalg.norm(s32.field(f) - s64.field(f))
        assert err <= 1e-4 * max(total, gross), (f, err, total, gross)
    d32, d64 = s32.diag(), s64.diag()
    for k in ("mean", "sigma", "usigma", "emit"):
        np.testing.assert_allclose(d32[k], d64[k], rtol=1e-4, err_msg=k)


# ---- the neutralising charge faded over T (options.init_fields = 2, section 3's artificial ions)
FADE_CELLS = 10.0  # cells / c: 20 steps at the half-cell step


def _fade_s(w):
    return FADE_CELLS * w["grid"]["dx_m"] / 299792458.0


@pytest.mark.parametrize("case", ["beam_only", "beam_plasma_ions", "ragged"])
def test_fp64_neutraliser_fade_matches_oracle(case):
    """Fields and particles of the FP64 path against the oracle's through the fade and past it
    (the GPU's line DFTs and the oracle's FFTs give the charge's field to 1e-11, then the per-step
    bar); the Gauss residual (FP64 diagnostic, which counts the fading charge) stays put."""
    from paper_2411_04703_amd import abi
    w = _case(case)
    w["beam"]["charge_C"] = 3e-9
    ref, gpu = _pair(w, init_fields=2, neutral_fade_s=_fade_s(w))
    po.init_neutraliser(ref, _fade_s(w))
    from paper_2411_04703_amd.sim import derive
    gpu.diag(abi.PIC_DIAG_GAUSS)
    dv = derive(pin.scaled(w))
    # round-off is relative to the gross densities: the beam's own (the net charge at t' = 0 is the
    # beam and its neutraliser, which cancel) and the plasma's (electrons and ions cancel)
    scale = max(np.abs(ref.rho(1)).max(), dv["gamma_R"] * dv["n0_norm"])
    for n in (1, 5, 12, 20, 26):
        k = n - ref.info().step
        ref.step(k)
        gpu.step(k)
        _compare(ref, gpu, 1e-11 + 1e-12 * n, f"step {n}")
        d = gpu.diag(abi.PIC_DIAG_GAUSS)
        assert d["gauss_drift"] <= 1e-12 * scale, (n, d["gauss_drift"], scale)


def test_fp32_neutraliser_fade_tracks_fp64():
    from paper_2411_04703_amd import abi
    from paper_2411_04703_amd.sim import Sim
    w = _case("beam_plasma_ions")
    w["beam"]["charge_C"] = 3e-9
    nrm = pin.beam_normals(w["beam"]["n_macro"], 0)
    w = pin.scaled(w)
    w["frame"]["window_beta"] = po.Sim(w, nrm).info().bw
    s32 = Sim(w, nrm, precision=1, init_fields=2, neutral_fade_s=_fade_s(w))
    s64 = Sim(w, nrm, precision=0, init_fields=2, neutral_fade_s=_fade_s(w), max_steps=64)
    s32.diag(abi.PIC_DIAG_GAUSS)
    for n in (10, 26):
        s32.step(n - int(s32.diag()["step"]))
        s64.step(n - int(s64.diag()["step"]))
        i = po.Sim(w, nrm).info()
        gross = i.dt * i.gR * i.n0n * i.bR * math.sqrt(w["grid"]["nx"] * w["grid"]["ny"] * w["grid"]["nz"])
        total = math.sqrt(sum(np.linalg.norm(s64.field(f)) ** 2 for f in FIELDS))
        for f in FIELDS:
            err = np.linalg.norm(s32.field(f) - s64.field(f))
            assert err <= 1e-4 * max(total, gross), (n, f, err, total, gross)
        d = s32.diag(abi.PIC_DIAG_GAUSS)
        # FP32 fields and the 2^-f current quantum: the residual moves at FP32 round-off of the gross density
        dv = __import__("paper_2411_04703_amd.sim", fromlist=["derive"]).derive(w)
        assert d["gauss_drift"] <= 1e-5 * dv["gamma_R"] * dv["n0_norm"], (n, d["gauss_drift"])
