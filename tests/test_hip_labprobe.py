"""GPU parity of the lab-frame probe (pic_lab_probe): the sums over sampled
beam particles against the oracle's probe on the same run.

Bars: FP64 path 1e-10 relative on every sum (the oracle interpolates between
its stored positions, the GPU reconstructs the start of the step from the
momentum: equal up to round-off); FP32 path 1e-5 on the sums (FP32 offsets:
~1e-7 cells, times gamma_R in the lab) and 1e-5 absolute on |b|."""
import math

import numpy as np
import pytest

import picinputs as pin
from oracle import pyoracle as po
from test_oracle_labprobe import _ballistic_case, _steps_to

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_built")]


def _cases():
    w = pin.workload(0)  # undulator beam: the fields act while the probe samples
    w["grid"]["nz"] = 192
    w["beam"]["z_center_cells"] = 96
    return {"ballistic": _ballistic_case(4096), "undulator_beam": w}


def _run(name, precision):
    from paper_2411_04703_amd.sim import Sim
    w = _cases()[name]
    nrm = pin.beam_normals(w["beam"]["n_macro"], 3)
    ref = po.Sim(w, nrm)
    i = ref.info()
    zp = np.real(ref.particles(0)["z"])
    T = i.gR * i.bR * (zp.max() - i.zoff) + 7.0
    n = _steps_to(i, zp, T)
    k = 2 * math.pi / 20.0
    ww = pin.scaled(w)
    ww["frame"]["window_beta"] = i.bw
    gpu = Sim(ww, nrm, precision=precision, **({} if precision else {"max_steps": 64}))
    gpu.lab_probe(T, k)
    gpu.step(n)
    g = gpu.lab_probe_read()
    r = po.lab_probe(ref, n, T, k)
    assert not np.isnan(r["z_lab"]).any()
    return g, r


@pytest.mark.parametrize("name", ["ballistic", "undulator_beam"])
def test_fp64_lab_probe_matches_oracle(name):
    g, r = _run(name, 0)
    assert g["w"] == pytest.approx(r["w"], rel=1e-14)
    for key in ("c", "s", "z", "zz"):
        assert g[key] == pytest.approx(r[key], rel=1e-10, abs=1e-10 * r["w"]), (key, g[key], r[key])


@pytest.mark.parametrize("name", ["ballistic", "undulator_beam"])
def test_fp32_lab_probe_matches_oracle(name):
    g, r = _run(name, 1)
    assert g["w"] == pytest.approx(r["w"], rel=1e-6)
    assert g["z"] == pytest.approx(r["z"], rel=1e-5)
    assert g["zz"] == pytest.approx(r["zz"], rel=1e-5)
    bg = math.hypot(g["c"], g["s"]) / g["w"]
    br = math.hypot(r["c"], r["s"]) / r["w"]
    assert abs(bg - br) < 1e-5, (bg, br)


def test_probe_disarmed_adds_nothing():
    from paper_2411_04703_amd.sim import Sim
    w = _cases()["ballistic"]
    nrm = pin.beam_normals(w["beam"]["n_macro"], 3)
    s = Sim(w, nrm, precision=1)
    s.lab_probe(float("nan"), 0.0)
    s.step(5)
    assert all(v == 0.0 for v in s.lab_probe_read().values())
