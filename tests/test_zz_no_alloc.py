"""The allocation-free diagnostics entry point (pic_diag_static) against
pic_diag through the C-ABI: the same kernels and the same fixed-order
reductions, only the partial sums live in the library's static device array,
so every output field must be equal bit for bit.  Two contexts in a row, the
second smaller (the array keeps the first one's contents), each read twice
with steps in between, in both precisions; and the size limit."""
import pytest

import picinputs as pin
from paper_2411_04703_amd import abi

pytestmark = pytest.mark.gpu

ALL = abi.PIC_DIAG_MOMENTS | abi.PIC_DIAG_BUNCHING | abi.PIC_DIAG_ENERGY | abi.PIC_DIAG_GAUSS


def _cases():
    big = pin.scaled(pin.workload(1), nx=32, ny=32, nz=128, n_beam=65536, sigma=(3, 3, 12))
    small = pin.scaled(pin.workload(1), nx=16, ny=16, nz=64, n_beam=4096, sigma=(2, 2, 8))
    return big, small


GAUSS = ("gauss_max", "rho_max", "gauss_drift")


def _check_pair(s, gross, what):
    """pic_diag, pic_diag_static, pic_diag on one state.  Every value equal bit for bit, except
    the Gauss residual's: each call deposits the charge density anew with FP64 atomics (a
    different summation order each time, in both modes), so there the values agree to 1e-12 of
    the charge density and the drift between calls on one state is that round-off, not zero."""
    d1 = s.diag(ALL)
    d2 = s.diag(ALL, static=True)
    d3 = s.diag(ALL)
    for k in d1:
        if k in GAUSS:
            continue
        assert d2[k] == d1[k], (what, k, d1[k], d2[k])
        assert d3[k] == d2[k], (what, k, d2[k], d3[k])
    rho = max(d1["rho_max"], gross)  # round-off is relative to the gross plasma density too
    for d in (d2, d3):
        assert abs(d["gauss_max"] - d1["gauss_max"]) <= 1e-12 * rho, what
        assert abs(d["rho_max"] - d1["rho_max"]) <= 1e-12 * rho, what
        assert 0.0 <= d["gauss_drift"] <= 1e-12 * rho, what
    assert d1["n_beam"] > 0 and d1["n_plasma"] > 0 and d1["field_energy"] > 0 and d1["gauss_max"] > 0, what


@pytest.mark.parametrize("precision", [0, 1])
def test_static_diag_equals_pic_diag(precision):
    from paper_2411_04703_amd.sim import Sim
    from paper_2411_04703_amd.sim import derive
    for name, w in zip(("big", "small"), _cases()):
        dv = derive(w)
        gross = dv["gamma_R"] * dv["n0_norm"]
        s = Sim(w, pin.beam_normals(w["beam"]["n_macro"], 3), precision=precision,
                **({} if precision else {"max_steps": 64}))
        s.step(4)
        _check_pair(s, gross, (name, precision, 4))
        s.step(3)
        _check_pair(s, gross, (name, precision, 7))
        s.close()


def test_static_diag_rejects_more_partials_than_it_holds():
    from paper_2411_04703_amd.sim import Sim
    w = pin.scaled(pin.workload(1), nx=256, ny=256, nz=704, n_beam=0)  # 3 x 256-cell blocks > 2^19 partials
    w["plasma"]["n0_lab_cm3"] = 0.0
    w["frame"]["window_beta"] = 0.99
    s = Sim(w, pin.beam_normals(0, 0), precision=1)
    with pytest.raises(abi.PicError) as e:
        s.diag(ALL, static=True)
    assert e.value.status == abi.PIC_ERANGE
    d = s.diag(abi.PIC_DIAG_MOMENTS | abi.PIC_DIAG_ENERGY, static=True)  # without the Gauss partials it fits
    assert d == s.diag(abi.PIC_DIAG_MOMENTS | abi.PIC_DIAG_ENERGY)
    s.close()
