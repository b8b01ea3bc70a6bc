"""pic_init draws the beam's standard normals on the device from a seed when pic_beam.normals is
NULL.  The beam it starts from equals the beam started from the oracle's draws of the same seed
(oracle/rng.py, written separately from the published generator definitions) to FP64 rounding of
the transcendental functions in both precisions, and the draws depend on the seed alone."""
import numpy as np
import pytest

import picinputs as pin
from oracle import rng

pytestmark = pytest.mark.gpu

SEED = 0x0123456789ABCDEF
KEYS = ("x", "y", "z", "ux", "uy", "uz", "w")


def _pair(precision, seed=SEED):
    from paper_2411_04703_amd.sim import Sim
    w = pin.workload(0)
    n = w["beam"]["n_macro"]
    a = Sim(w, None, precision=precision, seed=seed)
    b = Sim(w, rng.beam_normals_from_seed(n, seed), precision=precision)
    return a, b


def test_fp64_seeded_beam_equals_the_oracle_draws():
    a, b = _pair(0)
    pa, pb = a.particles(0), b.particles(0)
    assert np.array_equal(pa["alive"], pb["alive"])
    for k in KEYS:
        np.testing.assert_allclose(pa[k], pb[k], rtol=1e-13, atol=1e-13, err_msg=k)
    da, db = a.diag(), b.diag()
    for k in ("mean", "sigma", "usigma", "emit"):
        np.testing.assert_allclose(da[k], db[k], rtol=1e-12, err_msg=k)


def test_fp32_seeded_beam_equals_the_oracle_draws():
    """FP32 split storage rounds each coordinate once from the FP64 beam: at most one FP32 ulp
    apart (a draw an FP64 ulp away from a rounding tie); the same particles start inside the
    band (the window's 64 planes leave a few of the 3-sigma tail outside); the moments to 1e-9."""
    a, b = _pair(1)
    pa, pb = a.particles(0), b.particles(0)
    assert (pa["alive"] == 1).sum() == (pb["alive"] == 1).sum() > 0.99 * pin.workload(0)["beam"]["n_macro"]
    for k in KEYS:
        xa, xb = np.sort(pa[k][pa["alive"] == 1]), np.sort(pb[k][pb["alive"] == 1])
        np.testing.assert_allclose(xa, xb, rtol=2.0 ** -22, atol=2.0 ** -24, err_msg=k)
    da, db = a.diag(), b.diag()
    for k in ("mean", "sigma", "usigma", "emit"):
        np.testing.assert_allclose(da[k], db[k], rtol=1e-9, err_msg=k)


def test_seeded_draws_depend_on_the_seed_alone():
    from paper_2411_04703_amd.sim import Sim
    w = pin.workload(0)
    a = Sim(w, None, precision=0, seed=SEED).particles(0)
    b = Sim(w, None, precision=0, seed=SEED).particles(0)
    c = Sim(w, None, precision=0, seed=SEED + 1).particles(0)
    for k in KEYS[:6]:
        assert np.array_equal(a[k], b[k]), k
        assert not np.array_equal(a[k], c[k]), k
