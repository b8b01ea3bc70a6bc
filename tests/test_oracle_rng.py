"""The oracle's seeded beam draws (oracle/rng.py): Philox4x32-10 pinned by the generator's published
known-answer vectors, the Box-Muller normals by what the mathematics fixes (moments, the normal
distribution's quantiles and tails, independence of the six rows), and the counter layout by the
prefix property (a particle's draws do not depend on how many particles there are)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import rng

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answer_vectors():
    kat = json.load(open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        out = rng.philox4x32_10([int(x, 16) for x in v["counter"]], [int(x, 16) for x in v["key"]])
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]], v


def test_philox_vectorised_equals_one_counter_at_a_time():
    ctr = [np.array([0, 1, 0xFFFFFFFF], dtype=np.uint64), np.array([5, 0, 7], dtype=np.uint64),
           np.array([1, 1, 1], dtype=np.uint64), np.array([0, 9, 0], dtype=np.uint64)]
    key = (0x12345678, 0x9ABCDEF0)
    many = rng.philox4x32_10(ctr, key)
    for i in range(3):
        one = rng.philox4x32_10([int(c[i]) for c in ctr], key)
        assert [int(w[i]) for w in many] == [int(x) for x in one]


N = 1 << 20


@pytest.fixture(scope="module")
def draws():
    return rng.beam_normals_from_seed(N, 12345)


def test_normals_moments_and_quantiles(draws):
    """Each row: mean 0 and variance 1 within five standard errors, Kolmogorov-Smirnov against
    the standard normal, and the two-sided 3-sigma tail (0.27 %)."""
    se = 1.0 / math.sqrt(N)
    for r in range(6):
        x = draws[r]
        assert abs(x.mean()) < 5 * se, r
        assert abs(x.var() - 1.0) < 5 * math.sqrt(2.0) * se, r
        assert stats.kstest(x, "norm").pvalue > 1e-4, r
        tail = np.mean(np.abs(x) > 3.0)
        assert abs(tail - 2 * stats.norm.sf(3.0)) < 5 * math.sqrt(2 * stats.norm.sf(3.0) / N), r


def test_rows_are_uncorrelated(draws):
    c = np.corrcoef(draws)
    off = c[~np.eye(6, dtype=bool)]
    assert np.max(np.abs(off)) < 5.0 / math.sqrt(N)
    # the two normals of one Box-Muller pair are independent: their squares too
    for r in (0, 2, 4):
        assert abs(np.corrcoef(draws[r] ** 2, draws[r + 1] ** 2)[0, 1]) < 5.0 / math.sqrt(N)


def test_prefix_property_and_seed_dependence():
    a = rng.beam_normals_from_seed(1000, 7)
    b = rng.beam_normals_from_seed(100, 7)
    assert np.array_equal(a[:, :100], b)
    c = rng.beam_normals_from_seed(100, 8)
    assert not np.any(c == b)
    # the key's high word matters too
    d = rng.beam_normals_from_seed(100, 7 + (1 << 32))
    assert not np.any(d == b)
