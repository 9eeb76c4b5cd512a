"""Pins for the oracle's Philox4x64-10 and Gaussian transform (CPU only)."""
import math

import numpy as np
import pytest

from oracle import normal, philox

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_philox_matches_numpy_independent_implementation():
    # numpy ships its own Philox4x64-10; it increments the counter before each
    # block, so its block for state counter c is the bijection of c + 1.
    gen = np.random.default_rng(123)
    for _ in range(20):
        key = gen.integers(0, 2**63, size=2, dtype=np.uint64) * np.uint64(2) + gen.integers(0, 2, size=2, dtype=np.uint64)
        c0 = int(gen.integers(0, 2**62))
        ref = np.random.Philox(key=key, counter=[c0, 7, 9, 11]).random_raw(8)
        ctr = np.array([[c0 + 1, 7, 9, 11], [c0 + 2, 7, 9, 11]], dtype=np.uint64)
        got = philox.philox4x64_10(ctr, key).reshape(-1)
        assert np.array_equal(got, ref)


def test_philox_known_answer_zero():
    # Known-answer vector of the Random123 distribution (counter 0, key 0),
    # re-derived through numpy's implementation (counter wraps from 2^64 - 1).
    ref = np.random.Philox(key=[0, 0], counter=[2**64 - 1] * 4).random_raw(4)
    got = philox.philox4x64_10(np.zeros((1, 4), dtype=np.uint64), np.zeros(2, dtype=np.uint64))[0]
    assert np.array_equal(got, ref)
    assert int(got[0]) == 0x16554D9ECA36314C


def test_mulhilo_against_python_ints():
    gen = np.random.default_rng(5)
    a = gen.integers(0, 2**64 - 1, size=1000, dtype=np.uint64, endpoint=True)
    b = gen.integers(0, 2**64 - 1, size=1000, dtype=np.uint64, endpoint=True)
    hi, lo = philox.mulhilo64(a, b)
    for x, y, h, l in zip(a[:200], b[:200], hi[:200], lo[:200]):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2**64 - 1)


def test_uniform_is_exact_and_open_interval():
    w = np.array([0, 1, 2**12 - 1, 2**12, 2**64 - 1], dtype=np.uint64)
    u = normal.uniform_from_words(w)
    assert u[0] == 2.0**-53 and u[2] == 2.0**-53
    assert u[3] == 2.0**-52 + 2.0**-53
    assert u[4] == 1.0 - 2.0**-53
    assert np.all((u > 0) & (u < 1))


def test_own_log_accuracy():
    gen = np.random.default_rng(7)
    u = np.concatenate([gen.random(100000), [2.0**-53, 0.5, 1 - 2.0**-53, 0.7071067811865476, 1.0]])
    u = u[u > 0]
    got = normal.own_log(u)
    ref = np.array([math.log(x) for x in u])
    ulps = np.abs(got - ref) / np.spacing(np.maximum(np.abs(ref), 1e-300))
    assert ulps.max() <= 4
    assert normal.own_log(np.array([1.0]))[0] == 0.0


def test_own_sincos_accuracy_and_symmetry():
    gen = np.random.default_rng(8)
    w = gen.integers(0, 2**64 - 1, size=100000, dtype=np.uint64, endpoint=True)
    u = normal.uniform_from_words(w)
    s, c = normal.own_sincos_2pi(w)
    # reference in extended precision via angle reduction on exact dyadics
    t = np.array([math.fmod(4 * x, 1.0) for x in u[:2000]])
    ref_s = np.array([math.sin(2 * math.pi * x) for x in u[:2000]])
    ref_c = np.array([math.cos(2 * math.pi * x) for x in u[:2000]])
    assert np.abs(s[:2000] - ref_s).max() < 2e-15
    assert np.abs(c[:2000] - ref_c).max() < 2e-15
    assert np.abs(s * s + c * c - 1).max() < 4e-16 * 8
    assert t.size == 2000
    # quarter-turn points are exact: u = 1/4 -> (1, 0)
    w_q = np.array([(1 << 62) - (1 << 11)], dtype=np.uint64)  # (w>>12) * 2^-52 + 2^-53 just below 1/4
    s_q, c_q = normal.own_sincos_2pi(w_q)
    assert abs(s_q[0] - 1.0) < 1e-15 and abs(c_q[0]) < 1e-15


def test_gaussian_moments_and_normality():
    from scipy import stats
    z = normal.gaussian_matrix(11, 200000, 1).ravel()
    assert abs(z.mean()) < 0.01
    assert abs(z.std() - 1) < 0.01
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the two members of a Box-Muller pair are uncorrelated
    blk = normal.normals_from_block(philox.block_words(3, 0, np.arange(50000, dtype=np.uint64)))
    assert abs(np.corrcoef(blk[:, 0], blk[:, 1])[0, 1]) < 0.02
    assert abs(np.corrcoef(blk[:, 1], blk[:, 2])[0, 1]) < 0.02


def test_gaussian_nesting_and_layout():
    a = normal.gaussian_matrix(1, 37, 5)
    b = normal.gaussian_matrix(1, 37, 9)
    assert np.array_equal(a, b[:, :5])
    flat = normal.gaussian_matrix(1, 37 * 9, 1).ravel()
    assert np.array_equal(b.T.reshape(-1), flat)  # column-major numbering
    # different streams and seeds differ
    assert not np.array_equal(normal.gaussian_matrix(1, 37, 5, stream=1), a)
    assert not np.array_equal(normal.gaussian_matrix(2, 37, 5), a)
    assert normal.gaussian_matrix(1, 0, 3).shape == (0, 3)
