"""Pins for the oracle's Gaussian test matrix (Algorithm 3, step 3).

The Philox4x64-10 rounds are pinned against numpy's own, independently
written Philox4x64-10 bit generator (numpy.random.Philox), which increments
its 256-bit counter before every block of four outputs.  The float32
logarithm and cosine / sine of the Box-Muller transform are pinned against
numpy's float64 log, cos and sin (error bounds of a few float32 ulps over dense
grids, the quadrant boundaries and the ends of the uniform range).  The Gaussian
output is pinned by distributional tests (moments, Kolmogorov-Smirnov against
the standard normal CDF) and by the Box-Muller radius identity.
"""
import numpy as np
import pytest
from scipy import stats

from oracle.philox import philox4x64_10, omega

MASK = (1 << 64) - 1


def _numpy_block(ctr, key):
    c = list(ctr)
    # numpy's generator pre-increments the 256-bit counter: start one below.
    for i in range(4):
        c[i] = (c[i] - 1) & MASK
        if c[i] != MASK:
            break
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("trial", range(8))
def test_philox_matches_numpy_philox(trial):
    rng = np.random.default_rng(100 + trial)
    for _ in range(25):
        ctr = [int(v) for v in rng.integers(0, 2 ** 64, size=4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2 ** 64, size=2, dtype=np.uint64)]
        mine = philox4x64_10(*[np.uint64(c) for c in ctr], np.uint64(key[0]), np.uint64(key[1]))
        assert [int(v) for v in mine] == _numpy_block(ctr, key)


def test_philox_edge_counters_match_numpy():
    for ctr, key in [((0, 0, 0, 0), (0, 0)), ((MASK, MASK, MASK, MASK), (MASK, MASK)),
                     ((0, 1, 0, 0), (7, 0)), ((5, 0, 0, 1), (0, 9))]:
        mine = philox4x64_10(*[np.uint64(c) for c in ctr], np.uint64(key[0]), np.uint64(key[1]))
        assert [int(v) for v in mine] == _numpy_block(list(ctr), key)


def test_philox_vectorised_equals_scalar():
    beta = np.arange(17, dtype=np.uint64)
    g = np.uint64(3)
    v = philox4x64_10(beta, g, np.uint64(0), np.uint64(0), np.uint64(42), np.uint64(2))
    for i in range(17):
        s = philox4x64_10(np.uint64(i), g, np.uint64(0), np.uint64(0), np.uint64(42), np.uint64(2))
        assert all(int(a[i]) == int(b) for a, b in zip(v, s))


def test_omega_is_standard_normal():
    z = omega(0, 1, 0, 50000, 8).ravel()
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.02
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # columns are uncorrelated
    c = np.corrcoef(omega(0, 2, 0, 20000, 6), rowvar=False)
    assert np.max(np.abs(c - np.eye(6))) < 0.05


def test_omega_box_muller_radius_identity():
    # entries 8g + 2j, 8g + 2j + 1 share the radius sqrt(-2 ln u), u from the low half of
    # word j: their squares sum to -2 ln u (up to float32 rounding)
    from oracle.philox import philox4x64_10 as ph
    w = omega(5, 3, 100, 140, 16)
    words = ph(np.arange(100, 140, dtype=np.uint64)[:, None], np.arange(2, dtype=np.uint64)[None, :],
               np.zeros((1, 1), np.uint64), np.zeros((1, 1), np.uint64), np.uint64(5), np.uint64(3))
    for j, x in enumerate(words):
        u = (((x & np.uint64(0xFFFFFFFF)) >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23
        np.testing.assert_allclose(w[:, 2 * j::8] ** 2 + w[:, 2 * j + 1::8] ** 2, -2 * np.log(u), rtol=2e-6)


def test_ln32_against_numpy_log():
    from oracle.philox import ln32
    grid = np.concatenate([
        (np.arange(0, 2 ** 23, 97, dtype=np.float64) + 0.5) * 2.0 ** -23,            # the uniforms' lattice
        np.array([2.0 ** -24, 1 - 2.0 ** -24, 0.5, 0.5 + 2.0 ** -24, 2 ** -0.5, 2 ** -0.5 + 1e-7, 0.25, 1e-6]),
    ]).astype(np.float32)
    ref = np.log(grid.astype(np.float64))
    err = np.abs(ln32(grid).astype(np.float64) - ref) / np.maximum(np.abs(ref), 1e-30)
    assert np.max(err) <= 4e-7
    assert ln32(np.float32(0.5)) == np.float32(-0.6931471824645996)   # e ln2 with ln f = 0 exactly


def test_cossin32_against_numpy():
    from oracle.philox import cossin32
    v = np.concatenate([(np.arange(0, 2 ** 23, 89, dtype=np.float64) + 0.5) * 2.0 ** -23,
                        np.array([0.0, 0.25, 0.5, 0.75, 0.25 - 2.0 ** -24, 0.5 - 2.0 ** -24, 1 - 2.0 ** -24])]).astype(np.float32)
    c, s = cossin32(v)
    th = 2 * np.pi * v.astype(np.float64)
    assert np.max(np.abs(c - np.cos(th))) <= 4e-7
    assert np.max(np.abs(s - np.sin(th))) <= 4e-7
    # quadrant ends land on the axes
    c4, s4 = cossin32(np.array([0.0, 0.25, 0.5, 0.75], dtype=np.float32))
    np.testing.assert_array_equal(c4, np.array([1, 0, -1, 0], dtype=np.float32))
    np.testing.assert_array_equal(s4, np.array([0, 1, 0, -1], dtype=np.float32))


def test_omega_values_are_float32():
    w = omega(11, 4, 0, 500, 19)
    np.testing.assert_array_equal(w, w.astype(np.float32).astype(np.float64))


def test_omega_rows_and_streams():
    full = omega(7, 2, 0, 300, 10)
    np.testing.assert_array_equal(full[120:170], omega(7, 2, 120, 170, 10))
    np.testing.assert_array_equal(full[:, :7], omega(7, 2, 0, 300, 7))
    assert not np.allclose(full, omega(7, 3, 0, 300, 10))
    assert not np.allclose(full, omega(8, 2, 0, 300, 10))
