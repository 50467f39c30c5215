"""Pins for the reference gradient of f(X) = ||X - TT_r(X)||^2 (Omega fixed):
central finite differences of the float64 oracle sweep itself (an independent code path:
numpy + LAPACK, no autodiff), the d = 2 Eckart-Young envelope grad f = 2 (X - Xhat), and
grad f = 0 at a noise-free tensor of TT rank below the target."""
import math

import numpy as np
import pytest

import synth
from oracle import grad, metrics, ttrbki


def _f(X, ranks, q, p, seed=0):
    cores = ttrbki.tt_rbki(X, ranks, q, p, seed=seed)
    return metrics.errors(X, cores)[0]


def test_loss_matches_oracle_sweep():
    w = synth.workload("tt20x4")
    X = synth.build_host(w)
    f, _ = grad.loss_and_grad(X, w.target_ranks(), w.q, w.p)
    assert abs(f - _f(X, w.target_ranks(), w.q, w.p)) <= 1e-10 * float(np.sum(X * X))


@pytest.mark.parametrize("case", ["tt20x4", "small5"])
def test_directional_finite_differences(case):
    if case == "tt20x4":
        w = synth.workload("tt20x4")
        X, ranks, q, p = synth.build_host(w), w.target_ranks(), w.q, w.p
    else:
        rng = np.random.default_rng(3)
        X = synth.tt_full_host(synth.tt_cores_random((5, 6, 7, 6), 3, 1.0, 5)) + 0.3 * rng.standard_normal((5, 6, 7, 6))
        ranks, q, p = [2, 3, 2], 1, 1
    _, g = grad.loss_and_grad(X, ranks, q, p)
    rng = np.random.default_rng(11)
    rms = math.sqrt(float(np.mean(X * X)))
    for _ in range(3):
        D = rng.standard_normal(X.shape)
        D /= np.linalg.norm(D)
        h = 1e-5 * rms * math.sqrt(X.size)
        fd = (_f(X + h * D, ranks, q, p) - _f(X - h * D, ranks, q, p)) / (2 * h)
        an = float(np.sum(g * D))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) * 10, (fd, an)


def test_coordinate_finite_differences():
    w = synth.workload("tt20x4")
    X = synth.build_host(w)
    _, g = grad.loss_and_grad(X, w.target_ranks(), w.q, w.p)
    rng = np.random.default_rng(2)
    idx = [tuple(rng.integers(0, 20, size=4)) for _ in range(12)]
    h = 1e-5
    for ix in idx:
        Xp, Xm = X.copy(), X.copy()
        Xp[ix] += h
        Xm[ix] -= h
        fd = (_f(Xp, w.target_ranks(), w.q, w.p) - _f(Xm, w.target_ranks(), w.q, w.p)) / (2 * h)
        assert abs(fd - g[ix]) <= 1e-6 * max(1.0, abs(g[ix])) + 1e-8, (ix, fd, g[ix])


def test_matrix_case_envelope():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((12, 30))
    _, g = grad.loss_and_grad(X, [4], 2, 3)
    cores = ttrbki.tt_rbki(X, [4], 2, 3)
    Xh = metrics.tt_full(cores)
    np.testing.assert_allclose(g, 2 * (X - Xh), atol=1e-10)


def test_zero_gradient_at_exact_low_rank():
    X = synth.tt_full_host(synth.tt_cores_random((6, 7, 8, 5), 2, 1.0, 9))
    f, g = grad.loss_and_grad(X, [3, 3, 3], 1, 2)
    # f = ||X||^2 - ||C||^2 cancels to rounding of ||X||^2
    assert abs(f) <= 1e-13 * float(np.sum(X * X))
    assert np.max(np.abs(g)) <= 1e-8 * math.sqrt(float(np.mean(X * X)))
