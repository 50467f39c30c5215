"""Pins for the oracle's TT-rSVD (Algorithm 2), TT-rSI (Algorithm 4) and TT-rBKI as printed
(Algorithm 3 with the row-space Krylov matrix), against what the mathematics fixes:

* first-r-columns truncation of an unpivoted QR keeps the span of the first r columns of
  its argument (QR is triangular), so the printed forms reduce to spans of r-column blocks:
    Algorithm 2:  span G_1 = span(A Omega_r),
    Algorithm 3:  span G_1 = span((A A^T) A Omega_r)       (any q >= 1, any p),
    Algorithm 4:  span G_1 = span((A A^T)^q A Omega_r)     (any p),
  with Omega_r the first r columns of Omega (whose columns do not depend on s);
* Rayleigh-Ritz over nested spaces: span(A Omega) and span((A A^T)^q A Omega) lie in the
  block Krylov space, so the first mode's residual of the column-space TT-RBKI is at most
  that of the Rayleigh-Ritz forms of Algorithms 2 and 4 (same Omega), and every residual is
  at least the Ky Fan tail sum_{i>r} sigma_i^2;
* noise-free tensors of TT rank <= r are reproduced exactly by every form.
"""
import numpy as np
import pytest

import synth
from oracle import metrics, ttrbki
from oracle.philox import omega


def _noisy(dims, r, eta, seed):
    w = synth.scaled_down(synth.workload("tt48x5"), dims, signal_rank=r, eta=eta, core_seed=seed, noise_seed=seed + 1)
    return synth.build_host(w)


def _span_residual(G, V):
    """||(I - G G^T) V|| / ||V|| for orthonormal G."""
    return float(np.linalg.norm(V - G @ (G.T @ V)) / np.linalg.norm(V))


def _first_core(cores):
    return cores[0].reshape(-1, cores[0].shape[2])


def _orth(V):
    return np.linalg.qr(V)[0]


X = _noisy((12, 10, 9, 8), 3, 0.2, 31)
A1 = X.reshape(12, -1)
R = 4


def test_rsvd_printed_spans_first_sketch_columns():
    c = ttrbki.tt_variant(X, [R] * 3, 0, 5, seed=2, method="rsvd", truncation="first")
    G = _first_core(c)
    Om = omega(2, 1, 0, A1.shape[1], R)
    assert _span_residual(G, A1 @ Om) <= 1e-12
    assert metrics.left_orthonormality(c) <= 1e-14
    # the oversampling columns are discarded: p does not change the result
    c0 = ttrbki.tt_variant(X, [R] * 3, 0, 0, seed=2, method="rsvd", truncation="first")
    assert metrics.rec_diff_sq(c, c0) <= 1e-24 * float(np.sum(X * X))


def test_rbki_printed_is_one_power_step_of_r_columns():
    c = ttrbki.tt_variant(X, [R] * 3, 3, 4, seed=5, method="rbki", truncation="first")
    G = _first_core(c)
    Om = omega(5, 1, 0, A1.shape[1], R)
    assert _span_residual(G, A1 @ (A1.T @ (A1 @ Om))) <= 1e-11
    # neither q >= 1 nor p changes the printed result
    c1 = ttrbki.tt_variant(X, [R] * 3, 1, 0, seed=5, method="rbki", truncation="first")
    assert metrics.rec_diff_sq(c, c1) <= 1e-20 * float(np.sum(X * X))
    with pytest.raises(ValueError):
        ttrbki.tt_variant(X, [R] * 3, 0, 4, seed=5, method="rbki", truncation="first")


@pytest.mark.parametrize("q", [1, 3])
def test_rsi_printed_is_power_iteration_of_r_columns(q):
    c = ttrbki.tt_variant(X, [R] * 3, q, 6, seed=7, method="rsi", truncation="first")
    G = _first_core(c)
    V = _orth(A1 @ omega(7, 1, 0, A1.shape[1], R))
    for _ in range(q):
        V = _orth(A1 @ (A1.T @ V))
    assert _span_residual(G, V) <= 1e-11
    c0 = ttrbki.tt_variant(X, [R] * 3, q, 0, seed=7, method="rsi", truncation="first")
    assert metrics.rec_diff_sq(c, c0) <= 1e-20 * float(np.sum(X * X))


def _rho1(cores):
    G = _first_core(cores)
    return float(np.sum((A1 - G @ (G.T @ A1)) ** 2))


def test_ritz_forms_nested_and_ky_fan():
    q, p, seed = 2, 3, 11
    sig = np.linalg.svd(A1, compute_uv=False)
    tail = float(np.sum(sig[R:] ** 2))
    rbki = _rho1(ttrbki.tt_rbki(X, [R] * 3, q, p, seed=seed))
    rsi = _rho1(ttrbki.tt_variant(X, [R] * 3, q, p, seed=seed, method="rsi", truncation="ritz"))
    rsvd = _rho1(ttrbki.tt_variant(X, [R] * 3, q, p, seed=seed, method="rsvd", truncation="ritz"))
    assert rbki <= rsi * (1 + 1e-12) and rbki <= rsvd * (1 + 1e-12)
    for rho in (rbki, rsi, rsvd):
        assert rho >= tail * (1 - 1e-12)
    # the printed truncations are no better than the Ritz forms built on the same Omega
    assert _rho1(ttrbki.tt_variant(X, [R] * 3, q, p, seed=seed, method="rsvd", truncation="first")) >= rsvd * (1 - 1e-12)


@pytest.mark.parametrize("method,truncation", [("rsvd", "first"), ("rsvd", "ritz"), ("rbki", "first"),
                                               ("rsi", "first"), ("rsi", "ritz")])
def test_variants_reproduce_low_rank_exactly(method, truncation):
    Z = synth.tt_full_host(synth.tt_cores_random((7, 8, 9, 6), 3, 1.0, 4))
    c = ttrbki.tt_variant(Z, [3, 3, 3], 2, 2, seed=1, method=method, truncation=truncation)
    assert metrics.rel_error(Z, c) <= 1e-12
    assert metrics.left_orthonormality(c) <= 1e-13
