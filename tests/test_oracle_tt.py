"""Pins for the oracle's TT-SVD and TT-RBKI against facts other than the oracle.

* Definition 2 / exactness: a noise-free tensor of TT rank <= target is
  reproduced to rounding by TT-SVD and by TT-RBKI.
* Theorem 1 (Oseledets, Thm 4.3): eps_TTSVD ||X|| <= sqrt(sum_k tau_{r_k+1}^2(X<k>)),
  with the tails taken from LAPACK SVDs of the *original* unfoldings.
* Definition 3 lower bound: any rank-r TT obeys ||X - Y||^2 >= max_k tau_{r_k+1}^2(X<k>).
* d = 2: TT-SVD is the truncated SVD (Eckart-Young), checked against numpy's SVD.
* Eq. (12): ||X - Xhat||^2 equals the sum of the per-mode projection residuals.
* Odeco tensor with i^-1 weights: the closed-form TT-SVD error.
* Saturated modes are exact truncated SVDs for any Omega.
* Nestedness / Ky Fan: rho_1 is non-increasing in q and bounded below by the tail.
* Algorithm 1's delta-truncation guarantee ||A - B|| <= eps ||A||.
"""
import math

import numpy as np
import pytest

import synth
from oracle import metrics, ttrbki


def _tails(X, ranks):
    return [metrics.unfolding_tail(X, k, ranks[k - 1] + 1) for k in range(1, X.ndim)]


def _lowrank(dims, r, seed):
    return synth.tt_full_host(synth.tt_cores_random(dims, r, 1.0, seed))


@pytest.mark.parametrize("dims,r", [((3, 4, 5, 6), 2), ((4, 4, 4, 4, 4), 3), ((6, 5, 4), 4)])
def test_exact_low_rank_reproduced(dims, r):
    X = _lowrank(dims, r, 11)
    targets = [r + 1] * (len(dims) - 1)
    for cores in (ttrbki.tt_svd(X, targets), ttrbki.tt_rbki(X, targets, q=2, p=2, seed=3)):
        assert metrics.rel_error(X, cores) <= 1e-12
        assert metrics.left_orthonormality(cores) <= 1e-13


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_theorem1_and_lower_bound(seed):
    rng = np.random.default_rng(seed)
    X = _lowrank((5, 6, 7, 5), 3, seed) + 0.05 * rng.standard_normal((5, 6, 7, 5))
    ranks = [2, 3, 2]
    tails = _tails(X, ranks)
    x2 = float(np.sum(X * X))
    for cores in (ttrbki.tt_svd(X, ranks), ttrbki.tt_rbki(X, ranks, q=1, p=1, seed=seed)):
        e2 = metrics.errors(X, cores)[0]
        assert e2 >= max(tails) * (1 - 1e-12)
    e2_svd = metrics.errors(X, ttrbki.tt_svd(X, ranks))[0]
    assert e2_svd <= sum(tails) * (1 + 1e-12)
    assert e2_svd <= x2


def test_matrix_case_is_eckart_young():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((30, 45))
    for r in (1, 7, 30):
        cores = ttrbki.tt_svd(X, [r])
        sig = np.linalg.svd(X, compute_uv=False)
        assert abs(metrics.errors(X, cores)[0] - np.sum(sig[r:] ** 2)) <= 1e-10 * np.sum(sig ** 2)


def test_tt_svd_tail_identity():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((4, 5, 6, 7))
    ranks = [3, 6, 4]
    cores, tails = ttrbki.tt_svd(X, ranks, diagnostics=True)
    e2 = metrics.errors(X, cores)[0]
    assert abs(e2 - sum(float(np.sum(t)) for t in tails)) <= 1e-12 * float(np.sum(X * X))


@pytest.mark.parametrize("name,dims", [("tt20x4", None), ("tt24x6", (6, 6, 6, 6, 6)), ("tt48x5", (8, 8, 8, 8))])
def test_pythagorean_identity_eq12(name, dims):
    w = synth.workload(name)
    if dims:
        w = synth.scaled_down(w, dims)
    X = synth.build_host(w)
    cores, modes = ttrbki.tt_rbki(X, w.target_ranks(), w.q, w.p, 0, diagnostics=True)
    e2, x2, _ = metrics.errors(X, cores)
    assert abs(sum(m.rho for m in modes) - e2) <= 1e-12 * x2


def test_odeco_closed_form():
    # X0 = sum_{i<=R} i^-1 u_i o v_i o w_i o z_i with orthonormal factors: every unfolding has
    # singular values {1/i}, and TT-SVD at rank r leaves exactly sum_{i>r} i^-2.
    R, r = 12, 5
    w = synth.scaled_down(synth.workload("odeco256x4"), (16, 16, 16, 16), signal_rank=R, noise="none")
    X = synth.build_host(w)
    tot = sum(i ** -2.0 for i in range(1, R + 1))
    want = math.sqrt(sum(i ** -2.0 for i in range(r + 1, R + 1)) / tot)
    assert abs(metrics.rel_error(X, ttrbki.tt_svd(X, [r] * 3)) - want) <= 1e-12
    # w = (q+1)(r+p) = 3*8 = 24 >= 16 = m: every mode is saturated; the Krylov space spans all
    assert abs(metrics.rel_error(X, ttrbki.tt_rbki(X, [r] * 3, q=2, p=3, seed=0)) - want) <= 1e-12
    # regular first mode with a Krylov space that contains the whole rank-12 range
    w2 = synth.scaled_down(synth.workload("odeco256x4"), (40, 40, 40), signal_rank=R, noise="none")
    X2 = synth.build_host(w2)
    cores, modes = ttrbki.tt_rbki(X2, [r, r], q=1, p=9, seed=1, diagnostics=True)
    assert modes[0].kind == "regular"
    assert abs(metrics.rel_error(X2, cores) - want) <= 1e-10


def test_odeco_closed_form_constant_of_256_workload():
    # Stored decimal of sqrt(sum_{i=33}^{50} i^-2 / sum_{i=1}^{50} i^-2) for the 50-term, rank-32 case.
    with open(__file__.replace("test_oracle_tt.py", "golden/odeco_r32_R50.txt")) as f:
        stored = float(f.read().split()[0])
    val = math.sqrt(sum(i ** -2.0 for i in range(33, 51)) / sum(i ** -2.0 for i in range(1, 51)))
    assert abs(val - stored) < 5e-11


def test_saturated_modes_equal_tt_svd_for_any_seed():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((6, 7, 8, 5))
    ranks = [3, 4, 3]
    ref = ttrbki.tt_svd(X, ranks)
    for seed in (0, 1, 99):
        cores, modes = ttrbki.tt_rbki(X, ranks, q=3, p=4, seed=seed, diagnostics=True)
        assert all(m.kind != "regular" for m in modes)
        x2 = float(np.sum(X * X))
        assert metrics.rec_diff_sq(ref, cores) <= 1e-24 * x2 * 1e4


def test_krylov_depth_monotone_and_ky_fan():
    w = synth.scaled_down(synth.workload("tt48x5"), (30, 30, 30), signal_rank=8)
    X = synth.build_host(w)
    A1 = X.reshape(30, -1)
    sig = np.linalg.svd(A1, compute_uv=False)
    r = 6
    prev = None
    for q in range(0, 4):
        _, modes = ttrbki.tt_rbki(X, [r, r], q=q, p=1, seed=2, diagnostics=True)
        rho = modes[0].rho
        assert modes[0].kind == "regular"
        assert rho >= float(np.sum(sig[r:] ** 2)) * (1 - 1e-12)
        if prev is not None:
            assert rho <= prev * (1 + 1e-10)
        prev = rho


def test_delta_truncated_tt_svd_guarantee():
    rng = np.random.default_rng(3)
    X = _lowrank((6, 6, 6, 6), 3, 8) + 1e-2 * rng.standard_normal((6, 6, 6, 6))
    for eps in (0.5, 0.1, 0.02, 1e-3):
        cores = ttrbki.tt_svd_delta(X, eps)
        assert metrics.rel_error(X, cores) <= eps * (1 + 1e-12)
    # a loose tolerance recovers the signal rank
    cores = ttrbki.tt_svd_delta(X, 0.05)
    assert [c.shape[2] for c in cores[:-1]] == [3, 3, 3]


def test_zero_tensor_and_completion():
    X = np.zeros((4, 5, 6))
    cores = ttrbki.tt_rbki(X, [3, 3], q=1, p=1, seed=0)
    assert metrics.left_orthonormality(cores) <= 1e-15
    assert metrics.errors(X, cores)[0] == 0.0
    G = ttrbki.complete_columns(np.zeros((7, 0)), 7, 4)
    np.testing.assert_allclose(G.T @ G, np.eye(4), atol=1e-15)


def test_rank_clamping_plan():
    modes = ttrbki.plan_modes([8] * 10, [16] * 9, q=2, p=8)
    kinds = [m.kind for m in modes]
    assert modes[0].r == 8 and kinds[0] == "identity"
    assert modes[-1].r == 8
    assert [m.m for m in modes[:3]] == [8, 64, 128]
    assert kinds[1] == "saturated" and kinds[2] == "regular"


def test_noisy_ordering_rbki_vs_sketch_only():
    # Section 4: on noisy data the Krylov variant is at least as accurate as the q = 0 sketch
    w = synth.scaled_down(synth.workload("tt48x5"), (16, 16, 16, 16), signal_rank=6, eta=0.3)
    X = synth.build_host(w)
    e_svd = metrics.rel_error(X, ttrbki.tt_svd(X, [6] * 3))
    e0 = metrics.rel_error(X, ttrbki.tt_rbki(X, [6] * 3, q=0, p=2, seed=0))
    e3 = metrics.rel_error(X, ttrbki.tt_rbki(X, [6] * 3, q=3, p=2, seed=0))
    assert e_svd <= e3 * (1 + 1e-9)
    assert e3 <= e0 * (1 + 1e-9)
    assert e3 <= 1.02 * e_svd


def test_metrics_against_dense():
    rng = np.random.default_rng(2)
    a = synth.tt_cores_random((3, 4, 5), 2, 1.0, 1)
    b = synth.tt_cores_random((3, 4, 5), 2, 1.0, 2)
    A, B = metrics.tt_full(a), metrics.tt_full(b)
    assert abs(metrics.tt_inner(a, b) - float(np.sum(A * B))) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(B)
    assert abs(metrics.rec_diff_sq(a, b) - float(np.sum((A - B) ** 2))) <= 1e-12 * float(np.sum(A * A + B * B))
    X = A + 0.1 * rng.standard_normal(A.shape)
    e2, x2, xinf = metrics.errors(X, a)
    assert abs(e2 - np.sum((X - A) ** 2)) <= 1e-12 * x2
    assert xinf == np.max(np.abs(A))
    # a gauge change between cores leaves the interface subspaces and the tensor unchanged
    X = rng.standard_normal((4, 5, 6))
    cores = ttrbki.tt_svd(X, [3, 4])
    Rm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    g = [cores[0] @ Rm, np.einsum("ab,bic->aic", Rm.T, cores[1]), cores[2]]
    assert max(metrics.interface_sines(cores, g)) <= 1e-7
    assert metrics.rec_diff_sq(cores, g) <= 1e-24 * 1e4


def test_orth_tau_rank_revealing():
    rng = np.random.default_rng(12)
    # exact rank 4 inside 10 columns: four directions survive, spanning range(P)
    B = rng.standard_normal((50, 4)) @ rng.standard_normal((4, 10))
    Q = ttrbki.orth_tau(B, float(np.linalg.norm(B)), 1e-10)
    assert Q.shape[1] == 4
    np.testing.assert_allclose(Q.T @ Q, np.eye(4), atol=1e-14)
    assert np.linalg.norm(B - Q @ (Q.T @ B)) <= 1e-13 * np.linalg.norm(B)
    # well-separated spectrum: the kept span equals the dominant left singular subspace
    U0, _ = np.linalg.qr(rng.standard_normal((60, 8)))
    V0, _ = np.linalg.qr(rng.standard_normal((8, 8)))
    sig = np.array([1, 0.9, 0.8, 0.7, 1e-7, 1e-8, 1e-9, 1e-10])
    P = U0 @ np.diag(sig) @ V0.T
    Q = ttrbki.orth_tau(P, 1.0, 1e-5)
    assert Q.shape[1] == 4
    c = np.linalg.svd(Q.T @ U0[:, :4], compute_uv=False)
    assert np.min(c) >= 1 - 1e-9
    assert ttrbki.orth_tau(np.zeros((5, 3)), 0.0, 1e-10).shape[1] == 0


@pytest.mark.parametrize("name,dims,chg", [("odeco256x4", (96, 24, 20, 10), {"signal_rank": 8, "ranks": 6}),
                                           ("tt48x5", (16, 16, 16, 16), {}), ("tt20x4", None, {})])
def test_gram_first_products_equal_streamed(name, dims, chg):
    # A (A^T Z) = (A A^T) Z and B B^T = Q^T (A A^T) Q by associativity: the Gram-first form of
    # the Krylov products gives the same approximation to rounding
    w = synth.workload(name)
    if dims:
        w = synth.scaled_down(w, dims, **chg)
    X = synth.build_host(w)
    a, ma = ttrbki.tt_rbki(X, w.target_ranks(), w.q, w.p, 0, diagnostics=True)
    b, mb = ttrbki.tt_rbki(X, w.target_ranks(), w.q, w.p, 0, diagnostics=True, gram_first=True)
    assert any(m.kind == "regular" for m in ma)
    x2 = float(np.sum(X * X))
    assert abs(metrics.rel_error(X, a) - metrics.rel_error(X, b)) <= 1e-12
    assert metrics.rec_diff_sq(a, b) <= 1e-22 * x2
    assert [m.kept for m in ma] == [m.kept for m in mb]
