"""Error metrics and TT utilities for the oracle (float64, CPU).

* relative error  eps = ||A - Ahat||_F / ||A||_F   (Section 4)
* PSNR = 10 log10( numel * ||Ahat||_inf^2 / ||A - Ahat||_F^2 )  (Section 4,
  written for third-order tensors there; numel replaces I1 I2 I3)
* tail energy tau_j^2(X) = sum_{i >= j} sigma_i^2(X)  (Definition 3)
* TT reconstruction (Definition 2: contraction of consecutive cores over the
  shared rank index), streamed over the first index so that only one slab of
  the dense tensor exists at a time.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np


def tt_full(cores: Sequence[np.ndarray]) -> np.ndarray:
    cur = cores[0].reshape(cores[0].shape[1], cores[0].shape[2])
    for c in cores[1:]:
        cur = (cur @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
    return cur.reshape([c.shape[1] for c in cores])


def _slabs(cores: Sequence[np.ndarray], max_rows: int = 1 << 22):
    """Yield (i0, i1, dense slab of rows i0..i1-1 of the first index)."""
    I1 = cores[0].shape[1]
    rest = int(np.prod([c.shape[1] for c in cores[1:]], dtype=np.int64))
    step = max(1, max_rows // max(rest, 1))
    # right interface (r1 x rest) is formed once when it is small enough, else per slab
    for i0 in range(0, I1, step):
        i1 = min(I1, i0 + step)
        cur = cores[0][0, i0:i1, :]
        for c in cores[1:]:
            cur = (cur @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
        yield i0, i1, cur.reshape(i1 - i0, rest)


def errors(X: np.ndarray, cores: Sequence[np.ndarray]):
    """(||X - Xhat||_F^2, ||X||_F^2, ||Xhat||_inf), streaming over the first index."""
    Xm = X.reshape(X.shape[0], -1)
    e2 = x2 = 0.0
    xinf = 0.0
    for i0, i1, slab in _slabs(cores):
        xs = Xm[i0:i1].astype(np.float64)
        d = xs - slab
        e2 += float(np.sum(d * d))
        x2 += float(np.sum(xs * xs))
        xinf = max(xinf, float(np.max(np.abs(slab))) if slab.size else 0.0)
    return e2, x2, xinf


def rel_error(X: np.ndarray, cores: Sequence[np.ndarray]) -> float:
    e2, x2, _ = errors(X, cores)
    return math.sqrt(e2 / x2) if x2 > 0 else math.sqrt(e2)


def psnr(X: np.ndarray, cores: Sequence[np.ndarray]) -> float:
    e2, _, xinf = errors(X, cores)
    return 10.0 * math.log10(X.size * xinf * xinf / e2)


def rec_diff_sq(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> float:
    """||TT(a) - TT(b)||_F^2 computed entrywise (no cancellation-prone inner products)."""
    tot = 0.0
    for (i0, i1, sa), (_, _, sb) in zip(_slabs(a), _slabs(b)):
        d = sa - sb
        tot += float(np.sum(d * d))
    return tot


def tt_inner(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> float:
    """<TT(a), TT(b)> by the left-to-right contraction of core pairs."""
    W = np.ones((1, 1))
    for ca, cb in zip(a, b):
        # W_k[alpha, beta] = sum_{a,b,i} W[a,b] ca[a,i,alpha] cb[b,i,beta]
        T = np.einsum("ab,aix->bix", W, ca)
        W = np.einsum("bix,biy->xy", T, cb)
    return float(W[0, 0])


def interface_sines(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> List[float]:
    """sin of the largest principal angle between the left interface subspaces, per bond.

    For left-orthonormal cores the interface U_{<=k} (I_1..I_k x r_k, the chain
    G_1 x G_2 x ... x G_k of Definition 2) has orthonormal columns.  The sines of the
    principal angles between span(U_a) and span(U_b) are the singular values of
    D_k = (I - U_a U_a^T) U_b = U_b - U_a M_k with M_k = U_a^T U_b, which follows
    M_k = G_a^T (M_{k-1} (x) I) G_b core by core.  D_k is formed entrywise, one slab of
    rows (one value of the first index) at a time, so small angles keep full relative
    accuracy (the cosines alone resolve no sine below about 1e-8).  One value per bond
    k = 1..d-1; the ranks of a and b must agree.
    """
    d = len(a)
    Ms = []
    M = np.ones((1, 1))
    for k in range(1, d):
        T = np.einsum("ab,aix->bix", M, a[k - 1])
        M = np.einsum("bix,biy->xy", T, b[k - 1])
        Ms.append(M)
    S = [np.zeros((m.shape[1], m.shape[1])) for m in Ms]
    for i1 in range(a[0].shape[1]):
        ua, ub = a[0][0, i1:i1 + 1, :], b[0][0, i1:i1 + 1, :]
        for k in range(1, d):
            if k > 1:
                ua = (ua @ a[k - 1].reshape(a[k - 1].shape[0], -1)).reshape(-1, a[k - 1].shape[2])
                ub = (ub @ b[k - 1].reshape(b[k - 1].shape[0], -1)).reshape(-1, b[k - 1].shape[2])
            D = ub - ua @ Ms[k - 1]
            S[k - 1] += D.T @ D
    out = []
    for Sk in S:
        ev = np.linalg.eigvalsh(0.5 * (Sk + Sk.T)) if Sk.size else np.zeros(1)
        out.append(float(math.sqrt(max(0.0, min(1.0, float(ev.max()))))))
    return out


def left_orthonormality(cores: Sequence[np.ndarray]) -> float:
    """max_k ||G_k^T G_k - I||_max over the first d-1 cores (as r_{k-1} I_k x r_k)."""
    worst = 0.0
    for c in cores[:-1]:
        G = c.reshape(-1, c.shape[2])
        worst = max(worst, float(np.max(np.abs(G.T @ G - np.eye(G.shape[1])))))
    return worst


def unfolding_tail(X: np.ndarray, k: int, j: int) -> float:
    """tau_j^2 of the k-th unfolding X<k> = reshape(X, I1..Ik x I_{k+1}..I_N) (Definition 3), j >= 1."""
    m = int(np.prod(X.shape[:k]))
    sig = np.linalg.svd(X.reshape(m, -1), compute_uv=False)
    return float(np.sum(sig[j - 1:] ** 2))
