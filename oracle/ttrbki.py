"""TT-SVD (Algorithm 1) and TT-RBKI (Algorithm 3) in plain float64 numpy.

Conventions (shared with the GPU library by specification, not by code):

* Tensors are row-major (C order), first index slowest.  The k-th unfolding
  A_k (Definition 1; Algorithm 3, step 2) is the previous carry C_{k-1}
  viewed as an m_k x n_k matrix with m_k = r_{k-1} I_k and
  n_k = I_{k+1} ... I_N; no data is permuted.
* Ranks are clamped, never rejected: r_k = min(target_k, m_k, n_k).
  With s_k = r_k + p and w_k = (q+1) s_k a mode is
    identity   if r_k == m_k            (G_k = I, the carry is A_k itself),
    saturated  if w_k >= min(m_k, n_k)  (the block Krylov space spans the
                                         whole range: exact truncated SVD),
    regular    otherwise.
* Regular modes build the block Krylov space in column-space form
  K = [A Omega, (A A^T) A Omega, ..., (A A^T)^q A Omega]  (q+1 blocks of s
  columns; the paper's step 4 writes the row-space blocks
  (A^T A)^j Omega, j = 1..q, and step 6 maps them back with A, so
  span(A U) of the paper is contained in span(K)).  Each block is fed
  forward orthonormalised, projected against the earlier blocks twice
  (classical Gram-Schmidt, repeated once), and rank-revealed: the economy QR
  of step 5 is taken with column pivoting (Householder QRCP), and only the
  leading pivoted columns with |R_jj| > tau_k * ||Y_j||_F are kept; tau_k
  follows the precision mode k streams (see TAU).
* Truncation (steps 6-9) is by Rayleigh-Ritz on span(Q): with B = Q^T A the
  top-r eigenvectors U~ of B B^T give G_k = Q U~ and the carry
  C_k = G_k^T A_k (step 10's  A x_1 Q^T).  If fewer than r_k directions
  survive, G_k is completed by e_1, e_2, ... made orthogonal to the columns
  already present (classical Gram-Schmidt twice), skipping any unit vector
  whose orthogonal remainder has squared norm <= 1/(4 m).
* The last core is the final carry reshaped (step 12).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.linalg

from .philox import omega

# Drop thresholds tau of the rank-revealing orthonormalisation (Algorithm 3, step 5, read
# as a QR with column pivoting), relative to ||Y_j||_F of the block.  tau is chosen per
# mode from the arithmetic that forms that mode's Krylov blocks:
#   * float64 streams accumulate in float64: 1e-10;
#   * float32 streams accumulate in float32 (unit roundoff 2^-24): 1e-5;
#   * bfloat16 streams round the streamed block to bf16 but still form every column as A
#     times a vector, accumulated in float32.  The rounding perturbs which vectors span the
#     Krylov space, not whether a computed column lies in range(A), so the level that
#     separates real directions from accumulation error is the float32 one: 1e-5.
TAU = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-5}


def stream_precisions(precision: str, modes) -> List[str]:
    """Precision of the data each mode streams: the tensor's own up to and including the
    first mode that forms a carry, the carry's afterwards (float64 carries for a float64
    tensor, float32 otherwise)."""
    carry = "f64" if precision == "f64" else "f32"
    out, cur = [], precision
    for mi in modes:
        out.append(cur)
        if mi.kind != "identity":
            cur = carry
    return out

# Column chunk for streamed products over the wide unfoldings.
_CHUNK = 1 << 17


@dataclasses.dataclass
class ModeInfo:
    k: int
    m: int
    n: int
    r: int
    s: int
    w: int
    kind: str
    kept: int = 0                       # surviving Krylov directions (regular modes)
    ritz: Optional[np.ndarray] = None   # all Rayleigh-Ritz / squared singular values, descending
    tau: float = 0.0                    # drop threshold used in this mode
    rho: float = 0.0                    # ||A_k - G_k C_k||_F^2
    completed: int = 0                  # completion vectors added


def plan_modes(dims: Sequence[int], targets: Sequence[int], q: int, p: int) -> List[ModeInfo]:
    """Per-mode shapes and kinds after rank clamping."""
    d = len(dims)
    if d < 2:
        raise ValueError("need d >= 2")
    if len(targets) != d - 1:
        raise ValueError("need d-1 target ranks")
    out = []
    r_prev = 1
    for k in range(1, d):
        m = r_prev * int(dims[k - 1])
        n = int(np.prod(np.array(dims[k:], dtype=np.int64)))
        r = int(min(int(targets[k - 1]), m, n))
        if r < 1:
            raise ValueError("target ranks must be >= 1")
        s = r + p
        w = (q + 1) * s
        if r == m:
            kind = "identity"
        elif w >= min(m, n):
            kind = "saturated"
        else:
            kind = "regular"
        out.append(ModeInfo(k=k, m=m, n=n, r=r, s=s, w=w, kind=kind))
        r_prev = r
    return out


def complete_columns(G: np.ndarray, m: int, r: int) -> np.ndarray:
    """Append e_1, e_2, ... (orthogonalised against present columns) up to r columns."""
    cols = [G[:, i] for i in range(G.shape[1])]
    thresh = 1.0 / (4.0 * m)
    i = 0
    while len(cols) < r:
        if i >= m:
            raise RuntimeError("completion failed")
        v = np.zeros(m)
        v[i] = 1.0
        if cols:
            Gc = np.stack(cols, axis=1)
            v = v - Gc @ (Gc.T @ v)
            v = v - Gc @ (Gc.T @ v)
        nv2 = float(v @ v)
        if nv2 > thresh:
            cols.append(v / math.sqrt(nv2))
        i += 1
    return np.stack(cols, axis=1) if cols else np.zeros((m, 0))


def orth_tau(P: np.ndarray, ref: float, tau: float) -> np.ndarray:
    """Rank-revealing economy QR of P: Householder QR with column pivoting
    (LAPACK geqp3, whose |R_jj| are non-increasing); returns the first k columns of
    Q, k = number of pivots with |R_jj| > tau * ref."""
    if P.shape[1] == 0:
        return P
    Q, R, _ = scipy.linalg.qr(P, mode="economic", pivoting=True)
    k = int(np.sum(np.abs(np.diag(R)) > tau * ref))
    return Q[:, :k]


def _left_svd(A: np.ndarray):
    """Left singular vectors and values of a (possibly very wide) matrix A."""
    m, n = A.shape
    if n > 4 * m:
        # A^T = Q R (Householder), A = R^T Q^T: left singular pairs of A are those of R^T.
        R = np.linalg.qr(A.T, mode="r")
        U, sig, _ = np.linalg.svd(R.T, full_matrices=False)
    else:
        U, sig, _ = np.linalg.svd(A, full_matrices=False)
    return U, sig


def _gram_chunks(A: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """M = B B^T with B = Q^T A, accumulated over column chunks of A."""
    w = Q.shape[1]
    M = np.zeros((w, w))
    for j0 in range(0, A.shape[1], _CHUNK):
        B = Q.T @ A[:, j0:j0 + _CHUNK]
        M += B @ B.T
    return M


def _sketch(A: np.ndarray, seed: int, k: int, s: int) -> np.ndarray:
    """Y0 = A Omega_k, with Omega_k drawn chunk by chunk (never stored whole)."""
    m, n = A.shape
    Y = np.zeros((m, s))
    for j0 in range(0, n, _CHUNK):
        j1 = min(n, j0 + _CHUNK)
        Y += A[:, j0:j1] @ omega(seed, k, j0, j1, s)
    return Y


def _krylov_product(A: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """A (A^T Z), chunked over columns of A."""
    Y = np.zeros((A.shape[0], Z.shape[1]))
    for j0 in range(0, A.shape[1], _CHUNK):
        Aj = A[:, j0:j0 + _CHUNK]
        Y += Aj @ (Aj.T @ Z)
    return Y


def _carry(G: np.ndarray, A: np.ndarray) -> np.ndarray:
    return G.T @ A


def _residual_sq(A: np.ndarray, G: np.ndarray, C: np.ndarray) -> float:
    tot = 0.0
    for j0 in range(0, A.shape[1], _CHUNK):
        D = A[:, j0:j0 + _CHUNK] - G @ C[:, j0:j0 + _CHUNK]
        tot += float(np.sum(D * D))
    return tot


def _saturated_basis(A: np.ndarray, r: int, tau: float):
    """Exact top-r left singular vectors; directions with sigma <= tau*||sigma_1..r|| are completed."""
    m = A.shape[0]
    U, sig = _left_svd(A)
    top = sig[:r]
    ref = math.sqrt(float(np.sum(top * top)))
    valid = top > tau * ref
    G = U[:, :r][:, valid]
    nv = G.shape[1]
    if nv < r:
        G = complete_columns(G, m, r)
    return G, sig ** 2, r - nv


def _regular_basis(A: np.ndarray, k: int, r: int, s: int, q: int, seed: int, tau: float, gram_first: bool = False):
    """Block Krylov basis and Rayleigh-Ritz truncation of one regular mode.  With
    ``gram_first`` the products A (A^T Z) and B B^T = Q^T A A^T Q are taken through the
    m x m Gram A A^T formed once (the same quantities by associativity)."""
    m = A.shape[0]
    Gm = None
    if gram_first:
        Gm = np.zeros((m, m))
        for j0 in range(0, A.shape[1], _CHUNK):
            Aj = A[:, j0:j0 + _CHUNK]
            Gm += Aj @ Aj.T
    # Step 3-4 (sketch): Y0 = A Omega, orthonormalised with drops.
    Y = _sketch(A, seed, k, s)
    Qs = [orth_tau(Y, float(np.linalg.norm(Y)), tau)]
    # Krylov blocks j = 1..q on the orthonormal previous block.
    for _ in range(q):
        Y = Gm @ Qs[-1] if gram_first else _krylov_product(A, Qs[-1])
        Qp = np.concatenate(Qs, axis=1)
        P = Y - Qp @ (Qp.T @ Y)
        P = P - Qp @ (Qp.T @ P)
        Qs.append(orth_tau(P, float(np.linalg.norm(Y)), tau))
    Q = np.concatenate(Qs, axis=1)
    kept = Q.shape[1]
    # Rayleigh-Ritz: top-r eigenvectors of B B^T, B = Q^T A.
    M = Q.T @ Gm @ Q if gram_first else _gram_chunks(A, Q)
    M = 0.5 * (M + M.T)
    lam, V = np.linalg.eigh(M)
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    V = V[:, order]
    take = min(r, kept)
    G = Q @ V[:, :take]
    comp = 0
    if take < r:
        G = complete_columns(G, m, r)
        comp = r - take
    return G, lam, kept, comp


def tt_rbki(X: np.ndarray, targets: Sequence[int], q: int, p: int, seed: int = 0,
            tau: Optional[float] = None, precision: str = "f64", diagnostics: bool = False,
            residuals: bool = True, gram_first: bool = False):
    """TT-RBKI (Algorithm 3) in the form stated in the module docstring.

    Returns the list of cores (r_{k-1}, I_k, r_k) and, if ``diagnostics``, the
    per-mode ModeInfo list (with ``residuals`` also rho_k, one more pass per mode).
    ``gram_first`` takes the Krylov products of regular modes through A_k A_k^T.
    """
    X = np.asarray(X, dtype=np.float64)
    dims = list(X.shape)
    d = len(dims)
    modes = plan_modes(dims, targets, q, p)
    taus = [TAU[sp] if tau is None else float(tau) for sp in stream_precisions(precision, modes)]
    cores = []
    C = X.reshape(1, -1)
    for mi, tau_k in zip(modes, taus):
        mi.tau = tau_k
        A = C.reshape(mi.m, mi.n)
        if mi.kind == "identity":
            G = np.eye(mi.m)
            Cn = A.copy()
            mi.ritz = None
        elif mi.kind == "saturated":
            G, mi.ritz, mi.completed = _saturated_basis(A, mi.r, tau_k)
            Cn = _carry(G, A)
        else:
            G, mi.ritz, mi.kept, mi.completed = _regular_basis(A, mi.k, mi.r, mi.s, q, seed, tau_k, gram_first)
            Cn = _carry(G, A)
        if diagnostics and residuals:
            mi.rho = _residual_sq(A, G, Cn) if mi.kind != "identity" else 0.0
        r_prev = mi.m // dims[mi.k - 1]
        cores.append(G.reshape(r_prev, dims[mi.k - 1], mi.r))
        C = Cn
    cores.append(C.reshape(modes[-1].r, dims[-1], 1))
    return (cores, modes) if diagnostics else cores


def tt_svd(X: np.ndarray, targets: Sequence[int], diagnostics: bool = False):
    """Fixed-rank TT-SVD (Algorithm 1 with prescribed ranks instead of delta).

    Every mode takes the top-r_k left singular vectors of the processed
    unfolding (r_k clamped to min(target, m_k, n_k)); the carry is G^T A = S V^T.
    With ``diagnostics`` also returns the discarded squared singular values per mode.
    """
    X = np.asarray(X, dtype=np.float64)
    dims = list(X.shape)
    d = len(dims)
    if len(targets) != d - 1:
        raise ValueError("need d-1 target ranks")
    cores, tails = [], []
    C = X.reshape(1, -1)
    r_prev = 1
    for k in range(1, d):
        m = r_prev * dims[k - 1]
        n = C.size // m
        r = int(min(int(targets[k - 1]), m, n))
        A = C.reshape(m, n)
        U, sig = _left_svd(A)
        G = U[:, :r]
        tails.append(sig[r:] ** 2)
        C = G.T @ A
        cores.append(G.reshape(r_prev, dims[k - 1], r))
        r_prev = r
    cores.append(C.reshape(r_prev, dims[-1], 1))
    return (cores, tails) if diagnostics else cores


def tt_svd_delta(X: np.ndarray, eps: float):
    """delta-truncated TT-SVD (Algorithm 1): delta = eps/sqrt(N-1) * ||A||_F,
    each rank the smallest whose discarded tail energy is <= delta^2."""
    X = np.asarray(X, dtype=np.float64)
    dims = list(X.shape)
    d = len(dims)
    delta = eps / math.sqrt(d - 1) * float(np.linalg.norm(X.ravel()))
    cores = []
    C = X.reshape(1, -1)
    r_prev = 1
    for k in range(1, d):
        m = r_prev * dims[k - 1]
        n = C.size // m
        A = C.reshape(m, n)
        U, sig = _left_svd(A)
        tail = np.concatenate([np.cumsum((sig ** 2)[::-1])[::-1], [0.0]])  # tail[j] = sum_{i>=j} sig_i^2
        r = next(j for j in range(1, len(sig) + 1) if tail[j] <= delta * delta)
        G = U[:, :r]
        C = G.T @ A
        cores.append(G.reshape(r_prev, dims[k - 1], r))
        r_prev = r
    cores.append(C.reshape(r_prev, dims[-1], 1))
    return cores


# ---------------------------------------------------------------------------------------
# The paper's comparison drivers and its literal form of TT-RBKI.
#
# Algorithms 2, 3 and 4 as printed truncate each mode to the first r_n columns of an
# unpivoted economy QR (MATLAB qr(., 0); here LAPACK's Householder geqrf through
# numpy.linalg.qr).  Algorithm 3 as printed builds its Krylov matrix in the row space,
# K = [A^T A Omega, ..., (A^T A)^q Omega] (n x q s, no Omega block), orthonormalises it
# (U), maps it back (Y = A U) and takes the first r_n columns of qr(Y).  The Rayleigh-Ritz
# forms ("ritz") replace that truncation by the r_n leading Ritz directions of the final
# basis, as the column-space TT-RBKI above does.  Mode kinds for the printed forms: G = I
# when r_n = m (any orthonormal basis of R^m gives the same tensor); every other mode
# follows the printed steps, except r_n = n < m, where the span is range(A) itself and the
# truncated SVD stands in (it spans the same space).
# ---------------------------------------------------------------------------------------

def _householder_q(M: np.ndarray) -> np.ndarray:
    """Q of the unpivoted economy Householder QR of M (LAPACK geqrf/orgqr)."""
    return np.linalg.qr(M, mode="reduced")[0]


def _ritz_truncate(A: np.ndarray, Q: np.ndarray, r: int) -> np.ndarray:
    """Rayleigh-Ritz: the r leading eigenvectors of B B^T, B = Q^T A, mapped by Q."""
    M = _gram_chunks(A, Q)
    lam, V = np.linalg.eigh(0.5 * (M + M.T))
    order = np.argsort(lam)[::-1]
    take = min(r, Q.shape[1])
    G = Q @ V[:, order[:take]]
    return complete_columns(G, A.shape[0], r) if take < r else G


def _sketch_cols(A: np.ndarray, seed: int, k: int, s: int) -> np.ndarray:
    return _sketch(A, seed, k, s)


def _variant_basis(A: np.ndarray, k: int, r: int, s: int, q: int, seed: int, method: str, truncation: str,
                   tau: float) -> np.ndarray:
    m, n = A.shape
    if method == "rsvd":
        # Algorithm 2: Y = A Omega (step 4), [Q, ~] = qr(Y, 0) (step 5)
        Y = _sketch_cols(A, seed, k, s)
        if truncation == "first":
            return _householder_q(Y)[:, :r]
        return _ritz_truncate(A, orth_tau(Y, float(np.linalg.norm(Y)), tau), r)
    if method == "rbki":
        # Algorithm 3 as printed (steps 3-8)
        if q < 1:
            raise ValueError("Algorithm 3 as printed needs q >= 1 (its Krylov matrix has q blocks)")
        Om = np.concatenate([omega(seed, k, j0, min(n, j0 + _CHUNK), s) for j0 in range(0, n, _CHUNK)], axis=0)
        blocks, cur = [], Om
        for _ in range(q):
            cur = A.T @ (A @ cur)                      # (A^T A)^j Omega
            blocks.append(cur)
        K = np.concatenate(blocks, axis=1)             # step 4: n x q s
        U = _householder_q(K)                          # step 5
        Y = A @ U                                      # step 6
        return _householder_q(Y)[:, :r]                # steps 7-8
    if method == "rsi":
        # Algorithm 4: Y = A Omega, Q_0 = qr(Y); per iteration Yhat = A^T Q, Qhat = qr(Yhat),
        # Y = A Qhat, Q = qr(Y) (steps 4-11); then Q(:, 1:r) (step 12)
        Y = _sketch_cols(A, seed, k, s)
        Q = _householder_q(Y) if truncation == "first" else orth_tau(Y, float(np.linalg.norm(Y)), tau)
        for _ in range(q):
            Qh = _householder_q(A.T @ Q)
            Y = A @ Qh
            Q = _householder_q(Y) if truncation == "first" else orth_tau(Y, float(np.linalg.norm(Y)), tau)
        if truncation == "first":
            return Q[:, :r]
        return _ritz_truncate(A, Q, r)
    raise ValueError(method)


def tt_variant(X: np.ndarray, targets: Sequence[int], q: int, p: int, seed: int = 0, method: str = "rsi",
               truncation: str = "first", tau: Optional[float] = None, precision: str = "f64"):
    """TT-rSVD (method "rsvd", Algorithm 2), TT-rBKI as printed ("rbki", Algorithm 3 with
    the row-space Krylov matrix; truncation must be "first") or TT-rSI ("rsi", Algorithm 4),
    with the printed first-r-columns truncation ("first") or Rayleigh-Ritz ("ritz").
    Returns the cores (r_{k-1}, I_k, r_k).  Omega_k is the same seeded Gaussian matrix as
    in tt_rbki (its column c does not depend on s)."""
    if method == "rbki" and truncation != "first":
        raise ValueError("the Rayleigh-Ritz form of TT-RBKI is tt_rbki")
    X = np.asarray(X, dtype=np.float64)
    dims = list(X.shape)
    modes = plan_modes(dims, targets, q, p)
    taus = [TAU[sp] if tau is None else float(tau) for sp in stream_precisions(precision, modes)]
    cores = []
    C = X.reshape(1, -1)
    for mi, tau_k in zip(modes, taus):
        A = C.reshape(mi.m, mi.n)
        if mi.r == mi.m:
            G = np.eye(mi.m)
            Cn = A.copy()
        else:
            if mi.r == mi.n or (truncation == "ritz" and
                                (mi.s if method != "rbki" else mi.w) >= min(mi.m, mi.n)):
                G = _saturated_basis(A, mi.r, tau_k)[0]
            else:
                G = _variant_basis(A, mi.k, mi.r, mi.s, q, seed, method, truncation, tau_k)
            Cn = G.T @ A
        r_prev = mi.m // dims[mi.k - 1]
        cores.append(G.reshape(r_prev, dims[mi.k - 1], mi.r))
        C = Cn
    cores.append(C.reshape(modes[-1].r, dims[-1], 1))
    return cores
