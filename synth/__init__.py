"""Seeded synthetic workloads for TT approximation experiments.

This module only *builds input tensors*: low-TT-rank signals, orthogonally
decomposable (odeco) signals and scaled noise.  It holds none of the
arithmetic of the approximation method itself (no sketching, no Krylov
products, no orthonormalisation, no truncation), so that the CPU oracle and
the GPU library can both consume its outputs without sharing method code.

Every workload is defined by a small set of numpy-seeded factors (cores,
factor matrices) plus a noise law.  ``build_host`` materialises the tensor
in float64 with numpy; ``build_device`` materialises it with torch on a GPU
for sizes that do not fit a host-side build comfortably.  The two builders
draw their noise from different generators (numpy vs torch), so a tensor
built on the host and one built on the device are *different* samples of the
same law; every comparison feeds one and the same array to both sides.

Workload structure follows the paper's experiments (low-rank signal plus
noise, heavy-tailed noise, Section 4 of arXiv:2308.01480) at the sizes of the
benchmark configurations.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "workload", "tt_cores_random", "tt_full_host",
    "odeco_factors", "build_host", "build_device", "scaled_down", "eta_from_snr_db",
    "power_function_host", "decaying_diagonal_host",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """A synthetic tensor recipe plus the TT-RBKI run parameters used on it."""
    name: str
    dims: tuple
    signal: str            # "tt" | "odeco" | "power" | "diag"
    signal_rank: int       # bond rank of the TT signal / number of odeco terms
    core_std: float        # std of i.i.d. Gaussian TT core entries
    noise: str             # "gauss" | "student2" | "none"
    eta: float             # noise level: ||E||_F = eta * ||X0||_F
    core_seed: int
    noise_seed: int
    ranks: int             # target TT rank (clamped per bond by the method)
    p: int                 # oversampling
    q: int                 # Krylov depth
    omega_seed: int = 0
    odeco_decay: float = 1.0   # odeco weights i^-decay
    power_h: float = 5.0       # "power": x = (i_1^h + ... + i_N^h)^(-1/h), 1-based indices
    diag_T: int = 50           # "diag": frontal slice j = diag(1 (min(T, j) times), 10^-D, 10^-2D, ...)
    diag_D: float = 1.0

    @property
    def d(self) -> int:
        return len(self.dims)

    @property
    def numel(self) -> int:
        return int(np.prod(np.array(self.dims, dtype=np.int64)))

    def target_ranks(self) -> List[int]:
        return [self.ranks] * (self.d - 1)


# The five benchmark workloads (sizes, signal laws, noise laws, run parameters).
WORKLOADS = {
    "tt20x4": Workload("tt20x4", (20, 20, 20, 20), "tt", 5, 1.0, "gauss", 1e-3,
                       1001, 2001, ranks=5, p=5, q=2),
    "tt48x5": Workload("tt48x5", (48,) * 5, "tt", 20, 1.0, "student2", 1e-2,
                       1002, 2002, ranks=20, p=10, q=3),
    "odeco256x4": Workload("odeco256x4", (256,) * 4, "odeco", 50, 1.0, "gauss", 5e-2,
                           1003, 2003, ranks=32, p=8, q=4),
    "tt8x10": Workload("tt8x10", (8,) * 10, "tt", 16, 1.0 / math.sqrt(16.0), "gauss", 1e-3,
                       1004, 2004, ranks=16, p=8, q=2),
    "tt24x6": Workload("tt24x6", (24,) * 6, "tt", 12, 1.0, "gauss", 1e-2,
                       1005, 2005, ranks=12, p=6, q=2),
}


def eta_from_snr_db(snr_db: float) -> float:
    """Relative noise norm ||E|| / ||X0|| of a signal-to-noise ratio in dB measured on the
    signal's own power: SNR = 10 log10(||X0||^2 / ||E||^2)."""
    return 10.0 ** (-snr_db / 20.0)


# The paper's synthetic workloads (Section 4): the fifth-order power-function tensor
# (45^5, h = 5; Figures 1, 8, 9: ranks 2..11, p = 2, noise 5 dB) and the spectrum-decaying
# diagonal tensor (500^3, T = 50, D = 1; Figure 2: ranks 5..100, p = 2).  q is not stated
# in the paper; 2 is used here.
WORKLOADS.update({
    "power45x5": Workload("power45x5", (45,) * 5, "power", 0, 0.0, "none", 0.0, 0, 2005,
                          ranks=5, p=2, q=2),
    "power45x5_snr5": Workload("power45x5_snr5", (45,) * 5, "power", 0, 0.0, "gauss", eta_from_snr_db(5.0),
                               0, 2006, ranks=5, p=2, q=2),
    "diag500x3": Workload("diag500x3", (500, 500, 500), "diag", 0, 0.0, "none", 0.0, 0, 2007,
                          ranks=20, p=2, q=2),
})


def power_function_host(dims: Sequence[int], h: float) -> np.ndarray:
    """x_{i_1..i_N} = 1 / (i_1^h + ... + i_N^h)^(1/h) with 1-based indices (the power-function
    tensor of Section 4)."""
    acc = np.zeros(tuple(int(v) for v in dims))
    for k, I in enumerate(dims):
        shape = [1] * len(dims)
        shape[k] = int(I)
        acc = acc + (np.arange(1, I + 1, dtype=np.float64) ** h).reshape(shape)
    return acc ** (-1.0 / h)


def _diag_values(n: int, T: int, D: float, j1: int) -> np.ndarray:
    """Diagonal of frontal slice j1 (1-based): min(T, j1) ones, then 10^-D, 10^-2D, ...
    (evaluated in float64: the tail underflows to zero as it would in any IEEE double
    evaluation of the printed formula)."""
    ones = min(T, j1)
    ex = np.arange(1, n - ones + 1, dtype=np.float64) * D
    return np.concatenate([np.ones(ones), 10.0 ** (-ex)])


def decaying_diagonal_host(dims: Sequence[int], T: int, D: float) -> np.ndarray:
    """I x I x J tensor whose j-th frontal slice X[:, :, j] is the diagonal matrix of
    _diag_values (Section 4's spectrum-decaying tensor)."""
    I, I2, J = (int(v) for v in dims)
    assert I == I2, "frontal slices are square"
    X = np.zeros((I, I, J))
    idx = np.arange(I)
    for j in range(J):
        X[idx, idx, j] = _diag_values(I, T, D, j + 1)
    return X


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def scaled_down(w: Workload, dims: Sequence[int], **changes) -> Workload:
    """Same laws and run parameters on a smaller shape (CI-sized twins)."""
    return dataclasses.replace(w, name=w.name + "_small", dims=tuple(int(x) for x in dims), **changes)


def _bond_ranks(dims: Sequence[int], r: int) -> List[int]:
    """Feasible TT bond ranks (1, r1..r_{d-1}, 1) for a signal of nominal rank r."""
    d = len(dims)
    out = [1]
    for k in range(1, d):
        left = int(np.prod(dims[:k], dtype=np.float64))
        right = int(np.prod(dims[k:], dtype=np.float64))
        out.append(int(min(r, left, right)))
    out.append(1)
    return out


def tt_cores_random(dims: Sequence[int], r: int, std: float, seed: int) -> List[np.ndarray]:
    """I.i.d. N(0, std^2) TT cores of shape (r_{k-1}, I_k, r_k)."""
    rng = np.random.default_rng(seed)
    br = _bond_ranks(dims, r)
    return [rng.standard_normal((br[k], dims[k], br[k + 1])) * std for k in range(len(dims))]


def tt_full_host(cores: Sequence[np.ndarray]) -> np.ndarray:
    """Dense tensor from TT cores (row-major, first index slowest)."""
    cur = cores[0].reshape(cores[0].shape[1], cores[0].shape[2])
    for c in cores[1:]:
        cur = cur @ c.reshape(c.shape[0], -1)
        cur = cur.reshape(-1, c.shape[2])
    dims = [c.shape[1] for c in cores]
    return cur.reshape(dims)


def _haar_orthonormal(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """n x k matrix with Haar-distributed orthonormal columns (Mezzadri 2007)."""
    g = rng.standard_normal((n, k))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def odeco_factors(w: Workload):
    """Factor matrices U^(k) (I_k x R) and weights i^-decay of the odeco signal."""
    rng = np.random.default_rng(w.core_seed)
    R = w.signal_rank
    us = [_haar_orthonormal(rng, I, R) for I in w.dims]
    wts = np.arange(1, R + 1, dtype=np.float64) ** (-w.odeco_decay)
    return us, wts


def _odeco_full_host(us, wts) -> np.ndarray:
    # X0 = sum_i w_i u_i^(1) o u_i^(2) o ... o u_i^(d); built as a chain of Khatri-Rao products.
    cur = us[0] * wts[None, :]
    for u in us[1:]:
        cur = (cur[:, None, :] * u[None, :, :]).reshape(-1, u.shape[1])
    return cur.sum(axis=1).reshape([u.shape[0] for u in us])


def _student2_from_uniform(u):
    # Student-t with 2 degrees of freedom by inversion of its CDF.
    return (2.0 * u - 1.0) / np.sqrt(2.0 * u * (1.0 - u))


def build_host(w: Workload) -> np.ndarray:
    """Float64 tensor of the workload, built on the host, scaled to RMS 1."""
    if w.signal == "tt":
        x0 = tt_full_host(tt_cores_random(w.dims, w.signal_rank, w.core_std, w.core_seed))
    elif w.signal == "odeco":
        x0 = _odeco_full_host(*odeco_factors(w))
    elif w.signal == "power":
        x0 = power_function_host(w.dims, w.power_h)
    elif w.signal == "diag":
        x0 = decaying_diagonal_host(w.dims, w.diag_T, w.diag_D)
    else:
        raise ValueError(w.signal)
    x = _add_noise_host(x0, w)
    nrm = np.linalg.norm(x.ravel())
    if nrm > 0:
        x *= math.sqrt(x.size) / nrm
    return np.ascontiguousarray(x)


def _add_noise_host(x0: np.ndarray, w: Workload) -> np.ndarray:
    if w.noise == "none" or w.eta == 0.0:
        return x0.copy()
    rng = np.random.default_rng(w.noise_seed)
    if w.noise == "gauss":
        e = rng.standard_normal(x0.shape)
    elif w.noise == "student2":
        u = rng.random(x0.shape)
        u = np.where(u == 0.0, 0.5, u)
        e = _student2_from_uniform(u)
    else:
        raise ValueError(w.noise)
    e *= w.eta * np.linalg.norm(x0.ravel()) / np.linalg.norm(e.ravel())
    return x0 + e


def build_device(w: Workload, dtype=None, device: str = "cuda", chunk_rows: Optional[int] = None):
    """The workload's tensor built with torch on ``device`` and stored as ``dtype``.

    The signal factors are the same numpy-seeded factors as ``build_host``;
    the dense signal and the noise are generated in float64 chunks on the
    device (noise from a seeded torch generator), then the whole tensor is
    scaled to RMS 1 and cast to ``dtype``.  Peak extra memory is a few
    float64 chunks, never a float64 copy of the whole tensor.
    """
    import torch
    dtype = dtype or torch.float64
    dims = list(w.dims)
    lead = dims[0]
    rest = int(np.prod(dims[1:], dtype=np.int64))
    out = torch.empty((lead, rest), dtype=dtype, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(w.noise_seed)
    if w.signal == "tt":
        cores = [torch.from_numpy(c).to(device) for c in
                 tt_cores_random(w.dims, w.signal_rank, w.core_std, w.core_seed)]
        # right interface: R (r1 x rest) = contraction of cores 2..d
        right = cores[-1].reshape(cores[-1].shape[0], -1)
        for c in reversed(cores[1:-1]):
            right = (c.reshape(-1, c.shape[2]) @ right).reshape(c.shape[0], -1)
        left = cores[0].reshape(lead, -1)
        signal_row = lambda i0, i1: left[i0:i1] @ right
    elif w.signal == "power":
        # sum_{k>1} i_k^h over the trailing multi-index, then the leading index per row
        tail = torch.zeros(1, dtype=torch.float64, device=device)
        for I in dims[1:]:
            v = torch.arange(1, I + 1, dtype=torch.float64, device=device) ** w.power_h
            tail = (tail[:, None] + v[None, :]).reshape(-1)
        h = w.power_h
        signal_row = lambda i0, i1: (
            (torch.arange(i0 + 1, i1 + 1, dtype=torch.float64, device=device) ** h)[:, None] + tail[None, :]) ** (-1.0 / h)
    elif w.signal == "diag":
        I, J = dims[0], dims[2]
        vals = torch.from_numpy(np.stack([_diag_values(I, w.diag_T, w.diag_D, j + 1) for j in range(J)], 1)).to(device)

        def signal_row(i0, i1):
            blk = torch.zeros((i1 - i0, I, J), dtype=torch.float64, device=device)
            ii = torch.arange(i0, i1, device=device)
            blk[ii - i0, ii, :] = vals[i0:i1]
            return blk.reshape(i1 - i0, -1)
    else:
        us, wts = odeco_factors(w)
        us_t = [torch.from_numpy(u).to(device) for u in us]
        right = us_t[-1]
        for u in reversed(us_t[1:-1]):
            right = (u[:, None, :] * right[None, :, :]).reshape(-1, u.shape[1])
        left = us_t[0] * torch.from_numpy(wts).to(device)[None, :]
        signal_row = lambda i0, i1: left[i0:i1] @ right.T
    # Pass 1 accumulates ||S||^2, ||E||^2 and <S,E> chunk by chunk; pass 2 regenerates the
    # same noise stream (restored generator state) and writes (S + a E) * b in one rounding.
    step = chunk_rows or max(1, int(2 ** 27 // max(rest, 1)))
    state = gen.get_state()
    s0 = se = cr = 0.0
    for i0 in range(0, lead, step):
        i1 = min(lead, i0 + step)
        blk = signal_row(i0, i1)
        s0 += float(torch.sum(blk * blk))
        e = _noise_chunk_device(w, (i1 - i0, rest), gen, device)
        if e is not None:
            se += float(torch.sum(e * e))
            cr += float(torch.sum(blk * e))
    a = (w.eta * math.sqrt(s0) / math.sqrt(se)) if se > 0 else 0.0
    x_sq = s0 + 2.0 * a * cr + a * a * se
    b = math.sqrt(w.numel / x_sq) if x_sq > 0 else 1.0
    gen.set_state(state)
    for i0 in range(0, lead, step):
        i1 = min(lead, i0 + step)
        blk = signal_row(i0, i1)
        e = _noise_chunk_device(w, (i1 - i0, rest), gen, device)
        if e is not None:
            blk = blk + a * e
        out[i0:i1] = (blk * b).to(dtype)
    return out.reshape(dims)


def _noise_chunk_device(w: Workload, shape, gen, device):
    import torch
    if w.noise == "none" or w.eta == 0.0:
        return None
    if w.noise == "gauss":
        return torch.randn(shape, generator=gen, device=device, dtype=torch.float64)
    if w.noise == "student2":
        u = torch.rand(shape, generator=gen, device=device, dtype=torch.float64)
        u = torch.where(u == 0.0, torch.full_like(u, 0.5), u)
        return (2.0 * u - 1.0) / torch.sqrt(2.0 * u * (1.0 - u))
    raise ValueError(w.noise)
