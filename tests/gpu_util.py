"""Helpers shared by the GPU tests (no method arithmetic here)."""
import math

import numpy as np
import torch

DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def to_dev(a: np.ndarray, dt: str) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(DT[dt]).contiguous()


def to_dt_host(a: np.ndarray, dt: str) -> np.ndarray:
    """float64 copy of ``a`` after rounding to dtype ``dt`` (on the CPU)."""
    return torch.from_numpy(np.ascontiguousarray(a)).to(DT[dt]).to(torch.float64).numpy()


def round_bf16(a: np.ndarray) -> np.ndarray:
    """float64 values rounded once to bfloat16 (8 significant bits, ties to even), the
    library's own narrowing of float64 operands (normal range only)."""
    mant, ex = np.frexp(np.asarray(a, dtype=np.float64))
    return np.ldexp(np.rint(mant * 256.0) / 256.0, ex)


def stored_f64(t: torch.Tensor) -> np.ndarray:
    """Exact float64 copy of the values a GPU tensor stores."""
    return t.to(torch.float64).cpu().numpy()


def bound_check(got: np.ndarray, ref: np.ndarray, scale: np.ndarray, tol: float):
    """|got - ref| <= tol * scale elementwise, where scale = |A||B| bounds the products summed."""
    err = np.abs(got - ref)
    worst = float(np.max(err / np.maximum(scale, 1e-300)))
    assert worst <= tol, f"max error/scale = {worst:.3e} > {tol:.1e}"
    return worst


def announce(msg: str):
    print(f"[gpu-case] {msg}", flush=True)


# ---- checker metrics computed with plain torch float64 on the GPU (no library kernels),
#      for tensors whose host-side metric passes would take minutes ----

def _dev_cores(cores, device="cuda"):
    return [torch.from_numpy(np.ascontiguousarray(c)).to(device) for c in cores]


def _dev_slab(cores_t, i1):
    """Row i1 of the first index of the TT tensor (Definition 2), as 1 x (I_2..I_d), float64."""
    cur = cores_t[0][0, i1:i1 + 1, :]
    for c in cores_t[1:]:
        cur = (cur @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
    return cur.reshape(1, -1)


def dev_compare(x: torch.Tensor, a, b):
    """(||X - Xhat_a||^2, ||X - Xhat_b||^2, ||X||^2, ||Xhat_a - Xhat_b||^2), float64 sums
    over slabs of the first index; x is a GPU tensor of any float dtype, a and b host cores."""
    at, bt = _dev_cores(a, x.device), _dev_cores(b, x.device)
    xm = x.reshape(x.shape[0], -1)
    ea = eb = x2 = dd = 0.0
    for i1 in range(x.shape[0]):
        xs = xm[i1:i1 + 1].to(torch.float64)
        sa, sb = _dev_slab(at, i1), _dev_slab(bt, i1)
        ea += float(torch.sum((xs - sa) ** 2))
        eb += float(torch.sum((xs - sb) ** 2))
        x2 += float(torch.sum(xs * xs))
        dd += float(torch.sum((sa - sb) ** 2))
    return ea, eb, x2, dd


def dev_interface_sines(a, b):
    """Per bond, sin of the largest principal angle between the left interfaces of two
    left-orthonormal TTs: the largest singular value of U_b - U_a (U_a^T U_b), formed slab
    by slab (the same definition as the oracle's metric, evaluated with torch on the GPU)."""
    at, bt = _dev_cores(a), _dev_cores(b)
    d = len(at)
    Ms, M = [], torch.ones((1, 1), dtype=torch.float64, device="cuda")
    for k in range(1, d):
        T = torch.einsum("ab,aix->bix", M, at[k - 1])
        M = torch.einsum("bix,biy->xy", T, bt[k - 1])
        Ms.append(M)
    S = [torch.zeros((m.shape[1], m.shape[1]), dtype=torch.float64, device="cuda") for m in Ms]
    for i1 in range(at[0].shape[1]):
        ua, ub = at[0][0, i1:i1 + 1, :], bt[0][0, i1:i1 + 1, :]
        for k in range(1, d):
            if k > 1:
                ua = (ua @ at[k - 1].reshape(at[k - 1].shape[0], -1)).reshape(-1, at[k - 1].shape[2])
                ub = (ub @ bt[k - 1].reshape(bt[k - 1].shape[0], -1)).reshape(-1, bt[k - 1].shape[2])
            D = ub - ua @ Ms[k - 1]
            S[k - 1] += D.T @ D
    out = []
    for Sk in S:
        ev = float(torch.linalg.eigvalsh(0.5 * (Sk + Sk.T)).max().cpu())
        out.append(math.sqrt(max(0.0, min(1.0, ev))))
    return out
