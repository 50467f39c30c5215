"""MI355X-native randomized block-Krylov tensor-train approximation (TT-RBKI).

Thin Python binding of the C-ABI library ``libttrbki.so`` (see include/ttrbki.h).
This module only marshals arguments: torch provides device memory and the current
HIP stream, and every step of the computation runs in the library's HIP kernels.
There is no fallback: if the library has not been built, every call raises.

    cores = tt_rbki(x, ranks, q, p, seed)      # x: cuda tensor, float64/float32/bfloat16
    e2, x2, xinf = tt_error(x, cores)          # ||X - Xhat||^2, ||X||^2, ||Xhat||_inf
    f, dfdx = loss_grad(x, ranks, q, p, seed)  # ||X - TT_r(X)||^2 and its gradient
    f = rbki_loss_value(x, ranks, q, p, seed)  # the loss alone (sweep + streamed error)
    f = rbki_loss(x, ranks, q, p, seed)        # a torch.autograd function (backward: reverse sweep)
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import torch

__all__ = ["tt_rbki", "check", "tt_error", "loss_grad", "TTRBKILoss", "rbki_loss", "rbki_loss_value", "plan", "omega", "sketch", "krylov", "carry", "gram", "sym_eig", "sym_eig_top", "orth",
           "library_path", "TTRError", "TTR_F64", "TTR_F32", "TTR_BF16"]

TTR_F64, TTR_F32, TTR_BF16 = 0, 1, 2
MAX_D = 64
_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libttrbki.so")
_lib = None


class TTRError(RuntimeError):
    pass


class _Options(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("method", ctypes.c_int32), ("literal", ctypes.c_int32),
                ("krylov_form", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


METHODS = {"rbki": 0, "rsi": 1, "rsvd": 2}
KRYLOV_FORMS = {"auto": 0, "streamed": 1, "gram": 2}


class PlanT(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("q", ctypes.c_int32), ("p", ctypes.c_int32),
                ("x_dtype", ctypes.c_int32), ("carry_dtype", ctypes.c_int32), ("tau", ctypes.c_double),
                ("dims", ctypes.c_int64 * MAX_D), ("ranks", ctypes.c_int64 * (MAX_D + 1)),
                ("m", ctypes.c_int64 * MAX_D), ("n", ctypes.c_int64 * MAX_D),
                ("s", ctypes.c_int32 * MAX_D), ("w", ctypes.c_int32 * MAX_D), ("kind", ctypes.c_int32 * MAX_D),
                ("two_pass", ctypes.c_int32 * MAX_D), ("core_elems", ctypes.c_int64 * MAX_D),
                ("workspace_bytes", ctypes.c_size_t), ("grad_workspace_bytes", ctypes.c_size_t),
                ("method", ctypes.c_int32), ("literal", ctypes.c_int32),
                ("gram_first", ctypes.c_int32 * MAX_D)]

    @property
    def ranks_list(self) -> List[int]:
        return [int(self.ranks[i]) for i in range(self.d + 1)]

    @property
    def kinds(self) -> List[str]:
        names = {0: "identity", 1: "saturated", 2: "regular"}
        return [names[int(self.kind[i])] for i in range(self.d - 1)]


_P = ctypes.c_void_p
_I32, _I64, _U64, _SZ, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double
_PI64 = ctypes.POINTER(ctypes.c_int64)

_SIGNATURES = {
    "ttr_plan": (_I32, [_I32, _PI64, _PI64, _I32, _I32, _I32, ctypes.POINTER(_Options), ctypes.POINTER(PlanT)]),
    "ttr_rbki": (_I32, [_P, _I32, _I32, _PI64, _PI64, _I32, _I32, _U64, ctypes.POINTER(_Options), _P, _P, _SZ, _P]),
    "ttr_rbki_loss_grad": (_I32, [_P, _I32, _I32, _PI64, _PI64, _I32, _I32, _U64, ctypes.POINTER(_Options), _P, _P,
                                  _P, _SZ, _P]),
    "ttr_tt_error_workspace": (_SZ, [_I32, _PI64, _PI64]),
    "ttr_tt_error": (_I32, [_P, _I32, _I32, _PI64, _PI64, _P, _P, _P, _SZ, _P]),
    "ttr_block_workspace": (_SZ, [_I64, _I64, _I32, _I32]),
    "ttr_omega": (_I32, [_U64, _I32, _I64, _I64, _I32, _P, _P]),
    "ttr_sketch": (_I32, [_P, _I32, _I64, _I64, _U64, _I32, _I32, _P, _P, _SZ, _P]),
    "ttr_krylov": (_I32, [_P, _I32, _I64, _I64, _P, _I32, _P, _I32, _P, _SZ, _P]),
    "ttr_krylov_timed": (_I32, [_P, _I32, _I64, _I64, _P, _I32, _P, _I32, _P, _SZ, _P, _P, _P]),
    "ttr_carry": (_I32, [_P, _I32, _I64, _I64, _P, _I32, _P, _I32, _P, _SZ, _P]),
    "ttr_gram": (_I32, [_P, _I32, _I64, _I64, _P, _P, _SZ, _P]),
    "ttr_gram_sketch": (_I32, [_P, _I32, _I64, _I64, _U64, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "ttr_gram_sketch_timed": (_I32, [_P, _I32, _I64, _I64, _U64, _I32, _I32, _P, _P, _I32, _P, _SZ, _P, _P, _P]),
    "ttr_sym_eig_workspace": (_SZ, [_I32]),
    "ttr_sym_eig": (_I32, [_P, _I32, _P, _P, _P, _SZ, _P]),
    "ttr_orth_workspace": (_SZ, [_I64, _I32]),
    "ttr_orth": (_I32, [_P, _I64, _I32, _D, _D, _P, _P, _P, _SZ, _P]),
    "ttr_sym_eig_top": (_I32, [_P, _I32, _I32, _P, _P, _P, _SZ, _P]),
    "ttr_check": (_I32, [_P, _P]),
    "ttr_rbki_noalloc": (_I32, [_P, _I32, _I32, _PI64, _PI64, _I32, _I32, _U64, ctypes.POINTER(_Options), _P, _P]),
    "ttr_strerror": (ctypes.c_char_p, [_I32]),
    "ttr_last_error_detail": (ctypes.c_char_p, []),
}


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise TTRError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build() or "
                           "python -m paper_2308_01480_amd.build (no CPU fallback exists)")
        lib = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != 0:
        lib = _load()
        raise TTRError(f"{lib.ttr_strerror(rc).decode()} ({rc}): {lib.ttr_last_error_detail().decode()}")


def _dtype_code(t: torch.dtype) -> int:
    if t == torch.float64:
        return TTR_F64
    if t == torch.float32:
        return TTR_F32
    if t == torch.bfloat16:
        return TTR_BF16
    raise TTRError(f"unsupported dtype {t}")


def _i64(vals: Sequence[int]):
    arr = (ctypes.c_int64 * max(1, len(vals)))(*[int(v) for v in vals])
    return arr


def _opts(tau: Optional[float], method: str = "rbki", literal: bool = False, krylov: str = "auto"):
    o = _Options()
    o.tau = float(tau) if tau else 0.0
    if method not in METHODS:
        raise TTRError(f"unknown method {method!r}: one of {sorted(METHODS)}")
    if krylov not in KRYLOV_FORMS:
        raise TTRError(f"unknown krylov form {krylov!r}: one of {sorted(KRYLOV_FORMS)}")
    o.method = METHODS[method]
    o.literal = 1 if literal else 0
    o.krylov_form = KRYLOV_FORMS[krylov]
    return ctypes.byref(o)


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _require_cuda(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise TTRError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise TTRError(f"{name} must be contiguous (row-major)")


def plan(dims: Sequence[int], ranks, q: int, p: int, dtype: torch.dtype = torch.float64,
         tau: Optional[float] = None, method: str = "rbki", literal: bool = False, krylov: str = "auto") -> PlanT:
    """Clamped ranks, mode kinds and workspace size of a sweep (host only)."""
    lib = _load()
    d = len(dims)
    tr = [int(ranks)] * (d - 1) if isinstance(ranks, int) else list(ranks)
    out = PlanT()
    _check(lib.ttr_plan(d, _i64(dims), _i64(tr), int(q), int(p), _dtype_code(dtype),
                        _opts(tau, method, literal, krylov), ctypes.byref(out)))
    return out


def check(workspace: torch.Tensor):
    """Raise TTRError (TTR_ENUMERIC) when the last sweep or gradient call that used this
    workspace met non-finite values; waits for the current stream."""
    _check(_load().ttr_check(_ptr(workspace), ctypes.c_void_p(_stream(workspace.device))))


def tt_rbki(x: torch.Tensor, ranks, q: int, p: int, seed: int = 0, tau: Optional[float] = None,
            workspace: Optional[torch.Tensor] = None, check_finite: bool = False, method: str = "rbki",
            literal: bool = False, krylov: str = "auto") -> List[torch.Tensor]:
    """TT-RBKI sweep of the dense GPU tensor ``x``; returns float64 cores (r_{k-1}, I_k, r_k).
    ``method`` "rsi" / "rsvd" selects TT-rSI (Algorithm 4) / TT-rSVD (Algorithm 2);
    ``literal`` the first-r-columns truncation as printed instead of Rayleigh-Ritz;
    ``krylov`` "streamed" / "gram" forces how TT-RBKI forms its products (default: planner).
    With ``check_finite`` the call waits for the sweep and raises on non-finite values."""
    lib = _load()
    _require_cuda(x, "x")
    dims = list(x.shape)
    d = len(dims)
    tr = [int(ranks)] * (d - 1) if isinstance(ranks, int) else list(ranks)
    pl = plan(dims, tr, q, p, x.dtype, tau, method, literal, krylov)
    rk = pl.ranks_list
    cores = [torch.empty((rk[k], dims[k], rk[k + 1]), dtype=torch.float64, device=x.device) for k in range(d)]
    if workspace is None or workspace.numel() < pl.workspace_bytes:
        workspace = torch.empty(max(1, pl.workspace_bytes), dtype=torch.uint8, device=x.device)
    ptrs = (ctypes.c_void_p * d)(*[c.data_ptr() for c in cores])
    _check(lib.ttr_rbki(_ptr(x), _dtype_code(x.dtype), d, _i64(dims), _i64(tr), int(q), int(p),
                        ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), _opts(tau, method, literal, krylov),
                        ctypes.cast(ptrs, ctypes.c_void_p),
                        _ptr(workspace), ctypes.c_size_t(workspace.numel()), ctypes.c_void_p(_stream(x.device))))
    if check_finite:
        check(workspace)
    return cores


def tt_rbki_noalloc(x: torch.Tensor, ranks, q: int, p: int, seed: int = 0, tau: Optional[float] = None,
                    cores: Optional[List[torch.Tensor]] = None) -> List[torch.Tensor]:
    """tt_rbki on the library's own device scratch (ttr_rbki_noalloc): no workspace is
    allocated; ``cores`` may be given (float64, the planned shapes) to allocate nothing."""
    lib = _load()
    _require_cuda(x, "x")
    dims = list(x.shape)
    d = len(dims)
    tr = [int(ranks)] * (d - 1) if isinstance(ranks, int) else list(ranks)
    if cores is None:
        rk = plan(dims, tr, q, p, x.dtype, tau).ranks_list
        cores = [torch.empty((rk[k], dims[k], rk[k + 1]), dtype=torch.float64, device=x.device) for k in range(d)]
    ptrs = (ctypes.c_void_p * d)(*[c.data_ptr() for c in cores])
    _check(lib.ttr_rbki_noalloc(_ptr(x), _dtype_code(x.dtype), d, _i64(dims), _i64(tr), int(q), int(p),
                                ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), _opts(tau),
                                ctypes.cast(ptrs, ctypes.c_void_p), ctypes.c_void_p(_stream(x.device))))
    return cores


def loss_grad(x: torch.Tensor, ranks, q: int, p: int, seed: int = 0, tau: Optional[float] = None,
              workspace: Optional[torch.Tensor] = None, check_finite: bool = False):
    """(f, df/dX) with f = ||X - TT_r(X)||_F^2 of the TT-RBKI sweep, Omega fixed by ``seed``.

    ``f`` is a 0-dim float64 device tensor, ``df/dX`` has x's shape and dtype
    (float64 or float32)."""
    lib = _load()
    _require_cuda(x, "x")
    dims = list(x.shape)
    d = len(dims)
    tr = [int(ranks)] * (d - 1) if isinstance(ranks, int) else list(ranks)
    pl = plan(dims, tr, q, p, x.dtype, tau)
    if pl.grad_workspace_bytes == 0:
        raise TTRError("the gradient entry supports float64/float32 input with regular modes of m <= 4096")
    if workspace is None or workspace.numel() < pl.grad_workspace_bytes:
        workspace = torch.empty(pl.grad_workspace_bytes, dtype=torch.uint8, device=x.device)
    dx = torch.empty_like(x)
    loss = torch.empty((), dtype=torch.float64, device=x.device)
    _check(lib.ttr_rbki_loss_grad(_ptr(x), _dtype_code(x.dtype), d, _i64(dims), _i64(tr), int(q), int(p),
                                  ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), _opts(tau), _ptr(dx), _ptr(loss),
                                  _ptr(workspace), ctypes.c_size_t(workspace.numel()),
                                  ctypes.c_void_p(_stream(x.device))))
    if check_finite:
        check(workspace)
    return loss, dx


def rbki_loss_value(x: torch.Tensor, ranks, q: int, p: int, seed: int = 0, tau: Optional[float] = None,
                    workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """f = ||X - TT_r(X)||_F^2 without the gradient: the sweep (ttr_rbki) then the streamed
    error (ttr_tt_error) of its cores; a 0-dim float64 device tensor."""
    cores = tt_rbki(x, ranks, q, p, seed, tau, workspace)
    return tt_error(x, cores)[0]


class TTRBKILoss(torch.autograd.Function):
    """f(X) = ||X - TT_r(X)||_F^2 through the TT-RBKI sweep with Omega fixed by the seed.

    forward runs the sweep and the streamed error only and keeps X; backward calls the
    library's reverse sweep (ttr_rbki_loss_grad), which recomputes the Krylov space, and
    scales df/dX by the incoming gradient."""

    @staticmethod
    def forward(ctx, x, ranks, q, p, seed, tau):
        xc = x.contiguous()
        ctx.save_for_backward(xc)
        ctx.args = (ranks, q, p, seed, tau)
        return rbki_loss_value(xc, ranks, q, p, seed, tau)

    @staticmethod
    def backward(ctx, gout):
        (xc,) = ctx.saved_tensors
        _, g = loss_grad(xc, *ctx.args)
        return g * gout.to(g.dtype), None, None, None, None, None


def rbki_loss(x: torch.Tensor, ranks, q: int, p: int, seed: int = 0, tau: Optional[float] = None) -> torch.Tensor:
    return TTRBKILoss.apply(x, ranks, q, p, seed, tau)


def tt_error(x: torch.Tensor, cores: Sequence[torch.Tensor]) -> torch.Tensor:
    """Device tensor (||X - Xhat||_F^2, ||X||_F^2, ||Xhat||_inf) in float64."""
    lib = _load()
    _require_cuda(x, "x")
    d = x.dim()
    dims = list(x.shape)
    ranks = [1] + [int(c.shape[2]) for c in cores[:-1]] + [1]
    for c in cores:
        _require_cuda(c, "core")
        if c.dtype != torch.float64:
            raise TTRError("cores must be float64")
    nbytes = lib.ttr_tt_error_workspace(d, _i64(dims), _i64(ranks))
    ws = torch.empty(max(1, nbytes), dtype=torch.uint8, device=x.device)
    out = torch.empty(3, dtype=torch.float64, device=x.device)
    ptrs = (ctypes.c_void_p * d)(*[c.data_ptr() for c in cores])
    _check(lib.ttr_tt_error(_ptr(x), _dtype_code(x.dtype), d, _i64(dims), _i64(ranks),
                            ctypes.cast(ptrs, ctypes.c_void_p), _ptr(out), _ptr(ws), ctypes.c_size_t(ws.numel()),
                            ctypes.c_void_p(_stream(x.device))))
    return out


def _block_ws(a: torch.Tensor, cols: int) -> torch.Tensor:
    lib = _load()
    m, n = a.shape
    nbytes = lib.ttr_block_workspace(m, n, cols, _dtype_code(a.dtype))
    if nbytes == 0:
        raise TTRError("invalid block shape")
    return torch.empty(nbytes, dtype=torch.uint8, device=a.device)


def omega(seed: int, k: int, beta0: int, nrows: int, s: int, device="cuda") -> torch.Tensor:
    """Rows beta0..beta0+nrows-1 of the Gaussian test matrix Omega_k (float64)."""
    lib = _load()
    out = torch.empty((nrows, s), dtype=torch.float64, device=device)
    _check(lib.ttr_omega(ctypes.c_uint64(seed), k, beta0, nrows, s, _ptr(out),
                         ctypes.c_void_p(_stream(out.device))))
    return out


def sketch(a: torch.Tensor, seed: int, k: int, s: int) -> torch.Tensor:
    """Y = A Omega_k (m x s float64) for a row-major m x n GPU matrix A."""
    lib = _load()
    _require_cuda(a, "a")
    m, n = a.shape
    y = torch.empty((m, s), dtype=torch.float64, device=a.device)
    ws = _block_ws(a, s)
    _check(lib.ttr_sketch(_ptr(a), _dtype_code(a.dtype), m, n, ctypes.c_uint64(seed), k, s, _ptr(y), _ptr(ws),
                          ws.numel(), ctypes.c_void_p(_stream(a.device))))
    return y


def krylov(a: torch.Tensor, z: torch.Tensor, force_two_pass: bool = False) -> torch.Tensor:
    """Y = A (A^T Z) for A (m x n) and float64 Z (m x s)."""
    lib = _load()
    _require_cuda(a, "a")
    _require_cuda(z, "z")
    m, n = a.shape
    s = z.shape[1]
    y = torch.empty((m, s), dtype=torch.float64, device=a.device)
    ws = _block_ws(a, s)
    _check(lib.ttr_krylov(_ptr(a), _dtype_code(a.dtype), m, n, _ptr(z.to(torch.float64).contiguous()), s, _ptr(y),
                          int(force_two_pass), _ptr(ws), ws.numel(), ctypes.c_void_p(_stream(a.device))))
    return y


def krylov_timed(a: torch.Tensor, z: torch.Tensor, reps: int):
    """Y = A (A^T Z) on the one-pass fused path with the streaming kernel launched `reps`
    times back to back between two HIP events that the library records on the current
    stream; returns (Y, average milliseconds per launch of that kernel)."""
    lib = _load()
    _require_cuda(a, "a")
    _require_cuda(z, "z")
    m, n = a.shape
    s = z.shape[1]
    y = torch.empty((m, s), dtype=torch.float64, device=a.device)
    ws = _block_ws(a, s)
    zz = z.to(torch.float64).contiguous()
    st = torch.cuda.current_stream(a.device)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)  # creates the events; the library records them again around the kernel
    e1.record(st)
    _check(lib.ttr_krylov_timed(_ptr(a), _dtype_code(a.dtype), m, n, _ptr(zz), s, _ptr(y), int(reps), _ptr(ws),
                                ws.numel(), ctypes.c_void_p(e0.cuda_event), ctypes.c_void_p(e1.cuda_event),
                                ctypes.c_void_p(st.cuda_stream)))
    e1.synchronize()
    return y, e0.elapsed_time(e1) / reps


def carry(a: torch.Tensor, g: torch.Tensor) -> torch.Tensor:
    """C = G^T A (s x n): float64 for float64 A, float32 otherwise."""
    lib = _load()
    _require_cuda(a, "a")
    m, n = a.shape
    s = g.shape[1]
    cdt = torch.float64 if a.dtype == torch.float64 else torch.float32
    c = torch.empty((s, n), dtype=cdt, device=a.device)
    ws = _block_ws(a, s)
    gg = g.to(torch.float64).contiguous()
    _check(lib.ttr_carry(_ptr(a), _dtype_code(a.dtype), m, n, _ptr(gg), s, _ptr(c), _dtype_code(cdt), _ptr(ws),
                         ws.numel(), ctypes.c_void_p(_stream(a.device))))
    return c


def gram(a: torch.Tensor) -> torch.Tensor:
    """A A^T (m x m, float64) for m <= 128."""
    lib = _load()
    _require_cuda(a, "a")
    m, n = a.shape
    out = torch.empty((m, m), dtype=torch.float64, device=a.device)
    ws = _block_ws(a, 1)
    _check(lib.ttr_gram(_ptr(a), _dtype_code(a.dtype), m, n, _ptr(out), _ptr(ws), ws.numel(),
                        ctypes.c_void_p(_stream(a.device))))
    return out


def gram_sketch(a: torch.Tensor, seed: int, k: int, s: int):
    """(A A^T, A Omega_k) in one pass over A (m <= 256), Omega_k drawn inside the kernel."""
    lib = _load()
    _require_cuda(a, "a")
    m, n = a.shape
    gm = torch.empty((m, m), dtype=torch.float64, device=a.device)
    y = torch.empty((m, s), dtype=torch.float64, device=a.device)
    ws = _block_ws(a, s)
    _check(lib.ttr_gram_sketch(_ptr(a), _dtype_code(a.dtype), m, n, ctypes.c_uint64(seed), k, s, _ptr(gm), _ptr(y),
                               _ptr(ws), ws.numel(), ctypes.c_void_p(_stream(a.device))))
    return gm, y


def gram_sketch_timed(a: torch.Tensor, seed: int, k: int, s: int, reps: int):
    """gram_sketch with its streaming kernel launched `reps` times back to back between two
    HIP events that the library records on the current stream; returns (gm, y, average
    milliseconds per launch of that kernel)."""
    lib = _load()
    _require_cuda(a, "a")
    m, n = a.shape
    gm = torch.empty((m, m), dtype=torch.float64, device=a.device)
    y = torch.empty((m, s), dtype=torch.float64, device=a.device)
    ws = _block_ws(a, s)
    st = torch.cuda.current_stream(a.device)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    e1.record(st)
    _check(lib.ttr_gram_sketch_timed(_ptr(a), _dtype_code(a.dtype), m, n, ctypes.c_uint64(seed), k, s, _ptr(gm),
                                     _ptr(y), int(reps), _ptr(ws), ws.numel(), ctypes.c_void_p(e0.cuda_event),
                                     ctypes.c_void_p(e1.cuda_event), ctypes.c_void_p(st.cuda_stream)))
    e1.synchronize()
    return gm, y, e0.elapsed_time(e1) / reps


def _eig_ws(n: int, device) -> torch.Tensor:
    nbytes = int(_load().ttr_sym_eig_workspace(int(n)))
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def sym_eig(a: torch.Tensor):
    """(vecs, vals) of a symmetric positive semi-definite float64 matrix (n <= 256), decreasing."""
    lib = _load()
    _require_cuda(a, "a")
    n = a.shape[0]
    vecs = torch.empty((n, n), dtype=torch.float64, device=a.device)
    vals = torch.empty(n, dtype=torch.float64, device=a.device)
    ws = _eig_ws(n, a.device)
    _check(lib.ttr_sym_eig(_ptr(a.contiguous()), n, _ptr(vecs), _ptr(vals), _ptr(ws), ctypes.c_size_t(ws.numel()),
                           ctypes.c_void_p(_stream(a.device))))
    return vecs, vals


def orth(p: torch.Tensor, ref_norm: float, tau: float):
    """(Q, k): rank-revealing orthonormal basis of the float64 block p (m x s, s <= 64);
    the first k columns of Q are kept pivots with |R_jj| > tau * ref_norm, the rest zero."""
    lib = _load()
    _require_cuda(p, "p")
    m, s = p.shape
    q = torch.empty((m, s), dtype=torch.float64, device=p.device)
    kept = torch.zeros(1, dtype=torch.int32, device=p.device)
    nbytes = int(lib.ttr_orth_workspace(m, s))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=p.device)
    _check(lib.ttr_orth(_ptr(p.contiguous()), m, s, float(ref_norm), float(tau), _ptr(q), _ptr(kept), _ptr(ws),
                        ctypes.c_size_t(nbytes), ctypes.c_void_p(_stream(p.device))))
    return q, int(kept.cpu())


def sym_eig_top(a: torch.Tensor, r: int):
    """(vecs[:, :r], vals[:r]) leading eigenpairs of a symmetric PSD float64 matrix (n <= 256)."""
    lib = _load()
    _require_cuda(a, "a")
    n = a.shape[0]
    vecs = torch.zeros((n, n), dtype=torch.float64, device=a.device)
    vals = torch.empty(n, dtype=torch.float64, device=a.device)
    ws = _eig_ws(n, a.device)
    _check(lib.ttr_sym_eig_top(_ptr(a.contiguous()), n, int(r), _ptr(vecs), _ptr(vals), _ptr(ws),
                               ctypes.c_size_t(ws.numel()), ctypes.c_void_p(_stream(a.device))))
    return vecs[:, :r], vals[:r]
