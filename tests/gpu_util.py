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
