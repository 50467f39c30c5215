"""Gaussian test matrices Omega for the sketch step (Algorithm 3, step 3).

The paper only asks for "a random Gaussian matrix" per mode.  Both the oracle
and the GPU library draw the *same* matrix, each from its own implementation
of one published counter-based generator:

* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): 10 rounds of the 4x64 Philox S-box with the round
  multipliers and Weyl key increments given there.
* Box-Muller (1958) in float64: a pair of uniforms (u1, u2) gives
  sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2).

Entry (beta, c) of Omega_k (n_k x s_k, mode k counted from 1) is defined by:
  key     = (seed, k)                 two 64-bit words
  counter = (beta, c // 4, 0, 0)      four 64-bit words
  x0..x3  = Philox4x64-10(counter, key)
  u_j     = ((x_j >> 12) + 1/2) * 2^-52      exactly representable, in (0, 1)
  c % 4 == 0, 1 :  sqrt(-2 ln u0) * cos(2 pi u1),  sqrt(-2 ln u0) * sin(2 pi u1)
  c % 4 == 2, 3 :  sqrt(-2 ln u2) * cos(2 pi u3),  sqrt(-2 ln u2) * sin(2 pi u3)
where 2 pi is the float64 nearest to 2 pi and the product 2 pi * u is rounded
once to float64 before cos/sin.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a: np.ndarray, b: np.uint64):
    """(hi, lo) 64-bit halves of the 128-bit product a*b, from 32-bit limbs."""
    a_lo = a & _LO32
    a_hi = a >> _S32
    b_lo = b & _LO32
    b_hi = b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    lo = (ll & _LO32) | ((mid & _LO32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x64 with 10 rounds; all arguments uint64 (arrays broadcast)."""
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) for v in (c0, c1, c2, c3))
        k0 = np.asarray(k0, dtype=np.uint64)
        k1 = np.asarray(k1, dtype=np.uint64)
        for _ in range(10):
            hi0, lo0 = _mulhilo64(x0, _M0)
            hi1, lo1 = _mulhilo64(x2, _M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = k0 + _W0
            k1 = k1 + _W1
    return x0, x1, x2, x3


_TWO_PI = 6.283185307179586   # float64 nearest to 2*pi
_INV_2_52 = 2.0 ** -52


def _uniform(x: np.ndarray) -> np.ndarray:
    return ((x >> np.uint64(12)).astype(np.float64) + 0.5) * _INV_2_52


def omega(seed: int, k: int, beta0: int, beta1: int, s: int) -> np.ndarray:
    """Rows beta0..beta1-1 of Omega_k (an (beta1-beta0) x s float64 array)."""
    nb = beta1 - beta0
    ng = (s + 3) // 4
    beta = np.arange(beta0, beta1, dtype=np.uint64)[:, None]
    g = np.arange(ng, dtype=np.uint64)[None, :]
    z = np.zeros((1, 1), dtype=np.uint64)
    key0 = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    key1 = np.uint64(k)
    x0, x1, x2, x3 = philox4x64_10(beta, g, z, z, key0, key1)
    out = np.empty((nb, ng * 4), dtype=np.float64)
    for (xa, xb, col) in ((x0, x1, 0), (x2, x3, 2)):
        rad = np.sqrt(-2.0 * np.log(_uniform(xa)))
        th = _TWO_PI * _uniform(xb)
        out[:, col::4] = rad * np.cos(th)
        out[:, col + 1::4] = rad * np.sin(th)
    return out[:, :s]
