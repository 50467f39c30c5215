"""Gaussian test matrices Omega for the sketch step (Algorithm 3, step 3).

Test infrastructure: this module belongs to the CPU oracle and is used only by the
tests, the smoke check and the benchmark's CPU baseline.

The paper only asks for "a random Gaussian matrix" per mode.  Both the oracle
and the GPU library draw the *same* matrix, each from its own implementation
of one published counter-based generator and one fixed transform:

* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): 10 rounds of the 4x64 Philox S-box with the round
  multipliers and Weyl key increments given there.
* Box-Muller (1958): a pair of uniforms (u, v) gives
  sqrt(-2 ln u) * (cos 2 pi v, sin 2 pi v), evaluated in IEEE float32 arithmetic by
  the fixed sequence of correctly rounded operations below (+, -, *, /, sqrt; no fused
  multiply-add), so that every implementation that follows it produces the same bits.

Entry (beta, c) of Omega_k (n_k x s_k, mode k counted from 1) is defined by:
  key     = (seed, k)                 two 64-bit words
  counter = (beta, c // 8, 0, 0)      four 64-bit words
  x0..x3  = Philox4x64-10(counter, key)
  j = (c % 8) // 2;  a = low 32 bits of x_j, b = high 32 bits of x_j
  u = ((a >> 9) + 1/2) 2^-23,  v = ((b >> 9) + 1/2) 2^-23      exact float32, in (0, 1)
  c even:  sqrt(-2 ln32(u)) * cos32(v)        c odd:  sqrt(-2 ln32(u)) * sin32(v)
ln32: u = 2^e f with f in [1, 2) read from the bits, halved (e + 1) when f > sqrt 2;
  t = (f - 1) / (f + 1), w = t t, p = ((((1/11 w + 1/9) w + 1/7) w + 1/5) w + 1/3) w + 1,
  ln32(u) = e ln2 + (t + t) p   (the atanh series of ln f, truncated after t^11).
cos32 / sin32: y = 4 v, q = floor(y), x = (y - q) (pi/2); Taylor polynomials in x^2 of
  sin x (to x^13) and cos x (to x^14) by Horner's rule, then the quadrant q rotates
  (cos, sin) by q pi/2.
The float32 constants are those in _K (hexadecimal, exact).
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


# float32 constants of the transform (exact values, hexadecimal)
_K = {name: np.float32(float.fromhex(h)) for name, h in {
    "INV3": "0x1.555556p-2", "INV5": "0x1.99999ap-3", "INV7": "0x1.24924ap-3", "INV9": "0x1.c71c72p-4",
    "INV11": "0x1.745d18p-4", "LN2": "0x1.62e430p-1", "SQRT2": "0x1.6a09e6p+0", "HALFPI": "0x1.921fb6p+0",
    "S3": "-0x1.555556p-3", "S5": "0x1.111112p-7", "S7": "-0x1.a01a02p-13", "S9": "0x1.71de3ap-19",
    "S11": "-0x1.ae6456p-26", "S13": "0x1.612462p-33",
    "C2": "-0x1.000000p-1", "C4": "0x1.555556p-5", "C6": "-0x1.6c16c2p-10", "C8": "0x1.a01a02p-16",
    "C10": "-0x1.27e4fcp-22", "C12": "0x1.1eed8ep-29", "C14": "-0x1.93974ap-37"}.items()}
_ONE = np.float32(1.0)


def _uniform23(w: np.ndarray) -> np.ndarray:
    """((w >> 9) + 1/2) 2^-23 for 32-bit words w: exact float32 values in (0, 1)."""
    return ((w >> np.uint64(9)).astype(np.float32) + np.float32(0.5)) * np.float32(2.0 ** -23)


def ln32(u: np.ndarray) -> np.ndarray:
    """ln u for float32 u in (0, 1) by the module's fixed float32 operation sequence."""
    u = np.asarray(u, dtype=np.float32)
    bits = u.view(np.uint32)
    e = (bits >> np.uint32(23)).astype(np.int32) - 127
    f = ((bits & np.uint32(0x7FFFFF)) | np.uint32(0x3F800000)).view(np.float32)
    big = f > _K["SQRT2"]
    f = np.where(big, f * np.float32(0.5), f)
    e = e + big.astype(np.int32)
    t = (f - _ONE) / (f + _ONE)
    w = t * t
    p = _K["INV11"] * w + _K["INV9"]
    p = p * w + _K["INV7"]
    p = p * w + _K["INV5"]
    p = p * w + _K["INV3"]
    p = p * w + _ONE
    return e.astype(np.float32) * _K["LN2"] + (t + t) * p


def cossin32(v: np.ndarray):
    """(cos 2 pi v, sin 2 pi v) for float32 v in [0, 1) by the fixed float32 sequence."""
    v = np.asarray(v, dtype=np.float32)
    y = v * np.float32(4.0)
    q = y.astype(np.int32)
    x = (y - q.astype(np.float32)) * _K["HALFPI"]
    x2 = x * x
    sp = _K["S13"] * x2 + _K["S11"]
    for c in ("S9", "S7", "S5", "S3"):
        sp = sp * x2 + _K[c]
    sp = sp * x2 + _ONE
    sn = x * sp
    cs = _K["C14"] * x2 + _K["C12"]
    for c in ("C10", "C8", "C6", "C4", "C2"):
        cs = cs * x2 + _K[c]
    cs = cs * x2 + _ONE
    cos_out = np.select([q == 0, q == 1, q == 2], [cs, -sn, -cs], sn).astype(np.float32)
    sin_out = np.select([q == 0, q == 1, q == 2], [sn, cs, -sn], -cs).astype(np.float32)
    return cos_out, sin_out


def omega(seed: int, k: int, beta0: int, beta1: int, s: int) -> np.ndarray:
    """Rows beta0..beta1-1 of Omega_k (an (beta1-beta0) x s float64 array of float32 values)."""
    nb = beta1 - beta0
    ng = (s + 7) // 8
    beta = np.arange(beta0, beta1, dtype=np.uint64)[:, None]
    g = np.arange(ng, dtype=np.uint64)[None, :]
    z = np.zeros((1, 1), dtype=np.uint64)
    key0 = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    key1 = np.uint64(k)
    words = philox4x64_10(beta, g, z, z, key0, key1)
    out = np.empty((nb, ng * 8), dtype=np.float64)
    for j, x in enumerate(words):
        u = _uniform23(x & _LO32)
        v = _uniform23(x >> _S32)
        rad = np.sqrt(np.float32(-2.0) * ln32(u))
        cs, sn = cossin32(v)
        out[:, 2 * j::8] = rad * cs
        out[:, 2 * j + 1::8] = rad * sn
    return out[:, :s]
