"""Counter-based normal deviates for the Gaussian white noise.

The paper does not say how its Gaussian realisation is drawn (Sec. VI A only
calls Phi Gaussian).  Here one standard normal per lattice site comes from

* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): key = (seed, 0), counter = (site, 0, 0, 0), where
  site = (x N + y) N + z;
* two uniforms in (0, 1) from output words 0 and 1:
  u = (2 (w >> 12) + 1) * 2^-53, exact in binary64;
* Box-Muller (cosine branch): w = sqrt(-2 ln u1) * cos(2 pi u2).

The logarithm and the cosine are defined below by an explicit sequence of
IEEE-754 binary64 additions, subtractions, multiplications and divisions
(plus exact frexp/floor), with no fused multiply-add, so that any
implementation that follows the same sequence produces the same bits:

ln(u):  u = m 2^e with m in [1, 2); if m > sqrt(2): m /= 2, e += 1;
        s = (m - 1)/(m + 1); z = s s;
        p = Horner_z(1/1, 1/3, 1/5, ..., 1/25)  (13 coefficients 1/(2k+1));
        ln u = e * LN2 + (s + s) * p.
cos(2 pi u), u in (0, 1):
        t = 4u; q = floor(t); f = t - q;
        g = 1 - f if f > 1/2 else f;  x = g * (pi/2); z = x x;
        C = Horner_z((-1)^k/(2k)!,   k = 0..9);
        S = x * Horner_z((-1)^k/(2k+1)!, k = 0..9);
        (cf, sf) = (S, C) if f > 1/2 else (C, S)   # cos, sin of pi f / 2
        result = [cf, -sf, -cf, sf][q].
"""
from __future__ import annotations

import math

import numpy as np

U64 = np.uint64
M32 = U64(0xFFFFFFFF)
PHILOX_M0 = U64(0xD2E7470EE14C6C93)
PHILOX_M1 = U64(0xCA5A826395121157)
PHILOX_W0 = U64(0x9E3779B97F4A7C15)
PHILOX_W1 = U64(0xBB67AE8584CAA73B)

LN2 = 0.6931471805599453
SQRT2 = 1.4142135623730951
PIO2 = 1.5707963267948966
LN_COEF = [1.0 / (2 * k + 1) for k in range(13)]
COS_COEF = [(-1) ** k / math.factorial(2 * k) for k in range(10)]
SIN_COEF = [(-1) ** k / math.factorial(2 * k + 1) for k in range(10)]


def _mulhilo(a: np.ndarray, b: np.uint64):
    """Full 64x64 -> 128-bit product as (hi, lo), from 32-bit halves."""
    a0 = a & M32
    a1 = a >> U64(32)
    b0 = b & M32
    b1 = b >> U64(32)
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> U64(32)) + (p01 & M32) + (p10 & M32)
    hi = p11 + (p01 >> U64(32)) + (p10 >> U64(32)) + (mid >> U64(32))
    lo = a * b
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on 4x64-bit counters (arrays) with a 2x64-bit key."""
    with np.errstate(over="ignore"):
        c = [np.asarray(c0, dtype=U64), np.asarray(c1, dtype=U64),
             np.asarray(c2, dtype=U64), np.asarray(c3, dtype=U64)]
        k = [U64(k0), U64(k1)]
        for r in range(10):
            if r > 0:
                k = [k[0] + PHILOX_W0, k[1] + PHILOX_W1]
            hi0, lo0 = _mulhilo(c[0], PHILOX_M0)
            hi1, lo1 = _mulhilo(c[2], PHILOX_M1)
            c = [hi1 ^ c[1] ^ k[0], lo1, hi0 ^ c[3] ^ k[1], lo0]
    return c


def uniform_open(w: np.ndarray) -> np.ndarray:
    """(2 (w >> 12) + 1) * 2^-53: an exact binary64 uniform in (0, 1)."""
    j = (w >> U64(12)).astype(np.float64)
    return (j * 2.0 + 1.0) * (2.0 ** -53)


def _horner(z, coef):
    p = np.full_like(z, coef[-1])
    for c in reversed(coef[:-1]):
        p = p * z
        p = p + c
    return p


def ln_spec(u: np.ndarray) -> np.ndarray:
    u = np.asarray(u, dtype=np.float64)
    m0, e0 = np.frexp(u)
    m = m0 * 2.0
    e = (e0 - 1).astype(np.float64)
    big = m > SQRT2
    m = np.where(big, m * 0.5, m)
    e = np.where(big, e + 1.0, e)
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    p = _horner(z, LN_COEF)
    t = s + s
    return e * LN2 + t * p


def cos2pi_spec(u: np.ndarray) -> np.ndarray:
    u = np.asarray(u, dtype=np.float64)
    t = u * 4.0
    q = np.floor(t)
    f = t - q
    hi = f > 0.5
    g = np.where(hi, 1.0 - f, f)
    x = g * PIO2
    z = x * x
    C = _horner(z, COS_COEF)
    S = x * _horner(z, SIN_COEF)
    cf = np.where(hi, S, C)
    sf = np.where(hi, C, S)
    qi = q.astype(np.int64)
    return np.choose(qi, [cf, -sf, -cf, sf])


def normals_from_words(w0: np.ndarray, w1: np.ndarray) -> np.ndarray:
    u1 = uniform_open(w0)
    u2 = uniform_open(w1)
    lnu = ln_spec(u1)
    r = np.sqrt(lnu * -2.0)
    return r * cos2pi_spec(u2)


def site_words(seed: int, sites: np.ndarray):
    z = np.zeros_like(sites, dtype=U64)
    return philox4x64_10(sites.astype(U64), z, z, z, seed, 0)


def white_noise(N: int, seed: int, chunk: int = 1 << 22) -> np.ndarray:
    """One N(0,1) deviate per site, site = (x N + y) N + z, as an N^3 array."""
    total = N ** 3
    out = np.empty(total, dtype=np.float64)
    for start in range(0, total, chunk):
        sites = np.arange(start, min(total, start + chunk), dtype=np.uint64)
        w = site_words(seed, sites)
        out[start:start + len(sites)] = normals_from_words(w[0], w[1])
    return out.reshape(N, N, N)
