"""Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11) and the Gaussian random matrices built from it.

The paper draws its random vectors from rand() or a Mersenne Twister,
post-processed to a uniform or normal distribution (Sec. 3.2).  Those
generators are sequential; a counter-based generator instead gives every
entry of R^r and R^c directly from its (row, column) address, so columns
appended when d grows (Sec. 3.3) never depend on the growth history.

Definition used here (independently implemented on the GPU side):

* one Philox4x64-10 call with key (seed, 0) and counter (q, j, s, 0) yields
  four 64-bit words w0..w3 for column j of stream s (s = 0 for R^r, 1 for
  R^c) and rows 4q .. 4q+3;
* each word becomes u = ((w >> 12) + 1/2) * 2^-52, a uniform in (0, 1)
  (exact in float64: 53 significant bits at most);
* Box-Muller: (u0, u1) -> rows 4q, 4q+1 and (u2, u3) -> rows 4q+2, 4q+3 as
  r cos(2 pi u_b), r sin(2 pi u_b) with r = sqrt(-2 ln u_a).

Pins: the raw words equal NumPy's own Philox bit generator (a library
implementation of the same published function); the normals pass mean,
variance and Kolmogorov-Smirnov checks.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.uint64, b: np.ndarray):
    """128-bit product of the 64-bit constant a and the array b, as (hi, lo)."""
    a_lo = a & _LO32
    a_hi = a >> _S32
    b_lo = b & _LO32
    b_hi = b >> _S32
    p00 = a_lo * b_lo
    p01 = a_lo * b_hi
    p10 = a_hi * b_lo
    p11 = a_hi * b_hi
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """ctr: (..., 4) uint64, key: (..., 2) uint64 (broadcastable).
    Returns (..., 4) uint64 output words."""
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.array(ctr[..., i], dtype=np.uint64) for i in range(4))
        k0 = np.array(key[..., 0], dtype=np.uint64)
        k1 = np.array(key[..., 1], dtype=np.uint64)
        for _ in range(10):
            hi0, lo0 = _mulhilo(_M0, c0)
            hi1, lo1 = _mulhilo(_M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            k0 = k0 + _W0
            k1 = k1 + _W1
    return np.stack(np.broadcast_arrays(c0, c1, c2, c3), axis=-1)


def uniform_from_words(w: np.ndarray) -> np.ndarray:
    """u = ((w >> 12) + 0.5) * 2^-52, exactly representable, in (0, 1)."""
    return ((w >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def gaussian_columns(seed: int, stream: int, n: int, col0: int, col1: int) -> np.ndarray:
    """Rows 0..n-1, columns col0..col1-1 of the Gaussian matrix of the given
    stream (0 = R^r, 1 = R^c).  Returns an n x (col1-col0) float64 array."""
    ncol = col1 - col0
    nq = (n + 3) // 4
    out = np.empty((nq * 4, ncol))
    if ncol == 0 or n == 0:
        return out[:n]
    q = np.arange(nq, dtype=np.uint64)
    two_pi = 2.0 * np.pi
    for jj, j in enumerate(range(col0, col1)):
        ctr = np.zeros((nq, 4), dtype=np.uint64)
        ctr[:, 0] = q
        ctr[:, 1] = np.uint64(j)
        ctr[:, 2] = np.uint64(stream)
        key = np.array([seed, 0], dtype=np.uint64)
        w = philox4x64_10(ctr, key)
        u = uniform_from_words(w)
        r01 = np.sqrt(-2.0 * np.log(u[:, 0]))
        r23 = np.sqrt(-2.0 * np.log(u[:, 2]))
        t01 = two_pi * u[:, 1]
        t23 = two_pi * u[:, 3]
        col = np.empty((nq, 4))
        col[:, 0] = r01 * np.cos(t01)
        col[:, 1] = r01 * np.sin(t01)
        col[:, 2] = r23 * np.cos(t23)
        col[:, 3] = r23 * np.sin(t23)
        out[:, jj] = col.reshape(-1)
    return out[:n]
