"""Orthonormal 1-D Haar transform -- Eq. (8); Haar per Sec. 5.

For x of length 2^n the transform repeats, from the finest level up,
    s'[i] = (s[2i] + s[2i+1]) / sqrt(2),   d[i] = (s[2i] - s[2i+1]) / sqrt(2)
and lays the result out coarse to fine:
    [ s^(0)[0], d^(0)[0], d^(1)[0..1], d^(2)[0..3], ..., d^(n-1)[0..2^(n-1)-1] ]
so coefficient j >= 1 of level m = floor(log2 j) covers the dyadic block
b = j - 2^m of length 2^(n-m).  The matrix H is orthogonal (H^T H = I), so
(T H^T)(H E) = T E as Eq. (8) requires.  Lists shorter than a power of two
are zero-padded at the end.
"""
from __future__ import annotations

import numpy as np

INV_SQRT2 = 1.0 / np.sqrt(2.0)


def next_pow2(n: int) -> int:
    return 1 << (int(n) - 1).bit_length()


def pad(x, n_pad, axis=-1):
    x = np.asarray(x)
    width = [(0, 0)] * x.ndim
    width[axis] = (0, n_pad - x.shape[axis])
    return np.pad(x, width)


def haar(x, axis=-1):
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    n = x.shape[-1]
    assert n & (n - 1) == 0, "length must be a power of two"
    parts = []
    s = x
    while s.shape[-1] > 1:
        a, b = s[..., 0::2], s[..., 1::2]
        parts.append((a - b) * INV_SQRT2)
        s = (a + b) * INV_SQRT2
    parts.append(s)
    out = np.concatenate(parts[::-1], axis=-1)
    return np.moveaxis(out, -1, axis)


def ihaar(c, axis=-1):
    c = np.moveaxis(np.asarray(c, dtype=np.float64), axis, -1)
    n = c.shape[-1]
    s = c[..., 0:1]
    m = 1
    while m < n:
        d = c[..., m:2 * m]
        nxt = np.empty(c.shape[:-1] + (2 * m,))
        nxt[..., 0::2] = (s + d) * INV_SQRT2
        nxt[..., 1::2] = (s - d) * INV_SQRT2
        s = nxt
        m *= 2
    return np.moveaxis(s, -1, axis)


def matrix(n):
    """Dense H (n x n) with H @ x == haar(x)."""
    return haar(np.eye(n), axis=0)
