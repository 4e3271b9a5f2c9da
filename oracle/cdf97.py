"""CDF 9/7 biorthogonal wavelet along the Morton-ordered output list -- the
spatial transform w_1 of Sec. 3.2 (Eq. 9, 10), 9/7 per Sec. 5.

TEST INFRASTRUCTURE ONLY (see the package header).

Filters, from their definition.  With y = sin^2(w/2) the Daubechies
half-band product for four vanishing moments is
    P(y) = 1 + 4 y + 10 y^2 + 20 y^3 .
The 9/7 pair splits P at its one real root r:
    analysis low-pass   h(w) ~ cos^4(w/2) * P(y) / (1 - y/r)     (9 taps)
    synthesis low-pass  f(w) ~ cos^4(w/2) * (1 - y/r)             (7 taps)
each scaled to a DC gain of sqrt(2) (near-orthonormal), and the analysis
high-pass is the modulated synthesis low-pass, g[m] = (-1)^m f[m], centred
on the odd sample (Nyquist gain sqrt(2)).

One level on a list x of length n >= 8, with whole-sample symmetric
extension (x[-i] = x[i], x[n-1+i] = x[n-1-i]):
    low[i]  = sum_{m=-4..4} h[m] x[2i + m],      i < ceil(n/2)
    high[i] = sum_{m=-3..3} g[m] x[2i + 1 + m],  i < floor(n/2)
Levels repeat on the low band while it has at least 8 entries (or for a
given number of levels); the coefficients are laid out coarse to fine:
    [ low_J, high_J, high_{J-1}, ..., high_1 ].
The inverse w_1^{-1} (Step 5 of Sec. 4) is the exact inverse of this
analysis operator, taken level by level with a sparse solve.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

MIN_SPLIT = 8          # a level splits a list of at least this many entries


@functools.lru_cache(maxsize=None)
def filters():
    """(h [9], g [7], r): analysis low-pass h[-4..4], analysis high-pass
    g[-3..3] and the real root r of P."""
    roots = np.roots([20.0, 10.0, 4.0, 1.0])
    r = float(roots[np.abs(roots.imag) < 1e-12].real[0])
    # Laurent coefficient arrays (centred) of cos^2(w/2) and y = sin^2(w/2)
    c2 = np.array([0.25, 0.5, 0.25])
    y1 = np.array([-0.25, 0.5, -0.25])
    y2 = np.convolve(y1, y1)
    # P(y) / (1 - y/r) = q0 + q1 y + q2 y^2 (exact division: r is a root)
    q2, q1, q0 = np.polydiv([20.0, 10.0, 4.0, 1.0], [-1.0 / r, 1.0])[0]
    q = q0 * np.pad([1.0], 2) + q1 * np.pad(y1, 1) + q2 * y2
    c4 = np.convolve(c2, c2)
    h = np.convolve(c4, q)
    f = np.convolve(c4, np.array([0.0, 1.0, 0.0]) - y1 / r)
    h *= np.sqrt(2.0) / h.sum()
    f *= np.sqrt(2.0) / f.sum()
    g = f * (-1.0) ** np.abs(np.arange(-3, 4))
    return h, g, r


def band_sizes(n: int, levels: int = 0):
    """Lengths of the lists split at each level, finest first ([n, ceil(n/2),
    ...]); ``levels`` = 0 splits while the list has at least 8 entries."""
    sizes = []
    while n >= MIN_SPLIT and (levels == 0 or len(sizes) < levels):
        sizes.append(n)
        n = (n + 1) // 2
    if levels and len(sizes) < levels:
        raise ValueError(f"{levels} levels need at least {MIN_SPLIT} entries at the coarsest")
    return sizes


def _fold(i: int, n: int) -> int:
    """Whole-sample symmetric extension index (one reflection suffices for
    the filter reach when n >= 8)."""
    if i < 0:
        i = -i
    if i > n - 1:
        i = 2 * (n - 1) - i
    return i


@functools.lru_cache(maxsize=64)
def analysis_matrix(n: int):
    """One level as a sparse n x n matrix: rows [low; high]."""
    h, g, _ = filters()
    rows, cols, vals = [], [], []
    n_lo = (n + 1) // 2
    for i in range(n_lo):
        for m in range(-4, 5):
            rows.append(i)
            cols.append(_fold(2 * i + m, n))
            vals.append(h[m + 4])
    for i in range(n // 2):
        for m in range(-3, 4):
            rows.append(n_lo + i)
            cols.append(_fold(2 * i + 1 + m, n))
            vals.append(g[m + 3])
    # duplicates (reflected taps landing on one sample) are summed
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def forward(x, levels: int = 0):
    """w_1 along axis 0 of x [n, ...] -> coefficients [n, ...]."""
    x = np.asarray(x, dtype=np.float64)
    out = x.reshape(x.shape[0], -1).copy()
    for n in band_sizes(x.shape[0], levels):
        out[:n] = analysis_matrix(n) @ out[:n]
    return out.reshape(x.shape)


def inverse(z, levels: int = 0):
    """w_1^{-1} along axis 0: solves each level's analysis system, coarsest
    first."""
    z = np.asarray(z, dtype=np.float64)
    out = z.reshape(z.shape[0], -1).copy()
    for n in reversed(band_sizes(z.shape[0], levels)):
        lu = spla.splu(analysis_matrix(n).tocsc())
        out[:n] = lu.solve(out[:n])
    return out.reshape(z.shape)
