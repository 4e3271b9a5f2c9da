"""Real spherical harmonics and the unshadowed clamped-cosine transfer.

The irradiance E(x_i) of Eq. (6) (and Eq. 11 with visibility V = 1, no
Fresnel factor, as in precomputed radiance transfer of Sloan et al., which
the paper builds on in Sec. 3) is E_i = sum_lm T[i,lm] L[lm] with

    T[i, lm] = int_S2 max(n_i . w, 0) Y_lm(w) dw = Ahat_l Y_lm(n_i)

(Funk-Hecke), where Ahat_l = 2 pi int_0^1 t P_l(t) dt.  E is not clamped, so
E is linear in L and can be negative.

Basis: real orthonormal SH, index l*l + l + m (l-major, m = -l..l), without
the Condon-Shortley phase:
    Y_l0  = K_l0 P_l(z)
    Y_lm  = sqrt(2) K_lm Re[(x+iy)^m] Pt_l^m(z)   (m > 0)
    Y_l-m = sqrt(2) K_lm Im[(x+iy)^m] Pt_l^m(z)   (m > 0)
with K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and Pt_l^m = P_l^m / sin^m.
"""
from __future__ import annotations

import math

import numpy as np


def n_coeffs(lmax: int) -> int:
    return (lmax + 1) ** 2


def lmax_of(n_sh: int) -> int:
    l = int(round(math.sqrt(n_sh))) - 1
    assert (l + 1) ** 2 == n_sh, n_sh
    return l


def _pt(lmax, z):
    """Pt[l][m] = associated Legendre P_l^m(z) / (1-z^2)^(m/2), m >= 0."""
    P = [[None] * (lmax + 1) for _ in range(lmax + 1)]
    for m in range(lmax + 1):
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        P[m][m] = np.full_like(z, dfact)
        if m + 1 <= lmax:
            P[m + 1][m] = z * (2 * m + 1) * P[m][m]
        for l in range(m + 2, lmax + 1):
            P[l][m] = ((2 * l - 1) * z * P[l - 1][m] - (l + m - 1) * P[l - 2][m]) / (l - m)
    return P


def real_sh(lmax, dirs):
    """Y[..., l*l+l+m] for unit direction(s) ``dirs`` [..., 3]."""
    dirs = np.asarray(dirs, dtype=np.float64)
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    P = _pt(lmax, z)
    out = np.empty(dirs.shape[:-1] + (n_coeffs(lmax),))
    xy = x + 1j * y
    powm = [np.ones_like(xy)]
    for m in range(1, lmax + 1):
        powm.append(powm[-1] * xy)
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            K = math.sqrt((2 * l + 1) / (4 * math.pi)
                          * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                out[..., l * l + l] = K * P[l][0]
            else:
                c = math.sqrt(2.0) * K * P[l][m]
                out[..., l * l + l + m] = c * powm[m].real
                out[..., l * l + l - m] = c * powm[m].imag
    return out


def legendre(l, t):
    return _pt(l, np.asarray(t, dtype=np.float64))[l][0]


def clamped_cosine_coeffs(lmax):
    """Ahat_l = 2 pi int_0^1 t P_l(t) dt by Gauss-Legendre (exact here)."""
    t, wts = np.polynomial.legendre.leggauss(32)
    t = 0.5 * (t + 1.0)
    wts = 0.5 * wts
    return np.array([2.0 * math.pi * np.sum(wts * t * legendre(l, t))
                     for l in range(lmax + 1)])


def transfer(normals, n_sh):
    """T[i, lm] = Ahat_l Y_lm(n_i)  -> [N, n_sh] float64."""
    lmax = lmax_of(n_sh)
    Y = real_sh(lmax, normals)
    ah = clamped_cosine_coeffs(lmax)
    scale = np.concatenate([np.full(2 * l + 1, ah[l]) for l in range(lmax + 1)])
    return Y * scale[None, :]
