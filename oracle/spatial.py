"""Spatial (output-side) compression of the truncated transport and its
rendering form -- Sec. 3.2 (Eq. 9, 10; precompute Step 2), Steps 2, 4 and 5
of Sec. 4.

TEST INFRASTRUCTURE ONLY (see the package header).

Given the Step-1 rows W_k^S (each row (p, k) keeps its n_keep coefficients,
the rest zeroed; ``transport.Scene``), per PCA term k:

    Z_k[u, j] = (w_1 W_k^S[:, j])[u]       w_1 = CDF 9/7 along the Morton-
                                            ordered output index (``cdf97``)
    S2(k)     = the fewest entries of Z_k, largest |z| first (ties to the
                lower flat index u * n_cols + j), whose energy sum of z^2
                reaches tau times the energy of all of Z_k
    y[q, u, ch]       = sum_k g[mat(q), ch, k] sum_{(u, j) in S2(k)} Z_k[u, j] Ehat[q, j, ch]
    B[q, perm[p], ch] = (w_1^{-1} y[q, :, ch])[p]

With tau = 1 every non-zero coefficient is kept (also those too small to
move the float64 energy sum) and, w_1 being invertible, B equals the Step-1
radiance exactly.
"""
from __future__ import annotations

import numpy as np

from . import cdf97
from .transport import mat_of


class Spatial:
    def __init__(self, scene, energy: float, levels: int = 0):
        if not 0.0 < energy <= 1.0:
            raise ValueError("energy fraction must be in (0, 1]")
        self.sc = scene
        self.energy = energy
        self.levels = levels
        self.sizes = cdf97.band_sizes(scene.N, levels)
        Wt, _ = scene.truncated_rows(np.arange(scene.N))          # [K, N, n]
        self.Z = np.stack([cdf97.forward(Wt[k], levels) for k in range(Wt.shape[0])])
        self.keep = self.select(energy)

    def select(self, energy: float):
        """Boolean kept mask [K, N, n] of S2 for the given energy fraction."""
        Kk, N, n = self.Z.shape
        keep = np.zeros(self.Z.shape, dtype=bool)
        flat_idx = np.arange(N * n)
        if energy >= 1.0:
            return self.Z != 0.0                     # all of it, however small
        for k in range(Kk):
            a = np.abs(self.Z[k]).ravel()
            order = np.lexsort((flat_idx, -a))       # |z| descending, then index
            cum = np.cumsum(a[order] ** 2)
            if cum[-1] == 0.0:
                continue
            cut = int(np.searchsorted(cum, energy * cum[-1]))   # first cum >= tau * total
            keep[k].ravel()[order[:cut + 1]] = True
        return keep

    def stats(self, keep=None):
        """(kept entries per term [K], retained energy fraction per term [K])."""
        keep = self.keep if keep is None else keep
        z2 = self.Z ** 2
        tot = z2.reshape(z2.shape[0], -1).sum(axis=1)
        kept = np.where(keep, z2, 0.0).reshape(z2.shape[0], -1).sum(axis=1)
        return keep.reshape(keep.shape[0], -1).sum(axis=1), kept / np.where(tot > 0, tot, 1.0)

    def render(self, L, theta, keep=None, E=None):
        """Radiance [n_out, N, 3] (original vertex order) with kept set
        ``keep`` (default: this object's S2)."""
        sc, w = self.sc, self.sc.w
        keep = self.keep if keep is None else keep
        Eh = sc.ehat(L, E)                                         # [n_out, n, 3]
        g = sc.g(theta)                                            # [m, ch, k]
        y = np.zeros((w.n_out, sc.N, 3))
        for k in range(self.Z.shape[0]):
            Zk = np.where(keep[k], self.Z[k], 0.0)
            for q in range(w.n_out):
                y[q] += (Zk @ Eh[q]) * g[mat_of(w, q), :, k][None, :]
        B = np.empty_like(y)
        for q in range(w.n_out):
            B[q][sc.perm] = cdf97.inverse(y[q], self.levels)
        return B
