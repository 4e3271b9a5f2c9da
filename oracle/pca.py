"""PCA factorisation of the dipole table -- Sec. 2.2, Eq. (5).

R_d(r, sigma) ~ sum_k S_k(sigma) b_k(r).  The table M holds R_d sampled on
512 materials (rows) x 256 distances (columns); M = U S V, and the rows of V
(right singular vectors) are the discrete basis functions b_k on the
r-nodes.  For an arbitrary material the weight is the projection of R_d onto
b_k (Sec. 2.2 and rendering Step 3 of Sec. 4):

    g_k(sigma) = sum_m R_d(r_m; sigma) b_k[m].

Readings: M is not centred; the inner product is the plain sum over the
nodes; each b_k is signed so that its entry of largest magnitude is
positive; the nodes are r_m = r_max (m/255)^2 with r_max bounding every
vertex distance; between nodes b_k is interpolated linearly in r.  The
material grid is 8x8x8 (sigma_a, sigma_s' log-spaced, eta linear).
"""
from __future__ import annotations

import numpy as np

from . import dipole


def r_nodes(r_max, n_r=256):
    m = np.arange(n_r, dtype=np.float64)
    return r_max * (m / (n_r - 1)) ** 2


def material_grid(spec):
    sa = np.geomspace(spec["sigma_a"][0], spec["sigma_a"][1], spec["sigma_a"][2])
    ss = np.geomspace(spec["sigma_s"][0], spec["sigma_s"][1], spec["sigma_s"][2])
    et = np.linspace(spec["eta"][0], spec["eta"][1], spec["eta"][2])
    g = np.stack(np.meshgrid(sa, ss, et, indexing="ij"), axis=-1).reshape(-1, 3)
    return g


def table(rn, mats):
    """M[material, node] = R_d(r_node; material)."""
    return dipole.rd(rn[None, :], mats[:, 0:1], mats[:, 1:2], mats[:, 2:3])


def basis(M, K=None):
    """Right singular vectors of M, sign-normalised -> [K or all, n_r]."""
    _, s, Vt = np.linalg.svd(M, full_matrices=False)
    idx = np.argmax(np.abs(Vt), axis=1)
    sgn = np.sign(Vt[np.arange(Vt.shape[0]), idx])
    Vt = Vt * sgn[:, None]
    if K is not None:
        Vt = Vt[:K]
    return Vt, s


def weights(theta, rn, b):
    """g[..., k] = sum_m R_d(r_m; theta) b_k[m] for theta [..., 3]."""
    th = np.asarray(theta)
    R = dipole.rd(rn, th[..., 0:1], th[..., 1:2], th[..., 2:3])   # [..., n_r]
    return R @ b.T


def weight_grads(theta, rn, b):
    """dg[..., k, p] = sum_m b_k[m] dR_d(r_m; theta)/dtheta_p."""
    th = np.asarray(theta)
    _, da, ds, de = dipole.rd_grad(rn, th[..., 0:1], th[..., 1:2], th[..., 2:3])
    return np.stack([da @ b.T, ds @ b.T, de @ b.T], axis=-1)


def interp(b, rn, r):
    """Piecewise-linear b_k(r) on the nodes: returns [K, *r.shape]."""
    return np.stack([np.interp(r, rn, bk) for bk in b])
