"""FP64 adjoint of the O-B radiance map (the method's discrete operator).

The paper computes no gradients; these follow from the linearity of Eq. (7)
and (8) in the irradiance and from the chain rule through the PCA weights of
Sec. 2.2 and the dipole formula Eq. (4).  For an upstream gradient
Bbar[q, vertex, ch] (original vertex order):

    vbar: gbar[q, ch, k]    = sum_p Bbar[q, perm[p], ch] v_k[q, p, ch]
          thetabar[m, ch,:] = sum_{q: mat(q)=m} sum_k gbar[q, ch, k] dg[m, ch, k, :]
          dg[m, ch, k, :]   = sum_m' b_k[m'] dR_d(r_m'; theta[m, ch]) / dtheta
    Ebar: Ehatbar[q, :, ch] = sum_k g[mat(q), ch, k] W_k(trunc)^T Bbar[q, perm, ch]
          Ebar[q, :, ch]    = A o (H^T Ehatbar)[:N]        (Morton order)
          Lbar[l, :, ch]    = sum_{q: light(q)=l} T^T Ebar[q, :, ch]

``rows`` restricts the sum to the given Morton rows, which equals the full
adjoint for an upstream gradient supported on those rows only.
"""
from __future__ import annotations

import numpy as np

from . import haar, pca
from .transport import light_of, mat_of


def grad(scene, L, theta, Bbar, rows=None, block=64):
    """Returns (Lbar [n_light, n_sh, 3], thetabar [n_cfg, 3, 3]).

    Bbar: [n_out, len(rows) or N, 3], indexed like the Morton rows (rows
    given) or by original vertex id (rows None).
    """
    w = scene.w
    if rows is None:
        rows = np.arange(scene.N)
        Bb = np.asarray(Bbar)[:, scene.perm, :]
    else:
        rows = np.asarray(rows)
        Bb = np.asarray(Bbar)
    Eh = scene.ehat(L)                                   # [n_out, n, 3]
    g = scene.g(theta)                                   # [n_cfg, 3, K]
    dg = pca.weight_grads(theta, scene.rn, scene.b)      # [n_cfg, 3, K, 3]
    G = np.stack([g[mat_of(w, q)] for q in range(w.n_out)])   # [n_out, 3, K]
    n_cols = Eh.shape[1]
    gbar = np.zeros((w.n_out, 3, scene.K))
    ehbar = np.zeros((w.n_out, n_cols, 3))
    for s in range(0, len(rows), block):
        pr = rows[s:s + block]
        bb = Bb[:, s:s + len(pr), :]                     # [n_out, P, 3]
        cols, vals = scene.kept_lists(pr)                # [K, P, nk]
        v = np.einsum("kpn,qkpnc->kqpc", vals, Eh[:, cols, :])
        gbar += np.einsum("qpc,kqpc->qck", bb, v)
        # each kept W_k[p, j] sends g_k Bbar[p] back to column j
        contrib = np.einsum("qck,kpn,qpc->qkpnc", G, vals, bb)
        np.add.at(ehbar, (slice(None), cols.reshape(-1)), contrib.reshape(w.n_out, -1, 3))
    thbar = np.zeros((w.n_cfg, 3, 3))
    for q in range(w.n_out):
        thbar[mat_of(w, q)] += np.einsum("ck,ckp->cp", gbar[q], dg[mat_of(w, q)])
    if scene.wavelet == "none":
        ebar = ehbar
    else:
        ebar = haar.ihaar(ehbar, axis=1)[:, :scene.N, :]
    ebar = ebar * scene.area[scene.perm][None, :, None]
    Tm = scene.T[scene.perm]                             # [N, n_sh]
    Lbar = np.zeros((w.n_light, Tm.shape[1], 3))
    for q in range(w.n_out):
        Lbar[light_of(w, q)] += Tm.T @ ebar[q]
    return Lbar, thbar


def l2_loss(B, Bt):
    return 0.5 * float(np.sum((B - Bt) ** 2))


def fd_grad(scene, L, theta, Bt, rel=1e-4, floor=1e-7):
    """Central finite differences of 0.5||B(L, theta) - Bt||^2 (O-B)."""
    def loss(Lx, thx):
        return l2_loss(scene.render(Lx, thx), Bt)

    gL = np.zeros_like(L)
    for idx in np.ndindex(L.shape):
        h = max(rel * abs(L[idx]), floor)
        Lp, Lm = L.copy(), L.copy()
        Lp[idx] += h
        Lm[idx] -= h
        gL[idx] = (loss(Lp, theta) - loss(Lm, theta)) / (2 * h)
    gT = np.zeros_like(theta)
    for idx in np.ndindex(theta.shape):
        h = max(rel * abs(theta[idx]), floor)
        tp, tm = theta.copy(), theta.copy()
        tp[idx] += h
        tm[idx] -= h
        gT[idx] = (loss(L, tp) - loss(L, tm)) / (2 * h)
    return gL, gT
