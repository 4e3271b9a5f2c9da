"""Radiance of the translucent object: plain gather (O-A) and method form (O-B).

Column convention.  A launch renders ``n_out`` (lighting, material) sets of 3
RGB channels.  Output set q uses lighting ``light(q)`` and material
``mat(q)``: when both counts are equal they pair up one to one, otherwise the
single lighting (or single material) is shared by every set.

O-A  (Eq. 1-4 and 6, with the Fresnel and 1/pi factors left out so that the
radiance is B = sum R_d E dA):

    B_A[q, o, ch] = sum_i R_d(|x_o - x_i|; theta[mat(q), ch]) E[q, i, ch] A_i,
    E[q, i, ch]   = sum_lm T[i, lm] L[light(q), lm, ch].

O-B  (the discrete operator the method evaluates; Eq. 7 and 8, precompute
Step 1 of Sec. 3.2, rendering Steps 1-4 of Sec. 4):

    g[m, ch, k]   = sum_m' R_d(r_m'; theta[m, ch]) b_k[m']           (Step 3)
    K_k[p, p']    = btilde_k(|x_perm[p] - x_perm[p']|)  (Morton order)  (Eq. 7)
    W_k[p, :]     = Haar(pad(K_k[p, :]))                              (Eq. 8)
    S(p, k)       = the n_keep largest |W_k[p, j]|, ties to the lower j
    Ehat[q, :, ch]= Haar(pad(A o E[q, :, ch]))  (Morton order)        (Step 1)
    B_B[q, perm[p], ch] = sum_k g[mat(q), ch, k]
                          sum_{j in S(p,k)} W_k[p, j] Ehat[q, j, ch]   (Steps 2, 4)

With wavelet = "none" W_k = K_k and Ehat = A o E (the plain matrix form of
Eq. 7).  The area weight sits on the irradiance side (Eq. 6 integrates E dA);
the rows W_k are the Haar transform of the symmetric kernel alone.
"""
from __future__ import annotations

import numpy as np

import synth

from . import dipole, geometry, haar, pca, sh


def light_of(w, q):
    return q if w.n_light > 1 else 0


def mat_of(w, q):
    return q if w.n_cfg > 1 else 0


class Scene:
    """Everything the oracle derives from the seeded mesh of a workload."""

    def __init__(self, w, V=None, F=None, K=None):
        if V is None:
            V, F = synth.make_mesh(w)
        self.w = w
        self.V, self.F = V, F
        self.N = V.shape[0]
        self.n_pad = haar.next_pow2(self.N)
        self.area = geometry.vertex_areas(V, F)
        self.normal = geometry.vertex_normals(V, F)
        self.perm = geometry.morton_perm(V)
        self.T = sh.transfer(self.normal, w.n_sh)                # original order
        self.rn = pca.r_nodes(w.r_max, synth.N_R_NODES)
        self.mats = pca.material_grid(synth.MATERIAL_GRID)
        self.M = pca.table(self.rn, self.mats)
        self.b, self.sv = pca.basis(self.M, w.K if K is None else K)
        self.K = self.b.shape[0]
        self.n_keep = w.n_keep
        self.wavelet = w.wavelet

    # -- lighting side ----------------------------------------------------
    def irradiance(self, L):
        """E[q, i, ch] in original vertex order."""
        w = self.w
        return np.stack([self.T @ L[light_of(w, q)] for q in range(w.n_out)])

    def ehat(self, L=None, E=None):
        """Ehat[q, j, ch]: Haar of the area-weighted Morton-ordered E, with
        E = T L from SH lighting L, or a given irradiance E[light, i, ch]
        (original vertex order; output set q uses light(q))."""
        if E is None:
            Eq = self.irradiance(L)
        else:
            E = np.asarray(E, dtype=np.float64)
            Eq = np.stack([E[light_of(self.w, q)] for q in range(self.w.n_out)])
        Ew = Eq[:, self.perm, :] * self.area[self.perm][None, :, None]
        if self.wavelet == "none":
            return Ew
        return haar.haar(haar.pad(Ew, self.n_pad, axis=1), axis=1)

    # -- material side ----------------------------------------------------
    def g(self, theta):
        """g[m, ch, k]."""
        return pca.weights(theta, self.rn, self.b)

    # -- transport rows ---------------------------------------------------
    def kernel_rows(self, p_rows):
        """K_k[p, p'] for Morton positions p_rows -> [K, len(p_rows), N]."""
        Vm = self.V[self.perm]
        d = Vm[p_rows][:, None, :] - Vm[None, :, :]
        r = np.sqrt(np.einsum("abi,abi->ab", d, d))
        return pca.interp(self.b, self.rn, r)

    def wavelet_rows(self, p_rows):
        """Untruncated W_k rows [K, len(p_rows), n_cols] in float64."""
        Kr = self.kernel_rows(p_rows)
        if self.wavelet == "none":
            return Kr
        return haar.haar(haar.pad(Kr, self.n_pad, axis=-1), axis=-1)

    def select(self, Wr):
        """Boolean mask of the kept set S over the last axis of Wr.

        Keeps the n_keep entries of largest magnitude; among equal
        magnitudes the lower index wins.
        """
        n = Wr.shape[-1]
        nk = min(self.n_keep, n)
        if nk >= n:
            return np.ones(Wr.shape, dtype=bool)
        a = np.abs(Wr)
        thr = np.partition(a, n - nk, axis=-1)[..., n - nk:n - nk + 1]
        gt = a > thr
        need = nk - gt.sum(axis=-1, keepdims=True)
        eq = a == thr
        eq_rank = np.cumsum(eq, axis=-1)
        return gt | (eq & (eq_rank <= need))

    def truncated_rows(self, p_rows):
        """(W rows with dropped entries zeroed, kept mask), both [K, P, n]."""
        Wr = self.wavelet_rows(p_rows)
        keep = self.select(Wr)
        return np.where(keep, Wr, 0.0), keep

    def kept_lists(self, p_rows):
        """Kept (cols, vals) per row, cols ascending: [K, P, n_keep] each."""
        Wt, keep = self.truncated_rows(p_rows)
        Kk, P, n = keep.shape
        nk = min(self.n_keep, n)
        cols = np.nonzero(keep.reshape(-1, n))[1].reshape(Kk, P, nk)
        vals = np.take_along_axis(Wt, cols, axis=-1)
        return cols, vals

    def transport(self, p_rows, Eh):
        """v[k, q, p, ch] = sum over j in S(p, k) of W_k[p, j] Ehat[q, j, ch]."""
        cols, vals = self.kept_lists(p_rows)            # [K, P, nk]
        return np.einsum("kpn,qkpnc->kqpc", vals, Eh[:, cols, :])

    # -- radiance ---------------------------------------------------------
    def render_rows(self, L, theta, p_rows, block=64, keep_v=False, E=None):
        """O-B radiance at Morton positions p_rows -> B[q, len(p_rows), ch].

        With keep_v also returns v[k, q, P, ch] = sum_j W_k[p, j] Ehat[q, j, ch].
        """
        w = self.w
        Eh = self.ehat(L, E)                    # [n_out, n, 3]
        g = self.g(theta)                       # [n_cfg, 3, K]
        G = np.stack([g[mat_of(w, q)] for q in range(w.n_out)])   # [n_out,3,K]
        p_rows = np.asarray(p_rows)
        B = np.zeros((w.n_out, len(p_rows), 3))
        V = np.zeros((self.K, w.n_out, len(p_rows), 3)) if keep_v else None
        for s in range(0, len(p_rows), block):
            pr = p_rows[s:s + block]
            v = self.transport(pr, Eh)                  # [K, n_out, P, 3]
            B[:, s:s + len(pr), :] = np.einsum("qck,kqpc->qpc", G, v)
            if keep_v:
                V[:, :, s:s + len(pr), :] = v
        return (B, V) if keep_v else B

    def render(self, L, theta, block=64, E=None):
        """O-B radiance for every vertex, original order -> [n_out, N, 3]."""
        Bm = self.render_rows(L, theta, np.arange(self.N), block=block, E=E)
        B = np.empty_like(Bm)
        B[:, self.perm, :] = Bm
        return B

    def render_vertices(self, L, theta, vertex_ids, block=64):
        """O-B radiance at original vertex ids -> [n_out, len(ids), 3]."""
        inv = np.empty(self.N, dtype=np.int64)
        inv[self.perm] = np.arange(self.N)
        return self.render_rows(L, theta, inv[np.asarray(vertex_ids)], block=block)

    # -- plain gather (O-A) -----------------------------------------------
    def gather_plain(self, L, theta, vertex_ids=None, interpolated=False, block=128):
        """O-A: brute-force dipole gather at original vertex ids.

        interpolated=True replaces R_d by its piecewise-linear interpolant on
        the r-nodes (O-A'), which O-B reproduces exactly at full rank and
        without truncation.
        """
        w = self.w
        ids = np.arange(self.N) if vertex_ids is None else np.asarray(vertex_ids)
        E = self.irradiance(L) * self.area[None, :, None]     # [n_out, N, 3]
        out = np.zeros((w.n_out, len(ids), 3))
        for s in range(0, len(ids), block):
            vi = ids[s:s + block]
            d = self.V[vi][:, None, :] - self.V[None, :, :]
            r = np.sqrt(np.einsum("abi,abi->ab", d, d))
            for q in range(w.n_out):
                th = theta[mat_of(w, q)]
                for ch in range(3):
                    if interpolated:
                        Rt = np.interp(r, self.rn, dipole.rd(self.rn, *th[ch]))
                    else:
                        Rt = dipole.rd(r, *th[ch])
                    out[q, s:s + len(vi), ch] = Rt @ E[q, :, ch]
        return out
