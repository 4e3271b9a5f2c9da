"""Seeded synthetic inputs shared by the oracle and the GPU library's tests.

This module holds no arithmetic of the rendering method.  It only draws the
objects the method is applied to: an icosphere surface with radial noise, SH
lighting coefficients, dipole material parameters, and sampled row indices,
plus the numeric recipe of each workload (sizes, seeds, ranges).  Everything
the method computes from these (areas, normals, Morton order, SH transfer,
the PCA basis, transport rows, irradiance, radiance) is implemented twice,
independently: once in ``oracle/`` and once in the HIP library.

The paper's own test objects (Angel, Beethoven, Candle; Sec. 5) are not
available; icospheres of 642 .. 163842 vertices stand in for them, with the
paper's compression levels (about 1% of the Haar coefficients per row, Sec. 5)
at the largest size.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---------------------------------------------------------------------------
# Workload recipes.
# ---------------------------------------------------------------------------


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    subdiv: int            # icosphere subdivision level, N = 10*4^s + 2
    radius: float          # mm
    noise: float           # radial noise half-width (fraction of radius)
    n_sh: int              # SH coefficients per channel ((lmax+1)^2)
    K: int                 # PCA terms
    keep: float | None     # fraction of N kept per (row, k); None = untruncated
    storage: str           # "f64" | "f32" | "bf16" | "f16"  (W and T storage)
    wavelet: str           # "haar" | "none" (plain spatial form of Eq. 7)
    n_light: int           # SH lighting sets per launch
    n_cfg: int             # material sets per launch
    seed: int              # base of the per-workload seeds
    sample_rows: int = 0   # >0: parity on this many seeded sampled output rows
    description: str = ""

    @property
    def n_vertices(self) -> int:
        return 10 * 4 ** self.subdiv + 2

    @property
    def n_pad(self) -> int:
        n = self.n_vertices
        return 1 << (n - 1).bit_length()

    @property
    def n_keep(self) -> int:
        if self.keep is None:
            return self.n_pad if self.wavelet == "haar" else self.n_vertices
        return int(round(self.keep * self.n_vertices))

    @property
    def n_out(self) -> int:
        return max(self.n_light, self.n_cfg)

    @property
    def r_max(self) -> float:
        # Upper bound of any vertex-to-vertex distance on the noisy sphere.
        return 2.0 * self.radius * (1.0 + self.noise)

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# Material sample set used to build the PCA table M (512 materials):
# an 8x8x8 grid, sigma_a and sigma_s' log-spaced, eta linear.
MATERIAL_GRID = dict(
    sigma_a=(5e-4, 0.1, 8),
    sigma_s=(0.25, 4.0, 8),
    eta=(1.1, 1.6, 8),
)
N_R_NODES = 256            # r samples of the dipole table; r_m = r_max*(m/255)^2

# Material draw ranges per RGB channel.
SIGMA_A_RANGE = (0.001, 0.05)     # 1/mm
SIGMA_S_RANGE = (0.5, 3.0)        # 1/mm (reduced scattering sigma_s')
ETA_DEFAULT = 1.3

WORKLOADS = {
    "dense-f64-642": Workload("dense-f64-642", subdiv=3, radius=10.0, noise=0.02, n_sh=16, K=4,
                   keep=None, storage="f64", wavelet="none", n_light=1,
                   n_cfg=1, seed=1,
                   description="plain method, FP64, dense transport, N=642"),
    "haar-f32-10242": Workload("haar-f32-10242", subdiv=5, radius=10.0, noise=0.02, n_sh=25, K=6,
                   keep=0.05, storage="f32", wavelet="haar", n_light=1,
                   n_cfg=1, seed=2,
                   description="FP32 wavelet-sparse, N=10242, 5% kept"),
    "grad-f64-642": Workload("grad-f64-642", subdiv=3, radius=10.0, noise=0.02, n_sh=25, K=4,
                   keep=None, storage="f64", wavelet="none", n_light=1,
                   n_cfg=1, seed=3,
                   description="differentiable, N=642, 75 SH coefficients"),
    "batch64-bf16-40962": Workload("batch64-bf16-40962", subdiv=6, radius=10.0, noise=0.02, n_sh=25, K=8,
                   keep=0.02, storage="bf16", wavelet="haar", n_light=64,
                   n_cfg=64, seed=4,
                   description="batched BF16, N=40962, 2% kept, 64 pairs"),
    "large-f16-163842": Workload("large-f16-163842", subdiv=7, radius=10.0, noise=0.02, n_sh=36, K=8,
                   keep=0.01, storage="f16", wavelet="haar", n_light=16,
                   n_cfg=1, seed=5, sample_rows=2048,
                   description="large FP16, N=163842, 1% kept, 16 lights"),
}


def seeds(w: Workload) -> dict:
    """Per-purpose seeds of a workload."""
    return dict(mesh=12339 + w.seed, light=22030 + w.seed,
                material=31000 + w.seed, rows=41000 + w.seed,
                target=51000 + w.seed, probe=61000 + w.seed,
                irradiance=71000 + w.seed)


# ---------------------------------------------------------------------------
# Icosphere with radial noise.
# ---------------------------------------------------------------------------

def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
    ], dtype=np.float64)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    # Orient every face counter-clockwise seen from outside.
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


def icosphere(subdiv: int):
    """Unit icosphere: returns (vertices [N,3] float64, faces [F,3] int64).

    Each level splits every triangle into four, projecting the new edge
    midpoints onto the unit sphere; N = 10*4^s + 2.
    """
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(subdiv):
        cache: dict = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            idx = cache.get(key)
            if idx is None:
                m = np.add(verts[i], verts[j]) * 0.5
                m = m / np.linalg.norm(m)
                verts.append(tuple(m))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int64)
    return np.array(verts, dtype=np.float64), f


def make_mesh(w: Workload):
    """Noisy icosphere of workload ``w``: (vertices [N,3] mm, faces [F,3]).

    Every vertex is moved radially to R*(1+u), u ~ U[-noise, noise] i.i.d.
    """
    v, f = icosphere(w.subdiv)
    rng = np.random.default_rng(seeds(w)["mesh"])
    u = rng.uniform(-w.noise, w.noise, size=v.shape[0])
    return v * (w.radius * (1.0 + u))[:, None], f


# ---------------------------------------------------------------------------
# Lighting and materials.
# ---------------------------------------------------------------------------

def make_lighting(w: Workload, n_light: int | None = None, seed=None):
    """SH lighting [n_light, n_sh, 3] ~ N(0,1), DC coefficient made positive."""
    n = w.n_light if n_light is None else n_light
    rng = np.random.default_rng(seeds(w)["light"] if seed is None else seed)
    L = rng.standard_normal((n, w.n_sh, 3))
    L[:, 0, :] = np.abs(L[:, 0, :])
    return L


def make_irradiance(w: Workload, n_light: int | None = None, seed=None):
    """A per-vertex irradiance [n_light, N, 3] ~ U(0, 2), original vertex
    order: an input supplied in place of SH lighting (e.g. from a shadowing
    or local-light pass)."""
    n = w.n_light if n_light is None else n_light
    rng = np.random.default_rng(seeds(w)["irradiance"] if seed is None else seed)
    return rng.uniform(0.0, 2.0, size=(n, w.n_vertices, 3))


def make_materials(w: Workload, n_cfg: int | None = None, seed=None):
    """Materials [n_cfg, 3 channels, (sigma_a, sigma_s', eta)] in 1/mm."""
    n = w.n_cfg if n_cfg is None else n_cfg
    rng = np.random.default_rng(seeds(w)["material"] if seed is None else seed)
    th = np.empty((n, 3, 3))
    th[:, :, 0] = rng.uniform(*SIGMA_A_RANGE, size=(n, 3))
    th[:, :, 1] = rng.uniform(*SIGMA_S_RANGE, size=(n, 3))
    th[:, :, 2] = ETA_DEFAULT
    return th


def perturb_target(w: Workload, L, theta):
    """Target parameters for the L2-loss gradient workload.

    sigma_a and sigma_s' scaled by (1+U[-0.2,0.2]), eta ~ U[1.2,1.5] and
    every SH coefficient scaled by (1+U[-0.1,0.1]).
    """
    rng = np.random.default_rng(seeds(w)["target"])
    th = np.array(theta, dtype=np.float64, copy=True)
    th[..., 0] *= 1.0 + rng.uniform(-0.2, 0.2, size=th[..., 0].shape)
    th[..., 1] *= 1.0 + rng.uniform(-0.2, 0.2, size=th[..., 1].shape)
    th[..., 2] = rng.uniform(1.2, 1.5, size=th[..., 2].shape)
    Lt = np.array(L, dtype=np.float64) * (1.0 + rng.uniform(-0.1, 0.1, size=np.shape(L)))
    return Lt, th


def sample_rows(w: Workload, n: int | None = None):
    """Sorted, distinct seeded output vertex ids (original numbering)."""
    n = w.sample_rows if n is None else n
    rng = np.random.default_rng(seeds(w)["rows"])
    return np.sort(rng.choice(w.n_vertices, size=min(n, w.n_vertices), replace=False))


def get(name: str) -> Workload:
    return WORKLOADS[name]
