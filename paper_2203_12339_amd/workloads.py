"""Loaded renderers for the seeded synthetic workloads.

Takes the mesh and recipe from ``synth`` (inputs only) and runs the
library's own precompute (geometry, PCA basis, transport rows).
"""
from __future__ import annotations

import synth

from .tlt import Renderer, prepare_scene


def scene_for(w: synth.Workload, K=None):
    V, F = synth.make_mesh(w)
    return prepare_scene(V, F, w.n_sh, w.K if K is None else K, synth.N_R_NODES, w.r_max,
                         synth.MATERIAL_GRID)


def renderer_for(w: synth.Workload, device: int = 0, scene=None, K=None, layout="auto",
                 tile_vertices=0) -> Renderer:
    sc = scene_for(w, K) if scene is None else scene
    r = Renderer(device)
    r.load_transport(sc, w.n_keep, storage=w.storage, wavelet=w.wavelet, layout=layout,
                     tile_vertices=tile_vertices)
    r.scene = sc
    r.workload = w
    return r
