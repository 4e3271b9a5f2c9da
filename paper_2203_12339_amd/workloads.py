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
                 tile_vertices=0, tuned=True, bf16_head=True, tile_sparse=0) -> Renderer:
    """A renderer with the workload's transport loaded.  With ``tuned`` (and
    no explicit tile size) the autotuner's recorded shape for exactly this
    workload is applied, if there is one.  ``bf16_head=False`` builds BF16
    tiles without the residual words of the coarsest columns; ``tile_sparse``
    picks the tile form (0 built-in, 1 dense, 2 fragment-sparse)."""
    sc = scene_for(w, K) if scene is None else scene
    entry = None
    if tuned and tile_vertices == 0 and layout != "rows" and K is None:
        from .autotune import lookup
        entry = lookup(w)
        if entry is not None:
            tile_vertices = entry["tile_vertices"]
            tile_sparse = tile_sparse or entry.get("tile_sparse", 0)
    r = Renderer(device)
    if not bf16_head:
        r.set_tuning("bf16_head", 1)
    if tile_sparse:
        r.set_tuning("tile_sparse", tile_sparse)
    r.load_transport(sc, w.n_keep, storage=w.storage, wavelet=w.wavelet, layout=layout,
                     tile_vertices=tile_vertices)
    if entry is not None:
        r.set_tuning("tile_chunk", entry["tile_chunk"])
        r.set_tuning("tile_shape", entry.get("tile_shape", 0))
    r.scene = sc
    r.workload = w
    r.tuning = entry
    return r
