"""Autotuner of the transport launch shape.

For one workload it sweeps, on the GPU at hand, the tile block size (the
vertices whose rows share one column union, which fixes both the bytes
streamed per kept coefficient and the operand reuse), for 16-bit blocks
of 128 and 256 rows the tile form (dense, or only the fragments holding a
kept coefficient) and the wave shape (m-tiles and column tiles per wave),
and the number of k-steps whose irradiance rows the tile kernel stages at
once.  Each shape is
timed with the library's own stage timing (transport kernel only, every
stage recomputed), and the fastest is recorded in a table keyed by what
fixes the kernel's shape: storage type, PCA terms, output columns, vertex
count and kept coefficients per row.  ``renderer_for`` applies a recorded
entry when the workload matches it exactly; otherwise the library's built-in
choice stands.  Results do not depend on the shape beyond float32 summation
order (the tests check every shape against the FP64 oracle).

    python -m paper_2203_12339_amd.autotune --config haar-f32-10242 [--write tuning.json]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def key_of(storage: str, K: int, C: int, N: int, n_keep: int) -> str:
    return f"{storage}/K{K}/C{C}/N{N}/keep{n_keep}"


def workload_key(w) -> str:
    return key_of(w.storage, w.K, 3 * w.n_out, w.n_vertices, w.n_keep)


def vertex_candidates(K: int, storage: str = "f32") -> list:
    """Tile block sizes the tile kernel supports: V*K rows, 48..128 and a
    multiple of 16, or 256 rows with 16-bit storage."""
    vs = [V for V in range(1, 129) if (V * K) % 16 == 0 and 48 <= V * K <= 128]
    if storage != "f32" and 256 % K == 0:
        vs.append(256 // K)
    return vs


def chunk_candidates(storage: str) -> list:
    """Caps on the staged k-steps (0 = as many as fit)."""
    return [0, 128, 64, 32] if storage == "f32" else [0, 8, 4]


def shape_candidates(storage: str, rows: int) -> list:
    """Wave shapes of 16-bit tiles with eight or sixteen 16-row m-tiles
    (0 = built-in: two m-tiles and three 16-column tiles per wave); other
    tiles have one."""
    if storage == "f32":
        return [0]
    return [0, 241, 432] if rows == 128 else [0, 241] if rows == 256 else [0]


def form_candidates(storage: str, rows: int) -> list:
    """Tile forms (0 = built-in, 1 = dense, 2 = fragment-sparse): 16-bit
    blocks of 128 rows are dense by default, those of 256 rows sparse; both
    sizes also try the other form."""
    if storage == "f32" or rows not in (128, 256):
        return [0]
    return [0, 2] if rows == 128 else [0, 1]


def load_table(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def lookup(w, path: str = TABLE):
    """The recorded shape for workload ``w``, or None."""
    return load_table(path).get(workload_key(w))


def _time_transport(r, B, steps: int) -> float:
    import torch

    from .tlt import FORCE_FULL
    for _ in range(5):
        r.render_raw(B.data_ptr(), FORCE_FULL)
    torch.cuda.synchronize()
    r.profile(True)
    for _ in range(steps):
        r.render_raw(B.data_ptr(), FORCE_FULL)
    torch.cuda.synchronize()
    ms, n = r.profile_read("transport")
    r.profile(False)
    return 1e3 * ms / max(n, 1)


def tune(w, device: int = 0, steps: int = 64, log=print) -> dict:
    """Sweeps the tile shapes of workload ``w``; returns the table entry."""
    import torch

    import synth

    from .tlt import Renderer
    from .workloads import scene_for

    if w.storage == "f64":
        raise ValueError("float64 storage runs the row kernel only; nothing to tune")
    scene = scene_for(w)
    dev = torch.device("cuda", device)
    L = torch.tensor(synth.make_lighting(w), dtype=torch.float32, device=dev)
    th = torch.tensor(synth.make_materials(w), dtype=torch.float64, device=dev)
    B = torch.empty((w.n_out, w.n_vertices, 3), dtype=torch.float32, device=dev)
    results = []
    forms = ("built-in", "dense", "sparse")
    for V in vertex_candidates(w.K, w.storage):
        for form in form_candidates(w.storage, V * w.K):
            r = Renderer(device)
            try:
                if form:
                    r.set_tuning("tile_sparse", form)
                r.load_transport(scene, w.n_keep, storage=w.storage, wavelet=w.wavelet,
                                 layout="tiles", tile_vertices=V)
                r.set_lighting(L)
                r.set_material(th)
                for shape in shape_candidates(w.storage, V * w.K):
                    r.set_tuning("tile_shape", shape)
                    for kc in chunk_candidates(w.storage):
                        r.set_tuning("tile_chunk", kc)
                        us = _time_transport(r, B, steps)
                        results.append({"tile_vertices": V, "tile_sparse": form, "tile_chunk": kc,
                                        "tile_shape": shape, "transport_us": round(us, 2)})
                        log(f"[autotune] {w.name}: V={V} form={forms[form]} "
                            f"shape={shape or 'built-in'} chunk={kc or 'max'}: {us:.1f} us")
            finally:
                r.close()
    best = min(results, key=lambda e: e["transport_us"])
    return {"key": workload_key(w), "workload": w.name, "tile_vertices": best["tile_vertices"],
            "tile_sparse": best["tile_sparse"], "tile_chunk": best["tile_chunk"],
            "tile_shape": best["tile_shape"], "transport_us": best["transport_us"],
            "device": torch.cuda.get_device_name(device), "steps": steps,
            "tuned": time.strftime("%Y-%m-%d"), "sweep": results}


def main(argv=None) -> int:
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--config", action="append", required=True, choices=sorted(synth.WORKLOADS))
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--write", default=None, help="table to merge the entries into")
    args = ap.parse_args(argv)
    table = load_table(args.write) if args.write else {}
    for name in args.config:
        e = tune(synth.get(name), steps=args.steps,
                 log=lambda *a: print(*a, file=sys.stderr, flush=True))
        table[e["key"]] = e
        print(json.dumps({k: e[k] for k in ("key", "tile_vertices", "tile_sparse", "tile_chunk",
                                            "tile_shape", "transport_us")}),
              flush=True)
    if args.write:
        with open(args.write, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
