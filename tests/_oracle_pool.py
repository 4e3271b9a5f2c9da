"""The FP64 oracle on many output rows, spread over the host cores (test
infrastructure).  The GPU tests hold the GPU in their own process, so the
pool runs in a fresh interpreter started from there (this file as a script),
which imports only numpy, synth and oracle and forks its workers before any
GPU library could be loaded.

oracle_rows(name, kw, p_rows, bb, n_kept) -> dict with
  ref   [n_out, P, 3]   O-B radiance at the Morton positions p_rows
  gL/gT                 the FP64 adjoint restricted to those rows for the
                        upstream gradient bb [n_out, P, 3] (if given)
  cols  [K, n_kept, n]  kept columns of the first n_kept rows
"""
from __future__ import annotations

import json
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

_SCENE = None
_INPUT = None


def _run_job(job):
    from oracle import adjoint
    kind, idx = job
    L, th, rows, bb = _INPUT
    if kind == "kept":
        cols, _ = _SCENE.kept_lists(rows[idx])
        return cols
    ref = _SCENE.render_rows(L, th, rows[idx], block=16)
    if bb is None:
        return ref, None, None
    gL, gT = adjoint.grad(_SCENE, L, th, bb[:, idx, :], rows=rows[idx], block=16)
    return ref, gL, gT


def _child(inp, out):
    import multiprocessing as mp

    import synth
    from oracle.transport import Scene
    global _SCENE, _INPUT
    with np.load(inp) as z:
        name, kw = str(z["name"]), json.loads(str(z["kw"]))
        rows = z["rows"]
        bb = z["bb"] if "bb" in z.files else None
        n_kept = int(z["n_kept"])
    w = synth.get(name).with_(**kw)
    _SCENE = Scene(w)
    _INPUT = (synth.make_lighting(w), synth.make_materials(w), rows, bb)
    n = max(1, min(16, os.cpu_count() or 1))
    splits = [c for c in np.array_split(np.arange(len(rows)), 4 * n) if len(c)]
    kept = [c for c in np.array_split(np.arange(n_kept), n) if len(c)]
    with mp.get_context("fork").Pool(n) as pool:
        res = pool.map(_run_job, [("rows", c) for c in splits])
        kc = pool.map(_run_job, [("kept", c) for c in kept])
    d = {"ref": np.concatenate([r[0] for r in res], axis=1)}
    if bb is not None:
        d["gL"] = sum(r[1] for r in res)
        d["gT"] = sum(r[2] for r in res)
    if kc:
        d["cols"] = np.concatenate(kc, axis=1)
    np.savez(out, **d)


def oracle_rows(name, kw, p_rows, bb=None, n_kept=0, timeout=900):
    with tempfile.TemporaryDirectory(dir="/tmp") as d:
        inp, out = os.path.join(d, "in.npz"), os.path.join(d, "out.npz")
        extra = {} if bb is None else {"bb": np.asarray(bb, dtype=np.float64)}
        np.savez(inp, name=name, kw=json.dumps(kw), rows=np.asarray(p_rows, dtype=np.int64),
                 n_kept=n_kept, **extra)
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
                   PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), inp, out], env=env,
                           capture_output=True, text=True, timeout=timeout)
        if r.returncode != 0:
            raise RuntimeError("oracle pool failed: " + r.stderr[-2000:])
        with np.load(out) as z:
            return {k: z[k] for k in z.files}


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    _child(sys.argv[1], sys.argv[2])
