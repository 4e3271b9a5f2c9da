#!/usr/bin/env python3
"""Throughput of the per-frame translucent transport on one MI355X.

A step is one full pass of the hot path over one batch of synthetic input:
material weights g_k (FP64), irradiance E = T L (MFMA) with its Haar
transform, and the wavelet-sparse transport with K-term fusion written in
original vertex order -- every stage recomputed (TLT_FORCE_FULL).  With
--backward the step also runs the adjoint.  Inputs are resident in HBM
before timing starts.  Prints one JSON line on stdout; progress goes to
stderr.

  python bench.py [--config large-f16-163842|batch64-bf16-40962|haar-f32-10242]
                  [--steps K] [--warmup W] [--gpus 1] [--[no-]backward]

The default workload is the large one (163842 vertices, 1% of the Haar
coefficients kept in FP16, 16 lightings) with forward and adjoint in every
step, its error taken against the FP64 oracle on its 2048 seeded output
vertices.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
SAMPLE = 8                     # one timed step in SAMPLE
FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# sources that fix the transport kernel, its launch shape and the layout of
# the data it reads (kept rows, tiles, irradiance coefficients)
TRANSPORT_SOURCES = ("csrc/k_tiles.hip", "csrc/k_build.hip", "csrc/k_prep.hip",
                     "csrc/device_common.h", "csrc/index_maps.h", "csrc/kernels.h", "csrc/api.hip",
                     "tuning.json")


def kernel_hash():
    """Hash of the transport's sources: stored counter readings are valid
    only for the kernel and data layout they were taken on."""
    h = hashlib.sha256()
    for f in TRANSPORT_SOURCES:
        with open(os.path.join(ROOT, "paper_2203_12339_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload, C):
    """HBM bytes per transport launch from committed rocprofv3 counters, if
    they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"transport_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_hash") != kernel_hash() or d.get("columns") != C:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(w, L, th, budget_s=12.0, pool=None):
    """The FP64 oracle (O-B) on a bounded sample of output rows, 1 thread
    (drawn from ``pool`` when given, else from all vertices)."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle.transport import Scene
    import contextlib
    sc = Scene(w)
    rng = np.random.default_rng(12345)
    limit = threadpool_limits(limits=1) if threadpool_limits else contextlib.nullcontext()
    cand = np.arange(w.n_vertices) if pool is None else np.asarray(pool)
    with limit:
        probe = rng.choice(cand, size=min(16, len(cand)), replace=False)
        t0 = time.perf_counter()
        sc.render_vertices(L, th, probe, block=16)
        per_row = (time.perf_counter() - t0) / len(probe)
        n = int(min(len(cand), max(16, budget_s / max(per_row, 1e-6))))
        rows = np.sort(rng.choice(cand, size=n, replace=False))
        t0 = time.perf_counter()
        ref = sc.render_vertices(L, th, rows, block=32)
        dt = time.perf_counter() - t0
    return rows, ref, dt


def _quantiles(ms):
    import numpy as np
    a = np.asarray(ms)
    return {"median_ms": round(float(np.median(a)), 5), "p10_ms": round(float(np.percentile(a, 10)), 5),
            "p90_ms": round(float(np.percentile(a, 90)), 5), "n": int(a.size)}


def copy_bandwidth(mib=1024, reps=10):
    """Reference HBM rates on this machine with library kernels, timed with
    events: a device copy of `mib` MiB (read + write counted) and a sum over
    it (read only), and a read of it with the transport's 16-byte buffer loads
    (the library's read probe, best of three grid sizes); (copy, read, probe)
    in GB/s."""
    import torch
    from paper_2203_12339_amd import tlt
    src = torch.empty(mib << 18, dtype=torch.float32, device="cuda:0")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    sink = torch.empty((), dtype=torch.float32, device="cuda:0")
    dst.copy_(src)
    torch.sum(src, dim=0, out=sink)
    torch.cuda.synchronize()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    copy = 2 * (mib << 20) / timed(lambda: dst.copy_(src)) / 1e9
    read = (mib << 20) / timed(lambda: torch.sum(src, dim=0, out=sink)) / 1e9
    folds = torch.empty(4096 * 4, dtype=torch.int32, device="cuda:0")
    own = 0.0
    for blocks in (1024, 2048, 4096):
        tlt.read_probe(src, folds, blocks)
        own = max(own, (mib << 20) / timed(lambda: tlt.read_probe(src, folds, blocks)) / 1e9)
    del src, dst, folds
    torch.cuda.synchronize()
    log(f"[bench] {mib} MiB: device copy {copy:.0f} GB/s (read + write), sum {read:.0f} GB/s (read), "
        f"16-byte buffer-load read {own:.0f} GB/s")
    return copy, read, own


def per_step_timing(args, r, step, B):
    """Per-step time distributions, each step bracketed by events on the
    launch stream: warm (back to back), cold (a read of a scratch buffer evicts the
    Infinity Cache before every step, outside the bracket) and
    replay of the step captured once as a HIP graph (its output checked
    against the eager one)."""
    import torch
    n = args.dist_steps
    cur = torch.cuda.current_stream

    def bracketed(fn, pre=None):
        ms = []
        for i in range(n):
            if pre is not None:
                pre(i)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(cur())
            fn()
            e1.record(cur())
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return ms

    out = {"warm": _quantiles(bracketed(step))}
    # a read of the scratch evicts the caches without leaving dirty lines
    # whose write-back would compete with the step
    scratch = torch.ones(args.evict_mib << 18, dtype=torch.float32, device=B.device)
    sink = torch.empty((), dtype=torch.float32, device=B.device)
    r.profile(True)
    out["cold"] = _quantiles(bracketed(step, pre=lambda i: torch.sum(scratch, dim=0, out=sink)))
    ms_tr, n_tr = r.profile_read("combine" if args.material_edit else "transport")
    r.profile(False)
    out["cold"]["evict_mib"] = args.evict_mib
    out["cold"]["transport_us"] = round(1e3 * ms_tr / max(n_tr, 1), 2)
    del scratch
    torch.cuda.synchronize()
    eager = B.clone()
    try:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(cur())
        with torch.cuda.stream(side):
            step()
        cur().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            step()
        torch.cuda.synchronize()
        B.zero_()
        gms = bracketed(g.replay)
        torch.cuda.synchronize()
        diff = float((B - eager).abs().max() / eager.abs().max().clamp_min(1e-300))
        out["graph"] = dict(_quantiles(gms), max_rel_diff_vs_eager=diff)
        del g
    except Exception as e:  # pragma: no cover - reported, not fatal
        out["graph"] = {"error": str(e)[:200]}
    torch.cuda.synchronize()
    log("[bench] per-step: " + "; ".join(
        f"{k} median {v['median_ms']:.4f} ms (p10 {v['p10_ms']:.4f}, p90 {v['p90_ms']:.4f})"
        for k, v in out.items() if "median_ms" in v))
    return out


_SCENE = None


def _oracle_chunk(args):
    """Forward radiance of a chunk of output vertices and, with an upstream
    gradient on them, that chunk's share of the adjoint (the restricted-rows
    adjoint is linear and additive over disjoint row sets)."""
    import numpy as np

    from oracle import adjoint
    L, th, rows, bb = args
    ref = _SCENE.render_vertices(L, th, rows, block=32)
    if bb is None:
        return ref, None, None
    inv = np.empty(_SCENE.N, dtype=np.int64)
    inv[_SCENE.perm] = np.arange(_SCENE.N)
    gL, gT = adjoint.grad(_SCENE, L, th, bb, rows=inv[rows], block=32)
    return ref, gL, gT


def oracle_all_cores_child(name, rows_path, bb_path, out_path):
    """Child process of the CPU baseline (no GPU in it): the same oracle on
    the same sample, split over a fork pool of the host cores; with an
    upstream gradient also the FP64 adjoint on those rows.  Writes the
    results to out_path (.npz) and prints the timing."""
    global _SCENE
    import multiprocessing as mp

    import numpy as np

    import synth
    from oracle.transport import Scene
    w = synth.get(name)
    L, th = synth.make_lighting(w), synth.make_materials(w)
    _SCENE = Scene(w)
    rows = np.load(rows_path)
    bb = np.load(bb_path) if bb_path != "-" else None        # [n_out, len(rows), 3]
    n = max(1, min(16, os.cpu_count() or 1))
    splits = [c for c in np.array_split(np.arange(len(rows)), 4 * n) if len(c)]
    jobs = [(L, th, rows[c], None if bb is None else bb[:, c, :]) for c in splits]
    with mp.get_context("fork").Pool(n) as pool:
        pool.map(_oracle_chunk, [(L, th, rows[:1], None)] * n)        # workers up
        t0 = time.perf_counter()
        res = pool.map(_oracle_chunk, jobs)
        dt = time.perf_counter() - t0
    ref = np.concatenate([r[0] for r in res], axis=1)
    out = {"ref": ref}
    if bb is not None:
        out["gL"] = sum(r[1] for r in res)
        out["gT"] = sum(r[2] for r in res)
    np.savez(out_path, **out)
    print(json.dumps({"value": round(len(rows) * w.n_out / dt, 3), "cores": n,
                      "seconds": round(dt, 2), "adjoint": bb is not None}), flush=True)


def cpu_all_cores(w, rows, bb=None):
    """Runs oracle_all_cores_child in a fresh interpreter (this process holds
    the GPU; the child never touches it) -> (timing dict, results) or None."""
    import subprocess
    import tempfile

    import numpy as np
    with tempfile.TemporaryDirectory(dir="/tmp") as d:
        path = os.path.join(d, "rows.npy")
        np.save(path, np.asarray(rows))
        bpath = "-"
        if bb is not None:
            bpath = os.path.join(d, "bb.npy")
            np.save(bpath, np.asarray(bb))
        opath = os.path.join(d, "out.npz")
        env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
        try:
            out = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-all-cores",
                                  w.name, path, bpath, opath], capture_output=True, text=True,
                                 timeout=600, env=env)
        except subprocess.TimeoutExpired:
            log("[bench] all-cores oracle timed out")
            return None
        if out.returncode != 0:
            log(f"[bench] all-cores oracle failed: {out.stderr[-300:]}")
            return None
        with np.load(opath) as z:
            res = {k: z[k] for k in z.files}
        return json.loads(out.stdout.strip().splitlines()[-1]), res


def main():
    if len(sys.argv) == 6 and sys.argv[1] == "--oracle-all-cores":
        oracle_all_cores_child(*sys.argv[2:6])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="large-f16-163842",
                    choices=["large-f16-163842", "batch64-bf16-40962", "haar-f32-10242"])
    ap.add_argument("--backward", action=argparse.BooleanOptionalAction, default=None,
                    help="include the adjoint in every step (default: for the workload that "
                         "states forward + adjoint, large-f16-163842)")
    ap.add_argument("--tile", type=int, default=0, help="columns per lane (0 = tuned default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain", action="store_true",
                    help="use the (column, value) row kernel instead of the tiles")
    ap.add_argument("--folded", action="store_true",
                    help="relight through the folded lighting transport B = sum_k g_k P_k L")
    ap.add_argument("--material-edit", action="store_true",
                    help="time material edits: each step sets one of two material sets and "
                         "renders from the kept per-term transport (Steps 3 and 4 only)")
    ap.add_argument("--spatial", type=float, default=0.0, metavar="ENERGY",
                    help="render through the spatially compressed transport (CDF 9/7 over the "
                         "output vertices) keeping this fraction of the coefficient energy")
    ap.add_argument("--dist-steps", type=int, default=100,
                    help="steps of the per-step timing passes (warm, cold, graph replay); 0 skips them")
    ap.add_argument("--evict-mib", type=int, default=512,
                    help="scratch read before each cold step (evicts the 256 MB Infinity Cache)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.backward is None:
        args.backward = args.config == "large-f16-163842" and not (
            args.folded or args.spatial or args.material_edit)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the transport "
              "shards by Morton row blocks without communication in the forward pass, but "
              "this build measures the single-GPU kernel.", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py is single-process; WORLD_SIZE > 1 is not supported", file=sys.stderr)
        sys.exit(2)
    for mode, excl in (("spatial", ("folded", "backward", "plain")), ("folded", ("backward", "plain")),
                       ("material_edit", ("backward", "folded", "spatial"))):
        if getattr(args, mode) and any(getattr(args, e) for e in excl):
            print(f"--{mode.replace('_', '-')} excludes " + ", ".join(f"--{e}" for e in excl),
                  file=sys.stderr)
            sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2203_12339_amd import tlt
    from paper_2203_12339_amd.workloads import renderer_for

    w = synth.get(args.config)
    dev = torch.device("cuda", 0)
    log(f"[bench] {w.name}: {w.description}; N={w.n_vertices} K={w.K} n_keep={w.n_keep} "
        f"storage={w.storage} n_light={w.n_light} n_mat={w.n_cfg}")
    t0 = time.perf_counter()
    r = renderer_for(w, device=0)
    if args.tile:
        r.set_tile(args.tile)
    log(f"[bench] precompute + load {time.perf_counter() - t0:.1f}s")
    try:
        ti = r.tile_info()
        log(f"[bench] tiles: {ti['vertices']} vertices per block, {ti['blocks']} blocks, "
            f"{ti['entries']} entries, {ti['fragments']} fragments "
            f"({'sparse' if ti['sparse'] else 'dense'}), {ti['value_bytes']} value bytes")
    except tlt.TltError:
        pass   # no tiles loaded (rows layout)
    sp = None
    if args.spatial:
        t0 = time.perf_counter()
        r.load_spatial(args.spatial)
        nnz, levels, _, e_k = r.spatial_info()
        step1 = w.n_vertices * w.K * w.n_keep
        sp = {"energy": args.spatial, "nnz": int(nnz), "step1_nnz": step1,
              "kept_fraction": round(nnz / step1, 4), "levels": int(levels),
              "precompute_s": round(time.perf_counter() - t0, 2)}
        log(f"[bench] spatial compression: {nnz} of {step1} entries kept "
            f"({nnz / step1:.3f}), {levels} levels, {sp['precompute_s']} s")
    L = synth.make_lighting(w)
    th = synth.make_materials(w)
    ldt = torch.float64 if w.storage == "f64" else torch.float32
    sh = torch.tensor(L, dtype=ldt, device=dev)
    tt = torch.tensor(th, dtype=torch.float64, device=dev)
    r.set_lighting(sh)
    r.set_material(tt)
    B = torch.empty((w.n_out, w.n_vertices, 3), dtype=ldt, device=dev)
    dB = torch.randn_like(B) if args.backward else None

    flags = tlt.FORCE_FULL | (tlt.SAVE_FOR_BACKWARD if args.backward else 0) | \
        (tlt.PLAIN_ROWS if args.plain else 0) | (tlt.FOLDED_LIGHTING if args.folded else 0) | \
        (tlt.SPATIAL if args.spatial else 0)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe} MiB read + {args.copy_probe} MiB written")
        del src, dst
    dSH = torch.empty((w.n_light, w.n_sh, 3), dtype=ldt, device=dev)
    dTh = torch.empty((w.n_cfg, 3, 3), dtype=torch.float64, device=dev)

    def step():
        r.render_raw(B.data_ptr(), flags)
        if args.backward:
            r.render_backward(dB, dSH, dTh)

    if args.material_edit:
        # one full render keeps v_k; every step then edits the material --
        # new values written into the material buffer on the device, then
        # set_material (no host round trip: the values are validated by the
        # weights kernel) -- and renders: the weights and the combine over the
        # kept v_k (Steps 3 and 4 only).  The step is graph-capturable.
        r.render_raw(B.data_ptr(), flags | tlt.KEEP_TERMS)
        mats = [tt.clone(), torch.tensor(synth.make_materials(w, seed=4242), dtype=torch.float64, device=dev)]
        edit = [0]

        def step():
            edit[0] ^= 1
            tt.copy_(mats[edit[0]])
            r.set_material(tt)
            r.render_raw(B.data_ptr(), tlt.PLAIN_ROWS if args.plain else 0)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    r.profile(True)
    r.profile_pause()
    torch.cuda.synchronize()
    # Every SAMPLE-th step of the timed region carries the stage timing
    # events (they add a few microseconds of dispatch latency to the steps
    # they time, so timing every step would understate the throughput).
    t0 = time.perf_counter()
    for i in range(args.steps):
        timed = i % SAMPLE == 0
        if timed:
            r.profile_resume()
        step()
        if timed:
            r.profile_pause()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_tr, n_tr = r.profile_read("combine" if args.material_edit else "transport")
    stage_ms = {s: r.profile_read(s) for s in ("weights", "irradiance", "transport", "adjoint")
                + (("inverse",) if args.spatial else ()) + (("combine",) if args.material_edit else ())}
    r.profile(False)
    if args.material_edit:
        # back to the first material set, so the accuracy check below sees
        # a material edit rendered through the kept v_k
        tt.copy_(mats[0])
        r.set_material(tt)
        r.render_raw(B.data_ptr(), tlt.PLAIN_ROWS if args.plain else 0)
    assert r.material_status() == tlt.OK
    ms_per_step = 1e3 * elapsed / args.steps
    shaded = w.n_vertices * w.n_out
    value = shaded * args.steps / elapsed
    log(f"[bench] {args.steps} steps in {elapsed:.3f}s -> {ms_per_step:.4f} ms/step; "
        + ", ".join(f"{k} {v[0] / max(v[1], 1) * 1e3:.1f}us" for k, v in stage_ms.items()))

    timing = per_step_timing(args, r, step, B) if args.dist_steps > 0 else None
    copy_gbs = copy_bandwidth() if args.dist_steps > 0 else None

    # roofline of the dominant kernel (the transport)
    C = 3 * w.n_out
    vsz = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[w.storage]
    esz = 8 if w.storage == "f64" else 4
    nnz = w.n_vertices * w.K * w.n_keep
    n_rows = w.n_pad if w.wavelet == "haar" else w.n_vertices
    if args.spatial:
        # kept entries (column word + value) read once, Ehat read once, y
        # written once (the inverse's own traffic is its stage's)
        alg_bytes = sp["nnz"] * (4 + esz) + n_rows * C * esz + w.n_vertices * C * esz
        kernel, traffic = "k_sp_rows", None
        flops = 2.0 * sp["nnz"] * C
    elif args.material_edit:
        # kept v_k (K x N x Cs) read once, B written once
        cs = (C + 15) // 16 * 16
        alg_bytes = w.K * w.n_vertices * cs * esz + w.n_vertices * C * esz
        kernel, traffic = "k_combine", None
        flops = 2.0 * w.K * w.n_vertices * C
    elif args.folded:
        # P_k rows read once (Psh >= n_sh columns, as stored: an FP16 copy
        # with 16-bit storage), B written once
        psh = next(v for v in (4, 8, 12, 16, 24, 28, 32, 36, 48, 64) if v >= w.n_sh)
        psz = 2 if w.storage in ("f16", "bf16") else esz
        alg_bytes = w.K * w.n_vertices * psh * psz + w.n_vertices * C * esz
        kernel, traffic = "k_folded", None
        flops = 2.0 * w.K * w.n_vertices * w.n_sh * C
    else:
        # kept (index, value) entries read once, Ehat read once, B written
        # once (the adjoint needs nothing saved by the forward pass)
        alg_bytes = nnz * (4 + vsz) + n_rows * C * esz + w.n_vertices * C * esz
        kernel = "k_stream" if args.plain else "k_tiles"
        traffic = None if args.plain else stored_traffic(w.name, C)
        flops = 2.0 * nnz * C
    avg_s = ms_tr / max(n_tr, 1) * 1e-3
    warm = {"kernel_us": round(avg_s * 1e6, 2), "achieved": round(alg_bytes / avg_s / 1e9, 1),
            "frac": round(alg_bytes / avg_s / 1e9 / HBM_PEAK_GBS, 4)}
    cold = None
    if timing and "transport_us" in timing.get("cold", {}):
        cold_s = timing["cold"]["transport_us"] * 1e-6
        cold = {"kernel_us": timing["cold"]["transport_us"], "achieved": round(alg_bytes / cold_s / 1e9, 1),
                "frac": round(alg_bytes / cold_s / 1e9 / HBM_PEAK_GBS, 4)}
    # A transport whose bytes fit the 256 MB Infinity Cache is reported from
    # the cold steps (the cache evicted before each); larger ones stream from
    # HBM either way and are reported from the timed region.
    fits_cache = alg_bytes <= 1.05 * (256 << 20)
    prim = cold if (fits_cache and cold is not None) else warm
    roofline = {"bound": "hbm", "achieved": prim["achieved"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": prim["frac"],
                "traffic": traffic, "kernel": kernel,
                "kernel_us": prim["kernel_us"], "kernel_launches_timed": n_tr,
                "algorithmic_bytes": alg_bytes,
                "basis": ("cold steps (Infinity Cache evicted before each)" if prim is cold
                          else "timed region (every 8th step)"),
                "warm": warm}
    if copy_gbs:
        roofline["reference_GBps"] = {"copy": round(copy_gbs[0], 1), "read": round(copy_gbs[1], 1),
                                      "buffer_load_read": round(copy_gbs[2], 1),
                                      "source": "torch copy_ and sum, and the library's read "
                                                "probe, over 1 GiB on this GPU"}
    if cold is not None:
        roofline["cold"] = cold
    if traffic:
        # the tiles store fewer bytes than the algorithmic count (no index per
        # kept coefficient, and no fragment without a kept one), so the
        # measured HBM bytes over the same kernel time say how well it streams
        phys = traffic / (prim["kernel_us"] * 1e-6) / 1e9
        roofline["physical"] = {"GBps": round(phys, 1), "frac": round(phys / HBM_PEAK_GBS, 4),
                                "basis": "traffic / kernel_us"}
        if copy_gbs:
            roofline["physical"]["frac_of_read_probe"] = round(phys / copy_gbs[2], 4)
    roofline_adj = None
    if args.backward and stage_ms["adjoint"][1] > 0:
        # the lighting-transfer product P read once and the upstream
        # gradient read once (partial sums and outputs are a few MB)
        psh = next(v for v in (4, 8, 12, 16, 24, 28, 32, 36, 48, 64) if v >= w.n_sh)
        adj_bytes = (w.K * w.n_vertices * psh + w.n_vertices * C) * esz
        adj_s = stage_ms["adjoint"][0] / stage_ms["adjoint"][1] * 1e-3
        roofline_adj = {"bound": "hbm", "achieved": round(adj_bytes / adj_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(adj_bytes / adj_s / 1e9 / HBM_PEAK_GBS, 4),
                        "stage_us": round(adj_s * 1e6, 2), "algorithmic_bytes": adj_bytes,
                        "kernels": "adjoint stage (all its launches)"}
    ai = flops / alg_bytes

    # accuracy of this very output on a sample of rows + the CPU oracle time
    Bh = B.cpu().numpy()
    cpu = None
    rel_err = None
    grad_err = None
    err_rows = None
    if args.spatial and not args.no_cpu_baseline:
        log("[bench] no CPU baseline for the spatial path: its oracle needs every output "
            "coefficient (dense per-term CDF 9/7 transforms), not a sample of rows")
    if not args.no_cpu_baseline and not args.spatial:
        def rel(got, ref):
            got = np.asarray(got, dtype=np.float64)
            return float((np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)).max())

        # the workload's own seeded output vertices (2048 for the large one),
        # else the single-thread sample drawn below
        stated = synth.sample_rows(w) if w.sample_rows else None
        log("[bench] timing the FP64 oracle on a sample of rows, 1 thread ...")
        rows1, ref1, dt = cpu_baseline(w, L, th, pool=stated)
        cpu = {"value": round(len(rows1) * w.n_out / dt, 3), "unit": "vertices/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{len(rows1)} seeded output vertices x {w.n_out} configs of {w.name}, "
                         f"O-B float64 (row precompute + transport), 1 thread, {dt:.1f}s"}
        log(f"[bench] oracle {cpu['value']} vertices/s on 1 thread")
        err_rows = stated if stated is not None else rows1
        bb = None
        if args.backward:
            # one more forward + adjoint with the upstream gradient on the
            # error rows only: the oracle's restricted-rows adjoint is then
            # the full one
            bb = np.random.default_rng(11).standard_normal((w.n_out, len(err_rows), 3))
            dBm = torch.zeros_like(B)
            dBm[:, torch.as_tensor(err_rows, device=dev), :] = torch.as_tensor(bb, dtype=B.dtype, device=dev)
            r.render_raw(B.data_ptr(), flags)
            r.render_backward(dBm, dSH, dTh)
            torch.cuda.synchronize()
            Bh = B.cpu().numpy()
            gL_gpu, gT_gpu = dSH.cpu().numpy(), dTh.cpu().numpy()
        allc = cpu_all_cores(w, err_rows, bb)
        if allc is not None:
            t_all, res = allc
            cpu["all_cores"] = {"value": t_all["value"], "unit": "vertices/s", "cores": t_all["cores"],
                                "sample": f"{len(err_rows)} seeded output vertices, a fork pool of "
                                          f"one-thread workers" + (", forward + adjoint" if bb is not None else "")}
            log(f"[bench] oracle on {t_all['cores']} cores: {t_all['value']} vertices/s")
            rel_err = rel(Bh[:, err_rows, :], res["ref"])
            if bb is not None:
                grad_err = {"lighting": float(np.abs(gL_gpu - res["gL"]).max() / np.abs(res["gL"]).max()),
                            "material": float(np.abs(gT_gpu - res["gT"]).max() / np.abs(res["gT"]).max())}
        else:
            err_rows = rows1
            rel_err = rel(Bh[:, rows1, :], ref1)
        log(f"[bench] GPU rel err on {len(err_rows)} rows {rel_err:.3e}"
            + (f"; gradients {grad_err}" if grad_err else ""))

    out = {
        "metric": "shaded vertices/sec (K-term wavelet transport) at stated rel. err; % HBM peak",
        "value": round(value, 1),
        "unit": "vertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {w.description}",
            "n_vertices": w.n_vertices, "K": w.K, "n_keep": w.n_keep, "n_sh": w.n_sh,
            "storage": w.storage, "lightings": w.n_light, "materials": w.n_cfg,
            "columns": C, "backward": bool(args.backward), "tile": r.tile(),
            "material_edit": bool(args.material_edit),
            "layout": ("spatial" if args.spatial else "folded lighting" if args.folded
                       else ("rows" if args.plain else "tiles")),
            "spatial": sp,
            "tile_shape": ({"tile_vertices": r.tuning["tile_vertices"], "tile_chunk": r.tuning["tile_chunk"],
                            "wave_shape": r.tuning.get("tile_shape", 0) or "built-in",
                            "source": "autotuner table"} if getattr(r, "tuning", None) else "built-in"),
            "rel_err_vs_fp64_oracle": rel_err,
            "rel_err_rows": None if err_rows is None else int(len(err_rows)),
            "grad_rel_err_vs_fp64_oracle": grad_err,
            "precision": ("f64 storage and arithmetic" if w.storage == "f64" else
                          f"{w.storage} storage of W and T, f32 accumulation, f64 material weights"),
            "arith_intensity_flop_per_byte": round(ai, 3),
            "stage_us": {k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in stage_ms.items()},
        },
        "roofline": roofline,
        "roofline_adjoint": roofline_adj,
        "cpu_baseline": cpu,
        "timing": timing,
    }
    print(json.dumps(out), flush=True)
    r.close()


if __name__ == "__main__":
    main()
