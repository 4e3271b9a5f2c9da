"""CPU tests of the native library: exports, host precompute, error paths.

No GPU work is called here: only the host-side entry points
(tlt_prepare_scene, tlt_build_rows) and symbol lookup.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle.transport import Scene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
tlt = pytest.importorskip("paper_2203_12339_amd.tlt")
from paper_2203_12339_amd.workloads import scene_for  # noqa: E402


def _header_functions():
    src = open(os.path.join(ROOT, "include", "tlt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_library_exports_every_declared_function():
    names = _header_functions()
    assert {"load_transport", "set_material", "set_lighting", "render",
            "render_backward"} <= set(names)
    lib = ctypes.CDLL(tlt.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tlt.EXPORTED)
    assert "gfx950" in tlt.version()


@pytest.mark.parametrize("name", ["dense-f64-642", "haar-f32-10242", "large-f16-163842"])
def test_prepare_scene_matches_oracle(name):
    w = synth.get(name)
    if name == "large-f16-163842":
        w = w.with_(subdiv=4)
    sc = scene_for(w)
    o = Scene(w)
    p = o.perm
    assert np.array_equal(sc["perm"], p)                       # index work: exact
    np.testing.assert_allclose(sc["position"], o.V[p], rtol=0, atol=0)
    np.testing.assert_allclose(sc["area"], o.area[p], rtol=1e-13)
    np.testing.assert_allclose(sc["normal"], o.normal[p], atol=1e-14)
    np.testing.assert_allclose(sc["transfer"], o.T[p], atol=1e-13)
    np.testing.assert_allclose(sc["r_nodes"], o.rn, rtol=1e-15, atol=0)
    np.testing.assert_allclose(sc["basis"], o.b, atol=1e-12)
    np.testing.assert_allclose(sc["singular_values"], o.sv, rtol=1e-10, atol=1e-13 * o.sv[0])


@pytest.mark.parametrize("name,kw", [
    ("haar-f32-10242", {}),
    ("dense-f64-642", {}),
    ("dense-f64-642", dict(wavelet="haar")),
    ("batch64-bf16-40962", dict(subdiv=4)),
    ("large-f16-163842", dict(subdiv=3)),
    ("haar-f32-10242", dict(subdiv=0, keep=0.5)),
], ids=["haar-f32-10242", "dense-f64-642:plain", "dense-f64-642:haar-full", "batch64-bf16-40962:shrunk", "large-f16-163842:shrunk", "tiny"])
def test_build_rows_match_oracle(name, kw):
    w = synth.get(name).with_(**kw)
    sc = scene_for(w)
    o = Scene(w)
    rows = np.unique(np.concatenate([np.arange(0, w.n_vertices, max(1, w.n_vertices // 40)),
                                     [w.n_vertices - 1]]))
    col, val = tlt.build_rows(sc, w.n_keep, w.wavelet, rows)
    oc, ov = o.kept_lists(rows)
    oc = oc.transpose(1, 0, 2)
    ov = ov.transpose(1, 0, 2)
    assert np.array_equal(col, oc)                             # kept sets: exact
    np.testing.assert_allclose(val, ov, rtol=1e-11, atol=1e-13 * np.abs(ov).max())


def test_host_error_paths():
    V, F = synth.icosphere(1)
    grid = synth.MATERIAL_GRID
    with pytest.raises(tlt.TltError) as ei:
        tlt.prepare_scene(V, F, 17, 4, 256, 2.0, grid)         # not a square count
    assert ei.value.status == -1
    with pytest.raises(tlt.TltError):
        tlt.prepare_scene(V, F, 16, 0, 256, 2.0, grid)         # K = 0
    Fb = F.copy()
    Fb[0, 0] = 10 ** 6
    with pytest.raises(tlt.TltError):
        tlt.prepare_scene(V, Fb, 16, 4, 256, 2.0, grid)        # face out of range
    sc = tlt.prepare_scene(V, F, 16, 4, 256, 2.0, grid)
    with pytest.raises(tlt.TltError):
        tlt.build_rows(sc, 1000, "haar", [0])                  # n_keep > n_pad
    with pytest.raises(tlt.TltError):
        tlt.build_rows(sc, 4, "haar", [42])                    # row out of range
    assert "row out of range" in tlt._last_error(None).decode()


def test_read_probe_rejects_bad_arguments_before_any_device_call():
    """The read probe validates its arguments on the host: these calls
    return TLT_E_ARG without launching anything (no GPU needed)."""
    import ctypes
    P = ctypes.c_void_p
    dummy = P(16)   # never dereferenced: every call below is rejected first
    for buf, nbytes, out, blocks in ((None, 32, dummy, 4),     # no buffer
                                     (dummy, 24, dummy, 4),    # not a multiple of 16
                                     (dummy, -16, dummy, 4),   # negative size
                                     (dummy, 32, None, 4),     # no output
                                     (dummy, 32, dummy, 0)):   # no workgroups
        assert tlt.STATUS[tlt._read_probe(buf, nbytes, out, blocks, None)] == "TLT_E_ARG"
    assert "bad arguments" in tlt._last_error(None).decode()


def test_autotune_candidates_and_table():
    """Every candidate tile shape is one the tile kernel accepts, and the
    recorded table (if any) only names such shapes."""
    from paper_2203_12339_amd import autotune
    for K in (4, 6, 8, 12, 16):
        for V in autotune.vertex_candidates(K):
            assert (V * K) % 16 == 0 and 48 <= V * K <= 128
        for V in autotune.vertex_candidates(K, "f16"):
            assert (V * K) % 16 == 0 and (48 <= V * K <= 128 or V * K == 256)
    assert autotune.vertex_candidates(6) == [8, 16]
    assert autotune.vertex_candidates(8, "bf16") == [6, 8, 10, 12, 14, 16, 32]
    for key, e in autotune.load_table().items():
        storage, K = key.split("/")[0], int(key.split("/")[1][1:])
        assert storage in ("f32", "bf16", "f16")
        assert e["tile_vertices"] in autotune.vertex_candidates(K, storage)
        assert e["tile_chunk"] in autotune.chunk_candidates(storage)
        assert e.get("tile_shape", 0) in autotune.shape_candidates(storage, e["tile_vertices"] * K)
        assert e.get("tile_sparse", 0) in autotune.form_candidates(storage, e["tile_vertices"] * K)
        assert e["key"] == key
    assert autotune.form_candidates("f16", 256) == [0, 1] and autotune.form_candidates("bf16", 128) == [0, 2]
    assert autotune.form_candidates("f32", 128) == [0] and autotune.form_candidates("f16", 112) == [0]
    assert autotune.shape_candidates("bf16", 128) == [0, 241, 432]
    assert autotune.shape_candidates("f32", 128) == [0] and autotune.shape_candidates("f16", 112) == [0]


def _check_kept_sets(s, energy, lib_keys, lib_vals, scale):
    """The library's kept set equals the oracle's except, possibly, entries
    whose rank at the cut is decided by rounding: both sets must retain the
    energy fraction, and any entry in one set only must be no larger than
    every entry the other keeps (relative 1e-9)."""
    ora = np.argwhere(s.keep)                                   # (k, u, j)
    ora_keys = set(map(tuple, ora.tolist()))
    lib = set(lib_keys)
    only = lib ^ ora_keys
    mags = {kk: abs(s.Z[kk]) for kk in only}
    for kk, m in mags.items():
        k = kk[0]
        kept_min = np.abs(s.Z[k][s.keep[k]]).min()
        assert m <= kept_min * (1 + 1e-9), (kk, m, kept_min)
    assert len(only) <= 2 * s.Z.shape[0], len(only)
    z = np.array([s.Z[k, u, j] for (k, u, j) in lib_keys])
    np.testing.assert_allclose(lib_vals, z, rtol=0, atol=1e-12 * scale)
    for k in range(s.Z.shape[0]):
        tot = (s.Z[k] ** 2).sum()
        got = sum(s.Z[kk] ** 2 for kk in lib if kk[0] == k)
        assert got >= energy * tot * (1 - 1e-12) or energy >= 1.0


@pytest.mark.parametrize("name,kw,energy", [
    ("haar-f32-10242", dict(subdiv=2, keep=0.25), 0.97),
    ("haar-f32-10242", dict(subdiv=2, keep=0.25), 1.0),
    ("dense-f64-642", dict(subdiv=2), 0.95),
    ("haar-f32-10242", dict(subdiv=3, keep=None), 0.98),
], ids=["haar-162-0.97", "haar-162-all", "plain-162-0.95", "haar-642-0.98"])
def test_spatial_rows_match_oracle(name, kw, energy):
    """Host precompute Step 2 (Sec. 3.2) against the oracle: same CDF 9/7
    coefficients and, up to rounding at the cut, the same kept sets."""
    from oracle.spatial import Spatial
    w = synth.get(name).with_(**kw)
    if kw.get("keep", 0) is None:
        w = w.with_(keep=64 / w.n_vertices)
    sc = scene_for(w)
    o = Scene(w)
    s = Spatial(o, energy)
    col, val = tlt.build_rows(sc, w.n_keep, w.wavelet, np.arange(w.n_vertices))
    n_cols = w.n_pad if w.wavelet == "haar" else w.n_vertices
    rp, k, j, v = tlt.spatial_rows(col, val, n_cols, energy)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == len(k)
    u = np.repeat(np.arange(w.n_vertices), np.diff(rp))
    # rows hold their entries in (k, j) order
    key = k * n_cols + j
    for a, b in zip(rp[:-1], rp[1:]):
        assert np.all(np.diff(key[a:b]) > 0)
    _check_kept_sets(s, energy, list(zip(k.tolist(), u.tolist(), j.tolist())), v,
                     np.abs(s.Z).max())
    if energy >= 1.0:
        assert len(k) == int((s.Z != 0).sum())


def test_spatial_rows_error_paths():
    col = np.zeros((4, 1, 2), np.int32)
    val = np.ones((4, 1, 2))
    with pytest.raises(tlt.TltError):
        tlt.spatial_rows(col, val, 4, 0.9)                     # fewer than 8 vertices
    col = np.zeros((16, 1, 2), np.int32)
    col[:, 0, 1] = 1
    val = np.ones((16, 1, 2))
    with pytest.raises(tlt.TltError):
        tlt.spatial_rows(col, val, 16, 0.0)                    # energy outside (0, 1]
    with pytest.raises(tlt.TltError):
        tlt.spatial_rows(col, val, 16, 0.9, levels=5)          # too many levels for 16
    bad = col.copy()
    bad[3, 0, 0] = 99
    with pytest.raises(tlt.TltError):
        tlt.spatial_rows(bad, val, 16, 0.9)                    # column out of range
    rp, k, j, v = tlt.spatial_rows(col, val, 16, 1.0, levels=1)
    assert rp[-1] == len(v) > 0


@pytest.mark.parametrize("n,levels", [(8, 0), (13, 0), (642, 0), (2562, 0), (1000, 3)])
def test_spatial_synthesis_operator_is_the_oracle_inverse(n, levels):
    """Step 5 of Sec. 4 as a sparse matrix: equals the oracle's exact inverse
    of the CDF 9/7 analysis (a sparse solve per level), and keeps only the
    structural non-zeros (a few tens per output)."""
    from oracle import cdf97
    rp, col, w = tlt.spatial_synthesis(n, levels)
    assert rp[0] == 0 and rp[-1] == len(w)
    M = np.zeros((n, n))
    M[np.repeat(np.arange(n), np.diff(rp)), col] = w
    ref = cdf97.inverse(np.eye(n), levels)
    assert np.abs(M - ref).max() < 1e-13
    assert np.all(np.abs(ref[M == 0]) < 1e-13)
    assert np.diff(rp).max() <= 8 * (len(cdf97.band_sizes(n, levels)) + 2)
