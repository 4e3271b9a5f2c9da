"""ctypes binding of libtlt.so (argument marshalling only).

Every computation runs inside the library: host precompute in C++, the
per-frame path in HIP kernels on the GPU.  PyTorch supplies device memory
and the current HIP stream.  If the library is missing this module raises
at import time; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtlt.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
WAVELET_NONE, WAVELET_HAAR = 0, 1
SAVE_FOR_BACKWARD, FORCE_FULL, PLAIN_ROWS, FOLDED_LIGHTING, SPATIAL, KEEP_TERMS = 1, 2, 4, 8, 16, 32
LAYOUTS = {"auto": 0, "rows": 1, "tiles": 2}
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16}

OK = 0
W_MATERIAL_OUT_OF_RANGE = 1
W_BF16_NO_RESIDUAL = 2
E_ARG, E_STATE, E_OOM, E_HIP, E_FORMAT = -1, -2, -3, -4, -5
STATUS = {0: "TLT_OK", 1: "TLT_W_MATERIAL_OUT_OF_RANGE", 2: "TLT_W_BF16_NO_RESIDUAL",
          -1: "TLT_E_ARG", -2: "TLT_E_STATE", -3: "TLT_E_OOM", -4: "TLT_E_HIP", -5: "TLT_E_FORMAT"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
# torch first: it brings its own HIP runtime, and the library must bind to
# that same runtime (two runtimes in one process do not share devices).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

_p = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class SceneDesc(ctypes.Structure):
    _fields_ = [
        ("n_vertices", ctypes.c_int32), ("n_faces", ctypes.c_int32),
        ("vertices", _f64p), ("faces", _i32p),
        ("n_sh", ctypes.c_int32), ("K", ctypes.c_int32), ("n_r", ctypes.c_int32),
        ("r_max", ctypes.c_double),
        ("mat_lo", ctypes.c_double * 3), ("mat_hi", ctypes.c_double * 3),
        ("mat_n", ctypes.c_int32 * 3),
        ("perm", _i32p), ("position", _f64p), ("area", _f64p), ("normal", _f64p),
        ("transfer", _f64p), ("r_nodes", _f64p), ("basis", _f64p),
        ("singular_values", _f64p),
    ]


class TransportDesc(ctypes.Structure):
    _fields_ = [
        ("n_vertices", ctypes.c_int32), ("n_pad", ctypes.c_int32), ("n_sh", ctypes.c_int32),
        ("K", ctypes.c_int32), ("n_r", ctypes.c_int32), ("wavelet", ctypes.c_int32),
        ("value_dtype", ctypes.c_int32), ("transfer_dtype", ctypes.c_int32),
        ("n_keep", ctypes.c_int64),
        ("col", _i32p), ("val", _p), ("position", _f64p), ("transfer", _f64p),
        ("area", _f64p), ("perm", _i32p), ("r_nodes", _f64p), ("basis", _f64p),
        ("mat_range", _f64p), ("layout", ctypes.c_int32), ("tile_vertices", ctypes.c_int32),
        ("val_is_f64", ctypes.c_int32),
    ]


class SpatialDesc(ctypes.Structure):
    _fields_ = [
        ("energy", ctypes.c_double), ("levels", ctypes.c_int32), ("threads", ctypes.c_int32),
        ("col", _i32p), ("val", _f64p),
    ]


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_prepare_scene = _sig("tlt_prepare_scene", ctypes.c_int, ctypes.POINTER(SceneDesc))
_create = _sig("tlt_create", ctypes.c_int, ctypes.POINTER(_p), ctypes.c_int)
_destroy = _sig("tlt_destroy", None, _p)
_last_error = _sig("tlt_last_error", ctypes.c_char_p, _p)
_load_transport = _sig("load_transport", ctypes.c_int, _p, ctypes.POINTER(TransportDesc))
_check_transport = _sig("tlt_check_transport", ctypes.c_int, ctypes.POINTER(TransportDesc))
_set_material = _sig("set_material", ctypes.c_int, _p, ctypes.c_int, _p, _p)
_material_status = _sig("tlt_material_status", ctypes.c_int, _p, _p)
_set_lighting = _sig("set_lighting", ctypes.c_int, _p, ctypes.c_int, _p)
_render = _sig("render", ctypes.c_int, _p, _p, _p, ctypes.c_int)
_render_backward = _sig("render_backward", ctypes.c_int, _p, _p, _p, _p, _p)
_render_backward_noalloc = _sig("render_backward_noalloc", ctypes.c_int, _p, _p, _p, _p, _p)
_tile_info = _sig("tlt_tile_info", ctypes.c_int, _p, _p, _p, _p, _p, _p, _p)
_read_rows = _sig("tlt_read_rows", ctypes.c_int, _p, ctypes.c_int64,
                  ctypes.POINTER(ctypes.c_int64), _i32p, _f64p)
_read_state = _sig("tlt_read_state", ctypes.c_int, _p, ctypes.c_int, _p,
                   ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int))
_set_tile = _sig("tlt_set_tile", ctypes.c_int, _p, ctypes.c_int)
_get_tile = _sig("tlt_get_tile", ctypes.c_int, _p)
_version = _sig("tlt_version", ctypes.c_char_p)
_set_tuning = _sig("tlt_set_tuning", ctypes.c_int, _p, ctypes.c_int32, ctypes.c_int32)
_set_irradiance = _sig("set_irradiance", ctypes.c_int, _p, ctypes.c_int, _p)
_spatial_rows = _sig("tlt_spatial_rows", ctypes.c_int, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                     ctypes.c_int64, _i32p, _f64p, ctypes.c_double, ctypes.c_int32,
                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint32), _f64p,
                     ctypes.c_int64)
_spatial_synthesis = _sig("tlt_spatial_synthesis", ctypes.c_int, ctypes.c_int32, ctypes.c_int32,
                          _i32p, _i32p, _f64p, ctypes.c_int64)
_set_view = _sig("set_view", ctypes.c_int, _p, _f64p, _f64p, _f64p)
_read_probe = _sig("tlt_read_probe", ctypes.c_int, _p, ctypes.c_int64, _p, ctypes.c_int, _p)
_load_spatial = _sig("load_spatial", ctypes.c_int, _p, ctypes.POINTER(SpatialDesc))
_spatial_info = _sig("tlt_spatial_info", ctypes.c_int, _p, ctypes.POINTER(ctypes.c_int64),
                     _i32p, ctypes.POINTER(ctypes.c_int64), _f64p)
_read_spatial = _sig("tlt_read_spatial", ctypes.c_int, _p, ctypes.c_int64, ctypes.c_int64,
                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint32), _f64p,
                     ctypes.c_int64)
_profile_enable = _sig("tlt_profile_enable", ctypes.c_int, _p, ctypes.c_int)
_profile_read = _sig("tlt_profile_read", ctypes.c_int, _p, ctypes.c_int,
                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64))
_build_rows = _sig("tlt_build_rows", ctypes.c_int, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _f64p, _f64p, _f64p,
                   ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _i32p, _f64p)

EXPORTED = ["tlt_prepare_scene", "tlt_build_rows", "tlt_create", "tlt_destroy", "tlt_last_error", "load_transport",
            "tlt_check_transport", "tlt_material_status",
            "set_material", "set_lighting", "render", "render_backward", "render_backward_noalloc",
            "tlt_read_rows", "tlt_tile_info",
            "tlt_read_state", "tlt_set_tile", "tlt_get_tile", "tlt_version",
            "tlt_set_tuning", "tlt_profile_enable", "tlt_profile_read", "set_irradiance",
            "load_spatial", "tlt_spatial_info", "tlt_read_spatial", "tlt_spatial_rows",
            "tlt_spatial_synthesis", "set_view", "tlt_read_probe"]

TUNE_TILE_CHUNK, TUNE_STREAM_WAVES_PER_CU, TUNE_STREAM_EPL, TUNE_STREAM_NT = 1, 2, 3, 4
TUNE_SPATIAL_LANES, TUNE_SPATIAL_UNROLL, TUNE_SPATIAL_SYNTH_LANES, TUNE_SPATIAL_SEGMENT = 5, 6, 7, 8
TUNE_TILE_SHAPE, TUNE_IRRADIANCE_HAAR, TUNE_BF16_HEAD, TUNE_TILE_SPARSE = 9, 10, 11, 12
TUNE_FOLDED_FP32 = 13
TUNING_KEYS = {"tile_chunk": TUNE_TILE_CHUNK, "stream_waves_per_cu": TUNE_STREAM_WAVES_PER_CU,
               "stream_epl": TUNE_STREAM_EPL, "stream_nt": TUNE_STREAM_NT,
               "spatial_lanes": TUNE_SPATIAL_LANES, "spatial_unroll": TUNE_SPATIAL_UNROLL,
               "spatial_synth_lanes": TUNE_SPATIAL_SYNTH_LANES,
               "spatial_segment": TUNE_SPATIAL_SEGMENT, "tile_shape": TUNE_TILE_SHAPE,
               "irradiance_haar": TUNE_IRRADIANCE_HAAR, "bf16_head": TUNE_BF16_HEAD,
               "tile_sparse": TUNE_TILE_SPARSE, "folded_fp32": TUNE_FOLDED_FP32}


class TltError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(status, ctx=None, allow=(OK,)):
    if status in allow:
        return status
    msg = _last_error(ctx).decode(errors="replace")
    raise TltError(status, msg)


def version() -> str:
    return _version().decode()


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# ---------------------------------------------------------------------------
# Host precompute
# ---------------------------------------------------------------------------

def prepare_scene(vertices, faces, n_sh, K, n_r, r_max, grid):
    """Geometry + PCA precompute in the library (host C++, float64).

    grid: dict(sigma_a=(lo, hi, n), sigma_s=(lo, hi, n), eta=(lo, hi, n)).
    Returns a dict of numpy arrays (Morton order where per vertex).
    """
    V = np.ascontiguousarray(vertices, dtype=np.float64)
    F = np.ascontiguousarray(faces, dtype=np.int32)
    N = V.shape[0]
    n_mat = int(np.prod([grid[k][2] for k in ("sigma_a", "sigma_s", "eta")]))
    out = dict(perm=np.empty(N, np.int32), position=np.empty((N, 3)), area=np.empty(N),
               normal=np.empty((N, 3)), transfer=np.empty((N, n_sh)), r_nodes=np.empty(n_r),
               basis=np.empty((K, n_r)), singular_values=np.empty(min(n_mat, n_r)))
    d = SceneDesc()
    d.n_vertices, d.n_faces = N, F.shape[0]
    d.vertices, d.faces = _ptr(V, ctypes.c_double), _ptr(F, ctypes.c_int32)
    d.n_sh, d.K, d.n_r, d.r_max = n_sh, K, n_r, float(r_max)
    keys = ("sigma_a", "sigma_s", "eta")
    d.mat_lo = (ctypes.c_double * 3)(*[grid[k][0] for k in keys])
    d.mat_hi = (ctypes.c_double * 3)(*[grid[k][1] for k in keys])
    d.mat_n = (ctypes.c_int32 * 3)(*[grid[k][2] for k in keys])
    d.perm = _ptr(out["perm"], ctypes.c_int32)
    for k in ("position", "area", "normal", "transfer", "r_nodes", "basis", "singular_values"):
        setattr(d, k, _ptr(out[k], ctypes.c_double))
    _check(_prepare_scene(ctypes.byref(d)), None)
    out["mat_range"] = np.array([[grid[k][0], grid[k][1]] for k in keys], dtype=np.float64)
    return out


def build_rows(scene, n_keep, wavelet, morton_rows):
    """Host float64 transport rows (as load_transport builds them) for the
    given Morton positions -> (col [R, K, n_keep] int32, val [R, K, n_keep])."""
    pos = np.ascontiguousarray(scene["position"], dtype=np.float64)
    rn = np.ascontiguousarray(scene["r_nodes"], dtype=np.float64)
    b = np.ascontiguousarray(scene["basis"], dtype=np.float64)
    N = pos.shape[0]
    K = b.shape[0]
    n_cols = (1 << (N - 1).bit_length()) if wavelet == "haar" else N
    rows = np.ascontiguousarray(morton_rows, dtype=np.int64)
    col = np.empty((len(rows), K, n_keep), np.int32)
    val = np.empty((len(rows), K, n_keep), np.float64)
    _check(_build_rows(N, n_cols, K, rn.shape[0], WAVELET_HAAR if wavelet == "haar" else WAVELET_NONE,
                       n_keep, _ptr(pos, ctypes.c_double), _ptr(rn, ctypes.c_double),
                       _ptr(b, ctypes.c_double), len(rows), _ptr(rows, ctypes.c_int64),
                       _ptr(col, ctypes.c_int32), _ptr(val, ctypes.c_double)), None)
    return col, val


# ---------------------------------------------------------------------------
# Context wrapper
# ---------------------------------------------------------------------------

def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def spatial_rows(col, val, n_cols, energy, levels=0):
    """Host spatial compression of float64 Step-1 rows col/val [N, K, n_keep]
    -> (rowptr [N+1], k, j, values) of the kept entries of Z over u."""
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    N, K, n_keep = col.shape
    rp = np.zeros(N + 1, np.int64)
    st = _spatial_rows(N, n_cols, K, n_keep, _ptr(col, ctypes.c_int32), _ptr(val, ctypes.c_double),
                       float(energy), int(levels), _ptr(rp, ctypes.c_int64), None, None, 0)
    m = int(rp[-1])
    if st != OK and m == 0:
        _check(st, None)
    cw = np.zeros(max(m, 1), np.uint32)
    v = np.zeros(max(m, 1), np.float64)
    _check(_spatial_rows(N, n_cols, K, n_keep, _ptr(col, ctypes.c_int32), _ptr(val, ctypes.c_double),
                         float(energy), int(levels), _ptr(rp, ctypes.c_int64),
                         _ptr(cw, ctypes.c_uint32), _ptr(v, ctypes.c_double), m), None)
    return rp, (cw[:m] >> 24).astype(np.int64), (cw[:m] & 0xFFFFFF).astype(np.int64), v[:m]


def read_probe(buf, out, blocks):
    """Streams the CUDA tensor ``buf`` once (measurement of the read rate);
    ``out``: int32 CUDA tensor of at least blocks * 4 elements."""
    assert buf.is_cuda and out.is_cuda and out.numel() >= blocks * 4
    _check(_read_probe(ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                       ctypes.c_void_p(out.data_ptr()), blocks, _stream()), None)


def spatial_synthesis(n, levels=0):
    """w_1^{-1} over a list of n as CSR over the output position ->
    (rowptr [n+1], coefficient index, weight)."""
    rp = np.zeros(n + 1, np.int32)
    st = _spatial_synthesis(n, levels, _ptr(rp, ctypes.c_int32), None, None, 0)
    m = int(rp[-1])
    if st != OK and m == 0:
        _check(st, None)
    col = np.zeros(max(m, 1), np.int32)
    w = np.zeros(max(m, 1), np.float64)
    _check(_spatial_synthesis(n, levels, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32),
                              _ptr(w, ctypes.c_double), m), None)
    return rp, col[:m].astype(np.int64), w[:m]


class _Desc:
    """A TransportDesc with the numpy arrays its pointers refer to kept alive."""

    def __init__(self, scene, n_keep, storage="f32", wavelet="haar", col=None, val=None,
                 layout="auto", tile_vertices=0, transfer=None):
        N = scene["perm"].shape[0]
        self.N = N
        self.n_pad = 1 << (N - 1).bit_length()
        self.vdt = DTYPES[storage]
        self.n_sh = scene["transfer"].shape[1]
        self.K = scene["basis"].shape[0]
        self.wavelet = WAVELET_HAAR if wavelet == "haar" else WAVELET_NONE
        self.perm = np.ascontiguousarray(scene["perm"], dtype=np.int32)
        self.arrs = {k: np.ascontiguousarray(scene[k], dtype=np.float64)
                     for k in ("position", "transfer", "area", "r_nodes", "basis")}
        self.mr = np.ascontiguousarray(scene.get("mat_range"), dtype=np.float64) \
            if scene.get("mat_range") is not None else None
        d = TransportDesc()
        d.n_vertices, d.n_pad, d.n_sh, d.K = N, self.n_pad, self.n_sh, self.K
        d.n_r = self.arrs["r_nodes"].shape[0]
        d.wavelet = self.wavelet
        d.value_dtype = self.vdt
        d.transfer_dtype = DTYPES[transfer] if transfer else self.vdt
        d.n_keep = int(n_keep)
        d.layout = LAYOUTS[layout]
        d.tile_vertices = int(tile_vertices)
        if col is not None:
            # rows in the storage type's bits (uint16 for BF16/F16), or float64
            # values that the library rounds to storage itself
            self.col = np.ascontiguousarray(col, dtype=np.int32)
            self.val = np.ascontiguousarray(val)
            if self.val.dtype == np.float64 and self.vdt != F64:
                d.val_is_f64 = 1
            else:
                want = {F64: np.float64, F32: np.float32, BF16: np.uint16, F16: np.uint16}[self.vdt]
                assert self.val.dtype == want, (self.val.dtype, want)
            assert self.col.size == N * self.K * int(n_keep) and self.val.size == self.col.size
            d.col = _ptr(self.col, ctypes.c_int32)
            d.val = self.val.ctypes.data_as(ctypes.c_void_p)
        d.position = _ptr(self.arrs["position"], ctypes.c_double)
        d.transfer = _ptr(self.arrs["transfer"], ctypes.c_double)
        d.area = _ptr(self.arrs["area"], ctypes.c_double)
        d.perm = _ptr(self.perm, ctypes.c_int32)
        d.r_nodes = _ptr(self.arrs["r_nodes"], ctypes.c_double)
        d.basis = _ptr(self.arrs["basis"], ctypes.c_double)
        if self.mr is not None:
            d.mat_range = _ptr(self.mr, ctypes.c_double)
        self.desc = d


def check_transport(scene, n_keep, **kw):
    """Host-only validation of a transport description (tlt_check_transport):
    the status load_transport would return for it before any device work;
    raises TltError on an error."""
    d = _Desc(scene, n_keep, **kw)
    return _check(_check_transport(ctypes.byref(d.desc)), None)


class Renderer:
    """One library context holding one loaded transport.

    The C-ABI calls of the same names: load_transport, set_material,
    set_lighting, render, render_backward.
    """

    def __init__(self, device: int = 0):
        import torch
        self.device = device
        self.torch_device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        _check(_create(ctypes.byref(h), device), None)
        self._h = h
        self.loaded = False
        self._keep = []
        self.generation = 0   # counts renders and loads (autograd checks it)

    def close(self):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return _last_error(self._h).decode(errors="replace")

    # -- transport --------------------------------------------------------
    def load_transport(self, scene, n_keep, storage="f32", wavelet="haar", col=None, val=None,
                       layout="auto", tile_vertices=0, transfer=None):
        """transfer: storage of T (default: the storage of W; F64 only with F64).
        col/val: caller-given rows [N*K, n_keep] (val float64, or the storage
        type's bits).  Returns the status (TLT_OK or the warning
        TLT_W_BF16_NO_RESIDUAL)."""
        d = _Desc(scene, n_keep, storage=storage, wavelet=wavelet, col=col, val=val, layout=layout,
                  tile_vertices=tile_vertices, transfer=transfer)
        self.N, self.n_pad = d.N, d.n_pad
        self.n_sh, self.K = d.n_sh, d.K
        self.fp64 = d.vdt == F64
        self.storage = storage
        self.wavelet = d.wavelet
        self.n_keep = int(n_keep)
        self.perm = d.perm
        self.load_status = _check(_load_transport(self._h, ctypes.byref(d.desc)), self._h,
                                  allow=(OK, W_BF16_NO_RESIDUAL))
        self.loaded = True
        self.generation += 1
        return self

    # -- view -------------------------------------------------------------
    def set_view(self, eye, scene=None):
        """Applies (1/pi) F_t(eta, w_o) toward ``eye`` (mm) in later renders;
        None removes it.  Positions and normals from ``scene`` (default: the
        loaded one)."""
        if eye is None:
            return _check(_set_view(self._h, None, None, None), self._h)
        sc = self.scene if scene is None else scene
        e = np.ascontiguousarray(eye, dtype=np.float64)
        pos = np.ascontiguousarray(sc["position"], dtype=np.float64)
        nrm = np.ascontiguousarray(sc["normal"], dtype=np.float64)
        return _check(_set_view(self._h, _ptr(e, ctypes.c_double), _ptr(pos, ctypes.c_double),
                                _ptr(nrm, ctypes.c_double)), self._h)

    # -- spatial compression ----------------------------------------------
    def load_spatial(self, energy, levels=0, threads=0, scene=None, col=None, val=None):
        """Spatially compresses the loaded transport (load_spatial); the
        float64 Step-1 rows come from ``col``/``val`` [N, K, n_keep] or are
        rebuilt on the host from ``scene`` (default: the loaded scene)."""
        if col is None:
            sc = self.scene if scene is None else scene
            col, val = build_rows(sc, self.n_keep, "haar" if self.wavelet == WAVELET_HAAR else "none",
                                  np.arange(self.N))
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        assert col.shape == (self.N, self.K, self.n_keep) and val.shape == col.shape
        d = SpatialDesc()
        d.energy, d.levels, d.threads = float(energy), int(levels), int(threads)
        d.col = _ptr(col, ctypes.c_int32)
        d.val = _ptr(val, ctypes.c_double)
        return _check(_load_spatial(self._h, ctypes.byref(d)), self._h)

    def spatial_info(self):
        """(kept entries, levels, kept entries per term, retained energy per term)."""
        nnz = ctypes.c_int64()
        lv = ctypes.c_int32()
        nk = np.zeros(self.K, np.int64)
        ek = np.zeros(self.K, np.float64)
        _check(_spatial_info(self._h, ctypes.byref(nnz), ctypes.byref(lv),
                             _ptr(nk, ctypes.c_int64), _ptr(ek, ctypes.c_double)), self._h)
        return nnz.value, lv.value, nk, ek

    def read_spatial(self, u0=0, n_u=None):
        """Kept entries of output coefficients u0 .. u0+n_u-1 ->
        (rowptr [n_u+1], k, j, values)."""
        n_u = self.N - u0 if n_u is None else n_u
        rp = np.zeros(n_u + 1, np.int64)
        _read_spatial(self._h, u0, n_u, _ptr(rp, ctypes.c_int64), None, None, 0)
        m = int(rp[-1])
        cw = np.zeros(max(m, 1), np.uint32)
        v = np.zeros(max(m, 1), np.float64)
        _check(_read_spatial(self._h, u0, n_u, _ptr(rp, ctypes.c_int64), _ptr(cw, ctypes.c_uint32),
                             _ptr(v, ctypes.c_double), m), self._h)
        return rp, (cw[:m] >> 24).astype(np.int64), (cw[:m] & 0xFFFFFF).astype(np.int64), v[:m]

    # -- inputs -----------------------------------------------------------
    def set_irradiance(self, E):
        """E: CUDA tensor [n_light, N, 3] (original vertex order; float64 for
        F64 storage) used instead of SH lighting until set_lighting."""
        import torch
        want = torch.float64 if self.fp64 else torch.float32
        assert E.is_cuda and E.dtype == want and E.is_contiguous(), (E.dtype, want)
        assert E.shape[1] == self.N and E.shape[2] == 3
        self._E = E
        self.n_light = E.shape[0]
        return _check(_set_irradiance(self._h, E.shape[0], ctypes.c_void_p(E.data_ptr())), self._h)

    def set_material(self, theta):
        """theta: CUDA float64 tensor [n_mat, 3, 3] (read and validated on the
        device by the next render; see material_status)."""
        import torch
        assert theta.is_cuda and theta.dtype == torch.float64 and theta.is_contiguous()
        assert theta.dim() == 3 and theta.shape[1:] == (3, 3), tuple(theta.shape)
        self._theta = theta
        self.n_mat = theta.shape[0]
        return _check(_set_material(self._h, theta.shape[0], ctypes.c_void_p(theta.data_ptr()),
                                    _stream()), self._h)

    def material_status(self):
        """Waits for the current stream; TLT_OK or TLT_W_MATERIAL_OUT_OF_RANGE
        for the materials rendered since the last call, TltError(TLT_E_ARG)
        if one was invalid (tlt_material_status)."""
        return _check(_material_status(self._h, _stream()), self._h,
                      allow=(OK, W_MATERIAL_OUT_OF_RANGE))

    def set_lighting(self, sh):
        """sh: CUDA tensor [n_light, n_sh, 3] (float64 for F64 storage)."""
        import torch
        want = torch.float64 if self.fp64 else torch.float32
        assert sh.is_cuda and sh.dtype == want and sh.is_contiguous(), (sh.dtype, want)
        assert sh.shape[1] == self.n_sh and sh.shape[2] == 3
        self._sh = sh
        self.n_light = sh.shape[0]
        return _check(_set_lighting(self._h, sh.shape[0], ctypes.c_void_p(sh.data_ptr())), self._h)

    @property
    def n_out(self):
        return max(self.n_light, self.n_mat)

    def out_dtype(self):
        import torch
        return torch.float64 if self.fp64 else torch.float32

    def render(self, out=None, save=False, force=False, plain=False, folded=False, spatial=False,
               keep=False):
        """save: render_backward may differentiate this render; keep: keep the
        per-term transport v_k so that a material-only change reruns Steps 3-4
        only (render flags TLT_SAVE_FOR_BACKWARD, TLT_KEEP_TERMS)."""
        import torch
        if out is None:
            out = torch.empty((self.n_out, self.N, 3), dtype=self.out_dtype(),
                              device=self.torch_device)
        else:
            assert out.is_cuda and out.dtype == self.out_dtype() and out.is_contiguous()
            assert tuple(out.shape) == (self.n_out, self.N, 3), tuple(out.shape)
        flags = (SAVE_FOR_BACKWARD if save else 0) | (FORCE_FULL if force else 0) | \
            (PLAIN_ROWS if plain else 0) | (FOLDED_LIGHTING if folded else 0) | \
            (SPATIAL if spatial else 0) | (KEEP_TERMS if keep else 0)
        self.render_status = _check(_render(self._h, ctypes.c_void_p(out.data_ptr()), _stream(), flags),
                                    self._h, allow=(OK, W_BF16_NO_RESIDUAL))
        self.generation += 1
        return out

    def render_raw(self, out_ptr: int, flags: int):
        """Render into a raw device pointer (for graph capture and timing)."""
        self.generation += 1
        return _check(_render(self._h, ctypes.c_void_p(out_ptr), _stream(), flags), self._h,
                      allow=(OK, W_BF16_NO_RESIDUAL))

    def render_backward(self, dB, dSH=None, dTheta=None, noalloc=False):
        """Adjoint of the last render (render_backward); noalloc=True calls
        render_backward_noalloc (the library's static scratch; pass dSH and
        dTheta to keep the call free of allocations here too)."""
        import torch
        assert dB.is_cuda and dB.dtype == self.out_dtype(), (dB.dtype, self.out_dtype())
        assert tuple(dB.shape) == (self.n_out, self.N, 3), (tuple(dB.shape), (self.n_out, self.N, 3))
        dB = dB.contiguous()
        if dSH is None:
            dSH = torch.empty((self.n_light, self.n_sh, 3), dtype=self.out_dtype(),
                              device=self.torch_device)
        else:
            assert dSH.is_cuda and dSH.dtype == self.out_dtype() and dSH.is_contiguous()
            assert tuple(dSH.shape) == (self.n_light, self.n_sh, 3), tuple(dSH.shape)
        if dTheta is None:
            dTheta = torch.empty((self.n_mat, 3, 3), dtype=torch.float64,
                                 device=self.torch_device)
        else:
            assert dTheta.is_cuda and dTheta.dtype == torch.float64 and dTheta.is_contiguous()
            assert tuple(dTheta.shape) == (self.n_mat, 3, 3), tuple(dTheta.shape)
        fn = _render_backward_noalloc if noalloc else _render_backward
        _check(fn(self._h, ctypes.c_void_p(dB.data_ptr()),
                                ctypes.c_void_p(dSH.data_ptr()),
                                ctypes.c_void_p(dTheta.data_ptr()), _stream()), self._h)
        return dSH, dTheta

    # -- diagnostics ------------------------------------------------------
    def read_rows(self, rows):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        col = np.empty((len(rows), self.n_keep), np.int32)
        val = np.empty((len(rows), self.n_keep), np.float64)
        _check(_read_rows(self._h, len(rows), _ptr(rows, ctypes.c_int64),
                          _ptr(col, ctypes.c_int32), _ptr(val, ctypes.c_double)), self._h)
        return col, val

    def tile_info(self):
        """Shape of the loaded tiles (tlt_tile_info)."""
        v, sp = ctypes.c_int32(), ctypes.c_int32()
        nb, ne, nf, nbytes = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_tile_info(self._h, ctypes.byref(v), ctypes.byref(nb), ctypes.byref(ne), ctypes.byref(nf),
                          ctypes.byref(nbytes), ctypes.byref(sp)), self._h)
        return {"vertices": v.value, "blocks": nb.value, "entries": ne.value, "fragments": nf.value,
                "value_bytes": nbytes.value, "sparse": bool(sp.value)}

    def read_state(self, which):
        nbytes = ctypes.c_size_t()
        stride = ctypes.c_int()
        _check(_read_state(self._h, which, None, ctypes.byref(nbytes), ctypes.byref(stride)),
               self._h)
        buf = np.empty(nbytes.value, np.uint8)
        _check(_read_state(self._h, which, buf.ctypes.data_as(ctypes.c_void_p),
                           ctypes.byref(nbytes), ctypes.byref(stride)), self._h)
        return buf, stride.value

    def ehat(self):
        buf, cs = self.read_state(0)
        dt = np.float64 if self.fp64 else np.float32
        rows = self.n_pad if self.wavelet == WAVELET_HAAR else self.N
        return buf.view(dt).reshape(rows, cs)

    def g(self):
        buf, _ = self.read_state(1)
        return buf.view(np.float64).reshape(self.n_mat, 3, self.K)

    def dg(self):
        buf, _ = self.read_state(2)
        return buf.view(np.float64).reshape(self.n_mat, 3, self.K, 3)

    STAGES = {"weights": 0, "irradiance": 1, "transport": 2, "adjoint": 3, "combine": 4,
              "inverse": 5}

    def profile(self, enable=True):
        """Clear the stage totals and enable timing (True), or pause it."""
        _check(_profile_enable(self._h, 1 if enable else 0), self._h)

    def profile_pause(self):
        _check(_profile_enable(self._h, 0), self._h)

    def profile_resume(self):
        """Resume timing without waiting or clearing the totals."""
        _check(_profile_enable(self._h, 2), self._h)

    def profile_read(self, stage):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(_profile_read(self._h, self.STAGES.get(stage, stage), ctypes.byref(ms),
                             ctypes.byref(n)), self._h)
        return ms.value, n.value

    def set_tuning(self, key, value: int):
        """key: a TUNING_KEYS name or TUNE_* code; value 0 = built-in choice."""
        _check(_set_tuning(self._h, TUNING_KEYS.get(key, key), int(value)), self._h)

    def set_tile(self, cpl: int):
        _check(_set_tile(self._h, int(cpl)), self._h)

    def tile(self) -> int:
        return int(_get_tile(self._h))
