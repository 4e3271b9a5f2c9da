"""CPU tests of the transport description checks of the C ABI.

load_transport runs every host check before it touches the device; the same
checks are exported as tlt_check_transport (no GPU, no context), so each
refusal -- TLT_E_ARG for sizes, dtypes, layouts and values, TLT_E_FORMAT for
a malformed permutation or malformed rows -- is exercised here without a GPU.
"""
import ctypes

import numpy as np
import pytest

import synth

tlt = pytest.importorskip("paper_2203_12339_amd.tlt")
from paper_2203_12339_amd.workloads import scene_for  # noqa: E402

W = synth.get("haar-f32-10242").with_(subdiv=2)      # N = 162, n_pad = 256, K = 6


@pytest.fixture(scope="module")
def scene():
    return scene_for(W)


@pytest.fixture(scope="module")
def rows(scene):
    col, val = tlt.build_rows(scene, W.n_keep, "haar", np.arange(W.n_vertices))
    return col, val


def _status(d):
    return tlt._check_transport(ctypes.byref(d.desc))


def _desc(scene, **kw):
    """A description over private copies of the scene's arrays (the tests
    below corrupt them in place)."""
    args = dict(storage="f32", wavelet="haar")
    args.update(kw)
    own = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    return tlt._Desc(own, W.n_keep, **args)


def test_valid_descriptions_pass(scene, rows):
    col, val = rows
    assert _status(_desc(scene)) == tlt.OK
    assert _status(_desc(scene, col=col, val=val)) == tlt.OK                   # float64 rows
    assert _status(_desc(scene, col=col, val=val.astype(np.float32))) == tlt.OK
    assert _status(_desc(scene, storage="bf16", col=col, val=val)) == tlt.OK
    assert _status(_desc(scene, storage="f64", transfer="f64")) == tlt.OK
    assert tlt.check_transport(scene, W.n_keep, storage="f16") == tlt.OK


@pytest.mark.parametrize("field,value,what", [
    ("n_vertices", 0, "n_vertices"),
    ("wavelet", 7, "wavelet"),
    ("n_pad", 512, "n_pad"),
    ("n_sh", 0, "n_sh"),
    ("n_sh", 65, "n_sh"),
    ("K", 0, "K must"),
    ("n_r", 1, "n_r"),
    ("n_keep", 0, "n_keep"),
    ("n_keep", 257, "n_keep"),
    ("value_dtype", 9, "dtype"),
    ("transfer_dtype", -1, "dtype"),
    ("transfer_dtype", tlt.F64, "F64"),
    ("layout", 5, "layout"),
    ("tile_vertices", -1, "tile_vertices"),
    ("val_is_f64", 1, "val_is_f64"),
    ("val_is_f64", 2, "val_is_f64"),
])
def test_bad_sizes_and_codes_are_arg_errors(scene, field, value, what):
    d = _desc(scene)
    setattr(d.desc, field, value)
    assert _status(d) == tlt.E_ARG
    assert what in tlt._last_error(None).decode()


@pytest.mark.parametrize("field", ["transfer", "area", "perm", "r_nodes", "basis"])
def test_null_geometry_is_an_arg_error(scene, field):
    d = _desc(scene)
    setattr(d.desc, field, None)
    assert _status(d) == tlt.E_ARG


def test_rows_or_positions_are_needed(scene, rows):
    d = _desc(scene)
    d.desc.position = None                             # no rows and nothing to build them from
    assert _status(d) == tlt.E_ARG
    d = _desc(scene, col=rows[0], val=rows[1])
    d.desc.val = None                                  # columns without values
    assert _status(d) == tlt.E_ARG


def test_layouts_that_cannot_be_tiled(scene):
    d = _desc(scene, storage="f64", transfer="f64", layout="tiles")
    assert _status(d) == tlt.E_ARG                     # F64 has no tile form
    d = _desc(scene, layout="tiles", tile_vertices=5)  # 5 * K = 30 rows: not a multiple of 16
    assert _status(d) == tlt.E_ARG
    assert _status(_desc(scene, layout="rows", tile_vertices=5)) == tlt.OK


def test_device_build_limits():
    w = synth.get("haar-f32-10242")                   # N = 10242, n_pad = 16384
    sc = scene_for(w)
    assert tlt.check_transport(sc, 8192) == tlt.OK
    assert tlt.check_transport(sc, 16384) == tlt.OK   # every coefficient: no selection
    with pytest.raises(tlt.TltError) as ei:
        tlt.check_transport(sc, 8193)                 # longer than the device selection sorts
    assert ei.value.status == tlt.E_ARG
    assert "device build" in str(ei.value)


def test_permutation_must_be_a_bijection(scene):
    d = _desc(scene)
    d.perm[3] = d.perm[4]                              # a repeated vertex
    assert _status(d) == tlt.E_FORMAT
    assert "permutation" in tlt._last_error(None).decode()
    d = _desc(scene)
    d.perm[0] = W.n_vertices                           # out of range
    assert _status(d) == tlt.E_FORMAT
    d = _desc(scene)
    d.perm[0] = -1
    assert _status(d) == tlt.E_FORMAT


@pytest.mark.parametrize("bad", [0.0, -1e-3, np.nan, np.inf])
def test_areas_must_be_positive_and_finite(scene, bad):
    d = _desc(scene)
    d.arrs["area"][7] = bad
    assert _status(d) == tlt.E_ARG
    assert "areas" in tlt._last_error(None).decode()


def test_malformed_rows_are_format_errors(scene, rows):
    col, val = rows
    n_cols = W.n_pad
    cases = []
    c = col.copy().reshape(-1, W.n_keep)
    c[5, 3] = n_cols                                   # column past the padded length
    cases.append((c, "out of range in row 5"))
    c = col.copy().reshape(-1, W.n_keep)
    c[11, 0] = -1
    cases.append((c, "out of range in row 11"))
    c = col.copy().reshape(-1, W.n_keep)
    c[17, [2, 3]] = c[17, [3, 2]]                      # two columns swapped
    cases.append((c, "not ascending in row 17"))
    c = col.copy().reshape(-1, W.n_keep)
    c[23, 4] = c[23, 3]                                # a repeated column
    cases.append((c, "not ascending in row 23"))
    for c, msg in cases:
        d = _desc(scene, col=c, val=val)
        assert _status(d) == tlt.E_FORMAT, msg
        assert msg in tlt._last_error(None).decode()


def test_row_values_must_match_the_storage_type(scene, rows):
    col, val = rows
    with pytest.raises(AssertionError):
        _desc(scene, storage="bf16", col=col, val=val.astype(np.float32))
    bits = (val.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    assert _status(_desc(scene, storage="bf16", col=col, val=bits)) == tlt.OK
