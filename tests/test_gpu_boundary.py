"""GPU tests of the C ABI's loading paths (through the library).

- rows precomputed on the host (tlt_build_rows, the offline Step 1 of the
  precompute in Sec. 3.2) and handed to load_transport in col/val give the
  same transport as the rows the library builds on the device: the same
  kept sets, the same stored values, the same radiance, and the oracle's;
- BF16 rows handed in as BF16 values load with the warning
  TLT_W_BF16_NO_RESIDUAL, as does a BF16 render through the row kernel;
- a context that loads a second transport renders it correctly through the
  row kernel (whose row partition belongs to the transport it was made for).
"""
import numpy as np
import pytest

import synth
from _helpers import dev_tensor, light_dtype, normwise, oracle_scene, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2203_12339_amd import tlt  # noqa: E402
from paper_2203_12339_amd.workloads import renderer_for, scene_for  # noqa: E402

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 5e-3, "f16": 5e-3}


def _render(r, w, L, th, **kw):
    r.set_lighting(dev_tensor(L, light_dtype(w)))
    r.set_material(dev_tensor(th, "f64"))
    B = r.render(force=True, **kw)
    torch.cuda.synchronize()
    return B.cpu().numpy()


@pytest.mark.parametrize("name,kw", [("haar-f32-10242:2562", dict(subdiv=4, n_light=2, n_cfg=2)),
                                     ("batch64-bf16-40962:2562", dict(subdiv=4, n_light=8, n_cfg=8)),
                                     ("large-f16-163842:642", dict(subdiv=3, n_light=4, n_cfg=1))],
                         ids=["f32", "bf16", "f16"])
def test_host_built_rows_load_like_device_built(name, kw):
    w = synth.get(name.split(":")[0]).with_(**kw)
    say(f"[rows in] {name}: N={w.n_vertices} K={w.K} n_keep={w.n_keep} storage={w.storage}")
    sc = scene_for(w)
    col, val = tlt.build_rows(sc, w.n_keep, w.wavelet, np.arange(w.n_vertices))
    col = col.reshape(w.n_vertices * w.K, w.n_keep)
    val = val.reshape(w.n_vertices * w.K, w.n_keep)
    L = synth.make_lighting(w)
    th = synth.make_materials(w)
    ref = oracle_scene(w).render(L, th)

    r_dev = tlt.Renderer(0)
    assert r_dev.load_transport(sc, w.n_keep, storage=w.storage, wavelet=w.wavelet).load_status == tlt.OK
    r_host = tlt.Renderer(0)
    st = r_host.load_transport(sc, w.n_keep, storage=w.storage, wavelet=w.wavelet, col=col, val=val).load_status
    assert st == tlt.OK                                # float64 values: BF16 tiles keep residual words
    rows = np.arange(0, w.n_vertices * w.K, 7)
    c_dev, v_dev = r_dev.read_rows(rows)
    c_host, v_host = r_host.read_rows(rows)
    assert np.array_equal(c_dev, c_host)               # the same kept sets (exact)
    assert np.array_equal(c_host, col[rows])
    # values: the device build and the host build agree to the last float32 bit
    # but one; both are rounded to storage by the same rule here
    same = float(np.mean(v_dev == v_host))
    say(f"[rows in] {name}: stored values bit-equal {100 * same:.3f}%")
    assert same > 0.99
    B_dev = _render(r_dev, w, L, th)
    B_host = _render(r_host, w, L, th)
    e_dd, e_ho = normwise(B_host, B_dev), normwise(B_host, ref)
    say(f"[rows in] {name}: host-built vs device-built {e_dd:.2e}; vs oracle {e_ho:.3e}")
    assert e_dd <= {"f32": 1e-6, "bf16": 1e-4, "f16": 1e-4}[w.storage], e_dd
    assert e_ho <= TOL[w.storage], e_ho
    if w.storage == "bf16":
        # the same rows as BF16 bits: no residual words, reported as a warning
        bits = tlt.Renderer(0)
        b16 = (val.astype(np.float32).view(np.uint32) + 0x7FFF
               + ((val.astype(np.float32).view(np.uint32) >> 16) & 1)) >> 16
        st = bits.load_transport(sc, w.n_keep, storage="bf16", wavelet=w.wavelet, col=col,
                                 val=b16.astype(np.uint16)).load_status
        assert st == tlt.W_BF16_NO_RESIDUAL
        Bb = _render(bits, w, L, th)
        assert bits.render_status == tlt.W_BF16_NO_RESIDUAL
        assert normwise(Bb, ref) <= TOL["bf16"]
        # the row kernel of a residual-carrying transport warns as well
        _render(r_host, w, L, th, plain=True)
        assert r_host.render_status == tlt.W_BF16_NO_RESIDUAL
        _render(r_host, w, L, th)
        assert r_host.render_status == tlt.OK
        bits.close()
    r_dev.close()
    r_host.close()


def test_second_transport_on_one_context_row_kernel():
    """Two transports of >= 8192 vertices loaded one after the other into one
    context: the row kernel's partition (equal row ranges per wave, split
    vertices cleared before their atomic completion) is rebuilt for the
    second, whose radiance matches the oracle even over a dirty output."""
    w1 = synth.get("haar-f32-10242")
    w2 = w1.with_(seed=w1.seed + 17, K=4)               # another mesh and row count
    say(f"[reload] N={w1.n_vertices}: K={w1.K} then K={w2.K}, plain rows")
    r = renderer_for(w1)
    L = synth.make_lighting(w1)
    th = synth.make_materials(w1)
    B1 = _render(r, w1, L, th, plain=True)
    assert normwise(B1, oracle_scene(w1).render(L, th)) <= TOL["f32"]
    r.load_transport(scene_for(w2), w2.n_keep, storage="f32", wavelet="haar")
    L2 = synth.make_lighting(w2)
    th2 = synth.make_materials(w2)
    r.set_lighting(dev_tensor(L2, "f32"))
    r.set_material(dev_tensor(th2, "f64"))
    out = torch.full((w2.n_out, w2.n_vertices, 3), 1.0e3, device="cuda:0")
    r.render(out=out, force=True, plain=True)
    torch.cuda.synchronize()
    e = normwise(out.cpu().numpy(), oracle_scene(w2).render(L2, th2))
    say(f"[reload] second transport, row kernel: normwise {e:.3e}")
    assert e <= TOL["f32"], e
    r.close()
