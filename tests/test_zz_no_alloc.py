"""render_backward_noalloc (the adjoint with the library's static device
scratch, for callers that cannot allocate) against render_backward, through
the C ABI: two calls in a row on one GPU, the second with a smaller input
(fewer vertices and columns).  Both entry points run the same kernels on the
same inputs, so their gradients must agree exactly; the small case is also
checked against the FP64 oracle adjoint at the storage tolerance."""
import numpy as np
import pytest

import synth
from _helpers import dev_tensor, oracle_scene, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2203_12339_amd.workloads import renderer_for  # noqa: E402

# 2562 vertices x 48 columns (FP16), then 642 vertices x 9 columns (FP32)
CASES = [("large-f16-163842", dict(subdiv=4, n_light=16, n_cfg=1)),
         ("haar-f32-10242", dict(subdiv=3, n_light=3, n_cfg=3))]
TOL = {"f32": 1e-5, "f16": 5e-3}


def test_noalloc_adjoint_matches_allocating_one():
    from oracle import adjoint
    for i, (name, kw) in enumerate(CASES):
        w = synth.get(name).with_(**kw)
        say(f"[noalloc] call {i + 1}: {name} N={w.n_vertices} columns={3 * w.n_out} storage={w.storage}")
        r = renderer_for(w)
        L, th = synth.make_lighting(w), synth.make_materials(w)
        r.set_lighting(dev_tensor(L, "f32"))
        r.set_material(dev_tensor(th, "f64"))
        B = r.render(save=True, force=True)
        bb = np.random.default_rng(5 + i).standard_normal(tuple(B.shape))
        dB = dev_tensor(bb, "f32")
        dSH = torch.full((w.n_light, w.n_sh, 3), float("nan"), dtype=torch.float32, device="cuda:0")
        dTh = torch.full((w.n_cfg, 3, 3), float("nan"), dtype=torch.float64, device="cuda:0")
        # the static-scratch entry point first, before this context ever allocated its own
        r.render_backward(dB, dSH, dTh, noalloc=True)
        torch.cuda.synchronize()
        gL, gT = dSH.cpu().numpy(), dTh.cpu().numpy()
        rL, rT = r.render_backward(dB)
        rL, rT = rL.cpu().numpy(), rT.cpu().numpy()
        assert np.all(np.isfinite(gL)) and np.all(np.isfinite(gT))
        assert np.array_equal(gL, rL), np.abs(gL - rL).max()
        assert np.array_equal(gT, rT), np.abs(gT - rT).max()
        if w.n_vertices <= 642:
            o = oracle_scene(w)
            oL, oT = adjoint.grad(o, L, th, bb)
            for g, ref, what in ((gL, oL, "lighting"), (gT, oT, "material")):
                err = np.abs(g - ref).max() / np.abs(ref).max()
                say(f"[noalloc] {name}: {what} gradient vs FP64 oracle {err:.3e}")
                assert err <= TOL[w.storage], err
        r.close()
