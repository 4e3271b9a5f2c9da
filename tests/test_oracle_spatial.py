"""Pins of the spatial-compression oracle: the CDF 9/7 transform w_1 (9/7 per
Sec. 5) and the energy-thresholded output-side compression of Sec. 3.2
(Eq. 9, 10; precompute Step 2) with the inverse of Step 5 of Sec. 4."""
import numpy as np
import pytest

import synth
from oracle import cdf97
from oracle.spatial import Spatial
from oracle.transport import Scene

# The CDF 9/7 analysis filters as published (Cohen, Daubechies and Feauveau
# 1992; the irreversible filter of JPEG 2000), low-pass with DC gain 1 and
# high-pass with Nyquist gain 2: centre tap first, then the taps at +-1, +-2 ...
PUBLISHED_LOW = [0.602949018236, 0.266864118443, -0.078223266529, -0.016864118443, 0.026748757411]
PUBLISHED_HIGH = [1.115087052457, -0.591271763114, -0.057543526229, 0.091271763114]
# Its lifting factorisation (Daubechies and Sweldens 1998), as used by JPEG 2000
LIFT = (-1.586134342059924, -0.052980118572961, 0.882911075530934, 0.443506852043971)
LIFT_K = 1.230174104914001


def test_filters_match_published_taps():
    h, g, r = cdf97.filters()
    assert h.shape == (9,) and g.shape == (7,)
    np.testing.assert_allclose(h[4:] / np.sqrt(2), PUBLISHED_LOW, atol=2e-12)
    np.testing.assert_allclose(h[:5][::-1] / np.sqrt(2), PUBLISHED_LOW, atol=2e-12)
    np.testing.assert_allclose(g[3:] * np.sqrt(2), PUBLISHED_HIGH, atol=2e-12)
    np.testing.assert_allclose(g[:4][::-1] * np.sqrt(2), PUBLISHED_HIGH, atol=2e-12)
    assert abs(1 + 4 * r + 10 * r ** 2 + 20 * r ** 3) < 1e-14


def test_vanishing_moments():
    """Four vanishing moments: the high-pass kills cubics, the low-pass has
    a fourth-order zero at Nyquist."""
    h, g, _ = cdf97.filters()
    m9, m7 = np.arange(-4, 5), np.arange(-3, 4)
    for p in range(4):
        assert abs((g * m7.astype(float) ** p).sum()) < 1e-12, p
        assert abs((h * (-1.0) ** m9 * m9.astype(float) ** p).sum()) < 1e-12, p
    assert abs(h.sum() - np.sqrt(2)) < 1e-14
    assert abs((g * (-1.0) ** m7).sum() - np.sqrt(2)) < 1e-14


def _lifting_level(x):
    """One analysis level by the lifting steps, symmetric at both ends."""
    x = np.array(x, dtype=np.float64)
    n = len(x)

    def at(i):
        return x[-i if i < 0 else (2 * (n - 1) - i if i > n - 1 else i)]
    for c, parity in zip(LIFT, (1, 0, 1, 0)):
        upd = [x[i] + c * (at(i - 1) + at(i + 1)) for i in range(parity, n, 2)]
        x[parity::2] = upd
    return np.concatenate([x[0::2] * np.sqrt(2) / LIFT_K, x[1::2] * LIFT_K / np.sqrt(2)])


@pytest.mark.parametrize("n", [8, 9, 10, 13, 16, 31, 64, 101])
def test_one_level_equals_lifting(n):
    x = np.random.default_rng(n).standard_normal(n)
    np.testing.assert_allclose(cdf97.analysis_matrix(n) @ x, _lifting_level(x), atol=1e-13)


def test_synthesis_filters_in_the_interior():
    """Away from the ends the inverse of one level is the synthesis bank:
    low coefficient i -> f centred on 2i, high coefficient i -> the
    modulated analysis low-pass centred on 2i+1."""
    h, g, _ = cdf97.filters()
    f = g * (-1.0) ** np.abs(np.arange(-3, 4))
    n = 64
    n_lo = n // 2
    for i, band in ((12, "low"), (13, "high")):
        z = np.zeros(n)
        z[i if band == "low" else n_lo + i] = 1.0
        x = cdf97.inverse(z, levels=1)
        if band == "low":
            np.testing.assert_allclose(x[2 * i - 3:2 * i + 4], f, atol=1e-13)
            assert np.abs(np.delete(x, range(2 * i - 3, 2 * i + 4))).max() < 1e-13
        else:
            hs = h * (-1.0) ** np.abs(np.arange(-4, 5))
            np.testing.assert_allclose(x[2 * i + 1 - 4:2 * i + 1 + 5], hs, atol=1e-13)


@pytest.mark.parametrize("n", [8, 12, 642, 1000, 2562])
def test_multilevel_layout_inverse_and_constants(n):
    sizes = cdf97.band_sizes(n)
    assert sizes[0] == n and (sizes[-1] + 1) // 2 < 8 <= sizes[-1]
    x = np.random.default_rng(n).standard_normal((n, 3))
    z = cdf97.forward(x)
    np.testing.assert_allclose(cdf97.inverse(z), x, atol=1e-11)
    # near-orthonormal: white noise keeps its energy within a few percent
    # (short lists are dominated by the reflected ends)
    if n >= 600:
        assert 0.9 < (z ** 2).sum() / (x ** 2).sum() < 1.1
    # a constant has no detail at any level, ends included
    zc = cdf97.forward(np.full(n, 2.5))
    n_low = (sizes[-1] + 1) // 2
    assert np.abs(zc[n_low:]).max() < 1e-12
    assert np.abs(zc[:n_low] - 2.5 * np.sqrt(2) ** len(sizes)).max() < 1e-11


def test_spatial_untruncated_equals_step1_render():
    """tau = 1 keeps every non-zero coefficient: w_1^{-1} w_1 = I gives the
    Step-1 radiance (itself pinned by the dense sums)."""
    w = synth.get("haar-f32-10242").with_(subdiv=2, n_light=2, n_cfg=2, keep=0.25)
    sc = Scene(w)
    L, th = synth.make_lighting(w), synth.make_materials(w)
    s = Spatial(sc, energy=1.0)
    B = s.render(L, th)
    ref = sc.render(L, th)
    np.testing.assert_allclose(B, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    E = synth.make_irradiance(w)
    np.testing.assert_allclose(s.render(None, th, E=E), sc.render(None, th, E=E),
                               rtol=0, atol=1e-12 * np.abs(ref).max())


def test_energy_selection_is_the_minimal_largest_set():
    """S2 by brute force on a small case: retained energy reaches tau, no
    dropped entry is larger than a kept one, and dropping the smallest kept
    entry falls below tau."""
    w = synth.get("haar-f32-10242").with_(subdiv=2, keep=0.25)
    s = Spatial(Scene(w), energy=0.97)
    for k in range(s.Z.shape[0]):
        z2 = s.Z[k] ** 2
        kept = z2[s.keep[k]]
        tot = z2.sum()
        assert kept.sum() >= 0.97 * tot * (1 - 1e-14)
        assert kept.sum() - kept.min() < 0.97 * tot
        dropped = z2[~s.keep[k]]
        assert dropped.size == 0 or dropped.max() <= kept.min()
    cnt, frac = s.stats()
    assert (frac >= 0.97 - 1e-12).all() and (cnt < s.Z[0].size).all()


def test_spatial_compression_shrinks_and_error_follows_energy():
    """More retained energy, more kept entries and a smaller deviation from
    the Step-1 radiance (information, not a parity bound)."""
    w = synth.get("haar-f32-10242").with_(subdiv=3, keep=None)
    w = w.with_(keep=64 / w.n_vertices)
    sc = Scene(w)
    L, th = synth.make_lighting(w), synth.make_materials(w)
    ref = sc.render(L, th)
    s = Spatial(sc, energy=0.95)
    errs, counts = [], []
    for tau in (0.95, 0.98, 0.995):
        keep = s.select(tau)
        counts.append(keep.sum())
        B = s.render(L, th, keep=keep)
        errs.append(np.abs(B - ref).max() / np.abs(ref).max())
    step1_nnz = w.K * w.n_vertices * w.n_keep
    assert counts[0] < counts[1] < counts[2]
    assert errs[0] > errs[2]
    assert counts[0] < step1_nnz
