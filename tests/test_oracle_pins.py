"""Pins of the FP64 oracle against facts other than itself (CPU only).

Each test checks the oracle against a closed form, a library routine, a
quadrature, a hand-worked example under tests/golden/, an invariant, or a
brute-force evaluation -- chosen so a dropped term, wrong sign, wrong index
or transposed operand in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import sph_harm_y

import synth
from oracle import adjoint, dipole, geometry, haar, pca, sh
from oracle.transport import Scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MATS = [(0.001, 0.5, 1.3), (0.05, 3.0, 1.3), (0.02, 1.0, 1.5), (0.01, 2.0, 1.1)]


# --------------------------------------------------------------------------
# Dipole R_d, Eq. (4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("th", MATS)
def test_rd_integrates_to_total_diffuse_reflectance(th):
    """2 pi int r R_d dr equals the dipole's closed-form total reflectance.

    Fails for each of the garbled-symbol alternatives (1/d instead of 1/d_v,
    sigma_t' = sigma_s + sigma_s', sigma_tr with sigma_s, z_v without the
    4A/3 term)."""
    val = quad(lambda r: 2 * np.pi * r * dipole.rd(r, *th), 0, np.inf,
               limit=500, epsabs=0, epsrel=1e-13)[0]
    assert val == pytest.approx(dipole.total_reflectance(*th), rel=1e-11)


def test_fdr_printed_polynomial():
    # F_dr(1.3) by hand from the printed coefficients.
    e = 1.3
    v = -1.440 / 1.69 + 0.710 / 1.3 + 0.668 + 0.0636 * 1.3
    assert dipole.fdr(e) == pytest.approx(v, rel=1e-15)
    assert dipole.fdr(e) == pytest.approx(0.444763, abs=1e-6)
    assert dipole.a_coef(e) == pytest.approx(2.60207, abs=1e-5)


@pytest.mark.parametrize("th", MATS)
def test_rd_grad_complex_step(th):
    r = np.array([0.0, 0.05, 0.7, 3.0, 11.0, 20.4])
    R, *grads = dipole.rd_grad(r, *th)
    np.testing.assert_allclose(R, dipole.rd(r, *th), rtol=1e-15)
    h = 1e-30
    for p in range(3):
        x = [complex(v) for v in th]
        x[p] += 1j * h
        cs = dipole.rd(r, *x).imag / h
        np.testing.assert_allclose(grads[p], cs, rtol=1e-12, atol=0)


@pytest.mark.parametrize("th", MATS[:3])
def test_sphere_uniform_closed_form(th):
    R = 10.0
    val = quad(lambda r: 2 * np.pi * r * dipole.rd(r, *th), 0, 2 * R,
               limit=500, epsabs=0, epsrel=1e-13)[0]
    assert val == pytest.approx(dipole.sphere_uniform_response(R, *th), rel=1e-11)


# --------------------------------------------------------------------------
# Spherical harmonics and transfer
# --------------------------------------------------------------------------

def _sphere_quadrature(n_t=24, n_p=48):
    z, wz = np.polynomial.legendre.leggauss(n_t)
    ph = (np.arange(n_p) + 0.5) * 2 * np.pi / n_p
    Z, PH = np.meshgrid(z, ph, indexing="ij")
    s = np.sqrt(1 - Z**2)
    d = np.stack([s * np.cos(PH), s * np.sin(PH), Z], -1).reshape(-1, 3)
    wts = (wz[:, None] * np.full(n_p, 2 * np.pi / n_p)[None, :]).reshape(-1)
    return d, wts


def test_sh_orthonormal():
    d, wts = _sphere_quadrature()
    Y = sh.real_sh(5, d)
    G = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(36), atol=1e-13)


def test_sh_closed_forms_and_library():
    rng = np.random.default_rng(0)
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    x, y, z = d.T
    Y = sh.real_sh(5, d)
    np.testing.assert_allclose(Y[:, 0], 0.5 / math.sqrt(math.pi), rtol=1e-15)
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(Y[:, 1:4], c1 * np.stack([y, z, x], 1), rtol=1e-14)
    np.testing.assert_allclose(Y[:, 6], math.sqrt(5 / (16 * math.pi)) * (3 * z * z - 1),
                               rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Y[:, 8], math.sqrt(15 / (16 * math.pi)) * (x * x - y * y),
                               rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(Y[:, 4], math.sqrt(15 / (4 * math.pi)) * x * y,
                               rtol=1e-13, atol=1e-15)
    # scipy's complex SH (with Condon-Shortley phase) mapped to this basis.
    th, ph = np.arccos(z), np.arctan2(y, x)
    for l in range(6):
        for m in range(l + 1):
            ys = sph_harm_y(l, m, th, ph)
            if m == 0:
                np.testing.assert_allclose(Y[:, l * l + l], ys.real, atol=1e-14)
            else:
                f = math.sqrt(2) * (-1) ** m
                np.testing.assert_allclose(Y[:, l * l + l + m], f * ys.real, atol=1e-14)
                np.testing.assert_allclose(Y[:, l * l + l - m], f * ys.imag, atol=1e-14)


def test_clamped_cosine_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "clamped_cosine.txt"))
            if l.strip() and not l.startswith("#")]
    ah = sh.clamped_cosine_coeffs(5)
    for l, v in rows:
        assert ah[int(l)] == pytest.approx(float(v), abs=1e-14)


def test_transfer_matches_hemisphere_quadrature():
    """T[i,lm] = int max(n.w,0) Y_lm(w) dw, integrated in a frame around n."""
    rng = np.random.default_rng(1)
    n = rng.standard_normal((6, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    T = sh.transfer(n, 36)
    t, wt = np.polynomial.legendre.leggauss(40)
    t = 0.5 * (t + 1)
    wt = 0.5 * wt
    n_p = 64
    ph = (np.arange(n_p) + 0.5) * 2 * np.pi / n_p
    for i in range(n.shape[0]):
        a = np.array([1.0, 0, 0]) if abs(n[i, 0]) < 0.9 else np.array([0, 1.0, 0])
        u = np.cross(n[i], a)
        u /= np.linalg.norm(u)
        v = np.cross(n[i], u)
        T_, P_ = np.meshgrid(t, ph, indexing="ij")
        s = np.sqrt(1 - T_**2)
        dirs = (s * np.cos(P_))[..., None] * u + (s * np.sin(P_))[..., None] * v \
            + T_[..., None] * n[i]
        wts = wt[:, None] * np.full(n_p, 2 * np.pi / n_p)[None, :] * T_
        Y = sh.real_sh(5, dirs.reshape(-1, 3))
        ref = (Y * wts.reshape(-1, 1)).sum(0)
        np.testing.assert_allclose(T[i], ref, atol=1e-12)


# --------------------------------------------------------------------------
# Geometry
# --------------------------------------------------------------------------

def test_icosahedron_areas_golden():
    vals = dict(l.split() for l in open(os.path.join(GOLDEN, "icosahedron.txt"))
                if l.strip() and not l.startswith("#"))
    V, F = synth.icosphere(0)
    A = geometry.vertex_areas(V, F)
    np.testing.assert_allclose(A, float(vals["vertex_area"]), rtol=1e-14)
    assert A.sum() == pytest.approx(float(vals["total_area"]), rel=1e-14)
    e = np.linalg.norm(V[F[0, 0]] - V[F[0, 1]])
    assert e == pytest.approx(float(vals["edge"]), rel=1e-14)
    # On the regular solid each vertex normal is the radial direction.
    np.testing.assert_allclose(geometry.vertex_normals(V, F), V, atol=1e-14)


def test_vertex_normals_weight_faces_by_area():
    """Reading 10 on a vertex where the weighting shows: vertex 0 lies on a
    face of area 1/2 with normal +z and a face of area 3/2 with normal +x,
    so its area-weighted normal is (3, 0, 1)/sqrt(10) (a plain average of
    the face normals would give (1, 0, 1)/sqrt(2)), and its area is
    (1/2 + 3/2)/3.  Worked by hand."""
    V = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 3, 0], [0, 0, 1]])
    F = np.array([[0, 1, 2], [0, 3, 4]])
    n = geometry.vertex_normals(V, F)
    np.testing.assert_allclose(n[0], np.array([3.0, 0.0, 1.0]) / np.sqrt(10.0), rtol=0, atol=1e-15)
    np.testing.assert_allclose(n[1], [0.0, 0.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(n[3], [1.0, 0.0, 0.0], atol=1e-15)
    A = geometry.vertex_areas(V, F)
    np.testing.assert_allclose(A, [2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 0.5, 0.5], rtol=1e-15)


def test_mesh_sizes_and_areas():
    for s, n in [(0, 12), (1, 42), (2, 162), (3, 642)]:
        w = synth.get("dense-f64-642").with_(subdiv=s)
        V, F = synth.make_mesh(w)
        assert V.shape[0] == n == w.n_vertices
        A = geometry.vertex_areas(V, F)
        tri = 0.5 * np.linalg.norm(geometry.face_cross(V, F), axis=1).sum()
        assert A.sum() == pytest.approx(tri, rel=1e-13)
        r = np.linalg.norm(V, axis=1)
        assert np.all(r >= w.radius * (1 - w.noise) - 1e-12)
        assert np.all(r <= w.radius * (1 + w.noise) + 1e-12)
    # Euler characteristic of a closed genus-0 triangulation.
    V, F = synth.icosphere(3)
    assert V.shape[0] - 3 * F.shape[0] // 2 + F.shape[0] == 2


def test_morton_hand_example_and_bijection():
    # Four points on the bbox corners/centre of [0,1]^3.
    V = np.array([[1.0, 1.0, 1.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    k = geometry.morton_keys(V)
    top = (1 << 21) - 1
    assert int(k[1]) == 0
    # x only: bits at positions 3b+2 for every b
    assert int(k[2]) == sum(1 << (3 * b + 2) for b in range(21))
    assert int(k[3]) == sum(1 << (3 * b) for b in range(21))
    assert int(k[0]) == (1 << 63) - 1
    assert top == 2097151
    assert list(geometry.morton_perm(V)) == [1, 3, 2, 0]
    V, F = synth.make_mesh(synth.get("haar-f32-10242"))
    p = geometry.morton_perm(V)
    assert np.array_equal(np.sort(p), np.arange(V.shape[0]))
    keys = geometry.morton_keys(V)[p]
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)
    # Locality: consecutive Morton vertices are much closer than random pairs.
    step = np.linalg.norm(np.diff(V[p], axis=0), axis=1).mean()
    rnd = np.linalg.norm(V - V[np.random.default_rng(0).permutation(V.shape[0])], axis=1).mean()
    assert step < 0.1 * rnd


# --------------------------------------------------------------------------
# Haar, Eq. (8)
# --------------------------------------------------------------------------

def test_haar_golden():
    for line in open(os.path.join(GOLDEN, "haar_worked.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        a, b = line.split(";")
        x = np.array(a.split(), dtype=float)
        y = np.array(b.split(), dtype=float)
        np.testing.assert_allclose(haar.haar(x), y, rtol=1e-15, atol=1e-15)


def test_haar_orthonormal_and_inverse():
    rng = np.random.default_rng(2)
    for n in (1, 2, 8, 64, 1024):
        H = haar.matrix(n)
        np.testing.assert_allclose(H.T @ H, np.eye(n), atol=1e-14)
        x = rng.standard_normal((3, n))
        c = haar.haar(x)
        np.testing.assert_allclose(haar.ihaar(c), x, atol=1e-13)
        np.testing.assert_allclose((c**2).sum(-1), (x**2).sum(-1), rtol=1e-13)
        # each detail row of H: +/- 2^(-(n-m)/2) on its dyadic block halves
        if n >= 8:
            j = 5                          # level m=2, block b=1
            blk = n // 4
            row = np.zeros(n)
            row[blk:blk + blk // 2] = 1
            row[blk + blk // 2:2 * blk] = -1
            np.testing.assert_allclose(H[j], row / math.sqrt(blk), atol=1e-15)


# --------------------------------------------------------------------------
# PCA, Eq. (5)
# --------------------------------------------------------------------------

def test_pca_full_rank_and_eckart_young():
    w = synth.get("haar-f32-10242")
    rn = pca.r_nodes(w.r_max)
    mats = pca.material_grid(synth.MATERIAL_GRID)
    M = pca.table(rn, mats)
    b, s = pca.basis(M)
    np.testing.assert_allclose(b @ b.T, np.eye(256), atol=1e-12)
    # full-rank reconstruction for materials inside and outside the table
    th = np.array([[0.013, 1.7, 1.3], [0.049, 0.6, 1.45], [0.002, 3.9, 1.2]])
    g = pca.weights(th, rn, b)
    R = dipole.rd(rn[None, :], th[:, 0:1], th[:, 1:2], th[:, 2:3])
    np.testing.assert_allclose(g @ b, R, rtol=0, atol=1e-12 * np.abs(R).max())
    for K in (4, 6, 8):
        MK = pca.weights(mats, rn, b[:K]) @ b[:K]
        resid = np.linalg.norm(M - MK)
        assert resid == pytest.approx(math.sqrt((s[K:] ** 2).sum()), rel=1e-8)
    # sign rule and descending spectrum
    assert np.all(np.diff(s) <= 0)
    assert np.all(b[np.arange(256), np.argmax(np.abs(b), axis=1)] > 0)


def test_weight_grads_complex_step():
    w = synth.get("dense-f64-642")
    rn = pca.r_nodes(w.r_max)
    M = pca.table(rn, pca.material_grid(synth.MATERIAL_GRID))
    b, _ = pca.basis(M, 8)
    th = np.array([0.02, 1.3, 1.4])
    dg = pca.weight_grads(th, rn, b)
    for p in range(3):
        x = th.astype(complex)
        x[p] += 1e-30j
        np.testing.assert_allclose(dg[:, p], pca.weights(x, rn, b).imag / 1e-30,
                                   rtol=1e-11, atol=1e-14 * np.abs(dg).max())


# --------------------------------------------------------------------------
# Transport: O-B against O-A' and closed forms
# --------------------------------------------------------------------------

def _small(wavelet, subdiv=2, **kw):
    w = synth.get("dense-f64-642").with_(subdiv=subdiv, wavelet=wavelet, keep=None, **kw)
    return w, Scene(w, K=256)


@pytest.mark.parametrize("wavelet", ["none", "haar"])
def test_full_rank_untruncated_equals_interpolated_gather(wavelet):
    """K = 256, no truncation: O-B == O-A' (R_d interpolated on the nodes).

    Pins the Morton permutation, the area weighting, the Haar rows, the
    irradiance side and the PCA weights together (Eq. 7 and 8)."""
    w, s = _small(wavelet, n_light=2, n_cfg=2)
    L = synth.make_lighting(w)
    th = synth.make_materials(w)
    B = s.render(L, th)
    Bi = s.gather_plain(L, th, interpolated=True)
    np.testing.assert_allclose(B, Bi, rtol=0, atol=1e-11 * np.abs(Bi).max())


def test_uniform_sphere_converges_to_closed_form():
    """DC lighting on a noise-free sphere gives E = sqrt(pi)/2 L00 everywhere
    and B -> E * sphere_uniform_response; the gather converges O(h^2)."""
    th = np.array([[[0.01, 1.0, 1.3]] * 3])
    errs = []
    for s_ in (2, 3, 4):
        w = synth.get("dense-f64-642").with_(subdiv=s_, noise=0.0, n_sh=1, wavelet="none")
        sc = Scene(w, K=4)
        L = np.zeros((1, 1, 3))
        L[0, 0, :] = 1.0
        E = sc.irradiance(L)
        np.testing.assert_allclose(E, math.sqrt(math.pi) / 2, rtol=1e-14)
        B = sc.gather_plain(L, th)
        ref = math.sqrt(math.pi) / 2 * dipole.sphere_uniform_response(10.0, 0.01, 1.0, 1.3)
        errs.append(np.abs(B - ref).max() / ref)
    assert errs[-1] < 0.01
    assert errs[1] < errs[0] / 2.5 and errs[2] < errs[1] / 2.5


def test_linearity_and_reciprocity():
    w = synth.get("dense-f64-642").with_(subdiv=2, n_light=3, n_cfg=1, keep=None, wavelet="haar")
    s = Scene(w)
    L = synth.make_lighting(w)
    th = synth.make_materials(w)
    B = s.render(L, th)
    # linearity: lighting 2 := 2*L0 - 0.5*L1
    L2 = L.copy()
    L2[2] = 2 * L[0] - 0.5 * L[1]
    B2 = s.render(L2, th)
    np.testing.assert_allclose(B2[2], 2 * B[0] - 0.5 * B[1], atol=1e-12 * np.abs(B).max())
    # reciprocity: E1^T D_A B(E0) == E0^T D_A B(E1), kernel symmetric in (o, i)
    E = s.irradiance(L)
    a = s.area
    lhs = np.einsum("i,ic,ic->c", a, E[1], B[0])
    rhs = np.einsum("i,ic,ic->c", a, E[0], B[1])
    np.testing.assert_allclose(lhs, rhs, rtol=1e-11)


def test_supplied_irradiance_path():
    """Step 1 of Sec. 4 with E given instead of T L: E = T L reproduces the
    SH path; Haar of A*E keeps the energy (orthonormal) and its scaling
    coefficient is the area-weighted sum over sqrt(n_pad); untruncated, the
    radiance is the dense sum of Eq. (7) over the PCA kernels."""
    w = synth.get("dense-f64-642").with_(subdiv=1, n_light=2, n_cfg=2, keep=None, wavelet="haar")
    s = Scene(w)
    L = synth.make_lighting(w)
    th = synth.make_materials(w)
    E_tl = np.stack([s.T @ L[l] for l in range(w.n_light)])
    np.testing.assert_allclose(s.ehat(E=E_tl), s.ehat(L), rtol=0, atol=1e-13)
    E = synth.make_irradiance(w)
    assert E.shape == (2, s.N, 3) and E.min() >= 0
    Eh = s.ehat(E=E)
    AE = E * s.area[None, :, None]
    np.testing.assert_allclose((Eh ** 2).sum(axis=1), (AE ** 2).sum(axis=1), rtol=1e-12)
    np.testing.assert_allclose(Eh[:, 0, :], AE.sum(axis=1) / np.sqrt(s.n_pad), rtol=1e-12)
    B = s.render(None, th, E=E)
    g = s.g(th)                                            # [m, ch, k]
    Kr = s.kernel_rows(np.arange(s.N))                     # [k, p, p'] Morton order
    AEm = AE[:, s.perm, :]
    ref = np.einsum("qck,kpr,qrc->qpc", g, Kr, AEm)
    Bm = B[:, s.perm, :]
    np.testing.assert_allclose(Bm, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_selection_matches_brute_force_sort():
    w = synth.get("dense-f64-642").with_(subdiv=1, keep=0.25, wavelet="haar")
    s = Scene(w)
    rng = np.random.default_rng(3)
    Wr = rng.integers(-4, 5, size=(3, 7, 64)).astype(float)   # many ties
    keep = s.select(Wr)
    nk = w.n_keep
    for idx in np.ndindex(Wr.shape[:-1]):
        row = Wr[idx]
        order = sorted(range(64), key=lambda j: (-abs(row[j]), j))[:nk]
        assert set(np.flatnonzero(keep[idx])) == set(order)


def test_truncation_keeps_the_largest_and_reduces_to_dense():
    w = synth.get("haar-f32-10242").with_(subdiv=3, keep=0.05)
    s = Scene(w)
    cols, vals = s.kept_lists(np.arange(0, s.N, 37))
    assert cols.shape[-1] == w.n_keep == round(0.05 * 642)
    assert np.all(np.diff(cols, axis=-1) > 0)
    Wr = s.wavelet_rows(np.arange(0, s.N, 37))
    thr = np.sort(np.abs(Wr), axis=-1)[..., -w.n_keep]
    assert np.all(np.abs(vals) >= thr[..., None])
    # untruncated wavelet rows reproduce the spatial kernel (Eq. 8)
    Kr = s.kernel_rows(np.arange(5))
    np.testing.assert_allclose(haar.ihaar(s.wavelet_rows(np.arange(5)))[..., :s.N], Kr,
                               atol=1e-13)


# --------------------------------------------------------------------------
# Adjoint
# --------------------------------------------------------------------------

def test_adjoint_dot_product_and_fd():
    w = synth.get("grad-f64-642").with_(subdiv=1, wavelet="haar", keep=0.3)
    s = Scene(w)
    L = synth.make_lighting(w)
    th = synth.make_materials(w)
    Lt, tht = synth.perturb_target(w, L, th)
    Bt = s.render(Lt, tht)
    B = s.render(L, th)
    gL, gT = adjoint.grad(s, L, th, B - Bt)
    # dot-product test in the lighting direction (B is linear in L)
    rng = np.random.default_rng(4)
    dL = rng.standard_normal(L.shape)
    bb = rng.standard_normal(B.shape)
    lhs = np.sum(bb * s.render(dL, th))
    gLb, _ = adjoint.grad(s, L, th, bb)
    assert lhs == pytest.approx(np.sum(gLb * dL), rel=1e-12)
    fL, fT = adjoint.fd_grad(s, L, th, Bt)
    np.testing.assert_allclose(gL, fL, rtol=1e-6, atol=1e-9 * np.abs(fL).max())
    np.testing.assert_allclose(gT, fT, rtol=1e-6, atol=1e-9 * np.abs(fT).max())
    # bands 3 and 5 of the clamped-cosine transfer are zero
    w5 = w.with_(n_sh=36)
    s5 = Scene(w5)
    L5 = synth.make_lighting(w5)
    g5, _ = adjoint.grad(s5, L5, th, s5.render(L5, th))
    big = np.abs(g5).max()
    for l in (3, 5):
        assert np.abs(g5[:, l * l:(l + 1) ** 2]).max() < 1e-13 * big


def test_adjoint_on_sampled_rows_equals_masked_full():
    w = synth.get("haar-f32-10242").with_(subdiv=2, keep=0.1, n_light=2, n_cfg=2)
    s = Scene(w)
    L = synth.make_lighting(w)
    th = synth.make_materials(w)
    rows = np.array([3, 17, 40, 41, 100])
    rng = np.random.default_rng(5)
    bb = rng.standard_normal((2, len(rows), 3))
    full = np.zeros((2, s.N, 3))
    full[:, s.perm[rows], :] = bb
    a = adjoint.grad(s, L, th, bb, rows=rows)
    b = adjoint.grad(s, L, th, full)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-14 * np.abs(y).max())
