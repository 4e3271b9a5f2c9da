"""Pins of the Fresnel factor (Eq. 3 and the outgoing factor of Eq. 6)."""
import numpy as np
import pytest

import synth
from oracle import dipole, fresnel
from oracle.transport import Scene


@pytest.mark.parametrize("eta", [1.1, 1.3, 1.45, 1.6])
def test_normal_and_grazing_incidence(eta):
    # normal incidence: F_r = ((eta - 1) / (eta + 1))^2
    assert abs(fresnel.fresnel_t(eta, 1.0) - 4 * eta / (eta + 1) ** 2) < 1e-15
    assert fresnel.fresnel_t(eta, 1e-9) < 1e-8 and fresnel.fresnel_t(eta, -0.3) == 0.0
    # Brewster angle tan(theta) = eta: the p wave is fully transmitted
    th = np.arctan(eta)
    c, s = np.cos(th), np.sin(th)
    ct = np.sqrt(1 - (s / eta) ** 2)
    rs = (c - eta * ct) / (c + eta * ct)
    assert abs(fresnel.fresnel_r(eta, c) - 0.5 * rs * rs) < 1e-15


@pytest.mark.parametrize("eta", [1.1, 1.2, 1.3, 1.4, 1.5, 1.6])
def test_internal_diffuse_reflectance_matches_printed_fdr(eta):
    """The F_dr polynomial printed with Eq. (4) is a fit of the internal
    diffuse Fresnel reflectance; the Fresnel function integrated over the
    inside hemisphere reproduces it to the fit's accuracy (2e-3)."""
    fit = dipole.fdr(eta)
    assert abs(fresnel.internal_diffuse_reflectance(eta) - fit) < 2e-3


def test_view_factor_shape_and_range():
    w = synth.get("haar-f32-10242").with_(subdiv=2, n_light=2, n_cfg=2)
    sc = Scene(w)
    th = synth.make_materials(w)
    eye = np.array([30.0, 10.0, -5.0])
    f = fresnel.view_factor(sc, eye, th)
    assert f.shape == (w.n_out, sc.N, 3)
    assert f.min() >= 0.0 and f.max() <= 1.0 / np.pi
    d = eye[None, :] - sc.V
    back = np.einsum("ij,ij->i", sc.normal, d) <= 0
    assert back.any() and (~back).any()
    assert np.all(f[:, back, :] == 0.0) and np.all(f[:, ~back, :] > 0.0)
