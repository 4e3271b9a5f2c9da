"""Fresnel transmittance and the outgoing factor of Eq. (3) and (6).

TEST INFRASTRUCTURE ONLY (see the package header).

The dipole BSSRDF of Eq. (3) carries (1/pi) F_t(eta, w_i) ... F_t(eta, w_o);
the method's radiance, the last line of Eq. (6), keeps the outgoing factor
(1/pi) F_t(eta, w_o) in front of the transport and folds the incident one
into E.  F_t = 1 - F_r with F_r the unpolarised Fresnel reflectance of a
smooth dielectric boundary, air (index 1) outside and index eta inside, for
an outside direction at angle theta to the normal:

    sin t = sin(theta) / eta,
    r_s = (cos theta - eta cos t) / (cos theta + eta cos t),
    r_p = (eta cos theta - cos t) / (eta cos theta + cos t),
    F_r = (r_s^2 + r_p^2) / 2.

A vertex seen from behind (n . w_o <= 0) sends no radiance toward the eye:
its factor is 0.
"""
from __future__ import annotations

import numpy as np

from .transport import mat_of


def fresnel_r(eta, cos_o):
    """Reflectance for outside incidence at cos(theta) = cos_o in [0, 1]."""
    eta = np.asarray(eta, dtype=np.float64)
    c = np.asarray(cos_o, dtype=np.float64)
    s2 = (1.0 - c * c) / (eta * eta)
    ct = np.sqrt(1.0 - s2)
    rs = (c - eta * ct) / (c + eta * ct)
    rp = (eta * c - ct) / (eta * c + ct)
    return 0.5 * (rs * rs + rp * rp)


def fresnel_t(eta, cos_o):
    """Transmittance F_t = 1 - F_r; 0 for cos_o <= 0."""
    c = np.asarray(cos_o, dtype=np.float64)
    cc = np.clip(c, 0.0, 1.0)
    return np.where(c > 0.0, 1.0 - fresnel_r(eta, cc), 0.0)


def internal_diffuse_reflectance(eta, n=20001):
    """Hemispherical (cosine-weighted) reflectance for light inside the
    medium: 2 int_0^{pi/2} F_r,in(theta) cos sin dtheta, with the inside
    reflectance equal to the outside one at the refracted angle and 1 past
    the critical angle.  The dipole's F_dr polynomial (Eq. 4) fits this."""
    th = np.linspace(0.0, np.pi / 2, n)
    s_out = eta * np.sin(th)
    tir = s_out >= 1.0
    cos_out = np.sqrt(np.clip(1.0 - s_out * s_out, 0.0, 1.0))
    fr = np.where(tir, 1.0, fresnel_r(eta, cos_out))
    f = fr * np.cos(th) * np.sin(th)
    return 2.0 * np.trapezoid(f, th)


def view_factor(scene, eye, theta):
    """(1/pi) F_t(eta[mat(q), ch], w_o(v)) for every output set q, vertex v
    (original order) and channel: [n_out, N, 3]."""
    w = scene.w
    eye = np.asarray(eye, dtype=np.float64)
    d = eye[None, :] - scene.V
    cos_o = np.einsum("ij,ij->i", scene.normal, d) / np.linalg.norm(d, axis=1)
    theta = np.asarray(theta, dtype=np.float64)
    out = np.empty((w.n_out, scene.N, 3))
    for q in range(w.n_out):
        for ch in range(3):
            out[q, :, ch] = fresnel_t(theta[mat_of(w, q), ch, 2], cos_o) / np.pi
    return out
