"""Dipole diffuse reflectance R_d(r; sigma_a, sigma_s', eta) -- Sec. 2.1, Eq. (4).

Readings of the printed formula (the source text is garbled in places):

* the second dipole term uses 1/d_v (the printed "1/d" has no subscript);
* sigma_t' = sigma_a + sigma_s' (printed as sigma_s + sigma_s');
* sigma_tr = sqrt(3 sigma_a sigma_t') (printed with sigma_s);
* z_v = z_r (1 + 4A/3) (the printed parenthesis is unbalanced);
* inputs are sigma_s' directly, so the anisotropy g is not needed.

Only with these readings does R_d integrate over the plane to the known
total diffuse reflectance of the dipole model (``total_reflectance``); the
tests check that integral numerically.  All functions accept complex input
so the derivatives can be checked with the complex-step method.
"""
from __future__ import annotations

import numpy as np

FOUR_PI = 4.0 * np.pi


def fdr(eta):
    """Diffuse Fresnel reflectance fit F_dr(eta) as printed in Sec. 2.1."""
    return -1.440 / eta**2 + 0.710 / eta + 0.668 + 0.0636 * eta


def dfdr_deta(eta):
    return 2.880 / eta**3 - 0.710 / eta**2 + 0.0636


def a_coef(eta):
    """Boundary coefficient A = (1 + F_dr) / (1 - F_dr)."""
    f = fdr(eta)
    return (1.0 + f) / (1.0 - f)


def _params(sa, ss, eta):
    st = sa + ss                      # sigma_t'
    alpha = ss / st                   # reduced albedo alpha'
    str_ = np.sqrt(3.0 * sa * st)     # effective transport coefficient
    zr = 1.0 / st
    A = a_coef(eta)
    cv = 1.0 + 4.0 * A / 3.0
    zv = zr * cv
    return st, alpha, str_, zr, A, cv, zv


def _term(z, d, s):
    """z (s + 1/d) exp(-s d) / d^2, one pole of the dipole."""
    return z * (s + 1.0 / d) * np.exp(-s * d) / d**2


def rd(r, sa, ss, eta):
    """R_d(r) of Eq. (4) (units 1/mm^2 for r in mm, sigma in 1/mm)."""
    st, alpha, s, zr, A, cv, zv = _params(sa, ss, eta)
    dr = np.sqrt(r * r + zr * zr)
    dv = np.sqrt(r * r + zv * zv)
    return alpha / FOUR_PI * (_term(zr, dr, s) + _term(zv, dv, s))


def _dterm_ds(z, d, s):
    # d/ds of z (s + 1/d) e^{-s d} / d^2  =  -s z e^{-s d} / d
    return -s * z * np.exp(-s * d) / d


def _dterm_dz(z, d, s):
    # total derivative w.r.t. z with d = sqrt(r^2 + z^2)
    e = np.exp(-s * d)
    h = (s + 1.0 / d) * e / d**2
    hp = -e / d**2 * (s * s + 3.0 * s / d + 3.0 / d**2)
    return h + z * hp * (z / d)


def rd_grad(r, sa, ss, eta):
    """(R_d, dR_d/dsigma_a, dR_d/dsigma_s', dR_d/deta) by the chain rule."""
    st, alpha, s, zr, A, cv, zv = _params(sa, ss, eta)
    dr = np.sqrt(r * r + zr * zr)
    dv = np.sqrt(r * r + zv * zv)
    S = _term(zr, dr, s) + _term(zv, dv, s)
    R = alpha / FOUR_PI * S
    dS_ds = _dterm_ds(zr, dr, s) + _dterm_ds(zv, dv, s)
    dS_dzr = _dterm_dz(zr, dr, s)
    dS_dzv = _dterm_dz(zv, dv, s)

    # partials of the intermediate quantities
    dalpha = (-ss / st**2, sa / st**2, 0.0)
    ds = (3.0 * (st + sa) / (2.0 * s), 3.0 * sa / (2.0 * s), 0.0)
    dzr = (-1.0 / st**2, -1.0 / st**2, 0.0)
    dA = 2.0 / (1.0 - fdr(eta)) ** 2 * dfdr_deta(eta)
    dzv = (cv * dzr[0], cv * dzr[1], zr * 4.0 / 3.0 * dA)

    out = [R]
    for p in range(3):
        dSp = dS_ds * ds[p] + dS_dzr * dzr[p] + dS_dzv * dzv[p]
        out.append(dalpha[p] / FOUR_PI * S + alpha / FOUR_PI * dSp)
    return tuple(out)


def total_reflectance(sa, ss, eta):
    """Closed-form integral of R_d over the plane (Jensen et al.'s dipole).

    2*pi * int_0^inf r R_d(r) dr
      = alpha'/2 (1 + exp(-4/3 A sqrt(3(1-alpha')))) exp(-sqrt(3(1-alpha'))).
    Used only as an independent pin of ``rd``.
    """
    st = sa + ss
    alpha = ss / st
    A = a_coef(eta)
    q = np.sqrt(3.0 * (1.0 - alpha))
    return alpha / 2.0 * (1.0 + np.exp(-4.0 / 3.0 * A * q)) * np.exp(-q)


def sphere_uniform_response(R, sa, ss, eta):
    """Dipole response of a uniformly lit sphere of radius R, per unit E.

    On a sphere the area at distance r from any point is 2*pi*r dr for
    r in [0, 2R], so int_sphere R_d dA = int_0^{2R} 2 pi r R_d(r) dr, which has
    the closed form below (each pole integrates to z [e^{-s z} -
    e^{-s D}/D]/... evaluated at D = sqrt(4R^2 + z^2)).  Independent pin of
    the whole discrete gather in the limit of fine meshes.
    """
    st, alpha, s, zr, A, cv, zv = _params(sa, ss, eta)
    out = 0.0
    for z in (zr, zv):
        D = np.sqrt(4.0 * R * R + z * z)
        out = out + np.exp(-s * z) - z * np.exp(-s * D) / D
    return alpha / 2.0 * out
