"""Continuum (anisotropic) Green function in the line-mode representation (FP64 oracle;
test infrastructure only).

Section 3.1, eq. cgf: the continuum Green function is homogeneous of degree -1,
G_cgf(r) = |r|^{-1} F(r_hat).  For a cubic crystal F is the circle integral
    G_K(x) = 1/(8 pi^2 |x|) * integral over unit n normal to x of Gamma(n)^{-1}
with the acoustic tensor Gamma_ik(n) = C_ijkl n_j n_l (the anisotropic Kelvin solution
of a unit point force).  A lattice point force is a unit force, and D(q) -> Omega Gamma(q)
at small q, so the lattice Green function approaches G_K itself far from the source.

Line-mode representation.  Appendix B's lattice function, transformed along the line
(period c = a/sqrt2, site (n0, n1, n2) at (n0 + n1/2) c along the line), has the far
field (Poisson summation over the layer index; aliases decay like exp(-2 pi rho/c)):
    G_cgf(m; dn1, dn2) = (1/c) exp(i pi theta0 dn1) G^_K(kappa, r_perp),
    theta0 = m/N_z in [0, 1/2],  kappa = 2 pi theta0 / c,
    G^_K(kappa, r_perp) = integral dz G_K(r_perp + z t) exp(-i kappa z).
Homogeneity gives G^_K(kappa, lambda r) = G^_K(lambda kappa, r).

The z integral is evaluated by subtracting the two leading terms of the large-|z|
expansion G_K(r + z t) = G0/|z| + g1 z/|z|^3 + O(|z|^-3), G0 = G_K(t), g1 = (r.grad)G_K(t),
in regularised forms.  By homogeneity the problem is solved at rho = 1 with s = kappa rho:
G0/sqrt(z^2 + 1) and g1 z/(z^2 + 1)^{3/2} transform to 2 G0 K0(s) and -2 i s g1 K0(s)
(modified Bessel K0), and the O(|z|^-3) remainder is integrated by the trapezoid rule on
[-Z, Z].  At kappa = 0 the
transform diverges logarithmically (the Green function of the infinite line); the m = 0
value is defined by dropping 2 G0 log(kappa) (a constant gauge, which the method removes:
Section 3.1 and Appendix B, constant C).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import k0, k1

from .lattice import elastic_constants_nn_fcc

C_LINE = 1.0 / math.sqrt(2.0)                       # period along [1-10], a = 1
T_HAT = np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)  # line direction
E1 = np.array([0.0, 0.0, 1.0])                       # in-plane axes: [001]
E2 = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)      # and [110]/sqrt2
EULER_GAMMA = 0.57721566490153286060651209008240243


def cubic_stiffness(c11: float, c12: float, c44: float) -> np.ndarray:
    """Full C_ijkl of a cubic crystal in its cube axes."""
    c = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    v = 0.0
                    if i == j and k == l:
                        v += c12
                    if (i == k and j == l) or (i == l and j == k):
                        v += c44
                    if i == j == k == l:
                        v = c11
                    c[i, j, k, l] = v
    return c


def kelvin_green(x: np.ndarray, cijkl: np.ndarray, n_psi: int = 64) -> np.ndarray:
    """G_K(x) for points x[..., 3] (x != 0): circle integral of Gamma(n)^{-1} over unit n
    normal to x (trapezoid rule, exponentially convergent for this periodic integrand)."""
    x = np.asarray(x, dtype=np.float64)
    r = np.linalg.norm(x, axis=-1)
    xh = x / r[..., None]
    # orthonormal pair normal to xh
    helper = np.where(np.abs(xh[..., 0:1]) < 0.9, np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]))
    u = np.cross(xh, helper)
    u /= np.linalg.norm(u, axis=-1, keepdims=True)
    v = np.cross(xh, u)
    psi = 2.0 * np.pi * np.arange(n_psi) / n_psi
    n = np.cos(psi)[:, None] * u[..., None, :] + np.sin(psi)[:, None] * v[..., None, :]   # [..., P, 3]
    gam = np.einsum("ijkl,...j,...l->...ik", cijkl, n, n)
    inv = np.linalg.inv(gam)
    integral = inv.mean(axis=-3) * 2.0 * np.pi
    return integral / (8.0 * np.pi ** 2 * r[..., None, None])


def kelvin_isotropic(x: np.ndarray, mu: float, nu: float) -> np.ndarray:
    """Closed-form Kelvin solution of an isotropic solid (for pinning kelvin_green)."""
    x = np.asarray(x, dtype=np.float64)
    r = np.linalg.norm(x, axis=-1)
    outer = np.einsum("...i,...j->...ij", x, x) / (r ** 2)[..., None, None]
    return ((3.0 - 4.0 * nu) * np.eye(3) + outer) / (16.0 * np.pi * mu * (1.0 - nu) * r[..., None, None])


def nn_fcc_stiffness(spring_k: float = 1.0) -> np.ndarray:
    return cubic_stiffness(*elastic_constants_nn_fcc(spring_k))


def in_plane_vector(dn1, dn2) -> np.ndarray:
    """Physical in-plane position r_perp of column offset (dn1, dn2) (a = 1)."""
    dn1 = np.asarray(dn1, dtype=np.float64)
    dn2 = np.asarray(dn2, dtype=np.float64)
    x = 0.5 * dn1
    y = (dn1 + 2.0 * dn2) / (2.0 * math.sqrt(2.0))
    return x[..., None] * E1 + y[..., None] * E2


def mixed_kelvin(kappa: float, r_perp: np.ndarray, cijkl: np.ndarray, z_max: float = 400.0,
                 dz: float = 1.0 / 64.0, n_psi: int = 48) -> np.ndarray:
    """G^_K(kappa, r_perp) = integral dz G_K(r_perp + z t) exp(-i kappa z), complex [3, 3];
    kappa = 0 returns the regularised value (2 G0 log kappa dropped)."""
    r_perp = np.asarray(r_perp, dtype=np.float64)
    rho = float(np.linalg.norm(r_perp))
    rh = r_perp / rho
    g0 = kelvin_green(T_HAT, cijkl, n_psi)
    h = 1e-4
    g1 = (kelvin_green(T_HAT + h * rh, cijkl, n_psi) - kelvin_green(T_HAT - h * rh, cijkl, n_psi)) / (2 * h)
    # unit-rho problem (homogeneity): G^_K(kappa, r) = G^_K(kappa rho, r_hat)
    s = kappa * rho
    z = np.arange(-z_max, z_max + 0.5 * dz, dz)
    pts = rh[None, :] + z[:, None] * T_HAT[None, :]
    g = kelvin_green(pts, cijkl, n_psi)
    d = np.sqrt(z * z + 1.0)
    rem = g - g0[None] / d[:, None, None] - g1[None] * (z / d ** 3)[:, None, None]
    w = np.full(z.size, dz)
    w[0] = w[-1] = 0.5 * dz
    ph = np.exp(-1j * s * z)
    integral = np.einsum("z,zij->ij", w * ph, rem)
    if s > 0.0:
        # transforms of G0/sqrt(z^2+1) and g1 z/(z^2+1)^{3/2}
        asym = 2.0 * g0 * k0(s) + g1 * (-2j * s * k0(s))
    else:
        # 2 G0 K0(kappa rho) with the divergent -2 G0 log(kappa) dropped
        asym = 2.0 * g0 * (math.log(2.0) - EULER_GAMMA - math.log(rho))
    return integral + asym


def line_mode_cgf(nz: int, m: int, dn1: int, dn2: int, cijkl: np.ndarray, **kw) -> np.ndarray:
    """Far-field line-mode block (1/c) exp(i pi theta0 dn1) G^_K(2 pi theta0 / c, r_perp)."""
    theta0 = m / nz
    if theta0 > 0.5:
        raise ValueError("line modes 0..N_z/2 only")
    kappa = 2.0 * math.pi * theta0 / C_LINE
    r = in_plane_vector(dn1, dn2)
    return np.exp(1j * math.pi * theta0 * dn1) * mixed_kelvin(kappa, r, cijkl, **kw) / C_LINE


# The transform of g1 z/(z^2+1)^{3/2} used above: integral z exp(-i s z)(z^2+1)^{-3/2} dz
# = -2 i s K0(s); exposed for the pin test.
def transform_odd_asymptote(s: float) -> complex:
    return -2j * s * k0(s)


def transform_even_asymptote(s: float) -> float:
    return 2.0 * k0(s)


__all__ = ["kelvin_green", "kelvin_isotropic", "cubic_stiffness", "nn_fcc_stiffness", "mixed_kelvin",
           "line_mode_cgf", "in_plane_vector", "transform_odd_asymptote", "transform_even_asymptote",
           "C_LINE", "T_HAT", "E1", "E2", "k1"]
