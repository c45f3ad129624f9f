"""Pins for the oracle MLP (analytic gradient vs central differences) and for the
continuum Green function (isotropic closed form, Bessel transforms, far-field agreement
with the lattice Green function)."""
import math

import numpy as np
import pytest

from oracle import cgf, green, mlp


def test_mlp_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    sizes = (4, 7, 6, 5, 3)
    p = mlp.init_params(rng, sizes)
    x = rng.normal(size=(9, 4))
    t = rng.normal(size=(9, 3))
    w = rng.random(9) + 0.5
    _, g = mlp.loss_grad(p, x, t, w, sizes)
    h = 1e-6
    idx = rng.choice(p.size, size=40, replace=False)
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (mlp.loss(p + e, x, t, w, sizes) - mlp.loss(p - e, x, t, w, sizes)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd)), (k, fd, g[k])


def test_mlp_layout_and_size():
    assert mlp.n_params() == 8 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 12 + 12
    p = np.arange(mlp.n_params(), dtype=float)
    layers = mlp.unpack(p)
    assert layers[0][0].shape == (128, 8) and layers[0][0][0, 1] == 1.0 and layers[0][1][0] == 1024.0


def test_kelvin_matches_isotropic_closed_form():
    mu, nu = 1.3, 0.27
    lam = 2 * mu * nu / (1 - 2 * nu)
    c = cgf.cubic_stiffness(lam + 2 * mu, lam, mu)
    x = np.random.default_rng(1).normal(size=(30, 3))
    assert np.abs(cgf.kelvin_green(x, c) - cgf.kelvin_isotropic(x, mu, nu)).max() < 1e-14


def test_kelvin_is_homogeneous_and_symmetric():
    c = cgf.nn_fcc_stiffness()
    x = np.random.default_rng(2).normal(size=(10, 3))
    g1 = cgf.kelvin_green(x, c)
    assert np.allclose(cgf.kelvin_green(2.5 * x, c), g1 / 2.5, rtol=1e-13)
    assert np.allclose(cgf.kelvin_green(-x, c), g1, rtol=1e-13)
    assert np.allclose(g1, np.swapaxes(g1, -1, -2), atol=1e-15)


def test_odd_asymptote_transform():
    # integral z exp(-i s z) (z^2+1)^{-3/2} dz = -2 i s K0(s): absolutely convergent, check by quadrature
    for s in (0.3, 1.0, 4.0):
        z = np.linspace(-4000, 4000, 4_000_001)
        f = np.trapezoid(z * np.exp(-1j * s * z) / (z * z + 1) ** 1.5, z)
        assert abs(f - cgf.transform_odd_asymptote(s)) < 2e-6


@pytest.mark.slow
def test_cgf_is_the_far_field_of_the_lattice_green_function():
    # small line wavenumber: relative difference at the 1e-3 level, not growing with distance
    c = cgf.nn_fcc_stiffness()
    nz, m, big = 64, 1, 512
    g = green.line_mode_green(nz, big, big, m)
    rels = []
    for d in [(8, 4), (16, 8), (32, 16)]:
        gl = g[d[0] % big, d[1] % big]
        gc = cgf.line_mode_cgf(nz, m, d[0], d[1], c)
        rels.append(np.abs(gl - gc).max() / np.abs(gl).max())
    assert max(rels) < 1.5e-3
    # m = 0: lattice minus continuum is the same constant 3x3 (the gauge constant C) in
    # every direction and distance, up to lattice corrections and the finite torus; a wrong
    # coefficient of the logarithm would change it by O(1) between these points
    g0 = green.line_mode_green(nz, big, big, 0)
    diffs = []
    for d in [(20, 10), (20, -17), (40, -34), (-30, 2)]:
        diffs.append(g0[d[0] % big, d[1] % big] - cgf.line_mode_cgf(nz, 0, d[0], d[1], c).real)
    diffs = np.array(diffs)
    spread = np.abs(diffs - diffs.mean(axis=0)).max()
    assert spread < 5e-3 * np.abs(diffs).max()
