"""Pins for the real-space periodic lattice Green function oracle (Section 3.1, eqs.
G~inf, plgf_conv, plgf_poly, plgf_rich; Appendix B): Richardson extrapolation against
its defining expansion and a series with a known sum, the torus Green function against
the lattice equation, the exact membership of the near-field table, the matching
constant against the continuum, and the assembled periodic function against its own
symmetries, the line-periodic lattice equation and the independently computed line-mode
blocks of the Brillouin-zone assembly."""
import math

import numpy as np
import pytest

from oracle import cgf, green, lattice, plgf


@pytest.mark.parametrize("n,order", [(1, 5), (2, 3), (3, 4)])
def test_richardson_is_exact_for_its_expansion(n, order):
    rng = np.random.default_rng(n * 10 + order)
    q = rng.normal(size=(order + 1, 3, 3))
    k = np.arange(1, n + order + 1, dtype=float)
    seq = sum(q[j] * k[:, None, None] ** (-j) for j in range(order + 1))
    assert np.abs(plgf.richardson(seq, n, order) - q[0]).max() < 1e-10 * np.abs(q).max()


def test_richardson_accelerates_a_known_series():
    # sum_{i<=k} 1/i^2 = pi^2/6 - 1/k + 1/(2k^2) - ...: six terms, N = 5
    s = np.cumsum(1.0 / np.arange(1, 12) ** 2)
    direct = abs(s[5] - math.pi ** 2 / 6)
    rich = abs(plgf.richardson(s, 1, 5) - math.pi ** 2 / 6)
    assert rich < 1e-4 and rich < 1e-3 * direct
    assert abs(plgf.richardson(s, 5, 5) - math.pi ** 2 / 6) < 1e-6


def test_near_field_table_membership_is_exact():
    # independent enumeration in cube axes: fcc points (i, j, k)/2 with i + j + k even
    r = np.arange(-12, 13)
    x2 = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    x2 = x2[(x2.sum(axis=1) % 2 == 0) & ((x2 * x2).sum(axis=1) <= 100)]
    got = plgf.lattice_vectors(100)
    gx2 = np.rint(2.0 * got @ lattice.BASIS.T).astype(int)
    assert sorted(map(tuple, gx2)) == sorted(map(tuple, x2))
    assert (np.diff(plgf.four_r2(got)) >= 0).all()


def test_torus_green_solves_the_lattice_equation():
    L = 16
    gt = plgf.torus_green(L)
    nr = lattice.nn_index_offsets()
    p = lattice.bond_projectors()
    for n in ([0, 0, 0], [1, 0, 0], [2, -1, 3], [5, 7, -4]):
        n = np.array(n)
        lh = p.sum(axis=0) @ plgf.torus_at(gt, n)
        for b in range(12):
            lh -= p[b] @ plgf.torus_at(gt, n - nr[b])
        want = (np.eye(3) if not n.any() else 0.0) - np.eye(3) / L ** 3
        assert np.abs(lh - want).max() < 1e-12


def test_matching_constant_joins_the_continuum():
    # the torus background grows like (|r| / (L c))^3: L = 64 keeps it below 1 % at 7 a
    gi = plgf.InfiniteLatticeGreen(64, 100, 144)
    gt = plgf.torus_green(64)
    for lo, hi in ((64, 100), (144, 196), (196, 256)):      # inside r_cut, and 6-7 a, 7-8 a
        outer = plgf.lattice_vectors(hi, lo)
        x = outer.astype(float) @ lattice.BASIS.T
        gc = cgf.kelvin_green(x, cgf.nn_fcc_stiffness())
        joined = np.abs(plgf.torus_at(gt, outer) - gi.c - gc).max() / np.abs(gc).max()
        raw = np.abs(plgf.torus_at(gt, outer) - gc).max() / np.abs(gc).max()
        assert joined < 1e-2 and joined < 0.05 * raw, (lo, hi, joined, raw)


@pytest.fixture(scope="module")
def ginf32():
    return plgf.InfiniteLatticeGreen(32, 100, 144)


def test_periodic_green_symmetries(ginf32):
    nz = 16
    for n in ([3, 2, -1], [0, 4, -2], [11, -3, 5]):
        n = np.array(n)
        g = plgf.periodic_green(ginf32, n, nz)
        assert np.abs(g - plgf.periodic_green(ginf32, -n, nz)).max() < 1e-13 * np.abs(g).max()
        assert np.abs(g - g.T).max() < 1e-14 * np.abs(g).max()
        shifted = plgf.periodic_green(ginf32, n + np.array([nz, 0, 0]), nz)
        assert np.abs(g - shifted).max() < 3e-5 * np.abs(g).max()


def test_periodic_green_solves_the_line_lattice_equation(ginf32):
    # L_h G~ = delta (periodic along the line) - I / L^3 (the torus background of the
    # near-field table), up to the continuum images' lattice residual
    nz = 16
    nr = lattice.nn_index_offsets()
    p = lattice.bond_projectors()
    for n in ([0, 0, 0], [1, 0, 0], [0, 1, -1], [3, -2, 1]):
        n = np.array(n)
        lh = p.sum(axis=0) @ plgf.periodic_green(ginf32, n, nz)
        for b in range(12):
            lh -= p[b] @ plgf.periodic_green(ginf32, n - nr[b], nz)
        want = (np.eye(3) if not n.any() else 0.0) - np.eye(3) / 32 ** 3
        assert np.abs(lh - want).max() < 2e-6, (n, np.abs(lh - want).max())


def test_line_modes_agree_with_brillouin_zone_blocks():
    # independent method: line-mode blocks of the in-plane torus sum (m >= 1 carries no
    # gauge constant); the real-space construction differs by its continuum far field
    nz, m_torus = 8, 128
    gi = plgf.InfiniteLatticeGreen(64, 100, 144)
    ref = [green.line_mode_green(nz, m_torus, m_torus, m) for m in range(nz // 2 + 1)]
    for d1, d2 in ((0, 0), (1, 0), (2, -1), (3, 2)):
        f2 = plgf.periodic_line_modes(gi, d1, d2, nz)
        a2 = np.array([ref[m][d1 % m_torus, d2 % m_torus] for m in range(nz // 2 + 1)])
        scale = np.abs(a2[1:]).max()
        err = np.abs(f2[1:] - a2[1:]).max() / scale
        assert err < 1e-2, ((d1, d2), err)
