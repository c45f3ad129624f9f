"""Pins for the oracle's line-mode Green blocks and the apply chain (not GPU).

Each check ties the oracle to something other than itself: the brute-force
pseudo-inverse of the bond-assembled torus stiffness, a CG solve on the C1 torus,
the direct real-space circulant sum, and structural identities of a Green
operator of a symmetric positive semi-definite lattice operator."""
import numpy as np
import pytest

from oracle import green, supercell, apply as ap
import fbc_workloads as W


@pytest.mark.parametrize("nz,m1,m2", [(4, 4, 5), (8, 4, 6), (2, 6, 4)])
def test_ghat_equals_supercell_pinv(nz, m1, m2):
    kp = supercell.torus_pinv_dense(nz, m1, m2)
    err = 0.0
    for m in range(nz):
        g = green.line_mode_green(nz, m1, m2, m)
        for d1 in range(m1):
            for d2 in range(m2):
                s = np.zeros((3, 3), complex)
                for d0 in range(nz):
                    si = supercell.site_index(d0, d1, d2, nz, m1, m2)
                    s += kp[3 * si:3 * si + 3, 0:3] * np.exp(-2j * np.pi * m * d0 / nz)
                err = max(err, np.abs(s - g[d1, d2]).max())
    assert err < 1e-13


def test_tiny_config_apply_equals_bruteforce_cg():
    wl = W.make_single("tiny")
    c = wl.cells[0]
    g = green.green_modes_dense(c.nz, wl.bz, wl.bz, c.cols_b, c.cols_i)
    w = ap.apply_green(g, c.forces)
    wb = supercell.torus_response(c.nz, wl.bz, wl.bz, c.cols_i, c.cols_b, c.forces, rtol=1e-13)
    assert np.linalg.norm(w - wb) / np.linalg.norm(wb) < 1e-11


def test_micro_apply_equals_dense_pinv_product():
    wl = W.make_single("micro")
    c = wl.cells[0]
    kp = supercell.torus_pinv_dense(c.nz, wl.bz, wl.bz)
    wb = supercell.torus_response(c.nz, wl.bz, wl.bz, c.cols_i, c.cols_b, c.forces, pinv=kp)
    g = green.green_modes_dense(c.nz, wl.bz, wl.bz, c.cols_b, c.cols_i)
    w = ap.apply_green(g, c.forces)
    assert np.abs(w - wb).max() < 1e-13 * np.abs(wb).max() * 10


def _column_set():
    ci, cb = W.ring_columns(12, 20)
    return np.concatenate([ci, cb])


def test_hermitian_psd_reciprocity_and_block_symmetry():
    nz, m1 = 8, 32
    s = _column_set()
    for m in range(nz):
        g = green.line_mode_green(nz, m1, m1, m)
        blocks = green.gather_blocks(g, s, s)
        mat = green.dense_mode_matrix(blocks)
        assert np.abs(mat - mat.conj().T).max() < 1e-13 * np.abs(mat).max()
        ev = np.linalg.eigvalsh(mat)
        assert ev.min() > -1e-12 * ev.max()
        # reciprocity: G_ib = G_bi^H, i.e. g(-d) = g(d)^H
        gi = green.gather_blocks(g, s[:5], s[5:])
        gb = green.gather_blocks(g, s[5:], s[:5])
        assert np.allclose(gi, np.conj(np.swapaxes(np.swapaxes(gb, 0, 1), -1, -2)), atol=1e-14)
        # each 3x3 block is complex symmetric (centrosymmetric lattice)
        assert np.abs(blocks - np.swapaxes(blocks, -1, -2)).max() < 1e-14
        if m in (0, nz // 2):
            assert np.abs(blocks.imag).max() < 1e-14
        gc = green.line_mode_green(nz, m1, m1, (nz - m) % nz)
        assert np.allclose(gc, np.conj(g), atol=1e-14)


def test_fft_form_equals_direct_circulant_sum():
    wl = W.make_custom(nz=6, n_i=14, n_b=22, n_rhs=2, bz=16, seed=3)
    c = wl.cells[0]
    gr = green.green_real_space(c.nz, wl.bz, wl.bz)
    wd = ap.apply_direct(gr, c.cols_b, c.cols_i, c.forces)
    g = green.green_modes_dense(c.nz, wl.bz, wl.bz, c.cols_b, c.cols_i)
    w = ap.apply_green(g, c.forces)
    assert np.abs(w - wd).max() < 1e-13 * np.abs(wd).max() * 10


def test_linearity_and_gauge_invariance():
    wl = W.make_single("parity")
    c = wl.cells[0]
    g = green.green_modes_dense(c.nz, wl.bz, wl.bz, c.cols_b, c.cols_i)
    f = c.forces
    w1 = ap.apply_green(g, f[:1])
    w2 = ap.apply_green(g, f[1:2])
    w12 = ap.apply_green(g, f[:1] + 2.5 * f[1:2])
    assert np.allclose(w12, w1 + 2.5 * w2, atol=1e-14)
    # a constant 3x3 added to every m=0 block cancels for zero-net-force f
    gg = g.copy()
    const = np.random.default_rng(4).normal(size=(3, 3))
    const = const + const.T
    gg[0] += np.kron(np.ones((c.n_b, c.n_i)), const)
    assert np.abs(ap.apply_green(gg, f) - ap.apply_green(g, f)).max() < 1e-12
    # per-row gauge: subtracting any i-independent block per (b, m) also cancels
    gr = g.copy().reshape(g.shape[0], c.n_b, 3, c.n_i, 3)
    gr -= gr.mean(axis=3, keepdims=True)
    assert np.abs(ap.apply_green(gr.reshape(g.shape), f) - ap.apply_green(g, f)).max() < 1e-12


def test_pad_update_removes_mean():
    rng = np.random.default_rng(5)
    u = rng.normal(size=(3, 8, 20, 3)) + np.array([1.0, -2.0, 0.5])
    w = rng.normal(size=u.shape)
    un, mean = ap.pad_update(u, w, np.array([1.0, 0.3, -2.0]))
    assert np.abs(un.mean(axis=(1, 2))).max() < 1e-14
    assert np.allclose(un + mean[:, None, None, :], u - np.array([1.0, 0.3, -2.0])[:, None, None, None] * w)


def test_net_force_is_column_sum():
    f = W.make_single("micro").cells[0].forces
    assert np.abs(ap.net_force(f)).max() < 1e-15
