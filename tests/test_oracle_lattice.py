"""Pins for the lattice and force-constant model of the oracle (not GPU)."""
import numpy as np
import pytest

from oracle import lattice, supercell
import fbc_workloads as W


def test_basis_generates_fcc_shells():
    # coordination shells of fcc (a = 1): 12 at 1/sqrt2, 6 at 1, 24 at sqrt(3/2), 12 at sqrt2
    rng = np.arange(-4, 5)
    n = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3)
    x = n @ lattice.BASIS.T
    d = np.linalg.norm(x, axis=1)
    d = d[d > 1e-12]
    for r, cnt in ((1 / np.sqrt(2), 12), (1.0, 6), (np.sqrt(1.5), 24), (np.sqrt(2.0), 12)):
        assert np.sum(np.abs(d - r) < 1e-9) == cnt
    # every lattice point has cubic coordinates that are multiples of 1/2 with even sum*2
    assert np.allclose(2 * x, np.rint(2 * x))
    assert np.all(np.rint(2 * x).sum(axis=1) % 2 == 0)


def test_nn_offsets_are_bonds():
    offs = lattice.nn_index_offsets()
    x = offs @ lattice.BASIS.T
    assert np.allclose(np.linalg.norm(x, axis=1), 1 / np.sqrt(2))
    s = {tuple(o) for o in offs}
    assert len(s) == 12 and all(tuple(-o) in s for o in offs)


def test_sum_rule_and_symbol_basics():
    p = lattice.bond_projectors()
    assert np.allclose(p.sum(axis=0), 4 * np.eye(3))
    assert np.allclose(lattice.dynamical_matrix(np.zeros(3)), 0.0)
    rng = np.random.default_rng(0)
    th = rng.random((50, 3))
    d = lattice.dynamical_matrix(th)
    assert np.allclose(d, np.swapaxes(d, -1, -2))
    for shift in np.eye(3, dtype=int):
        assert np.allclose(lattice.dynamical_matrix(th + shift), d, atol=1e-13)
    assert np.min(np.linalg.eigvalsh(d)) > 0.0
    # D(q) = K_h(0) + sum_R K_h(R) e^{-i q.R} with K_h(R) = -k Rhat Rhat^T, K_h(0) = 4k I
    offs = lattice.nn_index_offsets()
    ph = np.exp(-2j * np.pi * th @ offs.T)
    d2 = 4 * np.eye(3) - np.einsum("nb,bij->nij", ph, p)
    assert np.allclose(d2.imag, 0, atol=1e-14) and np.allclose(d2.real, d, atol=1e-13)


def test_long_wave_limit_matches_textbook_elastic_constants():
    # D(q) -> Omega * C_ijkl q_j q_l with C11 = 2k/a, C12 = C44 = k/a for NN central springs
    c11, c12, c44 = lattice.elastic_constants_nn_fcc()
    rng = np.random.default_rng(1)
    g = lattice.reciprocal_basis()
    for _ in range(5):
        th = rng.normal(size=3)
        eps = 1e-4
        q = 2 * np.pi * (eps * th) @ g         # cartesian wavevector
        d = lattice.dynamical_matrix(eps * th)
        ref = lattice.ATOMIC_VOLUME * lattice.acoustic_tensor(q, c11, c12, c44)
        assert np.allclose(d, ref, rtol=1e-6, atol=1e-14 * np.abs(ref).max())


def test_torus_stiffness_structure():
    k = supercell.torus_stiffness(4, 4, 6).toarray()
    assert np.allclose(k, k.T)
    ones = np.tile(np.eye(3), (k.shape[0] // 3, 1))
    assert np.allclose(k @ ones, 0.0)
    ev = np.linalg.eigvalsh(k)
    assert ev[0] > -1e-12 and np.sum(np.abs(ev) < 1e-10) == 3


def test_column_positions_match_basis_projection():
    cols = np.array([[0, 0], [1, 0], [0, 1], [3, -2], [-5, 7]])
    xy = W.column_xy(cols)
    ex = np.array([0.0, 0.0, 1.0])
    ey = np.array([1.0, 1.0, 0.0]) / np.sqrt(2)
    x = cols[:, 0:1] * lattice.BASIS[:, 1] + cols[:, 1:2] * lattice.BASIS[:, 2]
    assert np.allclose(xy[:, 0], x @ ex) and np.allclose(xy[:, 1], x @ ey)
    # the line direction b0 projects to the origin
    assert np.allclose([lattice.BASIS[:, 0] @ ex, lattice.BASIS[:, 0] @ ey], 0)


@pytest.mark.parametrize("n_i,n_b,lo_i,hi_i,lo_b,hi_b", [
    (96, 192, 3.46, 4.64, 4.69, 6.59),
    (1024, 2048, 42.018, 43.340, 43.363, 45.929),
])
def test_ring_rule(n_i, n_b, lo_i, hi_i, lo_b, hi_b):
    ci, cb = W.ring_columns(n_i, n_b)
    assert ci.shape == (n_i, 2) and cb.shape == (n_b, 2)
    ri = np.hypot(*W.column_xy(ci).T)
    rb = np.hypot(*W.column_xy(cb).T)
    assert abs(ri.min() - lo_i) < 0.01 and abs(ri.max() - hi_i) < 0.01
    assert abs(rb.min() - lo_b) < 0.01 and abs(rb.max() - hi_b) < 0.01
    assert rb.min() > ri.max()
    assert len({tuple(c) for c in np.concatenate([ci, cb])}) == n_i + n_b
    # R_i = n_i / (2 pi rho w) lies inside the interface band
    r0 = n_i / (2 * np.pi * W.RHO * W.RING_WIDTH)
    assert ri.min() <= r0 <= ri.max()


def test_forces_zero_net_and_seeded():
    a = W.make_single("tiny").cells[0].forces
    b = W.make_single("tiny").cells[0].forces
    assert np.array_equal(a, b)
    assert np.abs(a.sum(axis=2)).max() < 1e-14
    assert 0.08 < a.std() < 0.12
