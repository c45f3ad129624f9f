"""Pins for the H-matrix oracle (Appendix C): the cross approximation against matrices of
known rank, the cluster trees and the block partition against their defining properties,
and the H-matrix product against the dense product of the Brillouin-zone blocks at the
paper's accuracy bound."""
import math

import numpy as np
import pytest

import fbc_workloads as W
from oracle import green, hmat


@pytest.mark.parametrize("rank", [1, 3, 7])
def test_aca_recovers_a_matrix_of_known_rank(rank):
    rng = np.random.default_rng(rank)
    u = rng.normal(size=(40, rank)) + 1j * rng.normal(size=(40, rank))
    v = rng.normal(size=(30, rank)) + 1j * rng.normal(size=(30, rank))
    a = u @ v.T
    f = hmat.aca(lambda i: a[i], lambda j: a[:, j], 40, 30, 1e-12, 64)
    assert f is not None and f[0].shape[1] <= rank + 2          # two terms at rounding level end it
    assert np.abs(f[0] @ f[1].T - a).max() < 1e-12 * np.abs(a).max()


def test_aca_cross_interpolates_pivot_rows_and_columns():
    # after k steps the approximation reproduces the chosen rows and columns exactly
    x = np.linspace(0.0, 1.0, 25)
    y = np.linspace(3.0, 4.0, 20)
    a = 1.0 / np.abs(x[:, None] - y[None, :]) + 0j          # smooth kernel, separated sets
    u, v = hmat.aca(lambda i: a[i], lambda j: a[:, j], 25, 20, 1e-10, 64)
    approx = u @ v.T
    assert np.linalg.norm(approx - a) < 1e-8 * np.linalg.norm(a)
    assert u.shape[1] < 12                                   # far fewer than min(25, 20)


def _cols():
    c = W.make_custom(16, 400, 800, 1, 256, seed=31).cells[0]
    return c


def test_cluster_tree_properties():
    c = _cols()
    root = hmat.cluster_tree(c.cols_b, 20)
    stack, leaves = [root], []
    while stack:
        t = stack.pop()
        if t.children:
            a, b = t.children
            assert sorted(np.concatenate([a.idx, b.idx]).tolist()) == sorted(t.idx.tolist())
            assert abs(len(a.idx) - len(b.idx)) <= 1
            stack += t.children
        else:
            assert len(t.idx) <= 20
            leaves.append(t)
    assert sorted(np.concatenate([l.idx for l in leaves]).tolist()) == list(range(len(c.cols_b)))


def test_partition_covers_every_entry_once():
    c = _cols()
    tb, ti = hmat.cluster_tree(c.cols_b, 20), hmat.cluster_tree(c.cols_i, 20)
    cover = np.zeros((len(c.cols_b), len(c.cols_i)), dtype=int)
    for kind, t, s in hmat.partition(tb, ti, 2):
        cover[np.ix_(t.idx, s.idx)] += 1
        if kind == "dense":
            assert not t.children and not s.children
        else:
            assert hmat.admissible(t, s, 2)
    assert (cover == 1).all()


def test_admissibility_matches_its_real_valued_statement():
    c = _cols()
    tb, ti = hmat.cluster_tree(c.cols_b, 20), hmat.cluster_tree(c.cols_i, 20)
    diam = lambda xy: float(np.hypot(*(xy.max(axis=0) - xy.min(axis=0))))
    checked = 0
    for t in (tb, tb.children[0], tb.children[0].children[1]):
        for s in (ti, ti.children[1], ti.children[1].children[0], ti.children[0].children[0]):
            xy_t, xy_s = hmat.column_xy(c.cols_b[t.idx]), hmat.column_xy(c.cols_i[s.idx])
            gap = np.maximum(0.0, np.maximum(xy_s.min(axis=0) - xy_t.max(axis=0), xy_t.min(axis=0) - xy_s.max(axis=0)))
            lhs, rhs = min(diam(xy_t), diam(xy_s)), 2.0 * float(np.hypot(*gap))
            if abs(lhs - rhs) > 1e-9 * max(lhs, rhs, 1.0):
                assert (lhs <= rhs) == hmat.admissible(t, s, 2)
                checked += 1
    assert checked >= 6


@pytest.mark.parametrize("m", [0, 1])
def test_hmatrix_product_within_the_accuracy_bound(m):
    c = _cols()
    a = green.green_modes_dense(16, 256, 256, c.cols_b, c.cols_i, modes=[m])[0]
    tb, ti = hmat.cluster_tree(c.cols_b, 20), hmat.cluster_tree(c.cols_i, 20)
    rng = np.random.default_rng(m)
    x = rng.normal(size=(a.shape[1], 3)) + 1j * rng.normal(size=(a.shape[1], 3))
    yd = a @ x
    errs = []
    for eps in (1e-3, 1e-5, 1e-8):
        h = hmat.HMatrix(a, tb, ti, 2, eps)
        errs.append(np.linalg.norm(h.matvec(x) - yd) / np.linalg.norm(yd))
        assert errs[-1] < 10 * eps, (eps, errs[-1])
        assert h.stored_entries() < 0.6 * a.size
    assert errs[0] > errs[1] > errs[2]
