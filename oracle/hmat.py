"""H-matrix form of the per-mode Green blocks (FP64 oracle; test infrastructure only).

Appendix C builds the hierarchical matrix in three steps:
* Step 1, cluster trees of the pad and interface index sets by geometric clustering
  (binary space partitioning) down to a minimal block size b_min;
* Step 2, the block partition: starting from the roots, a block t x s is kept as a
  low-rank leaf when min(diam t, diam s) <= gamma dist(t, s) (eq. geom_adm), a dense leaf
  when both clusters are leaves, and is subdivided otherwise;
* Step 3, the low-rank factors of every admissible block by adaptive cross approximation
  (eq. aca): R^k = R^{k-1} - R^{k-1}_{:, j_k} R^{k-1}_{i_k, :} / R^{k-1}_{i_k, j_k}, with
  i_k chosen heuristically and j_k the largest entry of the residual row (partial
  pivoting), stopped when the rank-1 update is below eps times the approximation.
Parameters of the paper: b_min = 20, gamma = 2, eps = 1e-5.

Readings (each also listed in the design notes):
* the line direction is diagonalised by the line transform, so the H-matrix is built for
  each line mode m of the complex matrix G^(m) (3 n_b x 3 n_i, 3 x 3 blocks); the
  periodic images s+ and s- of eq. geom_adm lie on the same in-plane position as s, so the
  criterion is evaluated in the plane;
* clusters hold atom columns (3 matrix rows or columns each); positions are the in-plane
  column positions, compared through the integers X = n1 (= 2x) and Y = n1 + 2 n2
  (= 2 sqrt2 y);
* a cluster is split along the longer side of its bounding box at the median (ties by
  column index), the first half taking floor(size / 2) columns;
* diam and dist are taken on the bounding boxes of the clusters (the supersets the
  appendix names for practical use): diam the box diagonal, dist the distance between the
  two boxes.  The text's centroid distance would admit, on ring geometries, blocks of two
  half rings whose ends touch, whose near pairs are not of low rank (measured: 8 % error
  at line mode 7 of the medium cell).  gamma is an integer (the paper's value is 2) and
  the criterion is decided exactly: 8 diam^2 = 2 dX^2 + dY^2, 8 dist^2 = 2 gX^2 + gY^2
  with gX, gY the gaps between the boxes in X and Y;
* rows and columns of a block follow the tree order (a cluster lists its first child's
  columns, then its second's);
* ACA: i_1 is the first row of the block, i_{k+1} the unused row of largest |u_k|;
  stop when |u_k| |v_k| <= eps ||S_k||_F (S_k the current approximation, norm updated
  incrementally) holds for two consecutive terms (one small term can come from a row
  that misses the block's large entries); a block whose rank would exceed max_rank is
  stored dense.
"""
from __future__ import annotations

import math

import numpy as np


def column_xy(cols: np.ndarray) -> np.ndarray:
    """In-plane coordinates (x, y) of columns (n1, n2), a = 1."""
    c = np.asarray(cols, dtype=np.float64)
    return np.stack([0.5 * c[:, 0], (c[:, 0] + 2.0 * c[:, 1]) / (2.0 * math.sqrt(2.0))], axis=1)


class Cluster:
    def __init__(self, idx: np.ndarray, cols: np.ndarray):
        self.idx = idx                                   # column indices (into cols)
        X = cols[idx, 0].astype(np.int64)
        Y = cols[idx, 0].astype(np.int64) + 2 * cols[idx, 1].astype(np.int64)
        self.xlo, self.xhi, self.ylo, self.yhi = int(X.min()), int(X.max()), int(Y.min()), int(Y.max())
        self.n = len(idx)
        self.sx, self.sy = int(X.sum()), int(Y.sum())
        self.diam8 = 2 * (self.xhi - self.xlo) ** 2 + (self.yhi - self.ylo) ** 2      # 8 diam^2
        self.children: list[Cluster] = []


def cluster_tree(cols: np.ndarray, b_min: int, idx: np.ndarray | None = None) -> Cluster:
    """Step 1: binary space partitioning until a cluster holds at most b_min columns."""
    cols = np.asarray(cols)
    if idx is None:
        idx = np.arange(len(cols))
    node = Cluster(idx, cols)
    if len(idx) > b_min:
        dx, dy = node.xhi - node.xlo, node.yhi - node.ylo
        # extent_x = dx / 2 >= extent_y = dy / (2 sqrt 2)  <=>  2 dx^2 >= dy^2
        if 2 * dx * dx >= dy * dy:
            key = cols[idx, 0].astype(np.int64)
        else:
            key = cols[idx, 0].astype(np.int64) + 2 * cols[idx, 1].astype(np.int64)
        order = np.lexsort((idx, key))
        srt = idx[order]
        h = len(idx) // 2
        node.children = [cluster_tree(cols, b_min, srt[:h]), cluster_tree(cols, b_min, srt[h:])]
        node.idx = np.concatenate([node.children[0].idx, node.children[1].idx])   # tree order
    return node


def admissible(t: Cluster, s: Cluster, gamma: int) -> bool:
    """eq. geom_adm in the plane on bounding boxes: min(diam t, diam s) <= gamma dist(t, s),
    squared and scaled to integers (exact)."""
    gx = max(0, s.xlo - t.xhi, t.xlo - s.xhi)
    gy = max(0, s.ylo - t.yhi, t.ylo - s.yhi)
    return min(t.diam8, s.diam8) <= gamma * gamma * (2 * gx * gx + gy * gy)


def partition(t: Cluster, s: Cluster, gamma: int, out=None) -> list:
    """Step 2: leaves (kind, t, s) with kind 'lr' (admissible) or 'dense'."""
    if out is None:
        out = []
    if admissible(t, s, gamma):
        out.append(("lr", t, s))
    elif not t.children and not s.children:
        out.append(("dense", t, s))
    else:
        tc = t.children or [t]
        sc = s.children or [s]
        for a in tc:
            for b in sc:
                partition(a, b, gamma, out)
    return out


def expand(idx: np.ndarray) -> np.ndarray:
    """Matrix rows/columns of a set of atom columns (3 components each)."""
    return (3 * np.asarray(idx)[:, None] + np.arange(3)[None, :]).reshape(-1)


def aca(get_row, get_col, n_rows: int, n_cols: int, eps: float, max_rank: int):
    """Step 3, eq. aca with partial pivoting.  get_row(i) / get_col(j) return a row / column
    of the block.  Returns (U [n_rows, k], V [n_cols, k]) with block ~ U V^T, or None when
    the rank would exceed max_rank."""
    us, vs = [], []
    used = np.zeros(n_rows, dtype=bool)
    i = 0
    norm2 = 0.0
    small = 0
    while True:
        row = get_row(i).astype(np.complex128)
        for u, v in zip(us, vs):
            row = row - u[i] * v
        used[i] = True
        j = int(np.argmax(np.abs(row)))
        piv = row[j]
        if piv == 0:
            # the residual row vanishes: try the next unused row, stop when none is left
            free = np.flatnonzero(~used)
            if free.size == 0:
                break
            i = int(free[0])
            continue
        v = row / piv
        col = get_col(j).astype(np.complex128)
        for uu, vv in zip(us, vs):
            col = col - vv[j] * uu
        u = col
        # ||S_k||_F^2 = ||S_{k-1}||_F^2 + 2 Re sum_l (u_l^H u)(v_l^H v) + |u|^2 |v|^2
        cross = 0.0
        for uu, vv in zip(us, vs):
            cross += 2.0 * float(np.real(np.vdot(uu, u) * np.vdot(vv, v)))
        nu, nv = float(np.linalg.norm(u)), float(np.linalg.norm(v))
        norm2 = norm2 + cross + (nu * nv) ** 2
        us.append(u)
        vs.append(v)
        if len(us) > max_rank:
            return None
        small = small + 1 if nu * nv <= eps * math.sqrt(max(norm2, 0.0)) else 0
        if small == 2:
            break
        mag = np.abs(u)
        mag[used] = -1.0
        if mag.max() < 0:
            break
        i = int(np.argmax(mag))
    if not us:
        return np.zeros((n_rows, 0), complex), np.zeros((n_cols, 0), complex)
    return np.stack(us, axis=1), np.stack(vs, axis=1)


class HMatrix:
    """H-matrix of one dense complex matrix A (3 n_b x 3 n_i) on the given trees."""

    def __init__(self, a: np.ndarray, tree_b: Cluster, tree_i: Cluster, gamma: int, eps: float,
                 max_rank: int = 64):
        self.shape = a.shape
        self.blocks = []
        for kind, t, s in partition(tree_b, tree_i, gamma):
            rows, cols = expand(t.idx), expand(s.idx)
            if kind == "lr":
                f = aca(lambda i: a[rows[i], cols], lambda j: a[rows, cols[j]], len(rows), len(cols), eps,
                        max_rank)
                if f is not None:
                    self.blocks.append(("lr", rows, cols, f))
                    continue
            self.blocks.append(("dense", rows, cols, a[np.ix_(rows, cols)]))

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = H x for x [3 n_i, R] (complex)."""
        y = np.zeros((self.shape[0],) + x.shape[1:], dtype=np.complex128)
        for kind, rows, cols, f in self.blocks:
            if kind == "lr":
                u, v = f
                y[rows] += u @ (v.T @ x[cols])
            else:
                y[rows] += f @ x[cols]
        return y

    def stored_entries(self) -> int:
        n = 0
        for kind, rows, cols, f in self.blocks:
            n += (f[0].size + f[1].size) if kind == "lr" else f.size
        return n
