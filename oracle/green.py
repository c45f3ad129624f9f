"""Line-mode lattice Green blocks by Brillouin-zone summation (FP64 oracle; test
infrastructure only).

Appendix B: G_inf = F^{-1}{ F{K_h}^{-1} } with the semi-discrete transform
F{f}(k) = sum_r f(r) e^{-i k.r}.  On the torus Z_Nz x Z_M1 x Z_M2 (periodic along
the line with l3 = Nz c, Section 2.1; in-plane torus M1 x M2 standing in for the
infinite plane) the inverse transform is a finite sum over the grid
theta = (m/Nz, m1/M1, m2/M2), and the term q = 0, where F{K_h} is singular, is
dropped (pseudo-inverse gauge; Section 3.1: the Green function is unique only up
to a constant).  Transforming the real-space Green function along the line,
    G^(m; dn1, dn2) = sum_dn0 G(dn0, dn1, dn2) e^{-2 pi i m dn0 / Nz}
                    = (1/(M1 M2)) sum_{m1,m2} D(theta)^{-1} e^{2 pi i (m1 dn1/M1 + m2 dn2/M2)},
which depends on the column offset (dn1, dn2) only (Section 3.2: entries depend on
r_ij only).  The block coupling pad column b to interface column i at mode m is
G^(m; n_b - n_i)  (target minus source).
"""
from __future__ import annotations

import numpy as np

from .lattice import dynamical_matrix


def dinv_grid(nz: int, m1: int, m2: int, m: int, spring_k: float = 1.0) -> np.ndarray:
    """D(theta)^{-1} on the in-plane grid for line mode m, [M1, M2, 3, 3]; zero at q = 0."""
    t1 = np.arange(m1) / m1
    t2 = np.arange(m2) / m2
    th = np.empty((m1, m2, 3))
    th[..., 0] = m / nz
    th[..., 1] = t1[:, None]
    th[..., 2] = t2[None, :]
    d = dynamical_matrix(th, spring_k)
    zero = (m % nz == 0)
    if zero:
        d[0, 0] = np.eye(3)          # placeholder, overwritten below
    dinv = np.linalg.inv(d)
    if zero:
        dinv[0, 0] = 0.0
    return dinv


def line_mode_green(nz: int, m1: int, m2: int, m: int, spring_k: float = 1.0) -> np.ndarray:
    """g_m(dn1, dn2) on the whole in-plane torus, complex [M1, M2, 3, 3]."""
    return np.fft.ifft2(dinv_grid(nz, m1, m2, m, spring_k), axes=(0, 1))


def gather_blocks(g: np.ndarray, cols_b: np.ndarray, cols_i: np.ndarray) -> np.ndarray:
    """Blocks G^_{bi} = g(n_b - n_i mod M), shape [n_b, n_i, 3, 3]."""
    m1, m2 = g.shape[0], g.shape[1]
    d1 = (cols_b[:, None, 0].astype(np.int64) - cols_i[None, :, 0]) % m1
    d2 = (cols_b[:, None, 1].astype(np.int64) - cols_i[None, :, 1]) % m2
    return g[d1, d2]


def dense_mode_matrix(blocks: np.ndarray) -> np.ndarray:
    """[n_b, n_i, 3, 3] blocks -> [3 n_b, 3 n_i] matrix (row 3b+c, column 3i+d)."""
    n_b, n_i = blocks.shape[:2]
    return blocks.transpose(0, 2, 1, 3).reshape(3 * n_b, 3 * n_i)


def green_modes_dense(nz: int, m1: int, m2: int, cols_b: np.ndarray, cols_i: np.ndarray,
                      modes=None, spring_k: float = 1.0) -> np.ndarray:
    """Dense per-mode matrices [n_modes, 3 n_b, 3 n_i] (modes default to 0..Nz/2)."""
    if modes is None:
        modes = range(nz // 2 + 1)
    out = []
    for m in modes:
        out.append(dense_mode_matrix(gather_blocks(line_mode_green(nz, m1, m2, m, spring_k), cols_b, cols_i)))
    return np.stack(out)


def green_real_space(nz: int, m1: int, m2: int, spring_k: float = 1.0) -> np.ndarray:
    """Real-space torus Green function G(n0, n1, n2), [Nz, M1, M2, 3, 3], from the 3-D
    inverse transform of D^{-1} (q = 0 dropped); used for the direct circulant check."""
    t0 = np.arange(nz) / nz
    t1 = np.arange(m1) / m1
    t2 = np.arange(m2) / m2
    th = np.stack(np.meshgrid(t0, t1, t2, indexing="ij"), axis=-1)
    d = dynamical_matrix(th, spring_k)
    d[0, 0, 0] = np.eye(3)
    dinv = np.linalg.inv(d)
    dinv[0, 0, 0] = 0.0
    g = np.fft.ifftn(dinv, axes=(0, 1, 2))
    return g.real.copy()
