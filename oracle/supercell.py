"""Brute-force periodic supercell (FP64 oracle; test infrastructure only).

Section 2.3.2 defines the Green operator of the periodic harmonic problem by
G L_h = I.  On a finite torus Z_Nz x Z_M1 x Z_M2 of primitive cells, L_h is the
stiffness matrix K of the nearest-neighbour central springs (Section 2.2.1),
assembled bond by bond from the spring energy (k/2) sum_bonds (Rhat.(u_j-u_i))^2,
with no reference to the Fourier symbol.  K is singular (uniform translations),
so the Green operator of the torus is the Moore-Penrose pseudo-inverse K^+,
i.e. the gauge in which the Green function is defined up to the constant the
paper says it is unique up to (Section 3.1).  Site index s = (n0*M1 + n1)*M2 + n2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .lattice import bond_projectors, nn_index_offsets


def torus_stiffness(nz: int, m1: int, m2: int, spring_k: float = 1.0) -> sp.csr_matrix:
    """Sparse 3N x 3N stiffness of the torus supercell, assembled from bonds (+= so that
    bonds that wrap onto the same pair of sites on a small torus add up)."""
    dims = np.array([nz, m1, m2])
    n_sites = int(dims.prod())
    idx = np.arange(n_sites)
    n0, rem = np.divmod(idx, m1 * m2)
    n1, n2 = np.divmod(rem, m2)
    offs = nn_index_offsets()
    proj = bond_projectors()
    rows, cols, vals = [], [], []
    # each bond once: keep one of every +/-R pair
    for b in range(offs.shape[0]):
        o = offs[b]
        if tuple(o) < tuple(-o):
            continue
        t0 = (n0 + o[0]) % nz
        t1 = (n1 + o[1]) % m1
        t2 = (n2 + o[2]) % m2
        tgt = (t0 * m1 + t1) * m2 + t2
        kp = spring_k * proj[b]
        for (a_s, b_s, sign) in ((idx, idx, 1.0), (tgt, tgt, 1.0), (idx, tgt, -1.0), (tgt, idx, -1.0)):
            for i in range(3):
                for j in range(3):
                    rows.append(3 * a_s + i)
                    cols.append(3 * b_s + j)
                    vals.append(np.full(n_sites, sign * kp[i, j]))
    k = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(3 * n_sites, 3 * n_sites))
    return k.tocsr()


def torus_pinv_dense(nz: int, m1: int, m2: int, spring_k: float = 1.0) -> np.ndarray:
    """Dense pseudo-inverse K^+ (micro tori only)."""
    k = torus_stiffness(nz, m1, m2, spring_k).toarray()
    return np.linalg.pinv(k, rcond=1e-12, hermitian=True)


def site_index(n0, n1, n2, nz, m1, m2):
    return ((np.asarray(n0) % nz) * m1 + (np.asarray(n1) % m1)) * m2 + (np.asarray(n2) % m2)


def torus_response(nz: int, m1: int, m2: int, cols_i: np.ndarray, cols_b: np.ndarray,
                   f: np.ndarray, spring_k: float = 1.0, pinv: np.ndarray | None = None,
                   rtol: float = 1e-14) -> np.ndarray:
    """w = K^+ F read at the pad sites, for interface forces f[R][nz][n_i][3].

    F places f on the interface sites of the torus.  With a dense K^+ the product is
    taken directly; otherwise K w = F is solved by conjugate gradients from zero (the
    iterates stay in range(K) when sum F = 0) and the uniform part is projected out,
    which gives the minimum-norm (pseudo-inverse) solution.  Returns w[R][nz][n_b][3].
    """
    f = np.asarray(f, dtype=np.float64)
    n_rhs, _, n_i, _ = f.shape
    n_b = cols_b.shape[0]
    n_sites = nz * m1 * m2
    layers = np.arange(nz)
    s_i = site_index(layers[:, None], cols_i[None, :, 0], cols_i[None, :, 1], nz, m1, m2)  # [nz, n_i]
    s_b = site_index(layers[:, None], cols_b[None, :, 0], cols_b[None, :, 1], nz, m1, m2)  # [nz, n_b]
    out = np.empty((n_rhs, nz, n_b, 3))
    kmat = None if pinv is not None else torus_stiffness(nz, m1, m2, spring_k)
    for r in range(n_rhs):
        big = np.zeros((n_sites, 3))
        np.add.at(big, s_i.ravel(), f[r].reshape(-1, 3))
        rhs = big.ravel()
        if pinv is not None:
            u = pinv @ rhs
        else:
            u, info = spla.cg(kmat, rhs, rtol=rtol, atol=0.0, maxiter=20000)
            if info != 0:
                raise RuntimeError(f"CG did not converge (info={info})")
            u = u.reshape(n_sites, 3)
            u -= u.mean(axis=0, keepdims=True)
            u = u.ravel()
        out[r] = u.reshape(n_sites, 3)[s_b.ravel()].reshape(nz, n_b, 3)
    return out
