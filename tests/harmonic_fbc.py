"""Algorithm 1 with L = L_h on a line-periodic cell: the caller's side of the FBC loop
(test infrastructure, not part of the library).

The atomistic model is the harmonic nearest-neighbour spring model itself, so the
atomistic problem (AH) is a sparse linear solve and the coupled problem's solution is
the global harmonic solution u* = G f_ext (Section 2.3.1; Remark 1: the method then
converges in two steps).  Sets, in atom columns (every layer):

* A    -- atomistic domain: columns with in-plane radius <= r_a;
* i+   -- continuum columns bonded to A (the pad that A's atoms see, and the interface
          where the incompatibility force lives, eq. flexbc.finc);
* i++  -- i+ plus the continuum columns bonded to i+: where the displacement must be
          known to evaluate the incompatibility force (Section 2.3.2).

The pad update u^{i++} <- u^{i++} - alpha G^{i++|i+} f_in plus mean removal is the
library's fbc_relax_step (or, on the CPU, the oracle); everything else here is the
caller: the (AH) solve and the incompatibility force
f_in = L_h^{i+|A}[u_{k+1}] + L_h^{i+|i++}[u_k].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import fbc_workloads as W
from oracle import lattice


class HarmonicDisc:
    def __init__(self, nz: int, r_a: float, spring_k: float = 1.0):
        self.nz = nz
        self.k = spring_k
        bonds = lattice.nn_index_offsets()                     # [12, 3] (dn0, dn1, dn2)
        proj = lattice.bond_projectors()                        # [12, 3, 3]
        self.bonds, self.proj = bonds, proj
        lim = int(np.ceil(4 * r_a)) + 8
        n1, n2 = np.meshgrid(np.arange(-lim, lim + 1), np.arange(-2 * lim, 2 * lim + 1), indexing="ij")
        cand = np.stack([n1.ravel(), n2.ravel()], axis=1)
        rho = np.linalg.norm(W.column_xy(cand), axis=1)
        col_a = cand[rho <= r_a]
        in_a = {tuple(c) for c in col_a}
        dcol = {(int(b[1]), int(b[2])) for b in bonds}

        def nbrs(c):
            return [(c[0] + d1, c[1] + d2) for d1, d2 in dcol]

        ip = sorted({n for c in in_a for n in nbrs(c) if n not in in_a})
        ip_set = set(ip)
        ipp_extra = sorted({n for c in ip for n in nbrs(c) if n not in in_a and n not in ip_set})
        self.cols_a = np.array(sorted(in_a), dtype=np.int32)
        self.cols_ip = np.array(ip, dtype=np.int32)                        # i+
        self.cols_ipp = np.array(ip + ipp_extra, dtype=np.int32)           # i++ (i+ first)
        self.n_a, self.n_ip, self.n_ipp = len(self.cols_a), len(self.cols_ip), len(self.cols_ipp)
        # global column numbering: A, then i++
        allc = np.concatenate([self.cols_a, self.cols_ipp])
        self.gidx = {tuple(c): g for g, c in enumerate(allc)}
        self.n_g = len(allc)
        self.k_a = self._rows(range(self.n_a))                             # rows of A atoms
        self.k_ip = self._rows(range(self.n_a, self.n_a + self.n_ip))      # rows of i+ atoms
        # dof permutations
        dof = np.arange(3 * nz * self.n_g).reshape(nz, self.n_g, 3)
        self.dof_a = dof[:, :self.n_a].ravel()
        self.dof_p = dof[:, self.n_a:].ravel()
        kaa = self.k_a[:, self.dof_a].tocsc()
        self.k_ap = self.k_a[:, self.dof_p].tocsr()
        self.lu = spla.splu(kaa)

    def _rows(self, gcols) -> sp.csr_matrix:
        """L_h rows, L_h[u](x) = sum_bonds k P_b (u(x) - u(x + R_b)), for the atoms of the
        given global columns in every layer; columns are all dofs (A and i++)."""
        nz, ng = self.nz, self.n_g
        gcols = list(gcols)
        allc = np.concatenate([self.cols_a, self.cols_ipp])
        rows, cols, vals = [], [], []
        for li, g in enumerate(gcols):
            c = allc[g]
            for n0 in range(nz):
                r0 = 3 * (n0 * len(gcols) + li)
                for b, (d0, d1, d2) in enumerate(self.bonds):
                    tgt = self.gidx[(int(c[0] + d1), int(c[1] + d2))]
                    m0 = (n0 + int(d0)) % nz
                    kp = self.k * self.proj[b]
                    for a in range(3):
                        for e in range(3):
                            rows += [r0 + a, r0 + a]
                            cols += [3 * (n0 * ng + g) + e, 3 * (m0 * ng + tgt) + e]
                            vals += [kp[a, e], -kp[a, e]]
        shape = (3 * nz * len(gcols), 3 * nz * ng)
        return sp.csr_matrix((vals, (rows, cols)), shape=shape)

    def solve_ah(self, f_ext_a: np.ndarray, u_p: np.ndarray) -> np.ndarray:
        """(AH): L_h^{A|A} u_A = f_ext - L_h^{A|i++} u_p (pad held), u arrays [nz][n][3]."""
        rhs = f_ext_a.ravel() - self.k_ap @ u_p.ravel()
        return self.lu.solve(rhs).reshape(self.nz, self.n_a, 3)

    def incompatibility_force(self, u_a: np.ndarray, u_p: np.ndarray) -> np.ndarray:
        """f_in on i+ (eq. flexbc.finc): L_h at the i+ atoms with the new atomistic and the
        old continuum displacements; [nz][n_ip][3]."""
        v = np.concatenate([u_a, u_p], axis=1)
        return (self.k_ip @ v.ravel()).reshape(self.nz, self.n_ip, 3)


def external_force(disc: HarmonicDisc, seed: int, radius: float = 1.6) -> np.ndarray:
    """Random forces on the A atoms within `radius` of the axis, zero total net force."""
    rng = np.random.default_rng(seed)
    rho = np.linalg.norm(W.column_xy(disc.cols_a), axis=1)
    f = np.zeros((disc.nz, disc.n_a, 3))
    sel = rho <= radius
    f[:, sel] = rng.normal(0.0, 0.1, size=(disc.nz, int(sel.sum()), 3))
    f[:, sel] -= f[:, sel].mean(axis=(0, 1))
    return f


def run_loop(disc: HarmonicDisc, f_ext: np.ndarray, update, n_iter: int):
    """Algorithm 1 from u_0 = 0 for n_iter iterations.  update(f_in, k) must apply lines
    5-8 to the pad state it holds and return the new pad displacements [nz][n_ipp][3].
    Returns (u_A, u_pad, history of ||f_in||_inf)."""
    u_p = np.zeros((disc.nz, disc.n_ipp, 3))
    hist = []
    u_a = None
    for k in range(n_iter):
        u_a = disc.solve_ah(f_ext, u_p)                       # atomistic solve with fixed pad
        f_in = disc.incompatibility_force(u_a, u_p)           # incompatibility forces
        hist.append(float(np.abs(f_in).max()))
        u_p = update(f_in, k)                                 # relaxation, pad update, mean
    return u_a, u_p, hist
