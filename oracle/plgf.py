"""Real-space periodic lattice Green function (FP64 oracle; test infrastructure only).

Section 3.1 builds the line-periodic Green function from the Green function of the
infinite lattice instead of computing it for every period:

* eq. (G~inf): G~inf(r) = G_inf(r) for |r| <= r_cut and the continuum Green function
  G_cgf(r) (eq. cgf, homogeneous of degree -1) beyond;
* eq. (plgf_conv): G~(r) = sum_i [G~inf(r + i l3 t) - G~inf(i l3 t)], t the line
  direction, l3 the period; subtracting the images of the origin keeps the sum finite;
* eq. (plgf_poly): the partial sums G~_n over |i| <= n behave like
  Q0 + Q1/n + Q2/n^2 + ..., and eq. (plgf_rich) takes Q0 by Richardson extrapolation
  from G~_n, ..., G~_{n+N} (the paper uses n + N = 6 images, N = 5).

Appendix B computes G_inf within r_cut by Brillouin-zone integration and, beyond it,
uses G_cgf; a constant C = G_inf(r') - G_cgf(r') at large r' is subtracted from the
computed G_inf values so the two pieces join.

Readings (each also listed in the design notes):
* G_inf within r_cut is evaluated as the Green function of the L x L x L torus of the
  primitive cell (Brillouin-zone sum on the L^3 grid, q = 0 dropped), which differs from
  G_inf by a constant plus terms of order (|r| / (L c))^3 relative;
* C is the mean of G_torus - G_cgf over the lattice vectors of the shell
  r_cut < |r| <= r_match (a symmetric shell, so the anisotropic lattice corrections of
  order |r|^-3 average out to leading order);
* r_cut and r_match are given as 4 |r|^2 (integers for fcc with a = 1), so that the
  membership of a lattice vector is decided exactly.

Coordinates: a lattice vector is n = (n0, n1, n2) in the primitive basis of
``lattice.BASIS`` (b0 along the line [1-10]); its position is B n (cube axes, a = 1).
A line of N_z layers has the period l3 t = N_z b0.
"""
from __future__ import annotations

import math

import numpy as np

from .cgf import kelvin_green, nn_fcc_stiffness
from .green import green_real_space
from .lattice import BASIS


def four_r2(n: np.ndarray) -> np.ndarray:
    """4 |B n|^2 as integers (2 B n has integer components for fcc)."""
    x2 = np.rint(2.0 * (np.asarray(n, dtype=np.float64) @ BASIS.T)).astype(np.int64)
    return (x2 * x2).sum(axis=-1)


def lattice_vectors(r2x4_max: int, r2x4_min: int = -1) -> np.ndarray:
    """All primitive-basis vectors n with r2x4_min < 4|B n|^2 <= r2x4_max, sorted by
    (4|B n|^2, n0, n1, n2)."""
    binv = np.linalg.inv(BASIS)
    bound = int(math.ceil(math.sqrt(r2x4_max / 4.0) * np.abs(binv).sum(axis=1).max())) + 1
    rng = np.arange(-bound, bound + 1)
    n = np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), axis=-1).reshape(-1, 3)
    d2 = four_r2(n)
    keep = (d2 <= r2x4_max) & (d2 > r2x4_min)
    n, d2 = n[keep], d2[keep]
    order = np.lexsort((n[:, 2], n[:, 1], n[:, 0], d2))
    return n[order]


def torus_green(L: int, spring_k: float = 1.0) -> np.ndarray:
    """Green function of the L^3 torus of the primitive cell, [L, L, L, 3, 3] (Appendix B,
    inverse semi-discrete transform on the L^3 grid, q = 0 dropped)."""
    return green_real_space(L, L, L, spring_k)


def torus_at(gt: np.ndarray, n: np.ndarray) -> np.ndarray:
    L = gt.shape[0]
    n = np.asarray(n) % L
    return gt[n[..., 0], n[..., 1], n[..., 2]]


def matching_constant(gt: np.ndarray, r2x4_cut: int, r2x4_match: int, n_psi: int = 64) -> np.ndarray:
    """C = mean over the shell r_cut < |r| <= r_match of G_torus(r) - G_cgf(r) (Appendix B)."""
    shell = lattice_vectors(r2x4_match, r2x4_cut)
    x = shell.astype(np.float64) @ BASIS.T
    diff = torus_at(gt, shell) - kelvin_green(x, nn_fcc_stiffness(), n_psi)
    return diff.mean(axis=0)


class InfiniteLatticeGreen:
    """G~inf of eq. (G~inf): the table of G_inf - C within r_cut, the continuum beyond."""

    def __init__(self, L: int, r2x4_cut: int, r2x4_match: int, n_psi: int = 64, spring_k: float = 1.0):
        gt = torus_green(L, spring_k)
        self.c = matching_constant(gt, r2x4_cut, r2x4_match, n_psi)
        self.vectors = lattice_vectors(r2x4_cut)
        self.table = torus_at(gt, self.vectors) - self.c
        self.index = {tuple(v): k for k, v in enumerate(self.vectors.tolist())}
        self.r2x4_cut = r2x4_cut
        self.n_psi = n_psi
        self.stiffness = nn_fcc_stiffness(spring_k)

    def __call__(self, n: np.ndarray) -> np.ndarray:
        """G~inf at lattice vectors n[..., 3] -> [..., 3, 3]."""
        n = np.asarray(n, dtype=np.int64)
        flat = n.reshape(-1, 3)
        out = np.empty((flat.shape[0], 3, 3))
        inside = four_r2(flat) <= self.r2x4_cut
        if inside.any():
            out[inside] = self.table[[self.index[tuple(v)] for v in flat[inside].tolist()]]
        if (~inside).any():
            x = flat[~inside].astype(np.float64) @ BASIS.T
            out[~inside] = kelvin_green(x, self.stiffness, self.n_psi)
        return out.reshape(n.shape[:-1] + (3, 3))


def partial_sums(ginf: InfiniteLatticeGreen, n: np.ndarray, nz: int, k_max: int) -> np.ndarray:
    """G~_k(r) for k = 1..k_max (eq. plgf_poly): sum over |i| <= k of
    G~inf(n + i N_z e0) - G~inf(i N_z e0).  Returns [k_max, ..., 3, 3]."""
    n = np.asarray(n, dtype=np.int64)
    e0 = np.array([nz, 0, 0], dtype=np.int64)
    out = []
    acc = ginf(n) - ginf(np.zeros(3, dtype=np.int64))
    for k in range(1, k_max + 1):
        for i in (-k, k):
            acc = acc + ginf(n + i * e0) - ginf(i * e0)
        out.append(acc.copy())
    return np.stack(out)


def richardson_weights(n: int, order: int) -> np.ndarray:
    """Weights w_i of eq. (plgf_rich): Q0 = sum_{i=0}^{N} w_i G~_{n+i},
    w_i = (n+i)^N (-1)^(i+N) / (i! (N-i)!)."""
    return np.array([(n + i) ** order * (-1.0) ** (i + order) / (math.factorial(i) * math.factorial(order - i))
                     for i in range(order + 1)])


def richardson(seq: np.ndarray, n: int, order: int) -> np.ndarray:
    """Q0 from seq[k - 1] = G~_k (k = 1, 2, ...) using G~_n .. G~_{n+N}."""
    w = richardson_weights(n, order)
    return np.tensordot(w, seq[n - 1:n + order], axes=(0, 0))


def periodic_green(ginf: InfiniteLatticeGreen, n: np.ndarray, nz: int, n_rich: int = 1, order: int = 5) -> np.ndarray:
    """G~(r) of eq. (plgf_conv), Richardson-extrapolated (eq. plgf_rich)."""
    return richardson(partial_sums(ginf, n, nz, n_rich + order), n_rich, order)


def periodic_line_modes(ginf: InfiniteLatticeGreen, dn1: int, dn2: int, nz: int, n_rich: int = 1,
                        order: int = 5) -> np.ndarray:
    """Line transform of G~ at column offset (dn1, dn2): sum over the layer offset dn0 of
    G~(dn0, dn1, dn2) e^{-2 pi i m dn0 / N_z}, m = 0..N_z/2 -> [N_z/2 + 1, 3, 3]."""
    n = np.array([[d0, dn1, dn2] for d0 in range(nz)], dtype=np.int64)
    g = periodic_green(ginf, n, nz, n_rich, order)
    return np.fft.rfft(g, axis=0)
