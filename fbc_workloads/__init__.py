"""Seeded synthetic workloads for the line-periodic FBC boundary update.

This module only builds inputs: the column sets of an interface ring and a pad
(boundary) ring, and Gaussian interface forces with zero net force per layer.
It holds none of the method's arithmetic (no force constants, no Green
function, no transforms), so the CPU oracle and the GPU library can both be fed
from it without sharing any code of the method.

Geometry (index space).  The fcc lattice with lattice constant a = 1 is written
in the primitive basis b0 = (1/2,-1/2,0), b1 = (1/2,0,1/2), b2 = (1/2,1/2,0)
(cubic coordinates).  b0 points along the dislocation line [1-10]; its length
c = 1/sqrt(2) is the period of one atom column.  A lattice site is the integer
triple (n0, n1, n2); the atom column is (n1, n2) and the layer is n0 mod N_z, so
every column holds exactly one atom per layer and the cell is periodic along the
line with period l3 = N_z c (Section 2.1: the domain is one period of a lattice
that is periodic along x3).  Projected onto the plane normal to the line, with
in-plane axes [001] and [110]/sqrt(2), column (n1, n2) sits at
x = n1/2, y = (n1 + 2 n2)/(2 sqrt 2).

Ring rule (the paper fixes no shape for the pad and interface sets, Section
2.2.2): with column density rho = 2 sqrt(2) / a^2 and ring width w = 1.35 a the
interface radius is R_i = n_i / (2 pi rho w).  The interface set is the n_i
columns closest to the circle of radius R_i; the pad set is the n_b columns of
smallest radius strictly outside the largest interface radius.  Ties are broken
by polar angle, then by (n1, n2).  Both sets are returned sorted by polar angle
(then radius), which keeps neighbouring columns close in memory.

Forces: i.i.d. normal with variance 1e-2 (standard deviation 0.1), drawn in
FP64 from numpy's PCG64 generator, then projected to zero net force per layer
and component by subtracting the mean over columns.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

RHO = 2.0 * math.sqrt(2.0)   # columns per unit area in the plane normal to [1-10]
RING_WIDTH = 1.35


def column_xy(cols: np.ndarray) -> np.ndarray:
    """In-plane coordinates (x along [001], y along [110]/sqrt2) of columns (n1, n2)."""
    cols = np.asarray(cols, dtype=np.int64)
    n1 = cols[..., 0].astype(np.float64)
    n2 = cols[..., 1].astype(np.float64)
    return np.stack([0.5 * n1, (n1 + 2.0 * n2) / (2.0 * math.sqrt(2.0))], axis=-1)


def _radius2_x8(n1: np.ndarray, n2: np.ndarray) -> np.ndarray:
    """8 r^2 as an exact integer: 2 n1^2 + (n1 + 2 n2)^2."""
    return 2 * n1 * n1 + (n1 + 2 * n2) ** 2


def ring_columns(n_i: int, n_b: int) -> tuple[np.ndarray, np.ndarray]:
    """Interface and pad column sets, int32 arrays of shape [n][2] holding (n1, n2)."""
    if n_i <= 0 or n_b <= 0:
        raise ValueError("ring sizes must be positive")
    r_i = n_i / (2.0 * math.pi * RHO * RING_WIDTH)
    # enough area for both rings with a generous margin
    r_max = r_i + 3.0 * (n_b / (2.0 * math.pi * RHO * max(r_i, 1.0))) + 4.0 * RING_WIDTH + 4.0
    n1_lim = int(math.ceil(2.0 * r_max)) + 2
    n2_lim = int(math.ceil(2.0 * math.sqrt(2.0) * r_max + n1_lim)) + 2
    n1, n2 = np.meshgrid(np.arange(-n1_lim, n1_lim + 1), np.arange(-n2_lim, n2_lim + 1), indexing="ij")
    n1 = n1.ravel()
    n2 = n2.ravel()
    r2x8 = _radius2_x8(n1, n2)
    keep = r2x8 <= int(8.0 * r_max * r_max)
    n1, n2, r2x8 = n1[keep], n2[keep], r2x8[keep]
    r = np.sqrt(r2x8 / 8.0)
    xy = column_xy(np.stack([n1, n2], axis=1))
    ang = np.arctan2(xy[:, 1], xy[:, 0])

    order = np.lexsort((n2, n1, ang, np.abs(r - r_i)))
    sel_i = order[:n_i]
    r_cut = r2x8[sel_i].max()
    outside = np.nonzero(r2x8 > r_cut)[0]
    order_b = outside[np.lexsort((n2[outside], n1[outside], ang[outside], r2x8[outside]))]
    if order_b.size < n_b:
        raise RuntimeError("candidate disc too small for the pad ring")
    sel_b = order_b[:n_b]

    def _sorted(sel):
        o = np.lexsort((n2[sel], n1[sel], r2x8[sel], ang[sel]))
        s = sel[o]
        return np.stack([n1[s], n2[s]], axis=1).astype(np.int32)

    return _sorted(sel_i), _sorted(sel_b)


def gaussian_forces(rng: np.random.Generator, n_rhs: int, nz: int, n_i: int,
                    sigma: float = 0.1, zero_net_force: bool = True) -> np.ndarray:
    """Interface forces f[r][n0][i][3] (FP64) with zero net force per layer and component."""
    f = rng.normal(0.0, sigma, size=(n_rhs, nz, n_i, 3))
    if zero_net_force:
        f -= f.mean(axis=2, keepdims=True)
    return np.ascontiguousarray(f)


@dataclass
class Cell:
    """One line-periodic dislocation cell: layers, column sets and right-hand sides."""
    nz: int
    cols_i: np.ndarray
    cols_b: np.ndarray
    n_rhs: int
    forces: np.ndarray = field(repr=False)

    @property
    def n_i(self) -> int:
        return int(self.cols_i.shape[0])

    @property
    def n_b(self) -> int:
        return int(self.cols_b.shape[0])


@dataclass
class Workload:
    name: str
    cells: list
    bz: int            # in-plane torus size M1 = M2 of the Brillouin-zone grid
    spring_k: float = 1.0
    lattice_a: float = 1.0
    description: str = ""

    @property
    def total_rhs(self) -> int:
        return sum(c.n_rhs for c in self.cells)


# name -> (nz, n_i, n_b, n_rhs, bz, seed, description)
SINGLE_CELL = {
    "tiny":   (8, 96, 192, 1, 64, 1000,
               "N_z=8, n_i=96 (ring radius 4a), n_b=192, 1 RHS"),
    "medium": (128, 1024, 2048, 8, 1024, 1001,
               "N_z=128, n_i=1024, n_b=2048, 8 RHS (65 modes, 6144x3072 complex blocks)"),
    "large":  (256, 2048, 4096, 64, 2048, 1002,
               "N_z=256, n_i=2048, n_b=4096, 64 RHS (129 modes, 12288x6144 complex blocks)"),
    "long":   (1024, 4096, 8192, 16, 4096, 1004,
               "N_z=1024, n_i=4096, n_b=8192, 16 RHS (513 modes, 24576x12288 complex blocks)"),
    # small cases for parity tests: several tiles and ragged tails, oracle in seconds
    "parity": (16, 100, 170, 3, 64, 7, "N_z=16, n_i=100, n_b=170, 3 RHS, M=64"),
    "micro":  (4, 10, 14, 2, 8, 11, "N_z=4, n_i=10, n_b=14, 2 RHS, M=8"),
}


def make_single(name: str, n_rhs: int | None = None, with_forces: bool = True) -> Workload:
    nz, n_i, n_b, rhs, bz, seed, desc = SINGLE_CELL[name]
    if n_rhs is not None:
        rhs = n_rhs
    rng = np.random.default_rng(seed)
    ci, cb = ring_columns(n_i, n_b)
    f = gaussian_forces(rng, rhs, nz, n_i) if with_forces else np.zeros((0,))
    return Workload(name=name, cells=[Cell(nz, ci, cb, rhs, f)], bz=bz, description=desc)


def make_custom(nz: int, n_i: int, n_b: int, n_rhs: int, bz: int, seed: int,
                zero_net_force: bool = True) -> Workload:
    rng = np.random.default_rng(seed)
    ci, cb = ring_columns(n_i, n_b)
    f = gaussian_forces(rng, n_rhs, nz, n_i, zero_net_force=zero_net_force)
    return Workload(name=f"custom-{nz}-{n_i}-{n_b}-{n_rhs}-{bz}", cells=[Cell(nz, ci, cb, n_rhs, f)], bz=bz,
                    description=f"N_z={nz}, n_i={n_i}, n_b={n_b}, {n_rhs} RHS")


def make_batched(n_cells: int = 32, seed: int = 1003, bz: int = 2048,
                 nz_choices=(32, 64, 128, 256, 512), n_i_range=(256, 2048),
                 rhs_range=(1, 16), with_forces: bool = True) -> Workload:
    """Independent cells of uneven size: N_z from nz_choices, n_i uniform in n_i_range,
    n_b = 2 n_i, 1..16 RHS each."""
    rng = np.random.default_rng(seed)
    nzs = rng.choice(np.asarray(nz_choices), size=n_cells)
    nis = rng.integers(n_i_range[0], n_i_range[1] + 1, size=n_cells)
    rhs = rng.integers(rhs_range[0], rhs_range[1] + 1, size=n_cells)
    cells = []
    for c in range(n_cells):
        ci, cb = ring_columns(int(nis[c]), 2 * int(nis[c]))
        f = gaussian_forces(rng, int(rhs[c]), int(nzs[c]), int(nis[c])) if with_forces else np.zeros((0,))
        cells.append(Cell(int(nzs[c]), ci, cb, int(rhs[c]), f))
    return Workload(name=f"batched-{n_cells}", cells=cells, bz=bz,
                    description=f"{n_cells} cells, N_z in {tuple(nz_choices)}, n_i in {n_i_range}, n_b=2n_i, RHS in {rhs_range}")
