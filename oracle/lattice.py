"""FCC lattice with nearest-neighbour central springs (FP64 oracle; test infrastructure only).

Section 2.1 (eq. flexbc.bravais): a Bravais lattice sum_i a_i b_i.  Here fcc, a = 1,
written in the primitive basis b0 = (1/2,-1/2,0) (along the line [1-10]),
b1 = (1/2,0,1/2), b2 = (1/2,1/2,0).

Section 2.2.1: the harmonic operator L_h[u](x) = sum_y K_h(x - y) u(y) with a
nearest-neighbour force-constant tensor.  For central springs of stiffness k on
the 12 bonds R in (a/2)<110>:  K_h(R) = -k Rhat Rhat^T and K_h(0) = -sum_R K_h(R).

Appendix B: the Fourier symbol of K_h is
    D(q) = sum_R K_h(R) e^{-i q.R} = k sum_R Rhat Rhat^T (1 - cos q.R),
written here as 2 k sum_R Rhat Rhat^T sin^2(q.R / 2) (same quantity, no
cancellation near q = 0).  q is given by fractional coordinates theta along the
reciprocal basis, so q.(sum_j n_j b_j) = 2 pi theta.n.
"""
from __future__ import annotations

import itertools

import numpy as np

BASIS = np.array([[0.5, -0.5, 0.0],
                  [0.5, 0.0, 0.5],
                  [0.5, 0.5, 0.0]]).T          # columns b0, b1, b2 (cubic coordinates, a = 1)


def nn_vectors(a: float = 1.0) -> np.ndarray:
    """The 12 nearest-neighbour bond vectors (a/2)<110> in cubic coordinates."""
    out = []
    for i, j in itertools.combinations(range(3), 2):
        for si, sj in itertools.product((1.0, -1.0), repeat=2):
            v = np.zeros(3)
            v[i], v[j] = si * a / 2, sj * a / 2
            out.append(v)
    return np.array(out)


def nn_index_offsets() -> np.ndarray:
    """Integer primitive-basis coordinates n_R of the 12 bonds (B n_R = R)."""
    n = np.linalg.solve(BASIS, nn_vectors().T).T
    ni = np.rint(n)
    assert np.max(np.abs(n - ni)) < 1e-12
    return ni.astype(np.int64)


def bond_projectors() -> np.ndarray:
    """Rhat Rhat^T for the 12 bonds, shape [12, 3, 3]."""
    r = nn_vectors()
    rh = r / np.linalg.norm(r, axis=1, keepdims=True)
    return np.einsum("bi,bj->bij", rh, rh)


def dynamical_matrix(theta: np.ndarray, spring_k: float = 1.0) -> np.ndarray:
    """D(q) for q given by fractional reciprocal coordinates theta[..., 3] (Appendix B).

    Returns a real symmetric array [..., 3, 3].
    """
    theta = np.asarray(theta, dtype=np.float64)
    nr = nn_index_offsets().astype(np.float64)          # [12, 3]
    p = bond_projectors()                                # [12, 3, 3]
    phase = theta @ nr.T                                 # [..., 12]  (q.R / 2pi)
    s2 = np.sin(np.pi * phase) ** 2                      # (1 - cos q.R) / 2
    return 2.0 * spring_k * np.einsum("...b,bij->...ij", s2, p)


def elastic_constants_nn_fcc(spring_k: float = 1.0, a: float = 1.0) -> tuple[float, float, float]:
    """Textbook cubic constants of the nearest-neighbour central-force fcc crystal:
    C11 = 2k/a, C12 = C44 = k/a (Cauchy relation holds)."""
    return 2.0 * spring_k / a, spring_k / a, spring_k / a


def acoustic_tensor(qvec: np.ndarray, c11: float, c12: float, c44: float) -> np.ndarray:
    """Gamma_ik(q) = C_ijkl q_j q_l for a cubic crystal in its cube axes (cubic coordinates)."""
    q = np.asarray(qvec, dtype=np.float64)
    g = np.empty(q.shape[:-1] + (3, 3))
    qq = q * q
    tot = qq.sum(axis=-1)
    for i in range(3):
        for k in range(3):
            if i == k:
                g[..., i, i] = c11 * qq[..., i] + c44 * (tot - qq[..., i])
            else:
                g[..., i, k] = (c12 + c44) * q[..., i] * q[..., k]
    return g


def reciprocal_basis() -> np.ndarray:
    """Rows g_j with g_j . b_l = delta_jl (q = 2 pi sum_j theta_j g_j)."""
    return np.linalg.inv(BASIS)


ATOMIC_VOLUME = abs(np.linalg.det(BASIS))   # a^3 / 4
