"""Harmonic pad update by line transforms (FP64 oracle; test infrastructure only).

Section 2.3.2, eq. flexbc.up=Gpipl*fipl: u^p_{k+1} = u^p_k - G^{p|i+}[f_in].  The
Green matrix has entries G(r_ij) that depend only on the separation (Section 3.2)
and the cell is periodic along the line (Section 2.1), so G^{p|i+} is
block-circulant in the layer index and a discrete Fourier transform over layers
block-diagonalises it:
  1. f^_i(m) = sum_n0 f_i(n0) e^{-2 pi i m n0 / Nz}           (forward, unnormalised)
  2. w^_b(m) = sum_i G^_{bi}(m) f^_i(m)                        (one matrix product per mode)
  3. w_b(n0) = (1/Nz) sum_m w^_b(m) e^{+2 pi i m n0 / Nz}      (inverse)
Real forces give Hermitian spectra, so modes 0..Nz/2 suffice (rfft / irfft).

Update step of Algorithm 1 and eq. mean(u^p)=0: u^p <- u^p - alpha w, then the mean
of each Cartesian component over all pad atoms of all layers is subtracted.
"""
from __future__ import annotations

import numpy as np


def net_force(f: np.ndarray) -> np.ndarray:
    """Per RHS, layer and component: sum over interface columns, [R, Nz, 3]."""
    return np.asarray(f).sum(axis=2)


def line_rfft(f: np.ndarray) -> np.ndarray:
    """[R, Nz, n, 3] real -> [R, Nz/2+1, n, 3] complex (step 1)."""
    return np.fft.rfft(np.asarray(f, dtype=np.float64), axis=1)


def line_irfft(uh: np.ndarray, nz: int) -> np.ndarray:
    """[R, Nz/2+1, n, 3] complex -> [R, Nz, n, 3] real, with the 1/Nz factor (step 3)."""
    return np.fft.irfft(uh, n=nz, axis=1)


def apply_green(gmodes: np.ndarray, f: np.ndarray) -> np.ndarray:
    """w = G^{p|i+} f for every RHS.  gmodes: [Nz/2+1, 3 n_b, 3 n_i]; f: [R, Nz, n_i, 3].
    Returns w [R, Nz, n_b, 3]."""
    n_rhs, nz, n_i, _ = f.shape
    n_modes = nz // 2 + 1
    assert gmodes.shape[0] == n_modes and gmodes.shape[2] == 3 * n_i
    n_b = gmodes.shape[1] // 3
    fh = line_rfft(f).reshape(n_rhs, n_modes, 3 * n_i)
    wh = np.empty((n_rhs, n_modes, 3 * n_b), dtype=np.complex128)
    for m in range(n_modes):
        wh[:, m, :] = (gmodes[m] @ fh[:, m, :].T).T
    return line_irfft(wh.reshape(n_rhs, n_modes, n_b, 3), nz)


def apply_direct(greal: np.ndarray, cols_b: np.ndarray, cols_i: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Real-space circulant sum w_b(n0) = sum_{n0'} sum_i G(n0 - n0', n_b - n_i) f_i(n0')
    (Section 3.2, eq. impl.up=Gpipl*fipl_mvm, written per atom); O(Nz^2 n_b n_i)."""
    nz, m1, m2 = greal.shape[:3]
    n_rhs = f.shape[0]
    n_b = cols_b.shape[0]
    d1 = (cols_b[:, None, 0].astype(np.int64) - cols_i[None, :, 0]) % m1
    d2 = (cols_b[:, None, 1].astype(np.int64) - cols_i[None, :, 1]) % m2
    w = np.zeros((n_rhs, nz, n_b, 3))
    for n0 in range(nz):
        for n0p in range(nz):
            gb = greal[(n0 - n0p) % nz][d1, d2]               # [n_b, n_i, 3, 3]
            w[:, n0] += np.einsum("bicd,rid->rbc", gb, f[:, n0p])
    return w


def pad_update(u: np.ndarray, w: np.ndarray, alpha) -> tuple[np.ndarray, np.ndarray]:
    """u <- u - alpha w, then subtract the per-component mean over all pad atoms and
    layers (update step of Algorithm 1; eq. mean(u^p)=0).  alpha: scalar or [R].
    Returns (u_new, removed_mean[R, 3])."""
    a = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (u.shape[0],))
    v = u - a[:, None, None, None] * w
    mean = v.mean(axis=(1, 2))
    return v - mean[:, None, None, :], mean
