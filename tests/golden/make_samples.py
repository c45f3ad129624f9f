"""Writes sampled expected outputs of the FP64 oracle at full workload sizes.

For a workload of fbc_workloads, the raw harmonic response w = G^{p|i+} f is evaluated
by the oracle (oracle/green.py, oracle/apply.py steps written out per mode) at a few
pad columns spread along the ring, for every layer and RHS, and stored with a digest
of the input forces.  Only oracle/ and the seeded input module are used.

    python tests/golden/make_samples.py medium large
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fbc_workloads as W  # noqa: E402
from oracle import apply as oap, green as ogr  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_columns(n_b: int, k: int = 5) -> np.ndarray:
    return np.unique(np.linspace(0, n_b - 1, k).round().astype(np.int64))


def force_digest(f: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(f).tobytes()).hexdigest()


def make(name: str) -> str:
    wl = W.make_single(name)
    c = wl.cells[0]
    sel = sample_columns(c.n_b)
    fh = oap.line_rfft(c.forces).reshape(c.n_rhs, c.nz // 2 + 1, 3 * c.n_i)
    wh = np.empty((c.n_rhs, c.nz // 2 + 1, 3 * sel.size), dtype=np.complex128)
    t0 = time.time()
    for m in range(c.nz // 2 + 1):
        g = ogr.line_mode_green(c.nz, wl.bz, wl.bz, m)
        gm = ogr.dense_mode_matrix(ogr.gather_blocks(g, c.cols_b[sel], c.cols_i))
        wh[:, m, :] = (gm @ fh[:, m, :].T).T
        if m % 16 == 0:
            print(f"{name}: mode {m}/{c.nz // 2} ({time.time() - t0:.0f} s)", flush=True)
    w = oap.line_irfft(wh.reshape(c.n_rhs, c.nz // 2 + 1, sel.size, 3), c.nz)
    out = os.path.join(HERE, f"{name}_samples.npz")
    np.savez_compressed(out, cols=sel, w=w, digest=force_digest(c.forces), bz=wl.bz)
    return out


if __name__ == "__main__":
    for n in sys.argv[1:] or ["medium"]:
        print(make(n))
