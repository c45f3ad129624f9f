"""Writes sampled expected outputs of the FP64 oracle at full workload sizes.

Two kinds of samples, both from the oracle (oracle/green.py, oracle/apply.py steps
written out per mode) and the seeded input module only:

  * `<name>_samples.npz`: the raw harmonic response w = G^{p|i+} f at a few pad columns
    spread along the ring, for every layer and RHS (all line modes evaluated);
  * `<name>_modes.npz`: the line spectrum w^(m) = G^(m) f^(m) (Section 2.3.2 in line-mode
    form) of the same response at a few line modes and pad columns, for every RHS.  Only
    the sampled modes are evaluated, so workloads whose Green function on the in-plane
    torus costs minutes per mode are checked at a bounded cost; the GPU side takes the
    forward line transform of its w at the sampled columns.  For the batched workload every
    cell gets its own sample (modes 0, 1, one seeded middle mode and N_z/2).

Each file stores a digest of the input forces.

    python tests/golden/make_samples.py medium large long:modes batched:modes
"""
import hashlib
import os
import sys
import time
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fbc_workloads as W  # noqa: E402
from oracle import apply as oap, green as ogr  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# line modes sampled per single-cell workload
MODES = {"long": (0, 1, 2, 37, 256, 511, 512), "large": (0, 1, 64, 128), "medium": (0, 1, 32, 64)}


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


def mode_spectrum(cell, bz: int, modes, cols, cache=None) -> np.ndarray:
    """w^(m) at the given modes and pad columns, [R, len(modes), len(cols), 3] complex."""
    fh = oap.line_rfft(cell.forces)                      # [R, Nz/2+1, n_i, 3]
    out = np.empty((cell.n_rhs, len(modes), len(cols), 3), dtype=np.complex128)
    for k, m in enumerate(modes):
        key = Fraction(int(m), cell.nz)                  # the Green function depends on m / N_z only
        g = cache.get(key) if cache is not None else None
        if g is None:
            g = ogr.line_mode_green(cell.nz, bz, bz, int(m))
            if cache is not None and (key.denominator <= 2 or key.numerator == 1):
                cache[key] = g                           # modes 0, N_z/2 and 1 recur across cells
        gm = ogr.dense_mode_matrix(ogr.gather_blocks(g, cell.cols_b[cols], cell.cols_i))
        f_m = fh[:, m].reshape(cell.n_rhs, 3 * cell.n_i)
        out[:, k] = (gm @ f_m.T).T.reshape(cell.n_rhs, len(cols), 3)
    return out


def make_modes(name: str) -> str:
    wl = W.make_single(name)
    c = wl.cells[0]
    cols = sample_columns(c.n_b, 64)
    modes = np.asarray(MODES[name], dtype=np.int64)
    t0 = time.time()
    wh = mode_spectrum(c, wl.bz, modes, cols)
    print(f"{name}: {len(modes)} modes x {len(cols)} columns in {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, f"{name}_modes.npz")
    np.savez_compressed(out, cols=cols, modes=modes, what=wh, digest=force_digest(c.forces), bz=wl.bz)
    return out


def make_batched_modes() -> str:
    wl = W.make_batched()
    rng = np.random.default_rng(2024)
    cache = {}
    arrays = {"n_cells": len(wl.cells), "bz": wl.bz}
    t0 = time.time()
    for k, c in enumerate(wl.cells):
        cols = sample_columns(c.n_b, 16)
        mid = int(rng.integers(2, c.nz // 2))
        modes = np.asarray(sorted({0, 1, mid, c.nz // 2}), dtype=np.int64)
        arrays[f"c{k}_cols"] = cols
        arrays[f"c{k}_modes"] = modes
        arrays[f"c{k}_what"] = mode_spectrum(c, wl.bz, modes, cols, cache)
        arrays[f"c{k}_digest"] = force_digest(c.forces)
        print(f"batched: cell {k} (N_z={c.nz}, n_i={c.n_i}, R={c.n_rhs}) modes {modes.tolist()} "
              f"({time.time() - t0:.0f} s)", flush=True)
    out = os.path.join(HERE, "batched_modes.npz")
    np.savez_compressed(out, **arrays)
    return out


if __name__ == "__main__":
    for n in sys.argv[1:] or ["medium"]:
        if n == "batched:modes":
            print(make_batched_modes())
        elif n.endswith(":modes"):
            print(make_modes(n.split(":")[0]))
        else:
            print(make(n))
