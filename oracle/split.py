"""BF16 hi+lo split representation, emulated on the host (FP64 oracle; test
infrastructure only).

A value x is held as hi + lo with hi = bf16(x) and lo = bf16(x - hi), both rounded
to nearest even.  bf16 keeps 8 significant bits, so |x - hi| <= 2^-8 |x| and
|x - hi - lo| <= 2^-8 |x - hi| <= 2^-16 |x| (for normal values).  The emulation
predicts the error of a reduced-precision apply; it is not a bitwise target.
"""
from __future__ import annotations

import numpy as np


def round_bf16(x) -> np.ndarray:
    """Round float32 values to the nearest bf16 (ties to even); returns float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).copy()
    nan = np.isnan(a)
    out[nan] = a[nan]
    return out


def split_bf16(x) -> tuple[np.ndarray, np.ndarray]:
    """x (FP64) -> (hi, lo) bf16 values stored as float32."""
    x = np.asarray(x, dtype=np.float64)
    hi = round_bf16(x.astype(np.float32))
    lo = round_bf16((x - hi.astype(np.float64)).astype(np.float32))
    return hi, lo
