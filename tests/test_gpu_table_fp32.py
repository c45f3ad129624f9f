"""Offset-table products on FP32 MFMA (options.table_fp32): at the line modes whose far
blocks are skipped the gathered FP64 blocks and f^ are rounded to FP32 (FP32 sums over 8
interface columns, FP64 across them); the modes without skipping stay on FP64 MFMA.
Against the oracle within the FP32 form's tolerance; different from the FP64 table
product (the FP32 path ran) but close to it; with the update and mean removal too."""
import numpy as np
import pytest

import fbc_workloads as W
from oracle import apply as oap

from test_gpu_parity import _ctx, _dev, oracle_green, oracle_update, rel_err, run_apply, split_cells, torch

pytestmark = pytest.mark.gpu


def _green(wl, **kw):
    dev = _dev()
    c = wl.cells[0]
    ctx = _ctx(wl.cells, wl.bz, form="dtable_fp64", **kw)
    f = torch.from_numpy(c.forces).to(dev)
    w = torch.zeros((c.n_rhs, c.nz, c.n_b, 3), dtype=torch.float64, device=dev)
    ctx.green_apply(f, w)
    assert ctx.sync_status() == 0
    skipped = ctx.info.skipped_fraction
    ctx.close()
    return w.cpu().numpy(), skipped


def test_table_fp32_green_apply_matches_oracle():
    # rings of radius ~17 / ~22: the upper modes skip most far chunks
    wl = W.make_custom(16, 400, 800, 3, 256, seed=31)
    w32, sk = _green(wl, table_fp32=True, skip_tol=1e-9)
    w64, _ = _green(wl, skip_tol=1e-9)
    assert sk > 0.05, sk
    ref = oap.apply_green(oracle_green(wl.cells[0], wl.bz), wl.cells[0].forces)
    e2, emax = rel_err(w32, ref)
    assert e2 < 1e-6 and emax < 3e-6, (e2, emax)
    d2, _ = rel_err(w32, w64)
    assert 1e-13 < d2 < 1e-6, d2        # the FP32 path ran, and agrees with FP64 to its rounding


@pytest.mark.parametrize("nz,n_i,n_b,R,bz", [(16, 400, 800, 9, 256), (32, 130, 300, 17, 128)])
def test_table_fp32_update_matches_oracle(nz, n_i, n_b, R, bz):
    wl = W.make_custom(nz, n_i, n_b, R, bz, seed=nz + R)
    rc, got, u0 = run_apply(wl, "dtable_fp64", alpha=0.9, table_fp32=True, skip_tol=1e-9)
    assert rc == 0
    ref = oracle_update(wl, u0, 0.9)
    e2, emax = rel_err(split_cells(wl, got)[0], ref[0])
    assert e2 < 1e-6 and emax < 3e-6, (e2, emax)
