"""GPU parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: FP64 forms <= 1e-10 relative (per RHS, 2-norm over all pad outputs, and
max-abs relative to the largest output); reduced forms at the bound stated per form.
Inputs come from the seeded workload module; expected values from oracle/ only.
"""
import numpy as np
import pytest

import fbc_workloads as W
from oracle import apply as oap, green as ogr, relax as orx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _ctx(cells, bz, **kw):
    from paper_2105_08798_amd import FBC
    return FBC(cells, bz, **kw)


_GCACHE = {}


def oracle_green(cell, bz):
    key = (cell.nz, bz, cell.cols_i.tobytes(), cell.cols_b.tobytes())
    if key not in _GCACHE:
        _GCACHE[key] = ogr.green_modes_dense(cell.nz, bz, bz, cell.cols_b, cell.cols_i)
    return _GCACHE[key]


def rel_err(got, ref):
    """max over RHS of ||got - ref|| / ||ref||, and max-abs error / max |ref|."""
    n = ref.shape[0]
    g = got.reshape(n, -1)
    r = ref.reshape(n, -1)
    per = np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)
    return float(per.max()), float(np.abs(g - r).max() / np.abs(r).max())


def run_apply(wl, form="fp64", alpha=1.0, seed=0, **kw):
    dev = _dev()
    ctx = _ctx(wl.cells, wl.bz, form=form, **kw)
    f = torch.from_numpy(np.concatenate([c.forces.ravel() for c in wl.cells])).to(dev)
    rng = np.random.default_rng(seed)
    u0 = [rng.normal(size=(c.n_rhs, c.nz, c.n_b, 3)) * 0.01 for c in wl.cells]
    u = torch.from_numpy(np.concatenate([x.ravel() for x in u0])).to(dev)
    ctx.apply(f, u, alpha=alpha)
    rc = ctx.sync_status()
    got = u.cpu().numpy()
    ctx.close()
    return rc, got, u0


def oracle_update(wl, u0, alpha=1.0):
    out = []
    for c, uc in zip(wl.cells, u0):
        w = oap.apply_green(oracle_green(c, wl.bz), c.forces)
        un, _ = oap.pad_update(uc, w, alpha)
        out.append(un)
    return out


def split_cells(wl, flat):
    out, off = [], 0
    for c in wl.cells:
        n = c.n_rhs * c.nz * c.n_b * 3
        out.append(flat[off:off + n].reshape(c.n_rhs, c.nz, c.n_b, 3))
        off += n
    return out


FP64_FORMS = ["fp64", "dtable_fp64"]


@pytest.mark.parametrize("form", FP64_FORMS)
@pytest.mark.parametrize("name", ["parity", "micro", "tiny"])
def test_fp64_apply_matches_oracle(name, form):
    wl = W.make_single(name)
    rc, got, u0 = run_apply(wl, form, alpha=0.7)
    assert rc == 0
    ref = oracle_update(wl, u0, 0.7)
    for g, r in zip(split_cells(wl, got), ref):
        e2, emax = rel_err(g, r)
        assert e2 < 1e-10 and emax < 1e-10, (name, e2, emax)


@pytest.mark.parametrize("nz,n_i,n_b,R,bz", [(2, 7, 11, 1, 16), (32, 33, 50, 9, 32), (64, 21, 40, 17, 16),
                                             (8, 1, 1, 2, 8), (16, 130, 260, 33, 64),
                                             (8, 20, 30, 2, 2048), (256, 20, 30, 2, 32), (16, 50, 80, 64, 64),
                                             (1024, 9, 13, 3, 16), (4, 12, 20, 1, 4096), (512, 17, 40, 5, 16),
                                             (1024, 30, 70, 9, 16), (2048, 5, 9, 2, 16)])
@pytest.mark.parametrize("form", FP64_FORMS)
def test_fp64_ragged_shapes(nz, n_i, n_b, R, bz, form):
    wl = W.make_custom(nz, n_i, n_b, R, bz, seed=nz + n_i)
    rc, got, u0 = run_apply(wl, form, alpha=1.3)
    assert rc == 0
    ref = oracle_update(wl, u0, 1.3)
    e2, emax = rel_err(split_cells(wl, got)[0], ref[0])
    assert e2 < 1e-10 and emax < 1e-10, (e2, emax)


@pytest.mark.parametrize("form", FP64_FORMS)
def test_fp64_assembled_blocks_match_oracle(form):
    _dev()
    wl = W.make_single("parity")
    c = wl.cells[0]
    ctx = _ctx(wl.cells, wl.bz, form=form)
    g = oracle_green(c, wl.bz)
    for m in (0, 1, c.nz // 2):
        got = ctx.block_rows(0, m, 0, c.n_b, c.n_i)
        ref = g[m]
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max(), m
    ctx.close()


def test_green_apply_is_raw_response():
    wl = W.make_single("parity")
    c = wl.cells[0]
    dev = _dev()
    ctx = _ctx(wl.cells, wl.bz, form="fp64")
    f = torch.from_numpy(c.forces).to(dev)
    w = torch.full((c.n_rhs, c.nz, c.n_b, 3), 7.0, dtype=torch.float64, device=dev)
    ctx.green_apply(f, w)
    assert ctx.sync_status() == 0
    ref = oap.apply_green(oracle_green(c, wl.bz), c.forces)
    e2, emax = rel_err(w.cpu().numpy(), ref)
    ctx.close()
    assert e2 < 1e-10 and emax < 1e-10


@pytest.mark.parametrize("form", FP64_FORMS + ["fp32", "split_fp16"])
def test_multi_cell_context_matches_per_cell_oracle(form):
    cells = W.make_custom(16, 30, 45, 3, 32, seed=1).cells + W.make_custom(8, 12, 20, 10, 32, seed=2).cells \
        + W.make_custom(32, 50, 60, 1, 32, seed=3).cells
    wl = W.Workload("three", cells, bz=32)
    rc, got, u0 = run_apply(wl, form, alpha=1.0)
    assert rc == 0
    tol = 1e-10 if form in FP64_FORMS else 1e-6
    for g, r in zip(split_cells(wl, got), oracle_update(wl, u0, 1.0)):
        e2, emax = rel_err(g, r)
        assert e2 < tol and emax < tol, (form, e2, emax)


@pytest.mark.parametrize("form,tol", [("split_fp16", 1e-6), ("fp32", 1e-6)])
def test_multi_cell_layer_net_forces(form, tol):
    """Cells of different line lengths in one context, some with per-layer net force
    (zero cell total) and some balanced: each cell's row-gauge compensation reads its own
    R_b(m) and s^ (the fused update at 16 and 512 layers, the inverse into w at 2048)."""
    specs = [(16, 30, 45, 3, 21, False), (512, 7, 13, 9, 22, True), (2048, 5, 9, 2, 23, False),
             (512, 6, 11, 5, 24, False)]
    cells = []
    for nz, n_i, n_b, R, seed, balanced in specs:
        c = W.make_custom(nz, n_i, n_b, R, 32, seed=seed, zero_net_force=False).cells[0]
        f = c.forces - c.forces.mean(axis=(1, 2), keepdims=True)
        if balanced:
            f = f - f.mean(axis=2, keepdims=True)
        else:
            assert np.abs(f.sum(axis=2)).max() > 1e-2
        c.forces = np.ascontiguousarray(f)
        cells.append(c)
    wl = W.Workload("mixed", cells, bz=32)
    rc, got, u0 = run_apply(wl, form, alpha=0.9)
    assert rc == 0
    for k, (g, r) in enumerate(zip(split_cells(wl, got), oracle_update(wl, u0, 0.9))):
        e2, emax = rel_err(g, r)
        assert e2 < tol and emax < 3 * tol, (form, k, e2, emax)


def test_net_force_violation_latched_and_u_untouched():
    wl = W.make_custom(8, 20, 30, 2, 16, seed=5, zero_net_force=False)
    rc, got, u0 = run_apply(wl, "fp64")
    from paper_2105_08798_amd.fbc import STATUS
    assert STATUS[rc] == "FBC_E_NETFORCE"
    assert np.array_equal(got, np.concatenate([x.ravel() for x in u0]))


def test_nonfinite_force_latched():
    wl = W.make_custom(8, 20, 30, 1, 16, seed=6)
    wl.cells[0].forces[0, 3, 4, 1] = np.nan
    rc, got, u0 = run_apply(wl, "fp64")
    from paper_2105_08798_amd.fbc import STATUS
    assert STATUS[rc] == "FBC_E_NONFINITE"
    assert np.array_equal(got, np.concatenate([x.ravel() for x in u0]))


def test_projection_of_net_force():
    wl = W.make_custom(16, 25, 40, 2, 16, seed=7, zero_net_force=False)
    rc, got, u0 = run_apply(wl, "fp64", project_netforce=True)
    assert rc == 0
    c = wl.cells[0]
    # the projection removes the net force of the whole cell (all atoms of all layers)
    fp = c.forces - c.forces.mean(axis=(1, 2), keepdims=True)
    w = oap.apply_green(oracle_green(c, wl.bz), fp)
    ref, _ = oap.pad_update(u0[0], w, 1.0)
    e2, emax = rel_err(got.reshape(ref.shape), ref)
    assert e2 < 1e-10 and emax < 1e-10


@pytest.mark.parametrize("form,tol", [("fp64", 1e-10), ("dtable_fp64", 1e-10), ("fp32", 1e-6),
                                      ("split_bf16", 2e-5), ("split_fp16", 1e-6)])
def test_layer_net_forces_with_zero_cell_total(form, tol):
    """Single layers may carry net force (as the incompatibility forces of Algorithm 1 do);
    only the cell total enters the gauge.  The reduced forms' row gauge is compensated
    exactly, so their error stays at the rounding level of the stored blocks."""
    wl = W.make_custom(32, 40, 70, 3, 32, seed=12, zero_net_force=False)
    c = wl.cells[0]
    c.forces = c.forces - c.forces.mean(axis=(1, 2), keepdims=True)
    assert np.abs(c.forces.sum(axis=2)).max() > 1e-2          # layers are not balanced
    rc, got, u0 = run_apply(wl, form, alpha=0.9)
    assert rc == 0
    ref = oracle_update(wl, u0, 0.9)[0]
    e2, emax = rel_err(got.reshape(ref.shape), ref)
    assert e2 < tol and emax < 3 * tol, (form, e2, emax)


@pytest.mark.parametrize("form,tol", [("fp32", 1e-6), ("split_bf16", 2e-5), ("split_fp16", 1e-6)])
def test_layer_net_forces_mixed_rhs(form, tol):
    """RHS whose layers are balanced sit beside RHS whose layers are not: the row-gauge
    compensation is switched per RHS (a balanced layer's net force is only rounding
    residue) and must stay on wherever a layer carries net force."""
    wl = W.make_custom(32, 40, 70, 6, 32, seed=13, zero_net_force=False)
    c = wl.cells[0]
    f = c.forces - c.forces.mean(axis=(1, 2), keepdims=True)
    for r in (2, 3, 5):                                       # balanced layers
        f[r] = f[r] - f[r].mean(axis=1, keepdims=True)
    c.forces = np.ascontiguousarray(f)
    for r in (0, 1, 4):
        assert np.abs(f[r].sum(axis=1)).max() > 1e-2
    assert np.abs(f[2].sum(axis=1)).max() < 1e-12
    rc, got, u0 = run_apply(wl, form, alpha=0.7)
    assert rc == 0
    ref = oracle_update(wl, u0, 0.7)[0]
    for r in range(6):
        e2, emax = rel_err(got.reshape(ref.shape)[r:r + 1], ref[r:r + 1])
        assert e2 < tol and emax < 3 * tol, (form, r, e2, emax)


@pytest.mark.parametrize("form,tol", [("fp32", 1e-6), ("split_bf16", 2e-5), ("split_fp16", 1e-6)])
@pytest.mark.parametrize("nz,n_i,n_b,R,bz", [(16, 50, 80, 20, 64), (8, 130, 260, 33, 64), (4, 40, 70, 64, 32)])
def test_reduced_forms_many_rhs(nz, n_i, n_b, R, bz, form, tol):
    """4 and 8 column tiles: the product kernels that share B through LDS."""
    wl = W.make_custom(nz, n_i, n_b, R, bz, seed=nz + R)
    rc, got, u0 = run_apply(wl, form, alpha=1.0)
    assert rc == 0
    ref = oracle_update(wl, u0, 1.0)[0]
    e2, emax = rel_err(got.reshape(ref.shape), ref)
    assert e2 < tol and emax < 3 * tol, (form, e2, emax)


@pytest.mark.parametrize("form", ["fp32", "split_bf16", "split_fp16"])
def test_projection_in_reduced_forms(form):
    wl = W.make_custom(16, 25, 40, 2, 16, seed=8, zero_net_force=False)
    rc, got, u0 = run_apply(wl, form, project_netforce=True)
    assert rc == 0
    c = wl.cells[0]
    fp = c.forces - c.forces.mean(axis=(1, 2), keepdims=True)
    ref, _ = oap.pad_update(u0[0], oap.apply_green(oracle_green(c, wl.bz), fp), 1.0)
    e2, _ = rel_err(got.reshape(ref.shape), ref)
    assert e2 < (2e-5 if form == "split_bf16" else 1e-6), e2


@pytest.mark.parametrize("alpha_min", [0.0, 3.0])
@pytest.mark.parametrize("form", FP64_FORMS)
def test_relax_sequence_matches_oracle(form, alpha_min):
    _relax_sequence_check(W.make_single("parity"), form, alpha_min)


@pytest.mark.parametrize("nz,n_i,n_b,R", [(256, 9, 17, 3), (512, 7, 15, 9), (1024, 9, 13, 5), (1024, 6, 11, 16),
                                          (2048, 5, 9, 2)])
def test_relax_sequence_long_lines(nz, n_i, n_b, R):
    """Relaxation steps on long lines (the inverse transform into w with 1024 threads at 512
    and 1024 layers, 2 rows x 4 RHS pairs per work group): odd pad row counts leave the last
    group half full, and RHS counts off a multiple of 8 leave pairs of the last column tile
    empty; the step bound reads every group's partial maximum."""
    _relax_sequence_check(W.make_custom(nz, n_i, n_b, R, 16, seed=nz + n_b), "fp64", 0.0)


@pytest.mark.parametrize("form,tol", [("split_fp16", 1e-6), ("fp32", 1e-6)])
@pytest.mark.parametrize("nz,n_i,n_b,R", [(1024, 9, 13, 5), (512, 7, 15, 9), (2048, 5, 9, 3)])
def test_relax_sequence_unbalanced_layers_long_lines(nz, n_i, n_b, R, form, tol):
    """Relaxation steps whose residuals carry net force per layer (zero cell total), as the
    incompatibility forces of Algorithm 1 do: the reduced forms add the row-gauge
    compensation in the inverse transform into w.  Without the step bound the relaxation
    factors depend on the residuals alone and match the oracle's to rounding; u and the
    step size match to the form's bound."""
    wl = W.make_custom(nz, n_i, n_b, R, 16, seed=nz + n_b + 1, zero_net_force=False)
    _relax_sequence_check(wl, form, 0.0, du_max=0.0, tol=tol, balanced=False)


@pytest.mark.parametrize("shape", [None, (1024, 9, 13, 5), (512, 7, 15, 9), (16, 30, 45, 11), (2048, 5, 9, 2)])
@pytest.mark.parametrize("form", FP64_FORMS)
def test_relax_sequence_without_step_bound(form, shape):
    """Without the step bound the step factors are known before w: lines of 16-1024 layers
    take the fused inverse transform and update, whose work groups leave the maxima of |w|
    that step_inf reports (2048 layers still go through w)."""
    wl = W.make_single("parity") if shape is None else W.make_custom(*shape, 16, seed=sum(shape))
    _relax_sequence_check(wl, form, 0.0, du_max=0.0)


@pytest.mark.parametrize("du_max", [0.0, 0.05])
def test_relax_multi_cell(du_max):
    """Relaxation steps of a context whose cells take different update paths (16 and 512
    layers: the fused update without the step bound; 2048 layers: through w), each cell's
    RHS with their own relaxation factors: every cell against the oracle's sequence."""
    dev = _dev()
    from paper_2105_08798_amd import RELAX_OUT_DOUBLES, parse_relax_out
    cells = [W.make_custom(16, 30, 45, 3, 32, seed=31).cells[0], W.make_custom(2048, 5, 9, 2, 32, seed=32).cells[0],
             W.make_custom(512, 7, 13, 9, 32, seed=33).cells[0]]
    wl = W.Workload("mixed-relax", cells, bz=32)
    ctx = _ctx(wl.cells, wl.bz, form="fp64")
    rng = np.random.default_rng(17)
    seqs = []
    for c in cells:
        base = c.forces - c.forces.mean(axis=2, keepdims=True)
        seq = [base]
        for k in range(4):
            nxt = 0.6 * seq[-1] + 0.02 * rng.normal(size=base.shape) * (0.5 ** k)
            seq.append(nxt - nxt.mean(axis=2, keepdims=True))
        seqs.append(seq)
    u0 = [rng.normal(size=(c.n_rhs, c.nz, c.n_b, 3)) * 0.01 for c in cells]
    u = torch.from_numpy(np.concatenate([x.ravel() for x in u0])).to(dev)
    greens = [oracle_green(c, wl.bz) for c in cells]
    states = [orx.RelaxState(n_rhs=c.n_rhs, relax=True, du_max=du_max, tol_f=0.2) for c in cells]
    uref = [x.copy() for x in u0]
    ctx.relax_begin(relax=True, du_max=du_max, tol_f=0.2)
    out = torch.zeros(sum(c.n_rhs for c in cells) * RELAX_OUT_DOUBLES, dtype=torch.float64, device=dev)
    for k in range(len(seqs[0])):
        f = np.concatenate([seqs[i][k].ravel() for i in range(len(cells))])
        ctx.relax_step(torch.from_numpy(f).to(dev), u, out)
        assert ctx.sync_status() == 0
        got = parse_relax_out(out)
        r0 = 0
        for i, c in enumerate(cells):
            uref[i], oref = orx.relax_step(states[i], seqs[i][k], uref[i], lambda x, g=greens[i]: oap.apply_green(g, x))
            for r in range(c.n_rhs):
                assert abs(got[r0 + r]["alpha"] - oref["alpha"][r]) <= 1e-10 * abs(oref["alpha"][r]), (k, i, r)
                assert abs(got[r0 + r]["step_inf"] - oref["step_inf"][r]) <= 1e-10 * oref["step_inf"][r], (k, i, r)
            r0 += c.n_rhs
        for i, (g_, r_) in enumerate(zip(split_cells(wl, u.cpu().numpy()), uref)):
            e2, emax = rel_err(g_, r_)
            assert e2 < 1e-10 and emax < 1e-10, (k, i, e2, emax)
    ctx.close()


def _relax_sequence_check(wl, form, alpha_min, du_max=0.05, tol=1e-10, balanced=True):
    c = wl.cells[0]
    dev = _dev()
    from paper_2105_08798_amd import RELAX_OUT_DOUBLES, parse_relax_out
    ctx = _ctx(wl.cells, wl.bz, form=form)
    g = oracle_green(c, wl.bz)
    rng = np.random.default_rng(11)
    # residual sequence with partly contracting, partly rotating directions; balanced
    # layers, or net force per layer with a zero cell total
    axes = 2 if balanced else (1, 2)
    base = c.forces - c.forces.mean(axis=axes, keepdims=True)
    if not balanced:
        assert np.abs(base.sum(axis=2)).max() > 1e-2
    seq = [base]
    for k in range(5):
        nxt = 0.6 * seq[-1] + 0.2 * rng.normal(size=base.shape) * 0.1 * (0.5 ** k)
        nxt -= nxt.mean(axis=axes, keepdims=True)
        seq.append(nxt)
    u0 = rng.normal(size=(c.n_rhs, c.nz, c.n_b, 3)) * 0.01
    u = torch.from_numpy(u0).to(dev)
    st = orx.RelaxState(n_rhs=c.n_rhs, relax=True, du_max=du_max, tol_f=0.2, alpha_min=alpha_min)
    ctx.relax_begin(relax=True, du_max=du_max, tol_f=0.2, alpha_min=alpha_min)
    out = torch.zeros(c.n_rhs * RELAX_OUT_DOUBLES, dtype=torch.float64, device=dev)
    uref = u0.copy()
    for fk in seq:
        ctx.relax_step(torch.from_numpy(fk).to(dev), u, out)
        assert ctx.sync_status() == 0
        uref, oref = orx.relax_step(st, fk, uref, lambda f: oap.apply_green(g, f))
        got = parse_relax_out(out)
        for r in range(c.n_rhs):
            assert abs(got[r]["alpha"] - oref["alpha"][r]) <= 1e-10 * abs(oref["alpha"][r])
            assert abs(got[r]["f_inf"] - oref["f_inf"][r]) <= 1e-15 * oref["f_inf"][r]
            assert abs(got[r]["step_inf"] - oref["step_inf"][r]) <= tol * oref["step_inf"][r]
            assert got[r]["converged"] == bool(oref["converged"][r])
            # the removed mean, against the size of the displacements
            scale = np.abs(uref[r]).max()
            assert np.abs(np.array(got[r]["mean_removed"]) - oref["mean_removed"][r]).max() <= tol * scale
        e2, emax = rel_err(u.cpu().numpy(), uref)
        assert e2 < tol and emax < (1 if tol == 1e-10 else 3) * tol
    ctx.close()


@pytest.mark.parametrize("form,tol", [("split_fp16", 1e-6), ("fp32", 1e-6), ("split_bf16", 2e-5)])
@pytest.mark.parametrize("nz,n_i,n_b,R", [(1024, 9, 13, 9), (512, 7, 15, 5), (256, 12, 21, 16), (2048, 5, 9, 3)])
def test_layer_net_forces_long_lines(nz, n_i, n_b, R, form, tol):
    """Per-layer net force on long lines, RHS with balanced layers beside RHS without: the
    fused update stages the row-gauge compensation of each work group's rows before it
    gathers the product records (1024 threads at 512 and 1024 layers, 256 below); 2048
    layers take the inverse transform into w."""
    wl = W.make_custom(nz, n_i, n_b, R, 16, seed=nz + n_b + 2, zero_net_force=False)
    c = wl.cells[0]
    f = c.forces - c.forces.mean(axis=(1, 2), keepdims=True)
    for r in range(1, R, 3):                                  # balanced layers
        f[r] = f[r] - f[r].mean(axis=1, keepdims=True)
    c.forces = np.ascontiguousarray(f)
    assert np.abs(f[0].sum(axis=1)).max() > 1e-2
    rc, got, u0 = run_apply(wl, form, alpha=0.8)
    assert rc == 0
    ref = oracle_update(wl, u0, 0.8)[0]
    for r in range(R):
        e2, emax = rel_err(got.reshape(ref.shape)[r:r + 1], ref[r:r + 1])
        assert e2 < tol and emax < 3 * tol, (form, r, e2, emax)


@pytest.mark.parametrize("form,bound", [("fp32", 1e-6), ("split_bf16", 2e-5), ("split_fp16", 1e-6)])
def test_reduced_forms_error_bound(form, bound):
    wl = W.make_single("parity")
    c = wl.cells[0]
    dev = _dev()
    ctx = _ctx(wl.cells, wl.bz, form=form)
    f = torch.from_numpy(c.forces).to(dev)
    w = torch.zeros((c.n_rhs, c.nz, c.n_b, 3), dtype=torch.float64, device=dev)
    ctx.green_apply(f, w)
    assert ctx.sync_status() == 0
    ctx.close()
    ref = oap.apply_green(oracle_green(c, wl.bz), c.forces)
    e2, emax = rel_err(w.cpu().numpy(), ref)
    print(f"{form}: rel err {e2:.3e} (max-abs {emax:.3e})")
    assert e2 < bound, (form, e2)


@pytest.mark.parametrize("form,bound", [("fp32", 1e-6), ("split_fp16", 1e-6)])
@pytest.mark.parametrize("R", [3, 10])
def test_rhs_of_very_different_scale(form, bound, R):
    """RHS whose forces differ by many orders of magnitude in one call (a converged
    residual beside one that is not, as in a batched Algorithm 1 loop): every RHS keeps
    its own relative error.  The split-FP16 operand scale is per RHS."""
    _dev()
    wl = W.make_custom(16, 60, 100, R, 32, seed=31)
    c = wl.cells[0]
    scales = np.array([1.0, 1e-4, 1e-8, 1e-2, 1e-6][:R] + [10.0 ** (-k) for k in range(max(0, R - 5))])
    c.forces = np.ascontiguousarray(c.forces * scales[:, None, None, None])
    dev = _dev()
    ctx = _ctx(wl.cells, wl.bz, form=form)
    f = torch.from_numpy(c.forces).to(dev)
    w = torch.zeros((c.n_rhs, c.nz, c.n_b, 3), dtype=torch.float64, device=dev)
    ctx.green_apply(f, w)
    assert ctx.sync_status() == 0
    ctx.close()
    got = w.cpu().numpy()
    ref = oap.apply_green(oracle_green(c, wl.bz), c.forces)
    for r in range(R):
        e2, emax = rel_err(got[r:r + 1], ref[r:r + 1])
        print(f"{form} R={R} rhs {r} scale {scales[r]:.0e}: rel err {e2:.2e}", flush=True)
        assert e2 < bound and emax < 3 * bound, (form, r, scales[r], e2, emax)


def test_repeated_apply_is_bitwise_reproducible():
    wl = W.make_single("parity")
    dev = _dev()
    ctx = _ctx(wl.cells, wl.bz, form="fp64")
    c = wl.cells[0]
    f = torch.from_numpy(c.forces).to(dev)
    outs = []
    for _ in range(3):
        u = torch.zeros((c.n_rhs, c.nz, c.n_b, 3), dtype=torch.float64, device=dev)
        ctx.apply(f, u, alpha=1.0)
        assert ctx.sync_status() == 0
        outs.append(u.cpu().numpy())
    ctx.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


@pytest.mark.parametrize("form", ["fp64", "dtable_fp64"])
def test_graph_replay_matches_eager(form):
    """Captured update replayed several times, with eager work and synchronisation between
    replays; every replay must equal the eager result bitwise (same kernels, same order)."""
    dev = _dev()
    cells = W.make_custom(16, 40, 70, 3, 32, seed=21).cells + W.make_custom(32, 20, 30, 9, 32, seed=22).cells
    wl = W.Workload("two", cells, bz=32)
    ctx = _ctx(wl.cells, wl.bz, form=form)
    f = torch.from_numpy(np.concatenate([c.forces.ravel() for c in wl.cells])).to(dev)
    n_u = sum(c.n_rhs * c.nz * c.n_b * 3 for c in wl.cells)
    u0 = torch.from_numpy(np.random.default_rng(3).normal(size=n_u) * 0.01).to(dev)
    s = torch.cuda.Stream()
    ref = u0.clone()
    ctx.apply(f, ref, alpha=0.9)
    assert ctx.sync_status() == 0
    u = torch.empty_like(u0)
    for rep in range(4):
        with torch.cuda.stream(s):
            u.copy_(u0)
            ctx.apply_graph(f, u, alpha=0.9, stream=s)
        s.synchronize()
        junk = torch.randn(1000, device=dev).sum().item()      # eager work between replays
        assert np.isfinite(junk)
        assert ctx.sync_status(stream=s) == 0
        assert torch.equal(u, ref), rep
    ctx.close()


@pytest.mark.parametrize("form", ["fp64", "dtable_fp64", "split_bf16", "split_fp16"])
def test_autotune_keeps_results(form):
    dev = _dev()
    wl = W.make_single("parity")
    c = wl.cells[0]
    ctx = _ctx(wl.cells, wl.bz, form=form)
    f = torch.from_numpy(c.forces).to(dev)
    w = torch.zeros((c.n_rhs, c.nz, c.n_b, 3), dtype=torch.float64, device=dev)
    res = ctx.autotune(f, w, reps=2)
    assert res["n_candidates"] >= 3 and res["gemm_ms"] > 0
    assert ctx.info.nsplit == res["nsplit"] and ctx.info.job_order == res["order"]
    w.zero_()
    ctx.green_apply(f, w)
    assert ctx.sync_status() == 0
    ref = oap.apply_green(oracle_green(c, wl.bz), c.forces)
    e2, emax = rel_err(w.cpu().numpy(), ref)
    ctx.close()
    assert e2 < {"split_bf16": 2e-5, "split_fp16": 1e-6}.get(form, 1e-10), (form, res, e2)


@pytest.mark.parametrize("form,tol", [("fp64", 1e-14), ("dtable_fp64", 1e-14), ("fp32", 1e-6),
                                      ("split_fp16", 1e-6), ("split_bf16", 2e-5)])
def test_negligible_block_skipping(form, tol):
    """High line modes decay with kappa rho: the product skips the K chunks of a row tile
    whose blocks are all below the skip tolerance.  FP64 forms: identical to the unskipped
    product to rounding; reduced forms: within their tolerance of the oracle."""
    dev = _dev()
    # rings of radius ~17 / ~22: at the upper modes many pad tiles are far from most
    # interface chunks
    wl = W.make_custom(16, 400, 800, 3, 256, seed=31)
    c = wl.cells[0]
    f = torch.from_numpy(c.forces).to(dev)
    out = {}
    for tag, st in (("skip", 0.0), ("full", -1.0)):
        ctx = _ctx(wl.cells, wl.bz, form=form, skip_tol=st)
        w = torch.zeros((c.n_rhs, c.nz, c.n_b, 3), dtype=torch.float64, device=dev)
        ctx.green_apply(f, w)
        assert ctx.sync_status() == 0
        out[tag] = (w.cpu().numpy(), ctx.info.skipped_fraction, ctx.info.product_bytes)
        ctx.close()
    assert out["skip"][1] > 0.05 and out["full"][1] == 0.0, (out["skip"][1], out["full"][1])
    if form in FP64_FORMS:
        e2, emax = rel_err(out["skip"][0], out["full"][0])
        assert e2 < tol and emax < tol, (e2, emax)
    else:
        assert out["skip"][2] < out["full"][2]
    ref = oap.apply_green(oracle_green(c, wl.bz), c.forces)
    e2, _ = rel_err(out["skip"][0], ref)
    assert e2 < max(tol, 1e-10), (form, e2)


@pytest.mark.parametrize("form", ["dtable_fp64", "fp64", "fp32", "split_fp16"])
def test_work_lists_give_identical_results(form):
    """Every order of the work list (incl. the persistent work-queue kernels) partitions
    the same products, so for a given number of K slices
    the update is bit-identical; other slice counts change only the rounding.  The
    persistent kernel's queue is reset for the next launch (repeated calls and graph
    replays agree)."""
    dev = _dev()
    cells = W.make_custom(16, 30, 45, 3, 32, seed=1).cells + W.make_custom(8, 12, 20, 10, 32, seed=2).cells \
        + W.make_custom(32, 50, 60, 1, 32, seed=3).cells
    wl = W.Workload("three", cells, bz=32)
    f = torch.from_numpy(np.concatenate([c.forces.ravel() for c in wl.cells])).to(dev)
    n_u = sum(c.n_rhs * c.nz * c.n_b * 3 for c in wl.cells)
    ctx = _ctx(wl.cells, wl.bz, form=form)
    ref = None
    stream = torch.cuda.Stream()
    for nsplit in (2, 1):
        ref_split = None
        for order in (0, 1, 2, 3, 4):
            ctx.set_work_list(nsplit, order)
            assert ctx.info.nsplit == nsplit and ctx.info.job_order == order
            for rep in range(2):
                w = torch.zeros(n_u, dtype=torch.float64, device=dev)
                ctx.green_apply(f, w)
                assert ctx.sync_status() == 0
                got = w.cpu().numpy()
                if ref_split is None:
                    ref_split = got
                assert np.array_equal(got, ref_split), (nsplit, order, rep)
        if ref is not None:      # other slice counts: rounding only
            tol = 1e-13 if form in FP64_FORMS else 1e-6
            assert np.abs(ref_split - ref).max() <= tol * np.abs(ref).max()
        ref = ref_split
    # persistent lists (one, and one per XCD) replayed from a captured graph, with eager
    # calls in between
    for order in (3, 4):
        ctx.set_work_list(1, order)
        u0 = torch.zeros(n_u, dtype=torch.float64, device=dev)
        u_eager = u0.clone()
        ctx.apply(f, u_eager, alpha=1.0)
        torch.cuda.synchronize()
        u = torch.empty_like(u0)          # one buffer: the first call captures, the rest replay
        for rep in range(3):
            u.copy_(u0)
            torch.cuda.synchronize()
            ctx.apply_graph(f, u, alpha=1.0, stream=stream)
            stream.synchronize()
            assert np.array_equal(u.cpu().numpy(), u_eager.cpu().numpy()), (order, rep)
            w = torch.zeros(n_u, dtype=torch.float64, device=dev)
            ctx.green_apply(f, w)
            assert np.array_equal(w.cpu().numpy(), ref), (order, rep)
    assert ctx.sync_status() == 0
    ctx.close()


def test_work_list_arguments_checked():
    _dev()
    wl = W.make_single("parity")
    from paper_2105_08798_amd.fbc import FbcError
    ctx = _ctx(wl.cells, wl.bz, form="fp64")
    for nsplit, order in ((0, 0), (1, 5), (1, -1), (1 << 20, 0)):
        with pytest.raises(FbcError):
            ctx.set_work_list(nsplit, order)
    ctx.close()


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_relax_checkpoint_resume_is_bitwise(form):
    # checkpoint after three steps, resume in a fresh context of the same cells (same
    # default work list), continue: every later step equals the uninterrupted run bit for bit
    wl = W.make_single("parity")
    c = wl.cells[0]
    dev = _dev()
    from paper_2105_08798_amd import RELAX_OUT_DOUBLES, FbcError
    rng = np.random.default_rng(21)
    seq = [c.forces]
    for k in range(5):
        nxt = 0.6 * seq[-1] + 0.02 * rng.normal(size=c.forces.shape) * (0.5 ** k)
        nxt -= nxt.mean(axis=2, keepdims=True)
        seq.append(nxt)
    u0 = torch.from_numpy(rng.normal(size=(c.n_rhs, c.nz, c.n_b, 3)) * 0.01).to(dev)
    opts = dict(relax=True, du_max=0.05, tol_f=0.2, alpha_min=0.0)

    def run(ctx, u, steps):
        outs = []
        for fk in steps:
            out = torch.zeros(c.n_rhs * RELAX_OUT_DOUBLES, dtype=torch.float64, device=dev)
            ctx.relax_step(torch.from_numpy(fk).to(dev), u, out)
            assert ctx.sync_status() == 0
            outs.append(out.cpu().numpy())
        return outs

    a = _ctx(wl.cells, wl.bz, form=form)
    a.relax_begin(**opts)
    ua = u0.clone()
    ref_out = run(a, ua, seq)
    a.close()

    b = _ctx(wl.cells, wl.bz, form=form)
    with pytest.raises(FbcError):
        b.relax_state()                          # no iteration yet
    b.relax_begin(**opts)
    ub = u0.clone()
    run(b, ub, seq[:3])
    state = b.relax_state()
    u_ckpt = ub.cpu()
    b.close()
    assert state["k"] == 3 and state["relax"] and state["du_max"] == 0.05
    assert np.array_equal(state["f_prev"].cpu().numpy(), seq[2].reshape(-1))

    r = _ctx(wl.cells, wl.bz, form=form)
    for bad in (dict(state, k=-1), dict(state, du_max=-1.0), dict(state, f_prev=None)):
        with pytest.raises((FbcError, TypeError)):
            r.set_relax_state(bad)
    r.set_relax_state(state)
    ur = u_ckpt.to(dev)
    got_out = run(r, ur, seq[3:])
    r.close()
    for g, e in zip(got_out, ref_out[3:]):
        assert np.array_equal(g, e)
    assert torch.equal(ur, ua)


@pytest.mark.parametrize("du_max", [0.05, 0.0])
@pytest.mark.parametrize("form", ["fp64", "split_fp16"])
def test_relax_step_graph_matches_eager(form, du_max):
    """Algorithm 1's update with Algorithm 2 replayed from a captured graph: the iteration
    index lives in device memory, so every replay takes the current k (relaxation from the
    third step on); each step equals the eager step bit for bit, with eager work between
    the replays, and the checkpointed index counts the replays."""
    wl = W.make_single("parity")
    c = wl.cells[0]
    dev = _dev()
    from paper_2105_08798_amd import RELAX_OUT_DOUBLES
    rng = np.random.default_rng(5)
    seq = [c.forces]
    for k in range(6):
        nxt = 0.5 * seq[-1] + 0.02 * rng.normal(size=c.forces.shape) * (0.5 ** k)
        nxt -= nxt.mean(axis=2, keepdims=True)
        seq.append(nxt)
    u0 = torch.from_numpy(rng.normal(size=(c.n_rhs, c.nz, c.n_b, 3)) * 0.01).to(dev)
    opts = dict(relax=True, du_max=du_max, tol_f=0.2, alpha_min=0.0)
    a = _ctx(wl.cells, wl.bz, form=form)
    g = _ctx(wl.cells, wl.bz, form=form)
    a.relax_begin(**opts)
    g.relax_begin(**opts)
    ua, ug = u0.clone(), u0.clone()
    fbuf = torch.empty(c.forces.size, dtype=torch.float64, device=dev)
    out_a = torch.zeros(c.n_rhs * RELAX_OUT_DOUBLES, dtype=torch.float64, device=dev)
    out_g = torch.zeros_like(out_a)
    stream = torch.cuda.Stream()
    alphas = []
    for k, fk in enumerate(seq):
        fdev = torch.from_numpy(fk.reshape(-1)).to(dev)
        a.relax_step(fdev, ua, out_a)
        fbuf.copy_(fdev)                          # the captured step reads this buffer
        torch.cuda.synchronize()
        g.relax_step_graph(fbuf, ug, out_g, stream=stream)
        stream.synchronize()
        assert a.sync_status() == 0 and g.sync_status() == 0
        assert torch.equal(ug, ua), k
        assert torch.equal(out_g, out_a), k
        from paper_2105_08798_amd import parse_relax_out
        o = parse_relax_out(out_g)
        assert all(r["k"] == k for r in o), (k, o)
        alphas.append([r["alpha"] for r in o])
    # relaxation takes over at k = 2 (the third step): alpha moves off 1
    assert all(x == 1.0 for x in alphas[0] + alphas[1])
    assert any(x != 1.0 for x in sum(alphas[2:], []))
    assert g.relax_state()["k"] == len(seq)
    a.close()
    g.close()


@pytest.mark.parametrize("form", ["fp64", "fp32", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("R", [3, 12, 20, 64])
def test_kernel_variants_are_bitwise_equal(form, R):
    """Every product kernel variant the autotuner may choose (ring depth, K steps per
    barrier) for each column-tile class gives bitwise the result of the default, which
    matches the oracle at the form's bound."""
    dev = _dev()
    wl = W.make_custom(8, 70, 110, R, 32, seed=R + 3)
    c = wl.cells[0]
    ctx = _ctx(wl.cells, wl.bz, form=form)
    f = torch.from_numpy(c.forces).to(dev)
    outs = []
    for v in range(ctx.info.n_variants):
        ctx.set_kernel_variant(v)
        assert ctx.info.kernel_variant == v and ctx.info.kernel_shape
        w = torch.zeros((c.n_rhs, c.nz, c.n_b, 3), dtype=torch.float64, device=dev)
        ctx.green_apply(f, w)
        assert ctx.sync_status() == 0
        outs.append(w.cpu().numpy())
        print(form, R, v, ctx.info.kernel_shape.decode(), flush=True)
    from paper_2105_08798_amd.fbc import FbcError
    with pytest.raises(FbcError):
        ctx.set_kernel_variant(ctx.info.n_variants)
    ctx.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    ref = oap.apply_green(oracle_green(c, wl.bz), c.forces)
    bound = {"fp64": 1e-10, "fp32": 1e-6, "split_bf16": 2e-5, "split_fp16": 1e-6}[form]
    e2, _ = rel_err(outs[0], ref)
    assert e2 < bound, (form, R, e2)


def test_autotune_cache_file(tmp_path):
    """The tuned choice is written to the cache file and applied untimed to a new context
    of the same configuration (bitwise the same result); other configurations miss."""
    dev = _dev()
    wl = W.make_custom(16, 60, 100, 9, 32, seed=4)
    c = wl.cells[0]
    path = str(tmp_path / "tune.txt")
    f = torch.from_numpy(c.forces).to(dev)
    w = torch.zeros((c.n_rhs, c.nz, c.n_b, 3), dtype=torch.float64, device=dev)
    a = _ctx(wl.cells, wl.bz, form="fp32")
    ra = a.autotune(f, w, reps=1, cache=path)
    assert not ra["from_cache"] and ra["n_candidates"] > 1
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("fbc-tune ")
    wa = torch.zeros_like(w)
    a.green_apply(f, wa)
    b = _ctx(wl.cells, wl.bz, form="fp32")
    rb = b.autotune(f, w, reps=1, cache=path)
    assert rb["from_cache"] and (rb["variant"], rb["nsplit"], rb["order"]) == (ra["variant"], ra["nsplit"], ra["order"])
    assert (b.info.kernel_variant, b.info.nsplit, b.info.job_order) == (ra["variant"], ra["nsplit"], ra["order"])
    wb = torch.zeros_like(w)
    b.green_apply(f, wb)
    assert a.sync_status() == 0 and b.sync_status() == 0
    assert torch.equal(wa, wb)
    # another form is another key: tuned and appended
    d = _ctx(wl.cells, wl.bz, form="fp64")
    rd = d.autotune(f, w, reps=1, cache=path)
    assert not rd["from_cache"] and len(open(path).read().splitlines()) == 2
    for x in (a, b, d):
        x.close()


@pytest.mark.parametrize("form", ["fp64", "split_fp16"])
def test_graph_replay_long_lines(form):
    """Lines of 1024 layers (the forward transform and the fused update on 1024-thread work
    groups with more than 64 KiB of LDS): a captured update replays bitwise like the eager
    one, also when the context's first call is the captured one."""
    dev = _dev()
    wl = W.make_custom(1024, 30, 70, 9, 16, seed=5)
    c = wl.cells[0]
    f = torch.from_numpy(c.forces).to(dev)
    u0 = torch.from_numpy(np.random.default_rng(4).normal(size=c.n_rhs * c.nz * c.n_b * 3) * 0.01).to(dev)
    s = torch.cuda.Stream()
    ctx = _ctx(wl.cells, wl.bz, form=form)
    u = torch.empty_like(u0)
    outs = []
    for rep in range(3):
        with torch.cuda.stream(s):
            u.copy_(u0)
            ctx.apply_graph(f, u, alpha=0.7, stream=s)
        s.synchronize()
        assert ctx.sync_status(stream=s) == 0
        outs.append(u.clone())
    ref = u0.clone()
    ctx.apply(f, ref, alpha=0.7)
    assert ctx.sync_status() == 0
    ctx.close()
    for rep, o in enumerate(outs):
        assert torch.equal(o, ref), rep
    if form == "fp64":
        exp = oracle_update(wl, [u0.cpu().numpy().reshape(c.n_rhs, c.nz, c.n_b, 3)], 0.7)[0]
        e2, emax = rel_err(ref.cpu().numpy().reshape(exp.shape), exp)
        assert e2 < 1e-10 and emax < 1e-10, (e2, emax)
