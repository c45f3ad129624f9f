#!/usr/bin/env python
"""Throughput of the line-periodic FBC pad update on one MI355X.

One step = one fbc_apply call: for every RHS of the cell, u <- u - G^{p|i+} f followed
by mean removal (net-force check, line rFFT, per-mode products, inverse rFFT, update,
mean), with f and u resident in HBM.  Prints one JSON line.

Default run (no flags): the headline on the long workload (N_z = 1024, n_i = 4096,
n_b = 8192, 16 RHS: the largest configuration, where the dense blocks would take 2.49 TB;
plain FP64 is the offset-table form there), with the forms FP64 offset table, FP32,
split FP16, split BF16 and the learned far field; the same line carries the large
workload (N_z = 256, n_i = 2048, n_b = 4096, 64 RHS: the precision form's configuration)
with the forms FP64, FP32, split BF16 and split FP16.

    python bench.py [--steps K] [--warmup W] [--workload long|large|medium|batched|plgf|hmat] [--forms ...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FBC boundary updates/sec + % MFMA/HBM roofline vs FP64 plain at 1e-6 rel err"
HBM_PEAK_GBS = 8000.0
# dense MFMA peak of the arithmetic each product runs on (TFLOP/s; the split forms run
# three BF16 / FP16 products per algorithmic one)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "split_bf16": 2500.0, "split_fp16": 2500.0, "dtable_fp64": 78.6,
               "surrogate": 78.6, "surrogate_fp32": 157.3}
MFMA_PER_ALG = {"split_bf16": 3.0, "split_fp16": 3.0}
F_BYTES = {"fp64": 16, "fp32": 8, "split_bf16": 8, "split_fp16": 8, "dtable_fp64": 16, "surrogate": 16,
           "surrogate_fp32": 16}
DTYPE = {"fp64": "f64", "fp32": "f32", "split_bf16": "bf16 hi+lo (fp32 acc)",
         "split_fp16": "fp16 hi+lo, power-of-two scaled (fp32 acc)", "dtable_fp64": "f64",
         "surrogate": "f64 (generated table; bf16 MLP on MFMA, fp32 acc)",
         "surrogate_fp32": "f32 MFMA on the generated f64 table, f64 across chunks and at modes without skipped "
                           "blocks (bf16 MLP on MFMA)"}
FP64_FORMS = ("fp64", "dtable_fp64")
DEFAULT_FORMS = {"long": ["dtable_fp64", "fp32", "split_fp16", "split_bf16", "surrogate", "surrogate_fp32"],
                 "large": ["fp64", "fp32", "split_bf16", "split_fp16"],
                 "medium": ["fp64", "fp32", "split_bf16", "split_fp16", "surrogate"],
                 "batched": ["dtable_fp64"]}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def io_bytes(cells, form: str) -> dict:
    """Bytes of the caller's arrays (f read, u read and written) and of the product's
    intermediate operands (f^ in, w^ out: R (3 n_i) and R (3 n_b) complex per mode)."""
    fu = fh = 0.0
    for c in cells:
        nm = c.nz // 2 + 1
        fu += c.n_rhs * c.nz * 3 * c.n_i * 8 + 2 * c.n_rhs * c.nz * 3 * c.n_b * 8
        fh += nm * c.n_rhs * (3 * c.n_i * F_BYTES[form] + 3 * c.n_b * 16)
    return dict(fu=fu, fhat_what=fh)


def kernel_matches(form: str, name: str) -> bool:
    """Whether a profiled kernel name is the product kernel of a form (either launch form:
    one work group per job, or the persistent work-queue kernel `..._pq`)."""
    name = name.replace("_pq<", "<")
    if form == "fp64":
        return name.startswith("k_gemm_f64<")
    if form == "fp32":
        return name.startswith("k_gemm_f32<")
    if form == "split_bf16":
        return name.startswith("k_gemm_split") and "bf16" in name
    if form == "split_fp16":
        return name.startswith("k_gemm_split") and "f16x8" in name
    return name.startswith("k_gemm_dtab<")


def measured_traffic(workload: str, form: str, product_bytes: float, tuned: dict | None):
    """HBM bytes per product launch from the committed counter runs, or None when they
    were taken on another workload, before the product kernels last changed, on a product
    of other algorithmic bytes (another set of kept blocks) or with another kernel variant
    or work list than the autotuner chose in this run."""
    import hashlib
    p = os.path.join(ROOT, "profiles", f"gemm_traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    t = json.load(open(p))
    src = open(os.path.join(ROOT, "paper_2105_08798_amd", "csrc", "gemm.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest() != t.get("gemm_source_sha256"):
        return None
    for name, v in t["kernels"].items():
        if not (kernel_matches(form, name) and v.get("form", form) == form):
            continue
        run = v.get("launch")
        if tuned is None or run is None or any(run.get(k) != tuned.get(k) for k in ("variant", "nsplit", "order")):
            continue
        return v["traffic_bytes"] if v.get("algorithmic_bytes") == product_bytes else None
    return None


_TRAINED = {}


def train_surrogate(torch, wl, steps: int, seed: int = 0, r_c: float = 6.0, s_exact: float = 12.0,
                    s_learn: float = 20.0, keep_net: bool = False):
    """Far-field object with a trained MLP.  Training data: lattice values of an offset-table
    context of a ring of 1280 interface / 2560 pad columns -- a geometry none of the
    workloads uses, so the timed cell's offsets are held out -- on the workload's line grid
    and in-plane torus; training runs on the library's own kernels.  The held-out error is
    the network's relative error on samples of the same table drawn with another seed."""
    import math
    import fbc_workloads as W
    from paper_2105_08798_amd import FBC, MLP, Surrogate
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    nz = max(c.nz for c in wl.cells)
    src = W.make_custom(nz, 1280, 2560, 1, wl.bz, seed=seed + 77)
    tab = FBC(src.cells, src.bz, form="dtable_fp64")
    sur = Surrogate(r_c=r_c)
    sur.set_exact_range(s_exact)
    sur.set_learn_range(s_learn)
    x, t = sur.training_set(tab, 1 << 19, seed=seed)
    xh, th = sur.training_set(tab, 1 << 13, seed=seed + 1000)     # one batch (max_batch rows)
    tab.close()
    del tab
    torch.cuda.empty_cache()
    t_data = time.perf_counter() - t0
    batch = 8192
    net = MLP(max_batch=batch, seed=seed + 1)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    n = x.shape[0]
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    t1 = time.perf_counter()
    for s in range(steps):
        idx = torch.randint(0, n, (batch,), device=dev, generator=g)
        lr = 2e-3 * 0.5 * (1 + math.cos(math.pi * s / steps)) + 1e-5
        net.loss_grad(x[idx].contiguous(), t[idx].contiguous(), loss)
        net.adam_step(lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    sur.set_mlp(net)
    yh = torch.empty_like(th)
    net.forward(xh, yh)
    torch.cuda.synchronize()
    held = float((torch.linalg.norm(yh - th) / torch.linalg.norm(th)).item())
    info = dict(samples=int(n), steps=steps, batch=batch, final_batch_loss=float(loss.item()),
                heldout_rel_err=held, r_c=r_c, s_exact=s_exact, s_learn=s_learn,
                data_s=t_data, train_s=t_train, source=f"offset table, {src.description}, M={src.bz}")
    log(f"surrogate: {n} samples in {t_data:.1f} s, {steps} Adam steps in {t_train:.1f} s, "
        f"last batch loss {info['final_batch_loss']:.3e}, held-out relative error {held:.3e}")
    if keep_net:
        return sur, info, net
    net.close()
    return sur, info


def golden(name: str):
    """Stored oracle samples of a workload: ('cols', npz) -- w at pad columns, every layer --
    or ('modes', npz) -- the line spectrum at sampled modes and pad columns -- or None."""
    for kind in ("samples", "modes"):
        p = os.path.join(ROOT, "tests", "golden", f"{name}_{kind}.npz")
        if os.path.exists(p):
            return ("cols" if kind == "samples" else "modes"), np.load(p)
    return None


def unbalanced_forces(c, seed: int = 5) -> np.ndarray:
    """The relaxation loop's incompatibility forces carry net force per layer (their cell
    total vanishes): the workload's forces plus a per-layer constant whose sum over the
    layers is zero."""
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, 0.05, size=(c.n_rhs, c.nz, 1, 3))
    v -= v.mean(axis=1, keepdims=True)
    return np.ascontiguousarray(c.forces + v)


def time_form(torch, wl, form: str, steps: int, warmup: int, graph: bool, tune: bool, keep_cols,
              train_steps: int = 20000, extras: bool = False,
              tune_cache: str | None = None, work_list: str | None = None,
              skip_tol: float = 0.0, gen_modes: int = 0) -> tuple[dict, np.ndarray | None]:
    """Times `steps` fbc_apply calls after `warmup`; returns the timings and the raw response
    w = G f at the pad columns keep_cols (every layer; one-cell workloads) or in full."""
    from paper_2105_08798_amd import FBC, RELAX_OUT_DOUBLES
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream() if graph else None
    sur = sur_info = None
    # surrogate_fp32: the learned form with its table products on FP32 MFMA (table_fp32)
    lib_form = "surrogate" if form.startswith("surrogate") else form
    if lib_form == "surrogate":
        key = (wl.description, train_steps)
        if key not in _TRAINED:            # one network per workload serves both learned forms
            _TRAINED[key] = train_surrogate(torch, wl, train_steps)
        sur, sur_info = _TRAINED[key]
    t0 = time.perf_counter()
    ctx = FBC(wl.cells, wl.bz, form=lib_form, surrogate=sur, skip_tol=skip_tol, gen_modes=gen_modes,
              table_fp32=form == "surrogate_fp32")
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    log(f"{form}: assembled in {t_asm:.2f} s (store {ctx.info.store_bytes / 1e9:.2f} GB, "
        f"{ctx.info.n_jobs} product work groups, {ctx.info.nsplit} K slices)")
    f = torch.from_numpy(np.concatenate([c.forces.ravel() for c in wl.cells])).to(dev)
    n_u = sum(c.n_rhs * c.nz * c.n_b * 3 for c in wl.cells)
    u = torch.zeros(n_u, dtype=torch.float64, device=dev)
    tuned = None
    if work_list and lib_form != "surrogate":
        var, nsplit, order = (int(x) for x in work_list.split(":"))
        ctx.set_kernel_variant(var)
        ctx.set_work_list(nsplit, order)
        tuned = dict(nsplit=nsplit, order=order, variant=var, forced=True, shape=ctx.info.kernel_shape.decode())
        log(f"{form}: work list set to {tuned}")
    elif tune:
        w = torch.zeros_like(u)
        tuned = ctx.autotune(f, w, reps=3, cache=tune_cache)
        del w
        log(f"{form}: autotuned work list {tuned}")
    ctx.timing(True)

    def step(ff=f):
        if graph:
            ctx.apply_graph(ff, u, alpha=1.0, stream=stream)
        else:
            ctx.apply(ff, u, alpha=1.0)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_read()
    rc = ctx.sync_status(stream=stream)
    if rc != 0:
        raise RuntimeError(f"{form}: status {rc} after warm-up")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gemm_ms, n_gemm = ctx.timing_read()
    if graph or n_gemm == 0:
        # launches inside a replayed graph carry no events: time the product eagerly
        for _ in range(min(steps, 20)):
            ctx.apply(f, u, alpha=1.0)
        gemm_ms, n_gemm = ctx.timing_read()
    ctx.timing(False)
    extra = {}
    if extras and len(wl.cells) == 1 and not graph:
        # the relaxation loop's forces (net force per layer, zero cell total): the update
        # adds the exact row-gauge compensation; and one fbc_relax_step per iteration
        c = wl.cells[0]
        fu = torch.from_numpy(unbalanced_forces(c)).to(dev)
        for _ in range(2):
            step(fu)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(fu)
        torch.cuda.synchronize()
        extra["unbalanced_ms_per_step"] = 1000.0 * (time.perf_counter() - t0) / steps
        out = torch.zeros(c.n_rhs * RELAX_OUT_DOUBLES, dtype=torch.float64, device=dev)
        ctx.relax_begin(relax=True, du_max=0.0, tol_f=1e-12)
        for _ in range(3):
            ctx.relax_step(fu, u, out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.relax_step(fu, u, out)
        torch.cuda.synchronize()
        extra["relax_step_ms"] = 1000.0 * (time.perf_counter() - t0) / steps
        del fu, out
        log(f"{form}: unbalanced forces {extra['unbalanced_ms_per_step']:.3f} ms/step, "
            f"relax step {extra['relax_step_ms']:.3f} ms")
    store_bytes = ctx.info.store_bytes
    prod = dict(bytes=ctx.info.product_bytes, flops=ctx.info.product_flops,
                skipped_fraction=ctx.info.skipped_fraction)
    rc = ctx.sync_status(stream=stream)
    if rc != 0:
        raise RuntimeError(f"{form}: status {rc} after the timed region")
    w = torch.zeros_like(u)
    ctx.green_apply(f, w)
    torch.cuda.synchronize()
    if keep_cols is not None and len(wl.cells) == 1:
        c = wl.cells[0]
        idx = torch.from_numpy(np.asarray(keep_cols)).to(dev)
        w_keep = w.view(c.n_rhs, c.nz, c.n_b, 3)[:, :, idx, :].cpu().numpy()
    else:
        w_keep = w.cpu().numpy()
    ctx.close()                      # a trained surrogate stays for the workload's other learned form
    del ctx, u, w, f
    torch.cuda.empty_cache()
    ms = 1000.0 * dt / steps
    total_rhs = sum(c.n_rhs for c in wl.cells)
    out = dict(ms_per_step=ms, updates_per_s=total_rhs / (ms / 1000.0), assembly_s=t_asm,
               store_bytes=int(store_bytes), autotune=tuned,
               gemm_ms=(gemm_ms / n_gemm) if n_gemm else None, gemm_launches_timed=n_gemm,
               graph=bool(graph), surrogate_training=sur_info, product=prod, **extra)
    log(f"{form}: {ms:.3f} ms/step, GEMM {out['gemm_ms']} ms, {out['updates_per_s']:.1f} updates/s")
    return out, w_keep


def rel_err(got: np.ndarray, ref: np.ndarray) -> float:
    """max over RHS of ||got - ref||_2 / ||ref||_2"""
    n = ref.shape[0]
    g = got.reshape(n, -1)
    r = ref.reshape(n, -1)
    return float((np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)).max())


def oracle_error(kind: str, gold, w_cols: np.ndarray) -> float:
    """Error of the GPU response at the golden columns against the oracle: relative per RHS
    over every sampled value (w itself, or its line spectrum at the sampled modes)."""
    if kind == "cols":
        return rel_err(w_cols, gold["w"])
    spec = np.fft.rfft(w_cols, axis=1)[:, gold["modes"]]
    return rel_err(spec, gold["what"])


def cpu_baseline(wl, name: str) -> dict:
    """The FP64 oracle (NumPy pocketfft and BLAS) timed on a bounded sample of the same
    workload: one line mode's product (all pad rows, all RHS; its blocks assembled
    untimed) and the line transforms and update of one RHS, each the median of 5 runs after
    a warm-up, scaled to the whole call (products x modes, transforms x RHS).  Also with
    BLAS on one thread (product on one eighth of the rows, median of 3 after a warm-up)."""
    from oracle import apply as oap, green as ogr
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count()
    c = wl.cells[0]
    nm = c.nz // 2 + 1
    m = nm // 3
    t0 = time.perf_counter()
    gm = ogr.dense_mode_matrix(ogr.gather_blocks(ogr.line_mode_green(c.nz, wl.bz, wl.bz, m), c.cols_b, c.cols_i))
    t_asm = time.perf_counter() - t0
    x = np.ascontiguousarray(oap.line_rfft(c.forces[:, :, :, :])[:, m].reshape(c.n_rhs, 3 * c.n_i).T)

    def med(fn, reps):
        fn()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    t_prod = med(lambda: gm @ x, 5)
    f1 = c.forces[:1]
    u1 = np.zeros((1, c.nz, c.n_b, 3))
    wh1 = np.ones((1, nm, c.n_b, 3), dtype=np.complex128)

    def transforms():
        oap.line_rfft(f1)
        oap.pad_update(u1, oap.line_irfft(wh1, c.nz), 1.0)

    t_tr = med(transforms, 5)
    t_call = t_prod * nm + t_tr * c.n_rhs
    out = dict(value=c.n_rhs / t_call, unit="FBC updates/s", cores=int(cores), kind="oracle",
               sample=f"{name}: line mode {m} of {nm} (its blocks assembled untimed in {t_asm:.1f} s), product "
                      f"of all {3 * c.n_b} rows x {c.n_rhs} RHS, median of 5 after a warm-up, x {nm} modes; "
                      f"line transforms + update of 1 RHS, median of 5, x {c.n_rhs} RHS; call {t_call:.2f} s",
               cpu=_cpu_model())
    if threadpool_limits is not None:
        rows = max(1, gm.shape[0] // 8)
        gs = np.ascontiguousarray(gm[:rows])
        with threadpool_limits(limits=1):
            t1 = med(lambda: gs @ x, 3) * gm.shape[0] / rows
        t_call1 = t1 * nm + t_tr * c.n_rhs
        out["value_1thread"] = c.n_rhs / t_call1
        out["sample_1thread"] = f"product of {rows} of {gm.shape[0]} rows on one BLAS thread, median of 3, scaled"
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def roofline_of(form: str, r: dict) -> dict:
    """Roofline of the product kernel of one form: algorithmic bytes (the stored blocks it
    does not skip, f^ and w^) or flops (8 per complex multiply-add of those blocks) per
    launch over its average launch time, against the roof its arithmetic intensity puts it
    under."""
    gm = r["gemm_ms"]
    b, fl = r["product"]["bytes"], r["product"]["flops"]
    gbs = b / (gm * 1e-3) / 1e9
    tfs = fl / (gm * 1e-3) / 1e12
    peak = PEAK_TFLOPS[form]
    mfma_bound = fl * MFMA_PER_ALG.get(form, 1.0) / b > peak * 1e3 / HBM_PEAK_GBS
    if mfma_bound:
        return dict(bound="mfma", achieved=tfs, peak=peak, unit="TFLOP/s", frac=tfs / peak,
                    flops_per_launch=fl, bytes_per_launch=b)
    return dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS,
                bytes_per_launch=b, flops_per_launch=fl)


def run_workload(torch, args, name: str, forms: list, extras_for=None) -> dict:
    """Every form of one workload; errors against the oracle's stored samples (and against
    the workload's FP64 form at the same columns)."""
    import fbc_workloads as W
    wl = W.make_batched() if name == "batched" else W.make_single(name)
    log(f"workload {name}: {wl.description}, M={wl.bz}")
    g = golden(name) if len(wl.cells) == 1 else None
    keep = g[1]["cols"] if g else None
    if g is not None:
        import hashlib
        dg = hashlib.sha256(np.ascontiguousarray(wl.cells[0].forces).tobytes()).hexdigest()
        if str(g[1]["digest"]) != dg:
            log(f"{name}: stored oracle samples do not match the seeded forces; ignored")
            g, keep = None, None
    res = {}
    for form in forms:
        r, w = time_form(torch, wl, form, args.steps, args.warmup, args.graph,
                         not args.no_autotune and not form.startswith("surrogate"), keep, args.train_steps,
                         extras=(form == extras_for), tune_cache=args.tune_cache, work_list=args.work_list,
                         skip_tol=args.skip_tol, gen_modes=args.gen_modes)
        r["w"] = w
        res[form] = r
    ref_form = next((f for f in FP64_FORMS if f in res), None)
    out_forms = {}
    for form, r in res.items():
        io = io_bytes(wl.cells, form)
        e_fp64 = None
        if ref_form is not None:
            e_fp64 = 0.0 if form == ref_form else rel_err(r["w"], res[ref_form]["w"]) \
                if len(wl.cells) == 1 else None
        e_or = oracle_error(g[0], g[1], r["w"]) if g is not None else None
        roof = roofline_of(form, r) if r["gemm_ms"] else None
        g_kept = r["product"]["bytes"] - io["fhat_what"] if form not in ("dtable_fp64", "surrogate",
                                                                            "surrogate_fp32") else None
        out_forms[form] = dict(
            updates_per_s=r["updates_per_s"], ms_per_step=r["ms_per_step"], gemm_ms=r["gemm_ms"],
            roofline=roof, rel_err_vs_oracle=e_or, oracle_samples=(g[0] if g else None),
            rel_err_vs_fp64_gpu=e_fp64, rel_err_reference=ref_form,
            call_GBs=((g_kept + io["fu"]) / (r["ms_per_step"] * 1e-3) / 1e9) if g_kept is not None else None,
            assembly_s=r["assembly_s"], graph=r["graph"], store_GB=r["store_bytes"] / 1e9,
            autotune=r["autotune"], surrogate_training=r["surrogate_training"],
            skipped_fraction=r["product"]["skipped_fraction"], product_bytes=r["product"]["bytes"],
            product_flops=r["product"]["flops"],
            **{k: r[k] for k in ("unbalanced_ms_per_step", "relax_step_ms") if k in r})
        if roof:
            log(f"{name}/{form}: {r['updates_per_s']:.1f} updates/s, product {roof['achieved']:.1f} {roof['unit']} "
                f"({roof['frac']:.2f} of {roof['bound']}), err vs oracle {e_or}")

    def err_of(f):
        e = out_forms[f]["rel_err_vs_oracle"]
        return out_forms[f]["rel_err_vs_fp64_gpu"] if e is None else e

    ok = [f for f in out_forms if err_of(f) is not None and err_of(f) <= 1e-6] or \
         [f for f in out_forms if f in FP64_FORMS]
    head = max(ok, key=lambda f: out_forms[f]["updates_per_s"]) if ok else forms[0]
    for sur, _ in _TRAINED.values():
        sur.close()
    _TRAINED.clear()
    return dict(wl=wl, forms=out_forms, head=head, err_of=err_of, ref_form=ref_form)


# Real-space periodic Green function (fbc_plgf_eval): algorithmic FP64 flops of one
# continuum evaluation (64 circle nodes x 69 flops: node vector 9, acoustic tensor 24,
# symmetric inverse 30, accumulation 6; wave sum 36; set-up 48) and of one image term.
PLGF_FLOPS_KELVIN = 64 * 69 + 36 + 48
PLGF_FLOPS_IMAGE = 12
FP64_VECTOR_PEAK = 78.6


def bench_plgf(args, torch) -> dict:
    """Line-periodic Green function at every (column offset, layer offset) of the medium
    cell: 70,666 distinct offsets x 128 layers, paper parameters (r_cut = 5 a, six images,
    N = 5)."""
    import fbc_workloads as W
    from paper_2105_08798_amd import PeriodicGreen
    wl = W.make_single("medium")
    c = wl.cells[0]
    nz = c.nz
    d12 = np.unique((c.cols_b[:, None, :].astype(np.int64) - c.cols_i[None, :, :]).reshape(-1, 2), axis=0)
    disp = np.empty((len(d12) * nz, 3), dtype=np.int32)
    disp[:, 0] = np.tile(np.arange(nz), len(d12))
    disp[:, 1:] = np.repeat(d12, nz, axis=0)
    n_rich, order = 1, 5
    K = n_rich + order
    # continuum evaluations per call: images outside r_cut (4|B n|^2 > 100), integer test
    n_cgf = 0
    for i in range(-K, K + 1):
        a = disp[:, 0].astype(np.int64) + i * nz + disp[:, 1] + disp[:, 2]
        b = disp[:, 2].astype(np.int64) - disp[:, 0] - i * nz
        n_cgf += int(((a * a + b * b + disp[:, 1].astype(np.int64) ** 2) > 100).sum())
    origin_cgf = sum(1 for i in range(-K, K + 1) if 2 * (i * nz) ** 2 > 100)
    flops = (n_cgf + origin_cgf) * PLGF_FLOPS_KELVIN + disp.shape[0] * (2 * K + 1) * PLGF_FLOPS_IMAGE
    t0 = time.perf_counter()
    pg = PeriodicGreen(torus_l=64, r2x4_cut=100, r2x4_match=144, n_psi=64)
    torch.cuda.synchronize()
    t_table = time.perf_counter() - t0
    d = torch.from_numpy(disp).cuda()
    out = torch.empty((disp.shape[0], 6), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    for _ in range(args.warmup):
        pg.eval(d, out, nz, n_rich, order)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(args.steps):
        pg.eval(d, out, nz, n_rich, order)
    e1.record(st)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ev_ms = e0.elapsed_time(e1) / args.steps
    # parity on a seeded sample against the oracle
    from oracle import plgf as oplgf
    rng = np.random.default_rng(0)
    idx = rng.choice(disp.shape[0], 256, replace=False)
    ora = oplgf.InfiniteLatticeGreen(64, 100, 144, n_psi=64)
    ref = oplgf.periodic_green(ora, disp[idx].astype(np.int64), nz, n_rich, order)
    ref6 = np.stack([ref[:, i, j] for i, j in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))], axis=-1)
    got = out.cpu().numpy()[idx]
    err = float(np.abs(got - ref6).max() / np.abs(ref6).max())
    log(f"plgf: table {t_table:.2f} s, {disp.shape[0]} entries, {dt * 1e3:.3f} ms/call "
        f"({ev_ms:.3f} ms by events), {flops / (ev_ms * 1e-3) / 1e12:.1f} TFLOP/s, err {err:.1e}")
    line = {
        "metric": "line-periodic lattice Green blocks/s (real-space construction, Section 3.1)",
        "value": disp.shape[0] / dt, "unit": "3x3 blocks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"plgf: every (column offset, layer offset) of the medium cell "
                               f"({len(d12)} offsets x {nz} layers), r_cut = 5 a, torus 64^3, "
                               f"n = {n_rich}, N = {order}, 64 circle nodes",
                   "rel_err_vs_oracle_sample": err, "table_s": t_table},
        "roofline": {"bound": "alu", "achieved": flops / (ev_ms * 1e-3) / 1e12, "peak": FP64_VECTOR_PEAK,
                     "unit": "TFLOP/s", "frac": flops / (ev_ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK,
                     "traffic": None, "kernel": "k_plgf_eval", "flops_per_launch": flops},
    }
    if not args.no_cpu:
        sub = disp[rng.choice(disp.shape[0], 2048, replace=False)].astype(np.int64)
        t0 = time.perf_counter()
        oplgf.periodic_green(ora, sub, nz, n_rich, order)
        tc = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": len(sub) / tc, "unit": "3x3 blocks/s", "cores": 1, "kind": "oracle",
                                "sample": f"{len(sub)} seeded entries of the same workload (numpy, one thread)",
                                "cpu": _cpu_model()}
    pg.close()
    return line


def bench_hmat(args, torch) -> dict:
    """H-matrix form (Appendix C: b_min = 20, gamma = 2, eps = 1e-5) of every line mode of
    the medium cell, built from an FP64 offset-table context (no dense store); the H-matrix
    product over all modes against the dense FP64 product of the same cell."""
    import fbc_workloads as W
    from paper_2105_08798_amd import FBC, HMatrix
    wl = W.make_single("medium")
    c = wl.cells[0]
    nm, R = c.nz // 2 + 1, c.n_rhs
    dev = torch.device("cuda:0")
    tab = FBC(wl.cells, wl.bz, form="dtable_fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = HMatrix(tab, b_min=20, gamma=2, eps=1e-5, max_rank=args.max_rank)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    rng = np.random.default_rng(3)
    fh = rng.normal(size=(nm, 3 * c.n_i, R)) + 1j * rng.normal(size=(nm, 3 * c.n_i, R))
    x = torch.from_numpy(np.ascontiguousarray(np.stack([fh.real, fh.imag], axis=-1))).to(dev)
    y = torch.empty((nm, 3 * c.n_b, R, 2), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream()
    for _ in range(args.warmup):
        h.apply(x, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        h.apply(x, y)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # dense FP64 product of the same cell (its own kernel timing)
    ctx = FBC(wl.cells, wl.bz, form="fp64")
    f = torch.from_numpy(c.forces.ravel().copy()).to(dev)
    w = torch.zeros(R * c.nz * c.n_b * 3, dtype=torch.float64, device=dev)
    ctx.timing(True)
    for _ in range(3):
        ctx.green_apply(f, w)
    torch.cuda.synchronize()
    ctx.timing_read()
    for _ in range(10):
        ctx.green_apply(f, w)
    torch.cuda.synchronize()
    dense_ms, n_d = ctx.timing_read()
    dense_ms = dense_ms / max(n_d, 1)

    # whole fbc_apply steps: dense FP64 store, offset-table product, and the H-matrix
    # attached as the table context's product step
    def apply_ms(cx):
        u = torch.zeros(R * c.nz * c.n_b * 3, dtype=torch.float64, device=dev)
        for _ in range(2):
            cx.apply(f, u, alpha=1.0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            cx.apply(f, u, alpha=1.0)
        torch.cuda.synchronize()
        ms_ = 1000.0 * (time.perf_counter() - t) / args.steps
        u.zero_()
        cx.apply(f, u, alpha=1.0)
        return ms_, u.cpu().numpy()

    step_ms = {}
    step_ms["fp64"], u_dense = apply_ms(ctx)
    step_ms["dtable_fp64"], _ = apply_ms(tab)
    tab.set_hmat(h)
    step_ms["dtable_fp64+hmat"], u_h = apply_ms(tab)
    tab.set_hmat(None)
    upd_err = float(np.linalg.norm(u_h - u_dense) / np.linalg.norm(u_dense))
    log(f"hmat: fbc_apply ms/step {step_ms}; H-matrix update vs dense FP64 update {upd_err:.2e}")
    info = h.info
    from oracle import green
    yy = y.cpu().numpy()
    got = yy[..., 0] + 1j * yy[..., 1]
    errs = []
    for m in (0, 7, 64):
        a = green.green_modes_dense(c.nz, wl.bz, wl.bz, c.cols_b, c.cols_i, modes=[m])[0]
        ref = a @ fh[m]
        errs.append(float(np.linalg.norm(got[m] - ref) / np.linalg.norm(ref)))
    bytes_ = info.stored_entries * 16 + nm * 3 * (c.n_i + c.n_b) * R * 16
    log(f"hmat: build {t_build:.2f} s, {info.n_blocks} blocks ({info.n_low_rank} low rank), max rank "
        f"{info.max_rank_used}, stored {info.stored_entries / info.dense_entries:.3f} of dense, "
        f"{ms:.3f} ms per product (dense FP64 product {dense_ms:.3f} ms), errors {errs}")
    line = {
        "metric": "H-matrix products/s over all line modes (Appendix C form, FP64)",
        "value": 1e3 / ms, "unit": "products/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"hmat: medium cell (N_z = {c.nz}, n_i = {c.n_i}, n_b = {c.n_b}, {R} RHS, "
                               f"{nm} modes), b_min = 20, gamma = 2, eps = 1e-5, max rank {args.max_rank}",
                   "build_s": t_build, "n_blocks": info.n_blocks, "n_low_rank": info.n_low_rank,
                   "max_rank_used": info.max_rank_used, "n_over_rank": info.n_over_rank,
                   "stored_fraction": info.stored_entries / info.dense_entries,
                   "dense_fp64_product_ms": dense_ms, "rel_err_modes_0_7_64": errs,
                   "apply_ms_per_step": step_ms, "hmat_update_rel_err_vs_dense": upd_err},
        "roofline": {"bound": "hbm", "achieved": bytes_ / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_hmat_vt + k_hmat_y", "bytes_per_launch": bytes_},
    }
    h.close()
    tab.close()
    ctx.close()
    return line


def bench_hbm_read(args, torch) -> dict:
    """The device memory's practical streaming-read rate (fbc_probe_read: a plain read kernel,
    16-byte nontemporal loads, each work group its own contiguous share), for buffers of 16,
    64 and 128 GiB (the long workload's compact store holds 121.5 GB) and 512 to 4096 work
    groups, beside the 8 TB/s peak the roofline fractions are quoted against."""
    from paper_2105_08798_amd import probe_read
    rows = []
    for gib in (16, 64, 128):
        buf = torch.ones((gib << 30) // 8, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        for groups in (512, 1024, 2048, 4096):
            gbs = probe_read(buf, groups, reps=3)
            rows.append(dict(gib=gib, groups=groups, gbs=gbs, frac_of_peak=gbs / HBM_PEAK_GBS))
            log(f"{gib} GiB, {groups} groups: {gbs:.0f} GB/s")
        del buf
        torch.cuda.empty_cache()
    best = max(r["gbs"] for r in rows)
    return {"metric": "streaming-read rate of the device memory (plain read kernel)", "unit": "GB/s",
            "value": best, "peak": HBM_PEAK_GBS, "frac_of_peak": best / HBM_PEAK_GBS, "rows": rows,
            "data": "synthetic (a buffer of ones)"}


def bench_learned_budget(args, torch) -> dict:
    """Error budget of the learned far field on the long workload against the FP64 oracle's
    sampled line spectrum (tests/golden/long_modes.npz).  The surrogate keeps a line mode's
    exact lattice values out to the last block of exp(-s_exact) times the mode's largest,
    applies continuum + learned correction out to exp(-s_learn), the continuum alone
    beyond.  For (s_exact, s_learn) = (4, 12), (8, 16), (12, 20): the exact table's size,
    and the error with the continuum alone in the learned band, with the learned
    correction in BF16 weights, and with the same network's FP32 weights."""
    import fbc_workloads as W
    from paper_2105_08798_amd import FBC, MLP
    wl = W.make_single("long")
    c = wl.cells[0]
    kind, gold = golden("long")
    dev = torch.device("cuda:0")
    f = torch.from_numpy(c.forces).to(dev)
    cols = torch.from_numpy(np.asarray(gold["cols"])).to(dev)
    zero = MLP(max_batch=16, seed=0)
    zero.params(np.zeros(zero.n_params, dtype=np.float32))
    rows = []

    def err(sur):
        ctx = FBC(wl.cells, wl.bz, form="surrogate", surrogate=sur)
        store = ctx.info.store_bytes
        w = torch.zeros((c.n_rhs, c.nz, c.n_b, 3), dtype=torch.float64, device=dev)
        ctx.green_apply(f, w)
        if ctx.sync_status() != 0:
            raise RuntimeError("surrogate apply failed")
        w_cols = w[:, :, cols, :].cpu().numpy()
        ctx.close()
        del w
        torch.cuda.empty_cache()
        # whole sampled spectrum, and per sampled mode (relative to that mode's values)
        spec = np.fft.rfft(w_cols, axis=1)[:, gold["modes"]]
        ref = gold["what"]
        per_mode = [rel_err(spec[:, k], ref[:, k]) for k in range(ref.shape[1])]
        return oracle_error(kind, gold, w_cols), per_mode, store

    for s_exact, s_learn in ((4.0, 12.0), (8.0, 16.0), (12.0, 20.0)):
        sur, info, net = train_surrogate(torch, wl, args.train_steps, s_exact=s_exact, s_learn=s_learn,
                                         keep_net=True)
        e_bf16, m_bf16, store = err(sur)
        sur.set_mlp(net, fp32=True)
        e_fp32, m_fp32, _ = err(sur)
        sur.set_mlp(zero)
        e_cont, m_cont, _ = err(sur)
        row = dict(s_exact=s_exact, s_learn=s_learn, exact_table_bytes=int(store), continuum_only=e_cont,
                   learned_bf16=e_bf16, learned_fp32=e_fp32, modes=[int(m) for m in gold["modes"]],
                   per_mode_continuum_only=m_cont, per_mode_learned_bf16=m_bf16, per_mode_learned_fp32=m_fp32,
                   heldout_rel_err=info["heldout_rel_err"], train_s=info["train_s"], steps=info["steps"])
        log(f"budget s_exact={s_exact} s_learn={s_learn}: exact table {store / 1e9:.2f} GB; continuum "
            f"{e_cont:.3e}, learned bf16 {e_bf16:.3e}, fp32 {e_fp32:.3e}, held-out {info['heldout_rel_err']:.3e}")
        log(f"   per mode {row['modes']}: continuum {[f'{x:.1e}' for x in m_cont]}; "
            f"bf16 {[f'{x:.1e}' for x in m_bf16]}; fp32 {[f'{x:.1e}' for x in m_fp32]}")
        rows.append(row)
        net.close()
        sur.close()
    zero.close()
    return {"metric": "learned far field: relative pad-update error vs the FP64 oracle (sampled line spectrum)",
            "value": min(r["learned_bf16"] for r in rows), "unit": "relative error", "n_gpus": 1,
            "higher_is_better": False, "dtype": DTYPE["surrogate"], "data": "synthetic",
            "config": {"workload": f"long: {wl.description}, in-plane torus M={wl.bz}",
                       "oracle_samples": f"{len(gold['modes'])} line modes x {len(gold['cols'])} pad columns",
                       "train_steps": args.train_steps},
            "budget": rows}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=None,
                    help="one workload only (long, large, medium, batched, plgf, hmat, learned: the "
                         "learned far field's error budget, hbm: the memory's streaming-read rate); default: "
                         "long (headline) and large in one line")
    ap.add_argument("--forms", default=None, help="comma-separated forms of the headline workload")
    ap.add_argument("--graph", action="store_true", help="replay the update from a captured HIP graph")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default work list (the library's autotuner picks K slices and order otherwise)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: a stored choice for the same configuration is applied "
                         "untimed, a new one appended (keeps separate profiling runs on one work list)")
    ap.add_argument("--work-list", default=None, metavar="VARIANT:NSPLIT:ORDER",
                    help="product kernel variant and work list for every form instead of the autotuner's choice "
                         "(for counter runs of one launch configuration)")
    ap.add_argument("--skip-tol", type=float, default=0.0,
                    help="negligible-block tolerance of every form (0: the library's default per form, < 0: none)")
    ap.add_argument("--gen-modes", type=int, default=0,
                    help="learned form: table modes generated per chunk (0: the library's default)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--train-steps", type=int, default=20000, help="Adam steps of the surrogate's MLP")
    ap.add_argument("--max-rank", type=int, default=64, help="rank bound of the H-matrix workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.workload == "plgf":
        print(json.dumps(bench_plgf(args, torch)), flush=True)
        return 0
    if args.workload == "hmat":
        print(json.dumps(bench_hmat(args, torch)), flush=True)
        return 0
    if args.workload == "learned":
        print(json.dumps(bench_learned_budget(args, torch)), flush=True)
        return 0
    if args.workload == "hbm":
        print(json.dumps(bench_hbm_read(args, torch)), flush=True)
        return 0

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB write")
        del a, b

    name = args.workload or "long"
    forms = [s for s in (args.forms or ",".join(DEFAULT_FORMS[name])).split(",") if s]
    main_run = run_workload(torch, args, name, forms, extras_for="split_fp16")
    second = None
    if args.workload is None:
        second = run_workload(torch, args, "large", DEFAULT_FORMS["large"], extras_for="split_fp16")
    wl, out_forms, head = main_run["wl"], main_run["forms"], main_run["head"]
    h = out_forms[head]
    ref = main_run["ref_form"]
    roof = dict(h["roofline"])
    roof["traffic"] = measured_traffic(name, head, h["product_bytes"], h.get("autotune"))
    roof["kernel"] = f"per-mode product ({head})"
    line = {
        "metric": METRIC, "value": h["updates_per_s"], "unit": "FBC updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": h["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[head],
        "data": "synthetic",
        "config": {"workload": f"{name}: {wl.description}, in-plane torus M={wl.bz}",
                   "form": head, "rel_err": main_run["err_of"](head),
                   "rel_err_kind": ("vs the FP64 oracle at sampled line modes and pad columns"
                                    if h["oracle_samples"] == "modes" else
                                    "vs the FP64 oracle at sampled pad columns" if h["oracle_samples"] else
                                    "vs the FP64 form on the GPU"),
                   "graph": bool(args.graph), "fp64_plain_form": ref,
                   "fp64_plain_updates_per_s": out_forms[ref]["updates_per_s"] if ref else None,
                   "speedup_vs_fp64_plain": (h["updates_per_s"] / out_forms[ref]["updates_per_s"]) if ref else None},
        "roofline": roof,
        "forms": out_forms,
    }
    if second is not None:
        s2 = second["forms"]
        sref = second["ref_form"]
        line["large"] = {"workload": f"large: {second['wl'].description}, in-plane torus M={second['wl'].bz}",
                         "fastest_within_1e-6": second["head"], "fp64_plain_form": sref,
                         "speedup_vs_fp64_plain": (s2[second["head"]]["updates_per_s"] / s2[sref]["updates_per_s"])
                         if sref else None, "forms": s2}
    if not args.no_cpu and len(wl.cells) == 1:
        log("timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(wl, name)
        if second is not None:
            line["large"]["cpu_baseline"] = cpu_baseline(second["wl"], "large")
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
