"""Thin ctypes binding of libfbc.so (argument marshalling only).

Every step of the FBC update runs in the HIP library; this module converts Python
arguments to the C structs of include/fbc.h and passes device pointers of torch
tensors and the current HIP stream.  It raises if the built library is missing: there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfbc.so")

FBC_OK = 0
STATUS = {0: "FBC_OK", -1: "FBC_E_ARG", -2: "FBC_E_NOMEM", -3: "FBC_E_NETFORCE",
          -4: "FBC_E_NONFINITE", -5: "FBC_E_DEVICE", -6: "FBC_E_STATE", -7: "FBC_E_UNSUPPORTED"}
FORMS = {"fp64": 0, "fp32": 1, "split_bf16": 2, "dtable_fp64": 3, "surrogate": 4, "split_fp16": 5}

EXPORTED = [
    "fbc_default_options", "fbc_assemble_G", "fbc_apply", "fbc_green_apply", "fbc_relax_begin",
    "fbc_relax_step", "fbc_relax_get_state", "fbc_relax_set_state", "fbc_sync_status", "fbc_get_info", "fbc_copy_block_rows", "fbc_destroy",
    "fbc_last_error", "fbc_status_string", "fbc_timing", "fbc_timing_read", "fbc_apply_graph",
    "fbc_autotune", "fbc_set_work_list", "fbc_learned_last_error", "fbc_sur_create", "fbc_sur_destroy", "fbc_sur_set_mlp",
    "fbc_sur_eval", "fbc_sur_training_set", "fbc_mlp_create", "fbc_mlp_destroy", "fbc_mlp_num_params",
    "fbc_mlp_params", "fbc_mlp_grad", "fbc_mlp_loss_grad", "fbc_mlp_adam_step", "fbc_mlp_forward",
    "fbc_plgf_last_error", "fbc_plgf_create", "fbc_plgf_destroy", "fbc_plgf_table", "fbc_plgf_eval",
    "fbc_hmat_last_error", "fbc_hmat_create", "fbc_hmat_destroy", "fbc_hmat_get_info", "fbc_hmat_partition",
    "fbc_hmat_ranks", "fbc_hmat_apply", "fbc_mlp_forward_noalloc", "fbc_mlp_forward_noalloc_max_rows",
    "fbc_relax_step_graph", "fbc_autotune_cached", "fbc_set_kernel_variant", "fbc_sur_set_mlp_fp32",
    "fbc_sur_set_learn_range", "fbc_sur_set_exact_range", "fbc_set_hmat", "fbc_probe_read",
]


class FbcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Lattice(C.Structure):
    _fields_ = [("a", C.c_double), ("spring_k", C.c_double)]


class Cell(C.Structure):
    _fields_ = [("nz", C.c_int), ("n_i", C.c_int), ("n_b", C.c_int), ("n_rhs", C.c_int),
                ("cols_i", C.POINTER(C.c_int32)), ("cols_b", C.POINTER(C.c_int32))]


class Options(C.Structure):
    _fields_ = [("form", C.c_int), ("bz_m1", C.c_int), ("bz_m2", C.c_int),
                ("check_netforce", C.c_int), ("project_netforce", C.c_int),
                ("netforce_tol", C.c_double), ("row_gauge", C.c_int), ("surrogate", C.c_void_p),
                ("gen_modes", C.c_int), ("skip_tol", C.c_double), ("table_fp32", C.c_int)]


class RelaxOpts(C.Structure):
    _fields_ = [("relax", C.c_int), ("du_max", C.c_double), ("tol_f", C.c_double), ("alpha_min", C.c_double)]


class RelaxOut(C.Structure):
    _fields_ = [("alpha", C.c_double), ("f_inf", C.c_double), ("step_inf", C.c_double),
                ("mean_removed", C.c_double * 3), ("converged", C.c_int32), ("k", C.c_int32)]


RELAX_OUT_DOUBLES = C.sizeof(RelaxOut) // 8


class Info(C.Structure):
    _fields_ = [("n_cells", C.c_int), ("total_rhs", C.c_int), ("store_bytes", C.c_int64),
                ("scratch_bytes", C.c_int64), ("f_elems", C.c_int64), ("u_elems", C.c_int64),
                ("n_offsets", C.c_int64), ("nsplit", C.c_int), ("job_order", C.c_int),
                ("n_jobs", C.c_int), ("product_bytes", C.c_double), ("product_flops", C.c_double),
                ("skipped_fraction", C.c_double), ("kernel_variant", C.c_int), ("n_variants", C.c_int),
                ("kernel_shape", C.c_char * 96)]


class PlgfOpts(C.Structure):
    _fields_ = [("torus_l", C.c_int), ("r2x4_cut", C.c_int), ("r2x4_match", C.c_int), ("n_psi", C.c_int)]


class HmatOpts(C.Structure):
    _fields_ = [("b_min", C.c_int), ("gamma", C.c_int), ("eps", C.c_double), ("max_rank", C.c_int)]


class HmatInfo(C.Structure):
    _fields_ = [("n_blocks", C.c_int), ("n_low_rank", C.c_int), ("n_dense", C.c_int), ("max_rank_used", C.c_int),
                ("n_over_rank", C.c_int), ("stored_entries", C.c_double), ("dense_entries", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("nsplit", C.c_int), ("order", C.c_int), ("gemm_ms", C.c_double),
                ("n_candidates", C.c_int), ("call_ms", C.c_double), ("variant", C.c_int),
                ("from_cache", C.c_int)]


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = C.CDLL(path)
    vp, cp = C.c_void_p, C.c_char_p
    lib.fbc_default_options.argtypes = [C.POINTER(Options)]
    lib.fbc_default_options.restype = None
    lib.fbc_assemble_G.argtypes = [C.POINTER(Lattice), C.POINTER(Cell), C.c_int, C.POINTER(Options),
                                   vp, C.POINTER(vp)]
    lib.fbc_apply.argtypes = [vp, vp, vp, C.c_double, vp]
    lib.fbc_green_apply.argtypes = [vp, vp, vp, vp]
    lib.fbc_relax_begin.argtypes = [vp, C.POINTER(RelaxOpts), vp]
    lib.fbc_relax_step.argtypes = [vp, vp, vp, vp, vp]
    lib.fbc_relax_step_graph.argtypes = [vp, vp, vp, vp, vp]
    lib.fbc_relax_get_state.argtypes = [vp, C.POINTER(RelaxOpts), C.POINTER(C.c_int32), vp, vp, vp]
    lib.fbc_relax_set_state.argtypes = [vp, C.POINTER(RelaxOpts), C.c_int32, vp, vp, vp]
    lib.fbc_sync_status.argtypes = [vp, vp]
    lib.fbc_get_info.argtypes = [vp, C.POINTER(Info)]
    lib.fbc_copy_block_rows.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, vp]
    lib.fbc_apply_graph.argtypes = [vp, vp, vp, C.c_double, vp]
    lib.fbc_autotune.argtypes = [vp, vp, vp, C.c_int, C.POINTER(TuneResult), vp]
    lib.fbc_autotune_cached.argtypes = [vp, vp, vp, C.c_int, cp, C.POINTER(TuneResult), vp]
    lib.fbc_set_kernel_variant.argtypes = [vp, C.c_int]
    lib.fbc_set_work_list.argtypes = [vp, C.c_int, C.c_int, vp]
    lib.fbc_timing.argtypes = [vp, C.c_int]
    lib.fbc_timing_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    lib.fbc_destroy.argtypes = [vp]
    lib.fbc_destroy.restype = None
    lib.fbc_last_error.argtypes = [vp]
    lib.fbc_last_error.restype = cp
    lib.fbc_status_string.argtypes = [C.c_int]
    lib.fbc_status_string.restype = cp
    lib.fbc_learned_last_error.argtypes = []
    lib.fbc_learned_last_error.restype = cp
    lib.fbc_sur_create.argtypes = [C.POINTER(Lattice), C.c_double, vp, C.POINTER(vp)]
    lib.fbc_sur_destroy.argtypes = [vp]
    lib.fbc_sur_destroy.restype = None
    lib.fbc_sur_set_mlp.argtypes = [vp, vp, vp]
    lib.fbc_sur_set_mlp_fp32.argtypes = [vp, vp, vp]
    lib.fbc_sur_set_learn_range.argtypes = [vp, C.c_double]
    lib.fbc_sur_set_exact_range.argtypes = [vp, C.c_double]
    lib.fbc_sur_eval.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, vp, vp]
    lib.fbc_sur_training_set.argtypes = [vp, vp, C.c_int, C.c_uint64, vp, vp, C.POINTER(C.c_int), vp]
    lib.fbc_mlp_create.argtypes = [C.c_int, C.c_uint64, C.POINTER(vp)]
    lib.fbc_mlp_destroy.argtypes = [vp]
    lib.fbc_mlp_destroy.restype = None
    lib.fbc_mlp_num_params.argtypes = []
    lib.fbc_mlp_params.argtypes = [vp, vp, vp]
    lib.fbc_mlp_grad.argtypes = [vp, vp]
    lib.fbc_mlp_loss_grad.argtypes = [vp, vp, vp, C.c_int, vp, vp]
    lib.fbc_mlp_adam_step.argtypes = [vp, C.c_float, vp]
    lib.fbc_mlp_forward.argtypes = [vp, vp, vp, C.c_int, vp]
    lib.fbc_mlp_forward_noalloc.argtypes = [vp, vp, vp, C.c_int, vp]
    lib.fbc_mlp_forward_noalloc_max_rows.argtypes = []
    lib.fbc_mlp_forward_noalloc_max_rows.restype = C.c_int
    lib.fbc_plgf_last_error.argtypes = []
    lib.fbc_plgf_last_error.restype = cp
    lib.fbc_plgf_create.argtypes = [C.POINTER(Lattice), C.POINTER(PlgfOpts), vp, C.POINTER(vp)]
    lib.fbc_plgf_destroy.argtypes = [vp]
    lib.fbc_plgf_destroy.restype = None
    lib.fbc_plgf_table.argtypes = [vp, C.POINTER(C.c_int), vp, vp, vp]
    lib.fbc_plgf_eval.argtypes = [vp, vp, C.c_int64, C.c_int, C.c_int, C.c_int, vp, vp]
    lib.fbc_hmat_last_error.argtypes = []
    lib.fbc_hmat_last_error.restype = cp
    lib.fbc_hmat_create.argtypes = [vp, C.POINTER(HmatOpts), vp, C.POINTER(vp)]
    lib.fbc_hmat_destroy.argtypes = [vp]
    lib.fbc_hmat_destroy.restype = None
    lib.fbc_hmat_get_info.argtypes = [vp, C.POINTER(HmatInfo)]
    lib.fbc_hmat_partition.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_int64)]
    lib.fbc_hmat_ranks.argtypes = [vp, vp]
    lib.fbc_hmat_apply.argtypes = [vp, vp, vp, vp]
    lib.fbc_set_hmat.argtypes = [vp, vp, vp]
    lib.fbc_probe_read.argtypes = [vp, C.c_int64, C.c_int, C.c_int, C.POINTER(C.c_double), vp]
    for name in ("fbc_assemble_G", "fbc_apply", "fbc_green_apply", "fbc_relax_begin", "fbc_relax_step",
                 "fbc_relax_step_graph", "fbc_autotune_cached", "fbc_set_kernel_variant",
                 "fbc_sur_set_mlp_fp32", "fbc_sur_set_learn_range", "fbc_sur_set_exact_range", "fbc_set_hmat",
                 "fbc_relax_get_state", "fbc_relax_set_state",
                 "fbc_sync_status", "fbc_get_info", "fbc_copy_block_rows", "fbc_timing", "fbc_timing_read",
                 "fbc_apply_graph", "fbc_autotune", "fbc_set_work_list", "fbc_sur_create", "fbc_sur_set_mlp", "fbc_sur_eval",
                 "fbc_sur_training_set", "fbc_mlp_create", "fbc_mlp_num_params", "fbc_mlp_params",
                 "fbc_mlp_grad", "fbc_mlp_loss_grad", "fbc_mlp_adam_step", "fbc_mlp_forward",
                 "fbc_mlp_forward_noalloc", "fbc_plgf_create", "fbc_plgf_table", "fbc_plgf_eval", "fbc_hmat_create", "fbc_hmat_get_info",
                 "fbc_hmat_partition", "fbc_hmat_ranks", "fbc_hmat_apply", "fbc_probe_read"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dptr(t, dtype=None) -> int:
    import torch
    dtype = torch.float64 if dtype is None else dtype
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
    return t.data_ptr()


def _lcheck(lib, rc):
    if rc != FBC_OK:
        raise FbcError(rc, lib.fbc_learned_last_error().decode())


class FBC:
    """One assembled context (cells, Green store, scratch) on the current device."""

    def __init__(self, cells, bz: int | tuple, form: str = "fp64", spring_k: float = 1.0,
                 lattice_a: float = 1.0, check_netforce: bool = True, project_netforce: bool = False,
                 netforce_tol: float = 1e-10, row_gauge: bool = True, surrogate=None, gen_modes: int = 0,
                 skip_tol: float = 0.0, table_fp32: bool = False, stream=None):
        lib = load_library()
        self._lib = lib
        self.ctx = C.c_void_p()
        bz1, bz2 = (bz, bz) if isinstance(bz, int) else bz
        opt = Options()
        lib.fbc_default_options(C.byref(opt))
        opt.form = FORMS[form] if isinstance(form, str) else int(form)
        opt.bz_m1, opt.bz_m2 = int(bz1), int(bz2)
        opt.check_netforce = int(bool(check_netforce))
        opt.project_netforce = int(bool(project_netforce))
        opt.netforce_tol = float(netforce_tol)
        opt.row_gauge = int(bool(row_gauge))
        opt.surrogate = surrogate.handle.value if surrogate is not None else None
        opt.gen_modes = int(gen_modes)
        opt.skip_tol = float(skip_tol)
        opt.table_fp32 = int(bool(table_fp32))
        self._sur = surrogate          # the context reads it on every apply
        self.form = form
        self._keep = []
        arr = (Cell * len(cells))()
        for k, c in enumerate(cells):
            ci = np.ascontiguousarray(c.cols_i, dtype=np.int32)
            cb = np.ascontiguousarray(c.cols_b, dtype=np.int32)
            self._keep += [ci, cb]
            arr[k] = Cell(int(c.nz), int(ci.shape[0]), int(cb.shape[0]), int(c.n_rhs),
                          ci.ctypes.data_as(C.POINTER(C.c_int32)), cb.ctypes.data_as(C.POINTER(C.c_int32)))
        lat = Lattice(float(lattice_a), float(spring_k))
        st = _stream_handle(stream)
        rc = lib.fbc_assemble_G(C.byref(lat), arr, len(cells), C.byref(opt), st, C.byref(self.ctx))
        if rc != FBC_OK:
            raise FbcError(rc, lib.fbc_last_error(None).decode())
        self._keep = []
        self.info = self.get_info()

    def _check(self, rc):
        if rc != FBC_OK:
            raise FbcError(rc, self._lib.fbc_last_error(self.ctx).decode())

    def get_info(self) -> Info:
        info = Info()
        self._check(self._lib.fbc_get_info(self.ctx, C.byref(info)))
        return info

    def apply(self, f, u, alpha: float = 1.0, stream=None):
        self._check(self._lib.fbc_apply(self.ctx, _dptr(f), _dptr(u), float(alpha), _stream_handle(stream)))

    def apply_graph(self, f, u, alpha: float = 1.0, stream=None):
        self._check(self._lib.fbc_apply_graph(self.ctx, _dptr(f), _dptr(u), float(alpha), _stream_handle(stream)))

    def set_work_list(self, nsplit: int, order: int, stream=None):
        self._check(self._lib.fbc_set_work_list(self.ctx, int(nsplit), int(order), _stream_handle(stream)))
        self.info = self.get_info()

    def autotune(self, f, w, reps: int = 3, cache: str | None = None, stream=None) -> dict:
        """Tunes the product launch (kernel variant, K slices, order); with `cache` (a file
        path) a stored result for the same configuration is applied untimed, and a new one
        is appended."""
        r = TuneResult()
        if cache is None:
            self._check(self._lib.fbc_autotune(self.ctx, _dptr(f), _dptr(w), int(reps), C.byref(r),
                                               _stream_handle(stream)))
        else:
            self._check(self._lib.fbc_autotune_cached(self.ctx, _dptr(f), _dptr(w), int(reps),
                                                      os.fsencode(cache), C.byref(r), _stream_handle(stream)))
        self.info = self.get_info()
        return dict(nsplit=r.nsplit, order=r.order, gemm_ms=r.gemm_ms, n_candidates=r.n_candidates,
                    call_ms=r.call_ms, variant=r.variant, from_cache=bool(r.from_cache),
                    shape=self.info.kernel_shape.decode())

    def set_kernel_variant(self, variant: int):
        self._check(self._lib.fbc_set_kernel_variant(self.ctx, int(variant)))
        self.info = self.get_info()

    def set_hmat(self, h, stream=None):
        """Product step from the H-matrix h (an HMatrix of this context), or None: the
        offset-table product again."""
        self._check(self._lib.fbc_set_hmat(self.ctx, h.handle if h is not None else None, _stream_handle(stream)))
        self._hmat = h                       # keep it alive while attached
        self.info = self.get_info()

    def green_apply(self, f, w, stream=None):
        self._check(self._lib.fbc_green_apply(self.ctx, _dptr(f), _dptr(w), _stream_handle(stream)))

    def relax_begin(self, relax: bool = True, du_max: float = 0.0, tol_f: float = 1e-3,
                    alpha_min: float = 0.0, stream=None):
        o = RelaxOpts(int(bool(relax)), float(du_max), float(tol_f), float(alpha_min))
        self._check(self._lib.fbc_relax_begin(self.ctx, C.byref(o), _stream_handle(stream)))

    def relax_step(self, f, u, out=None, stream=None):
        """out: float64 CUDA tensor of at least total_rhs * RELAX_OUT_DOUBLES elements, or None."""
        optr = _dptr(out) if out is not None else None
        self._check(self._lib.fbc_relax_step(self.ctx, _dptr(f), _dptr(u), optr, _stream_handle(stream)))

    def relax_step_graph(self, f, u, out=None, stream=None):
        """relax_step replayed from a captured HIP graph (stream: a created torch stream)."""
        optr = _dptr(out) if out is not None else None
        self._check(self._lib.fbc_relax_step_graph(self.ctx, _dptr(f), _dptr(u), optr, _stream_handle(stream)))

    def relax_state(self, stream=None) -> dict:
        """Checkpoint of the relaxation: options, k, alpha_k per RHS (host array) and the
        previous raw incompatibility forces (float64 CUDA tensor in the layout of f)."""
        import torch
        info = self.get_info()
        o = RelaxOpts()
        k = C.c_int32()
        alpha = np.empty(info.total_rhs, dtype=np.float64)
        f_prev = torch.empty(info.f_elems, dtype=torch.float64, device="cuda")
        self._check(self._lib.fbc_relax_get_state(self.ctx, C.byref(o), C.byref(k), alpha.ctypes.data,
                                                  _dptr(f_prev), _stream_handle(stream)))
        return dict(relax=bool(o.relax), du_max=o.du_max, tol_f=o.tol_f, alpha_min=o.alpha_min, k=k.value,
                    alpha=alpha, f_prev=f_prev)

    def set_relax_state(self, state: dict, stream=None):
        """Loads a state from relax_state() (in place of relax_begin)."""
        o = RelaxOpts(int(bool(state["relax"])), float(state["du_max"]), float(state["tol_f"]),
                      float(state["alpha_min"]))
        alpha = np.ascontiguousarray(state["alpha"], dtype=np.float64)
        f_prev = state["f_prev"]
        self._check(self._lib.fbc_relax_set_state(self.ctx, C.byref(o), int(state["k"]), alpha.ctypes.data,
                                                  _dptr(f_prev) if f_prev is not None else None,
                                                  _stream_handle(stream)))

    def sync_status(self, stream=None) -> int:
        return self._lib.fbc_sync_status(self.ctx, _stream_handle(stream))

    def timing(self, enable: bool = True):
        self._check(self._lib.fbc_timing(self.ctx, int(bool(enable))))

    def timing_read(self) -> tuple[float, int]:
        ms = C.c_double()
        n = C.c_int()
        self._check(self._lib.fbc_timing_read(self.ctx, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def block_rows(self, cell: int, m: int, b0: int, b1: int, n_i: int) -> np.ndarray:
        out = np.empty((3 * (b1 - b0), 6 * n_i), dtype=np.float64)
        self._check(self._lib.fbc_copy_block_rows(self.ctx, cell, m, b0, b1, out.ctypes.data))
        return out[:, 0::2] + 1j * out[:, 1::2]

    def close(self):
        if self.ctx:
            self._lib.fbc_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """Trainable far-field correction network (FP32 parameters and Adam state on device)."""

    def __init__(self, max_batch: int, seed: int = 0):
        lib = load_library()
        self._lib = lib
        self.handle = C.c_void_p()
        _lcheck(lib, lib.fbc_mlp_create(int(max_batch), C.c_uint64(seed), C.byref(self.handle)))
        self.n_params = lib.fbc_mlp_num_params()
        self.max_batch = int(max_batch)

    def params(self, new: np.ndarray | None = None) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        src = None
        if new is not None:
            src = np.ascontiguousarray(new, dtype=np.float32)
            if src.size != self.n_params:
                raise ValueError("parameter vector has the wrong length")
        _lcheck(self._lib, self._lib.fbc_mlp_params(self.handle, out.ctypes.data,
                                                    None if src is None else src.ctypes.data))
        return out

    def grad(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        _lcheck(self._lib, self._lib.fbc_mlp_grad(self.handle, out.ctypes.data))
        return out

    def loss_grad(self, x, t, loss_out=None, stream=None):
        import torch
        n = int(x.shape[0])
        _lcheck(self._lib, self._lib.fbc_mlp_loss_grad(
            self.handle, _dptr(x, torch.float32), _dptr(t, torch.float32), n,
            None if loss_out is None else _dptr(loss_out, torch.float32), _stream_handle(stream)))

    def adam_step(self, lr: float, stream=None):
        _lcheck(self._lib, self._lib.fbc_mlp_adam_step(self.handle, C.c_float(lr), _stream_handle(stream)))

    def forward(self, x, y, stream=None):
        import torch
        _lcheck(self._lib, self._lib.fbc_mlp_forward(self.handle, _dptr(x, torch.float32),
                                                     _dptr(y, torch.float32), int(x.shape[0]),
                                                     _stream_handle(stream)))

    def forward_noalloc(self, x, y, stream=None):
        """The same forward pass with the activations in the library's static workspace."""
        import torch
        _lcheck(self._lib, self._lib.fbc_mlp_forward_noalloc(self.handle, _dptr(x, torch.float32),
                                                             _dptr(y, torch.float32), int(x.shape[0]),
                                                             _stream_handle(stream)))

    def noalloc_max_rows(self) -> int:
        return int(self._lib.fbc_mlp_forward_noalloc_max_rows())

    def close(self):
        if self.handle:
            self._lib.fbc_mlp_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """Continuum table plus BF16 inference weights of the far-field correction."""

    def __init__(self, r_c: float = 6.0, spring_k: float = 1.0, lattice_a: float = 1.0, stream=None):
        lib = load_library()
        self._lib = lib
        self.handle = C.c_void_p()
        self.r_c = float(r_c)
        lat = Lattice(float(lattice_a), float(spring_k))
        _lcheck(lib, lib.fbc_sur_create(C.byref(lat), self.r_c, _stream_handle(stream), C.byref(self.handle)))

    def set_mlp(self, net: MLP, stream=None, fp32: bool = False):
        """Inference weights from the network: BF16 (default) or, as a control, FP32."""
        fn = self._lib.fbc_sur_set_mlp_fp32 if fp32 else self._lib.fbc_sur_set_mlp
        _lcheck(self._lib, fn(self.handle, net.handle, _stream_handle(stream)))

    def set_learn_range(self, s_learn: float):
        """Upper end (kappa rho) of the learned band."""
        _lcheck(self._lib, self._lib.fbc_sur_set_learn_range(self.handle, float(s_learn)))

    def set_exact_range(self, s_exact: float):
        """kappa rho range of the exact lattice values (read when a context is created)."""
        _lcheck(self._lib, self._lib.fbc_sur_set_exact_range(self.handle, float(s_exact)))

    def eval(self, theta0, dn1, dn2, out, use_mlp: bool, stream=None):
        """theta0 float64, dn1/dn2 int32 (device); out float64 [n, 6, 2] (device)."""
        import torch
        n = int(theta0.shape[0])
        _lcheck(self._lib, self._lib.fbc_sur_eval(self.handle, _dptr(theta0), _dptr(dn1, torch.int32),
                                                  _dptr(dn2, torch.int32), n, int(bool(use_mlp)),
                                                  _dptr(out), _stream_handle(stream)))

    def training_set(self, table_ctx: "FBC", max_samples: int, seed: int, stream=None):
        """Returns (x [n, 8], t [n, 12]) float32 device tensors drawn from the table context."""
        import torch
        x = torch.empty((max_samples, 8), dtype=torch.float32, device="cuda")
        t = torch.empty((max_samples, 12), dtype=torch.float32, device="cuda")
        n = C.c_int()
        _lcheck(self._lib, self._lib.fbc_sur_training_set(self.handle, table_ctx.ctx, int(max_samples),
                                                          C.c_uint64(seed), x.data_ptr(), t.data_ptr(),
                                                          C.byref(n), _stream_handle(stream)))
        return x[:n.value], t[:n.value]

    def close(self):
        if self.handle:
            self._lib.fbc_sur_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PeriodicGreen:
    """Real-space line-periodic lattice Green function: near-field table within r_cut,
    continuum beyond, image sum with Richardson extrapolation (fbc_plgf_*)."""

    def __init__(self, torus_l: int = 64, r2x4_cut: int = 100, r2x4_match: int = 144, n_psi: int = 64,
                 spring_k: float = 1.0, lattice_a: float = 1.0, stream=None):
        lib = load_library()
        self._lib = lib
        self.handle = C.c_void_p()
        lat = Lattice(float(lattice_a), float(spring_k))
        opts = PlgfOpts(int(torus_l), int(r2x4_cut), int(r2x4_match), int(n_psi))
        self._check(lib.fbc_plgf_create(C.byref(lat), C.byref(opts), _stream_handle(stream), C.byref(self.handle)))

    def _check(self, rc):
        if rc != FBC_OK:
            raise FbcError(rc, self._lib.fbc_plgf_last_error().decode())

    def table(self):
        """(vectors int32 [T, 3], values float64 [T, 6], c float64 [6]) on the host."""
        import numpy as np
        n = C.c_int()
        self._check(self._lib.fbc_plgf_table(self.handle, C.byref(n), None, None, None))
        vec = np.zeros((n.value, 3), dtype=np.int32)
        val = np.zeros((n.value, 6))
        c = np.zeros(6)
        self._check(self._lib.fbc_plgf_table(self.handle, C.byref(n), vec.ctypes.data, val.ctypes.data,
                                             c.ctypes.data))
        return vec, val, c

    def eval(self, disp, out, nz: int, n_rich: int = 1, order: int = 5, stream=None):
        """disp int32 [n, 3], out float64 [n, 6] (device tensors)."""
        import torch
        n = int(disp.shape[0])
        self._check(self._lib.fbc_plgf_eval(self.handle, _dptr(disp, torch.int32) if n else None, n, int(nz),
                                            int(n_rich), int(order), _dptr(out) if n else None,
                                            _stream_handle(stream)))

    def close(self):
        if self.handle:
            self._lib.fbc_plgf_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HMatrix:
    """H-matrices of every line mode of a one-cell FP64 context (fbc_hmat_*)."""

    def __init__(self, ctx: "FBC", b_min: int = 20, gamma: int = 2, eps: float = 1e-5, max_rank: int = 64,
                 stream=None):
        lib = load_library()
        self._lib = lib
        self._ctx = ctx                      # the store must outlive this object
        self.handle = C.c_void_p()
        opts = HmatOpts(int(b_min), int(gamma), float(eps), int(max_rank))
        self._check(lib.fbc_hmat_create(ctx.ctx, C.byref(opts), _stream_handle(stream), C.byref(self.handle)))
        self.info = HmatInfo()
        self._check(lib.fbc_hmat_get_info(self.handle, C.byref(self.info)))

    def _check(self, rc):
        if rc != FBC_OK:
            raise FbcError(rc, self._lib.fbc_hmat_last_error().decode())

    def partition(self):
        """List of (kind, t columns, s columns); kind 1 low rank, 0 dense."""
        import numpy as np
        n = C.c_int64()
        self._check(self._lib.fbc_hmat_partition(self.handle, None, 0, C.byref(n)))
        buf = np.zeros(n.value, dtype=np.int32)
        self._check(self._lib.fbc_hmat_partition(self.handle, buf.ctypes.data, n.value, C.byref(n)))
        out, k = [], 0
        while k < len(buf):
            kind, nt, ns = int(buf[k]), int(buf[k + 1]), int(buf[k + 2])
            t = buf[k + 3:k + 3 + nt].copy()
            s = buf[k + 3 + nt:k + 3 + nt + ns].copy()
            out.append((kind, t, s))
            k += 3 + nt + ns
        return out

    def ranks(self, n_modes: int):
        import numpy as np
        r = np.zeros((n_modes, self.info.n_low_rank), dtype=np.int32)
        self._check(self._lib.fbc_hmat_ranks(self.handle, r.ctypes.data))
        return r

    def apply(self, fhat, what, stream=None):
        """fhat float64 [n_modes, 3 n_i, R, 2], what float64 [n_modes, 3 n_b, R, 2] (device)."""
        self._check(self._lib.fbc_hmat_apply(self.handle, _dptr(fhat), _dptr(what), _stream_handle(stream)))

    def close(self):
        if self.handle:
            self._lib.fbc_hmat_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_read(buf, groups: int, reps: int = 5, stream=None) -> float:
    """Streaming-read rate (GB/s) of the device buffer `buf` (a CUDA tensor, 16-byte aligned,
    a multiple of 16 bytes) with `groups` work groups: fbc_probe_read, a diagnostic for
    weighing the kernels against the memory's practical rate."""
    if not buf.is_contiguous():
        raise ValueError("probe_read needs a contiguous tensor")
    lib = load_library()
    out = C.c_double(0.0)
    rc = lib.fbc_probe_read(C.c_void_p(buf.data_ptr()), C.c_int64(buf.numel() * buf.element_size()), int(groups),
                            int(reps), C.byref(out), _stream_handle(stream))
    if rc != 0:
        raise FbcError(rc, f"fbc_probe_read: {lib.fbc_status_string(rc).decode()}")
    return out.value


def parse_relax_out(t) -> list[dict]:
    """Decodes the device relax-out buffer (copied to host) into dicts."""
    a = np.ascontiguousarray(t.detach().cpu().numpy()) if hasattr(t, "detach") else np.asarray(t)
    raw = a.view(np.uint8)
    out = []
    n = raw.size // C.sizeof(RelaxOut)
    for r in range(n):
        o = RelaxOut.from_buffer_copy(raw[r * C.sizeof(RelaxOut):(r + 1) * C.sizeof(RelaxOut)].tobytes())
        out.append(dict(alpha=o.alpha, f_inf=o.f_inf, step_inf=o.step_inf,
                        mean_removed=list(o.mean_removed), converged=bool(o.converged), k=o.k))
    return out
