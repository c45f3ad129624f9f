"""The C-ABI library loads, exports every symbol include/fbc.h declares, and rejects
invalid arguments before touching the device (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fbc.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fbc_[a-zA-Z_0-9]+)\s*\(", txt)))


def _lib():
    from paper_2105_08798_amd import fbc
    if not os.path.exists(fbc.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    return fbc, fbc.load_library()


def test_header_declares_the_documented_entry_points():
    names = _declared_functions()
    for n in ("fbc_assemble_G", "fbc_apply", "fbc_relax_step", "fbc_destroy", "fbc_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    fbc, lib = _lib()
    for n in _declared_functions():
        assert hasattr(lib, n), n
    assert set(fbc.EXPORTED) == set(_declared_functions())


def test_struct_layouts_match_header_sizes():
    fbc, _ = _lib()
    assert C.sizeof(fbc.Cell) == 32
    assert C.sizeof(fbc.RelaxOut) == 56
    assert C.sizeof(fbc.RelaxOpts) == 32
    assert C.sizeof(fbc.Options) == 72


def test_default_options():
    fbc, lib = _lib()
    o = fbc.Options()
    lib.fbc_default_options(C.byref(o))
    assert o.form == 0 and o.bz_m1 == 1024 and o.check_netforce == 1 and o.netforce_tol == 1e-10


def _assemble(lib, fbc, nz=8, n_i=4, n_b=6, n_rhs=1, bz=16, form=0, ncells=1, null_cols=False,
              k=1.0, table_fp32=0):
    ci = np.zeros((n_i, 2), np.int32)
    ci[:, 0] = np.arange(n_i)
    cb = np.zeros((n_b, 2), np.int32)
    cb[:, 0] = np.arange(n_b)
    cb[:, 1] = 5
    cell = fbc.Cell(nz, n_i, n_b, n_rhs, None if null_cols else ci.ctypes.data_as(C.POINTER(C.c_int32)),
                    cb.ctypes.data_as(C.POINTER(C.c_int32)))
    cells = (fbc.Cell * 1)(cell)
    opt = fbc.Options()
    lib.fbc_default_options(C.byref(opt))
    opt.bz_m1 = opt.bz_m2 = bz
    opt.form = form
    opt.table_fp32 = table_fp32
    lat = fbc.Lattice(1.0, k)
    out = C.c_void_p()
    rc = lib.fbc_assemble_G(C.byref(lat), cells, ncells, C.byref(opt), None, C.byref(out))
    return rc, out


@pytest.mark.parametrize("kw", [dict(nz=12), dict(nz=1), dict(nz=8192), dict(bz=12), dict(bz=4),
                                dict(n_i=0), dict(n_rhs=0), dict(form=9), dict(ncells=0),
                                dict(null_cols=True), dict(k=-1.0), dict(table_fp32=2),
                                dict(form=1, table_fp32=1), dict(form=5, table_fp32=1)])
def test_invalid_arguments_rejected_before_device_work(kw):
    fbc, lib = _lib()
    rc, out = _assemble(lib, fbc, **kw)
    assert rc == -1, (kw, rc)
    assert not out.value
    assert len(lib.fbc_last_error(None)) > 0


def test_null_context_calls_fail_cleanly():
    fbc, lib = _lib()
    assert lib.fbc_apply(None, None, None, 1.0, None) == -1
    assert lib.fbc_relax_step(None, None, None, None, None) == -1
    assert lib.fbc_sync_status(None, None) == -1
    assert lib.fbc_relax_get_state(None, None, None, None, None, None) == -1
    assert lib.fbc_relax_set_state(None, None, 0, None, None, None) == -1
    assert lib.fbc_relax_step_graph(None, None, None, None, None) == -1
    lib.fbc_destroy(None)
    assert lib.fbc_status_string(-3) == b"non-zero net force of a cell (all interface atoms of all layers)"


def test_surrogate_form_needs_a_surrogate_object():
    fbc, lib = _lib()
    rc, out = _assemble(lib, fbc, form=4)
    assert rc == -1 and not out.value


def test_learned_calls_reject_bad_arguments_on_the_host():
    fbc, lib = _lib()
    from oracle import mlp as omlp
    assert lib.fbc_mlp_num_params() == omlp.n_params()
    out = C.c_void_p()
    assert lib.fbc_mlp_create(0, C.c_uint64(1), C.byref(out)) == -1 and not out.value
    assert lib.fbc_mlp_create(1 << 23, C.c_uint64(1), C.byref(out)) == -1 and not out.value
    lat = fbc.Lattice(1.0, 1.0)
    assert lib.fbc_sur_create(None, 6.0, None, C.byref(out)) == -1 and not out.value
    assert lib.fbc_sur_create(C.byref(lat), -1.0, None, C.byref(out)) == -1 and not out.value
    assert lib.fbc_sur_create(C.byref(fbc.Lattice(1.0, -1.0)), 6.0, None, C.byref(out)) == -1
    assert lib.fbc_sur_eval(None, None, None, None, 1, 0, None, None) == -1
    assert lib.fbc_mlp_loss_grad(None, None, None, 1, None, None) == -1
    assert lib.fbc_mlp_adam_step(None, C.c_float(1e-3), None) == -1
    assert lib.fbc_learned_last_error()


def test_tune_result_layout_and_null_context_work_list():
    fbc, lib = _lib()
    assert C.sizeof(fbc.TuneResult) == 40
    assert lib.fbc_set_work_list(None, 1, 0, None) == -1


def test_read_probe_rejects_bad_arguments_on_the_host():
    fbc, lib = _lib()
    g = C.c_double(0.0)
    assert lib.fbc_probe_read(None, 1 << 20, 512, 1, C.byref(g), None) == -1
    fake = C.c_void_p(1 << 20)                    # never dereferenced: the checks come first
    assert lib.fbc_probe_read(fake, 24, 512, 1, C.byref(g), None) == -1        # not a multiple of 16
    assert lib.fbc_probe_read(fake, 1 << 20, 0, 1, C.byref(g), None) == -1
    assert lib.fbc_probe_read(fake, 1 << 20, 512, 0, C.byref(g), None) == -1
    assert lib.fbc_probe_read(fake, 1 << 20, 512, 1, None, None) == -1
    assert lib.fbc_probe_read(C.c_void_p((1 << 20) + 8), 1 << 20, 512, 1, C.byref(g), None) == -1   # alignment
