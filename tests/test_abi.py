"""The C-ABI library loads and exports every entry point include/rs.h declares,
and its host-only paths (defaults, argument checks, error strings) behave as
documented.  No call here touches a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2409_03807_amd", "librs.so")
HEADER = os.path.join(ROOT, "include", "rs.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(rs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2409_03807_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ["rs_create", "rs_destroy", "rs_decode", "rs_energy_grad_hess", "rs_newton_solve",
                 "rs_lipschitz_loss", "rs_last_error"]:
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_lists_every_symbol():
    from paper_2409_03807_amd.binding import SYMBOLS
    assert sorted(SYMBOLS) == declared_symbols()


def test_default_opts_and_errors_on_host(lib):
    from paper_2409_03807_amd.binding import SolveOpts
    o = SolveOpts()
    assert lib.rs_default_opts(C.byref(o)) == 0
    assert (o.max_iter, o.ls_max, o.c1, o.shrink, o.rel_tol, o.hess) == (50, 128, 1e-4, 0.5, 1e-6, 1)
    assert lib.rs_default_opts(None) == 1
    from paper_2409_03807_amd.binding import LbfgsOpts, MAX_HISTORY
    lo = LbfgsOpts()
    assert lib.rs_default_lbfgs_opts(C.byref(lo)) == 0
    # the paper's exits (Sec. 5): 128 line-search trials, 1024 iterations
    assert (lo.max_iter, lo.ls_max, lo.history, lo.c1, lo.shrink, lo.rel_tol) == (1024, 128, 10, 1e-4, 0.5, 1e-6)
    assert lib.rs_default_lbfgs_opts(None) == 1
    hdr = open(os.path.join(ROOT, "include", "rs.h")).read()
    assert f"#define RS_MAX_HISTORY {MAX_HISTORY}" in hdr
    lib.rs_last_error.restype = C.c_char_p
    lib.rs_last_error.argtypes = [C.c_void_p]
    assert lib.rs_last_error(None) == b"rs: null context"
    out = C.c_void_p(1)
    # NULL mesh is rejected before any device work, and *out is cleared
    assert lib.rs_create(None, None, None, None, None, 0, 1, C.byref(out)) == 1
    assert not out.value
    assert lib.rs_create(None, None, None, None, None, 0, 1, None) == 1
    assert lib.rs_destroy(None) == 0
    # calls on a NULL context report an unusable context
    assert lib.rs_newton_solve(None, 0, None, None, None, None, None, None, None, None) == 4
    assert lib.rs_lbfgs_solve(None, 0, None, None, None, None, None, None, None, None) == 4
    assert lib.rs_energy_grad_hess(None, 0, None, None, 0, None, None, None, None) == 4
    assert lib.rs_energy_param_grad(None, 0, None, None, 0, None, None, None, None) == 4
    n = C.c_int64(-1)
    assert lib.rs_param_count(None, C.byref(n)) == 4 and n.value == -1
