"""The C-ABI library builds for gfx950, loads, and exports every entry point
that include/floop.h declares (no GPU work is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "floop.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fl_[A-Za-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_1108_2473_amd as fl
    if not os.path.exists(fl.LIB_PATH):
        from paper_1108_2473_amd import build
        build.build()
    return fl.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("fl_create", "fl_destroy", "fl_set_stream", "fl_set_gauge", "fl_set_kappa", "fl_apply_D",
                 "fl_solve", "fl_loops_exact", "fl_loops_stochastic", "fl_loops_grad", "fl_last_error"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_defaults(lib):
    import paper_1108_2473_amd as fl
    assert "gfx950" in fl.version()
    p = fl._SolverParams()
    lib.fl_solver_params_default(ctypes.byref(p))
    assert p.solver == 0 and p.tol == 1e-12 and p.gauge_reals == 12 and p.inner_prec == fl.PREC_F32
    assert p.delta == 0.0 and p.truncated == 0  # 0: the solver chooses delta for the inner precision


def test_argument_checks_before_any_device_call(lib):
    """Odd or too small extents, a bad bc_t and lattices beyond the 32-bit
    addressing of a link array (including extents whose product overflows
    64 bits) are rejected before HIP is touched."""
    h = ctypes.c_void_p()
    big = 1 << 30
    for dims, bc in [((3, 4, 4, 4), -1), ((4, 4, 4, 0), -1), ((4, 4, 4, 4), 0), ((2, 2, 2, 1), 1),
                     ((64, 64, 64, 64), -1), ((big, big, big, big), -1)]:
        d = (ctypes.c_int * 4)(*dims)
        assert lib.fl_create(ctypes.byref(h), 0, d, bc) == -1
        assert lib.fl_last_error(None)
    assert lib.fl_create(None, 0, (ctypes.c_int * 4)(4, 4, 4, 4), -1) == -1
    # NULL context pointers are rejected
    assert lib.fl_set_kappa(None, 0.1) == -1
    assert lib.fl_destroy(None) == 0


def test_library_is_built_for_gfx950_only():
    """The build script targets gfx950 and disables packed-FP32 instructions."""
    from paper_1108_2473_amd import build
    src = open(build.__file__).read()
    assert 'ARCH = "gfx950"' in src and "-packed-fp32-ops" in src


def test_batched_loops_reject_a_context_given_twice(lib):
    """fl_loops_stochastic_multi compares the context pointers before using
    them: the same context twice would share one workspace (no GPU work and
    no dereference happens; the pointers here are placeholders)."""
    import paper_1108_2473_amd as fl
    dummy = ctypes.create_string_buffer(64)
    h = ctypes.cast(dummy, ctypes.c_void_p).value
    hs = (ctypes.c_void_p * 2)(h, h)
    nps = (fl._NoiseParams * 2)()
    g = (ctypes.c_int * 1)(0)
    outs = (ctypes.c_void_p * 2)(h, h)
    p = fl._SolverParams()
    lib.fl_solver_params_default(ctypes.byref(p))
    st = lib.fl_loops_stochastic_multi(hs, 2, nps, g, 1, ctypes.byref(p), ctypes.byref(p), outs, 0)
    assert st == -1
    assert b"twice" in lib.fl_last_error(None)
    assert dummy.raw == b"\0" * 64  # the placeholder was not written


def test_last_stats_argument_checks(lib):
    n = ctypes.c_longlong(-7)
    assert lib.fl_last_stats(None, None, 0, ctypes.byref(n)) == -1
    assert n.value == -7
