"""The C ABI without a GPU: the library loads, exports every function that
include/npga.h declares, and its host-side logic (defaults, status text,
workspace sizes, argument validation before any launch) behaves as the
header documents.  No call here reaches a kernel."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "npga.h")
LIB = os.path.join(ROOT, "paper_2604_02917_amd", "libnpga.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(npga_[a-z0-9_]+)\s*\(", text, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ["npga_solve", "npga_project", "npga_gradient", "npga_build_factor", "npga_sketch_str",
                 "npga_solve_batched", "npga_gradient_batched", "npga_batched_tune", "npga_to_bf16",
                 "npga_backward", "npga_status_string", "npga_default_options"]:
        assert must in names, must


def test_every_declared_symbol_is_exported(lib):
    missing = [name for name in declared_functions() if not hasattr(lib, name)]
    assert not missing, missing


def test_default_options_and_status_strings():
    from paper_2604_02917_amd import api
    o = api._Options()
    api._lib.npga_default_options(ctypes.byref(o))
    assert o.tol == 1e-6 and o.check_every == 5 and o.power_iters == 20 and o.step_estimator == 0
    assert o.step_safety == 1.05 and o.refine == 1 and o.batch_config == -1 and o.momentum == 0
    for code in range(9):
        assert api.status_string(code) and api.status_string(code) != "unknown status"
    assert api.status_string(99) == "unknown status"


def test_struct_layouts_match_the_binding():
    """The ctypes structures of the binding have the sizes of the C ones."""
    from paper_2604_02917_amd import api
    for which, st in enumerate([api._Options, api._Result, api._Factor, api._StrOptions, api._BackwardResult]):
        assert api._lib.npga_struct_size(which) == ctypes.sizeof(st), st.__name__
    assert api._lib.npga_struct_size(5) == 0
    o = api._Options()
    api._lib.npga_default_options(ctypes.byref(o))
    assert o.alpha == 0.0  # step estimated unless the caller fixes it


def test_workspace_sizes():
    from paper_2604_02917_amd import api
    lib = api._lib
    assert lib.npga_solve_workspace_size(0, 10, None) == 0
    assert lib.npga_solve_workspace_size(8193, 10, None) == 0
    a = lib.npga_solve_workspace_size(5440, 48374, None)
    assert a > 0 and a % 256 == 0
    # the batched workspace holds the single-solve region plus per-target buffers
    b1 = lib.npga_batched_workspace_size(2000, 20000, 1, None)
    b128 = lib.npga_batched_workspace_size(2000, 20000, 128, None)
    og = api._Options()
    lib.npga_default_options(ctypes.byref(og))
    og.path = 1   # the batched solver runs the fused sweep's layout
    assert b128 > b1 > lib.npga_solve_workspace_size(2000, 20000, ctypes.byref(og))
    assert lib.npga_batched_workspace_size(2000, 20000, 0, None) == 0
    assert lib.npga_batched_workspace_size(2000, 20000, 1025, None) == 0
    assert lib.npga_build_factor_workspace_size(64, 1) == 0
    assert lib.npga_sketch_workspace_size(64, 256, 32, 64) == 0   # ell > k


def test_invalid_arguments_rejected_before_launch():
    """Null or inconsistent arguments return NPGA_ERR_INVALID (1) without
    touching the device (there is none here)."""
    from paper_2604_02917_amd import api
    lib = api._lib
    res = api._Result()
    null = ctypes.c_void_p(0)
    assert lib.npga_solve(None, 0.0, None, null, ctypes.byref(res), null, 0, null) == 1
    f = api._Factor(64, 256, 62, 16, 16, 0.0, 0, 0)            # ld < n
    assert lib.npga_solve(ctypes.byref(f), 0.0, None, ctypes.c_void_p(16), ctypes.byref(res), null, 0,
                          null) == 1
    f = api._Factor(64, 256, 64, 16, 16, -1.0, 0, 0)           # gamma < 0
    assert lib.npga_gradient(ctypes.byref(f), ctypes.c_void_p(16), ctypes.c_void_p(16), null, null, 0,
                             null) == 1
    f = api._Factor(64, 256, 64, 16, 16, 0.0, 7, 0)            # unknown dtype
    assert lib.npga_gradient(ctypes.byref(f), ctypes.c_void_p(16), ctypes.c_void_p(16), null, null, 0,
                             null) == 1
    f = api._Factor(64, 256, 64, 16, 16, 0.0, 0, 0)
    r = (ctypes.c_double * 2)(0.0, float("nan"))              # non-finite target
    assert lib.npga_solve_batched(ctypes.byref(f), r, 2, None, ctypes.c_void_p(16), 64, None, null, 0,
                                  null) == 1
    o = api._Options()
    lib.npga_default_options(ctypes.byref(o))
    o.batch_config = 12                                        # out of range
    r = (ctypes.c_double * 1)(0.0)
    assert lib.npga_solve_batched(ctypes.byref(f), r, 1, ctypes.byref(o), ctypes.c_void_p(16), 64, None,
                                  null, 0, null) == 1
    # a valid request with no workspace reports NPGA_ERR_WORKSPACE (6)
    o.batch_config = -1
    assert lib.npga_solve_batched(ctypes.byref(f), r, 1, ctypes.byref(o), ctypes.c_void_p(16), 64, None,
                                  null, 0, null) == 6
    assert lib.npga_project(null, null, 4, 0.0, null, null, null, 0, null) == 1
    f = api._Factor(64, 256, 64, 16, 16, 0.0, 0, 0)
    assert lib.npga_backward(ctypes.byref(f), 0.0, null, null, null, null, 64, None, null, 0, null) == 1
    assert lib.npga_backward(ctypes.byref(f), 0.0, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16),
                             ctypes.c_void_p(16), 63, None, null, 0, null) == 1      # ldg < n
    assert lib.npga_backward(ctypes.byref(f), 0.0, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16),
                             null, 64, None, null, 0, null) == 6                     # no workspace
    og = api._Options()
    lib.npga_default_options(ctypes.byref(og))
    og.path = 1   # the adjoint runs on the fused sweep's layout
    assert lib.npga_backward_workspace_size(64, 256) > lib.npga_solve_workspace_size(64, 256, ctypes.byref(og))
    # a negative or non-finite fixed step is rejected
    o.alpha = -1.0
    assert lib.npga_solve_batched(ctypes.byref(f), r, 1, ctypes.byref(o), ctypes.c_void_p(16), 64, None,
                                  null, 0, null) == 1
    o.alpha = float("inf")
    assert lib.npga_solve_batched(ctypes.byref(f), r, 1, ctypes.byref(o), ctypes.c_void_p(16), 64, None,
                                  null, 0, null) == 1
    # backtracking and Dykstra's projections are single-solve options
    o.alpha = 0.0
    o.backtrack_rho = 0.5
    assert lib.npga_solve_batched(ctypes.byref(f), r, 1, ctypes.byref(o), ctypes.c_void_p(16), 64, None,
                                  null, 0, null) == 1
    o.backtrack_rho = 1.0                                      # out of (0, 1)
    assert lib.npga_solve(ctypes.byref(f), 0.0, ctypes.byref(o), ctypes.c_void_p(16), ctypes.byref(res), null, 0,
                          null) == 1
    o.backtrack_rho = 0.0
    o.projection = 1
    assert lib.npga_solve_batched(ctypes.byref(f), r, 1, ctypes.byref(o), ctypes.c_void_p(16), 64, None,
                                  null, 0, null) == 1


def test_build_script_runs_without_importing_the_package():
    """The build must work on a checkout with no library: the build script
    imports nothing from the package (whose import loads the library)."""
    src = open(os.path.join(ROOT, "paper_2604_02917_amd", "build.py")).read()
    assert "import paper_2604_02917_amd" not in src and "from paper_2604_02917_amd" not in src
    assert "from ." not in src
    entry = open(os.path.join(ROOT, "__graft_entry__.py")).read()
    assert "spec_from_file_location" in entry


def test_auto_path_rule():
    """NPGA_PATH_AUTO: the covariance path for a float32 factor with at least
    as many columns as assets (measured faster there), within its 4 GiB
    workspace bound; the fused sweep for fewer columns (an STR factor), a
    bfloat16 factor, or a covariance workspace past the bound."""
    from paper_2604_02917_amd import api
    lib = api._lib
    F32, BF16, GEMV, SYRK = 0, 1, 1, 2
    assert lib.npga_auto_path(5440, 48374, F32) == SYRK      # the full model, T >> n
    assert lib.npga_auto_path(5440, 5440, F32) == SYRK       # T = n
    assert lib.npga_auto_path(5440, 5439, F32) == GEMV       # T < n
    assert lib.npga_auto_path(5440, 512, F32) == GEMV        # an STR factor (ell = 512)
    assert lib.npga_auto_path(5440, 48374, BF16) == GEMV     # the covariance path needs float32
    assert lib.npga_auto_path(64, 256, F32) == SYRK
    assert lib.npga_auto_path(8192, 100000, F32) == GEMV     # Sigma + planes ~ 5.2 GB > 4 GiB
    assert lib.npga_auto_path(0, 10, F32) == -1 and lib.npga_auto_path(10, 10, 7) == -1
    # the workspace query sizes for the path AUTO takes
    o = api._Options()
    lib.npga_default_options(ctypes.byref(o))
    assert o.path == 0
    auto = lib.npga_solve_workspace_size(5440, 48374, ctypes.byref(o))
    o.path = SYRK
    assert auto == lib.npga_solve_workspace_size(5440, 48374, ctypes.byref(o))
    o.path = 0
    small = lib.npga_solve_workspace_size(5440, 512, ctypes.byref(o))
    o.path = GEMV
    assert small == lib.npga_solve_workspace_size(5440, 512, ctypes.byref(o)) < auto
    assert api.auto_path(5440, 48374) == "syrk" and api.auto_path(5440, 48374, "bf16") == "gemv"
