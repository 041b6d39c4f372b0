"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/p2o.h declares, and rejects bad arguments before it
touches the device."""
import ctypes
import os
import re

import pytest

import paper_2504_16344_amd as P
import p2o_synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        from paper_2504_16344_amd.build import build_library
        build_library()
    return P.load_library()


def header_symbols():
    text = open(os.path.join(ROOT, "include", "p2o.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(p2o_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert header_symbols() == sorted(P.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in header_symbols():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for code, name in P.STATUS.items():
        assert lib.p2o_status_string(code).decode()
    assert lib.p2o_status_string(99) == b"unknown status"


def test_setup_rejects_bad_arguments_on_host(lib):
    h = ctypes.c_void_p(123)
    # sizes < 1 and bad precision are refused before any device call
    assert lib.p2o_setup_begin(0, 5, 5, 0, None, ctypes.byref(h)) == 1
    assert h.value is None
    assert lib.p2o_setup_begin(5, 5, 0, 0, None, ctypes.byref(h)) == 1
    assert lib.p2o_setup_begin(5, 5, 5, 7, None, ctypes.byref(h)) == 1
    assert lib.p2o_setup_begin(5, 5, 5, 4, None, ctypes.byref(h)) == 1
    assert lib.p2o_setup_begin(5, 5, 5, 0, None, None) == 1
    assert lib.p2o_setup(None, 5, 5, 5, 0, None, ctypes.byref(h)) == 1
    # null handles
    assert lib.p2o_apply(None, 0, None, None, 1, None) == 1
    assert lib.p2o_setup_end(None, None) == 1
    assert lib.p2o_reserve(None, 1, None) == 1
    assert lib.p2o_get_info(None, None, None, None, None, None) == 1
    assert lib.p2o_hessian_assemble(None, 1.0, None, None, None) == 1
    assert lib.p2o_posterior_solve(None, None, None, None, 1, 1.0, 1, None, None) == 1
    assert lib.p2o_posterior_mean(None, None, None, None, 1, 1.0, None) == 1
    assert lib.p2o_posterior_invert(None, None, None, None) == 1
    assert lib.p2o_posterior_mean_kinv(None, None, None, None, 1, 1.0, None) == 1
    assert lib.p2o_posterior_mean_kinv_noalloc(None, None, None, None, 1, 1.0, None) == 1
    assert lib.p2o_read_bandwidth(None, 16, None, None) == 1
    assert lib.p2o_kernel_time(None, 0, None, None) == 1
    assert lib.p2o_last_hip_error(None) == 1
    lib.p2o_destroy(None)


def test_smooth_length():
    assert [P.smooth_length(n) for n in (1, 32, 200, 420, 97, 13)] == [2, 64, 400, 840, 196, 28]


def test_synth_device_library_exports():
    path = p2o_synth.LIB_PATH
    if not os.path.exists(path):
        from p2o_synth.build import build_library
        build_library()
    lib = p2o_synth.load_device_library()
    assert hasattr(lib, "synth_blocks_f64") and hasattr(lib, "synth_normals_f64")


def test_boundary_names_and_precision_values():
    """The boundary's names: p2o_setup (+ chunked), p2o_apply,
    p2o_hessian_assemble, p2o_posterior_solve, the batch and graph calls, and
    the precision tiers P2O_FP64 = 0, P2O_MIXED = 1 (bfloat16 hi+lo),
    P2O_FAST = 2 (bfloat16 hi only), plus the extra P2O_MIXED_FP16 = 3."""
    names = set(header_symbols())
    for name in ("p2o_setup", "p2o_setup_begin", "p2o_setup_columns", "p2o_setup_end",
                 "p2o_apply", "p2o_hessian_assemble", "p2o_posterior_solve",
                 "p2o_batch_create", "p2o_batch_apply", "p2o_graph_capture",
                 "p2o_graph_launch", "p2o_destroy", "p2o_status_string", "p2o_last_hip_error"):
        assert name in names, name
    text = open(os.path.join(ROOT, "include", "p2o.h")).read()
    vals = dict(re.findall(r"\b(P2O_[A-Z0-9_]+)\s*=\s*([A-Z0-9_]+)", text))
    assert vals["P2O_FP64"] == "0" and vals["P2O_MIXED"] == "1" and vals["P2O_FAST"] == "2"
    assert vals["P2O_MIXED_FP16"] == "3"
    assert vals["P2O_MIXED_BF16"] == "P2O_MIXED" and vals["P2O_FAST_BF16"] == "P2O_FAST"
    assert (P.FP64, P.MIXED, P.FAST, P.MIXED_FP16) == (0, 1, 2, 3)
    assert P.PREC_BY_NAME["mixed_bf16"] == P.MIXED and P.PREC_BY_NAME["fast_bf16"] == P.FAST
