"""The C ABI without a GPU: the library loads and exports every function that
include/lpgpu.h declares, the binding knows them all, and the host-only
entry points behave as documented."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpgpu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(lp_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lpgpu():
    from paper_2211_10979_amd import lpgpu as mod

    if not os.path.exists(mod.LIB_PATH):
        pytest.skip("liblpgpu.so not built")
    return mod


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lp_create", "lp_solve", "lp_get_solution", "lp_get_pivots", "lp_destroy", "lp_batch_create",
                 "lp_batch_solve", "lp_server_create", "lp_server_submit", "lp_server_poll"):
        assert must in names


# The boundary's entry points and the leading option fields, in this order.
BOUNDARY_CALLS = ["lp_options_default", "lp_tableau_bytes", "lp_create", "lp_solve", "lp_get_solution",
                  "lp_get_pivots", "lp_destroy", "lp_error_string", "lp_batch_create", "lp_batch_solve",
                  "lp_batch_get_solution", "lp_batch_get_pivots", "lp_batch_destroy", "lp_server_create",
                  "lp_server_submit", "lp_server_poll", "lp_server_stats", "lp_server_destroy"]
BOUNDARY_OPTIONS = ["eps_dual", "eps_pivot", "max_pivots", "record_pivots", "stream", "device_buffer",
                    "device_buffer_bytes"]


def struct_fields(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + ";", text).group(1)
    return re.findall(r"(\w+)\s*;", body)


def test_boundary_names_and_option_order():
    names = declared_functions()
    assert [n for n in BOUNDARY_CALLS if n not in names] == []
    fields = struct_fields("lp_options")
    assert fields[:len(BOUNDARY_OPTIONS)] == BOUNDARY_OPTIONS
    assert fields[len(BOUNDARY_OPTIONS):] == ["device", "bland_after", "tuning"]


def test_binding_layout_matches_the_header(lpgpu):
    assert [f for f, _ in lpgpu.lp_options._fields_] == struct_fields("lp_options")
    assert [f for f, _ in lpgpu.lp_tuning._fields_] == struct_fields("lp_tuning")


def test_every_declared_symbol_is_exported(lpgpu):
    lib = ctypes.CDLL(lpgpu.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_covers_the_header(lpgpu):
    assert set(declared_functions()) <= set(lpgpu.SIGNATURES), set(declared_functions()) - set(lpgpu.SIGNATURES)


def test_host_only_entry_points(lpgpu):
    lib = lpgpu.library()
    assert b"lpgpu" in lib.lp_version()
    assert lib.lp_error_string(lpgpu.LP_E_NEG_RHS)
    assert lib.lp_error_string(12345) == b"unknown code"
    o = lpgpu.lp_options_default()
    assert o.eps_dual == 1e-9 and o.eps_pivot == 1e-9 and o.record_pivots == 1 and not o.tuning
    assert lib.lp_options_default(None) == lpgpu.LP_E_INVAL
    t = lpgpu.lp_tuning_default()
    assert all(getattr(t, name) == 0 for name in lpgpu.TUNING_FIELDS)
    assert lib.lp_tuning_default(None) == lpgpu.LP_E_INVAL
    o = lpgpu.lp_options_default(fuse_pivots=4, eps_dual=1e-7)
    assert o.eps_dual == 1e-7 and o.tuning and o.tuning.contents.fuse_pivots == 4
    # tableau bytes: ld = m+1 rounded up to 16 doubles, W = n+m+1 columns
    assert lpgpu.lp_tableau_bytes(8000, 8000) == 8016 * 16001 * 8
    assert lpgpu.lp_tableau_bytes(15, 3) == 16 * 19 * 8
    assert lpgpu.lp_tableau_bytes(16, 3) == 32 * 20 * 8
    assert lpgpu.lp_tableau_bytes(0, 3) == 0


def test_null_arguments_are_rejected_without_a_device(lpgpu):
    lib = lpgpu.library()
    assert lib.lp_create(None, 1, 1, None, None, None, None) == lpgpu.LP_E_INVAL
    h = ctypes.c_void_p()
    assert lib.lp_create(ctypes.byref(h), 0, 1, None, None, None, None) == lpgpu.LP_E_INVAL
    assert lib.lp_solve(None) == lpgpu.LP_E_INVAL
    assert lib.lp_get_solution(None, None, None, None) == lpgpu.LP_E_INVAL
    lib.lp_destroy(None)  # NULL-safe
    lib.lp_batch_destroy(None)
    lib.lp_server_destroy(None)
    assert lib.lp_solve(None) == lpgpu.LP_E_INVAL
    assert "NULL" in lpgpu.lp_last_error()


def test_oracle_and_library_share_no_code():
    """The oracle is a separate C file built by gcc; the HIP sources never
    include or name it, and it never includes them."""
    csrc = os.path.join(ROOT, "paper_2211_10979_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "oracle" not in text.lower(), f
    otext = open(os.path.join(ROOT, "oracle", "tableau_simplex.c")).read()
    assert "#include \"" not in otext and "lpgpu" not in otext
    pytext = open(os.path.join(ROOT, "oracle", "__init__.py")).read()
    assert "paper_2211_10979_amd" not in pytext
