"""The C-ABI library loads and exports every function include/ocp_admm.h
declares; host-side argument checks reject bad input without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ocp_admm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ocp_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("ocp_create", "ocp_destroy", "ocp_set_lti", "ocp_set_qp", "ocp_set_bicycle", "ocp_solve",
                 "ocp_adjoint", "ocp_default_settings", "ocp_status_string", "ocp_supported",
                 "ocp_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2606_24039_amd import _abi

    lib = C.CDLL(_abi.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the ctypes mirror covers the same set
    assert sorted(n for n, _, _ in _abi.SIGNATURES) == declared_functions()


def test_struct_layouts_match_header_field_order():
    from paper_2606_24039_amd import _abi

    src = open(HEADER).read()
    body = re.search(r"typedef struct \{([^{}]*?)\} ocp_settings;", src, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"([a-z_0-9]+)\s*[,;]", body)
    assert fields == [f for f, _ in _abi.ocp_settings._fields_]


def test_defaults_and_host_side_errors():
    from paper_2606_24039_amd import _abi

    lib = _abi.lib()
    s = _abi.default_settings()
    assert (s.sigma, s.rho0, s.rho_f_scale, s.k_rho, s.k_ratio, s.max_admm) == (1e-6, 0.1, 1e3, 25, 5.0, 1000)
    assert lib.ocp_supported(12, 4, 16) == 1 and lib.ocp_supported(4, 2, 3) == 1
    assert lib.ocp_supported(40, 4, 4) == 0
    hz = (C.c_int32 * 2)(20, 20)
    h = C.c_void_p()
    bad = _abi.ocp_dims(2, 40, 4, 4, _abi.MODEL_LTI, 0, 0)
    assert lib.ocp_create(C.byref(bad), hz, C.byref(h)) == _abi.OCP_E_SHAPE
    neg = _abi.ocp_dims(0, 4, 2, 4, _abi.MODEL_LTI, 0, 0)
    assert lib.ocp_create(C.byref(neg), hz, C.byref(h)) == _abi.OCP_E_ARG
    zero_h = (C.c_int32 * 2)(20, 0)
    ok = _abi.ocp_dims(2, 4, 2, 4, _abi.MODEL_LTI, 0, 0)
    assert lib.ocp_create(C.byref(ok), zero_h, C.byref(h)) == _abi.OCP_E_ARG
    nbytes = C.c_size_t()
    assert lib.ocp_workspace_bytes(C.byref(ok), hz, C.byref(nbytes)) == _abi.OCP_OK and nbytes.value > 0
    assert lib.ocp_status_string(_abi.OCP_E_ORDER) == b"call order violated"
    assert lib.ocp_destroy(None) == _abi.OCP_OK
    # entry points that need a handle reject a null one before any device work
    assert lib.ocp_graph_capture(None, C.byref(s), None, None, None, None, None) == _abi.OCP_E_ARG
    assert lib.ocp_graph_launch(None, None) == _abi.OCP_E_ARG
    assert lib.ocp_profile(None, 1) == _abi.OCP_E_ARG
    assert lib.ocp_profile_read(None, None) == _abi.OCP_E_ARG
    assert lib.ocp_set_segmented(None, 128) == _abi.OCP_E_ARG
    assert lib.ocp_set_segmented_after(None, 150) == _abi.OCP_E_ARG
    assert lib.ocp_set_tail_workgroup(None, 200) == _abi.OCP_E_ARG
    assert lib.ocp_set_multiwave(None, 255) == _abi.OCP_E_ARG
    assert lib.ocp_autotune(None, C.byref(s), 1, None, None, None, None) == _abi.OCP_E_ARG


def test_product_path_has_no_cpu_fallback(monkeypatch):
    from paper_2606_24039_amd import _abi

    monkeypatch.setattr(_abi, "_LIB", None)
    monkeypatch.setattr(_abi, "LIB_PATH", "/nonexistent/libocp_admm.so")
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _abi.lib()
