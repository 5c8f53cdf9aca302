"""Host-only checks of the C ABI: the library loads and exports every symbol that
include/mgrt.h declares; calls without a device fail with an error code."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgrt.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(mgrt_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("mgrt_create", "mgrt_destroy", "mgrt_last_error", "mgrt_upload_mesh",
              "mgrt_upload_permittivity", "mgrt_forward_traces", "mgrt_jacobian_coarse",
              "mgrt_misfit_gradient", "mgrt_tv_invert_level", "mgrt_tv_invert_two_level",
              "mgrt_project_rows", "mgrt_projection_weights", "mgrt_upload_pml",
              "mgrt_stability_bound",
              "mgrt_last_timing", "mgrt_struct_sizes"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_1707_04605_amd import native
    lib = native.load()
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_null_and_device_errors_without_gpu():
    from paper_1707_04605_amd import native
    lib = native.load()
    assert lib.mgrt_create(0, None, None) == -1            # MGRT_E_ARG
    assert lib.mgrt_destroy(None) == -1
    assert lib.mgrt_last_error(None) == b"null context"
    t = native.Timing()
    assert lib.mgrt_last_timing(None, C.byref(t)) == -1
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if not has_gpu:
        h = C.c_void_p()
        assert lib.mgrt_create(0, None, C.byref(h)) == -4   # MGRT_E_HIP: no device here
        assert not h.value


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1707_04605_amd import native
    monkeypatch.setattr(native, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(native, "_lib", None)
    with pytest.raises(ImportError):
        native.load()


def test_struct_mirrors_match_the_library():
    """The binding's ctypes mirrors of mgrt_run_opts and mgrt_timing have the library's
    sizes (native.load also refuses a library that disagrees)."""
    from paper_1707_04605_amd import native
    lib = native.load()
    so, st = C.c_size_t(), C.c_size_t()
    assert lib.mgrt_struct_sizes(C.byref(so), C.byref(st)) == 0
    assert so.value == C.sizeof(native.RunOpts)
    assert st.value == C.sizeof(native.Timing)
