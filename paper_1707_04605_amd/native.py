"""ctypes loader of libmgrt.so (argument marshalling only).

The library is built in-tree by ``paper_1707_04605_amd/build.py``.  There is no
fallback: if the shared object is missing or fails to load, importing the binding raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgrt.so")

MGRT_OK = 0
ERRORS = {
    -1: "MGRT_E_ARG", -2: "MGRT_E_UNSTABLE", -3: "MGRT_E_OOM_PLAN", -4: "MGRT_E_HIP",
    -5: "MGRT_E_NONFINITE", -6: "MGRT_E_MESH", -7: "MGRT_E_STATE",
}
F_DEVICE_OUT = 1
F_TIMING = 2
F_SKIP_STABILITY = 8
F_NO_TUNE = 16
F_JAC_SPLIT = 32
F_JAC_DIRECT = 64
F_NO_GRAPH = 128
F_ONE_STEP = 512
F_JAC_PAIRED = 256
STEP_BATCHED = 0
STEP_PLAIN = 1
JAC_MG = 0
JAC_EXACT = 1
JAC_DECONV = 2
TV_AUTO = 0
TV_CG = 1


class MgrtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class RunOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("variant", C.c_int), ("batch", C.c_int),
                ("flags", C.c_int), ("mem_budget_gb", C.c_double), ("deconv_delta", C.c_double),
                ("launch", C.c_int)]


class Timing(C.Structure):
    _fields_ = [("step_launches", C.c_int64), ("step_ms_total", C.c_double),
                ("call_ms", C.c_double), ("node_updates", C.c_int64), ("nodes", C.c_int64),
                ("batch", C.c_int), ("precision", C.c_int), ("ell_width", C.c_int),
                ("ell_mean_width", C.c_double), ("variant", C.c_int),
                ("step_bytes", C.c_double), ("tune_us", C.c_double * 16),
                ("jac_split", C.c_int), ("graph_steps", C.c_int64),
                ("tune_b", C.c_int * 6), ("tune_b_us", C.c_double * 6),
                ("jac_runs", C.c_int), ("jac_sets", C.c_int), ("steps_per_launch", C.c_int)]


_lib = None

vp = C.c_void_p
i64 = C.c_int64
i32 = C.c_int32
dbl = C.c_double


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc for gfx950) first")
    # PyTorch ships its own HIP runtime under the same soname; load it first so that the
    # library binds to that one and the process holds a single HIP runtime (loading the
    # library first and torch afterwards leaves two, and device calls then fail)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    lib.mgrt_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
    lib.mgrt_destroy.argtypes = [vp]
    lib.mgrt_last_error.argtypes = [vp]
    lib.mgrt_last_error.restype = C.c_char_p
    lib.mgrt_upload_mesh.argtypes = [vp, C.c_int, i64, vp, i64, vp, i64, vp, vp, i64, vp, vp]
    lib.mgrt_upload_permittivity.argtypes = [vp, vp, vp]
    lib.mgrt_stability_bound.argtypes = [vp, C.POINTER(dbl)]
    lib.mgrt_forward_traces.argtypes = [vp, i64, vp, i32, vp, vp, dbl, i64, C.POINTER(RunOpts), vp]
    lib.mgrt_forward_traces_noalloc.argtypes = [vp, i64, vp, i32, vp, vp, dbl, i64,
                                                C.POINTER(RunOpts), vp]
    lib.mgrt_jacobian_coarse.argtypes = [vp, i64, vp, i32, vp, vp, dbl, i64, i32, vp, C.c_int,
                                         i64, vp, C.POINTER(RunOpts), vp]
    lib.mgrt_misfit_gradient.argtypes = [vp, i64, vp, i32, vp, vp, dbl, i64, vp, C.c_int,
                                         C.POINTER(RunOpts), vp]
    lib.mgrt_tv_invert_level.argtypes = [vp, i64, i64, vp, C.c_int, C.c_int, vp, vp, vp, vp,
                                         dbl, C.c_int, dbl, C.c_int, C.c_int, vp, vp]
    lib.mgrt_tv_invert_two_level.argtypes = [vp, i64, i64, vp, C.c_int, C.c_int, vp, C.c_int,
                                             vp, i64, vp, vp, vp, vp, vp, vp, vp, dbl,
                                             C.c_int, i64, dbl, C.c_int, C.c_int, vp, vp, vp,
                                             vp]
    lib.mgrt_upload_pml.argtypes = [vp, vp, vp]
    lib.mgrt_project_rows.argtypes = [vp, i64, C.c_int32, i64, vp, C.c_int, C.c_int, vp,
                                      C.c_int32, vp, vp]
    lib.mgrt_projection_weights.argtypes = [vp, C.c_int32, dbl, i64, vp]
    lib.mgrt_last_timing.argtypes = [vp, C.POINTER(Timing)]
    lib.mgrt_struct_sizes.argtypes = [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    so, st = C.c_size_t(), C.c_size_t()
    lib.mgrt_struct_sizes(C.byref(so), C.byref(st))
    if (so.value, st.value) != (C.sizeof(RunOpts), C.sizeof(Timing)):
        raise ImportError(f"{LIB_PATH}: mgrt_run_opts / mgrt_timing are {so.value} / "
                          f"{st.value} bytes, the binding's mirrors "
                          f"{C.sizeof(RunOpts)} / {C.sizeof(Timing)}; rebuild")
    _lib = lib
    return lib
