"""ctypes declarations of the C ABI in include/pflbm.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpflbm.so")
LIB_PATHS = {"d3q15": LIB_PATH,
             "d3q27": os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpflbm_d3q27.so")}

PFLBM_OK, PFLBM_ERR_ARG, PFLBM_ERR_STATE, PFLBM_ERR_HIP, PFLBM_ERR_UNSTABLE, \
    PFLBM_ERR_UNSUPPORTED = range(6)
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16s": 2}
COLLISIONS = {"bgk": 0, "mrt": 1}
STREAMING = {"ab": 0, "aa": 1}
FORCING = {"first": 0, "guo": 1}
STATES_WRITE_SRC_PHI, STATES_SKIP_DST_PHI = 1, 2
COPY_FORMS = {"w4": 0, "w16": 1, "w16_cached": 2, "soa43": 3, "soa43_nt": 4, "soa43_f64": 5,
              "soa43_f64_nt": 6}


class Desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_uint32), ("precision", C.c_int32), ("collision", C.c_int32),
                ("has_mask", C.c_int32), ("streaming", C.c_int32), ("forcing", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("tau_H", C.c_double), ("tau_L", C.c_double), ("mobility", C.c_double),
                ("xi", C.c_double), ("sigma", C.c_double), ("rho_H", C.c_double),
                ("rho_L", C.c_double), ("g", C.c_double * 3), ("s_high", C.c_double),
                ("fp16_scale_log2", C.c_double * 2), ("normal_eps", C.c_double),
                ("s_bulk", C.c_double), ("rho_g_ref", C.c_double)]


# name: (restype, argtypes)
SIGNATURES = {
    "pflbm_workspace_bytes": (C.c_size_t, [C.POINTER(Desc)]),
    "pflbm_create": (C.c_int, [C.POINTER(Desc), C.c_void_p, C.c_size_t, C.c_void_p,
                               C.POINTER(C.c_void_p)]),
    "pflbm_destroy": (C.c_int, [C.c_void_p]),
    "pflbm_set_params": (C.c_int, [C.c_void_p, C.POINTER(Params)]),
    "pflbm_set_mask": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pflbm_init_equilibrium": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pflbm_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "pflbm_set_check_interval": (C.c_int, [C.c_void_p, C.c_int64]),
    "pflbm_read_moments": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pflbm_read_phi": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pflbm_read_populations": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pflbm_reduce": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pflbm_reduce_static": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pflbm_state_bytes": (C.c_size_t, [C.c_void_p]),
    "pflbm_save_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pflbm_load_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "pflbm_step_states": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "pflbm_step_count": (C.c_int64, [C.c_void_p]),
    "pflbm_profile_step": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_double)]),
    "pflbm_sync": (C.c_int, [C.c_void_p]),
    "pflbm_lattice": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "pflbm_phase_q": (C.c_int32, []),
    "pflbm_adjoint_workspace_bytes": (C.c_size_t, [C.POINTER(Desc)]),
    "pflbm_adjoint_attach": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "pflbm_adjoint_reset": (C.c_int, [C.c_void_p]),
    "pflbm_adjoint_inject_phi": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pflbm_adjoint_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "pflbm_adjoint_init": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pflbm_adjoint_grads": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pflbm_hbm_copy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p]),
    "pflbm_pack_faces": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "pflbm_status_string": (C.c_char_p, [C.c_int]),
    "pflbm_last_error": (C.c_char_p, [C.c_void_p]),
}

_libs = {}
_ctx_lib = {}


def load(path: str = None, phase: str = "d3q15"):
    """Load the build of the given phase lattice: libpflbm.so ("d3q15", or the
    build named by $PFLBM_LIBRARY) or libpflbm_d3q27.so ("d3q27"); raises if
    it is missing (there is no fallback path)."""
    key = path or phase
    if key in _libs:
        return _libs[key]
    if path is None:
        path = (os.environ.get("PFLBM_LIBRARY") if phase == "d3q15" else None) or LIB_PATHS[phase]
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2206_11637_amd.build` "
            "(the HIP library is the only implementation of the step)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _libs[key] = lib
    return lib


def register(ctx, lib) -> None:
    """Remember which build a context belongs to (for its error messages)."""
    _ctx_lib[ctx.value] = lib


def unregister(ctx) -> None:
    _ctx_lib.pop(ctx.value, None)


class PFLBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(status: int, ctx=None, what: str = "") -> None:
    if status != PFLBM_OK:
        lib = _ctx_lib.get(ctx.value if ctx is not None else None) or load()
        detail = lib.pflbm_last_error(ctx).decode() if ctx else ""
        base = lib.pflbm_status_string(status).decode()
        raise PFLBMError(status, f"{what}: {base}" + (f": {detail}" if detail else ""))
