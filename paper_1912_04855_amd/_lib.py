"""ctypes declarations of the C ABI in include/csph.h (argument marshalling only).

The library is the in-tree ``libcsph.so`` built by ``paper_1912_04855_amd/build.py``.
Loading fails loudly when it is missing: there is no fallback path.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# CSPH_LIB may name another build of the same library (to compare builds)
LIB_PATH = os.environ.get("CSPH_LIB") or os.path.join(HERE, "libcsph.so")

OK, ERR_ARG, ERR_NOMEM, ERR_DEVICE, ERR_STATE, ERR_NONFINITE, ERR_NEG_DENSITY, ERR_NO_SIGNAL, \
    ERR_BUDGET = range(9)
F32, F64 = 0, 1
PERIODIC, OUTFLOW, INFLOW, REFLECT = 0, 1, 2, 3
CONSERVED, PRIMITIVE = 0, 1
LIM_MINMOD, LIM_MC, LIM_VANLEER, LIM_SUPERBEE = 0, 1, 2, 3
FLUX_SWEPT, FLUX_LF, FLUX_SWEPT_AV = 0, 1, 2

STATUS_NAMES = {0: "CSPH_OK", 1: "CSPH_ERR_ARG", 2: "CSPH_ERR_NOMEM", 3: "CSPH_ERR_DEVICE",
                4: "CSPH_ERR_STATE", 5: "CSPH_ERR_NONFINITE", 6: "CSPH_ERR_NEG_DENSITY",
                7: "CSPH_ERR_NO_SIGNAL", 8: "CSPH_ERR_BUDGET"}

# every entry point declared in include/csph.h
EXPORTS = [
    "csph_required_bytes", "csph_create", "csph_create_in", "csph_destroy", "csph_set_stream",
    "csph_set_state", "csph_set_potential", "csph_set_boundary", "csph_step", "csph_advance",
    "csph_get_state", "csph_get_time", "csph_set_time", "csph_totals", "csph_get_stage",
    "csph_last_error", "csph_batch_create", "csph_batch_add", "csph_batch_advance",
    "csph_batch_poll", "csph_batch_remove", "csph_batch_destroy", "csph_profile_enable",
    "csph_profile_read", "csph_set_tile_depth", "csph_set_tile_depths", "csph_get_tile_depths",
    "csph_autotune",
    "csph_batch_autotune", "csph_set_scheme", "csph_get_scheme", "csph_stream_probe",
    "csph_create_static", "csph_set_viscosity", "csph_set_self_gravity", "csph_set_source",
    "csph_fill_state", "csph_set_state_box", "csph_get_state_box",
]


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double),
                ("origin", C.c_double * 3), ("gamma", C.c_double), ("cfl", C.c_double),
                ("rho_vac", C.c_double), ("dtype", C.c_int32)]


class CsphError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libcsph.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run paper_1912_04855_amd/build.py or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, dp, st = C.c_void_p, C.POINTER(C.c_double), C.c_int32
    sig = {
        "csph_required_bytes": (C.c_size_t, [C.POINTER(GridDesc)]),
        "csph_create": (st, [C.POINTER(GridDesc), vp, C.POINTER(vp)]),
        "csph_create_in": (st, [C.POINTER(GridDesc), vp, vp, C.c_size_t, C.POINTER(vp)]),
        "csph_create_static": (st, [C.POINTER(GridDesc), vp, C.POINTER(vp)]),
        "csph_set_viscosity": (st, [vp, C.c_double]),
        "csph_set_self_gravity": (st, [vp, C.c_double]),
        "csph_set_source": (st, [vp, vp, C.c_double]),
        "csph_fill_state": (st, [vp, C.c_int32, vp]),
        "csph_set_state_box": (st, [vp, C.c_int32, vp, vp, vp]),
        "csph_get_state_box": (st, [vp, C.c_int32, vp, vp, vp]),
        "csph_destroy": (st, [vp]),
        "csph_set_stream": (st, [vp, vp]),
        "csph_set_state": (st, [vp, C.c_int32, vp]),
        "csph_set_potential": (st, [vp, vp]),
        "csph_set_boundary": (st, [vp, C.c_int32, C.c_int32, vp]),
        "csph_step": (st, [vp, C.c_double, dp]),
        "csph_advance": (st, [vp, C.c_double, C.c_int64, C.POINTER(C.c_int64)]),
        "csph_get_state": (st, [vp, C.c_int32, vp]),
        "csph_get_time": (st, [vp, dp, C.POINTER(C.c_int64)]),
        "csph_set_time": (st, [vp, C.c_double, C.c_int64]),
        "csph_totals": (st, [vp, vp]),
        "csph_get_stage": (st, [vp, C.c_int32, vp]),
        "csph_last_error": (C.c_char_p, []),
        "csph_batch_create": (st, [C.c_int32, vp, C.c_size_t, C.POINTER(vp)]),
        "csph_batch_add": (st, [vp, vp, C.c_int64, C.c_double, C.POINTER(C.c_int32)]),
        "csph_batch_advance": (st, [vp, C.c_int32, C.POINTER(C.c_int32)]),
        "csph_batch_poll": (st, [vp, vp, C.c_int32, C.POINTER(C.c_int32)]),
        "csph_batch_remove": (st, [vp, C.c_int32]),
        "csph_batch_destroy": (st, [vp]),
        "csph_profile_enable": (st, [vp, C.c_int32]),
        "csph_profile_read": (st, [vp, vp, vp, C.c_int32]),
        "csph_set_tile_depth": (st, [vp, C.c_int32]),
        "csph_set_tile_depths": (st, [vp, C.POINTER(C.c_int32)]),
        "csph_get_tile_depths": (st, [vp, C.POINTER(C.c_int32)]),
        "csph_stream_probe": (st, [C.c_int32, C.c_int32, C.c_int64, C.c_int32, vp, dp]),
        "csph_autotune": (st, [vp, C.c_int32, C.POINTER(C.c_int32), dp]),
        "csph_batch_autotune": (st, [vp, C.c_int32, C.POINTER(C.c_int32), dp]),
        "csph_set_scheme": (st, [vp, C.c_int32, C.c_int32]),
        "csph_get_scheme": (st, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(code, where):
    if code != OK:
        msg = load().csph_last_error().decode(errors="replace")
        raise CsphError(code, where, msg)
