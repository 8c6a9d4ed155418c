"""ctypes binding of libabs.so (include/abs.h).  Argument marshalling only: every
step of the estimator runs in the library's HIP kernels.  PyTorch supplies device
memory and streams.  There is no fallback: if the library is missing, loading fails."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libabs.so")

OK, ERR_INVALID, ERR_ALIAS, ERR_UNBOUND, ERR_DEVICE, ERR_JIT, ERR_NOMEM, ERR_EMPTY, ERR_SCRATCH = range(9)
FP32, BF16X3, FP16X3 = 0, 1, 2
W_UNIT, W_INV_COUNT, W_GIVEN = 0, 1, 2
C64, C128 = 0, 1
NEAREST, GAUSS7 = 0, 1
STAGE_CONTRACT, STAGE_COLPASS, STAGE_ROWPASS, STAGE_GRID = 0, 1, 2, 3
ALLOW_WRAP, ALLOW_DC, EVERY_LEVEL, ALL_MFMA = 1, 2, 4, 8
BEAM_NONE, BEAM_MWA, BEAM_GAUSS = 0, 1, 2


class PlanDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nbins", ctypes.c_int32),
                ("edges", ctypes.POINTER(ctypes.c_double)), ("du", ctypes.c_double),
                ("norm", ctypes.c_double), ("theta0", ctypes.c_double),
                ("precision", ctypes.c_int32), ("wmode", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("flags", ctypes.c_uint32), ("levels", ctypes.c_int32),
                ("nchan", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nbins", ctypes.c_int32), ("ntrip", ctypes.c_int64),
                ("npairs", ctypes.c_int64), ("ncols", ctypes.c_int64),
                ("plan_bytes", ctypes.c_int64), ("norm", ctypes.c_double),
                ("mfma_tiles", ctypes.c_int64), ("jit_parts", ctypes.c_int32),
                ("contract_parts", ctypes.c_int32), ("contract_jk", ctypes.c_int32),
                ("contract_block", ctypes.c_int32), ("contract_waves", ctypes.c_int32),
                ("weight_parts", ctypes.c_int32), ("weight_jk", ctypes.c_int32),
                ("weight_block", ctypes.c_int32), ("weight_waves", ctypes.c_int32),
                ("mfma_tiles_per_wave", ctypes.c_int32), ("mfma_depth", ctypes.c_int32),
                ("nlevels", ctypes.c_int32), ("ring0", ctypes.c_int32), ("nchan", ctypes.c_int32)]


class AbsError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s (status %d)" % (where, status_str(status), status))


_lib = None
_P = ctypes.c_void_p


def lib():
    """Load libabs.so once.  torch is imported first so that the library binds to the
    HIP runtime torch already loaded (one runtime per process)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime first)
    if not os.path.exists(LIB_PATH):
        raise ImportError("libabs.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, sz, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    sig = {
        "abs_plan": [ctypes.POINTER(PlanDesc), ctypes.POINTER(_P)],
        "abs_plan_info_get": [_P, ctypes.POINTER(PlanInfo)],
        "abs_plan_level_info": [_P, i32, ctypes.POINTER(PlanInfo), _P],
        "abs_plan_triplets": [_P, _P, _P, _P],
        "abs_plan_compile": [_P],
        "abs_plan_compile_part": [_P, i32],
        "abs_plan_code": [_P, i32, ctypes.POINTER(ctypes.c_uint64), _P, ctypes.POINTER(sz)],
        "abs_plan_set_code": [_P, i32, ctypes.c_uint64, _P, sz],
        "abs_plan_bind": [_P, _P, sz, _P],
        "abs_estimate_workspace": [_P, i32, i32, i32, ctypes.POINTER(sz)],
        "abs_grid_workspace": [_P, i64, i32, ctypes.POINTER(sz)],
        "abs_grid": [_P, i64, i32, _P, _P, _P, i32, _P, sz, _P, _P, _P, _P],
        "abs_grid_sort_workspace": [_P, i64, ctypes.POINTER(sz), ctypes.POINTER(sz)],
        "abs_grid_sort": [_P, i64, _P, _P, sz, _P, sz, _P, _P, _P, _P],
        "abs_grid_permute": [_P, i64, i32, _P, i64, _P, _P, _P],
        "abs_grid_sorted": [_P, _P, sz, i32, i64, _P, _P, _P, _P],
        "abs_estimate": [_P, i32, i32, _P, _P, i32, _P, _P, sz, _P, _P, _P],
        "abs_estimate_noalloc": [_P, i32, i32, _P, _P, i32, _P, _P, _P, _P],
        "abs_estimate_complex_workspace": [_P, i32, i32, i32, ctypes.POINTER(sz)],
        "abs_estimate_complex": [_P, i32, i32, _P, _P, i32, _P, _P, sz, _P, _P, _P],
        "abs_counts": [_P, _P, _P, sz, _P, _P],
        "abs_rebin_table": [_P, i32, _P, i32, i32, _P],
        "abs_rebin": [_P, i32, _P, i32, _P, _P, _P, _P, _P],
        "abs_ensemble": [i32, i32, _P, _P, _P, _P, _P, _P, _P],
        "abs_model_workspace": [_P, ctypes.POINTER(sz)],
        "abs_model_discrete": [_P, _P, _P, dbl, _P, sz, _P, _P],
        "abs_simulate_workspace": [i32, ctypes.POINTER(sz)],
        "abs_simulate": [i32, dbl, i32, dbl, dbl, i32, _P, i64, _P, _P, _P, sz, _P],
        "abs_sync": [_P, _P],
        "abs_profile": [_P, i32, _P, _P],
        "abs_destroy": [_P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.abs_status_str.argtypes = [ctypes.c_int]
    L.abs_status_str.restype = ctypes.c_char_p
    _lib = L
    return L


def status_str(s):
    try:
        return lib().abs_status_str(int(s)).decode()
    except Exception:
        return "status %d" % s


def check(s, where):
    if s != OK:
        raise AbsError(s, where)
