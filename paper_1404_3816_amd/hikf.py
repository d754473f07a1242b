"""ctypes binding of the C ABI in include/hikf.h and include/hikf_enkf.h
(argument marshalling only).

Every function keeps its C name and signature; device pointers are passed
as integers (``tensor.data_ptr()``) and streams as raw ``hipStream_t``
handles (``torch.cuda.current_stream().cuda_stream``).  All computation
happens in libhikf.so; importing this module fails loudly if the library
has not been built.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhikf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1404_3816_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

# status codes
HIKF_OK = 0
HIKF_E_INVALID = 1
HIKF_E_UNSUPPORTED = 2
HIKF_E_NOMEM = 3
HIKF_E_NOT_SPD = 4
HIKF_E_DEVICE = 5
# kernel families
HIKF_KERNEL_POWEXP = 0
HIKF_KERNEL_TEST_R2 = 1
# priors
HIKF_PRIOR_ZERO = 0
HIKF_PRIOR_SCALED_I = 1
HIKF_PRIOR_KERNEL = 2
# FMM precision
HIKF_FMM_F32 = 0
HIKF_FMM_F64 = 1
HIKF_FMM_BF16X3 = 2
HIKF_FMM_BF16 = 3
# size of the fixed workspace of hikf_cov_apply_noalloc
HIKF_NOALLOC_SCRATCH_BYTES = 32 << 20

c_i32, c_i64, c_dbl, c_vp, c_sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                   ctypes.c_void_p, ctypes.c_size_t)


class hikf_problem(ctypes.Structure):
    _fields_ = [
        ("dim", c_i32), ("n", c_i32), ("kernel_family", c_i32), ("prior_kind", c_i32),
        ("theta", c_dbl), ("ell", c_dbl), ("gamma", c_dbl), ("alpha", c_dbl),
        ("p", c_i32), ("reserved0", c_i32), ("nnz", c_i64),
        ("h_rowptr_dev", c_vp), ("h_col_dev", c_vp), ("h_val_dev", c_vp),
        ("r_diag_dev", c_vp), ("x0_dev", c_vp),
    ]


class hikf_options(ctypes.Structure):
    _fields_ = [("n_c", c_i32), ("fmm_precision", c_i32), ("direct", c_i32),
                ("timing", c_i32), ("riccati", c_i32), ("history", c_i32), ("graph", c_i32),
                ("sparse", c_i32), ("rowpass_variant", c_i32), ("reserved1", c_i32),
                ("tune_cache", ctypes.c_char_p), ("psd_guard", c_i32), ("reserved4", c_i32),
                ("m2l_eps", c_dbl)]


class hikf_plan_info(ctypes.Structure):
    _fields_ = [("resident_bytes", c_sz), ("scratch_bytes", c_sz), ("m", c_i64),
                ("depth", c_i32), ("r", c_i32), ("near_pairs", c_i64), ("far_pairs", c_i64),
                ("query_bytes", c_sz), ("rowpass_variant", c_i32), ("reserved3", c_i32)]


HIKF_NUM_PHASES = 12
PHASES = ("operators", "p2m", "m2m", "m2l", "l2l", "p2p", "init", "gather", "reduce",
          "pspace", "rowpass", "output")


class hikf_stats(ctypes.Structure):
    _fields_ = [("steps_applied", c_i64), ("last_status", c_i32), ("init_status", c_i32),
                ("min_pivot", c_dbl), ("negative_variances", c_i64),
                ("time_ms", c_dbl * HIKF_NUM_PHASES),
                ("time_count", c_i64 * HIKF_NUM_PHASES),
                ("rowpass_variant", c_i32), ("reserved2", c_i32),
                ("riccati_drift_g", c_dbl), ("riccati_drift_h", c_dbl),
                ("riccati_checks", c_i64), ("m2l_ranks", c_i32 * 20)]


class hikf_checkpoint_info(ctypes.Structure):
    _fields_ = [("problem_hash", ctypes.c_uint64), ("steps_applied", c_i64),
                ("steps_issued", c_i64), ("p", c_i32), ("carried", c_i32)]


class hikf_enkf_problem(ctypes.Structure):
    _fields_ = [("m", c_i64), ("p", c_i32), ("n_ens", c_i32), ("nnz", c_i64),
                ("h_rowptr_dev", c_vp), ("h_col_dev", c_vp), ("h_val_dev", c_vp),
                ("r_diag_dev", c_vp), ("timing", c_i32), ("tile_rows", c_i32)]


class hikf_enkf_plan_info(ctypes.Structure):
    _fields_ = [("resident_bytes", c_sz), ("ld", c_i32), ("gather_chunks", c_i32)]


HIKF_ENKF_PHASE_GATHER = 0
HIKF_ENKF_PHASE_NSPACE = 1
HIKF_ENKF_PHASE_TRANSFORM = 2
HIKF_ENKF_NUM_PHASES = 4


class hikf_enkf_stats(ctypes.Structure):
    _fields_ = [("steps_applied", c_i64), ("last_status", c_i32), ("init_status", c_i32),
                ("min_pivot", c_dbl), ("time_ms", c_dbl * HIKF_ENKF_NUM_PHASES),
                ("time_count", c_i64 * HIKF_ENKF_NUM_PHASES)]


_P = ctypes.POINTER

_SIGS = {
    "hikf_plan": (c_i32, [_P(hikf_problem), _P(hikf_options), _P(hikf_plan_info)]),
    "hikf_init": (c_i32, [_P(hikf_problem), _P(hikf_options), c_vp, c_sz, c_vp, c_sz, c_vp,
                          _P(c_vp)]),
    "hikf_step": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "hikf_step_batch": (c_i32, [_P(c_vp), _P(c_vp), _P(c_vp), _P(c_vp), c_i32, c_vp]),
    "hikf_cov_apply": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "hikf_cov_apply_noalloc": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "hikf_query": (c_i32, [c_vp, _P(hikf_stats)]),
    "hikf_export_state": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "hikf_import_state": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "hikf_export_checkpoint": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp,
                                       _P(hikf_checkpoint_info), c_vp]),
    "hikf_import_checkpoint": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp,
                                       _P(hikf_checkpoint_info), c_vp]),
    "hikf_export_cq": (c_i32, [c_vp, c_vp, c_vp]),
    "hikf_destroy": (None, [c_vp]),
    "hikf_status_string": (ctypes.c_char_p, [c_i32]),
    "hikf_last_error": (ctypes.c_char_p, [c_vp]),
    # include/hikf_enkf.h
    "hikf_enkf_plan": (c_i32, [_P(hikf_enkf_problem), _P(hikf_enkf_plan_info)]),
    "hikf_enkf_init": (c_i32, [_P(hikf_enkf_problem), c_vp, c_vp, c_sz, c_vp, _P(c_vp)]),
    "hikf_enkf_step": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "hikf_enkf_query": (c_i32, [c_vp, _P(hikf_enkf_stats)]),
    "hikf_enkf_export": (c_i32, [c_vp, c_vp, c_vp]),
    "hikf_enkf_import": (c_i32, [c_vp, c_vp, c_vp]),
    "hikf_enkf_destroy": (None, [c_vp]),
    "hikf_enkf_last_error": (ctypes.c_char_p, [c_vp]),
}

EXPORTED = tuple(_SIGS)

for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

hikf_plan = _lib.hikf_plan
hikf_init = _lib.hikf_init
hikf_step = _lib.hikf_step
hikf_step_batch = _lib.hikf_step_batch
hikf_cov_apply = _lib.hikf_cov_apply
hikf_cov_apply_noalloc = _lib.hikf_cov_apply_noalloc
hikf_query = _lib.hikf_query
hikf_export_state = _lib.hikf_export_state
hikf_import_state = _lib.hikf_import_state
hikf_export_checkpoint = _lib.hikf_export_checkpoint
hikf_import_checkpoint = _lib.hikf_import_checkpoint
hikf_export_cq = _lib.hikf_export_cq
hikf_destroy = _lib.hikf_destroy
hikf_status_string = _lib.hikf_status_string
hikf_last_error = _lib.hikf_last_error
hikf_enkf_plan = _lib.hikf_enkf_plan
hikf_enkf_init = _lib.hikf_enkf_init
hikf_enkf_step = _lib.hikf_enkf_step
hikf_enkf_query = _lib.hikf_enkf_query
hikf_enkf_export = _lib.hikf_enkf_export
hikf_enkf_import = _lib.hikf_enkf_import
hikf_enkf_destroy = _lib.hikf_enkf_destroy
hikf_enkf_last_error = _lib.hikf_enkf_last_error


class HikfError(RuntimeError):
    def __init__(self, status, where, detail=b""):
        msg = hikf_status_string(status).decode()
        if detail:
            msg += f" ({detail.decode(errors='replace')})"
        super().__init__(f"{where}: {msg}")
        self.status = status


def check(status, where, handle=None):
    """Raise HikfError for a non-OK status."""
    if status != HIKF_OK:
        raise HikfError(status, where, hikf_last_error(handle) if handle else b"")
    return status
