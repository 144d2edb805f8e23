"""ctypes declarations of the libsmc C ABI (include/smc.h).

Loads the in-tree ``libsmc.so``.  torch is imported first so that the HIP
runtime torch ships is the one the library binds to (both carry the soname
libamdhip64.so.7); device pointers and streams then come from torch.
There is no fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime before libsmc)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsmc.so")

SMC_OK, SMC_E_ARG, SMC_E_NONFINITE, SMC_E_DEGENERATE = 0, 1, 2, 3
SMC_E_NOMEM, SMC_E_DEVICE, SMC_E_UNSUPPORTED = 4, 5, 6
DTYPE_F32, DTYPE_F64 = 0, 1
TARGET_NONE, TARGET_GAUSS, TARGET_STUDENT, TARGET_LOGREG, TARGET_BEARING = 0, 1, 2, 3, 4
MODE_AUTO, MODE_FORCE, MODE_NEVER = 0, 1, 2
PREC_F64, PREC_BF16 = 0, 1

EXPORTS = ("smc_workspace_bytes", "smc_init", "smc_step", "smc_steps", "smc_sync_weights",
           "smc_resample", "smc_normalised_weights", "smc_redistribute",
           "smc_log_target", "smc_sync_error", "smc_destroy", "smc_status_string",
           "smc_batch_sampler_bytes", "smc_batch_workspace_bytes", "smc_batch_create",
           "smc_batch_attach", "smc_batch_detach", "smc_batch_step", "smc_batch_set_graph",
           "smc_batch_counts", "smc_batch_sync_error", "smc_batch_destroy",
           "smc_batch_particles", "smc_batch_set_group", "smc_resample_noalloc",
           "smc_batch_set_bucket_waves")
BATCH_DMAX, BATCH_EST_STRIDE = 64, 256
NOALLOC_MAX_N = 1 << 20


class SmcConfig(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("d", C.c_int32), ("x_dtype", C.c_int32), ("target", C.c_int32),
        ("mode", C.c_int32), ("ess_num", C.c_int32), ("ess_den", C.c_int32),
        ("sampler_id", C.c_uint32), ("loglik_precision", C.c_int32), ("seed", C.c_uint64),
        ("rw_sd", C.c_double), ("init_mean", C.c_double), ("init_sd", C.c_double),
        ("init_log_norm", C.c_double), ("log_norm", C.c_double),
        ("mean", C.c_void_p), ("prec", C.c_void_p), ("nu", C.c_double), ("mu", C.c_double),
        ("m_rows", C.c_int64), ("X", C.c_void_p), ("y", C.c_void_p), ("prior_prec", C.c_double),
        ("obs", C.c_void_p), ("n_obs", C.c_int32), ("lazy_reset", C.c_int32), ("delta", C.c_double),
        ("obs_var", C.c_double), ("obs_log_norm", C.c_double),
    ]


class SmcInfo(C.Structure):
    _fields_ = [
        ("m", C.c_double), ("logZ", C.c_double), ("ess", C.c_double), ("Z", C.c_double),
        ("Z2", C.c_double), ("S", C.c_uint64), ("U", C.c_uint64), ("Q2_hi", C.c_uint64),
        ("Q2_lo", C.c_uint64), ("K", C.c_int32), ("resampled", C.c_int32), ("err", C.c_int32),
        ("pad", C.c_int32), ("log_c", C.c_double),
    ]


INFO_BYTES = C.sizeof(SmcInfo)


class SmcBatchSampler(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("d", C.c_int32), ("mode", C.c_int32), ("ess_num", C.c_int32),
        ("ess_den", C.c_int32), ("sampler_id", C.c_uint32), ("pad0", C.c_int32),
        ("seed", C.c_uint64), ("rw_sd", C.c_double), ("init_mean", C.c_double),
        ("init_sd", C.c_double), ("init_log_norm", C.c_double), ("log_norm", C.c_double),
        ("mean", C.c_void_p), ("chol", C.c_void_p), ("x", C.c_void_p), ("logw", C.c_void_p),
        ("ws", C.c_void_p), ("ws_bytes", C.c_size_t),
    ]


class SmcError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s: %s (status %d)" % (where, status_string(code), code))


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsmc.so is not built (run paper_1905_10252_amd/build.py): %s"
                          % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, P = C.c_void_p, C.POINTER
    L.smc_workspace_bytes.argtypes = [P(SmcConfig)]
    L.smc_workspace_bytes.restype = C.c_size_t
    L.smc_init.argtypes = [P(vp), P(SmcConfig), vp, C.c_size_t, vp, vp, vp]
    L.smc_step.argtypes = [vp, vp, vp, vp, vp, vp]
    L.smc_steps.argtypes = [vp, vp, vp, C.c_int32, vp, vp, vp]
    L.smc_sync_weights.argtypes = [vp, vp, vp]
    L.smc_normalised_weights.argtypes = [vp, vp, C.c_int64, vp, vp]
    L.smc_resample.argtypes = [vp, vp, C.c_int64, C.c_uint64, C.c_int32, vp, vp, vp]
    L.smc_resample_noalloc.argtypes = [vp, C.c_int64, C.c_uint64, C.c_int32, C.c_int32,
                                       C.c_int32, vp, vp, vp]
    L.smc_redistribute.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int32, vp, vp, vp]
    L.smc_log_target.argtypes = [vp, vp, C.c_int64, vp, vp]
    L.smc_sync_error.argtypes = [vp, vp]
    L.smc_destroy.argtypes = [vp]
    L.smc_status_string.argtypes = [C.c_int]
    L.smc_status_string.restype = C.c_char_p
    for f in ("smc_init", "smc_step", "smc_steps", "smc_sync_weights", "smc_resample",
              "smc_resample_noalloc",
              "smc_normalised_weights", "smc_redistribute",
              "smc_log_target", "smc_sync_error", "smc_destroy"):
        getattr(L, f).restype = C.c_int
    L.smc_batch_sampler_bytes.argtypes = [P(SmcBatchSampler)]
    L.smc_batch_sampler_bytes.restype = C.c_size_t
    L.smc_batch_workspace_bytes.argtypes = [C.c_int32]
    L.smc_batch_workspace_bytes.restype = C.c_size_t
    L.smc_batch_create.argtypes = [P(vp), C.c_int32, vp, C.c_size_t, vp]
    L.smc_batch_attach.argtypes = [vp, C.c_int32, P(SmcBatchSampler), vp]
    L.smc_batch_detach.argtypes = [vp, C.c_int32, vp]
    L.smc_batch_step.argtypes = [vp, vp, vp, vp]
    L.smc_batch_set_graph.argtypes = [vp, C.c_int32]
    L.smc_batch_counts.argtypes = [vp, P(C.c_int32), P(C.c_int64)]
    L.smc_batch_particles.argtypes = [vp, C.c_int32, P(vp), P(vp), vp]
    L.smc_batch_set_group.argtypes = [vp, C.c_int32, vp]
    L.smc_batch_set_bucket_waves.argtypes = [vp, C.c_int32, C.c_int32]
    L.smc_batch_sync_error.argtypes = [vp, C.c_int32, vp]
    L.smc_batch_destroy.argtypes = [vp]
    for f in ("smc_batch_create", "smc_batch_attach", "smc_batch_detach", "smc_batch_step",
              "smc_batch_set_graph", "smc_batch_counts", "smc_batch_sync_error",
              "smc_batch_destroy", "smc_batch_particles", "smc_batch_set_group",
              "smc_batch_set_bucket_waves"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def status_string(code: int) -> str:
    return load().smc_status_string(code).decode()


def check(code: int, where: str) -> None:
    if code != SMC_OK:
        raise SmcError(code, where)
