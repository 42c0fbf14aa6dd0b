"""ctypes binding of libhf (argument marshalling only).

Every step of the pass runs in the HIP library; this module converts torch
tensors to device pointers and the current HIP stream, and raises on errors.
There is no fallback: without the built library, or without a gfx950 GPU, the
calls fail.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhf.so")

HF_OK, HF_ERR_INVALID, HF_ERR_NOMEM, HF_ERR_CAPACITY, HF_ERR_DEVICE, HF_ERR_UNSUPPORTED = range(6)
HF_OPT_RADIUS_SEARCH = 1
HF_RADIUS_HISTOGRAM, HF_RADIUS_BINS = 0, 1
STATUS = {0: "HF_OK", 1: "HF_ERR_INVALID", 2: "HF_ERR_NOMEM", 3: "HF_ERR_CAPACITY",
          4: "HF_ERR_DEVICE", 5: "HF_ERR_UNSUPPORTED"}

EXPORTS = ["hf_default_params", "hf_params_at_redshift", "hf_derived", "hf_create", "hf_destroy", "hf_last_error",
           "hf_get_stats", "hf_set_option", "hf_get_option", "hf_density", "hf_l0_fof", "hf_compaso", "hf_find", "hf_find_noalloc", "hf_find_grouped",
           "hf_count_pairs", "hf_halo_stats",
           "hf_find_batch", "hf_tune_batch", "hf_load_tuning", "hf_batch_groups",
           "hf_server_create", "hf_server_submit", "hf_server_wait",
           "hf_server_now", "hf_server_held_bytes", "hf_server_last_error", "hf_server_destroy"]


class HfParams(ctypes.Structure):
    _fields_ = [("box", ctypes.c_double), ("mean_density", ctypes.c_double),
                ("b_kernel", ctypes.c_double), ("l_fof", ctypes.c_double),
                ("delta_l0_min", ctypes.c_double), ("delta_l1", ctypes.c_double),
                ("delta_l2", ctypes.c_double),
                ("alpha_elig", ctypes.c_double), ("c_roche", ctypes.c_double),
                ("n_new_min", ctypes.c_double), ("particle_mass", ctypes.c_double),
                ("n_l1_min", ctypes.c_int32), ("self_count", ctypes.c_int32)]


class HfHalo(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int32), ("nucleus", ctypes.c_int32), ("l0_id", ctypes.c_int32),
                ("n", ctypes.c_int32), ("n_enclosed", ctypes.c_int32), ("x", ctypes.c_float),
                ("y", ctypes.c_float), ("z", ctypes.c_float), ("r", ctypes.c_float),
                ("mass", ctypes.c_float)]


class HfStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_float) for k in
                ("ms_bin", "ms_density", "ms_fof", "ms_segment", "ms_candidates", "ms_accept",
                 "ms_assign", "ms_output", "ms_total")] + \
               [(k, ctypes.c_int64) for k in
                ("n_cells", "n_members", "n_groups", "n_candidates", "n_found", "n_halos",
                 "n_dense_cells", "n_dense_chunks", "n_sparse", "n_hard")]


class HfHaloSummary(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int32), ("n", ctypes.c_int32), ("n_l2", ctypes.c_int32),
                ("l2max_nucleus", ctypes.c_int32), ("l2max_n", ctypes.c_int32),
                ("x_com", ctypes.c_float * 3), ("x_l2com", ctypes.c_float * 3),
                ("l2_mass", ctypes.c_float * 5), ("r_pct", ctypes.c_float * 9),
                ("vcirc_max", ctypes.c_float), ("rvcirc_max", ctypes.c_float)]


PCT = [10, 25, 33, 50, 67, 75, 90, 95, 98]   # the r_XX of hf_halo_summary.r_pct


class HfRequest(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("n", ctypes.c_int64), ("params", HfParams),
                ("density", ctypes.c_void_p), ("l0_id", ctypes.c_void_p),
                ("halo_id", ctypes.c_void_p), ("halos", ctypes.c_void_p),
                ("halos_cap", ctypes.c_int64)]


class HfResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("slot", ctypes.c_int32), ("n_halos", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("ms_gpu", ctypes.c_float),
                ("error", ctypes.c_char * 160)]


HALO_FIELDS = [f[0] for f in HfHalo._fields_]
HALO_WORDS = ctypes.sizeof(HfHalo) // 4   # 10 x 32-bit words per row

_lib = None


class HfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libhf.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_2110_11408_amd/build.py")
        lib = ctypes.CDLL(path)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        PP = ctypes.POINTER(HfParams)
        lib.hf_default_params.argtypes = [PP]
        lib.hf_default_params.restype = None
        lib.hf_derived.argtypes = [PP, I64, P]
        lib.hf_params_at_redshift.argtypes = [PP, ctypes.c_double, ctypes.c_double, PP]
        lib.hf_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), I32, ctypes.c_uint64]
        lib.hf_destroy.argtypes = [P]
        lib.hf_destroy.restype = None
        lib.hf_last_error.argtypes = [P]
        lib.hf_last_error.restype = ctypes.c_char_p
        lib.hf_get_stats.argtypes = [P, ctypes.POINTER(HfStats)]
        lib.hf_set_option.argtypes = [P, ctypes.c_int32, I64]
        lib.hf_get_option.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
        lib.hf_density.argtypes = [P, P, I64, PP, P, P]
        lib.hf_l0_fof.argtypes = [P, P, P, I64, PP, P, P, P]
        lib.hf_compaso.argtypes = [P, P, P, P, I64, PP, P, P, I64, P, P]
        lib.hf_find.argtypes = [P, P, I64, PP, P, P, P, P, I64, P, P]
        lib.hf_find_noalloc.argtypes = [P, P, I64, PP, P, P, P, P, I64, P, P]
        lib.hf_find_grouped.argtypes = [P, P, I64, PP, P, P, P, P, I64, P, P, P, P]
        lib.hf_count_pairs.argtypes = [P, P, I64, PP, P, P]
        lib.hf_halo_stats.argtypes = [P, P, P, P, I64, PP, I64, P, P, P, P]
        lib.hf_find_batch.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P, P, P, P, ctypes.c_int32, P]
        lib.hf_tune_batch.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P, P, P, P, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_float), P]
        lib.hf_load_tuning.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]
        lib.hf_batch_groups.argtypes = [P, ctypes.c_int32, I64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        lib.hf_server_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), I32, ctypes.c_int32,
                                         ctypes.c_uint64]
        lib.hf_server_submit.argtypes = [P, ctypes.POINTER(HfRequest), ctypes.POINTER(ctypes.c_int64)]
        lib.hf_server_wait.argtypes = [P, ctypes.c_int64, ctypes.POINTER(HfResult)]
        lib.hf_server_now.argtypes = [P]
        lib.hf_server_now.restype = ctypes.c_double
        lib.hf_server_held_bytes.argtypes = [P]
        lib.hf_server_held_bytes.restype = ctypes.c_uint64
        lib.hf_server_last_error.argtypes = [P]
        lib.hf_server_last_error.restype = ctypes.c_char_p
        lib.hf_server_destroy.argtypes = [P]
        lib.hf_server_destroy.restype = None
        for name in ("hf_derived", "hf_params_at_redshift", "hf_create", "hf_get_stats", "hf_set_option",
                     "hf_get_option", "hf_density", "hf_l0_fof",
                     "hf_compaso", "hf_find", "hf_find_noalloc", "hf_find_grouped", "hf_count_pairs", "hf_halo_stats", "hf_find_batch",
                     "hf_tune_batch", "hf_load_tuning", "hf_batch_groups",
                     "hf_server_create", "hf_server_submit", "hf_server_wait"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def default_params(**kw) -> HfParams:
    p = HfParams()
    load().hf_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def params_at_redshift(p: HfParams, omega_m0: float, z: float) -> HfParams:
    """hf_params_at_redshift: thresholds scaled to redshift z."""
    out = HfParams()
    st = load().hf_params_at_redshift(ctypes.byref(p), float(omega_m0), float(z), ctypes.byref(out))
    if st:
        raise HfError(st, "invalid cosmology")
    return out


def derived(p: HfParams, n: int) -> dict:
    out = (ctypes.c_double * 11)()
    st = load().hf_derived(ctypes.byref(p), int(n), out)
    if st:
        raise HfError(st, "invalid parameters")
    names = ["nbar", "b", "l", "b2", "l2", "norm", "K", "K2", "floor", "A6", "C3"]
    return dict(zip(names, list(out)))
