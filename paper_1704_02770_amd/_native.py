"""Loads libqkrylov.so (built in-tree) and declares the C signatures of include/qk.h.

torch is imported first so that the HIP runtime it ships is the one the
library binds to (both carry the soname libamdhip64.so.7); device pointers
and streams handed over from torch are then valid in the library.
There is no fallback: a missing library raises at import.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime before the library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqkrylov.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1704_02770_amd/build.py` (run by path from the repository root)")

lib = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)

i32, i64, f64, vp = C.c_int32, C.c_int64, C.c_double, C.c_void_p
P = C.POINTER


class HamParams(C.Structure):
    _fields_ = [("jxy", f64), ("jz", f64), ("pbc", i32), ("mode", i32)]


class KernelTime(C.Structure):
    _fields_ = [("ms_total", f64), ("launches", i64)]


class LaunchShape(C.Structure):
    _fields_ = [("threads", i32), ("blocks_per_cu", i32), ("blocked_wgs_per_cu", i32), ("blocked_llo", i32)]


class AdaptParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("dt_init", C.c_double), ("dt_max", C.c_double), ("max_steps", C.c_int32)]


class AdaptInfo(C.Structure):
    _fields_ = [("steps", C.c_int32), ("dt_min", C.c_double), ("dt_max", C.c_double), ("err_sum", C.c_double)]


class StepInfo(C.Structure):
    _fields_ = [("m_used", i32), ("status", i32), ("err_est", f64), ("beta0", f64)]


# device-memory callbacks of qk_set_allocator
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

# name -> (restype, argtypes); every symbol include/qk.h declares
SIGNATURES = {
    "qk_abi_version": (C.c_int, []),
    "qk_set_allocator": (i32, [ALLOC_FN, RELEASE_FN, vp]),
    "qk_last_error": (C.c_char_p, []),
    "qk_fields_quasiperiodic": (i32, [i32, f64, f64, P(f64), i32, P(f64)]),
    "qk_basis_build": (i32, [i32, i32, vp, P(vp)]),
    "qk_basis_dim": (i32, [vp, P(i64)]),
    "qk_basis_shape": (i32, [vp, P(i32), P(i32)]),
    "qk_basis_states": (i32, [vp, vp, vp]),
    "qk_basis_rank": (i32, [vp, P(C.c_uint64), i64, P(i64)]),
    "qk_basis_destroy": (None, [vp]),
    "qk_ham_create": (i32, [vp, P(HamParams), P(f64), i32, vp, P(vp)]),
    "qk_ham_set_fields": (i32, [vp, P(f64), i32, vp]),
    "qk_ham_get_fields": (i32, [vp, P(f64), i32]),
    "qk_ham_shape": (i32, [vp, P(i64), P(i32), P(i32)]),
    "qk_ham_apply": (i32, [vp, vp, vp, i32, vp]),
    "qk_ham_destroy": (None, [vp]),
    "qk_krylov_create": (i32, [vp, i32, i32, i32, P(vp)]),
    "qk_krylov_expm_step": (i32, [vp, vp, f64, vp, P(StepInfo)]),
    "qk_krylov_evolve": (i32, [vp, vp, f64, P(AdaptParams), vp, P(AdaptInfo)]),
    "qk_krylov_coefficients": (i32, [vp, i32, P(f64), P(f64), P(i32)]),
    "qk_krylov_destroy": (None, [vp]),
    "qk_krylov_profile": (i32, [vp, i32]),
    "qk_krylov_profile_read": (i32, [vp, P(KernelTime)]),
    "qk_krylov_set_shape": (i32, [vp, P(LaunchShape)]),
    "qk_krylov_get_shape": (i32, [vp, P(LaunchShape)]),
    "qk_krylov_autotune": (i32, [vp, f64, C.c_char_p, vp, P(LaunchShape)]),
    "qk_batch_create": (i32, [P(vp), P(vp), P(i64), i32, P(vp)]),
    "qk_batch_items": (i32, [vp, P(i32)]),
    "qk_batch_run": (i32, [vp, f64, i32, i32, vp, vp]),
    "qk_batch_run_autocorr": (i32, [vp, f64, i32, i32, vp, vp, vp]),
    "qk_batch_destroy": (None, [vp]),
    "qk_grad_return_prob": (i32, [vp, i64, f64, i32, i32, P(f64), P(f64), vp]),
    "qk_return_prob": (i32, [vp, i64, vp, vp, i32, i32, vp, vp]),
    "qk_return_prob_noalloc": (i32, [vp, i64, vp, vp, i32, i32, vp, vp]),
}

for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args
