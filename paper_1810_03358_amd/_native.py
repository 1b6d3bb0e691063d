"""ctypes declarations of the C ABI in include/ff.h and include/ff_learn.h
(libff_mi355x.so)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libff_mi355x.so")

FF_OK, FF_ERR_ARG, FF_ERR_HIP, FF_ERR_WORKSPACE, FF_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
FF_GD, FF_FGM, FF_CG, FF_LBFGS, FF_HB, FF_OGM = 0, 1, 2, 3, 4, 5
FF_FP64, FF_FP32_ACC64 = 0, 1
FF_CONVERGED, FF_MAX_ITER, FF_LS_FAILED, FF_NONFINITE_START, FF_DIVERGED = 0, 1, 2, 3, 4
FF_LS_DEFAULT, FF_LS_PAR, FF_LS_H = -1, 0, 1
FF_MIN_RESUME, FF_MIN_NO_CERTIFY = 1, 2
FF_CG_PRP, FF_CG_FR, FF_CG_HS, FF_CG_PRP_PLUS, FF_CG_CD, FF_CG_LS, FF_CG_DY = 0, 1, 2, 3, 4, 5, 6
FF_NOALLOC_SCRATCH_BYTES = 128 << 20

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class FFSystem(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32), ("q", _dp), ("sigma", _dp), ("eps", _dp),
        ("n_bonds", C.c_int32), ("bond", _ip), ("bond_k", _dp), ("bond_r0", _dp),
        ("n_angles", C.c_int32), ("angle", _ip), ("angle_k", _dp), ("angle_t0", _dp),
        ("n_dihedrals", C.c_int32), ("dihedral", _ip), ("dihedral_v", _dp),
        ("coulomb_c", C.c_double),
    ]


class FFMinParams(C.Structure):
    _fields_ = [
        ("method", C.c_int32), ("m", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32),
        ("precision", C.c_int32), ("linesearch", C.c_int32), ("ls_K", C.c_int32),
        ("h_init", C.c_double), ("k_plus", C.c_double), ("k_minus", C.c_double), ("eps_h", C.c_double),
        ("cg_restart", C.c_int32), ("flags", C.c_int32), ("cg_beta", C.c_int32), ("ls_par_g0", C.c_int32),
        ("fgm_restart", C.c_int32), ("hb_alpha", C.c_double), ("hb_beta", C.c_double),
    ]


class FFMinResult(C.Structure):
    _fields_ = [
        ("term", C.c_int32), ("iters", C.c_int32), ("evals", C.c_int32), ("evals_fp64", C.c_int32),
        ("energy", C.c_double), ("grad_inf", C.c_double), ("grad_2", C.c_double),
    ]


EXPORTS = ("ff_workspace_bytes", "ff_workspace_bytes_batch", "ff_create", "ff_create_batch", "ff_batch_size",
           "ff_destroy", "ff_energy_grad", "ff_minimize", "ff_get_trace", "ff_time_pair", "ff_default_params",
           "ff_last_error", "ff_num_tile_configs", "ff_tile_config_info", "ff_workspace_bytes_tiled",
           "ff_create_tiled", "ff_get_tiling", "ff_autotune_workspace_bytes", "ff_autotune", "ff_energy_profile",
           "ff_energy_grad_noalloc")

LEARN_EXPORTS = ("ff_learn_param_count", "ff_learn_workspace_bytes", "ff_learn_last_error", "ff_learn_features",
                 "ff_learn_gemm", "ff_learn_forward", "ff_learn_backward", "ff_learn_adam", "ff_learn_to_bf16",
                 "ff_learn_delta", "ff_learn_gather_rows", "ff_learn_displace", "ff_learn_select")
FF_LEARN_NEIGHBORS, FF_LEARN_FEATURES, FF_LEARN_HIDDEN, FF_LEARN_OUT_PAD = 16, 128, 128, 16

_lib = None


def load():
    """Load the HIP library; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1810_03358_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    lib.ff_workspace_bytes.argtypes = [C.POINTER(FFSystem), C.c_int32]
    lib.ff_workspace_bytes.restype = C.c_size_t
    lib.ff_create.argtypes = [C.POINTER(FFSystem), C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p,
                              C.POINTER(C.c_void_p)]
    lib.ff_create.restype = C.c_int
    lib.ff_workspace_bytes_batch.argtypes = [C.POINTER(FFSystem), C.c_int32, C.c_int32]
    lib.ff_workspace_bytes_batch.restype = C.c_size_t
    lib.ff_create_batch.argtypes = [C.POINTER(FFSystem), C.c_int32, C.c_void_p, C.c_size_t, C.c_int32,
                                    C.c_void_p, C.POINTER(C.c_void_p)]
    lib.ff_create_batch.restype = C.c_int
    lib.ff_batch_size.argtypes = [C.c_void_p]
    lib.ff_batch_size.restype = C.c_int32
    lib.ff_destroy.argtypes = [C.c_void_p]
    lib.ff_destroy.restype = C.c_int
    lib.ff_energy_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    lib.ff_energy_grad.restype = C.c_int
    lib.ff_energy_grad_noalloc.argtypes = [C.POINTER(FFSystem), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                           C.c_void_p]
    lib.ff_energy_grad_noalloc.restype = C.c_int
    lib.ff_minimize.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(FFMinParams), C.POINTER(FFMinResult),
                                C.c_void_p]
    lib.ff_minimize.restype = C.c_int
    lib.ff_get_trace.argtypes = [C.c_void_p, _dp, C.c_int32, C.c_void_p]
    lib.ff_get_trace.restype = C.c_int32
    lib.ff_time_pair.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, _dp]
    lib.ff_time_pair.restype = C.c_int
    lib.ff_default_params.argtypes = [C.POINTER(FFMinParams)]
    lib.ff_default_params.restype = None
    _ip = C.POINTER(C.c_int32)
    lib.ff_num_tile_configs.argtypes = []
    lib.ff_num_tile_configs.restype = C.c_int32
    lib.ff_tile_config_info.argtypes = [C.c_int32, _ip, _ip, _ip, _ip, _ip]
    lib.ff_tile_config_info.restype = C.c_int
    lib.ff_workspace_bytes_tiled.argtypes = [C.POINTER(FFSystem), C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                             C.c_int32]
    lib.ff_workspace_bytes_tiled.restype = C.c_size_t
    lib.ff_create_tiled.argtypes = [C.POINTER(FFSystem), C.c_int32, C.c_void_p, C.c_size_t, C.c_int32,
                                    C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.ff_create_tiled.restype = C.c_int
    lib.ff_get_tiling.argtypes = [C.c_void_p, _ip, _ip, _ip]
    lib.ff_get_tiling.restype = C.c_int
    lib.ff_autotune_workspace_bytes.argtypes = [C.POINTER(FFSystem), C.c_int32]
    lib.ff_autotune_workspace_bytes.restype = C.c_size_t
    lib.ff_autotune.argtypes = [C.POINTER(FFSystem), C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32,
                                C.c_int32, C.c_void_p, _ip, _ip, _dp]
    lib.ff_autotune.restype = C.c_int
    lib.ff_energy_profile.argtypes = [C.c_void_p, C.c_void_p, _dp, C.c_int32, _dp, C.c_int32, C.c_void_p]
    lib.ff_energy_profile.restype = C.c_int
    lib.ff_last_error.argtypes = []
    lib.ff_last_error.restype = C.c_char_p
    v, i32, i64, sz, f32, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_float, C.c_double
    lib.ff_learn_param_count.argtypes = []
    lib.ff_learn_param_count.restype = i32
    lib.ff_learn_workspace_bytes.argtypes = [i32]
    lib.ff_learn_workspace_bytes.restype = sz
    lib.ff_learn_last_error.argtypes = []
    lib.ff_learn_last_error.restype = C.c_char_p
    lib.ff_learn_features.argtypes = [i32, i32, v, v, v, v, v, v, v, v, v]
    lib.ff_learn_gemm.argtypes = [i32, i32, i32, v, i64, i64, v, i64, i64, v, i32, v, i64, v, i64, v]
    lib.ff_learn_forward.argtypes = [v, v, v, i32, v, sz, v, v]
    lib.ff_learn_backward.argtypes = [v, v, v, i32, v, sz, v, v, v, v]
    lib.ff_learn_adam.argtypes = [v, v, v, v, v, i32, f32, f32, f32, f32, v]
    lib.ff_learn_to_bf16.argtypes = [v, i64, v, v]
    lib.ff_learn_delta.argtypes = [v, v, i32, v, v]
    lib.ff_learn_gather_rows.argtypes = [v, v, i32, i32, v, v]
    lib.ff_learn_displace.argtypes = [v, v, i32, f64, v, v]
    lib.ff_learn_select.argtypes = [i32, i32, v, v, v, v, v, v, v, v, v]
    for name in LEARN_EXPORTS[3:]:
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().ff_last_error().decode()


def learn_last_error() -> str:
    return load().ff_learn_last_error().decode()
