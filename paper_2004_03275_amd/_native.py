"""ctypes binding of libamrv.so (the C-ABI in include/amrv.h).

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  Loading fails loudly if the library is missing; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamrv.so")

OK = 0
EINVAL = -1
EUNBALANCED = -2
ENONPHYSICAL = -3
ENOMEM = -4
EDEVICE = -5
ENOTSUP = -6
ENOTCONVERGED = -7

SCHED_PER_BLOCK = 0
SCHED_GRID = 1
SCHED_PERSISTENT = 2

ARITH_EXACT = 0
ARITH_FAST = 1

FLAG_LOHNER = 0
FLAG_MLP = 1
FLAG_MLP_FALLBACK = 2
MLP_NPARAM = 12546
MLP_NIN = 128


class Config(ctypes.Structure):
    """amrv_config: 20 int32 followed by 14 double."""

    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("block_nx", ctypes.c_int32 * 3),
        ("nghost", ctypes.c_int32),
        ("base_blocks", ctypes.c_int32 * 3),
        ("max_level", ctypes.c_int32),
        ("physics", ctypes.c_int32),
        ("flux", ctypes.c_int32),
        ("limiter", ctypes.c_int32),
        ("rk_stages", ctypes.c_int32),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("pad_", ctypes.c_int32),
        ("xmin", ctypes.c_double * 3),
        ("xmax", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("lohner_tol", ctypes.c_double),
        ("lohner_coarsen_frac", ctypes.c_double),
        ("lohner_eps", ctypes.c_double),
        ("lohner_w_rho", ctypes.c_double),
        ("lohner_w_p", ctypes.c_double),
        ("glm_cr", ctypes.c_double),
        ("cad", ctypes.c_double),
        ("cada_radius", ctypes.c_double),
    ]


class TrainCfg(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("pos_weight", ctypes.c_float), ("pos_weight_c", ctypes.c_float),
                ("t0", ctypes.c_int32)]


class MgConfig(ctypes.Structure):
    """amrv_mg_config (include/amrv_mg.h)."""

    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32), ("bc", ctypes.c_int32), ("nfields", ctypes.c_int32),
                ("pre_sweeps", ctypes.c_int32), ("post_sweeps", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("smoother", ctypes.c_int32), ("length", ctypes.c_double)]


class FmgConfig(ctypes.Structure):
    """amrv_fmg_config (include/amrv_mg.h)."""

    _fields_ = [("nleaves", ctypes.c_int64), ("base", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("pre_sweeps", ctypes.c_int32), ("post_sweeps", ctypes.c_int32),
                ("ndim", ctypes.c_int32), ("length", ctypes.c_double)]


class RdParams(ctypes.Structure):
    """amrv_rd_params (include/amrv_mg.h)."""

    _fields_ = [("model", ctypes.c_int32), ("pad", ctypes.c_int32), ("Du", ctypes.c_double), ("Dv", ctypes.c_double),
                ("p1", ctypes.c_double), ("p2", ctypes.c_double), ("p3", ctypes.c_double)]


class AmrvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"amrv error {code}: {msg}")
        self.code = code


_lib = None

# exported symbols and their signatures (also checked by the CPU test suite)
P = ctypes.c_void_p
SIGNATURES = {
    "amrv_workspace_bytes": ([ctypes.POINTER(Config), ctypes.c_int64, P, P], ctypes.c_size_t),
    "amrv_forest_create": ([ctypes.POINTER(Config), ctypes.c_int64, P, P, P, ctypes.c_size_t, P,
                            ctypes.POINTER(P)], ctypes.c_int),
    "amrv_forest_destroy": ([P], ctypes.c_int),
    "amrv_nvar": ([P], ctypes.c_int),
    "amrv_state_doubles": ([P], ctypes.c_int64),
    "amrv_set_state": ([P, P, ctypes.c_int64, ctypes.c_int32], ctypes.c_int),
    "amrv_get_state": ([P, P, ctypes.c_int64, ctypes.c_int32], ctypes.c_int),
    "amrv_max_dt": ([P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "amrv_glm_ch": ([P], ctypes.c_double),
    "amrv_advance": ([P, ctypes.c_double], ctypes.c_int),
    "amrv_flag_blocks": ([P, ctypes.c_int32, P, P], ctypes.c_int),
    "amrv_advance_cfl": ([P, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "amrv_mlp_set_weights": ([P, P, ctypes.c_int64], ctypes.c_int),
    "amrv_mlp_set_margin": ([P, ctypes.c_float], ctypes.c_int),
    "amrv_mlp_features": ([P, P, ctypes.c_int32], ctypes.c_int),
    "amrv_mlp_logits": ([P, P], ctypes.c_int),
    "amrv_mlp_fuse_features": ([P, ctypes.c_int32], ctypes.c_int),
    "amrv_mlp_train_workspace_bytes": ([ctypes.c_int32], ctypes.c_size_t),
    "amrv_mlp_train": ([P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P,
                        ctypes.POINTER(TrainCfg), P, ctypes.c_size_t, P, P, P], ctypes.c_int),
    "amrv_mlp_train_noalloc": ([P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P,
                                ctypes.POINTER(TrainCfg), P, P, P], ctypes.c_int),
    "amrv_set_schedule": ([P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "amrv_get_schedule": ([P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "amrv_set_variant": ([P, ctypes.c_int32], ctypes.c_int),
    "amrv_set_arithmetic": ([P, ctypes.c_int32], ctypes.c_int),
    "amrv_get_arithmetic": ([P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "amrv_get_variant": ([P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "amrv_autotune": ([P, ctypes.c_int32], ctypes.c_int),
    "amrv_autotune_report": ([P], ctypes.c_char_p),
    "amrv_use_graph": ([P, ctypes.c_int32], ctypes.c_int),
    "amrv_profile": ([P, ctypes.c_int32], ctypes.c_int),
    "amrv_profile_read": ([P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                           ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "amrv_regrid_plan": ([P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), P, P], ctypes.c_int),
    "amrv_regrid_plan_leaves": ([ctypes.POINTER(Config), ctypes.c_int64, P, P, P, ctypes.c_int64,
                                 ctypes.POINTER(ctypes.c_int64), P, P], ctypes.c_int),
    "amrv_regrid_transfer": ([P, P], ctypes.c_int),
    "amrv_synchronize": ([P], ctypes.c_int),
    "amrv_uniform_grid_copy": ([P, ctypes.c_int32, P, ctypes.c_int32], ctypes.c_int),
    "amrv_mg_workspace_bytes": ([ctypes.POINTER(MgConfig)], ctypes.c_size_t),
    "amrv_mg_create": ([ctypes.POINTER(MgConfig), P, ctypes.c_size_t, P, ctypes.POINTER(P)], ctypes.c_int),
    "amrv_mg_destroy": ([P], ctypes.c_int),
    "amrv_mg_solve": ([P, P, P, P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), P, P],
                      ctypes.c_int),
    "amrv_rd_step": ([P, ctypes.POINTER(RdParams), ctypes.c_int32, ctypes.c_double, ctypes.c_int32, P, P,
                      ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), P], ctypes.c_int),
    "amrv_mg_divb_project": ([P, P, P, P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "amrv_mg_set_coefficient": ([P, P], ctypes.c_int),
    "amrv_mg_profile": ([P, ctypes.c_int32], ctypes.c_int),
    "amrv_mg_profile_read": ([P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "amrv_fmg_workspace_bytes": ([ctypes.POINTER(FmgConfig), P, P], ctypes.c_size_t),
    "amrv_fmg_create": ([ctypes.POINTER(FmgConfig), P, P, P, ctypes.c_size_t, P, ctypes.POINTER(P)], ctypes.c_int),
    "amrv_fmg_destroy": ([P], ctypes.c_int),
    "amrv_fmg_levels": ([P, P], ctypes.c_int),
    "amrv_fmg_solve": ([P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "amrv_fmg_rd_step": ([P, ctypes.POINTER(RdParams), ctypes.c_int32, ctypes.c_double, ctypes.c_int32, P, P,
                          ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "amrv_fmg_divb_project": ([P, P, P, P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "amrv_last_error": ([], ctypes.c_char_p),
}


def lib():
    """Load libamrv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(rc: int):
    if rc != OK:
        raise AmrvError(rc, lib().amrv_last_error().decode())


def make_config(s) -> Config:
    """Config from a workloads.Scheme (or any object with the same fields)."""
    c = Config()
    c.ndim = s.ndim
    for d in range(3):
        c.block_nx[d] = s.block_nx[d]
        c.base_blocks[d] = s.base_blocks[d]
        c.xmin[d] = s.xmin[d]
        c.xmax[d] = s.xmax[d]
        c.bc[d][0] = s.bc
        c.bc[d][1] = s.bc
    c.nghost = s.nghost
    c.max_level = s.max_level
    c.physics = s.physics
    c.flux = s.flux
    c.limiter = s.limiter
    c.rk_stages = s.rk_stages
    c.gamma = s.gamma
    c.cfl = s.cfl
    c.lohner_tol = s.lohner_tol
    c.lohner_coarsen_frac = s.lohner_coarsen_frac
    c.lohner_eps = s.lohner_eps
    c.lohner_w_rho = s.lohner_w_rho
    c.lohner_w_p = s.lohner_w_p
    c.glm_cr = s.glm_cr
    c.cad = s.cad
    c.cada_radius = s.cada_radius
    return c


def regrid_plan_leaves(forest, flags) -> tuple:
    """Host-only regrid plan of a workloads.Forest: (level [m], ijk [m, 3])."""
    import numpy as np

    cfg = make_config(forest.scheme)
    lev = np.ascontiguousarray(forest.level, dtype=np.int32)
    ijk = np.ascontiguousarray(forest.ijk, dtype=np.int32)
    flags = np.ascontiguousarray(flags, dtype=np.int8)
    if flags.shape != (forest.n,):
        raise ValueError("one flag per leaf")
    # at most every leaf splits: one call with room for that
    cap = forest.n << forest.scheme.ndim
    m = ctypes.c_int64()
    out_l = np.empty(cap, dtype=np.int32)
    out_i = np.empty((cap, 3), dtype=np.int32)
    check(lib().amrv_regrid_plan_leaves(ctypes.byref(cfg), forest.n, lev.ctypes.data, ijk.ctypes.data,
                                        flags.ctypes.data, cap, ctypes.byref(m), out_l.ctypes.data,
                                        out_i.ctypes.data))
    return out_l[:m.value].copy(), out_i[:m.value].copy()
