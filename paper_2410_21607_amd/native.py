"""ctypes loader for the HIP library ``libsem.so`` (no fallback).

If the library is missing or fails to load, every entry point raises: the
product has no CPU path.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsem.so")

SEM_OK = 0
SEM_FP64, SEM_FP32 = 0, 1
SEM_SCATTER, SEM_GATHER = 0, 1
SEM_ASSEMBLE, SEM_FINALIZE = 0, 1
SEM_CRIT_SPEED, SEM_CRIT_VORTZ = 0, 1
SEM_MAX_N = 8
SEM_MAX_LEVEL = 12

c_int, c_double, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
c_i32p = ctypes.POINTER(ctypes.c_int32)
c_dp = ctypes.POINTER(ctypes.c_double)


class SemMeshDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nx0", ctypes.c_int32), ("ny0", ctypes.c_int32),
                ("n_z", ctypes.c_int32), ("n_col", ctypes.c_int32),
                ("h_col_level", c_i32p), ("h_col_ix", c_i32p), ("h_col_iy", c_i32p),
                ("Lx", c_double), ("Ly", c_double), ("h_z_edges", c_dp),
                ("periodic_x", ctypes.c_int32), ("periodic_y", ctypes.c_int32),
                ("f", c_double), ("g", c_double), ("R_d", c_double), ("c_p", c_double),
                ("p00", c_double)]


class SemMeshInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("n_z", ctypes.c_int32), ("nzn", ctypes.c_int32),
                ("ldz", ctypes.c_int32), ("max_level", ctypes.c_int32), ("n_col", ctypes.c_int64),
                ("n_elem", ctypes.c_int64), ("n_h", ctypes.c_int64), ("n_hh", ctypes.c_int64),
                ("n_dof", ctypes.c_int64), ("n_hang", ctypes.c_int64),
                ("n_local", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64)]


# name -> (restype, argtypes); every symbol declared in include/sem.h
SIGNATURES = {
    "sem_mesh_create": (c_int, [ctypes.POINTER(SemMeshDesc), ctypes.POINTER(c_void_p)]),
    "sem_mesh_destroy": (c_int, [c_void_p]),
    "sem_mesh_plan": (c_int, [ctypes.POINTER(SemMeshDesc), ctypes.POINTER(SemMeshInfo), c_dp, c_dp,
                              c_dp, c_dp]),
    "sem_mesh_get_info": (c_int, [c_void_p, ctypes.POINTER(SemMeshInfo)]),
    "sem_mesh_coords": (c_int, [c_void_p, c_dp, c_dp, c_dp]),
    "sem_mesh_set_reference": (c_int, [c_void_p, c_dp, c_dp, c_dp]),
    "sem_mesh_set_dissipation": (c_int, [c_void_p, c_double, c_double, c_double]),
    "sem_mesh_set_terrain": (c_int, [c_void_p, c_dp, c_dp, c_dp, c_dp]),
    "sem_mesh_heights": (c_int, [c_void_p, c_dp, c_dp]),
    "sem_mesh_get_epoch": (c_int, [c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "sem_nc_project": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "sem_rhs": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    "sem_dss": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "sem_stage_update": (c_int, [c_void_p, c_double, c_double, c_double, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p]),
    "sem_stage": (c_int, [c_void_p, c_double, c_double, c_double, c_void_p, c_void_p,
                          c_void_p, c_int, c_void_p]),
    "sem_stage_tune": (c_int, [c_void_p, c_int]),
    "sem_stage_get_tune": (c_int, [c_void_p, ctypes.POINTER(c_int)]),
    "sem_stage_set_layout": (c_int, [c_void_p, c_int, c_int]),
    "sem_stage_get_layout": (c_int, [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "sem_stage_autotune": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int,
                                   ctypes.POINTER(c_int), ctypes.POINTER(ctypes.c_float), c_void_p]),
    "amr_flag": (c_int, [c_void_p, c_void_p, c_int, c_dp, c_int, c_void_p, c_void_p, c_void_p]),
    "sem_adapt_columns": (c_int, [ctypes.POINTER(SemMeshDesc), c_void_p, c_int, ctypes.c_int32,
                                  c_i32p, c_i32p, c_i32p, ctypes.POINTER(ctypes.c_int32)]),
    "sem_transfer_create": (c_int, [c_void_p, c_void_p, ctypes.POINTER(c_void_p)]),
    "sem_transfer_apply": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "sem_transfer_destroy": (c_int, [c_void_p]),
    "sem_transfer_plan": (c_int, [ctypes.POINTER(SemMeshDesc), ctypes.POINTER(SemMeshDesc),
                                  ctypes.POINTER(ctypes.c_int64), c_i32p, c_i32p, c_dp]),
    "amr_features": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_dp, c_int,
                             ctypes.POINTER(ctypes.c_float), c_void_p, c_void_p, c_void_p]),
    "amr_forecast_flags": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p,
                                   c_void_p]),
    "sem_max_wind": (c_int, [c_void_p, c_void_p, c_double, c_double, c_double, c_double,
                             c_void_p, c_void_p]),
    "sem_forecast_labels": (c_int, [ctypes.POINTER(SemMeshDesc), ctypes.POINTER(SemMeshDesc),
                                    c_void_p, c_void_p]),
    "mlp_forward": (c_int, [c_void_p, c_void_p, ctypes.c_int64, c_void_p, c_void_p]),
    "mlp_backward": (c_int, [c_void_p, c_void_p, ctypes.c_int64, c_void_p, c_void_p,
                             ctypes.c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mlp_backward_noalloc": (c_int, [c_void_p, c_void_p, ctypes.c_int64, c_void_p, c_void_p,
                                     ctypes.c_int64, c_void_p, c_void_p, c_void_p]),
    "mlp_adam_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, ctypes.c_float, c_void_p]),
    "sem_last_error": (ctypes.c_char_p, []),
}

SEM_NFEAT = 16
SEM_MLP_NPARAM = 5443
SEM_MLP_WORK = 260
SEM_MLP_NOALLOC_MAX = 2048

_LIB = None


class SemError(RuntimeError):
    def __init__(self, name, code, msg):
        super().__init__(f"{name} failed ({code}): {msg}")
        self.code = code


def lib():
    """Load libsem.so once; raise if it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def call(name, *args):
    L = lib()
    rc = getattr(L, name)(*args)
    if rc != SEM_OK:
        raise SemError(name, rc, L.sem_last_error().decode())
    return rc
