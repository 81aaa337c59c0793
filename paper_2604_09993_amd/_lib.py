"""ctypes binding of libcis.so (argument marshalling only).

Every step of the discretization runs in the HIP kernels behind the C ABI
declared in include/cis.h; this module only loads the library and describes
its structs and signatures.  Loading fails loudly when the library is absent
or cannot be opened: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

from . import build as _build

LIB_PATH = _build.LIB

CIS_OK = 0
CIS_ERR_NULL = 1
CIS_ERR_DIM = 2
CIS_ERR_LAYOUT = 3
CIS_ERR_DTYPE = 4
CIS_ERR_WORKSPACE = 5
CIS_ERR_MODEL = 6
CIS_ERR_HIP = 7
CIS_ERR_UNSUPPORTED = 8
CIS_ERR_NONFINITE = 9
CIS_F64 = 0
CIS_F32 = 1
CIS_BATCH_DISCRETIZE = 1
CIS_BATCH_ADJOINT = 2
CIS_SCHED_GRID = 1
CIS_SCHED_PERSISTENT = 2
CIS_SCHED_TUNE = 3
CIS_SCHED_ADJ_1 = 0x10
CIS_SCHED_ADJ_2 = 0x20
CIS_SCHED_ADJ_3 = 0x30
CIS_SCHED_ADJ_4 = 0x100
CIS_SCHED_WAVES_1 = 0x40
CIS_SCHED_WAVES_2 = 0x80
CIS_SCHED_DEF_BODY = 0x200
CIS_SCHED_DEF_LANE = 0x400
CIS_SCHED_SPLIT = 0x800
CIS_SCHED_FUSED = 0x1000
CIS_COMPOSE_VALU = 0
CIS_COMPOSE_MFMA = 1
CIS_FORM_ONE_LAUNCH = 0
CIS_FORM_SPLIT = 1
CIS_FORM_BLOCKED = 2

# every symbol include/cis.h declares
EXPORTS = [
    "cis_version", "cis_status_string", "cis_last_error", "cis_model_create",
    "cis_model_destroy", "cis_model_dims", "cis_discretize", "cis_defects",
    "cis_adjoint_workspace_size", "cis_discretize_adjoint", "cis_batch_plan_create",
    "cis_batch_run", "cis_batch_graph_run", "cis_batch_plan_info", "cis_batch_plan_destroy",
    "cis_blocked_workspace_size", "cis_discretize_blocked", "cis_discretize_adjoint_noalloc",
    "cis_split_workspace_size", "cis_discretize_split", "cis_batch_plan_discretize_form",
    "cis_batch_run_part", "cis_impact_dims", "cis_impact_linearize", "cis_rkf_workspace_size",
    "cis_discretize_rkf", "cis_paper_dims", "cis_paper_workspace_size", "cis_discretize_paper",
    "cis_batch_plan_tuned_from_cache", "cis_ldl_symbolic", "cis_ldl_numeric", "cis_ldl_solve",
    "cis_single_tune",
]


class ModelDesc(ctypes.Structure):
    _fields_ = [
        ("n_bodies", ctypes.c_int32), ("n_joints", ctypes.c_int32),
        ("n_contacts", ctypes.c_int32),
        ("link_length", ctypes.c_void_p), ("joint_parent", ctypes.c_void_p),
        ("joint_child", ctypes.c_void_p), ("joint_anchor_parent", ctypes.c_void_p),
        ("joint_anchor_child", ctypes.c_void_p), ("joint_stiffness", ctypes.c_void_p),
        ("joint_damping", ctypes.c_void_p), ("contact_body", ctypes.c_void_p),
        ("contact_point", ctypes.c_void_p),
        ("gravity", ctypes.c_double), ("terrain_amplitude", ctypes.c_double),
        ("terrain_wavenumber", ctypes.c_double),
    ]


class Shape(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("substeps", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("ld_node", ctypes.c_int64), ("ld_int", ctypes.c_int64)]


class SingleChoice(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("compose", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("ms", ctypes.c_float)]


class Traj(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("N", ctypes.c_int32),
                ("substeps", ctypes.c_int32), ("ld_node", ctypes.c_int64),
                ("ld_int", ctypes.c_int64)] + [
        (name, ctypes.c_void_p) for name in
        ("X", "U", "s", "params", "A", "Bm", "Bp", "S", "defect", "xprop", "seed",
         "gX", "gU", "gs", "gparams")]


_lib = None


def load(build_if_missing: bool = True):
    """Open libcis.so (building it first only if no library exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError(f"libcis.so not found at {LIB_PATH}; run the package build")
        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, St = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
    lib.cis_version.restype = ctypes.c_char_p
    lib.cis_version.argtypes = []
    lib.cis_status_string.restype = ctypes.c_char_p
    lib.cis_status_string.argtypes = [St]
    lib.cis_last_error.restype = ctypes.c_char_p
    lib.cis_last_error.argtypes = []
    lib.cis_model_create.restype = St
    lib.cis_model_create.argtypes = [ctypes.POINTER(ModelDesc), ctypes.POINTER(P)]
    lib.cis_model_destroy.restype = None
    lib.cis_model_destroy.argtypes = [P]
    lib.cis_model_dims.restype = St
    lib.cis_model_dims.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32),
                                   ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.cis_discretize.restype = St
    lib.cis_discretize.argtypes = [P, ctypes.POINTER(Shape)] + [P] * 11
    lib.cis_defects.restype = St
    lib.cis_defects.argtypes = [P, ctypes.POINTER(Shape), P, P, P, P, P, P, P, I32, P]
    lib.cis_adjoint_workspace_size.restype = St
    lib.cis_adjoint_workspace_size.argtypes = [P, ctypes.POINTER(Shape),
                                               ctypes.POINTER(ctypes.c_size_t)]
    lib.cis_discretize_adjoint.restype = St
    lib.cis_discretize_adjoint.argtypes = ([P, ctypes.POINTER(Shape), P, P, P, P, P, I32]
                                           + [P] * 6 + [ctypes.c_size_t, P])
    lib.cis_discretize_adjoint_noalloc.restype = St
    lib.cis_discretize_adjoint_noalloc.argtypes = ([P, ctypes.POINTER(Shape), P, P, P, P, P, I32]
                                                   + [P] * 6)
    lib.cis_split_workspace_size.restype = St
    lib.cis_split_workspace_size.argtypes = [P, ctypes.POINTER(Shape),
                                             ctypes.POINTER(ctypes.c_size_t)]
    lib.cis_discretize_split.restype = St
    lib.cis_discretize_split.argtypes = ([P, ctypes.POINTER(Shape), P, P, P, P, I32]
                                         + [P] * 7 + [ctypes.c_size_t, P])
    lib.cis_blocked_workspace_size.restype = St
    lib.cis_blocked_workspace_size.argtypes = [P, ctypes.POINTER(Shape), I32,
                                               ctypes.POINTER(ctypes.c_size_t)]
    lib.cis_discretize_blocked.restype = St
    lib.cis_discretize_blocked.argtypes = ([P, ctypes.POINTER(Shape), P, P, P, P, I32, I32]
                                           + [P] * 7 + [ctypes.c_size_t, P])
    lib.cis_batch_plan_create.restype = St
    lib.cis_batch_plan_create.argtypes = [ctypes.POINTER(Traj), I32, I32, I32, I32, I32, I32, P,
                                          ctypes.POINTER(P)]
    lib.cis_batch_run.restype = St
    lib.cis_batch_run.argtypes = [P, I32, P]
    lib.cis_batch_run_part.restype = St
    lib.cis_batch_run_part.argtypes = [P, I32, I32, P]
    lib.cis_batch_graph_run.restype = St
    lib.cis_batch_graph_run.argtypes = [P, I32, P]
    lib.cis_batch_plan_info.restype = St
    lib.cis_batch_plan_info.argtypes = [P, I32] + [ctypes.POINTER(I32)] * 8
    lib.cis_batch_plan_discretize_form.restype = St
    lib.cis_batch_plan_discretize_form.argtypes = [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.cis_batch_plan_destroy.restype = None
    lib.cis_batch_plan_destroy.argtypes = [P]
    lib.cis_rkf_workspace_size.restype = St
    lib.cis_rkf_workspace_size.argtypes = [P, ctypes.POINTER(Shape), ctypes.POINTER(ctypes.c_size_t)]
    lib.cis_discretize_rkf.restype = St
    lib.cis_discretize_rkf.argtypes = ([P, ctypes.POINTER(Shape), P, P, P, P, I32]
                                       + [P] * 8 + [ctypes.c_size_t, P])
    lib.cis_batch_plan_tuned_from_cache.restype = St
    lib.cis_batch_plan_tuned_from_cache.argtypes = [P, I32, ctypes.POINTER(I32)]
    lib.cis_paper_dims.restype = St
    lib.cis_paper_dims.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.cis_paper_workspace_size.restype = St
    lib.cis_paper_workspace_size.argtypes = [P, ctypes.POINTER(Shape),
                                             ctypes.POINTER(ctypes.c_size_t)]
    lib.cis_discretize_paper.restype = St
    lib.cis_discretize_paper.argtypes = ([P, ctypes.POINTER(Shape), P, P, P, P]
                                         + [P] * 7 + [ctypes.c_size_t, P])
    lib.cis_impact_dims.restype = St
    lib.cis_impact_dims.argtypes = [P] + [ctypes.POINTER(I32)] * 3
    lib.cis_impact_linearize.restype = St
    lib.cis_impact_linearize.argtypes = ([P, I32, ctypes.c_int64] + [P] * 5
                                         + [ctypes.c_double, ctypes.c_double] + [P] * 6)
    lib.cis_single_tune.restype = St
    lib.cis_single_tune.argtypes = [P, ctypes.POINTER(Shape)] + [P] * 10 + \
        [ctypes.POINTER(SingleChoice), P]
    lib.cis_ldl_symbolic.restype = ctypes.c_int64
    lib.cis_ldl_symbolic.argtypes = [I32] + [P] * 5
    lib.cis_ldl_numeric.restype = I32
    lib.cis_ldl_numeric.argtypes = [I32] + [P] * 6 + [ctypes.c_double] * 2 + [P] * 6
    lib.cis_ldl_solve.restype = None
    lib.cis_ldl_solve.argtypes = [I32] + [P] * 5
    _lib = lib
    return lib


class CisError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"cis status {status}: {detail}")
        self.status = status


def check(status: int) -> None:
    if status != CIS_OK:
        lib = load()
        raise CisError(status, lib.cis_last_error().decode())
