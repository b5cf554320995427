"""ctypes declarations of the C ABI in include/maspncg.h.

Loading fails loudly when the built library is missing: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmaspncg.so")

MAS_F64, MAS_F32, MAS_BF16, MAS_F16 = 0, 1, 2, 3
PREC = {"f64": MAS_F64, "f32": MAS_F32, "bf16": MAS_BF16, "f16": MAS_F16}
BETA = {"fr": 1, "cd": 2, "dk": 3}
PRECOND = {"mas": 0, "bj3": 1}
HIERARCHY = {"morton": 0, "connectivity": 1}

STATUS = {0: "MAS_OK", 1: "MAS_ERR_INVALID_ARG", 2: "MAS_ERR_STATE", 3: "MAS_ERR_OOM",
          4: "MAS_ERR_HIP", 5: "MAS_ERR_NOT_SPD", 6: "MAS_ERR_NONFINITE", 7: "MAS_ERR_RANK"}


class MasConfig(ctypes.Structure):
    _fields_ = [
        ("num_levels", ctypes.c_int32),
        ("max_rank", ctypes.c_int32),
        ("cos_rot", ctypes.c_double),
        ("restart_delta", ctypes.c_double),
        ("eps_sing", ctypes.c_double),
        ("eps_abs", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("dhat", ctypes.c_double),
        ("h", ctypes.c_double),
        ("gravity", ctypes.c_double * 3),
        ("block_prec", ctypes.c_int32),
        ("coarse_prec", ctypes.c_int32),
        ("hess_prec", ctypes.c_int32),
        ("deterministic", ctypes.c_int32),
        ("prec_guard", ctypes.c_double),
        ("max_contacts", ctypes.c_int64),
        ("max_tris", ctypes.c_int64),
        ("max_edges", ctypes.c_int64),
        ("precond", ctypes.c_int32),
        ("hierarchy", ctypes.c_int32),
    ]


class MasMesh(ctypes.Structure):
    _fields_ = [
        ("num_vertices", ctypes.c_int64),
        ("num_tets", ctypes.c_int64),
        ("rest_x", ctypes.c_void_p),
        ("tets", ctypes.c_void_p),
        ("density", ctypes.c_void_p),
        ("youngs", ctypes.c_void_p),
        ("poisson", ctypes.c_void_p),
        ("num_links", ctypes.c_int64),
        ("links", ctypes.c_void_p),
        ("num_scenes", ctypes.c_int32),
        ("scene_offsets", ctypes.c_void_p),
    ]


class MasContacts(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64),
        ("key", ctypes.c_void_p),
        ("idx", ctypes.c_void_p),
        ("d", ctypes.c_void_p),
        ("grad", ctypes.c_void_p),
    ]


class MasStepOut(ctypes.Structure):
    _fields_ = [
        ("mu", ctypes.c_double), ("nu", ctypes.c_double), ("r", ctypes.c_double),
        ("gz", ctypes.c_double), ("gp", ctypes.c_double), ("gzp", ctypes.c_double),
        ("A11", ctypes.c_double), ("A12", ctypes.c_double), ("A22", ctypes.c_double),
        ("gnorm2", ctypes.c_double), ("znorm2", ctypes.c_double),
        ("fallback", ctypes.c_int32), ("restart_next", ctypes.c_int32),
        ("restart_used", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


STEP_FIELDS = [f for f, _ in MasStepOut._fields_]


class MasIterStats(ctypes.Structure):
    _fields_ = [
        ("contacts", ctypes.c_int64), ("active", ctypes.c_int64),
        ("n_new", ctypes.c_int64), ("n_rotated", ctypes.c_int64),
        ("n_stiffened", ctypes.c_int64), ("n_softened", ctypes.c_int64),
        ("rank_sum", ctypes.c_int64), ("rank_max", ctypes.c_int32), ("safe_rounds", ctypes.c_int32),
        ("safe_left", ctypes.c_int64), ("alpha_hist", ctypes.c_int64 * 8),
    ]

TIMERS = {"apply_l0": 0, "apply": 1, "hv_tets": 2, "hess_vec": 3, "update": 4, "capacitance": 5,
          "build": 6, "energy": 7, "subspace": 8, "ccd": 9, "contact": 10, "constraint_set": 11}

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double

SIGNATURES = {
    "mas_default_config": (None, [ctypes.POINTER(MasConfig)]),
    "mas_create": (_I32, [ctypes.POINTER(MasConfig), ctypes.POINTER(MasMesh), _P, ctypes.POINTER(_P), _P]),
    "mas_destroy": (_I32, [_P]),
    "mas_build": (_I32, [_P, _P, ctypes.POINTER(MasContacts)]),
    "mas_woodbury_update": (_I32, [_P, ctypes.POINTER(MasContacts), _P]),
    "mas_apply": (_I32, [_P, _P, _P]),
    "hess_vec": (_I32, [_P, _P, _P, _I32]),
    "pncg_subspace_step": (_I32, [_P, _P, _P, _P, _P, _P, _P, _I32, _P]),
    "pncg_subspace_step_noalloc": (_I32, [_P, _P, _P, _P, _P, _P, _P, _I32, _P]),
    "pncg_beta_step": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _P, _P, _I32, _P, _P]),
    "mas_energy_grad": (_I32, [_P, _P, _P, ctypes.POINTER(MasContacts), _P, _P]),
    "pncg_subspace_step_scenes": (_I32, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "mas_energy_grad_scenes": (_I32, [_P, _P, _P, ctypes.POINTER(MasContacts), _P, _P]),
    "mas_step_scenes": (_I32, [_P, _P, _P, _P, _P]),
    "mas_scenes": (_I32, [_P, _P, _P]),
    "mas_inertial_target": (_I32, [_P, _P, _P, _P]),
    "mas_next_frame": (_I32, [_P, _P, _P, _P, _P]),
    "mas_stencil_distance": (_I32, [_P, _P, _I64, _P, _P, _P, _P]),
    "mas_safe_step": (_I32, [_P, _P, _P, ctypes.POINTER(MasContacts), _D, _P, _P]),
    "mas_ccd_steps": (_I32, [_P, _P, _P, ctypes.c_int64, _P, _P, _P, _P, _P]),
    "mas_ccd_safe_step": (_I32, [_P, _P, _P, _D, _I64, _P, _P, _P, _D, _P, _P]),
    "mas_contact_distances": (_I32, [_P, _P, ctypes.c_int64, _P, _P, _P, _P, _P]),
    "mas_constraint_set": (_I32, [_P, _P, ctypes.c_double, ctypes.c_int64, _P, ctypes.c_int64, _P, ctypes.c_int64,
                                  _P, ctypes.c_int64, _P, _P, _P, _P, _P, _P]),
    "mas_sync_status": (_I32, [_P, ctypes.c_char_p, _I32]),
    "mas_read_stats": (_I32, [_P, ctypes.POINTER(MasIterStats)]),
    "mas_query": (_I32, [_P, _P, _P, _P, _P]),
    "mas_vertex_order": (_I32, [ctypes.POINTER(MasMesh), _I32, _I32, _P]),
    "mas_get_block": (_I32, [_P, _I32, _I64, _P]),
    "mas_block_precisions": (_I32, [_P, _I32, _P]),
    "mas_get_selection": (_I32, [_P, _P, _P]),
    "mas_status_string": (ctypes.c_char_p, [_I32]),
    "mas_profile_enable": (_I32, [_P, _I32]),
    "mas_profile_read": (_I32, [_P, _I32, _P, _P]),
    "mas_profile_select": (_I32, [_P, ctypes.c_uint32]),
}

_lib = None


class MasError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__("%s failed: %s (%d)" % (fn, STATUS.get(code, "?"), code))
        self.code = code


def lib():
    """The loaded libmaspncg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmaspncg.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(fn, code):
    if code != 0:
        raise MasError(fn, code)
