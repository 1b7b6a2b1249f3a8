"""ctypes binding of libpic (include/pic.h): argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libpic.so")

PIC_OK = 0
PIC_E_ARG = 1
PIC_E_HIP = 2
PIC_E_STATE = 3
PIC_E_CAPACITY = 1 << 8
PIC_E_CFL = 1 << 9
PIC_E_NONFINITE = 1 << 10
PIC_E_OUT_OF_TILE = 1 << 11
PIC_E_ADJ_MAP = 1 << 12
PIC_FP32 = 0
PIC_FP64 = 1
PIC_MAX_SPECIES = 4
PIC_HALF_B = 0
PIC_CURL_E = 1
PIC_ADD_J = 2
PIC_CURL_E_ADD_J = 3
PIC_TWO_HALF_B = 4
PIC_FUSED = 1
PIC_SORT_CELLS = 2
PIC_PUSH_HALF_B = 4
PIC_DEPOSIT_CURL_E = 8
PIC_ALL_SPECIES = 0xFFFFFFFF
PIC_OPT_ACC_WORKING = 1
PIC_OPT_PERSISTENT = 2
PIC_OPT_TRACK = 4
PIC_WALL_X = 1
PIC_PUSHER_BORIS = 0
PIC_PUSHER_VAY = 1
PIC_PUSHER_HC = 2

EXPORTS = ["pic_query", "pic_init_tiles", "pic_fdtd_step", "pic_push_interp", "pic_deposit_current",
           "pic_sort_migrate", "pic_step", "pic_inject", "pic_filter_current", "pic_graph_capture", "pic_graph_launch", "pic_error",
           "pic_diagnostics", "pic_diagnostics_static", "pic_diagnostics_boxes", "pic_adjoint_unpermute", "pic_adjoint_step", "pic_destroy", "pic_last_error"]

P = ctypes.c_void_p
I32 = ctypes.c_int32
U32 = ctypes.c_uint32
I64 = ctypes.c_int64
U64 = ctypes.c_uint64
DBL = ctypes.c_double


class PicConfig(ctypes.Structure):
    _fields_ = [
        ("dim", I32), ("precision", I32), ("n_species", I32), ("n_boxes", I32),
        ("tile", I32 * 3), ("block", I32), ("cfl", DBL),
        ("box_cells", P), ("charge", P), ("qm", P), ("mass", P), ("tile_capacity", P),
        ("capacity_factor", DBL), ("outbox_capacity", I32), ("options", U32), ("box_walls", P),
        ("pusher", I32), ("filter_passes", I32), ("fdtd_order", I32), ("inject_max", I64),
    ]


class PicLayout(ctypes.Structure):
    _fields_ = [
        ("total_bytes", U64), ("off_E", U64), ("off_B", U64), ("off_J", U64), ("off_pos", U64),
        ("off_u", U64), ("off_xold", U64), ("off_seg_offset", U64), ("off_seg_capacity", U64),
        ("off_seg_count", U64), ("off_error", U64), ("off_flags", U64), ("off_ids", U64),
        ("cells_total", I64), ("tiles_total", I64), ("capacity_total", I64), ("outbox_capacity", I64),
        ("elem_bytes", I32), ("reserved", I32),
    ]


class PicInitData(ctypes.Structure):
    _fields_ = [("count", P), ("pos", P), ("u", P), ("E", P), ("B", P)]


class PicDiag(ctypes.Structure):
    _fields_ = [
        ("field_energy", DBL), ("kinetic_energy", DBL), ("gauss_max", DBL), ("divb_max", DBL),
        ("charge_total", DBL), ("particles", I64), ("near_face", I64), ("error_bits", I32), ("reserved", I32),
        ("continuity_max", DBL),
    ]


_lib = None


class PicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpic error {code:#x}: {msg}")
        self.code = code


def lib():
    """Load libpic.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1906_06306_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "pic_query": [P, P, P],
            "pic_init_tiles": [P, P, P, U64, P, P, P],
            "pic_fdtd_step": [P, I32],
            "pic_push_interp": [P, U32, U32],
            "pic_deposit_current": [P, U32, U32],
            "pic_sort_migrate": [P, U32, P, P, I64],
            "pic_step": [P, U32],
            "pic_filter_current": [P, I32],
            "pic_inject": [P, I32, I32, I64, P, P],
            "pic_graph_capture": [P, I32, U32],
            "pic_graph_launch": [P],
            "pic_error": [P],
            "pic_diagnostics": [P, P],
            "pic_diagnostics_static": [P, P],
            "pic_diagnostics_boxes": [P, P],
            "pic_adjoint_unpermute": [P, P, P, P, P, I64],
            "pic_adjoint_step": [P, P, P, P, P],
            "pic_destroy": [P],
            "pic_last_error": [],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name == "pic_last_error" else I32
        _lib = L
    return _lib


def check(code: int) -> int:
    if code != PIC_OK:
        msg = lib().pic_last_error()
        raise PicError(code, msg.decode() if msg else "")
    return code
