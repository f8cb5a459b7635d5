"""ctypes loader for libpcgainv.so (argument marshalling only).

There is no fallback: if the shared library is missing or fails to load, every
entry point raises.  Build it with ``python -m paper_1210_1878_amd.build`` or
``__graft_entry__.build()``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcgainv.so")

OK, NOCONV, EINVAL, EBREAKDOWN, ENAN, EHIP, ENOMEM = 0, 1, -1, -2, -3, -4, -5
PERIODIC_X = 1
FP64, MIXED, MIXED_A32 = 0, 1, 2
REFINE_RESTART, REFINE_KEEP = 0, 1
NOALLOC_MAX_BYTES = 64 << 20   # PCGA_NOALLOC_MAX_BYTES


class PcgaError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str = ""):
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


class A5(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("diag", ctypes.c_void_p), ("ae", ctypes.c_void_p), ("an", ctypes.c_void_p)]


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


_p = ctypes.c_void_p
_pp = ctypes.POINTER(ctypes.c_void_p)
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_sz = ctypes.c_size_t
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pdbl = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "pcga_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "pcga_last_error": ([], ctypes.c_char_p),
    "pcga_stream_create": ([_pp], ctypes.c_int),
    "pcga_stream_destroy": ([_p], ctypes.c_int),
    "pcga_ainv_setup": ([ctypes.POINTER(A5), _dbl, _pp], ctypes.c_int),
    "pcga_ainv_setup_fill": ([ctypes.POINTER(A5), _dbl, _i32, _pp], ctypes.c_int),
    "pcga_fsai_band_setup": ([ctypes.POINTER(A5), _i32, _pp], ctypes.c_int),
    "pcga_ainv_setup_csr": ([ctypes.POINTER(Csr), _dbl, _i32, _pp], ctypes.c_int),
    "pcga_workspace_bytes_csr": ([ctypes.POINTER(Csr), _p, ctypes.c_int, _i32,
                                  ctypes.POINTER(_sz)], ctypes.c_int),
    "pcga_solver_create_csr": ([ctypes.POINTER(Csr), _p, ctypes.c_int, _i32, _p, _sz, _p, _pp],
                               ctypes.c_int),
    "pcga_ainv_info": ([_p, _pi64, _pi64], ctypes.c_int),
    "pcga_ainv_export": ([_p, _p, _p, _p, _p], ctypes.c_int),
    "pcga_ainv_import": ([_i64, _p, _p, _p, _p, _pp], ctypes.c_int),
    "pcga_ainv_free": ([_p], ctypes.c_int),
    "pcga_layout_info": ([_p, _i32, _p], ctypes.c_int),
    "pcga_workspace_bytes": ([ctypes.POINTER(A5), _p, ctypes.c_int, ctypes.POINTER(_sz)],
                             ctypes.c_int),
    "pcga_solver_create": ([ctypes.POINTER(A5), _p, ctypes.c_int, _p, _sz, _p, _pp],
                           ctypes.c_int),
    "pcga_solver_destroy": ([_p], ctypes.c_int),
    "pcga_workspace_bytes_ex": ([ctypes.POINTER(A5), _p, ctypes.c_int, _i32, ctypes.POINTER(_sz)],
                                ctypes.c_int),
    "pcga_solver_create_ex": ([ctypes.POINTER(A5), _p, ctypes.c_int, _i32, _p, _sz, _p, _pp],
                              ctypes.c_int),
    "pcga_solver_info": ([_p, _pi64, _pi64, _pi32, _pdbl, _pi32, _pi32], ctypes.c_int),
    "pcga_solver_tune": ([_p, _i32, _i32, _i32], ctypes.c_int),
    "pcga_solver_set_grids": ([_p, _i32, _i32, _i32], ctypes.c_int),
    "pcga_pcg_solve": ([_p, _p, _p, _dbl, _i32, _pi32, _p, _i32, _pi32, _pdbl], ctypes.c_int),
    "pcga_pcg_solve_noalloc": ([_p, _p, _p, _dbl, _i32, _pi32, _p, _i32, _pi32, _pdbl],
                               ctypes.c_int),
    "pcga_pcg_solve_mixed": ([_p, _p, _p, _dbl, _dbl, _i32, _i32, _pi32, _pi32, _p, _i32,
                              _pi32, _pdbl], ctypes.c_int),
    "pcga_pcg_solve_mixed_ex": ([_p, _p, _p, _dbl, _dbl, _i32, _i32, _i32, _pi32, _pi32, _p,
                                 _i32, _pi32, _pdbl], ctypes.c_int),
    "pcga_apply_a": ([_p, _p, _p], ctypes.c_int),
    "pcga_apply_prec": ([_p, _p, _p, _p], ctypes.c_int),
    "pcga_step_stencil": ([_p, _p, _p, _dbl, _p, _p, _pdbl], ctypes.c_int),
    "pcga_profile_iteration": ([_p, _p, _i32, _i32, _pdbl], ctypes.c_int),
    "pcga_ts_rhs": ([_p, _p, _p, _p, _p, _p], ctypes.c_int),
    "pcga_ts_eta": ([_p, _p, _p, _dbl, _p], ctypes.c_int),
    "pcga_ts_guess": ([_p, _p, _p, _dbl, _dbl, _p], ctypes.c_int),
    "pcga_batch_scratch_bytes": ([_i32, ctypes.POINTER(_sz)], ctypes.c_int),
    "pcga_batch_item_bytes": ([_p, _i32, ctypes.POINTER(_sz)], ctypes.c_int),
    "pcga_batch_create": ([_i32, _p, _sz, _p, _pp], ctypes.c_int),
    "pcga_batch_destroy": ([_p], ctypes.c_int),
    "pcga_batch_add": ([_p, _p, _i32, _p, _p, _p, _p, _sz, _dbl, _dbl, _i32, _i32, _pi32],
                       ctypes.c_int),
    "pcga_batch_add_ex": ([_p, _p, _i32, _p, _p, _p, _p, _sz, _dbl, _dbl, _i32, _i32, _i32, _pi32],
                       ctypes.c_int),
    "pcga_batch_run": ([_p, _i32, _pi32], ctypes.c_int),
    "pcga_batch_launch": ([_p, _i32], ctypes.c_int),
    "pcga_batch_wait": ([_p, _i32, _pi32, _pi32], ctypes.c_int),
    "pcga_batch_query": ([_p, _i32, _pi32, _pi32, _pi32, _pi32, _pdbl], ctypes.c_int),
    "pcga_batch_remove": ([_p, _i32], ctypes.c_int),
    "pcga_batch_set_chunk": ([_p, _i32], ctypes.c_int),
    "pcga_batch_set_grid": ([_p, _i32], ctypes.c_int),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libpcgainv.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first "
                              "(python -m paper_1210_1878_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(status: int, where: str, allow=(OK,)) -> int:
    if status in allow:
        return status
    L = load()
    raise PcgaError(status, where, L.pcga_last_error().decode(errors="replace"))
