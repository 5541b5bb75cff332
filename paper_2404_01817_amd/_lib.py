"""ctypes binding of libneat.so (the C ABI in include/neat.h).

Argument marshalling only: torch tensors provide device memory and streams;
every step of the computation runs in the library's HIP kernels.  The library
must have been built (``python -m paper_2404_01817_amd.build``); there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libneat.so")

NEAT_OK = 0
NEAT_PENDING = 1
FWD_AUTO, FWD_REG, FWD_LDS, FWD_REG2, FWD_TUNED, FWD_LVL, FWD_SEG = 0, 1, 2, 3, 4, 5, 6
TUNE_CANDIDATES = 5  # REG, REG2, LDS, LVL, SEG


class NeatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("neat error %d: %s" % (code, msg))
        self.code = code


class Dims(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("N_max", ctypes.c_int32),
                ("C_max", ctypes.c_int32), ("I", ctypes.c_int32), ("O", ctypes.c_int32)]


class BatchItem(ctypes.Structure):
    """neat_batch_item."""
    _fields_ = [("dims", Dims), ("nodes", ctypes.c_void_p), ("conns", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("program", ctypes.c_void_p),
                ("inputs", ctypes.c_void_p), ("input_genome_stride", ctypes.c_int64),
                ("B", ctypes.c_int32), ("grid_side", ctypes.c_int32),
                ("grid_first", ctypes.c_int64), ("outputs", ctypes.c_void_p)]


class ServerCfg(ctypes.Structure):
    """neat_server_cfg."""
    _fields_ = [("device", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("cap_bytes", ctypes.c_uint64), ("tune_cache_path", ctypes.c_char_p)]


class Request(ctypes.Structure):
    """neat_request."""
    _fields_ = [("pop_id", ctypes.c_int32), ("input_mode", ctypes.c_int32),
                ("inputs", ctypes.c_void_p), ("input_genome_stride", ctypes.c_int64),
                ("B", ctypes.c_int32), ("grid_side", ctypes.c_int32),
                ("grid_first", ctypes.c_int64), ("outputs", ctypes.c_void_p),
                ("tag", ctypes.c_uint64)]


class Result(ctypes.Structure):
    """neat_result."""
    _fields_ = [("status", ctypes.c_int32), ("tag", ctypes.c_uint64),
                ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class Stats(ctypes.Structure):
    """neat_stats."""
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("queued", ctypes.c_uint64),
                ("genome_inputs", ctypes.c_uint64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("throughput", ctypes.c_double),
                ("batched_requests", ctypes.c_uint64), ("resident_bytes", ctypes.c_uint64),
                ("peak_bytes", ctypes.c_uint64)]


INPUT_TENSOR, INPUT_GRID = 0, 1

_lib = None

# exported symbol -> (restype, argtypes)
_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
SIGNATURES = {
    "neat_program_bytes": (_sz, [ctypes.POINTER(Dims)]),
    "neat_program_stride": (_sz, [ctypes.POINTER(Dims)]),
    "neat_topo_sort": (_i32, [ctypes.POINTER(Dims), _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "neat_forward": (_i32, [ctypes.POINTER(Dims), _vp, _vp, _i64, _i32, _vp, _vp]),
    "neat_forward_ex": (_i32, [ctypes.POINTER(Dims), _vp, _vp, _i64, _i32, _vp, _i32, _vp]),
    "neat_autotune_forward": (_i32, [ctypes.POINTER(Dims), _vp, _vp, _i64, _i32, _vp, _i32,
                                     _vp, _vp, _vp]),
    "neat_tuned_variant": (_i32, [ctypes.POINTER(Dims), _i32, _i32, _i32]),
    "neat_tune_clear": (None, []),
    "neat_forward_grid": (_i32, [ctypes.POINTER(Dims), _vp, _i32, _i64, _i32, _vp, _vp]),
    "neat_apply_edits": (_i32, [ctypes.POINTER(Dims), _vp, _vp, _vp, _i32, _vp, _vp]),
    "neat_crossover": (_i32, [ctypes.POINTER(Dims), _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp,
                              _vp]),
    "neat_distance": (_i32, [ctypes.POINTER(Dims), _vp, _vp, _i32, _vp, _vp, ctypes.c_float,
                             ctypes.c_float, _vp, _vp]),
    "neat_substrate_forward": (_i32, [ctypes.POINTER(Dims), _vp, _i32, ctypes.c_float, _vp,
                                      _i32, _vp, _vp, _vp]),
    "neat_topo_sort_recurrent": (_i32, [ctypes.POINTER(Dims), _vp, _vp, _vp, _vp, _vp, _vp,
                                        _vp]),
    "neat_forward_recurrent": (_i32, [ctypes.POINTER(Dims), _vp, _vp, _i64, _i32, _i32, _vp,
                                      _vp]),
    "neat_forward_batch": (_i32, [ctypes.POINTER(BatchItem), _i32,
                                  ctypes.POINTER(ctypes.c_void_p), _vp]),
    "neat_batch_plan_free": (None, [_vp]),
    "neat_forward_batch_noalloc": (_i32, [ctypes.POINTER(BatchItem), _i32, _vp]),
    "neat_batch_plan_launches": (_i32, [_vp]),
    "neat_server_create": (_i32, [ctypes.POINTER(ServerCfg), ctypes.POINTER(ctypes.c_void_p)]),
    "neat_server_destroy": (_i32, [_vp]),
    "neat_server_register": (_i32, [_vp, ctypes.POINTER(Dims), _vp, _vp,
                                    ctypes.POINTER(ctypes.c_int32)]),
    "neat_submit": (_i32, [_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "neat_submit_many": (_i32, [_vp, ctypes.POINTER(Request), _i32,
                                ctypes.POINTER(ctypes.c_uint64)]),
    "neat_poll": (_i32, [_vp, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "neat_server_stats": (_i32, [_vp, ctypes.POINTER(Stats)]),
    "neat_server_reset_stats": (_i32, [_vp]),
    "neat_last_error": (ctypes.c_char_p, []),
    "neat_strerror": (ctypes.c_char_p, [_i32]),
}


def lib():
    """Load libneat.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libneat.so is not built; run `python -m paper_2404_01817_amd.build`")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def check(rc: int) -> int:
    if rc < 0:
        raise NeatError(rc, lib().neat_last_error().decode())
    return rc
