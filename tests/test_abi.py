"""The C-ABI library: it loads, exports every function include/neat.h
declares, and rejects invalid arguments on the host (no GPU needed: these
paths return before any HIP call)."""
import ctypes
import os
import re

import pytest

from paper_2404_01817_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(neat_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("neat_topo_sort", "neat_forward", "neat_program_bytes", "neat_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, "binding lacks " + n


def test_program_bytes_and_invalid_dims():
    lib = _lib.lib()
    d = _lib.Dims(10, 50, 200, 17, 6)
    nb = lib.neat_program_bytes(ctypes.byref(d))
    # P per-genome programs of 256-byte multiples, then the population area
    # (a 256-byte header and one word per genome, padded to 64 words)
    d1 = _lib.Dims(1, 50, 200, 17, 6)
    nb1 = lib.neat_program_bytes(ctypes.byref(d1))
    per = (nb1 - 512)
    assert nb > 0 and per > 0 and per % 256 == 0
    assert nb == 10 * per + 512
    for bad in [(1, 0, 4, 1, 1), (1, 8, 4, 0, 1), (1, 8, 4, 4, 5), (-1, 8, 4, 1, 1),
                (1, 2000, 4, 1, 1), (1, 8, -1, 1, 1)]:
        db = _lib.Dims(*bad)
        assert lib.neat_program_bytes(ctypes.byref(db)) == 0
        rc = lib.neat_topo_sort(ctypes.byref(db), None, None, None, None, None, None, None)
        assert rc == -1 and lib.neat_last_error()
        rc = lib.neat_forward(ctypes.byref(db), None, None, 0, 4, None, None)
        assert rc == -1
    # NULL dims, negative B, bad stride, bad grid arguments
    assert lib.neat_forward(None, None, None, 0, 4, None, None) == -1
    assert lib.neat_forward(ctypes.byref(d), None, None, 0, -1, None, None) == -1
    assert lib.neat_forward(ctypes.byref(d), ctypes.c_void_p(256), ctypes.c_void_p(256),
                            5, 4, ctypes.c_void_p(256), None) == -1
    assert b"stride" in lib.neat_last_error()
    assert lib.neat_forward_grid(ctypes.byref(d), None, 16, 0, 10, None, None) == -1  # I != 5
    d5 = _lib.Dims(1, 30, 120, 5, 1)
    assert lib.neat_forward_grid(ctypes.byref(d5), None, 16, 65530, 10, None, None) == -1
    assert lib.neat_forward_grid(ctypes.byref(d5), None, 1, 0, 1, None, None) == -1
    # P = 0 and B = 0 are accepted no-ops
    d0 = _lib.Dims(0, 8, 16, 3, 1)
    assert lib.neat_topo_sort(ctypes.byref(d0), None, None, None, None, None, None, None) == 0
    assert lib.neat_forward(ctypes.byref(d), None, None, 0, 0, None, None) == 0
    assert lib.neat_strerror(-4) == b"request larger than the admission cap"


def test_server_create_reports_errors_without_crashing():
    """Invalid configurations fail with NEAT_E_INVALID before touching a
    device; on a machine without a GPU a valid one fails with an error code
    too (never a silent host fallback)."""
    lib = _lib.lib()
    h = ctypes.c_void_p(None)
    bad = _lib.ServerCfg(0, 0, 1 << 20)  # max_inflight = 0
    rc = lib.neat_server_create(ctypes.byref(bad), ctypes.byref(h))
    assert rc < 0 and h.value is None
    assert lib.neat_server_create(None, ctypes.byref(h)) == -1
    assert lib.neat_submit(None, None, None) == -1
    assert lib.neat_poll(None, 1, None) == -1
    assert lib.neat_server_destroy(None) == -1


_COMPUTE = ["neat_topo_sort", "neat_forward", "neat_forward_ex", "neat_autotune_forward",
            "neat_forward_grid", "neat_distance", "neat_apply_edits", "neat_crossover",
            "neat_substrate_forward", "neat_topo_sort_recurrent", "neat_forward_recurrent",
            "neat_forward_batch", "neat_forward_batch_noalloc", "neat_server_create",
            "neat_server_destroy", "neat_server_register", "neat_submit", "neat_submit_many",
            "neat_poll", "neat_server_stats", "neat_server_reset_stats"]
_INTS = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_float)


def test_every_entry_point_refuses_null_arguments():
    """Every compute and server entry point, given NULL for each pointer
    (and 1 for each count), fails with NEAT_E_INVALID and a message before
    touching a device, so it behaves the same with or without a GPU."""
    lib = _lib.lib()
    for name in _COMPUTE:
        _, args = _lib.SIGNATURES[name]
        vals = [1 if a in _INTS else None for a in args]
        rc = getattr(lib, name)(*vals)
        assert rc == -1, (name, rc)
        assert lib.neat_last_error().decode(), name


def test_invalid_dims_are_refused_before_any_access():
    """Out-of-range dims fail with NEAT_E_INVALID naming the field; the
    (host) pointers passed are never dereferenced."""
    lib = _lib.lib()
    buf = (ctypes.c_float * 16)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    cases = [((1, 0, 4, 1, 1), "N_max"), ((1, 20000, 4, 1, 1), "N_max"),
             ((-1, 8, 4, 1, 1), "P"), ((1, 8, -1, 1, 1), "C_max"),
             ((1, 8, 1 << 20, 1, 1), "C_max"), ((1, 8, 4, 0, 1), "I"), ((1, 8, 4, 6, 3), "I")]
    for dims, field in cases:
        d = _lib.Dims(*dims)
        rc = lib.neat_topo_sort(ctypes.byref(d), p, p, p, p, p, p, None)
        assert rc == -1, dims
        assert field in lib.neat_last_error().decode(), (dims, lib.neat_last_error())
        rc = lib.neat_forward(ctypes.byref(d), p, p, 0, 1, p, None)
        assert rc == -1, dims
