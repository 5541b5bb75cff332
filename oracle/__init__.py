"""CPU oracle for the population forward of tensorized NEAT.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2404_01817_amd``) and neither imports the
other.

What lives here:

* ``neat_oracle.c`` (loaded through ctypes): the plain definition of the
  paper's inference (Section 3.3) on adjacency lists, in IEEE double, plus a
  float instantiation of the same code and a first-order fp32 error bound
  (``transform``, ``forward``); the recurrent reading by synchronous sweeps
  (``forward_recurrent``); and the gene-level operators of a generation:
  compatibility distance, crossover and the tensorized edits of Section 3.2
  (``distance``, ``crossover``, ``edit``).
* ``dense.py``: the paper's own dense formulation (N_order and the expanded
  connection tensor C_exp of Section 3.3) written out in numpy, used to
  cross-check the C oracle.
* ``substrate.py``: the HyperNEAT substrate layer (CPPN weights from the C
  oracle, threshold, numpy contraction) with its fp32 bound.

Status bits (per genome): BAD_VALUE 1, DUP_KEY 2, MISSING_IO 4, BAD_REF 8,
INTO_INPUT 16, DUP_EDGE 32, CYCLE 64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "neat_oracle.c")
_INC = os.path.join(_HERE, "neat_oracle_forward.inc")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

BAD_VALUE, DUP_KEY, MISSING_IO, BAD_REF, INTO_INPUT, DUP_EDGE, CYCLE = (
    1, 2, 4, 8, 16, 32, 64)

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math, no FMA
    contraction) into ``oracle/liboracle.so``."""
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(_SRC), os.path.getmtime(_INC))
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_transform.argtypes = [i32] * 5 + [vp] * 5
        lib.oracle_transform.restype = i32
        lib.oracle_transform_recurrent.argtypes = [i32] * 5 + [vp] * 5
        lib.oracle_transform_recurrent.restype = i32
        for name in ("oracle_forward_f64", "oracle_forward_f32"):
            fn = getattr(lib, name)
            fn.argtypes = [i32] * 5 + [vp, vp, vp, i64, i32, vp, vp]
            fn.restype = i32
        lib.oracle_edit.argtypes = [i32] * 3 + [vp, vp, i32, vp, vp]
        lib.oracle_edit.restype = i32
        lib.oracle_crossover.argtypes = [i32] * 3 + [vp] * 7
        lib.oracle_crossover.restype = i32
        lib.oracle_distance.argtypes = [i32] * 4 + [vp] * 4 + [ctypes.c_double] * 2 + [vp] * 2
        lib.oracle_distance.restype = i32
        for name in ("oracle_forward_recurrent_f64", "oracle_forward_recurrent_f32"):
            fn = getattr(lib, name)
            fn.argtypes = [i32] * 5 + [vp, vp, vp, i64, i32, i32, vp, vp]
            fn.restype = i32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _check_genomes(nodes, conns, I, O):
    nodes = np.ascontiguousarray(nodes, dtype=np.float32)
    conns = np.ascontiguousarray(conns, dtype=np.float32)
    if nodes.ndim != 3 or nodes.shape[2] != 5:
        raise ValueError("nodes must be [P, N_max, 5]")
    if conns.ndim != 3 or conns.shape[2] != 4 or conns.shape[0] != nodes.shape[0]:
        raise ValueError("conns must be [P, C_max, 4]")
    return nodes, conns


def transform(nodes, conns, I: int, O: int, recurrent: bool = False):
    """Transformation stage: returns (order [P,N_max] i32, level [P,N_max]
    i32, status [P] u32).  ``order`` lists node rows by (level, key), -1
    padded; rejected genomes get all -1 rows.  With ``recurrent`` cycles are
    allowed (CYCLE is never set), every valid row has level 0 and the order
    is plain key order."""
    nodes, conns = _check_genomes(nodes, conns, I, O)
    P, N, _ = nodes.shape
    C = conns.shape[1]
    order = np.empty((P, N), np.int32)
    level = np.empty((P, N), np.int32)
    status = np.empty((P,), np.uint32)
    fn = _load().oracle_transform_recurrent if recurrent else _load().oracle_transform
    rc = fn(P, N, C, I, O, _ptr(nodes), _ptr(conns), _ptr(order), _ptr(level), _ptr(status))
    if rc != 0:
        raise RuntimeError("oracle_transform failed: %d" % rc)
    return order, level, status


def _inputs(inputs, P, I, shared_inputs):
    x = np.ascontiguousarray(inputs, dtype=np.float32)
    if shared_inputs:
        if x.ndim != 2 or x.shape[1] != I:
            raise ValueError("shared inputs must be [B, I]")
        return x, x.shape[0], 0
    if x.ndim != 3 or x.shape[0] != P or x.shape[2] != I:
        raise ValueError("inputs must be [P, B, I]")
    return x, x.shape[1], x.shape[1] * I


def forward(nodes, conns, inputs, I: int, O: int, shared_inputs=False,
            precision="f64", with_beta=True):
    """Transformation + calculation.

    ``inputs`` is [P, B, I] (or [B, I] with ``shared_inputs``), float32.
    Returns outputs [P, B, O] (float64 or float32) and, for f64 with
    ``with_beta``, beta [P, B, O]: a first-order bound on the error of an fp32
    evaluation of the same graph (inf where fp32 may overflow)."""
    return _forward(nodes, conns, inputs, I, O, shared_inputs, precision, with_beta, None)


def forward_recurrent(nodes, conns, inputs, I: int, O: int, K: int, shared_inputs=False,
                      precision="f64", with_beta=True):
    """Recurrent transformation + K synchronous sweeps (a reading; see
    neat_oracle_forward.inc): v0 = inputs at the input keys, 0 elsewhere;
    every sweep recomputes every non-input node from the previous sweep's
    values; the outputs are the values after sweep K.  Returns as
    ``forward``."""
    if K < 0:
        raise ValueError("K must be >= 0")
    return _forward(nodes, conns, inputs, I, O, shared_inputs, precision, with_beta, K)


def _forward(nodes, conns, inputs, I, O, shared_inputs, precision, with_beta, K):
    nodes, conns = _check_genomes(nodes, conns, I, O)
    P, N, _ = nodes.shape
    C = conns.shape[1]
    x, B, stride = _inputs(inputs, P, I, shared_inputs)
    lib = _load()
    rec = K is not None
    extra = (K,) if rec else ()
    if precision == "f64":
        fn = lib.oracle_forward_recurrent_f64 if rec else lib.oracle_forward_f64
        y = np.empty((P, B, O), np.float64)
        beta = np.empty((P, B, O), np.float64) if with_beta else None
        rc = fn(P, N, C, I, O, _ptr(nodes), _ptr(conns), _ptr(x), stride, B, *extra, _ptr(y),
                _ptr(beta) if beta is not None else None)
        if rc != 0:
            raise RuntimeError("oracle forward (f64) failed: %d" % rc)
        return (y, beta) if with_beta else y
    if precision == "f32":
        fn = lib.oracle_forward_recurrent_f32 if rec else lib.oracle_forward_f32
        y = np.empty((P, B, O), np.float32)
        rc = fn(P, N, C, I, O, _ptr(nodes), _ptr(conns), _ptr(x), stride, B, *extra, _ptr(y),
                None)
        if rc != 0:
            raise RuntimeError("oracle forward (f32) failed: %d" % rc)
        return y
    raise ValueError("precision must be 'f64' or 'f32'")


def distance(nodes, conns, rnodes, rconns, c_disjoint=1.0, c_homologous=0.5):
    """Compatibility distance of every genome to every representative
    ([P, Q] float64) and its fp32 error bound (see neat_oracle.c)."""
    nodes, conns = _check_genomes(nodes, conns, 1, 1)
    rnodes, rconns = _check_genomes(rnodes, rconns, 1, 1)
    if rnodes.shape[1:] != nodes.shape[1:] or rconns.shape[1:] != conns.shape[1:]:
        raise ValueError("representatives must have the population's N_max and C_max")
    P, N, _ = nodes.shape
    Q, C = rnodes.shape[0], conns.shape[1]
    out = np.empty((P, Q), np.float64)
    bound = np.empty((P, Q), np.float64)
    rc = _load().oracle_distance(P, Q, N, C, _ptr(nodes), _ptr(conns), _ptr(rnodes),
                                 _ptr(rconns), float(c_disjoint), float(c_homologous),
                                 _ptr(out), _ptr(bound))
    if rc != 0:
        raise RuntimeError("oracle_distance failed: %d" % rc)
    return out, bound


EDIT_DTYPE = np.dtype([("genome", "<i4"), ("op", "<i4"), ("row", "<i4"), ("column", "<i4"),
                       ("v", "<f4", (5,))])
NODE_ADD, NODE_DEL, CONN_ADD, CONN_DEL, NODE_SET, CONN_SET = range(6)


def edit(nodes, conns, edits):
    """Apply the tensorized edits (EDIT_DTYPE records, see neat_oracle.c) to
    copies of nodes/conns; returns (nodes, conns, applied [n] i32)."""
    nodes = np.array(nodes, dtype=np.float32, copy=True, order="C")
    conns = np.array(conns, dtype=np.float32, copy=True, order="C")
    edits = np.ascontiguousarray(edits, dtype=EDIT_DTYPE)
    applied = np.empty((len(edits),), np.int32)
    rc = _load().oracle_edit(nodes.shape[0], nodes.shape[1], conns.shape[1], _ptr(nodes),
                             _ptr(conns), len(edits), _ptr(edits), _ptr(applied))
    if rc != 0:
        raise RuntimeError("oracle_edit failed: %d" % rc)
    return nodes, conns, applied


def crossover(nodes, conns, pairs, rn, rc):
    """Children of the parent pairs [Pc, 2] (fitter parent first) with the
    per-row uniform numbers rn [Pc, N_max], rc [Pc, C_max] (see
    neat_oracle.c); returns (child nodes, child conns)."""
    nodes, conns = _check_genomes(nodes, conns, 1, 1)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32)
    Pc = pairs.shape[0]
    N, C = nodes.shape[1], conns.shape[1]
    rn = np.ascontiguousarray(rn, dtype=np.float32).reshape(Pc, N)
    rc = np.ascontiguousarray(rc, dtype=np.float32).reshape(Pc, C)
    if pairs.ndim != 2 or pairs.shape[1] != 2 or pairs.min(initial=0) < 0 \
            or pairs.max(initial=0) >= nodes.shape[0]:
        raise ValueError("pairs must be [Pc, 2] parent indices")
    cn = np.empty((Pc, N, 5), np.float32)
    cc = np.empty((Pc, C, 4), np.float32)
    rc_ = _load().oracle_crossover(Pc, N, C, _ptr(nodes), _ptr(conns), _ptr(pairs), _ptr(rn),
                                   _ptr(rc), _ptr(cn), _ptr(cc))
    if rc_ != 0:
        raise RuntimeError("oracle_crossover failed: %d" % rc_)
    return cn, cc


def order_keys(nodes, order):
    """Express an order (node rows) as node keys, -1 padded."""
    nodes = np.asarray(nodes)
    P, N = order.shape
    out = np.full((P, N), -1, np.int64)
    for p in range(P):
        for i in range(N):
            r = order[p, i]
            if r >= 0:
                out[p, i] = int(nodes[p, r, 0])
    return out


def within_tolerance(y_gpu, y64, beta, atol=1e-5):
    """The parity rule for fp32 results against the f64 oracle.

    An output passes when
      * beta is infinite (fp32 may overflow there; only counted), or
      * the oracle value is NaN and the fp32 value is NaN too, or
      * |y_gpu - y64| <= atol + 2 * beta.
    Returns (ok_mask, stats)."""
    y_gpu = np.asarray(y_gpu, dtype=np.float64)
    y64 = np.asarray(y64, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    unbounded = np.isinf(beta)
    ref_nan = np.isnan(y64) & ~unbounded
    finite = ~unbounded & ~np.isnan(y64)
    err = np.where(finite, np.abs(y_gpu - y64), 0.0)
    err = np.where(np.isnan(err), np.inf, err)
    ok = unbounded | (ref_nan & np.isnan(y_gpu)) | (finite & (err <= atol + 2.0 * beta))
    well = finite & (beta <= 1e-6)
    stats = {
        "n": int(y64.size),
        "max_abs_err_well_conditioned": float(err[well].max()) if well.any() else 0.0,
        "max_abs_err": float(err[finite].max()) if finite.any() else 0.0,
        "n_ill_conditioned": int((finite & (beta > 1e-6)).sum()),
        "n_unbounded": int(unbounded.sum()),
        "n_nan_ref": int(ref_nan.sum()),
        "n_fail": int((~ok).sum()),
    }
    return ok, stats
