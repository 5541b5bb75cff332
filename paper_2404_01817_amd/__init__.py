"""MI355X-native population forward of tensorized NEAT (Wang et al., GECCO
2024): transformation (topological sort + program build) and calculation
(forward over population x inputs) as hand-written HIP kernels for gfx950
behind the C ABI of ``include/neat.h``.

The functions here marshal torch tensors into that ABI.  torch supplies
device memory and the current HIP stream; nothing is computed in Python.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

from ._lib import (FWD_AUTO, FWD_LDS, FWD_LVL, FWD_REG, FWD_REG2, FWD_SEG, FWD_TUNED,
                   TUNE_CANDIDATES,
                   INPUT_GRID, INPUT_TENSOR,
                   BatchItem, Dims, NeatError, Request, Result, ServerCfg, Stats, check, lib)

__all__ = ["Dims", "NeatError", "dims_of", "program_bytes", "topo_sort", "forward",
           "autotune_forward", "forward_grid", "forward_recurrent", "substrate_forward", "distance",
           "crossover", "edit"]


def _torch():
    import torch
    return torch


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    torch = _torch()
    # the current stream's handle without building a Stream object (a few
    # microseconds per call otherwise); the public path where torch lacks it
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return ctypes.c_void_p(raw(torch.cuda.current_device()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> Optional[ctypes.c_void_p]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f32(t, name):
    torch = _torch()
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("%s must be a contiguous float32 CUDA tensor" % name)


def dims_of(nodes, conns, I: int, O: int) -> Dims:
    if nodes.dim() != 3 or nodes.shape[2] != 5:
        raise ValueError("nodes must be [P, N_max, 5]")
    if conns.dim() != 3 or conns.shape[2] != 4 or conns.shape[0] != nodes.shape[0]:
        raise ValueError("conns must be [P, C_max, 4]")
    return Dims(nodes.shape[0], nodes.shape[1], conns.shape[1], I, O)


def program_bytes(dims: Dims) -> int:
    return int(lib().neat_program_bytes(ctypes.byref(dims)))


def program_words_per_genome(dims: Dims) -> int:
    """32-bit words between consecutive genomes' parts of the program."""
    return int(lib().neat_program_stride(ctypes.byref(dims))) // 4


def program_headers(dims: Dims, program):
    """The diagnostic header words [P, 16] of every genome (device tensor
    view; see neat_program_stride)."""
    w = program_words_per_genome(dims)
    return program[:dims.P * w].view(dims.P, w)[:, :16]


def topo_sort(nodes, conns, I: int, O: int, program=None, stream=None,
              want_order: bool = True, recurrent: bool = False, status=None):
    """Transformation stage.  nodes [P,N_max,5], conns [P,C_max,4] float32 on
    the GPU.  Returns (order, level, status, program) as device tensors
    (order/level None unless ``want_order``; program and status are written
    into the given tensors when passed).  ``recurrent``: cycles allowed,
    key order, a program for ``forward_recurrent``
    (neat_topo_sort_recurrent)."""
    torch = _torch()
    _dev_f32(nodes, "nodes")
    _dev_f32(conns, "conns")
    d = dims_of(nodes, conns, I, O)
    dev = nodes.device
    order = level = None
    if want_order:
        order = torch.empty((d.P, d.N_max), dtype=torch.int32, device=dev)
        level = torch.empty((d.P, d.N_max), dtype=torch.int32, device=dev)
    if status is None:
        status = torch.empty((d.P,), dtype=torch.int32, device=dev)
    elif status.numel() < d.P or status.dtype != torch.int32 or not status.is_cuda:
        raise ValueError("status must be an int32 device tensor of at least P elements")
    if program is None:
        program = torch.empty((max(program_bytes(d), 4) // 4,), dtype=torch.int32, device=dev)
    fn = lib().neat_topo_sort_recurrent if recurrent else lib().neat_topo_sort
    check(fn(ctypes.byref(d), _ptr(nodes), _ptr(conns), _ptr(order), _ptr(level), _ptr(status),
             _ptr(program), _stream(stream)))
    return order, level, status, program


def _io(dims, inputs, B, shared_inputs, outputs):
    torch = _torch()
    _dev_f32(inputs, "inputs")
    if shared_inputs:
        stride = 0
        if inputs.numel() < B * dims.I:
            raise ValueError("shared inputs smaller than B * I")
    else:
        stride = B * dims.I
        if inputs.numel() < dims.P * stride:
            raise ValueError("inputs smaller than P * B * I")
    if outputs is None:
        outputs = torch.empty((dims.P, B, dims.O), dtype=torch.float32, device=inputs.device)
    else:
        _dev_f32(outputs, "outputs")
        if outputs.numel() < dims.P * B * dims.O:
            raise ValueError("outputs smaller than P * B * O")
    return stride, outputs


def forward(dims: Dims, program, inputs, B: int, shared_inputs: bool = False,
            outputs=None, stream=None, variant: int = 0):
    """Calculation stage.  inputs [P,B,I] (or [B,I] when shared) float32 on the
    GPU; returns outputs [P,B,O]."""
    stride, outputs = _io(dims, inputs, B, shared_inputs, outputs)
    check(lib().neat_forward_ex(ctypes.byref(dims), _ptr(program), _ptr(inputs), stride, B,
                                _ptr(outputs), variant, _stream(stream)))
    return outputs



def autotune_forward(dims: Dims, program, inputs, B: int, outputs=None, reps: int = 5,
                     stream=None):
    """Time the forward variants on these buffers and record the fastest for
    the call's bucket (neat_autotune_forward); returns (latency winner, [ms
    of FWD_REG, FWD_REG2, FWD_LDS, FWD_LVL, FWD_SEG alone, then per copy on
    a full GPU]).  Later calls with variant=FWD_TUNED, and
    batches, use the recorded variant."""
    stride, outputs = _io(dims, inputs, B, False, outputs)
    v = ctypes.c_int32(0)
    ms = (ctypes.c_float * (2 * TUNE_CANDIDATES))()
    check(lib().neat_autotune_forward(ctypes.byref(dims), _ptr(program), _ptr(inputs), stride, B,
                                      _ptr(outputs), reps, ctypes.byref(v), ms, _stream(stream)))
    return v.value, [float(x) for x in ms]


def tune_clear() -> None:
    """Forget every tuned variant and detach any tune cache file
    (neat_tune_clear)."""
    lib().neat_tune_clear()


def tuned_variant(dims: Dims, B: int, grid: bool = False, throughput: bool = False) -> int:
    """The variant recorded for the call's bucket (neat_tuned_variant): the
    latency winner, or the throughput winner that batches use."""
    return check(lib().neat_tuned_variant(ctypes.byref(dims), B, int(grid), int(throughput)))

def distance(nodes, conns, rnodes, rconns, c_disjoint: float = 1.0,
             c_homologous: float = 0.5, out=None, stream=None):
    """Compatibility distance of every genome (nodes [P,N,5], conns [P,C,4])
    to every representative (rnodes [Q,N,5], rconns [Q,C,4]); returns
    [P, Q] float32 (neat_distance)."""
    torch = _torch()
    for t, name in ((nodes, "nodes"), (conns, "conns"), (rnodes, "rnodes"), (rconns, "rconns")):
        _dev_f32(t, name)
    d = dims_of(nodes, conns, 1, 1)
    if rnodes.shape[1:] != nodes.shape[1:] or rconns.shape[1:] != conns.shape[1:] \
            or rnodes.shape[0] != rconns.shape[0]:
        raise ValueError("representatives must have the population's N_max and C_max")
    Q = rnodes.shape[0]
    if out is None:
        out = torch.empty((d.P, Q), dtype=torch.float32, device=nodes.device)
    else:
        _dev_f32(out, "out")
        if out.numel() < d.P * Q:
            raise ValueError("out smaller than P * Q")
    check(lib().neat_distance(ctypes.byref(d), _ptr(nodes), _ptr(conns), Q, _ptr(rnodes),
                              _ptr(rconns), ctypes.c_float(c_disjoint),
                              ctypes.c_float(c_homologous), _ptr(out), _stream(stream)))
    return out


def edit(nodes, conns, edits, applied=None, stream=None):
    """Apply tensorized edits in place (neat_apply_edits): ``edits`` is a device
    uint8/int32 tensor holding neat_edit records (36 bytes each, sorted by
    genome); returns applied [n] int32."""
    torch = _torch()
    _dev_f32(nodes, "nodes")
    _dev_f32(conns, "conns")
    if not (edits.is_cuda and edits.is_contiguous() and edits.numel() * edits.element_size()
            % 36 == 0):
        raise ValueError("edits must be a contiguous CUDA tensor of 36-byte records")
    n = edits.numel() * edits.element_size() // 36
    d = dims_of(nodes, conns, 1, 1)
    if applied is None:
        applied = torch.empty((n,), dtype=torch.int32, device=nodes.device)
    check(lib().neat_apply_edits(ctypes.byref(d), _ptr(nodes), _ptr(conns), _ptr(edits), n,
                          _ptr(applied), _stream(stream)))
    return applied


def crossover(nodes, conns, pairs, rn, rc, child_nodes=None, child_conns=None, stream=None):
    """Children of the parent pairs [Pc, 2] (int32, fitter parent first) with
    uniform numbers rn [Pc, N_max], rc [Pc, C_max] (neat_crossover);
    returns (child nodes, child conns)."""
    torch = _torch()
    for t, name in ((nodes, "nodes"), (conns, "conns"), (rn, "rn"), (rc, "rc")):
        _dev_f32(t, name)
    if not (pairs.is_cuda and pairs.dtype == torch.int32 and pairs.is_contiguous()):
        raise ValueError("pairs must be a contiguous int32 CUDA tensor")
    d = dims_of(nodes, conns, 1, 1)
    Pc = pairs.shape[0]
    if pairs.dim() != 2 or pairs.shape[1] != 2 or rn.numel() < Pc * d.N_max \
            or rc.numel() < Pc * d.C_max:
        raise ValueError("pairs [Pc, 2], rn [Pc, N_max], rc [Pc, C_max]")
    if child_nodes is None:
        child_nodes = torch.empty((Pc, d.N_max, 5), dtype=torch.float32, device=nodes.device)
    if child_conns is None:
        child_conns = torch.empty((Pc, d.C_max, 4), dtype=torch.float32, device=nodes.device)
    check(lib().neat_crossover(ctypes.byref(d), _ptr(nodes), _ptr(conns), Pc, _ptr(pairs),
                               _ptr(rn), _ptr(rc), _ptr(child_nodes), _ptr(child_conns),
                               _stream(stream)))
    return child_nodes, child_conns


def substrate_forward(dims: Dims, program, side: int, x, threshold: float = 0.2,
                      weights=None, outputs=None, stream=None):
    """HyperNEAT substrate layer: CPPN weights on all side^2 x side^2 point
    pairs (written to ``weights`` [P, S, S]), thresholded, then
    tanh(x W') for the shared input planes x [B, S].  Returns
    (outputs [P, B, S], weights)."""
    torch = _torch()
    _dev_f32(x, "x")
    S = side * side
    if x.dim() != 2 or x.shape[1] != S:
        raise ValueError("x must be [B, side^2]")
    B = x.shape[0]
    if weights is None:
        weights = torch.empty((dims.P, S, S), dtype=torch.float32, device=x.device)
    else:
        _dev_f32(weights, "weights")
        if weights.numel() < dims.P * S * S:
            raise ValueError("weights smaller than P * S * S")
    if outputs is None:
        outputs = torch.empty((dims.P, B, S), dtype=torch.float32, device=x.device)
    else:
        _dev_f32(outputs, "outputs")
        if outputs.numel() < dims.P * B * S:
            raise ValueError("outputs smaller than P * B * S")
    check(lib().neat_substrate_forward(ctypes.byref(dims), _ptr(program), side,
                                       ctypes.c_float(threshold), _ptr(x), B, _ptr(weights),
                                       _ptr(outputs), _stream(stream)))
    return outputs, weights


def forward_recurrent(dims: Dims, program, inputs, B: int, K: int,
                      shared_inputs: bool = False, outputs=None, stream=None):
    """K synchronous sweeps of a recurrent network (program from
    ``topo_sort(..., recurrent=True)``); returns outputs [P,B,O]."""
    stride, outputs = _io(dims, inputs, B, shared_inputs, outputs)
    check(lib().neat_forward_recurrent(ctypes.byref(dims), _ptr(program), _ptr(inputs), stride,
                                       B, K, _ptr(outputs), _stream(stream)))
    return outputs


def forward_grid(dims: Dims, program, side: int, first: int, Q: int, outputs=None,
                 stream=None):
    """CPPN substrate queries generated in the kernel; returns [P,Q,O]."""
    torch = _torch()
    if outputs is None:
        outputs = torch.empty((dims.P, Q, dims.O), dtype=torch.float32, device=program.device)
    else:
        _dev_f32(outputs, "outputs")
        if outputs.numel() < dims.P * Q * dims.O:
            raise ValueError("outputs smaller than P * Q * O")
    check(lib().neat_forward_grid(ctypes.byref(dims), _ptr(program), side, first, Q,
                                  _ptr(outputs), _stream(stream)))
    return outputs


def batch_item(dims: Dims, program, outputs, inputs=None, B: int = 0,
               shared_inputs: bool = False, nodes=None, conns=None, status=None,
               grid_side: int = 0, grid_first: int = 0) -> BatchItem:
    """One population of a batch (neat_batch_item).  With nodes/conns the
    batch also runs its transformation into ``program`` (and ``status``).
    TENSOR mode: inputs [P,B,I] (or [B,I] when shared); GRID mode
    (grid_side > 0): B queries from grid_first."""
    if grid_side:
        stride = 0
    else:
        _dev_f32(inputs, "inputs")
        stride = 0 if shared_inputs else B * dims.I
    def addr(t):
        return None if t is None else t.data_ptr()

    it = BatchItem()
    it.dims = dims
    it.nodes, it.conns, it.status = addr(nodes), addr(conns), addr(status)
    it.program = addr(program)
    it.inputs = addr(inputs)
    it.input_genome_stride = stride
    it.B = B
    it.grid_side = grid_side
    it.grid_first = grid_first
    it.outputs = addr(outputs)
    return it


class BatchPlan:
    """A batch recorded into a HIP graph by neat_forward_batch; running it
    again with the same items replays the graph."""

    def __init__(self):
        self._h = ctypes.c_void_p(None)

    def run(self, items, stream=None):
        arr = (BatchItem * len(items))(*items)
        check(lib().neat_forward_batch(arr, len(items), ctypes.byref(self._h), _stream(stream)))

    @property
    def launches(self) -> int:
        return int(lib().neat_batch_plan_launches(self._h))

    def free(self):
        if self._h.value:
            lib().neat_batch_plan_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def forward_batch_noalloc(items, stream=None) -> None:
    """The batch of ``BatchPlan.run`` without device allocation
    (neat_forward_batch_noalloc): launched directly on the stream, work-unit
    tables in the library's static scratch area."""
    arr = (BatchItem * len(items))(*items) if items else None
    check(lib().neat_forward_batch_noalloc(arr, len(items), _stream(stream)))


class Server:
    """Resident populations and continuous batching (neat_server_*)."""

    def __init__(self, device: int = 0, cap_bytes: int = 64 << 30, max_inflight: int = 4,
                 tune_cache_path: str = None):
        cfg = ServerCfg(device, max_inflight, cap_bytes,
                        tune_cache_path.encode() if tune_cache_path else None)
        self._h = ctypes.c_void_p(None)
        check(lib().neat_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))

    def register(self, nodes, conns, I: int, O: int) -> int:
        """Copy a population (device tensors) into the server and transform
        it once; returns its id."""
        _dev_f32(nodes, "nodes")
        _dev_f32(conns, "conns")
        d = dims_of(nodes, conns, I, O)
        pid = ctypes.c_int32(-1)
        check(lib().neat_server_register(self._h, ctypes.byref(d), _ptr(nodes), _ptr(conns),
                                         ctypes.byref(pid)))
        return pid.value

    @staticmethod
    def request(pop_id: int, outputs, inputs=None, B: int = 0, shared_inputs=False,
                grid_side: int = 0, grid_first: int = 0, tag: int = 0, I: int = 0):
        """A request record for submit_many (arguments as submit)."""
        r = Request()
        r.pop_id = pop_id
        if grid_side:
            r.input_mode = INPUT_GRID
            r.grid_side, r.grid_first = grid_side, grid_first
        else:
            r.input_mode = INPUT_TENSOR
            r.inputs = inputs.data_ptr()
            r.input_genome_stride = 0 if shared_inputs else B * I
        r.B = B
        r.outputs = outputs.data_ptr()
        r.tag = tag
        return r

    def submit_many(self, requests) -> list:
        """Queue a list of request records (Server.request) in one call;
        returns their tickets.  On a refused request it raises: the ones
        before it are queued (their tickets are in the error's `tickets`)."""
        n = len(requests)
        arr = (Request * n)(*requests)
        tickets = (ctypes.c_uint64 * n)()
        rc = lib().neat_submit_many(self._h, arr, n, tickets)
        if rc < 0:
            err = NeatError(rc, lib().neat_last_error().decode())
            err.tickets = [t for t in tickets if t]
            raise err
        return list(tickets)

    def submit(self, pop_id: int, outputs, inputs=None, B: int = 0, shared_inputs=False,
               grid_side: int = 0, grid_first: int = 0, tag: int = 0, I: int = 0) -> int:
        """Queue one request; returns its ticket.  TENSOR mode needs I (the
        population's input count) unless the inputs are shared."""
        r = Request()
        r.pop_id = pop_id
        if grid_side:
            r.input_mode = INPUT_GRID
            r.grid_side, r.grid_first = grid_side, grid_first
        else:
            r.input_mode = INPUT_TENSOR
            r.inputs = inputs.data_ptr()
            r.input_genome_stride = 0 if shared_inputs else B * I
        r.B = B
        r.outputs = outputs.data_ptr()
        r.tag = tag
        t = ctypes.c_uint64(0)
        check(lib().neat_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """None while pending, else the Result (the ticket is then forgotten)."""
        res = Result()
        rc = check(lib().neat_poll(self._h, ticket, ctypes.byref(res)))
        return None if rc == 1 else res

    def wait(self, ticket: int, timeout_s: float = 60.0):
        import time
        t_end = time.monotonic() + timeout_s
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() > t_end:
                raise TimeoutError("ticket %d not done after %.1fs" % (ticket, timeout_s))
            time.sleep(20e-6)

    def stats(self) -> Stats:
        st = Stats()
        check(lib().neat_server_stats(self._h, ctypes.byref(st)))
        return st

    def reset_stats(self):
        check(lib().neat_server_reset_stats(self._h))

    def close(self):
        if self._h.value:
            check(lib().neat_server_destroy(self._h))
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
