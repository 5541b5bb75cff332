"""GPU: neat_forward_batch_noalloc (the batch without device allocation)
against neat_forward_batch on the same items, bit for bit, on two calls in a
row (the second with a smaller batch), plus the refusal of a batch whose
tables exceed the scratch area."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
from tests.parity import assert_parity
from workloads import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _neat():
    import paper_2404_01817_amd as neat
    return neat


def _same_bits(a, b):
    nan = np.isnan(a)
    return np.array_equal(nan, np.isnan(b)) and np.array_equal(a[~nan].view(np.uint32),
                                                                 b[~nan].view(np.uint32))


class _Buffers:
    """One population's device tensors for one entry point (its own program,
    status and outputs, so the two entry points share nothing they write)."""

    def __init__(self, pop, grid=None):
        neat = _neat()
        dev = torch.device("cuda:0")
        self.pop, self.grid = pop, grid
        self.nodes = torch.from_numpy(pop.nodes).to(dev)
        self.conns = torch.from_numpy(pop.conns).to(dev)
        self.d = neat.dims_of(self.nodes, self.conns, pop.I, pop.O)
        self.prog = torch.full((neat.program_bytes(self.d) // 4,), -7, dtype=torch.int32,
                               device=dev)
        self.status = torch.full((pop.P,), -7, dtype=torch.int32, device=dev)
        if grid is None:
            self.x = torch.from_numpy(pop.inputs).to(dev)
            self.B = pop.B
        else:
            self.x, self.B = None, grid[2]
        self.y = torch.full((pop.P, self.B, pop.O), 7.0, dtype=torch.float32, device=dev)

    def item(self):
        neat = _neat()
        kw = dict(nodes=self.nodes, conns=self.conns, status=self.status)
        if self.grid is None:
            return neat.batch_item(self.d, self.prog, self.y, inputs=self.x, B=self.B, **kw)
        side, first, Q = self.grid
        return neat.batch_item(self.d, self.prog, self.y, B=Q, grid_side=side, grid_first=first,
                               **kw)


def _workload(seed, n_pops, N_range, B_range, P_range, cppn_P):
    pops = synth.uneven(seed=seed, n_pops=n_pops, P_range=P_range, N_range=N_range,
                        B_range=B_range)
    grids = [None] * len(pops)
    if cppn_P:
        pops.append(synth.cppn(seed=seed + 100, P=cppn_P))
        grids.append((16, 333, 500))
    return pops, grids


def _run_both(pops, grids):
    neat = _neat()
    ref = [_Buffers(p, g) for p, g in zip(pops, grids)]
    new = [_Buffers(p, g) for p, g in zip(pops, grids)]
    plan = neat.BatchPlan()
    plan.run([b.item() for b in ref])
    neat.forward_batch_noalloc([b.item() for b in new])
    torch.cuda.synchronize()
    plan.free()
    return ref, new


def _check(ref, new, with_oracle):
    for k, (a, b) in enumerate(zip(ref, new)):
        ya, yb = a.y.cpu().numpy(), b.y.cpu().numpy()
        assert _same_bits(yb, ya), k
        assert torch.equal(a.status, b.status), k
        if with_oracle:
            p = b.pop
            if b.grid is None:
                y64, beta = oracle.forward(p.nodes, p.conns, p.inputs, p.I, p.O)
            else:
                q = synth.grid_queries(b.grid[1], b.grid[2])
                y64, beta = oracle.forward(p.nodes, p.conns, q, p.I, p.O, shared_inputs=True)
            assert_parity(yb, y64, beta, "noalloc item %d" % k)


def test_noalloc_batch_matches_the_recorded_batch_twice():
    """Two calls in a row: a batch of uneven populations (every slot class,
    tensor and grid items), then a smaller one; each equals
    neat_forward_batch on the same items bit for bit (outputs and status),
    and the first also the oracle within the parity rule."""
    print("noalloc: first call, 9 populations N_max 10..400 + CPPN grid", flush=True)
    pops, grids = _workload(41, 9, (10, 400), (1, 300), (3, 50), 10)
    ref, new = _run_both(pops, grids)
    _check(ref, new, with_oracle=True)
    print("noalloc: second call, 3 smaller populations", flush=True)
    pops, grids = _workload(42, 3, (10, 60), (1, 40), (2, 20), 0)
    ref, new = _run_both(pops, grids)
    _check(ref, new, with_oracle=True)


def test_noalloc_refuses_tables_beyond_the_scratch_area():
    """A batch whose work-unit tables exceed NEAT_NOALLOC_SCRATCH_BYTES is
    refused on the host with NEAT_E_TOO_LARGE before anything launches, and
    the entry point keeps working afterwards."""
    neat = _neat()
    from paper_2404_01817_amd import _lib
    pop = synth.uneven(seed=43, n_pops=1, P_range=(2, 2), N_range=(12, 12), B_range=(3, 3))[0]
    buf = _Buffers(pop)
    # a transformation item (88 B) and a work-unit item (120 B) each; N_max =
    # 12 needs no class list: 1300 x 208 B > 256 KiB
    items = [buf.item() for _ in range(1300)]
    arr = (_lib.BatchItem * len(items))(*items)
    rc = _lib.lib().neat_forward_batch_noalloc(arr, len(items), None)
    assert rc == -4, rc  # NEAT_E_TOO_LARGE
    assert b"scratch" in _lib.lib().neat_last_error()
    neat.forward_batch_noalloc([buf.item()])
    torch.cuda.synchronize()
    y64, beta = oracle.forward(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O)
    assert_parity(buf.y.cpu().numpy(), y64, beta, "after refusal")
