"""GPU parity of the recurrent path (neat_topo_sort_recurrent +
neat_forward_recurrent, through the C ABI) against the CPU oracle.

Status, order and level must match bit for bit; fp32 outputs must satisfy
the parity rule of ``oracle.within_tolerance`` (|y - y64| <= 1e-5 + 2 beta,
NaN where the oracle is NaN)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from tests.parity import assert_parity
from workloads import synth
from tests.helpers import genome, stack

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _neat():
    import paper_2404_01817_amd as neat
    return neat


def _gpu_rec(nodes, conns, I, O, x, K, shared=False):
    neat = _neat()
    dev = torch.device("cuda:0")
    tn = torch.from_numpy(np.ascontiguousarray(nodes)).to(dev)
    tc = torch.from_numpy(np.ascontiguousarray(conns)).to(dev)
    order, level, status, prog = neat.topo_sort(tn, tc, I, O, recurrent=True)
    d = neat.dims_of(tn, tc, I, O)
    tx = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    B = x.shape[0] if shared else x.shape[1]
    y = neat.forward_recurrent(d, prog, tx, B, K, shared_inputs=shared)
    torch.cuda.synchronize()
    return (order.cpu().numpy(), level.cpu().numpy(), status.cpu().numpy().astype(np.uint32),
            y.cpu().numpy())


def _rec_pop(seed, P, N, C, I, O, B, hidden=None):
    rng = np.random.default_rng(seed)
    pop = synth.make_population(rng, P, N, C, I, O, N - I - O if hidden is None else hidden,
                                synth._k_uniform(C), synth.CONTROL_ACTS, synth.ALL_AGGS,
                                recurrent=True)
    pop.inputs = rng.standard_normal((P, B, I), dtype=np.float32)
    return pop


def _check(pop, K, label):
    print("case", label, "K", K, flush=True)
    order, level, status, y = _gpu_rec(pop.nodes, pop.conns, pop.I, pop.O, pop.inputs, K)
    o_order, o_level, o_status = oracle.transform(pop.nodes, pop.conns, pop.I, pop.O,
                                                  recurrent=True)
    assert np.array_equal(status, o_status), label
    assert np.array_equal(order, o_order), label
    assert np.array_equal(level, o_level), label
    y64, beta = oracle.forward_recurrent(pop.nodes, pop.conns, pop.inputs, pop.I, pop.O, K)
    stats = assert_parity(y, y64, beta, label)


# (P, N_max, C_max, I, O, B): one-wave transformation groups, multi-wave
# groups, 128- and 224-slot rows and the N_max + 2 row layout (N_max = 500
# in tiles of 32 samples); B spanning several tiles with a ragged last one
SHAPES = [(37, 12, 30, 3, 2, 70), (24, 50, 200, 17, 6, 130), (11, 100, 400, 8, 3, 65),
          (7, 180, 720, 12, 4, 64), (5, 260, 1040, 10, 5, 33), (3, 500, 1500, 6, 3, 40)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "P%d_N%d_B%d" % (s[0], s[1], s[5]))
@pytest.mark.parametrize("K", [0, 1, 3, 8])
def test_recurrent_parity(shape, K):
    P, N, C, I, O, B = shape
    pop = _rec_pop(1000 + N + K, P, N, C, I, O, B)
    _check(pop, K, "P%d N%d B%d" % (P, N, B))


def test_recurrent_shared_inputs():
    pop = _rec_pop(7, 20, 40, 160, 5, 3, 1)
    x = np.random.default_rng(8).standard_normal((150, 5)).astype(np.float32)
    _, _, status, y = _gpu_rec(pop.nodes, pop.conns, 5, 3, x, 5, shared=True)
    y64, beta = oracle.forward_recurrent(pop.nodes, pop.conns, x, 5, 3, 5, shared_inputs=True)
    stats = assert_parity(y, y64, beta, "")


def test_recurrent_status_cases_bit_exact():
    """Cycles and self-loops accepted; every other fault flagged with NaN
    outputs (the cases of the oracle's recurrent status pins)."""
    base = {0: (0, 0, 1, 0, 0), 1: (1, 0, 1, 0, 0), 2: (2, 0, 1, 0, 0), 3: (9, 0, 1, 0, 0)}
    loop = {0: (0, 9, 1, 1.0), 1: (9, 2, 1, 1.0), 2: (2, 9, 1, 1.0), 3: (9, 9, 1, 0.5)}
    cases = [(base, loop), (base, {**loop, 4: (5, 9, 1, 1.0)}),
             (base, {**loop, 4: (9, 1, 1, 1.0)}), (base, {**loop, 4: (9, 9, 1, 2.0)}),
             (base, {**loop, 4: (9, 2, 0.5, 1.0)}), ({**base, 4: (9, 0, 1, 0, 0)}, loop),
             ({k: v for k, v in base.items() if k != 2}, {0: (0, 9, 1, 1.0)})]
    n, c = stack([genome(6, 8, a, b) for a, b in cases])
    x = np.random.default_rng(3).standard_normal((len(cases), 9, 2)).astype(np.float32)
    order, level, status, y = _gpu_rec(n, c, 2, 1, x, 4)
    o_order, o_level, o_status = oracle.transform(n, c, 2, 1, recurrent=True)
    assert status.tolist() == o_status.tolist() == [0, 8, 16, 32, 1, 2, 4]
    assert np.array_equal(order, o_order) and np.array_equal(level, o_level)
    y64, beta = oracle.forward_recurrent(n, c, x, 2, 1, 4)
    stats = assert_parity(y, y64, beta, "")
    assert np.all(np.isnan(y[1:]))


def test_dag_matches_feedforward_lds_store_bits():
    """An acyclic population after max-level + 1 sweeps gives exactly the
    bits of the feedforward calculation with the LDS value store (both run
    the same per-node operations in the same order)."""
    neat = _neat()
    pop = synth.control(seed=31, P=300, B=100)
    _, level, status = oracle.transform(pop.nodes, pop.conns, pop.I, pop.O)
    K = int(level.max()) + 1
    dev = torch.device("cuda:0")
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    tx = torch.from_numpy(pop.inputs).to(dev)
    d = neat.dims_of(tn, tc, pop.I, pop.O)
    _, _, _, prog = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False)
    y_ff = neat.forward(d, prog, tx, pop.B, variant=neat.FWD_LDS)
    _, _, _, prog_r = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False, recurrent=True)
    y_rec = neat.forward_recurrent(d, prog_r, tx, pop.B, K)
    torch.cuda.synchronize()
    a, b = y_ff.cpu().numpy(), y_rec.cpu().numpy()
    ok = status == 0
    assert np.array_equal(a[ok].view(np.uint32), b[ok].view(np.uint32))


def test_recurrent_empty_and_too_large():
    neat = _neat()
    dev = torch.device("cuda:0")
    pop = _rec_pop(5, 3, 20, 40, 4, 2, 1)
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    d = neat.dims_of(tn, tc, 4, 2)
    _, _, _, prog = neat.topo_sort(tn, tc, 4, 2, recurrent=True)
    x = torch.zeros((3, 0, 4), device=dev)
    y = neat.forward_recurrent(d, prog, x, 0, 3)          # B = 0: nothing to do
    assert y.shape == (3, 0, 2)
    with pytest.raises(neat.NeatError):
        neat.forward_recurrent(d, prog, torch.zeros((3, 5, 4), device=dev), 5, -1)
    with pytest.raises(neat.NeatError):    # beyond NEAT_MAX_SWEEPS
        neat.forward_recurrent(d, prog, torch.zeros((3, 5, 4), device=dev), 5, 65537)
    # N_max = 700 needs 2 x 702 LDS rows per lane: beyond 160 KiB even with
    # tiles of 32 samples
    big = neat.Dims(1, 700, 16, 4, 2)
    prog_b = torch.zeros((neat.program_bytes(big) // 4,), dtype=torch.int32, device=dev)
    with pytest.raises(neat.NeatError) as e:
        neat.forward_recurrent(big, prog_b, torch.zeros((1, 8, 4), device=dev), 8, 2)
    assert e.value.code == -4  # NEAT_E_TOO_LARGE
    torch.cuda.synchronize()


def test_recurrent_full_size_sampled():
    """The benchmark's recurrent workload (P=10000, N_max=50, C_max=200,
    B=1000, K=4) in its launch configuration; the oracle checks every output
    of a sample of genomes."""
    neat = _neat()
    pop = synth.recurrent_control()
    K = 4
    dev = torch.device("cuda:0")
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    tx = torch.from_numpy(pop.inputs).to(dev)
    d = neat.dims_of(tn, tc, pop.I, pop.O)
    _, _, st, prog = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False, recurrent=True)
    y = neat.forward_recurrent(d, prog, tx, pop.B, K)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    status = st.cpu().numpy().astype(np.uint32)
    _, _, o_status = oracle.transform(pop.nodes, pop.conns, pop.I, pop.O, recurrent=True)
    assert np.array_equal(status, o_status)
    sample = np.random.default_rng(0).choice(pop.P, 40, replace=False)
    sample = np.concatenate([sample, [0, pop.P - 1]])
    y64, beta = oracle.forward_recurrent(pop.nodes[sample], pop.conns[sample],
                                         pop.inputs[sample], pop.I, pop.O, K)
    stats = assert_parity(y[sample], y64, beta, "")
