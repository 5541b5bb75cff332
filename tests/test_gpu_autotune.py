"""GPU tests of the forward autotuner (neat_autotune_forward, through the C
ABI): the tuned variant is one of the five measured ones; tuning leaves
the outputs bit-identical to the automatic rule, and later calls with
FWD_TUNED and batches over tuned buckets give the same bits as untuned
calls, unless the segment mapping was recorded, whose sums and products
round in another order: then they match the oracle within the parity
rule."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from workloads import synth
from tests.parity import assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _clean_tune_table():
    """Every test here tunes: leave the process-wide table empty for the
    tests after it, which compare untuned bits."""
    yield
    import paper_2404_01817_amd as neat
    neat.tune_clear()

torch = pytest.importorskip("torch")


def _neat():
    import paper_2404_01817_amd as neat
    return neat


def _bits(t):
    return t.cpu().numpy().view(np.uint32)


class _Pop:
    def __init__(self, seed, P, B):
        neat = _neat()
        dev = torch.device("cuda:0")
        pop = synth.control(seed=seed, P=P, B=B)
        self.pop = pop
        self.B = B
        self.nodes = torch.from_numpy(pop.nodes).to(dev)
        self.conns = torch.from_numpy(pop.conns).to(dev)
        self.x = torch.from_numpy(pop.inputs).to(dev)
        self.d = neat.dims_of(self.nodes, self.conns, pop.I, pop.O)
        _, _, _, self.prog = neat.topo_sort(self.nodes, self.conns, pop.I, pop.O,
                                            want_order=False)
        self.y = torch.empty((P, B, pop.O), device=dev)

    def auto(self):
        return _neat().forward(self.d, self.prog, self.x, self.B)


@pytest.mark.parametrize("P,B", [(300, 130), (64, 17)])
def test_autotune_records_a_measured_variant(P, B):
    neat = _neat()
    p = _Pop(seed=P + B, P=P, B=B)
    ref = p.auto()
    v, ms = neat.autotune_forward(p.d, p.prog, p.x, B, outputs=p.y, reps=3)
    torch.cuda.synchronize()
    print("tuned", P, B, v, ms, flush=True)
    cands = [neat.FWD_REG, neat.FWD_REG2, neat.FWD_LDS, neat.FWD_LVL, neat.FWD_SEG]
    nc = len(cands)
    assert v in cands and len(ms) == 2 * nc
    assert all(m > 0 for m in ms)
    assert ms[cands.index(v)] == min(ms[:nc])
    vt = neat.tuned_variant(p.d, B, throughput=True)
    assert ms[nc + cands.index(vt)] == min(ms[nc:])
    assert neat.tuned_variant(p.d, B) == v
    y2 = neat.forward(p.d, p.prog, p.x, B, variant=neat.FWD_TUNED)
    torch.cuda.synchronize()
    for y in (p.y, y2):
        if v == neat.FWD_SEG:
            y64, beta = oracle.forward(p.pop.nodes, p.pop.conns, p.pop.inputs, p.pop.I, p.pop.O)
            assert_parity(y.cpu().numpy(), y64, beta, "tuned (segment mapping)")
        else:
            assert np.array_equal(_bits(y), _bits(ref))


def test_batch_over_tuned_buckets_matches_single_calls():
    neat = _neat()
    pops = [_Pop(seed=s, P=P, B=B) for s, P, B in ((1, 200, 100), (2, 150, 40), (3, 90, 300))]
    refs = [p.auto() for p in pops]
    neat.autotune_forward(pops[0].d, pops[0].prog, pops[0].x, pops[0].B, reps=2)
    neat.autotune_forward(pops[2].d, pops[2].prog, pops[2].x, pops[2].B, reps=2)
    plan = neat.BatchPlan()
    items = [neat.batch_item(p.d, p.prog, p.y, inputs=p.x, B=p.B) for p in pops]
    for _ in range(2):  # record, then replay
        for p in pops:
            p.y.fill_(float("nan"))
        plan.run(items)
        torch.cuda.synchronize()
        for p, r in zip(pops, refs):
            if neat.tuned_variant(p.d, p.B, throughput=True) == neat.FWD_SEG:
                y64, beta = oracle.forward(p.pop.nodes, p.pop.conns, p.pop.inputs, p.pop.I,
                                           p.pop.O)
                assert_parity(p.y.cpu().numpy(), y64, beta, "batch item (segment mapping)")
            else:
                assert np.array_equal(_bits(p.y), _bits(r))
    plan.free()


def test_autotune_arguments():
    neat = _neat()
    p = _Pop(seed=5, P=20, B=8)
    with pytest.raises(neat.NeatError):
        neat.autotune_forward(p.d, p.prog, p.x, 8, reps=0)
    with pytest.raises(neat.NeatError):
        neat.forward(p.d, p.prog, p.x, 8, variant=7)
    v, ms = neat.autotune_forward(p.d, p.prog, p.x, 0, reps=2)
    assert v == neat.FWD_AUTO and ms == [-1.0] * (2 * neat.TUNE_CANDIDATES)
    torch.cuda.synchronize()


def test_tune_cache_file_read_and_rewritten(tmp_path):
    """A server created with tune_cache_path loads the autotuner's table
    from that file (bucket values: N_max and C_max rounded up to powers of
    two, B to a power of two), and a later tuning rewrites the file with
    both winners of the tuned bucket."""
    neat = _neat()
    path = tmp_path / "tune.txt"
    # bucket (64, 256, 8) -> level mapping alone, segment mapping on a full GPU
    path.write_text("64 256 8 0 %d %d\n" % (neat.FWD_LVL, neat.FWD_SEG))
    server = neat.Server(max_inflight=1, tune_cache_path=str(path))
    d = neat.Dims(5, 50, 200, 17, 6)  # N_max 50 -> 64, C_max 200 -> 256
    assert neat.tuned_variant(d, 7) == neat.FWD_LVL        # B 7 -> 8
    assert neat.tuned_variant(d, 8, throughput=True) == neat.FWD_SEG
    assert neat.tuned_variant(d, 9) == neat.FWD_AUTO       # bucket 16: never tuned
    assert neat.tuned_variant(d, 7, grid=True) == neat.FWD_AUTO
    server.close()
    p = _Pop(seed=9, P=40, B=12)
    v, ms = neat.autotune_forward(p.d, p.prog, p.x, 12, reps=2)
    vt = neat.tuned_variant(p.d, 12, throughput=True)
    lines = {tuple(int(x) for x in l.split()) for l in path.read_text().splitlines() if l}
    assert (64, 256, 8, 0, neat.FWD_LVL, neat.FWD_SEG) in lines
    assert (64, 256, 16, 0, v, vt) in lines
