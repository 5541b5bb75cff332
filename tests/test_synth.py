"""Conformance of the seeded workload generators (shapes, NaN placement, DAGs,
enabled fraction, reproducibility).  Uses the oracle only to check that every
generated genome is accepted."""
import numpy as np

import oracle
from workloads import synth


def test_tiny_shape_and_values():
    p = synth.tiny()
    assert p.nodes.shape == (16, 8, 5) and p.conns.shape == (16, 16, 4)
    assert p.inputs.shape == (32, 3) and p.shared_inputs
    assert p.inputs.min() >= -1 and p.inputs.max() <= 1
    valid = ~np.isnan(p.nodes[:, :, 0])
    assert set(np.unique(p.nodes[:, :, 3][valid])) == {synth.ACT_SIGMOID}
    assert set(np.unique(p.nodes[:, :, 4][valid])) == {synth.AGG_SUM}
    _, _, status = oracle.transform(p.nodes, p.conns, p.I, p.O)
    assert (status == 0).all()


def test_control_conformance():
    p = synth.control(P=400, B=3)
    assert p.nodes.shape == (400, 50, 5) and p.conns.shape == (400, 200, 4)
    assert p.inputs.shape == (400, 3, 17)
    k = p.nodes[:, :, 0]
    # I/O keys at rows 0..22, hidden keys elsewhere and never equal to their row
    assert np.array_equal(k[:, :23], np.broadcast_to(np.arange(23), (400, 23)))
    hid = ~np.isnan(k[:, 23:])
    rows = np.broadcast_to(np.arange(23, 50), (400, 27))
    assert (k[:, 23:][hid] >= 23).all() and (k[:, 23:][hid] < 800).all()
    assert (k[:, 23:][hid] != rows[hid]).mean() > 0.9
    # NaN gaps inside the node and connection tensors, not only at the tail
    gaps = [np.isnan(k[p_, 23:]).any() and (~np.isnan(k[p_, 23:])).any() and
            not np.isnan(k[p_, -1]) for p_ in range(400)]
    assert any(gaps)
    en = p.conns[:, :, 2][~np.isnan(p.conns[:, :, 0])]
    assert set(np.unique(en)) <= {0.0, 1.0} and abs(en.mean() - 0.7) < 0.02
    _, level, status = oracle.transform(p.nodes, p.conns, p.I, p.O)
    assert (status == 0).all()
    acts = np.unique(p.nodes[:, :, 3][~np.isnan(k)])
    assert set(acts) == set(synth.CONTROL_ACTS)
    # response is 1 everywhere
    assert (p.nodes[:, :, 2][~np.isnan(k)] == 1).all()


def test_reproducible():
    a, b = synth.control(P=20, B=2), synth.control(P=20, B=2)
    assert np.array_equal(a.nodes, b.nodes, equal_nan=True)
    assert np.array_equal(a.conns, b.conns, equal_nan=True)
    assert np.array_equal(a.inputs, b.inputs)
    c = synth.control(seed=7, P=20, B=2)
    assert not np.array_equal(a.conns, c.conns, equal_nan=True)


def test_uneven_populations_are_valid():
    pops = synth.uneven(n_pops=4, P_range=(5, 20), N_range=(10, 400), B_range=(1, 8))
    for p in pops:
        assert p.C_max == 4 * p.N_max and 2 <= p.I <= 24 and 1 <= p.O <= 8
        _, _, status = oracle.transform(p.nodes, p.conns, p.I, p.O)
        assert (status == 0).all()


def test_grid_queries():
    c = synth.grid_coords()
    assert c[0] == -1 and c[-1] == 1 and c.dtype == np.float32
    # the coordinates are the fp32 roundings of (2i - 15) / 15
    for i in range(16):
        assert c[i] == np.float32(np.float64(2 * i - 15) / 15.0)
    q = synth.grid_queries()
    assert q.shape == (65536, 5) and (q[:, 4] == 1).all()
    assert np.array_equal(q[257], [c[1], c[0], c[1], c[0], 1.0])
    assert len(np.unique(q[:, :4], axis=0)) == 65536
    assert np.array_equal(synth.grid_queries(1000, 7), q[1000:1007])
