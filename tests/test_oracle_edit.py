"""Pins for the oracle's tensorized genome edits (Section 3.2): each edit's
row-level effect against its definition on hand-made genomes, sequential
additions filling the NaN rows in order, a full tensor refusing an
addition, add-then-remove restoring the tensors, independence of genomes,
and the transformation seeing an added node and connection."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import EDIT_DTYPE, NODE_ADD, NODE_DEL, CONN_ADD, CONN_DEL, NODE_SET, CONN_SET
from workloads import synth
from tests.helpers import genome, stack


def _edits(rows):
    e = np.zeros(len(rows), EDIT_DTYPE)
    for i, (g, op, row, col, v) in enumerate(rows):
        e[i] = (g, op, row, col, tuple(v) + (0.0,) * (5 - len(v)))
    return e


def _same(a, b):
    return np.array_equal(np.nan_to_num(a, nan=7.5e30), np.nan_to_num(b, nan=7.5e30))


def _base():
    return genome(5, 4, {0: (0, 0, 1, 0, 0), 1: (1, 0, 1, 0, 0), 3: (2, 0.5, 1, 2, 0)},
                  {1: (0, 2, 1, 0.5), 2: (1, 2, 1, -1.0)})


def test_each_edit_on_a_hand_made_genome():
    n, c = _base()
    n2, c2, ok = oracle.edit(n, c, _edits([
        (0, NODE_ADD, 0, 0, (9, 0.25, 1, 1, 0)),    # first NaN node row is row 2
        (0, NODE_ADD, 0, 0, (11, 0.0, 1, 3, 2)),    # then row 4
        (0, CONN_ADD, 0, 0, (9, 2, 1, 2.0)),        # first NaN connection row is row 0
        (0, CONN_DEL, 2, 0, ()),
        (0, NODE_SET, 3, 1, (-0.75,)),              # bias of node 2
        (0, CONN_SET, 1, 3, (4.0,)),                # weight of 0 -> 2
        (0, CONN_SET, 1, 2, (0.0,)),                # and disable it
        (0, NODE_DEL, 1, 0, ()),
    ]))
    assert ok.tolist() == [1] * 8
    assert n2[0, 2].tolist() == [9, 0.25, 1, 1, 0] and n2[0, 4].tolist() == [11, 0, 1, 3, 2]
    assert n2[0, 3].tolist() == [2, -0.75, 1, 2, 0] and np.all(np.isnan(n2[0, 1]))
    assert c2[0, 0].tolist() == [9, 2, 1, 2.0] and c2[0, 1].tolist() == [0, 2, 0, 4.0]
    assert np.all(np.isnan(c2[0, 2])) and np.all(np.isnan(c2[0, 3]))
    assert n2[0, 0].tolist() == n[0, 0].tolist()


def test_full_tensor_and_bad_edits_do_not_apply():
    n, c = _base()
    e = _edits([(0, NODE_ADD, 0, 0, (7, 0, 1, 0, 0))] * 3         # 2 NaN rows: the 3rd fails
               + [(0, NODE_SET, 0, 0, (5.0,)), (0, CONN_SET, 0, 1, (5.0,)),  # key columns
                  (0, NODE_DEL, 5, 0, ()), (1, NODE_DEL, 0, 0, ()), (0, 9, 0, 0, ())])
    n2, c2, ok = oracle.edit(n, c, e)
    assert ok.tolist() == [1, 1, 0, 0, 0, 0, 0, 0]
    assert np.all(~np.isnan(n2[0, :, 0]))
    assert _same(c2, c)


def test_add_then_remove_restores():
    pop = synth.control(seed=3, P=20, B=1)
    rows = []
    for g in range(pop.P):
        r = int(np.flatnonzero(np.isnan(pop.nodes[g, :, 0]))[0])
        rc = int(np.flatnonzero(np.isnan(pop.conns[g, :, 0]))[0])
        rows += [(g, NODE_ADD, 0, 0, (700 + g, 0.1, 1, 1, 0)), (g, NODE_DEL, r, 0, ()),
                 (g, CONN_ADD, 0, 0, (0, 17, 1, 0.3)), (g, CONN_DEL, rc, 0, ())]
    n2, c2, ok = oracle.edit(pop.nodes, pop.conns, _edits(rows))
    assert np.all(ok == 1)
    assert _same(n2, pop.nodes) and _same(c2, pop.conns)


def test_genomes_are_independent():
    pop = synth.control(seed=4, P=12, B=1)
    rng = np.random.default_rng(0)
    rows = [(int(rng.integers(0, 12)), int(rng.integers(0, 6)), int(rng.integers(0, 50)),
             int(rng.integers(1, 4)), tuple(rng.normal(size=5))) for _ in range(200)]
    e = _edits(rows)
    n_all, c_all, ok_all = oracle.edit(pop.nodes, pop.conns, e)
    for g in range(12):
        sel = e["genome"] == g
        n1e = e[sel].copy()
        n1e["genome"] = 0
        n1, c1, ok1 = oracle.edit(pop.nodes[g:g + 1], pop.conns[g:g + 1], n1e)
        assert _same(n1[0], n_all[g]) and _same(c1[0], c_all[g])
        assert np.array_equal(ok1, ok_all[sel])


def test_transformation_sees_the_edits():
    """Split connection 0 -> 2 with a new node 9 (NEAT's add-node mutation as
    edits): disable it, add node 9, add 0 -> 9 and 9 -> 2; the new node
    sits on level 1 and node 2 moves to level 2."""
    n, c = _base()
    n2, c2, ok = oracle.edit(n, c, _edits([
        (0, CONN_SET, 1, 2, (0.0,)), (0, NODE_ADD, 0, 0, (9, 0, 1, 0, 0)),
        (0, CONN_ADD, 0, 0, (0, 9, 1, 1.0)), (0, CONN_ADD, 0, 0, (9, 2, 1, 0.5))]))
    assert np.all(ok == 1)
    order, level, status = oracle.transform(n2, c2, 2, 1)
    assert status[0] == 0
    keys = {int(n2[0, r, 0]): int(level[0, r]) for r in range(5) if not np.isnan(n2[0, r, 0])}
    assert keys == {0: 0, 1: 0, 9: 1, 2: 2}
