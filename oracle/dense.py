"""The paper's dense formulation of feedforward inference, in numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 3.3 transforms a genome into a node order N_order and an expanded
connection tensor C_exp of shape |N|max x |N|max x noa(c), written by a
scatter over the connection rows: the cell addressed by a row's (in, out)
receives the row's attributes when the row is enabled and NaN otherwise, and
every cell not written stays NaN.  The calculation keeps a NaN-initialised
value vector v, writes the inputs into it, and then visits the nodes in
N_order, each time combining the non-NaN column of C_exp that ends at the
node: f_c multiplies the source value by the weight, f_n aggregates, adds the
bias and applies the activation.

This module writes exactly that, with two deviations that are readings of the
paper rather than changes to it:

* (in, out) are node keys, so the scatter goes through a key -> row map;
* only enabled rows are scattered (a disabled row leaves its cell NaN, which
  is what the rule produces when no enabled row shares the cell).

Its topological order is computed independently of the C oracle: repeatedly
take every remaining node whose C_exp column has no remaining source, in row
order.  Any valid order gives the same values, so this is a cross-check of
the C oracle's forward, not of its order.  It handles valid genomes only.
"""
from __future__ import annotations

import numpy as np


def _act(code: int, z: np.ndarray) -> np.ndarray:
    if code == 0:
        return z
    if code == 1:
        return np.tanh(z)
    if code == 2:
        return 1.0 / (1.0 + np.exp(-z))
    if code == 3:
        return np.where(np.isnan(z), z, np.where(z > 0, z, 0.0))
    if code == 4:
        return np.sin(z)
    if code == 5:
        return np.exp(-(z * z))
    if code == 6:
        return np.abs(z)
    raise ValueError("activation code %r" % code)


def _agg(code: int, terms: np.ndarray) -> np.ndarray:
    """terms: [B, m]; aggregation over axis 1, 0 when m == 0."""
    if terms.shape[1] == 0:
        return np.zeros(terms.shape[0])
    if code == 0:
        return terms.sum(axis=1)
    if code == 1:
        return terms.prod(axis=1)
    if code == 2:
        return terms.max(axis=1)   # numpy max propagates NaN
    if code == 3:
        return terms.min(axis=1)
    if code == 4:
        return terms.mean(axis=1)
    raise ValueError("aggregation code %r" % code)


def expand(nodes: np.ndarray, conns: np.ndarray):
    """Transformation: (order rows, C_exp [N, N] of weights with NaN holes)."""
    N = nodes.shape[0]
    keys = nodes[:, 0].astype(np.float64)
    row_of = {}
    for r in range(N):
        if not np.isnan(keys[r]):
            row_of[float(keys[r])] = r
    c_exp = np.full((N, N), np.nan)
    for c in conns.astype(np.float64):
        if np.isnan(c[0]) or c[2] != 1.0:
            continue
        c_exp[row_of[float(c[0])], row_of[float(c[1])]] = c[3]
    edge = ~np.isnan(c_exp)
    remaining = ~np.isnan(keys)
    order = []
    while remaining.any():
        blocked = (edge & remaining[:, None]).any(axis=0)
        ready = remaining & ~blocked
        if not ready.any():
            raise ValueError("cycle")
        order.extend(np.nonzero(ready)[0].tolist())
        remaining &= ~ready
    return np.array(order, dtype=np.int64), c_exp


def forward(nodes: np.ndarray, conns: np.ndarray, x: np.ndarray, I: int, O: int):
    """nodes [N,5], conns [C,4], x [B, I] -> y [B, O] in float64."""
    nodes = np.asarray(nodes, dtype=np.float32)
    order, c_exp = expand(nodes, conns)
    keys = nodes[:, 0].astype(np.float64)
    x = np.asarray(x, dtype=np.float64)
    B = x.shape[0]
    N = nodes.shape[0]
    v = np.full((B, N), np.nan)
    row_of = {float(keys[r]): r for r in range(N) if not np.isnan(keys[r])}
    for i in range(I):
        v[:, row_of[float(i)]] = x[:, i]
    for k in order:
        if keys[k] < I:
            continue
        col = c_exp[:, k]
        src = np.nonzero(~np.isnan(col))[0]
        terms = v[:, src] * col[src][None, :]
        a = _agg(int(nodes[k, 4]), terms)
        z = float(nodes[k, 1]) + float(nodes[k, 2]) * a
        v[:, k] = _act(int(nodes[k, 3]), z)
    return np.stack([v[:, row_of[float(I + j)]] for j in range(O)], axis=1)
