"""Small genome builders and the golden-fixture reader shared by the tests.

Nothing here computes the method: it only lays out node and connection rows
(Section 3.1 encoding) and parses text fixtures."""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def genome(N_max, C_max, nodes, conns):
    """nodes: {row: (key, bias, response, act, agg)}, conns: {row: (in, out,
    enabled, weight)} -> ([1,N_max,5], [1,C_max,4]) NaN-padded float32."""
    n = np.full((1, N_max, 5), np.nan, np.float32)
    c = np.full((1, C_max, 4), np.nan, np.float32)
    for r, v in nodes.items():
        n[0, r] = v
    for r, v in conns.items():
        c[0, r] = v
    return n, c


def stack(genomes):
    """[(nodes[1,N,5], conns[1,C,4]), ...] -> population with common N, C."""
    N = max(g[0].shape[1] for g in genomes)
    C = max(g[1].shape[1] for g in genomes)
    n = np.full((len(genomes), N, 5), np.nan, np.float32)
    c = np.full((len(genomes), C, 4), np.nan, np.float32)
    for i, (gn, gc) in enumerate(genomes):
        n[i, :gn.shape[1]] = gn[0]
        c[i, :gc.shape[1]] = gc[0]
    return n, c


def read_golden(name):
    """Parse a golden network fixture (see tests/golden/*.txt)."""
    out = {"nodes": {}, "conns": {}, "order": None, "level": {}, "cases": []}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            head, vals = tok[0], tok[1:]
            if head in ("I", "O", "N_max", "C_max"):
                out[head] = int(vals[0])
            elif head == "node":
                out["nodes"][int(vals[0])] = tuple(float(v) for v in vals[1:])
            elif head == "conn":
                out["conns"][int(vals[0])] = tuple(float(v) for v in vals[1:])
            elif head == "order":
                out["order"] = [int(v) for v in vals]
            elif head == "level":
                out["level"][int(vals[0])] = int(vals[1])
            elif head == "case":
                out["cases"].append([float(v) for v in vals])
    n, c = genome(out["N_max"], out["C_max"], out["nodes"], out["conns"])
    out["nodes_arr"], out["conns_arr"] = n, c
    cases = np.array(out["cases"], np.float64)
    out["x"] = cases[:, :out["I"]].astype(np.float32)
    out["y"] = cases[:, out["I"]:]
    return out
