#!/usr/bin/env python3
"""Benchmark: population forward of tensorized NEAT on one MI355X.

One step = the whole hot path over the control-policy workload: the
transformation (validation, topological sort, program build) of P = 10000
genomes (N_max = 50, C_max = 200, I = 17, O = 6) followed by the calculation
of every genome on its own B = 1000 input vectors.  Inputs are resident in
HBM before the timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--P", type=int, default=10000)
    ap.add_argument("--B", type=int, default=1000)
    ap.add_argument("--cpu-genomes", type=int, default=8000,
                    help="genomes of the workload the CPU oracle is timed on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, copy 256 MiB once (a plain copy kernel "
                         "of known size, which calibrates HBM byte counters)")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def program_bytes_read(O, n_valid, n_edges, I):
    """Algorithmic program bytes a forward reads once per genome: a 64-byte
    header, 4 bytes per output slot, 16 bytes per computed node (bias,
    response, activation and aggregation, edge count) and 8 bytes per enabled
    connection (source, weight).  The stored records are larger (64 bytes,
    with the first edges inline); this counts what the method needs."""
    n_comp = np.maximum(n_valid - I, 0)
    return int((64 + 4 * O + 16 * n_comp + 8 * n_edges).sum())


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the population forward has no "
              "cross-GPU exchange; shard genomes across GPUs by running one "
              "process per GPU.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2404_01817_amd as neat
    from paper_2404_01817_amd import synth

    dev = torch.device("cuda:0")
    t0 = time.time()
    pop = synth.control(P=args.P, B=args.B)
    log(args, "generated P=%d B=%d in %.1fs" % (pop.P, pop.B, time.time() - t0))
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    tx = torch.from_numpy(pop.inputs).to(dev)
    d = neat.dims_of(tn, tc, pop.I, pop.O)
    prog = torch.empty((neat.program_bytes(d) // 4,), dtype=torch.int32, device=dev)
    status = torch.empty((pop.P,), dtype=torch.int32, device=dev)
    out = torch.empty((pop.P, pop.B, pop.O), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    lib = neat.lib()

    def topo():
        neat._lib.check(lib.neat_topo_sort(ctypes.byref(d), ctypes.c_void_p(tn.data_ptr()),
                                           ctypes.c_void_p(tc.data_ptr()), None, None,
                                           ctypes.c_void_p(status.data_ptr()),
                                           ctypes.c_void_p(prog.data_ptr()), sp))

    def fwd():
        neat._lib.check(lib.neat_forward(ctypes.byref(d), ctypes.c_void_p(prog.data_ptr()),
                                         ctypes.c_void_p(tx.data_ptr()), pop.B * pop.I, pop.B,
                                         ctypes.c_void_p(out.data_ptr()), sp))

    for _ in range(args.warmup):
        topo()
        fwd()
    torch.cuda.synchronize()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        topo()
        ev[k][1].record(stream)
        fwd()
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    topo_ms = np.array([e[0].elapsed_time(e[1]) for e in ev])
    fwd_ms = np.array([e[1].elapsed_time(e[2]) for e in ev])
    step_ms = wall * 1e3 / args.steps
    units = pop.P * pop.B
    value = units / (step_ms / 1e3)

    # algorithmic bytes of the forward launch
    hdr = neat.program_headers(d, prog).cpu().numpy()
    st = status.cpu().numpy()
    n_bad = int((st != 0).sum())
    pbytes = program_bytes_read(pop.O, hdr[:, 0], hdr[:, 7], pop.I)  # valid nodes, edges
    fwd_bytes = pop.P * pop.B * (pop.I + pop.O) * 4 + pbytes
    fwd_avg_s = float(fwd_ms.mean()) / 1e3
    achieved = fwd_bytes / fwd_avg_s / 1e9
    roofline = {"kernel": "forward (lane per sample)", "bound": "hbm",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "algorithmic_bytes_per_launch": fwd_bytes,
                "bytes_per_genome_input": round(fwd_bytes / units, 2),
                "avg_launch_us": round(fwd_avg_s * 1e6, 1)}

    # each forward variant on the same program, for the record
    variants = {}
    for name, var in (("reg", neat.FWD_REG), ("reg2", neat.FWD_REG2), ("lds", neat.FWD_LDS)):
        try:
            t0e, t1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            neat.forward(d, prog, tx, pop.B, outputs=out, variant=var)
            t0e.record(stream)
            for _ in range(5):
                neat.forward(d, prog, tx, pop.B, outputs=out, variant=var)
            t1e.record(stream)
            torch.cuda.synchronize()
            variants[name] = round(t0e.elapsed_time(t1e) / 5, 4)
        except neat.NeatError:
            variants[name] = None

    if args.copy_probe:
        src = torch.ones((64 << 20,), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(args, "copy probe: 256 MiB read, 256 MiB written")
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        g = min(args.cpu_genomes, pop.P)
        t = time.perf_counter()
        oracle.forward(pop.nodes[:g], pop.conns[:g], pop.inputs[:g], pop.I, pop.O,
                       with_beta=False)
        dt = time.perf_counter() - t
        cpu = {"value": round(g * pop.B / dt, 1), "unit": "genome-inputs/s", "cores": 1,
               "kind": "oracle",
               "sample": "first %d genomes x %d inputs of the same workload, fp64, "
                         "transformation + calculation, single thread (%.1f s)"
                         % (g, pop.B, dt)}

    res = {
        "metric": "genome-input forwards/s", "value": round(value, 1),
        "unit": "genome-inputs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(step_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "control-policy population: P=%d genomes, N_max=50, "
                               "C_max=200, I=17, O=6, B=%d per-genome inputs, plain "
                               "per-population launch (sort + forward)" % (pop.P, pop.B),
                   "P": pop.P, "B": pop.B, "N_max": 50, "C_max": 200, "I": 17, "O": 6},
        "topo_ms": round(float(np.median(topo_ms)), 4),
        "forward_ms": round(float(np.median(fwd_ms)), 4),
        "forward_variant_ms": variants,
        "rejected_genomes": n_bad,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
