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
# fp32 vector peak without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# (fused multiply-add) x 2.4 GHz (packed fp32 would double it; the kernels are
# compiled without packed fp32 instructions)
VALU_PEAK_TFLOPS = 78.6
# algorithmic flops of an activation (identity, tanh, sigmoid, relu, sin,
# gaussian, abs): the arithmetic of its definition on the hardware's base-2
# exponential and reciprocal, sin as range reduction + two short polynomials
ACT_FLOPS = (0, 5, 4, 1, 15, 3, 1)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "forward_control_traffic.json")


def measured_profile():
    """From the committed counter profile of the control forward: HBM bytes
    per launch (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a
    plain copy of known size) and the kernel's average launch time in the
    rocprofv3 trace; (None, None) when the kernel sources have changed since
    they were taken."""
    import hashlib
    try:
        prof = json.load(open(TRAFFIC_PROFILE))
        h = hashlib.sha256()
        for f in prof["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest()[:16] != prof["source_hash"]:
            return None, None
        return int(prof["traffic_bytes_per_launch"]), prof.get("rocprof_avg_launch_us")
    except (OSError, KeyError, ValueError):
        return None, None


def ramp(args, torch, fn):
    """Run fn untimed until args.ramp_ms of wall time has passed, so that the
    GPU's clocks have left their idle state before the warmup and the timed
    steps: a GPU that was idle runs its first tens of milliseconds of work
    slower (the control step measured 0.234 ms over 20 steps after 3 warmup
    steps, 0.202 ms once warm)."""
    if args.ramp_ms <= 0:
        return
    torch.cuda.synchronize()
    t = time.perf_counter()
    while (time.perf_counter() - t) * 1e3 < args.ramp_ms:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ramp-ms", type=float, default=50.0,
                    help="untimed run of each workload's step before its warmup steps, "
                         "until this much wall time has passed (GPU clock ramp); 0: none")
    ap.add_argument("--P", type=int, default=10000)
    ap.add_argument("--B", type=int, default=1000)
    ap.add_argument("--cpu-genomes", type=int, default=10000,
                    help="genomes of the workload the CPU oracle is timed on")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="the oracle repeats its sample until this much CPU time has passed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-p-sweep", action="store_true",
                    help="skip the control step over P = 50 .. 10000 genomes")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--workloads", default="control,tiny,batched,served,cppn,recurrent,substrate,distance,"
                            "crossover,edit",
                    help="comma list: control (the headline line), batched (64 uneven "
                         "populations in one recorded batch), served (Poisson request "
                         "stream over 128 resident populations), cppn (grid queries), "
                         "recurrent (K sweeps of networks with cycles), substrate "
                         "(HyperNEAT substrate layer on the matrix cores), distance "
                         "(compatibility distance to species representatives), "
                         "crossover (children of genome pairs), edit (tensorized "
                         "mutation edits)")
    ap.add_argument("--served-burst", type=int, default=512,
                    help="requests of the saturation comparison (served burst against "
                         "plain per-request launches); 0 skips it")
    ap.add_argument("--served-seconds", type=float, default=60.0,
                    help="length of the served request stream (latency counted after "
                         "the first quarter)")
    ap.add_argument("--served-rate", type=float, default=200.0, help="requests per second")
    ap.add_argument("--served-sweep", default="1000,4000,16000,64000,256000",
                    help="further request rates (per second), each run for --sweep-seconds")
    ap.add_argument("--sweep-seconds", type=float, default=3.0)
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


def bench_p_sweep(args, torch, neat, pop, tn, tc, tx, hdr,
                  sizes=(50, 100, 200, 500, 1000, 2000, 5000, 10000)):
    """The control step (transformation + forward, B=1000) on the first P
    genomes of the control population for P from 50 to 10000, the paper's
    population axis: ms per step (median of 5 runs of 20 steps after a
    warmup), genome-inputs/s and the end-to-end HBM fraction of the step's
    algorithmic bytes (as step_roofline, over the P genomes)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    lib = neat.lib()
    out = []
    for P in sizes:
        if P > pop.P:
            continue
        d = neat.Dims(P, tn.shape[1], tc.shape[1], pop.I, pop.O)
        prog = torch.empty((neat.program_bytes(d) // 4,), dtype=torch.int32, device=dev)
        st = torch.empty((P,), dtype=torch.int32, device=dev)
        y = torch.empty((P, pop.B, pop.O), dtype=torch.float32, device=dev)
        n, c, x = tn[:P], tc[:P], tx[:P]

        def step():
            neat._lib.check(lib.neat_topo_sort(ctypes.byref(d), ctypes.c_void_p(n.data_ptr()),
                                               ctypes.c_void_p(c.data_ptr()), None, None,
                                               ctypes.c_void_p(st.data_ptr()),
                                               ctypes.c_void_p(prog.data_ptr()), sp))
            neat._lib.check(lib.neat_forward(ctypes.byref(d), ctypes.c_void_p(prog.data_ptr()),
                                             ctypes.c_void_p(x.data_ptr()), pop.B * pop.I, pop.B,
                                             ctypes.c_void_p(y.data_ptr()), sp))

        for _ in range(3):
            step()
        runs = []
        for _ in range(5):
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(20):
                step()
            torch.cuda.synchronize()
            runs.append((time.perf_counter() - t) * 1e3 / 20)
        ms = float(np.median(runs))
        pb = program_bytes_read(pop.O, hdr[:P, 0], hdr[:P, 7], pop.I)
        step_bytes = P * (20 * pop.N_max + 16 * pop.C_max + 4) + pb + \
            P * pop.B * (pop.I + pop.O) * 4 + pb
        out.append({"P": P, "ms_per_step": round(ms, 4), "min_ms": round(min(runs), 4),
                    "value": round(P * pop.B / (ms / 1e3), 1),
                    "hbm_frac_end_to_end": round(step_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)})
    return {"workload": "control step on the first P genomes of the control population, B=1000",
            "unit": "genome-inputs/s", "points": out}


def bench_control_forms(args, torch, neat, pop, tn, tc, tx, step_bytes, parts=10):
    """The control workload (P=10000, N_max=50, B=1000) as `parts`
    populations of P/parts genomes: plain (one neat_topo_sort and one
    neat_forward per population) against batched (all populations as one
    recorded batch, transformation + calculation per replay), and the whole
    population as a single batch item; each form's end-to-end HBM fraction
    from the step's algorithmic bytes (step_bytes)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    lib = neat.lib()
    bounds = [pop.P * k // parts for k in range(parts + 1)]
    chunks = []
    for k in range(parts):
        g0, g1 = bounds[k], bounds[k + 1]
        d = neat.Dims(g1 - g0, tn.shape[1], tc.shape[1], pop.I, pop.O)
        prog = torch.empty((neat.program_bytes(d) // 4,), dtype=torch.int32, device=dev)
        st = torch.empty((g1 - g0,), dtype=torch.int32, device=dev)
        y = torch.empty((g1 - g0, pop.B, pop.O), dtype=torch.float32, device=dev)
        chunks.append((d, tn[g0:g1], tc[g0:g1], tx[g0:g1], prog, st, y))

    def plain():
        for d, n, c, x, prog, st, y in chunks:
            neat._lib.check(lib.neat_topo_sort(ctypes.byref(d), ctypes.c_void_p(n.data_ptr()),
                                               ctypes.c_void_p(c.data_ptr()), None, None,
                                               ctypes.c_void_p(st.data_ptr()),
                                               ctypes.c_void_p(prog.data_ptr()), sp))
            neat._lib.check(lib.neat_forward(ctypes.byref(d), ctypes.c_void_p(prog.data_ptr()),
                                             ctypes.c_void_p(x.data_ptr()), pop.B * pop.I,
                                             pop.B, ctypes.c_void_p(y.data_ptr()), sp))

    items = [neat.batch_item(d, prog, y, inputs=x, B=pop.B, nodes=n, conns=c, status=st)
             for d, n, c, x, prog, st, y in chunks]
    d1 = neat.dims_of(tn, tc, pop.I, pop.O)
    prog1 = torch.empty((neat.program_bytes(d1) // 4,), dtype=torch.int32, device=dev)
    st1 = torch.empty((pop.P,), dtype=torch.int32, device=dev)
    y1 = torch.empty((pop.P, pop.B, pop.O), dtype=torch.float32, device=dev)
    one = [neat.batch_item(d1, prog1, y1, inputs=tx, B=pop.B, nodes=tn, conns=tc, status=st1)]
    plan, plan1 = neat.BatchPlan(), neat.BatchPlan()

    def timed(fn):
        ramp(args, torch, fn)
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / args.steps

    ms_plain = timed(plain)
    ms_batch = timed(lambda: plan.run(items))
    ms_one = timed(lambda: plan1.run(one))
    same = all(torch.equal(torch.nan_to_num(y, nan=7.5), torch.nan_to_num(y1[b0:b0 + y.shape[0]],
                                                                          nan=7.5))
               for (d, n, c, x, prog, st, y), b0 in zip(chunks, bounds))
    plan.free()
    plan1.free()
    units = pop.P * pop.B
    return {"workload": "the control workload as %d populations of %d genomes"
                        % (parts, pop.P // parts),
            "plain_ms": round(ms_plain, 4), "plain_launches": 2 * parts,
            "plain_value": round(units / (ms_plain / 1e3), 1),
            "batched_ms": round(ms_batch, 4),
            "batched_value": round(units / (ms_batch / 1e3), 1),
            "batched_speedup": round(ms_plain / ms_batch, 3),
            "one_item_batched_ms": round(ms_one, 4),
            "one_item_batched_value": round(units / (ms_one / 1e3), 1),
            "hbm_frac_end_to_end": {
                k: round(step_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                for k, ms in (("plain", ms_plain), ("batched", ms_batch),
                              ("one_item_batched", ms_one))},
            "outputs_identical": bool(same), "unit": "genome-inputs/s"}


def served_control(args, torch, neat, pop, tn, tc, tx, fwd_bytes, parts=10, bursts=20):
    """The control workload (P=10000, N_max=50, B=1000) served: its genomes
    registered as `parts` resident populations, then `bursts` rounds of one
    request per population (B=1000 inputs each, a round per neat_submit_many
    call) queued back to back and waited for at the end, against the same calculations as plain
    neat_forward launches one after another (programs resident in both
    forms).  Each round writes its own output buffers; the last round's
    outputs are compared bit for bit.  HBM fraction from the forward's
    algorithmic bytes (fwd_bytes per round)."""
    dev = torch.device("cuda:0")
    server = neat.Server(cap_bytes=64 << 30, max_inflight=4)
    bounds = [pop.P * k // parts for k in range(parts + 1)]
    ids, progs = [], []
    for k in range(parts):
        g0, g1 = bounds[k], bounds[k + 1]
        ids.append(server.register(tn[g0:g1].contiguous(), tc[g0:g1].contiguous(), pop.I, pop.O))
        _, _, _, pg = neat.topo_sort(tn[g0:g1], tc[g0:g1], pop.I, pop.O, want_order=False)
        progs.append((neat.dims_of(tn[g0:g1], tc[g0:g1], pop.I, pop.O), pg))
    xs = [tx[bounds[k]:bounds[k + 1]] for k in range(parts)]
    ys = [[torch.empty((bounds[k + 1] - bounds[k], pop.B, pop.O), device=dev)
           for k in range(parts)] for _ in range(bursts)]
    yp = [torch.empty_like(y) for y in ys[0]]

    def plain():
        for _ in range(bursts):
            for k in range(parts):
                neat.forward(progs[k][0], progs[k][1], xs[k], pop.B, outputs=yp[k])

    # each round handed over in one neat_submit_many call (one crossing per
    # round rather than per request), records built in advance
    rounds = [[server.request(ids[k], ys[r][k], inputs=xs[k], B=pop.B, I=pop.I,
                              tag=r * parts + k) for k in range(parts)] for r in range(bursts)]

    def served():
        pend = []
        for recs in rounds:
            pend += server.submit_many(recs)
        for t in pend:
            server.wait(t)

    times = {}
    for name, fn in (("plain", plain), ("served", served)):
        ramp(args, torch, fn)
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        times[name] = best
    server.reset_stats()
    served()
    torch.cuda.synchronize()
    st = server.stats()
    same = all(torch.equal(ys[-1][k].view(torch.int32), yp[k].view(torch.int32))
               for k in range(parts))
    server.close()
    gi = pop.P * pop.B * bursts

    def frac(sec):
        return round(fwd_bytes * bursts / sec / 1e9 / HBM_PEAK_GBS, 4)

    return {"workload": "the control workload served: %d resident populations of %d genomes, "
                        "%d rounds of one request each (B=%d) queued at once"
                        % (parts, pop.P // parts, bursts, pop.B),
            "plain_ms": round(times["plain"] * 1e3, 3),
            "plain_launches": parts * bursts,
            "plain_value": round(gi / times["plain"], 1),
            "served_ms": round(times["served"] * 1e3, 3),
            "served_value": round(gi / times["served"], 1),
            "served_speedup": round(times["plain"] / times["served"], 3),
            "hbm_frac_forward": {"plain": frac(times["plain"]), "served": frac(times["served"])},
            "batches": int(st.batches),
            "mean_requests_per_batch": round(st.batched_requests / max(1, st.batches), 2),
            "p50_ms": round(st.p50_ms, 3), "p99_ms": round(st.p99_ms, 3),
            "outputs_identical": bool(same), "unit": "genome-inputs/s"}


def bench_batched(args, torch, neat, synth):
    """64 uneven populations (P, N_max, B log-uniform; C_max = 4 N_max) run
    as one recorded batch: transformation + calculation of every population
    per replay, and the calculation alone."""
    dev = torch.device("cuda:0")
    t0 = time.time()
    pops = synth.uneven(seed=2)
    log(args, "generated %d uneven populations in %.1fs" % (len(pops), time.time() - t0))
    bufs = []
    for pop in pops:
        tn = torch.from_numpy(pop.nodes).to(dev)
        tc = torch.from_numpy(pop.conns).to(dev)
        tx = torch.from_numpy(pop.inputs).to(dev)
        d = neat.dims_of(tn, tc, pop.I, pop.O)
        prog = torch.empty((neat.program_bytes(d) // 4,), dtype=torch.int32, device=dev)
        st = torch.empty((pop.P,), dtype=torch.int32, device=dev)
        y = torch.empty((pop.P, pop.B, pop.O), dtype=torch.float32, device=dev)
        bufs.append((pop, d, tn, tc, tx, prog, st, y))
    full = [neat.batch_item(d, prog, y, inputs=tx, B=pop.B, nodes=tn, conns=tc, status=st)
            for pop, d, tn, tc, tx, prog, st, y in bufs]
    fwd_only = [neat.batch_item(d, prog, y, inputs=tx, B=pop.B)
                for pop, d, tn, tc, tx, prog, st, y in bufs]
    stream = torch.cuda.current_stream()

    def timed(fn, steps):
        ramp(args, torch, fn)
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def run_batches():
        res = {}
        for name, items in (("end_to_end", full), ("forward", fwd_only)):
            plan = neat.BatchPlan()
            res[name] = (timed(lambda: plan.run(items), args.steps), plan.launches)
            plan.free()
        return res

    untuned = run_batches()
    # the autotuner on every population (outside the timed region): the
    # batch uses each bucket's throughput winner, plain calls their latency
    # winner
    t_tune = time.time()
    tuned_to = {}
    for pop, d, tn, tc, tx, prog, st, y in bufs:
        neat.autotune_forward(d, prog, tx, pop.B, outputs=y, reps=3)
        v = neat.tuned_variant(d, pop.B, throughput=True)
        tuned_to[v] = tuned_to.get(v, 0) + 1
    log(args, "autotuned 64 populations in %.1fs: %s" % (time.time() - t_tune, tuned_to))
    res = run_batches()

    # the same work as plain per-population launches: transformation and
    # calculation of each population in turn, and the calculations alone
    def plain_e2e():
        for pop, d, tn, tc, tx, prog, st, y in bufs:
            neat.topo_sort(tn, tc, pop.I, pop.O, program=prog, status=st, want_order=False)
            neat.forward(d, prog, tx, pop.B, outputs=y, variant=neat.FWD_TUNED)

    def plain_fwd():
        for pop, d, tn, tc, tx, prog, st, y in bufs:
            neat.forward(d, prog, tx, pop.B, outputs=y, variant=neat.FWD_TUNED)

    ms_plain_e2e = timed(plain_e2e, max(3, args.steps // 4))
    ms_plain_fwd = timed(plain_fwd, max(3, args.steps // 4))
    units = sum(pop.P * pop.B for pop in pops)
    fwd_bytes = 0
    for pop, d, tn, tc, tx, prog, st, y in bufs:
        hdr = neat.program_headers(d, prog).cpu().numpy()
        fwd_bytes += pop.P * pop.B * (pop.I + pop.O) * 4
        fwd_bytes += program_bytes_read(pop.O, hdr[:, 0], hdr[:, 7], pop.I)
    ms_e2e, n_e2e = res["end_to_end"]
    ms_fwd, n_fwd = res["forward"]
    achieved = fwd_bytes / (ms_fwd / 1e3) / 1e9
    return {
        "workload": "uneven batch: 64 populations, P log-uniform [100, 4096], N_max "
                    "log-uniform [10, 400], C_max = 4 N_max, B log-uniform [1, 512]",
        "genomes": sum(pop.P for pop in pops), "genome_inputs": units,
        "ms_end_to_end": round(ms_e2e, 4), "launches_end_to_end": n_e2e,
        "value_end_to_end": round(units / (ms_e2e / 1e3), 1),
        "ms_forward": round(ms_fwd, 4), "launches_forward": n_fwd,
        "value_forward": round(units / (ms_fwd / 1e3), 1), "unit": "genome-inputs/s",
        "untuned": {"ms_end_to_end": round(untuned["end_to_end"][0], 4),
                    "ms_forward": round(untuned["forward"][0], 4)},
        "tuned_throughput_winners": {{0: "auto", 1: "reg", 2: "lds", 3: "reg2",
                                      5: "lvl"}.get(k, str(k)): v for k, v in tuned_to.items()},
        "plain": {"ms_end_to_end": round(ms_plain_e2e, 4), "ms_forward": round(ms_plain_fwd, 4),
                  "launches_end_to_end": 2 * len(pops), "launches_forward": len(pops),
                  "value_end_to_end": round(units / (ms_plain_e2e / 1e3), 1),
                  "value_forward": round(units / (ms_plain_fwd / 1e3), 1)},
        "batched_speedup_end_to_end": round(ms_plain_e2e / ms_e2e, 3),
        "batched_speedup_forward": round(ms_plain_fwd / ms_fwd, 3),
        "roofline_forward": {"bound": "hbm", "achieved": round(achieved, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(achieved / HBM_PEAK_GBS, 4),
                             "algorithmic_bytes_per_launch": fwd_bytes,
                             "note": "neither HBM nor ALU bounds this launch: with B of 1 "
                                     "to 512 most genomes' node chains are latency-bound "
                                     "at low occupancy (large genomes need 128-224 value "
                                     "registers per lane)"},
    }


def bench_tiny(args, torch, neat, synth):
    """The tiny workload (P = 16, N_max = 8, 32 shared inputs): latency of
    one transformation + calculation call pair through the C ABI, on the
    device (events over consecutive calls) and end to end on the host (each
    pair synchronized); and the same pair through the Python wrappers
    (argument checks on torch tensors included)."""
    dev = torch.device("cuda:0")
    pop = synth.tiny()
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    tx = torch.from_numpy(pop.inputs).to(dev)
    d = neat.dims_of(tn, tc, pop.I, pop.O)
    _, _, st, prog = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False)
    y = torch.empty((pop.P, pop.B, pop.O), device=dev)
    stream = torch.cuda.current_stream()
    lib = neat.lib()
    sp = ctypes.c_void_p(stream.cuda_stream)
    dref = ctypes.byref(d)
    a_n, a_c, a_s, a_p, a_x, a_y = [ctypes.c_void_p(t.data_ptr()) for t in (tn, tc, st, prog, tx, y)]

    def call():
        neat._lib.check(lib.neat_topo_sort(dref, a_n, a_c, None, None, a_s, a_p, sp))
        neat._lib.check(lib.neat_forward(dref, a_p, a_x, 0, pop.B, a_y, sp))

    def call_wrapped():
        neat.topo_sort(tn, tc, pop.I, pop.O, program=prog, status=st, want_order=False)
        neat.forward(d, prog, tx, pop.B, shared_inputs=True, outputs=y)

    def back_to_back(fn, n=500):
        for _ in range(20):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n * 1e3

    ramp(args, torch, call)
    dev_us = back_to_back(call)
    host = []
    for _ in range(200):
        t = time.perf_counter()
        call()
        torch.cuda.synchronize()
        host.append(time.perf_counter() - t)
    wrapped_us = back_to_back(call_wrapped)
    return {"workload": "tiny: P=16, N_max=8, C_max=16, I=3, O=1, 32 shared inputs, "
                        "transformation + calculation per call",
            "us_per_call_back_to_back": round(dev_us, 2),
            "us_per_call_synchronized_p50": round(float(np.median(host)) * 1e6, 2),
            "us_per_call_back_to_back_python_wrappers": round(wrapped_us, 2),
            "genome_inputs_per_call": pop.P * pop.B}


def served_stream(args, torch, neat, server, pool, ids, xpool, ypool, rate, seconds, seed,
                  tune=False):
    """One Poisson stream of requests over the resident pool: arrivals at
    `rate` per second for `seconds`, each request a uniform pool population
    with B log-uniform [1, 256] and inputs cut from xpool at a seed-derived
    offset.  Latency = completion - scheduled arrival, over arrivals after
    the first quarter."""
    rng = np.random.default_rng(seed)
    n_req = max(1, int(rate * seconds))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    which = rng.integers(0, len(pool), n_req)
    Bs = np.rint(np.exp(rng.uniform(0.0, np.log(256.0), n_req))).astype(np.int64)
    torch.cuda.synchronize()
    server.reset_stats()
    pending = {}  # ticket -> (k, submit delay)
    done = []     # (k, latency_s)
    y_at = 0
    late = 0
    t_start = time.perf_counter()

    def drain():
        for t in list(pending):
            r = server.poll(t)
            if r is not None:
                k, delay = pending.pop(t)
                done.append((k, delay + (r.t_done_ns - r.t_submit_ns) * 1e-9))

    for k in range(n_req):
        pop, B = pool[which[k]], int(Bs[k])
        nx, ny = pop.P * B * pop.I, pop.P * B * pop.O
        xo = int(rng.integers(0, xpool.numel() - nx))
        if y_at + ny > ypool.numel():
            while pending:  # wrap the output pool once earlier requests are done
                drain()
            y_at = 0
        while True:
            now = time.perf_counter() - t_start
            if now >= arrivals[k]:
                break
            drain()
            if arrivals[k] - now > 2e-4:
                time.sleep(1e-4)
        delay = time.perf_counter() - t_start - arrivals[k]
        late += delay > 1e-3
        t = server.submit(ids[which[k]], ypool[y_at:y_at + ny], inputs=xpool[xo:xo + nx],
                          B=B, I=pop.I, tag=k)
        pending[t] = (k, delay)
        y_at += ny
        if k % 64 == 63:
            drain()
    while pending:
        drain()
    wall = time.perf_counter() - t_start
    st = server.stats()
    lat = np.array([l for k, l in done if arrivals[k] >= 0.25 * seconds]) if n_req >= 8 \
        else np.array([l for _, l in done])
    gi = int(sum(pool[which[k]].P * int(Bs[k]) for k in range(n_req)))
    hbm = sum(pool[which[k]].P * int(Bs[k]) * (pool[which[k]].I + pool[which[k]].O) * 4
              for k in range(n_req))
    return {"rate_req_s": rate, "seconds": seconds, "requests": n_req,
            "offered_req_s": round(n_req / arrivals[-1], 1),
            "submitted_late_over_1ms": int(late),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "latency_counted": int(len(lat)), "genome_inputs": gi,
            "throughput": round(gi / wall, 1), "unit": "genome-inputs/s",
            "input_output_GBps": round(hbm / wall / 1e9, 2),
            "hbm_frac": round(hbm / wall / 1e9 / HBM_PEAK_GBS, 5),
            "batches": int(st.batches),
            "mean_requests_per_batch": round(st.batched_requests / max(1, st.batches), 2),
            "peak_footprint_GiB": round(st.peak_bytes / 2 ** 30, 3),
            "resident_GiB": round(st.resident_bytes / 2 ** 30, 3)}


def bench_served(args, torch, neat, synth):
    """Served path over 128 resident populations (P log-uniform [64, 8192],
    N_max log-uniform [8, 256], C_max = 4 N_max): the Poisson stream at the
    configured rate, a sweep of higher rates, a burst against plain
    per-request launches, and CPPN grid requests."""
    dev = torch.device("cuda:0")
    t0 = time.time()
    pool = synth.served_pool(seed=3)
    log(args, "generated %d resident populations in %.1fs" % (len(pool), time.time() - t0))
    server = neat.Server(cap_bytes=64 << 30, max_inflight=4)
    ids = []
    for pop in pool:
        tn = torch.from_numpy(pop.nodes).to(dev)
        tc = torch.from_numpy(pop.conns).to(dev)
        ids.append(server.register(tn, tc, pop.I, pop.O))
        del tn, tc
    gen = torch.Generator(device=dev)
    gen.manual_seed(3)
    xpool = torch.randn((1 << 30,), generator=gen, device=dev)  # 4 GiB
    ypool = torch.empty((1 << 30,), device=dev)
    main = served_stream(args, torch, neat, server, pool, ids, xpool, ypool,
                         args.served_rate, args.served_seconds, seed=3)
    log(args, "served stream: %s" % main)
    sweep = []
    for rate in [float(r) for r in args.served_sweep.split(",") if r]:
        sweep.append(served_stream(args, torch, neat, server, pool, ids, xpool, ypool, rate,
                                   args.sweep_seconds, seed=int(rate) + 7))
        log(args, "served sweep: %s" % sweep[-1])
    burst = served_burst(args, torch, neat, server, pool, ids, xpool, ypool) \
        if args.served_burst > 0 else None
    cppn = served_cppn(args, torch, neat, synth, server)
    server.close()
    out = {"workload": "served: Poisson %.0f req/s for %.0f s over 128 resident populations "
                       "(P log-uniform [64, 8192], N_max log-uniform [8, 256], C_max = 4 N_max), "
                       "B log-uniform [1, 256]" % (args.served_rate, args.served_seconds)}
    out.update(main)
    out["rate_sweep"] = sweep
    out["burst_vs_plain"] = burst
    out["cppn_grid_requests"] = cppn
    return out


def served_cppn(args, torch, neat, synth, server):
    """CPPN substrate queries served as batched GRID requests: the CPPN
    population (P = 1000, N_max = 30) registered on the server, the 65536
    queries of the 16 x 16 grid split into requests of 4096 queries, queued
    in one neat_submit_many call; against one plain neat_forward_grid call over the whole grid
    (outputs compared bit for bit).  Best of three."""
    dev = torch.device("cuda:0")
    pop = synth.cppn()
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    pid = server.register(tn, tc, pop.I, pop.O)
    d = neat.dims_of(tn, tc, pop.I, pop.O)
    _, _, _, prog = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False)
    Q, chunk = 65536, 4096
    yfull = torch.empty((pop.P, Q, pop.O), device=dev)
    parts = [torch.empty((pop.P, chunk, pop.O), device=dev) for _ in range(Q // chunk)]

    def plain():
        neat.forward_grid(d, prog, 16, 0, Q, outputs=yfull)
        torch.cuda.synchronize()

    recs = [server.request(pid, parts[k], B=chunk, grid_side=16, grid_first=k * chunk, tag=k)
            for k in range(len(parts))]

    def served():
        for t in server.submit_many(recs):
            server.wait(t)
        torch.cuda.synchronize()

    times = {}
    for name, fn in (("plain", plain), ("served", served)):
        fn()
        best = float("inf")
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            best = min(best, time.perf_counter() - t)
        times[name] = best
    server.reset_stats()
    served()
    st = server.stats()
    same = all(torch.equal(parts[k].view(torch.int32),
                           yfull[:, k * chunk:(k + 1) * chunk].contiguous().view(torch.int32))
               for k in range(len(parts)))
    gi = pop.P * Q
    return {"workload": "CPPN P=1000 (N_max=30) on all 65536 queries of a 16x16 grid as %d "
                        "GRID requests of %d queries" % (len(parts), chunk),
            "plain_ms": round(times["plain"] * 1e3, 3), "served_ms": round(times["served"] * 1e3, 3),
            "served_value": round(gi / times["served"], 1), "plain_value": round(gi / times["plain"], 1),
            "batches": int(st.batches),
            "mean_requests_per_batch": round(st.batched_requests / max(1, st.batches), 2),
            "p50_ms": round(st.p50_ms, 3), "p99_ms": round(st.p99_ms, 3),
            "outputs_identical": bool(same), "unit": "genome-inputs/s"}


def served_burst(args, torch, neat, server, pool, ids, xpool, ypool):
    """Saturation: the same requests (population and B drawn as in the
    stream) once queued to the server all at once (one neat_submit_many
    call), once as plain
    per-request forward launches one after another; programs are resident
    in both forms (the plain form's transformed before timing).  Best of
    three; the outputs of the two forms are compared bit for bit."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(4)
    reqs, xo, yo = [], 0, 0
    while len(reqs) < args.served_burst:
        j = int(rng.integers(0, len(pool)))
        B = int(np.rint(np.exp(rng.uniform(0.0, np.log(256.0)))))
        pop = pool[j]
        nx, ny = pop.P * B * pop.I, pop.P * B * pop.O
        if xo + nx > xpool.numel() or yo + ny > ypool.numel():
            break
        reqs.append((j, B, xo, nx, yo, ny))
        xo, yo = xo + nx, yo + ny
    progs = {}
    for j in sorted({r[0] for r in reqs}):
        pop = pool[j]
        tn = torch.from_numpy(pop.nodes).to(dev)
        tc = torch.from_numpy(pop.conns).to(dev)
        _, _, _, pg = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False)
        progs[j] = (neat.dims_of(tn, tc, pop.I, pop.O), pg)
        del tn, tc
    yplain = torch.empty((yo,), device=dev)

    def plain():
        for j, B, x0, nx, y0, ny in reqs:
            pop = pool[j]
            d, pg = progs[j]
            neat.forward(d, pg, xpool[x0:x0 + nx].view(pop.P, B, pop.I), B,
                         outputs=yplain[y0:y0 + ny].view(pop.P, B, pop.O))
        torch.cuda.synchronize()

    recs = [server.request(ids[j], ypool[y0:y0 + ny], inputs=xpool[x0:x0 + nx], B=B,
                           I=pool[j].I, tag=k)
            for k, (j, B, x0, nx, y0, ny) in enumerate(reqs)]

    def served():
        pending = set(server.submit_many(recs))
        while pending:
            for t in list(pending):
                if server.poll(t) is not None:
                    pending.discard(t)
        torch.cuda.synchronize()

    times = {}
    for name, fn in (("plain", plain), ("served", served)):
        fn()  # warm-up
        best = float("inf")
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            best = min(best, time.perf_counter() - t)
        times[name] = best
    same = bool(torch.equal(ypool[:yo].view(torch.int32), yplain.view(torch.int32)))
    gi = sum(pool[r[0]].P * r[1] for r in reqs)
    b0 = server.stats().batches
    served()
    nb = server.stats().batches - b0
    return {"requests": len(reqs), "genome_inputs": int(gi),
            "plain_ms": round(times["plain"] * 1e3, 3),
            "plain_value": round(gi / times["plain"], 1),
            "served_ms": round(times["served"] * 1e3, 3),
            "served_value": round(gi / times["served"], 1),
            "served_speedup": round(times["plain"] / times["served"], 3),
            "served_batches": int(nb), "outputs_identical": same,
            "unit": "genome-inputs/s"}


def bench_cppn(args, torch, neat, synth):
    """CPPN substrate queries: P = 1000 genomes (I = 5, O = 1, N_max = 30,
    C_max = 120, sin/gaussian/abs/tanh/sigmoid, sum) on all 65536 pairs of a
    16 x 16 grid, inputs generated in the kernel."""
    dev = torch.device("cuda:0")
    pop = synth.cppn()
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    d = neat.dims_of(tn, tc, pop.I, pop.O)
    _, _, st, prog = neat.topo_sort(tn, tc, pop.I, pop.O, want_order=False)
    Q = 65536
    y = torch.empty((pop.P, Q, pop.O), device=dev)
    ramp(args, torch, lambda: neat.forward_grid(d, prog, 16, 0, Q, outputs=y))
    for _ in range(max(1, args.warmup)):
        neat.forward_grid(d, prog, 16, 0, Q, outputs=y)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        neat.forward_grid(d, prog, 16, 0, Q, outputs=y)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    units = pop.P * Q
    # algorithmic flops per genome-input: 2 per enabled connection (multiply,
    # add), 2 per computed node (response, bias) plus its activation's
    flops = 0
    for g in range(pop.P):
        nd, cn = pop.nodes[g], pop.conns[g]
        live = ~np.isnan(nd[:, 0])
        comp = live & (nd[:, 0] >= pop.I)
        en = (~np.isnan(cn[:, 0])) & (cn[:, 2] == 1.0)
        flops += 2 * int(en.sum()) + int(sum(2 + ACT_FLOPS[int(a)] for a in nd[comp, 3]))
    tflops = flops * Q / (ms / 1e3) / 1e12
    return {"workload": "cppn: P=1000, N_max=30, C_max=120, I=5, O=1, 65536 grid queries "
                        "per genome generated in the kernel",
            "ms": round(ms, 4), "value": round(units / (ms / 1e3), 1),
            "unit": "genome-inputs/s", "output_GBps": round(units * 4 / (ms / 1e3) / 1e9, 1),
            "roofline": {"bound": "alu", "achieved": round(tflops, 2),
                         "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tflops / VALU_PEAK_TFLOPS, 4),
                         "flops_per_genome_input": round(flops / pop.P, 1)}}


MFMA_F32_PEAK_TFLOPS = 157.3


def bench_substrate(args, torch, neat, synth):
    """HyperNEAT substrate: P=1000 CPPNs paint a 256 x 256 weight matrix each
    (side 16 grid), threshold 0.2, then tanh(X W') for B=256 shared input
    planes; CPPN queries + substrate layer per step."""
    dev = torch.device("cuda:0")
    pop = synth.cppn()
    side, S = 16, 256
    X = torch.from_numpy(synth.substrate_inputs(B=256, side=side)).to(dev)
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    _, _, st, prog = neat.topo_sort(tn, tc, 5, 1, want_order=False)
    d = neat.dims_of(tn, tc, 5, 1)
    w = torch.empty((pop.P, S, S), dtype=torch.float32, device=dev)
    y = torch.empty((pop.P, X.shape[0], S), dtype=torch.float32, device=dev)
    ramp(args, torch, lambda: neat.substrate_forward(d, prog, side, X, 0.2, weights=w, outputs=y))
    for _ in range(max(1, args.warmup)):
        neat.substrate_forward(d, prog, side, X, 0.2, weights=w, outputs=y)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        neat.substrate_forward(d, prog, side, X, 0.2, weights=w, outputs=y)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # the CPPN part alone (the same grid calculation the call makes first)
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    for _ in range(args.steps):
        neat.forward_grid(d, prog, side, 0, S * S, outputs=w)
    g1.record(stream)
    torch.cuda.synchronize()
    ms_cppn = g0.elapsed_time(g1) / args.steps
    ms_layer = max(ms - ms_cppn, 1e-6)
    flops = 2.0 * pop.P * X.shape[0] * S * S
    tflops = flops / (ms_layer / 1e3) / 1e12
    return {"workload": "hyperneat substrate: P=1000 CPPNs (N_max=30), 16x16 grid (S=256), "
                        "threshold 0.2, B=256 shared input planes, tanh layer",
            "ms": round(ms, 4), "ms_cppn_weights": round(ms_cppn, 4),
            "ms_substrate_layer": round(ms_layer, 4),
            "value": round(pop.P * X.shape[0] / (ms / 1e3), 1), "unit": "genome-inputs/s",
            "roofline": {"kernel": "substrate layer, fp32 MFMA 16x16x4", "bound": "mfma",
                         "achieved": round(tflops, 2), "peak": MFMA_F32_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / MFMA_F32_PEAK_TFLOPS, 4),
                         "flops_per_launch": flops}}


def bench_distance(args, torch, neat, synth):
    """Compatibility distance (speciation): P=10000 control genomes against
    Q=64 species representatives."""
    dev = torch.device("cuda:0")
    pop = synth.control(P=args.P, B=1, with_inputs=False)
    rep = synth.control(seed=7, P=64, B=1, with_inputs=False)
    t = [torch.from_numpy(a).to(dev) for a in (pop.nodes, pop.conns, rep.nodes, rep.conns)]
    out = torch.empty((pop.P, rep.P), dtype=torch.float32, device=dev)
    ramp(args, torch, lambda: neat.distance(*t, out=out))
    for _ in range(max(1, args.warmup)):
        neat.distance(*t, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        neat.distance(*t, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    pairs = pop.P * rep.P
    # algorithmic HBM bytes: every genome's rows once (nodes 20 B,
    # connections 16 B per row), the representatives once (they stay in
    # L2), the distances
    gbytes = pop.P * (pop.nodes.shape[1] * 20 + pop.conns.shape[1] * 16)
    rbytes = rep.P * (rep.nodes.shape[1] * 20 + rep.conns.shape[1] * 16)
    return {"workload": "compatibility distance: P=%d control genomes (N_max=50, C_max=200) "
                        "against Q=64 representatives" % pop.P,
            "ms": round(ms, 4), "value": round(pairs / (ms / 1e3), 1), "unit": "pairs/s",
            "hbm_GBps": round((gbytes + rbytes + pairs * 4) / (ms / 1e3) / 1e9, 1)}


def bench_crossover(args, torch, neat, synth):
    """Crossover: P=10000 children of random pairs of control genomes."""
    dev = torch.device("cuda:0")
    pop = synth.control(P=args.P, B=1, with_inputs=False)
    rng = np.random.default_rng(14)
    pairs = torch.from_numpy(rng.integers(0, pop.P, (pop.P, 2)).astype(np.int32)).to(dev)
    rn = torch.from_numpy(rng.random((pop.P, 50)).astype(np.float32)).to(dev)
    rc = torch.from_numpy(rng.random((pop.P, 200)).astype(np.float32)).to(dev)
    tn, tc = torch.from_numpy(pop.nodes).to(dev), torch.from_numpy(pop.conns).to(dev)
    cn, cc = neat.crossover(tn, tc, pairs, rn, rc)
    ramp(args, torch, lambda: neat.crossover(tn, tc, pairs, rn, rc, cn, cc))
    for _ in range(max(1, args.warmup)):
        neat.crossover(tn, tc, pairs, rn, rc, cn, cc)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        neat.crossover(tn, tc, pairs, rn, rc, cn, cc)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # algorithmic bytes per child: both parents' rows read, the child's rows
    # written, one number per first-parent row, the pair
    per = 3 * (50 * 20 + 200 * 16) + (50 + 200) * 4 + 8
    return {"workload": "crossover: %d children of control-genome pairs (N_max=50, "
                        "C_max=200)" % pop.P,
            "ms": round(ms, 4), "value": round(pop.P / (ms / 1e3), 1), "unit": "children/s",
            "roofline": {"bound": "hbm", "achieved": round(pop.P * per / (ms / 1e3) / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(pop.P * per / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                         "bytes_per_child": per}}


def bench_edit(args, torch, neat, synth):
    """Tensorized edits: a mutation-sized batch over P=10000 control genomes
    (per genome one node addition, two connection additions, one connection
    removal and four attribute writes), applied in place."""
    dev = torch.device("cuda:0")
    pop = synth.control(P=args.P, B=1, with_inputs=False)
    rng = np.random.default_rng(16)
    per = 8
    rec = np.dtype([("genome", "<i4"), ("op", "<i4"), ("row", "<i4"), ("column", "<i4"),
                    ("v", "<f4", (5,))])
    e = np.zeros(pop.P * per, rec)
    e["genome"] = np.repeat(np.arange(pop.P), per)
    e["op"] = np.tile([0, 2, 2, 3, 4, 4, 5, 5], pop.P)
    e["row"] = rng.integers(0, 50, pop.P * per)
    e["column"] = np.tile([0, 0, 0, 0, 1, 2, 3, 2], pop.P)
    e["v"] = rng.normal(size=(pop.P * per, 5)).astype(np.float32)
    te = torch.from_numpy(e.view(np.uint8).copy()).to(dev)
    tn0, tc0 = torch.from_numpy(pop.nodes).to(dev), torch.from_numpy(pop.conns).to(dev)
    tn, tc = tn0.clone(), tc0.clone()
    applied = neat.edit(tn, tc, te)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ms = []
    for _ in range(args.steps):
        tn.copy_(tn0)
        tc.copy_(tc0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        neat.edit(tn, tc, te, applied=applied)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    ms = float(np.median(ms))
    return {"workload": "tensorized edits: %d control genomes x %d edits (node add, 2 "
                        "connection adds, connection removal, 4 attribute writes)"
                        % (pop.P, per),
            "ms": round(ms, 4), "value": round(pop.P * per / (ms / 1e3), 1),
            "unit": "edits/s", "applied": int(applied.sum().item())}


def bench_recurrent(args, torch, neat, synth):
    """Recurrent networks: the control shapes with cycles (P=10000, N_max=50,
    C_max=200, B=1000), K=4 synchronous sweeps; transformation + calculation
    per step."""
    dev = torch.device("cuda:0")
    pop = synth.recurrent_control(P=args.P, B=args.B)
    K = 4
    tn = torch.from_numpy(pop.nodes).to(dev)
    tc = torch.from_numpy(pop.conns).to(dev)
    tx = torch.from_numpy(pop.inputs).to(dev)
    d = neat.dims_of(tn, tc, pop.I, pop.O)
    prog = torch.empty((neat.program_bytes(d) // 4,), dtype=torch.int32, device=dev)
    out = torch.empty((pop.P, pop.B, pop.O), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        neat.topo_sort(tn, tc, pop.I, pop.O, program=prog, want_order=False, recurrent=True)
        neat.forward_recurrent(d, prog, tx, pop.B, K, outputs=out)

    ramp(args, torch, step)
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        neat.topo_sort(tn, tc, pop.I, pop.O, program=prog, want_order=False, recurrent=True)
        ev[k][1].record(stream)
        neat.forward_recurrent(d, prog, tx, pop.B, K, outputs=out)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    fwd_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    topo_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    units = pop.P * pop.B
    # algorithmic work per genome-input: K sweeps of 2 flops per enabled
    # connection plus 2 + the activation's per computed node
    hdr = neat.program_headers(d, prog).cpu().numpy()
    flops = 0
    for g in range(pop.P):
        if hdr[g, 2] != 0:
            continue
        nd = pop.nodes[g]
        comp = (~np.isnan(nd[:, 0])) & (nd[:, 0] >= pop.I)
        flops += 2 * int(hdr[g, 7]) + int(sum(2 + ACT_FLOPS[int(a)] for a in nd[comp, 3]))
    flops *= K * pop.B
    tflops = flops / (fwd_ms / 1e3) / 1e12
    fwd_bytes = units * (pop.I + pop.O) * 4 + program_bytes_read(pop.O, hdr[:, 0], hdr[:, 7],
                                                                 pop.I)
    return {"workload": "recurrent control-policy population: P=%d, N_max=50, C_max=200, "
                        "I=17, O=6, B=%d, cycles allowed, K=%d synchronous sweeps, "
                        "transformation + calculation" % (pop.P, pop.B, K),
            "ms_per_step": round(step_ms, 4), "topo_ms": round(topo_ms, 4),
            "forward_ms": round(fwd_ms, 4),
            "value": round(units / (step_ms / 1e3), 1), "unit": "genome-inputs/s",
            "rejected_genomes": int((hdr[:, 2] != 0).sum()),
            "roofline": {"kernel": "recurrent forward, 64-slot register store (read and "
                                   "write vectors)", "bound": "alu",
                         "achieved": round(tflops, 2), "peak": VALU_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / VALU_PEAK_TFLOPS, 4),
                         "flops_per_genome_input": round(flops / units, 1),
                         "hbm_GBps": round(fwd_bytes / (fwd_ms / 1e3) / 1e9, 1)}}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(pop, g, threads, precision, min_seconds):
    """Genome-inputs/s of the oracle (transformation + calculation) over the
    first g genomes, split into `threads` contiguous genome ranges evaluated
    concurrently (the oracle is C called through ctypes, which releases the
    GIL), repeated until min_seconds have passed."""
    import concurrent.futures as cf
    import oracle
    bounds = np.linspace(0, g, threads + 1).astype(int)
    parts = [(a, b) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]

    def run(ab):
        a, b = ab
        oracle.forward(pop.nodes[a:b], pop.conns[a:b], pop.inputs[a:b], pop.I, pop.O,
                       precision=precision, with_beta=False)

    passes, t = 0, time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=len(parts)) as ex:
        while True:
            list(ex.map(run, parts))
            passes += 1
            dt = time.perf_counter() - t
            if dt >= min_seconds or passes >= 50:
                break
    return passes * g * pop.B / dt, passes, dt


def cpu_baseline(args, pop):
    """The oracle timed on this machine's host cores: its fp32 instantiation
    with genomes split over all usable cores (at most 16, the host share of
    one GPU), the same on one core, and the fp64 reference on one core."""
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(usable, 16))
    g_all = min(args.cpu_genomes, pop.P)
    g_one = min(max(g_all // 8, 1), pop.P)
    sec = args.cpu_seconds
    v_all, n_all, t_all = _oracle_rate(pop, g_all, threads, "f32", sec)
    v_one, n_one, t_one = _oracle_rate(pop, g_one, 1, "f32", sec / 2)
    v_64, n_64, t_64 = _oracle_rate(pop, g_one, 1, "f64", sec / 2)
    return {"value": round(v_all, 1), "unit": "genome-inputs/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d genomes x %d inputs of the control workload, %d passes in %.1f s: "
                      "the oracle's fp32 instantiation (transformation + calculation), "
                      "genomes split over %d threads" % (g_all, pop.B, n_all, t_all, threads),
            "os_cpu_count": os.cpu_count(), "usable_cpus": usable, "cpu_model": _cpu_model(),
            "one_core_f32": {"value": round(v_one, 1), "cores": 1,
                             "sample": "%d genomes x %d inputs, %d passes in %.1f s"
                                       % (g_one, pop.B, n_one, t_one)},
            "one_core_f64": {"value": round(v_64, 1), "cores": 1,
                             "sample": "%d genomes x %d inputs, %d passes in %.1f s, the fp64 "
                                       "parity reference" % (g_one, pop.B, n_64, t_64)}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the population forward has no "
              "cross-GPU exchange; shard genomes across GPUs by running one "
              "process per GPU.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2404_01817_amd as neat
    from workloads import synth

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

    ramp(args, torch, lambda: (topo(), fwd()))
    for _ in range(args.warmup):
        topo()
        fwd()
    torch.cuda.synchronize()

    # the timed steps: transformation + forward, nothing else in the stream
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        topo()
        fwd()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    step_ms = wall * 1e3 / args.steps
    # per-kernel breakdown, from the same number of steps bracketed by events
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for k in range(args.steps):
        ev[k][0].record(stream)
        topo()
        ev[k][1].record(stream)
        fwd()
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    topo_ms = np.array([e[0].elapsed_time(e[1]) for e in ev])
    fwd_ms = np.array([e[1].elapsed_time(e[2]) for e in ev])
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
    traffic, prof_us = measured_profile()
    roofline = {"kernel": "forward, 64-slot register store, two samples per lane", "bound": "hbm",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": fwd_bytes,
                "bytes_per_genome_input": round(fwd_bytes / units, 2),
                "avg_launch_us": round(fwd_avg_s * 1e6, 1),
                # the same fraction from the committed rocprofv3 trace's average
                "rocprof_avg_launch_us": prof_us,
                "frac_rocprof": (round(fwd_bytes / (prof_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                                 if prof_us else None)}
    # the whole step against the same peak: the transformation reads the
    # node and connection rows and writes the status and the program (at
    # least what the forward reads of it), then the forward's bytes
    step_bytes = (pop.P * (20 * pop.N_max + 16 * pop.C_max + 4) + pbytes) + fwd_bytes
    step_roofline = {"bound": "hbm", "algorithmic_bytes_per_step": step_bytes,
                     "achieved": round(step_bytes / (step_ms / 1e3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(step_bytes / (step_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}

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

    # what a plain device copy (torch) reaches on this GPU, for context: a
    # 2 GiB copy (4 GiB moved), well past the on-package cache
    src = torch.ones((512 << 20,), dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 4 / (c0.elapsed_time(c1) / 5 / 1e3) / 1e9
    del src, dst
    roofline["copy_GBps"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(achieved / copy_gbs, 4)

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
        cpu = cpu_baseline(args, pop)

    psweep = bench_p_sweep(args, torch, neat, pop, tn, tc, tx, hdr) if not args.no_p_sweep else None

    workloads = set(args.workloads.split(","))
    forms = (bench_control_forms(args, torch, neat, pop, tn, tc, tx, step_bytes)
             if "batched" in workloads else None)
    # the latency-bound regime of small populations (the population sweep's
    # plain step is launch-bound below about 500 genomes)
    forms_small = (bench_control_forms(args, torch, neat, pop, tn, tc, tx, step_bytes, parts=100)
                   if "batched" in workloads else None)
    batched = bench_batched(args, torch, neat, synth) if "batched" in workloads else None
    served = bench_served(args, torch, neat, synth) if "served" in workloads else None
    served_ctl = (served_control(args, torch, neat, pop, tn, tc, tx, fwd_bytes)
                  if "served" in workloads else None)
    served_ctl_small = (served_control(args, torch, neat, pop, tn, tc, tx, fwd_bytes, parts=100)
                        if "served" in workloads else None)
    cppn = bench_cppn(args, torch, neat, synth) if "cppn" in workloads else None
    recurrent = (bench_recurrent(args, torch, neat, synth) if "recurrent" in workloads
                 else None)
    substrate = (bench_substrate(args, torch, neat, synth) if "substrate" in workloads
                 else None)
    distance = (bench_distance(args, torch, neat, synth) if "distance" in workloads
                else None)
    crossover = (bench_crossover(args, torch, neat, synth) if "crossover" in workloads
                 else None)
    edits = bench_edit(args, torch, neat, synth) if "edit" in workloads else None
    tiny = bench_tiny(args, torch, neat, synth) if "tiny" in workloads else None

    res = {
        "metric": "genome-input forwards/s", "value": round(value, 1),
        "unit": "genome-inputs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ramp_ms": args.ramp_ms, "ms_per_step": round(step_ms, 4),
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
        "step_roofline": step_roofline,
        "cpu_baseline": cpu,
        "p_sweep": psweep,
        "control_batched_vs_plain": forms,
        "control_batched_vs_plain_100_populations": forms_small,
        "control_served_vs_plain": served_ctl,
        "control_served_vs_plain_100_populations": served_ctl_small,
        "batched": batched,
        "served": served,
        "cppn": cppn,
        "recurrent": recurrent,
        "substrate": substrate,
        "distance": distance,
        "crossover": crossover,
        "edit": edits,
        "tiny": tiny,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
