#!/usr/bin/env python3
"""Benchmark of the sample-many path on one MI355X.

A step is one clifft_sample call over the whole workload (every shot of the
batch through the compiled stream: frames, noise, active vector, records),
with the program resident on the device and the outputs preallocated,
replayed from a captured HIP graph (--no-graph: launched eagerly).
Prints one JSON line (driver contract).

Default workload: rotated surface-code memory d = 3, 3 rounds,
circuit-level depolarizing p = 1e-3, 1e7 shots (the Pauli-frame
configuration of the benchmark table).  Other workloads: --workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shots/sec at matched detector-rate accuracy, FP32-batched vs FP64-plain"
# 32-bit VALU lane-ops/s at the rate the published FP32 vector figure implies
# (157.3 TFLOP/s = 2 flops x 128 lanes x 256 CUs x 2.4 GHz).  The 16-lane SIMD
# count (39.3 T) is not an upper bound here: the integer probe exceeds it.
PEAK_INT_OPS = 256 * 128 * 2.4e9
PEAK_FP32 = 157.3e12                 # FP32 vector FLOP/s
PEAK_FP64 = 78.6e12                  # FP64 vector FLOP/s
PEAK_HBM = 8.0e12                    # HBM3E bytes/s
PEAK_LDS = 256 * 128 * 2.4e9         # LDS bytes/s: 128 B/clk/CU


def measured_peak(bound, pk, torch):
    """Achievable rate on this device for the bound, from the library's
    probes timed with HIP events on the current stream: a 1 GiB device copy
    (read + write bytes) for "hbm", a 1 GiB read-only sweep for "hbm_read",
    16 full-rate VALU instructions per iteration for "alu".  None for other
    bounds."""
    if bound not in ("hbm", "hbm_read", "alu"):
        return None
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if bound in ("hbm", "hbm_read"):
        n = 1 << 30
        src = torch.empty(n, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        grid = 256 * 16
        if bound == "hbm":
            dst = torch.empty_like(src)
            run = lambda: pk.probe(0, dst, src, n, grid, st)
            work = 2.0 * n
        else:
            dst = torch.empty(grid * 256 * 16, dtype=torch.uint8, device="cuda")
            run = lambda: pk.probe(2, dst, src, n, grid, st)
            work = 1.0 * n
        unit = 1e9
    else:
        grid, iters = 256 * 16, 2048
        dst = torch.empty(grid * 256, dtype=torch.int32, device="cuda")
        run = lambda: pk.probe(1, dst, None, iters, grid, st)
        work, unit = 16.0 * iters * grid * 256, 1e12
    run()
    torch.cuda.synchronize()
    reps = 10
    e0.record(st)
    for _ in range(reps):
        run()
    e1.record(st)
    torch.cuda.synchronize()
    return work * reps / (e0.elapsed_time(e1) * 1e-3) / unit


def add_measured_peak(roof, pk, torch):
    """peak_measured: the larger achievable rate for the bound (for HBM, of a
    copy and a read-only sweep, since read-heavy kernels outrun a copy)."""
    m = measured_peak(roof["bound"], pk, torch)
    if m and roof["bound"] == "hbm":
        r = measured_peak("hbm_read", pk, torch)
        roof["probes"] = {"copy": m, "read": r}
        m = max(m, r)
    if m:
        roof["peak_measured"] = m
        roof["frac_measured"] = roof["achieved"] / m


def load_traffic(workload, precision, kernel):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they
    were taken on this kernel and its current sources."""
    from paper_2604_27058_amd.profiling import kernel_family, kernel_source_hash
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (workload, precision))
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    family = kernel_family(kernel)
    if d.get("kernel_family", "interpreter") != family or d.get("kernel_source_hash") != kernel_source_hash(family):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(text, shots_hint, seed):
    """The FP64 oracle timed on the host cores on a bounded sample."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    prog = oracle.Program(text)
    n = 4096
    t0 = time.perf_counter()
    prog.sample(n, seed=seed, threads=threads)
    dt = time.perf_counter() - t0
    # scale the sample to about 10 s of CPU time, within the workload's shots
    target = min(shots_hint, max(64, int(n * 10.0 / max(dt, 1e-6))))
    target = (target + 63) // 64 * 64
    t0 = time.perf_counter()
    meas, det, obs = prog.sample(target, seed=seed, threads=threads)
    dt = time.perf_counter() - t0
    return dict(value=target / dt, unit="shots/s", cores=threads, kind="oracle",
                sample="first %d shots of the workload (seed %d), FP64 oracle, %d threads, %.1f s"
                       % (target, seed, threads, dt)), (target, meas, det, obs)


def captured(fn, torch):
    """fn captured in a HIP graph (torch.cuda.CUDAGraph) after one eager
    call on a side stream; returns the replay callable."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g.replay, g


def bench_batch(args, w, pk, torch):
    """Batched workload: all circuits in one persistent FP32 launch, against
    the plain FP64 form (one clifft_sample call per circuit) on the same GPU."""
    import numpy as np
    texts = w["texts"]
    shots = [w["shots"]] * len(texts)
    seeds = list(range(len(texts)))
    progs = [pk.Program(t) for t in texts]
    precision = args.precision or "f32"
    if not args.no_autotune and not args.threads_per_shot:
        for p in progs:
            p.autotune(shots[0], precision)
            p.autotune(shots[0], "f64")  # the plain FP64 form below uses its own tuned shapes
    B = pk.Batch(progs, shots, seeds, precision=precision, threads_per_shot=args.threads_per_shot, grid=args.grid)
    outs, ws = B.alloc()
    stream = torch.cuda.current_stream()
    step = lambda: B.sample(outs, ws)
    if not args.no_graph:
        step, graph = captured(step, torch)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = sum(a.elapsed_time(b) for a, b in evs) / len(evs)
    total = sum(shots)
    value = total * args.steps / wall
    # plain FP64 form: one call per circuit, sequential, same shots and seeds
    L64 = pk.make_launch("f64")
    plain = [(p, p.alloc_outputs(n), p.alloc_workspace(L64)) for p, n in zip(progs, shots)]
    for p, o, wsp in plain:
        p.sample(shots[0], seed=0, launch=L64, outputs=o, workspace=wsp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (p, o, wsp) in enumerate(plain):
        p.sample(shots[i], seed=seeds[i], launch=L64, outputs=o, workspace=wsp)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    # matched accuracy: the FP32 batched records agree with the FP64 plain ones
    differing = 0
    for i, (p, o, _) in enumerate(plain):
        bm = [x.cpu().numpy().view(np.uint64) for x in B.records(outs, i)]
        pm = [x.cpu().numpy().view(np.uint64) for x in o]
        diff = np.zeros(bm[0].shape[1], np.uint64)
        for x, y in zip(bm, pm):
            if x.size:
                diff |= np.bitwise_or.reduce(x ^ y, axis=0)
        differing += int(sum(bin(int(v)).count("1") for v in diff))
    cost = [p.cost_model(precision) for p in progs]
    # every batched vector is in HBM; each program's bytes for the tier it runs on
    tiers = B.threads_per_shot
    vec_bytes = sum(c["vector_bytes_fused" if g == 1 else "vector_bytes_fused_group"] * n
                    for c, n, g in zip(cost, shots, tiers))
    table_bytes = sum(c["vector_bytes"] * n for c, n in zip(cost, shots))
    achieved = vec_bytes / (kernel_ms * 1e-3)
    line = {
        "metric": METRIC, "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": precision, "data": "synthetic",
        "config": {"workload": args.workload, "circuits": len(texts), "shots_per_circuit": shots[0],
                   "k_max": [p.k_max for p in progs], "threads_per_shot": B.threads_per_shot,
                   "graph": not args.no_graph, "parallelism": "all circuits in one persistent launch"},
        "fp64_plain": {"value": total / plain_s, "unit": "shots/s", "ms": plain_s * 1e3,
                       "speedup_of_fp32_batched": value / (total / plain_s),
                       "records_differing_shots": differing, "records_total_shots": total},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM, "work_model": "fused passes",
                     "unfused_table": {"achieved": table_bytes / (kernel_ms * 1e-3) / 1e9,
                                       "frac": table_bytes / (kernel_ms * 1e-3) / PEAK_HBM},
                     "traffic": None, "kernel_ms": kernel_ms},
    }
    add_measured_peak(line["roofline"], pk, torch)
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="surface_d3_r3")
    ap.add_argument("--precision", default=None, help="f32 or f64 (default: the workload's)")
    ap.add_argument("--threads-per-shot", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--vector-in-hbm", type=int, default=0, choices=(-1, 0, 1),
                    help="1 active vectors in HBM, -1 on chip, 0 automatic")
    ap.add_argument("--specialize", type=int, default=0, choices=(-1, 0, 1),
                    help="bit-sliced tier: 1 the program-specialized kernel, -1 the interpreter, 0 automatic")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="skip clifft_autotune before timing")
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying a captured graph")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="run one plain device copy of this many bytes first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (shards would run "
              "independent shot ranges keyed by the global shot index); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_27058_amd as pk
    from paper_2604_27058_amd import circuits

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    w = circuits.workload(args.workload)
    precision = args.precision or w["precision"]
    shots = w["shots"]
    seed = 0
    if len(w["texts"]) != 1:
        bench_batch(args, w, pk, torch)
        return
    text = w["texts"][0]
    prog = pk.Program(text)
    tuned = None
    explicit = args.threads_per_shot or args.grid or args.vector_in_hbm or args.specialize
    if not args.no_autotune and not explicit:
        tuned = prog.autotune(shots, precision)
    if args.specialize == 1:
        prog.specialize()
    launch = pk.make_launch(precision, threads_per_shot=args.threads_per_shot, grid=args.grid,
                            vector_in_hbm=args.vector_in_hbm, specialize=args.specialize)
    outs = prog.alloc_outputs(shots)
    ws = prog.alloc_workspace(launch)
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:
        src = torch.empty(args.calibrate_copy // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    step = lambda: prog.sample(shots, seed=seed, launch=launch, outputs=outs, workspace=ws)
    if not args.no_graph:
        step, graph = captured(step, torch)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = sum(a.elapsed_time(b) for a, b in evs) / len(evs)
    ms_per_step = wall * 1e3 / args.steps
    value = shots * args.steps / wall

    cost = prog.cost_model(precision)
    k = prog.k_max
    shape = prog.resolve_launch(shots, launch)
    bit_sliced = shape["threads_per_shot"] < 0
    if k == 0 and bit_sliced:
        # algorithmic work of the bit-sliced form: frame words shared by 32
        # shots, every per-shot draw and outcome bit counted in full
        achieved = cost["int_ops_bitsliced"] * shots / (kernel_ms * 1e-3)
        table = cost["int_ops"] * shots / (kernel_ms * 1e-3)
        roof = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_INT_OPS / 1e12, unit="Tops/s",
                    frac=achieved / PEAK_INT_OPS, work_model="bit-sliced",
                    int_ops_per_shot=round(cost["int_ops_bitsliced"], 3),
                    per_shot_table=dict(int_ops_per_shot=round(cost["int_ops"], 3), achieved=table / 1e12,
                                        frac=table / PEAK_INT_OPS))
    elif k == 0:
        achieved = cost["int_ops"] * shots / (kernel_ms * 1e-3)
        roof = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_INT_OPS / 1e12, unit="Tops/s",
                    frac=achieved / PEAK_INT_OPS, work_model="per-shot table")
    elif shape["vector_in_hbm"] == 1:
        # bytes the fused passes move (folded localization passes, deferred
        # expansions, carried branch sums); the unfused per-instruction table
        # beside it
        fused_key = "vector_bytes_fused" if shape["threads_per_shot"] == 1 else "vector_bytes_fused_group"
        achieved = cost[fused_key] * shots / (kernel_ms * 1e-3)
        table = cost["vector_bytes"] * shots / (kernel_ms * 1e-3)
        roof = dict(bound="hbm", achieved=achieved / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s", frac=achieved / PEAK_HBM,
                    work_model="fused passes", bytes_per_shot=round(cost[fused_key], 1),
                    unfused_table=dict(bytes_per_shot=round(cost["vector_bytes"], 1), achieved=table / 1e9,
                                       frac=table / PEAK_HBM))
    else:
        achieved = cost["vector_bytes"] * shots / (kernel_ms * 1e-3)
        roof = dict(bound="lds", achieved=achieved / 1e9, peak=PEAK_LDS / 1e9, unit="GB/s", frac=achieved / PEAK_LDS)
    roof["kernel"] = ("clifft_frames_spec" if shape["specialize"] == 1 else "k_frames") if bit_sliced else "k_sample"
    traffic = load_traffic(args.workload, precision, roof["kernel"])
    roof["traffic"] = traffic
    if traffic:
        vb = cost[fused_key] if shape["vector_in_hbm"] == 1 else cost["vector_bytes"]
        roof["traffic_over_algorithmic"] = traffic / max(1.0, (vb + cost["record_bytes"]) * shots)
    roof["kernel_ms"] = kernel_ms
    roof["work_per_shot"] = {kk: round(v, 3) for kk, v in cost.items()}
    add_measured_peak(roof, pk, torch)

    line = {
        "metric": METRIC, "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64" if k == 0 else precision, "data": "synthetic",
        "config": {"workload": args.workload, "shots": shots, "qubits": prog.num_qubits, "k_max": k,
                   "detectors": prog.num_detectors, "noise_sites": prog.num_noise_sites,
                   "precision": precision, "threads_per_shot": shape["threads_per_shot"],
                   "vector_in_hbm": shape["vector_in_hbm"] == 1, "grid": shape["grid"],
                   "specialized": shape["specialize"] == 1, "autotuned": tuned is not None,
                   "graph": not args.no_graph,
                   "parallelism": "shots across lanes/waves of one GPU"},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        import numpy as np
        cb, (n, om, od, oo) = cpu_baseline(text, shots, seed)
        line["cpu_baseline"] = cb
        # records of the sampled shots must equal the oracle's
        words = (n + 63) // 64
        gm = outs[0][:, :words].cpu().numpy().view(np.uint64)
        gd = outs[1][:, :words].cpu().numpy().view(np.uint64)
        go = outs[2][:, :words].cpu().numpy().view(np.uint64)
        diff = np.zeros(words, np.uint64)
        for g, o in ((gm, om), (gd, od), (go, oo)):
            if g.size:
                diff |= np.bitwise_or.reduce(g ^ o, axis=0)
        line["cpu_baseline"]["gpu_records_differing_on_sample"] = int(
            sum(bin(int(x)).count("1") for x in diff))
    print(json.dumps(line))


if __name__ == "__main__":
    main()
