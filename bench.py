#!/usr/bin/env python3
"""Benchmark of the sample-many path on one MI355X.

Default workload (the headline): 64 seeded heterogeneous near-Clifford
circuits (20-100 qubits, peak active dimension 4-16, 1e5 shots each).  A
step samples every shot of every circuit with the FP32 batched launch
(amplitudes FP32, reductions and renormalisation FP64); the plain form, one
FP64 clifft_sample call per circuit, is timed the same way beside it, and
both are checked against the FP64 oracle rate by rate (matched accuracy).
Programs are resident and outputs preallocated; steps replay a captured HIP
graph (--no-graph: launched eagerly).  Prints one JSON line.

Single-program workloads (--workload): one clifft_sample call over the
workload's shots per step, reported under their own metric name.
--postselect all post-selects every detector (shots end at their first
firing detector) and --faults R samples the stratum of exactly R faults
(clifft_sample_stratified); either way the plain form of the same program
is timed beside it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shots/sec at matched detector-rate accuracy, FP32-batched vs FP64-plain"
# single-program workloads are reported under their own name
METRIC_SINGLE = "shots/sec, one program per call (%s, %s)"
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


def cpu_baseline(text, shots_hint, seed, postselect=None, faults=None):
    """The FP64 oracle timed on the host cores on a bounded sample."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    prog = oracle.Program(text, postselect=postselect)
    n = 4096
    t0 = time.perf_counter()
    prog.sample(n, seed=seed, threads=threads, faults=faults)
    dt = time.perf_counter() - t0
    # scale the sample to about 10 s of CPU time, within the workload's shots
    target = min(shots_hint, max(64, int(n * 10.0 / max(dt, 1e-6))))
    target = (target + 63) // 64 * 64
    t0 = time.perf_counter()
    meas, det, obs = prog.sample(target, seed=seed, threads=threads, faults=faults)
    dt = time.perf_counter() - t0
    return dict(value=target / dt, unit="shots/s", cores=threads, cpu_model=cpu_model(), kind="oracle",
                sample="first %d shots of the workload (seed %d), FP64 oracle, %d threads, %.1f s"
                       % (target, seed, threads, dt)), (target, meas, det, obs)


def calibration_copy(nbytes, torch):
    """One plain device copy of nbytes (the HBM counters' calibration)."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


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


def time_steps(fn, steps, warmup, torch, graph=True):
    """The driver's timing contract for one form: `warmup` untimed calls,
    then exactly `steps` calls bracketed by device synchronisations, each also
    bracketed by HIP events on the launch stream.  Returns (wall seconds of
    the timed calls, per-step event times in ms, graph handle)."""
    g = None
    if graph:
        fn, g = captured(fn, torch)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in evs], g


def progress(msg):
    """One progress line on stderr (the JSON result alone goes to stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def median(xs):
    s = sorted(xs)
    n = len(s)
    return s[n // 2] if n % 2 else 0.5 * (s[n // 2 - 1] + s[n // 2])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def row_counts(words, shots):
    """Set bits per row of a record-major bit-packed array (first `shots` shots)."""
    import numpy as np
    w = np.ascontiguousarray(words, dtype=np.uint64)
    if w.size == 0:
        return np.zeros(w.shape[0], np.int64)
    nw = (shots + 63) // 64
    w = w[:, :nw].copy()
    rem = shots % 64
    if rem:
        w[:, -1] &= np.uint64((1 << rem) - 1)
    return np.unpackbits(w.view(np.uint8), axis=1).sum(axis=1).astype(np.int64)


def two_sample_5sigma(k1, n1, k2, n2, nsig=5.0):
    """Two-sample binomial test with pooled variance: per-row booleans."""
    import numpy as np
    k1, k2 = np.asarray(k1, float), np.asarray(k2, float)
    p = (k1 + k2) / (n1 + n2)
    sd = np.sqrt(np.maximum(p * (1 - p), 1e-300) * (1.0 / n1 + 1.0 / n2))
    return np.abs(k1 / n1 - k2 / n2) <= nsig * sd + 1.0 / min(n1, n2)


def differing_shots(a, b, shots):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    if a.size == 0:
        return 0
    nw = (shots + 63) // 64
    d = np.bitwise_or.reduce(a[:, :nw] ^ b[:, :nw], axis=0)
    rem = shots % 64
    if rem:
        d[-1] &= np.uint64((1 << rem) - 1)
    return int(np.unpackbits(d.view(np.uint8)).sum())


def bench_batch(args, w, pk, torch):
    """The headline comparison: every circuit of the set sampled by the
    batched launch in FP32 (amplitudes FP32; branch sums, renormalisation
    factors and rotation constants FP64) against the plain form, one FP64
    clifft_sample call per circuit, on the same GPU.  Both forms are timed
    the same way (captured graph, warm-up, `steps` timed replays).  Matched
    accuracy: every measurement, detector and observable rate of both forms
    passes a two-sample 5-sigma binomial test against the oracle on a prefix
    of each circuit's shots, and against each other at full size."""
    import numpy as np
    texts = w["texts"]
    n = len(texts)
    shots = [w["shots"]] * n
    seeds = list(range(n))
    progs = [pk.Program(t) for t in texts]
    total = sum(shots)
    if args.calibrate_copy:
        calibration_copy(args.calibrate_copy, torch)
    tuned = False
    t_tune = time.perf_counter()
    if not args.no_autotune and not args.threads_per_shot:
        for i, (p, s) in enumerate(zip(progs, shots)):
            # the plain FP64 form's per-program shapes (the batched launch
            # places programs by its own k_max rule)
            p.autotune(s, "f64")
            if i % 16 == 15:
                progress("autotuned %d of %d circuits (%.0f s)" % (i + 1, n, time.perf_counter() - t_tune))
        tuned = True
    tune_s = time.perf_counter() - t_tune
    graph = not args.no_graph

    # FP32, all circuits in one batched launch
    B = pk.Batch(progs, shots, seeds, precision="f32", threads_per_shot=args.threads_per_shot, grid=args.grid)
    outs, ws = B.alloc()
    wall32, ev32, g32 = time_steps(lambda: B.sample(outs, ws), args.steps, args.warmup, torch, graph)
    med32 = median(ev32)
    value = total * args.steps / wall32
    progress("FP32 batched: %.1f ms per step (median)" % med32)

    # FP64 plain: one call per circuit, in order, sharing one workspace
    L64 = pk.make_launch("f64")
    plain_outs = [p.alloc_outputs(s) for p, s in zip(progs, shots)]
    ws64_bytes = max(p.workspace_size(L64, s) for p, s in zip(progs, shots))
    ws64 = torch.empty(max(ws64_bytes, 1), dtype=torch.uint8, device="cuda") if ws64_bytes else None

    def plain_step():
        for i, p in enumerate(progs):
            p.sample(shots[i], seed=seeds[i], launch=L64, outputs=plain_outs[i], workspace=ws64)

    wall64, ev64, g64 = time_steps(plain_step, args.steps, args.warmup, torch, graph)
    med64 = median(ev64)
    value64 = total * args.steps / wall64
    progress("FP64 plain: %.1f ms per step (median)" % med64)
    torch.cuda.synchronize()

    rec32 = [[x.cpu().numpy().view(np.uint64) for x in B.records(outs, i)] for i in range(n)]
    rec64 = [[x.cpu().numpy().view(np.uint64) for x in o] for o in plain_outs]

    cost = [p.cost_model("f32") for p in progs]
    tiers = B.threads_per_shot
    vec_bytes = sum(c["vector_bytes_fused" if g == 1 else "vector_bytes_fused_batch"] * s
                    for c, s, g in zip(cost, shots, tiers))
    rec_bytes = sum(c["record_bytes"] * s for c, s in zip(cost, shots))
    table_bytes = sum(c["vector_bytes"] * s for c, s in zip(cost, shots))
    achieved = vec_bytes / (med32 * 1e-3)
    roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": achieved / PEAK_HBM, "kernel": "k_batch (the batched step: its queue kernels in order)",
            "work_model": "fused passes", "bytes_per_step": vec_bytes,
            "unfused_table": {"bytes_per_step": table_bytes, "achieved": table_bytes / (med32 * 1e-3) / 1e9,
                              "frac": table_bytes / (med32 * 1e-3) / PEAK_HBM},
            "kernel_ms": med32}
    traffic = load_traffic(args.workload, "f32", "k_batch")
    roof["traffic"] = traffic
    if traffic:
        roof["traffic_over_algorithmic"] = traffic / max(1.0, vec_bytes + rec_bytes)
    add_measured_peak(roof, pk, torch)

    line = {
        "metric": METRIC, "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall32 * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "circuits": n, "shots_per_circuit": shots[0],
                   "qubits": [p.num_qubits for p in progs], "k_max": [p.k_max for p in progs],
                   "threads_per_shot": tiers, "graph": graph, "autotuned": tuned,
                   "autotune_s": round(tune_s, 2),
                   "parallelism": "all circuits in one batched launch (shot-parallel on one GPU)"},
        "ms_median": med32,
        "fp64_plain": {"value": value64, "unit": "shots/s", "ms_per_step": wall64 * 1e3 / args.steps,
                       "ms_median": med64, "timing": "same as the FP32 form (graph replay, warm-up, steps)",
                       "speedup_of_fp32_batched": value / value64},
        "roofline": roof,
    }
    # agreement of the two GPU forms at full size
    rows_3264 = fails_3264 = diff_3264 = 0
    for i in range(n):
        for a, b in zip(rec32[i], rec64[i]):
            if a.size == 0:
                continue
            ok = two_sample_5sigma(row_counts(a, shots[i]), shots[i], row_counts(b, shots[i]), shots[i])
            rows_3264 += len(ok)
            fails_3264 += int((~ok).sum())
        diff_3264 += differing_shots(np.vstack([x for x in rec32[i] if x.size]),
                                     np.vstack([x for x in rec64[i] if x.size]), shots[i])
    line["fp64_plain"]["rates_5sigma_vs_fp32"] = {"rows": rows_3264, "failing": fails_3264}
    line["fp64_plain"]["records_differing_shots"] = diff_3264
    line["fp64_plain"]["records_total_shots"] = total
    if not args.no_cpu_baseline:
        cb = cpu_baseline_batch(texts, shots, seeds, rec32, rec64)
        line["cpu_baseline"] = cb
        line["matched_accuracy"] = (cb["rates_5sigma"]["fp32_batched"]["failing"] == 0
                                    and cb["rates_5sigma"]["fp64_plain"]["failing"] == 0 and fails_3264 == 0)
    print(json.dumps(line))


def cpu_baseline_batch(texts, shots, seeds, rec32, rec64, budget_s=15.0):
    """The FP64 oracle on the host cores, on the same prefix of every
    circuit's shots (sized from a short calibration run to about `budget_s`
    seconds); its rates test both GPU forms (two-sample 5 sigma per row), and
    its records equal the FP64 plain form's on the prefix."""
    import numpy as np
    import oracle
    threads = host_threads()
    oprogs = [oracle.Program(t) for t in texts]
    t0 = time.perf_counter()
    for p, sd in zip(oprogs, seeds):
        p.sample(64, seed=sd, threads=threads)
    cal = time.perf_counter() - t0  # one 64-shot range per circuit, one thread each
    per = int(64 * budget_s * threads / max(cal, 1e-6))
    per = max(64, min(min(shots), per // 64 * 64))
    progress("oracle prefix: %d shots per circuit" % per)
    t0 = time.perf_counter()
    orec = []
    for p, sd in zip(oprogs, seeds):
        orec.append(p.sample(per, seed=sd, threads=threads))
    dt = time.perf_counter() - t0
    res = {}
    for name, recs in (("fp32_batched", rec32), ("fp64_plain", rec64)):
        rows = fails = 0
        for i, (o, g) in enumerate(zip(orec, recs)):
            for a, b in zip(o, g):
                if a.size == 0:
                    continue
                ok = two_sample_5sigma(row_counts(b, shots[i]), shots[i], row_counts(a, per), per)
                rows += len(ok)
                fails += int((~ok).sum())
        res[name] = {"rows": rows, "failing": fails}
    diff64 = sum(differing_shots(np.vstack([x for x in o if x.size]), np.vstack([x for x in g if x.size]), per)
                 for o, g in zip(orec, rec64))
    diff32 = sum(differing_shots(np.vstack([x for x in o if x.size]), np.vstack([x for x in g if x.size]), per)
                 for o, g in zip(orec, rec32))
    return dict(value=per * len(texts) / dt, unit="shots/s", cores=threads, cpu_model=cpu_model(), kind="oracle",
                sample="first %d shots of each of the %d circuits (seed = circuit index), FP64 oracle, %d threads, "
                       "%.1f s" % (per, len(texts), threads, dt),
                rates_5sigma=res, prefix_shots_per_circuit=per,
                records_differing_on_prefix={"fp64_plain": diff64, "fp32_batched": diff32})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched64")
    ap.add_argument("--precision", default=None, help="f32 or f64 (default: the workload's)")
    ap.add_argument("--threads-per-shot", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--vector-in-hbm", type=int, default=0, choices=(-1, 0, 1),
                    help="1 active vectors in HBM, -1 on chip, 0 automatic")
    ap.add_argument("--specialize", type=int, default=0, choices=(-1, 0, 1),
                    help="bit-sliced tier: 1 the program-specialized kernel, -1 the interpreter, 0 automatic")
    ap.add_argument("--split", type=int, default=0, choices=(-1, 0, 1, 2, 3),
                    help="single-program workloads: clifft_launch.split (the split form's frame pass)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--postselect", default="none", choices=("none", "all"),
                    help="single-program workloads: post-select every detector")
    ap.add_argument("--faults", type=int, default=-1,
                    help="single-program workloads: sample the stratum of exactly this many faults")
    ap.add_argument("--no-autotune", action="store_true", help="skip clifft_autotune before timing")
    ap.add_argument("--no-graph", action="store_true", help="launch eagerly instead of replaying a captured graph")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="run one plain device copy of this many bytes first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (shards would run "
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
    post = None if args.postselect == "none" else "all"
    faults = args.faults if args.faults >= 0 else None
    prog = pk.Program(text, postselect=post)
    tuned = None
    explicit = args.threads_per_shot or args.grid or args.vector_in_hbm or args.specialize or args.split
    if not args.no_autotune and not explicit:
        tuned = prog.autotune(shots, precision)
    if args.specialize == 1:
        prog.specialize()
    launch = pk.make_launch(precision, threads_per_shot=args.threads_per_shot, grid=args.grid,
                            vector_in_hbm=args.vector_in_hbm, specialize=args.specialize, split=args.split)
    outs = prog.alloc_outputs(shots)
    ws = prog.alloc_workspace(launch, shots=shots)
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:
        calibration_copy(args.calibrate_copy, torch)
    if faults is None:
        step = lambda: prog.sample(shots, seed=seed, launch=launch, outputs=outs, workspace=ws)
    else:
        step = lambda: prog.sample_stratified(shots, faults, seed=seed, launch=launch, outputs=outs, workspace=ws)
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
    if post:
        roof["note"] = "work model counts every instruction of every shot; rejected shots skip their tail"
    add_measured_peak(roof, pk, torch)

    variant = ""
    if post:
        variant += ", every detector post-selected"
    if faults is not None:
        variant += ", stratum of %d faults" % faults
    line = {
        "metric": METRIC_SINGLE % (args.workload + variant, "u64 frames" if k == 0 else precision), "value": value,
        "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
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
    if post or faults is not None:
        import numpy as np
        if post:
            words = (shots + 63) // 64
            d = outs[1].cpu().numpy().view(np.uint64)
            rej = np.bitwise_or.reduce(d, axis=0) if d.size else np.zeros(words, np.uint64)
            nrej = sum(bin(int(x)).count("1") for x in rej)
            line["config"]["kept_fraction"] = 1.0 - nrej / shots
        if faults is not None:
            line["config"]["stratum_weight"] = prog.fault_count_pmf(faults)[faults]
        # the same program sampled plainly (no post-selection, no stratum),
        # same launch and timing
        plain = pk.Program(text)
        if tuned is not None:
            plain.autotune(shots, precision)
        pouts = plain.alloc_outputs(shots)
        pws = plain.alloc_workspace(launch, shots=shots)
        pstep = lambda: plain.sample(shots, seed=seed, launch=launch, outputs=pouts, workspace=pws)
        pwall, pev, _ = time_steps(pstep, args.steps, args.warmup, torch, graph=not args.no_graph)
        line["plain_form"] = {"value": shots * args.steps / pwall, "unit": "shots/s",
                              "kernel_ms": sum(pev) / len(pev),
                              "speedup": (shots * args.steps / wall) / (shots * args.steps / pwall)}
    if not args.no_cpu_baseline:
        import numpy as np
        cb, (n, om, od, oo) = cpu_baseline(text, shots, seed, postselect=post, faults=faults)
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
