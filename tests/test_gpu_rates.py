"""Rate-level and full-size agreement of the HIP path with the FP64 oracle.

The paper validates its sampler by comparing marginals within binomial
bounds (Section 3.3, Validation).  Here every measurement, detector and
observable rate of the GPU path at full shot count is tested against the
oracle with a two-sample 5-sigma binomial test, on the d = 5 + 10 T surface
code and on the benchmark's own 64-circuit batched set.  The forced-outcome
checks of the k = 20 stress program compare every branch probability and
the 2^20-amplitude vector with the oracle at the stated tolerances.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_2604_27058_amd as pk
from paper_2604_27058_amd import circuits
from stats import popcount_rows, two_sample_ok

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    yield


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def host_threads():
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def failing_rows(gpu_rows, n_gpu, ora_rows, n_ora, gpu_first=0):
    """Rows whose rates differ by more than 5 sigma (two-sample binomial).
    gpu_first: the GPU sample starts at this shot (so that it is disjoint
    from an oracle prefix drawn with the same seed)."""
    bad = []
    for g, o in zip(gpu_rows, ora_rows):
        if o.size == 0:
            continue
        if gpu_first:
            assert gpu_first % 64 == 0
            g = g[:, gpu_first // 64:]
        kg = popcount_rows(g, n_gpu)
        ko = popcount_rows(o, n_ora)
        for r in range(len(kg)):
            if not two_sample_ok(int(kg[r]), n_gpu, int(ko[r]), n_ora):
                bad.append((r, int(kg[r]) / n_gpu, int(ko[r]) / n_ora))
    return bad


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_rates_5sigma_surface_d5_t10_full(precision):
    """1e6 shots of the d = 5 + 10 T workload on the GPU (default launch)
    against 1e6 oracle shots of another seed: every one of the 145
    measurement, 120 detector and 1 observable rates within 5 sigma."""
    text = circuits.workload("surface_d5_r5_t10")["texts"][0]
    shots = 1_000_000
    gp = pk.Program(text)
    outs = gp.sample(shots, seed=200, launch=pk.make_launch(precision))
    torch.cuda.synchronize()
    g = [u64(x) for x in outs]
    o = oracle.Program(text).sample(shots, seed=100, threads=host_threads())
    bad = failing_rows(g, shots, o, shots)
    print("rows failing 5 sigma:", bad)
    assert not bad


def test_rates_5sigma_batched64_bench_set():
    """The benchmark's own 64 circuits (1e5 shots each, seed = circuit index)
    through the FP32 batched launch: every record rate of every circuit,
    shots 2048..1e5 (disjoint from the prefix), against a 2048-shot oracle
    prefix of the same seed; the FP64 plain form equals the oracle bit for
    bit on that prefix."""
    w = circuits.workload("batched64")
    texts = w["texts"]
    n = len(texts)
    shots = [w["shots"]] * n
    seeds = list(range(n))
    progs = [pk.Program(t) for t in texts]
    B = pk.Batch(progs, shots, seeds, precision="f32")
    outs = B.sample()
    torch.cuda.synchronize()
    pre = 2048
    L64 = pk.make_launch("f64")
    total_rows = 0
    bad_all = []
    for i, (t, p) in enumerate(zip(texts, progs)):
        o = oracle.Program(t).sample(pre, seed=seeds[i], threads=host_threads())
        g = [u64(x) for x in B.records(outs, i)]
        bad = failing_rows(g, shots[i] - pre, o, pre, gpu_first=pre)
        total_rows += sum(x.shape[0] for x in o)
        bad_all += [(i,) + b for b in bad]
        m64, d64, b64 = p.sample(pre, seed=seeds[i], launch=L64)
        torch.cuda.synchronize()
        for a, b in zip((u64(m64), u64(d64), u64(b64)), o):
            assert np.array_equal(a, b), "FP64 plain records differ from the oracle (circuit %d)" % i
    print("rows tested: %d; failing 5 sigma: %s" % (total_rows, bad_all))
    assert total_rows > 3000
    assert not bad_all


def _large_active_without_final_measurement():
    """The k = 20 stress program up to its final measurement (final k = 20)."""
    lines = circuits.workload("large_active_k20")["texts"][0].splitlines()
    while lines and (lines[-1].startswith("M ") or lines[-1].startswith("X_ERROR")):
        lines.pop()
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-5)])
def test_forced_k20_full_program(precision, tol):
    """One forced shot of the full k = 20 program (its own faults and
    outcomes from the oracle) on the shot-per-workgroup tier with vectors in
    HBM: every branch probability of its mid-circuit measurements, and the
    final 2^20-amplitude vector, within the stated relative tolerance."""
    import test_gpu_parity as tp
    text = _large_active_without_final_measurement()
    op = oracle.Program(text)
    gp = pk.Program(text)
    assert op.kmax == 20 and gp.k_max == 20
    faults = op.faults(17, 0)
    t0 = op.trace(17, 0, forced_faults=faults)
    t = op.trace(17, 0, forced_m=t0["m"], forced_faults=faults)
    assert t["error"] == 0 and t["k"] == 20
    fm = np.asarray(t["m"], np.uint32)[None, :]
    ff = np.asarray(faults, np.int32)[None, :]
    res = gp.sample_trace(1, seed=17, launch=pk.make_launch(precision, 256, vector_in_hbm=1),
                          forced_m=torch.from_numpy(fm), forced_faults=torch.from_numpy(ff))
    torch.cuda.synchronize()
    probs = res["probs"].cpu().numpy()[0]
    m = fm[0].astype(bool)
    pg = np.where(m, probs, 1.0 - probs)
    po = np.where(m, t["probs"], 1.0 - np.asarray(t["probs"]))
    worst_p = float(np.max(np.abs(pg - po) / po))
    phi = res["phi"].cpu().numpy()[0]
    gam = res["gamma"].cpu().numpy()[0]
    worst_v = tp._state_error(phi, gam, gp.final_slots(), t)
    print("k = 20 %s: worst relative probability error %.3g, vector error %.3g" % (precision, worst_p, worst_v))
    assert worst_p <= tol and worst_v <= tol
