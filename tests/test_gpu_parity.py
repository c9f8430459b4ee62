"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on
the same seeded inputs.

Bar: records bit-exact for Pauli-frame-only circuits; with FP64 amplitudes
records bit-exact on every circuit (the only possible difference is a
uniform draw falling between two probabilities that differ by rounding);
with FP32 amplitudes records identical except for such near-threshold
shots, bounded from the measured FP32-FP64 probability gap.  On
forced-outcome shots the probability of every forced outcome is within
1e-12 (FP64) or 2e-5 (FP32) relative, and gamma * phi (the global scalar
times the final active vector, after slot permutation only) within the same
tolerance relative to its norm.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_2604_27058_amd as pk
from paper_2604_27058_amd import circuits
from test_oracle_pins import random_small_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    yield


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def gpu_sample(text_or_prog, shots, seed=0, offset=0, **launch):
    p = text_or_prog if isinstance(text_or_prog, pk.Program) else pk.Program(text_or_prog)
    L = pk.make_launch(**launch) if launch else None
    # outputs start as garbage so that unwritten words are caught
    outs = tuple(x.fill_(-1) for x in p.alloc_outputs(shots))
    m, d, o = p.sample(shots, seed=seed, offset=offset, launch=L, outputs=outs)
    torch.cuda.synchronize()
    return u64(m), u64(d), u64(o)


def mismatched_shots(a, b, shots):
    """Shots whose records differ between two record-major bit arrays."""
    if a.size == 0:
        return 0
    diff = np.bitwise_or.reduce(a ^ b, axis=0)
    return int(sum(bin(int(w)).count("1") for w in diff))


def fp32_mismatch_bound(text, shots, seed=0, sample_shots=64, tail=1e-6, safety=4.0, forms=1):
    """Upper bound on the number of shots, out of `shots`, whose FP32
    records may differ from the FP64 (oracle) ones.  A record differs only
    when a measurement's uniform falls between its FP32 and FP64
    probabilities, so the expected count is the sum over shots and events of
    |P32 - P64| along a common trajectory.  That gap is measured on oracle
    trajectories forced onto the FP32 path (`sample_shots` of them), scaled
    to `shots` with a safety factor (and by `forms` when two FP32 forms are
    compared with each other), and the bound is the Poisson quantile of that
    mean at tail probability `tail`."""
    from scipy.stats import poisson
    op = oracle.Program(text)
    if op.nevents == 0:
        return 0
    gp = pk.Program(text)
    fm = np.zeros((sample_shots, op.nevents), np.uint32)
    ff = np.full((sample_shots, max(op.nsites, 1)), -1, np.int32)
    po = np.zeros((sample_shots, op.nevents))
    for s in range(sample_shots):
        faults = op.faults(seed, s)
        t = op.trace(seed, s, forced_faults=faults)
        fm[s] = t["m"]
        ff[s, : op.nsites] = faults
        po[s] = t["probs"]
    res = gp.sample_trace(sample_shots, seed=seed, launch=pk.make_launch("f32"), forced_m=torch.from_numpy(fm),
                          forced_faults=torch.from_numpy(ff[:, : op.nsites]), want_phi=False)
    torch.cuda.synchronize()
    gap = float(np.abs(res["probs"].cpu().numpy() - po).sum(axis=1).mean())
    mu = safety * forms * shots * gap
    return int(poisson.isf(tail, mu)) + 1 if mu > 0 else 0


def test_in_tree_library_is_the_one_loaded():
    gpu_sample(circuits.surface_code_memory(3, 1, 1e-3), 64)
    maps = open("/proc/self/maps").read()
    assert pk.LIB_PATH in maps


@pytest.mark.parametrize("G", [1, 64, 256, -32])
def test_surface_d3_bit_exact(G):
    text = circuits.workload("surface_d3_r3")["texts"][0]
    shots = 20000 + 37  # ragged last tile
    om, od, oo = oracle.Program(text).sample(shots, seed=11, threads=8)
    gm, gd, go = gpu_sample(text, shots, seed=11, threads_per_shot=G)
    assert np.array_equal(gm, om)
    assert np.array_equal(gd, od)
    assert np.array_equal(go, oo)


@pytest.mark.parametrize("G", [1, -32])
def test_surface_d3_high_noise_bit_exact_multi_chunk(G):
    # many faults per shot and more than one 4096-site survival chunk
    text = circuits.surface_code_memory(3, 120, 2e-2)
    p = oracle.Program(text)
    assert p.nchunks >= 2
    shots = 3000
    om, od, oo = p.sample(shots, seed=5, threads=8)
    gm, gd, go = gpu_sample(text, shots, seed=5, threads_per_shot=G)
    assert np.array_equal(gm, om) and np.array_equal(gd, od) and np.array_equal(go, oo)


@pytest.mark.parametrize("case", range(12))
def test_bit_sliced_frames_random_clifford_circuits(case):
    """Pauli-frame-only random circuits (W = 1..3 words, all noise types, MX,
    resets, detectors, observables included twice) on the bit-sliced tier."""
    rng = np.random.default_rng(1300 + case)
    n = [5, 70, 100, 30][case % 4]
    text = random_small_circuit(rng, n, 120, rotations=False)
    text += "OBSERVABLE_INCLUDE(1) rec[-1] rec[-2]\nOBSERVABLE_INCLUDE(1) rec[-1]\n"
    shots = 5000 + 13 * case
    om, od, oo = oracle.Program(text).sample(shots, seed=case, threads=8)
    gm, gd, go = gpu_sample(text, shots, seed=case, threads_per_shot=-32)
    assert np.array_equal(gm, om) and np.array_equal(gd, od) and np.array_equal(go, oo)


@pytest.mark.parametrize("G", [1, -32])
def test_shard_resume_bit_identical_gpu(G):
    text = circuits.surface_code_memory(3, 3, 1e-2)
    a = gpu_sample(text, 4096, seed=5, threads_per_shot=G)
    b = gpu_sample(text, 2048, seed=5, offset=0, threads_per_shot=G)
    c = gpu_sample(text, 2048, seed=5, offset=2048, threads_per_shot=G)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, np.concatenate([y, z], axis=1))


@pytest.mark.parametrize("G", [1, 64, 256])
def test_shard_resume_active_hbm_fp64(G):
    """Shards of an active-vector program on the HBM tiers (the cooperative
    ones OR single shots' record bits into zero-filled rows) join into the
    unsharded records bit for bit, and equal the oracle's."""
    text = circuits.workload("random_clifford_t_n8")["texts"][0]
    a = gpu_sample(text, 4096, seed=9, precision="f64", threads_per_shot=G, vector_in_hbm=1)
    b = gpu_sample(text, 2048, seed=9, offset=0, precision="f64", threads_per_shot=G, vector_in_hbm=1)
    c = gpu_sample(text, 2048, seed=9, offset=2048, precision="f64", threads_per_shot=G, vector_in_hbm=1)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, np.concatenate([y, z], axis=1))
    om, _, _ = oracle.Program(text).sample(4096, seed=9, threads=8)
    assert np.array_equal(a[0], om)


@pytest.mark.parametrize("case", range(16))
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_random_circuits_records(case, precision):
    rng = np.random.default_rng(100 + case)
    n = int(rng.integers(2, 6))
    text = random_small_circuit(rng, n, int(rng.integers(10, 45)))
    shots = 700
    om, od, oo = oracle.Program(text).sample(shots, seed=case, threads=4)
    gm, gd, go = gpu_sample(text, shots, seed=case, precision=precision)
    bad = mismatched_shots(np.vstack([om, od, oo]) if om.size else om, np.vstack([gm, gd, go]) if gm.size else gm,
                           shots)
    if precision == "f64":
        assert bad == 0
    else:
        assert bad <= fp32_mismatch_bound(text, shots, seed=case)


def _phi_in_oracle_order(phi_g, gslots, oslots):
    """Permute a GPU active vector (slot s holds virtual qubit gslots[s]) to
    the oracle's slot order."""
    pos = {q: t for t, q in enumerate(oslots)}
    i = np.arange(len(phi_g), dtype=np.int64)
    j = np.zeros_like(i)
    for s, q in enumerate(gslots):
        j |= ((i >> s) & 1) << pos[q]
    out = np.zeros_like(phi_g)
    out[j] = phi_g
    return out


def _state_error(phi_g, gamma_g, gslots, t):
    """Relative distance between gamma * phi of the GPU (slots permuted to
    the oracle's order) and of the oracle: the same vector of the
    frame-factored state with no phase alignment and no rescaling."""
    a = gamma_g * _phi_in_oracle_order(phi_g, gslots, list(t["slots"]))
    b = t["gamma"] * np.asarray(t["phi"])
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _forced_check(text, case, precision, tol, tier, rng):
    """Forces the faults and outcomes of oracle shots (plus extra faults) and
    compares every measurement's probability and the final vector."""
    op = oracle.Program(text)
    gp = pk.Program(text)
    shots = 8
    fm = np.zeros((shots, max(op.nevents, 1)), np.uint32)
    ff = np.full((shots, max(op.nsites, 1)), -1, np.int32)
    traces = []
    for s in range(shots):
        # force the faults and outcomes of an oracle shot (plus extra faults)
        faults = op.faults(case, s)
        for i in range(op.nsites):
            if rng.random() < 0.2:
                faults[i] = int(rng.integers(0, 1 if "ERROR" in text else 3))
        t0 = op.trace(case, s, forced_faults=faults)
        t = op.trace(case, s, forced_m=t0["m"], forced_faults=faults)
        assert t["error"] == 0
        fm[s, : op.nevents] = t["m"]
        ff[s, : op.nsites] = faults
        traces.append(t)
    L = pk.make_launch(precision) if tier is None else pk.make_launch(precision, tier[0], vector_in_hbm=tier[1])
    res = gp.sample_trace(shots, seed=case, launch=L, forced_m=torch.from_numpy(fm[:, : max(op.nevents, 0)]),
                          forced_faults=torch.from_numpy(ff[:, : max(op.nsites, 0)]))
    torch.cuda.synchronize()
    probs = res["probs"].cpu().numpy()
    phi = res["phi"].cpu().numpy()
    gam = res["gamma"].cpu().numpy()
    gslots = gp.final_slots()
    worst_p = worst_v = 0.0
    for s, t in enumerate(traces):
        if op.nevents:
            # relative error of the probability of each forced outcome
            m = fm[s, : op.nevents].astype(bool)
            pg = np.where(m, probs[s], 1.0 - probs[s])
            po = np.where(m, t["probs"], 1.0 - np.asarray(t["probs"]))
            assert (po > 0).all()
            worst_p = max(worst_p, float(np.max(np.abs(pg - po) / po)))
        k = t["k"]
        assert len(gslots) == k
        worst_v = max(worst_v, _state_error(phi[s, : 1 << k], gam[s], gslots, t))
    print("%s case %d: worst relative probability error %.3g, vector error %.3g" % (precision, case, worst_p, worst_v))
    assert worst_p <= tol and worst_v <= tol


@pytest.mark.parametrize("case", range(12))
@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-5)])
@pytest.mark.parametrize("tier", [None, (1, 1), (64, 1), (256, 1)], ids=["auto", "lane-hbm", "wave-hbm", "group-hbm"])
def test_forced_probabilities_and_amplitudes(case, precision, tol, tier):
    """Forced outcomes and faults of oracle shots: every measurement's
    probability and the final vector.  The HBM tiers collapse out of place
    through folded localization passes and deferred expansions (a Z or X
    measurement on a stored or a deferred slot)."""
    rng = np.random.default_rng(700 + case)
    n = int(rng.integers(2, 6))
    text = random_small_circuit(rng, n, int(rng.integers(10, 45))).rsplit("M ", 1)[0]  # keep the final vector
    _forced_check(text, case, precision, tol, tier, rng)


def active_rotation_circuit(rng, n, layers):
    """Every qubit expanded first (H, T), then Cliffords, rotations, noise and
    a few measurements on the active register: rotations whose generator has
    X support only on active qubits become an H pass on their pivot slot, with
    its localization passes before it and the diagonal rotation right after."""
    lines = ["H %d" % q for q in range(n)] + ["T %d" % q for q in range(n)]
    for _ in range(layers):
        q = int(rng.integers(0, n))
        r = rng.random()
        if r < 0.3:
            lines.append("%s %d" % (["H", "S", "S_DAG", "X"][int(rng.integers(0, 4))], q))
        elif r < 0.55:
            a, b = [int(v) for v in rng.choice(n, 2, replace=False)]
            lines.append("%s %d %d" % (["CX", "CZ"][int(rng.integers(0, 2))], a, b))
        elif r < 0.82:
            lines.append(["T %d" % q, "T_DAG %d" % q, "R_Z(%r) %d" % (float(rng.uniform(-3, 3)), q)][int(rng.integers(0, 3))])
        elif r < 0.9:
            lines.append("%s %d" % (["MX", "M"][int(rng.integers(0, 2))], q))
        else:
            lines.append("%s(%r) %d" % (["X_ERROR", "Z_ERROR", "DEPOLARIZE1"][int(rng.integers(0, 3))],
                                        float(rng.uniform(0.02, 0.1)), q))
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("case", range(8))
@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-5)])
@pytest.mark.parametrize("tier", [None, (1, 1), (64, 1), (256, 1)], ids=["auto", "lane-hbm", "wave-hbm", "group-hbm"])
def test_forced_active_rotations(case, precision, tol, tier):
    """H passes on active slots: on the HBM tiers they read their folded
    localization passes and apply the rotation that follows them in the same
    out-of-place pass (seeds 1300..1307 compile to several such passes)."""
    rng = np.random.default_rng(1300 + case)
    n = int(rng.integers(3, 6))
    text = active_rotation_circuit(rng, n, int(rng.integers(20, 40)))
    _forced_check(text, case, precision, tol, tier, rng)


def measurement_burst_circuit(rng, n):
    """n qubits expanded and entangled, then n - 1 of them measured one after
    another (X or Z basis, single-qubit Cliffords and Z faults between them):
    a chain of active measurements with only frame work and folded
    localization passes between consecutive ones, the case of paired
    collapses on the cooperative HBM tiers."""
    lines = ["H %d" % q for q in range(n)] + ["T %d" % q for q in range(n)]
    for _ in range(2 * n):
        a, b = [int(v) for v in rng.choice(n, 2, replace=False)]
        lines.append("%s %d %d" % (["CX", "CZ"][int(rng.integers(0, 2))], a, b))
        lines.append("%s %d" % (["T", "T_DAG", "H", "S"][int(rng.integers(0, 4))], int(rng.integers(0, n))))
    for q in [int(v) for v in rng.permutation(n)][: n - 1]:
        if rng.random() < 0.5:
            lines.append("%s %d" % (["H", "S", "S_DAG", "X", "Z"][int(rng.integers(0, 5))], q))
        if rng.random() < 0.3:
            lines.append("Z_ERROR(0.05) %d" % q)
        lines.append("%s %d" % (["MX", "M"][int(rng.integers(0, 2))], q))
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("case", range(8))
@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-5)])
@pytest.mark.parametrize("tier", [(64, 1), (256, 1), (1, 1)], ids=["wave-hbm", "group-hbm", "lane-hbm"])
def test_forced_measurement_chains(case, precision, tol, tier):
    """Chains of 5..7 active measurements (k from 6..8 down to 1): in FP64 on
    the wave and group HBM tiers consecutive measurements are sampled from
    joint branch sums and collapse in one pass (FP32 pairs only vectors of
    2^17 amplitudes or more, so here it checks the single collapses of the
    same kernels); every forced outcome's probability and the final vector
    against the oracle, as on the lane tier."""
    rng = np.random.default_rng(1500 + case)
    n = int(rng.integers(6, 9))
    _forced_check(measurement_burst_circuit(rng, n), case, precision, tol, tier, rng)


def deferred_chain_circuit(rng, n):
    """n fresh qubits expanded (H, then T or T_DAG) with at most two CX among
    them, then n - 1 of them measured one after another: the chain's first
    measurement reads four deferred expansions, so on the cooperative HBM
    tiers the first pair's sums and its double collapse go through the
    deferred phase factors."""
    lines = ["H %d" % q for q in range(n)] + ["%s %d" % (["T", "T_DAG"][int(rng.integers(0, 2))], q) for q in range(n)]
    for _ in range(int(rng.integers(0, 3))):
        a, b = [int(v) for v in rng.choice(n, 2, replace=False)]
        lines.append("CX %d %d" % (a, b))
    for q in [int(v) for v in rng.permutation(n)][: n - 1]:
        if rng.random() < 0.5:
            lines.append("%s %d" % (["S", "S_DAG", "X", "Z"][int(rng.integers(0, 4))], q))
        lines.append("%s %d" % (["MX", "M"][int(rng.integers(0, 2))], q))
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("case", range(8))
@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-5)])
@pytest.mark.parametrize("tier", [(64, 1), (256, 1)], ids=["wave-hbm", "group-hbm"])
def test_forced_deferred_measurement_chains(case, precision, tol, tier):
    """Chains whose first measurement reads deferred expansions: every forced
    outcome's probability and the final vector against the oracle."""
    rng = np.random.default_rng(1700 + case)
    n = int(rng.integers(5, 9))
    _forced_check(deferred_chain_circuit(rng, n), case, precision, tol, tier, rng)


@pytest.mark.parametrize("G,hbm", [(64, 1), (256, 1)])
def test_measurement_chains_fp64_records(G, hbm):
    """Both kinds of chain sampled freely (24 circuits each): FP64 records
    equal the oracle's."""
    for case in range(24):
        for gen, base in ((measurement_burst_circuit, 1500), (deferred_chain_circuit, 1700)):
            rng = np.random.default_rng(base + case)
            text = gen(rng, int(rng.integers(6, 9)) if base == 1500 else int(rng.integers(5, 9)))
            shots = 2000
            om, od, oo = oracle.Program(text).sample(shots, seed=case, threads=4)
            gm, gd, go = gpu_sample(text, shots, seed=case, precision="f64", threads_per_shot=G, vector_in_hbm=hbm)
            assert np.array_equal(gm, om), (gen.__name__, case)


TIERS = [(1, -1), (1, 1), (64, -1), (64, 1), (256, -1), (256, 1)]  # (threads per shot, vector in HBM)


@pytest.mark.parametrize("G,hbm", TIERS)
def test_clifford_t_n8_fp64_bit_exact(G, hbm):
    w = circuits.workload("random_clifford_t_n8")
    text = w["texts"][0]
    shots = w["shots"]
    om, _, _ = oracle.Program(text).sample(shots, seed=0, threads=8)
    gm, _, _ = gpu_sample(text, shots, seed=0, precision="f64", threads_per_shot=G, vector_in_hbm=hbm)
    assert np.array_equal(gm, om)


@pytest.mark.parametrize("G,hbm", TIERS)
def test_random_circuits_every_tier_fp64(G, hbm):
    for case in range(4):
        rng = np.random.default_rng(900 + case)
        text = random_small_circuit(rng, 5, 40)
        shots = 300
        om, od, oo = oracle.Program(text).sample(shots, seed=case, threads=4)
        gm, gd, go = gpu_sample(text, shots, seed=case, precision="f64", threads_per_shot=G, vector_in_hbm=hbm)
        assert np.array_equal(gm, om) and np.array_equal(gd, od) and np.array_equal(go, oo)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("G", [0, 64])
def test_surface_d5_t10_records(precision, G):
    text = circuits.workload("surface_d5_r5_t10")["texts"][0]
    shots = 4096 + 5
    om, od, oo = oracle.Program(text).sample(shots, seed=3, threads=8)
    gm, gd, go = gpu_sample(text, shots, seed=3, precision=precision, threads_per_shot=G)
    bad = mismatched_shots(np.vstack([om, od, oo]), np.vstack([gm, gd, go]), shots)
    if precision == "f64":
        assert bad == 0
    else:
        bound = fp32_mismatch_bound(text, shots, seed=3)
        print("FP32 shots differing: %d (bound %d)" % (bad, bound))
        assert bad <= bound


def test_large_active_k20_sampled_shots():
    text = circuits.workload("large_active_k20")["texts"][0]
    op = oracle.Program(text)
    shots = 4
    gm, _, _ = gpu_sample(text, shots, seed=0, precision="f32", threads_per_shot=256)
    om, _, _ = op.sample(shots, seed=0, threads=4)
    assert mismatched_shots(om, gm, shots) == 0


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batched_launch_matches_single_program_and_oracle(precision):
    """A heterogeneous batch (all three tiers, k_max 4..16, W = 1 and 2) in
    one launch: every program's records equal its single-program call (FP64:
    exactly; FP32: up to near-threshold shots) and, on a prefix, the oracle."""
    specs = circuits.batched_set(count=12, seed=4100)
    progs = [pk.Program(c["text"]) for c in specs]
    shots = [1000 + 37 * i for i in range(len(progs))]
    seeds = [11 + i for i in range(len(progs))]
    B = pk.Batch(progs, shots, seeds, precision=precision)
    assert set(B.threads_per_shot) == {1, 64, 256}
    outs = B.sample()
    torch.cuda.synchronize()
    for i, (c, p) in enumerate(zip(specs, progs)):
        bm = [u64(x) for x in B.records(outs, i)]
        sm = gpu_sample(p, shots[i], seed=seeds[i], precision=precision)
        bad = mismatched_shots(np.vstack([x for x in bm if x.size]), np.vstack([x for x in sm if x.size]), shots[i])
        # two FP32 forms may each differ from FP64 near a threshold
        bound = 0 if precision == "f64" else fp32_mismatch_bound(c["text"], shots[i], seed=seeds[i], forms=2)
        assert bad <= bound, (i, bad, bound)
        n = 64 if p.k_max <= 12 else 16
        om, _, _ = oracle.Program(c["text"]).sample(n, seed=seeds[i], threads=8)
        bad = mismatched_shots(om[:, :1], bm[0][:, :1] & np.uint64((1 << n) - 1 if n < 64 else ~np.uint64(0)), n)
        bound = 0 if precision == "f64" else fp32_mismatch_bound(c["text"], n, seed=seeds[i])
        assert bad <= bound, (i, bad, bound)


@pytest.mark.parametrize("cap", ["0", "1", "3"])
def test_bit_sliced_fault_list_overflow_path(cap, monkeypatch):
    """Low-noise programs precompute each lane's faults into a list; lanes
    whose faults overflow it re-draw them per block.  Shrinking the list
    forces that path; records must not change."""
    text = circuits.surface_code_memory(3, 5, 1e-3)
    shots = 40000 + 3
    om, od, oo = oracle.Program(text).sample(shots, seed=21, threads=8)
    monkeypatch.setenv("CLIFFT_FRAMES_LIST_CAP", cap)
    gm, gd, go = gpu_sample(text, shots, seed=21, threads_per_shot=-32)
    assert np.array_equal(gm, om) and np.array_equal(gd, od) and np.array_equal(go, oo)


def test_bit_sliced_multi_chunk_low_noise():
    """More than one survival chunk with the fault list (no LDS table)."""
    text = circuits.surface_code_memory(3, 120, 5e-5)
    p = oracle.Program(text)
    assert p.nchunks >= 2
    shots = 20000
    om, od, oo = p.sample(shots, seed=8, threads=8)
    gm, gd, go = gpu_sample(text, shots, seed=8, threads_per_shot=-32)
    assert np.array_equal(gm, om) and np.array_equal(gd, od) and np.array_equal(go, oo)


# ---------------------------------------------------------------- specialized kernel
def spec_sample(text, shots, seed=0, offset=0):
    p = pk.Program(text)
    p.specialize()
    return gpu_sample(p, shots, seed=seed, offset=offset, threads_per_shot=-32, specialize=1)


def test_specialized_surface_d3_bit_exact():
    text = circuits.workload("surface_d3_r3")["texts"][0]
    shots = 20000 + 37
    om, od, oo = oracle.Program(text).sample(shots, seed=11, threads=8)
    gm, gd, go = spec_sample(text, shots, seed=11)
    assert np.array_equal(gm, om) and np.array_equal(gd, od) and np.array_equal(go, oo)


@pytest.mark.parametrize("case", range(8))
def test_specialized_random_clifford_circuits(case):
    """Low-noise Pauli-frame-only random circuits (all noise types, MX,
    resets, detectors, an observable included twice) on the specialized
    kernel."""
    rng = np.random.default_rng(1500 + case)
    n = [5, 30, 40, 17][case % 4]
    text = random_small_circuit(rng, n, 90, rotations=False)
    # keep the circuit's structure, scale its noise down to the fault-list regime
    text = "\n".join(_scale_noise(line, 0.02) for line in text.splitlines()) + "\n"
    text += "OBSERVABLE_INCLUDE(1) rec[-1] rec[-2]\nOBSERVABLE_INCLUDE(1) rec[-1]\n"
    shots = 5000 + 13 * case
    om, od, oo = oracle.Program(text).sample(shots, seed=case, threads=8)
    gm, gd, go = spec_sample(text, shots, seed=case)
    assert np.array_equal(gm, om) and np.array_equal(gd, od) and np.array_equal(go, oo)


def _scale_noise(line, factor):
    import re
    m = re.match(r"^(\s*(?:DEPOLARIZE1|DEPOLARIZE2|X_ERROR|Y_ERROR|Z_ERROR))\(([^)]*)\)(.*)$", line)
    if not m:
        return line
    return "%s(%r)%s" % (m.group(1), float(m.group(2)) * factor, m.group(3))


@pytest.mark.parametrize("cap", ["1", "3"])
def test_specialized_fault_list_refill(cap, monkeypatch):
    """A lane whose faults exceed its list rebuilds the list above its last
    applied fault; shrinking the list forces that path."""
    text = circuits.surface_code_memory(3, 3, 1e-3)
    shots = 40000 + 3
    om, od, oo = oracle.Program(text).sample(shots, seed=21, threads=8)
    monkeypatch.setenv("CLIFFT_FRAMES_LIST_CAP", cap)
    gm, gd, go = spec_sample(text, shots, seed=21)
    assert np.array_equal(gm, om) and np.array_equal(gd, od) and np.array_equal(go, oo)


def test_specialized_shard_resume():
    text = circuits.surface_code_memory(3, 3, 1e-3)
    a = spec_sample(text, 4096 + 64, seed=5)
    b = spec_sample(text, 2048, seed=5, offset=0)
    c = spec_sample(text, 2048 + 64, seed=5, offset=2048)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, np.concatenate([y, z], axis=1))


def test_specialized_equals_interpreter_large():
    """At the benchmark size, the specialized kernel's records equal the
    bit-sliced interpreter's word for word (both are checked against the
    oracle at smaller sizes)."""
    text = circuits.workload("surface_d3_r3")["texts"][0]
    shots = 10_000_000
    p = pk.Program(text)
    p.specialize()
    a = gpu_sample(p, shots, seed=3, threads_per_shot=-32, specialize=-1)
    b = gpu_sample(p, shots, seed=3, threads_per_shot=-32, specialize=1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def _surface_d5_through_t_layer():
    """The d = 5 + 10 T workload cut after its T layer: final k = 10."""
    lines = circuits.workload("surface_d5_r5_t10")["texts"][0].splitlines()
    last = max(i for i, l in enumerate(lines) if l.startswith("T ") or l.startswith("T_DAG "))
    return "\n".join(lines[: last + 2]) + "\n"


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-5)])
@pytest.mark.parametrize("G,hbm", [(1, 1), (64, 1), (256, -1), (256, 1)])  # 64 shot-per-lane vectors of 2^10 exceed LDS
def test_forced_amplitudes_k10(precision, tol, G, hbm):
    """2^10 amplitudes after the T layer of the d = 5 workload, on forced
    shots (the oracle's own faults and outcomes), within the stated
    tolerance (vector-relative), and the branch probabilities of every
    forced outcome within the same relative tolerance."""
    text = _surface_d5_through_t_layer()
    op = oracle.Program(text)
    gp = pk.Program(text)
    assert op.kmax == 10 and gp.k_max == 10
    shots = 4
    fm = np.zeros((shots, op.nevents), np.uint32)
    ff = np.full((shots, op.nsites), -1, np.int32)
    traces = []
    for s in range(shots):
        faults = op.faults(31, s)
        t = op.trace(31, s, forced_faults=faults)
        fm[s] = t["m"]
        ff[s] = faults
        traces.append(t)
    res = gp.sample_trace(shots, seed=31, launch=pk.make_launch(precision, G, vector_in_hbm=hbm),
                          forced_m=torch.from_numpy(fm), forced_faults=torch.from_numpy(ff))
    torch.cuda.synchronize()
    probs = res["probs"].cpu().numpy()
    phi = res["phi"].cpu().numpy()
    gam = res["gamma"].cpu().numpy()
    gslots = gp.final_slots()
    for s, t in enumerate(traces):
        m = fm[s].astype(bool)
        pg = np.where(m, probs[s], 1.0 - probs[s])
        po = np.where(m, t["probs"], 1.0 - np.asarray(t["probs"]))
        assert np.max(np.abs(pg - po) / po) <= tol
        assert t["k"] == 10
        assert _state_error(phi[s, : 1 << 10], gam[s], gslots, t) <= tol


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-5)])
@pytest.mark.parametrize("G", [1, 64, 256])
def test_forced_probabilities_d5_full(precision, tol, G):
    """The whole d = 5 + 10 T workload on forced oracle shots with vectors in
    HBM: its first active measurement reads ten expansions, four of them
    deferred (the other six applied oldest first as the deferral fills), and
    every later one collapses out of place; each forced outcome's branch
    probability within the stated relative tolerance."""
    text = circuits.workload("surface_d5_r5_t10")["texts"][0]
    op = oracle.Program(text)
    gp = pk.Program(text)
    shots = 4
    fm = np.zeros((shots, op.nevents), np.uint32)
    ff = np.full((shots, op.nsites), -1, np.int32)
    traces = []
    for s in range(shots):
        faults = op.faults(41, s)
        t = op.trace(41, s, forced_faults=faults)
        fm[s] = t["m"]
        ff[s] = faults
        traces.append(t)
    res = gp.sample_trace(shots, seed=41, launch=pk.make_launch(precision, G, vector_in_hbm=1),
                          forced_m=torch.from_numpy(fm), forced_faults=torch.from_numpy(ff))
    torch.cuda.synchronize()
    probs = res["probs"].cpu().numpy()
    for s, t in enumerate(traces):
        m = fm[s].astype(bool)
        pg = np.where(m, probs[s], 1.0 - probs[s])
        po = np.where(m, t["probs"], 1.0 - np.asarray(t["probs"]))
        assert np.max(np.abs(pg - po) / po) <= tol
