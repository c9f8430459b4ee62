"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/clifft.h declares, its host compiler agrees with the oracle's on the
physical invariants of each workload, and errors come back as status codes.
No device work runs here."""
import os
import re
import subprocess

import pytest

import oracle
import paper_2604_27058_amd as pk
from paper_2604_27058_amd import circuits

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "clifft.h")).read()
    return sorted(set(re.findall(r"\b(clifft_[a-z_]+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    names = _declared_symbols()
    assert "clifft_sample" in names and "clifft_compile" in names
    out = subprocess.run(["nm", "-D", "--defined-only", pk.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = pk.lib()
    for n in names:
        assert hasattr(L, n)


@pytest.mark.parametrize("name", ["random_clifford_t_n8", "surface_d3_r3", "surface_d5_r5_t10", "large_active_k20"])
def test_compiler_agrees_with_oracle_on_invariants(name):
    w = circuits.workload(name)
    text = w["texts"][0]
    p = pk.Program(text)
    o = oracle.Program(text)
    assert p.k_max == o.kmax == w["kmax"]
    assert p.num_qubits == o.nq
    assert p.num_measurements == o.nrec
    assert p.num_detectors == o.ndet
    assert p.num_observables == o.nobs
    assert p.num_noise_sites == o.nsites
    assert p.num_events == o.nevents
    assert p.event_classes() == [int(c) for c in o.event_classes()]
    kp = p.k_profile()
    assert max(kp) == p.k_max and kp[-1] == o.k_profile()[-1]


def test_compiler_agrees_with_oracle_on_batched_set():
    for c in circuits.batched_set()[:16]:
        p = pk.Program(c["text"])
        o = oracle.Program(c["text"])
        assert p.k_max == o.kmax == c["k"]
        assert p.event_classes() == [int(x) for x in o.event_classes()]


def test_final_slots_hold_the_oracles_active_qubits():
    # slot order may differ (the GPU compiler refills a demoted slot from the
    # top), the set of active virtual qubits may not
    text = circuits.random_clifford_t(8, 40, 4, 0.0, seed=1000).replace("M 0 1 2 3 4 5 6 7", "")
    p = pk.Program(text)
    t = oracle.Program(text).trace(0, 0)
    assert sorted(p.final_slots()) == sorted(int(q) for q in t["slots"])


def test_status_codes():
    with pytest.raises(pk.ClifftError) as e:
        pk.Program("FOO 1\n")
    assert e.value.status == 2
    with pytest.raises(pk.ClifftError) as e:
        pk.Program("REPEAT 2 {\nH 0\n")
    assert e.value.status == 1
    with pytest.raises(pk.ClifftError) as e:
        pk.Program("H 300\n")
    assert e.value.status == 3
    with pytest.raises(pk.ClifftError) as e:
        pk.Program("DETECTOR rec[-1]\n")
    assert e.value.status == 1


def test_workspace_size_host_only():
    p = pk.Program(circuits.workload("large_active_k20")["texts"][0])
    n = p.workspace_size(pk.make_launch("f32", threads_per_shot=256, grid=4))
    assert n == 2 * 4 * (1 << 20) * 8  # two 2^20-amplitude buffers per workgroup
    small = pk.Program(circuits.workload("surface_d3_r3")["texts"][0])
    assert small.workspace_size() == 0


def test_specialize_host_only():
    """clifft_specialize generates and compiles the program-specialized
    bit-sliced kernel on the host (no GPU needed) and rejects programs that
    do not qualify."""
    p = pk.Program(circuits.surface_code_memory(3, 3, 1e-3))
    assert p.specialize() == ""
    assert p.specialize() == ""  # idempotent
    L = p.resolve_launch(10 ** 6, pk.make_launch("f32", -32, specialize=1))
    assert L["threads_per_shot"] == -32 and L["specialize"] == 1
    assert p.resolve_launch(10 ** 6, pk.make_launch("f32", -32))["specialize"] == -1
    with pytest.raises(pk.ClifftError, match="k_max = 0"):
        pk.Program(circuits.workload("surface_d5_r5_t10")["texts"][0]).specialize()
    with pytest.raises(pk.ClifftError, match="too long"):
        pk.Program(circuits.surface_code_memory(3, 40, 1e-5)).specialize()
    with pytest.raises(pk.ClifftError, match="too dense"):
        pk.Program(circuits.surface_code_memory(3, 3, 2e-2)).specialize()
    with pytest.raises(pk.ClifftError):
        p.resolve_launch(10 ** 6, pk.make_launch("f32", 1, specialize=1))
    assert p.resolve_launch(10 ** 6, pk.make_launch("f32", 1, specialize=-1))["specialize"] == 0  # not bit-sliced


def test_fused_byte_model_pins():
    """The fused-pass byte model the HBM rooflines are priced on.  Six fresh
    qubits expanded in a row with nothing reading the vector: four
    expansions stay deferred, the fifth and sixth each apply the oldest
    (reading and writing 2^0, then 2^1 stored amplitudes)."""
    n = 6
    text = "".join("H %d\n" % q for q in range(n)) + "".join("T %d\n" % q for q in range(n))
    p = pk.Program(text)
    assert p.k_max == n
    for prec, amp in (("f32", 8), ("f64", 16)):
        c = p.cost_model(prec)
        assert c["vector_bytes_fused"] == c["vector_bytes_fused_group"] == (2 * 1 + 2 * 2) * amp
        # the unfused table charges every expansion a read and a write of 2^k
        assert c["vector_bytes"] == sum(2 * (1 << k) * amp for k in range(n))


@pytest.mark.parametrize("name", ["random_clifford_t_n8", "surface_d5_r5_t10", "large_active_k20"])
def test_fused_byte_model_orders(name):
    """Fusing never adds bytes on either tier (the lane tier carries branch
    sums through deferred expansions; the cooperative tiers collapse pairs
    of measurements in one pass, so either can move fewer bytes), and the
    paired collapses never add bytes to the one-at-a-time collapses of the
    batched launch."""
    for text in circuits.workload(name)["texts"]:
        c = pk.Program(text).cost_model("f32")
        assert 0 < c["vector_bytes_fused"] <= c["vector_bytes"]
        assert 0 < c["vector_bytes_fused_group"] <= c["vector_bytes_fused_batch"] <= c["vector_bytes"]
    for spec in circuits.batched_set()[:16]:
        c = pk.Program(spec["text"]).cost_model("f32")
        assert c["vector_bytes_fused"] <= c["vector_bytes"]
        assert c["vector_bytes_fused_group"] <= c["vector_bytes_fused_batch"] <= c["vector_bytes"]


def test_compile_options():
    text = circuits.workload("random_clifford_t_n8")["texts"][0]
    assert pk.Program(text, k_limit=4).k_max == 4
    with pytest.raises(pk.ClifftError) as e:
        pk.Program(text, k_limit=3)
    assert e.value.status == 3
    with pytest.raises(pk.ClifftError) as e:
        pk.Program(text, hir_passes=8)
    assert e.value.status == 4
    with pytest.raises(pk.ClifftError) as e:
        pk.Program(text, drop_phases=2)
    assert e.value.status == 4
    # a rotation about a dormant Z string only changes the global scalar:
    # kept as one instruction, or left out on request
    ph = "T 0\nH 1\nT 1\nM 0 1\n"
    a, b = pk.Program(ph), pk.Program(ph, drop_phases=1)
    assert a.k_max == b.k_max == 1
    assert a.num_instructions == b.num_instructions + 1


@pytest.mark.parametrize("case", range(25))
def test_compiler_agrees_with_oracle_on_wide_gate_set(case):
    """R_X, R_Y, U3, rotations about Pauli products, MPP and feed-forward
    Paulis: the host compiler's k_max, event classes and record counts
    equal the oracle's (both lowered from the same circuit independently)."""
    from test_oracle_pins import random_wide_circuit
    import numpy as np
    rng = np.random.default_rng(8300 + case)
    text = random_wide_circuit(rng, int(rng.integers(2, 7)), int(rng.integers(10, 50)))
    p, o = pk.Program(text), oracle.Program(text)
    assert p.k_max == o.kmax
    assert p.num_measurements == o.nrec and p.num_events == o.nevents and p.num_detectors == o.ndet
    assert p.event_classes() == [int(c) for c in o.event_classes()]
    for hp in (1, 2, 3, 4):
        q = pk.Program(text, hir_passes=hp)
        assert q.k_max <= p.k_max and q.num_measurements == p.num_measurements


def test_wide_gate_parse_errors():
    for bad in ("MPP X0*X0\n", "MPP X0*Q1\n", "R_PAULI X0*Y1\n", "U3(0.1, 0.2) 0\n", "CX rec[-1] 0\n",
                "M 0\nCX 0 rec[-1]\n", "R_X 0\n", "H X0\n"):
        with pytest.raises(pk.ClifftError):
            pk.Program(bad)
        with pytest.raises(oracle.OracleError):
            oracle.Program(bad)


def test_postselect_compile_option():
    """Post-selected detectors (Section 3.2): counted in the program info,
    checked against the detectors the circuit has, kept out of the split
    form and the specialized kernel; the rest of the program is unchanged."""
    text = circuits.surface_code_memory(d=3, rounds=2, p=0.01, t_rotations=2, seed=1)
    plain = pk.Program(text)
    allp = pk.Program(text, postselect="all")
    some = pk.Program(text, postselect=[0, 3, 5])
    assert allp.num_postselected == plain.num_detectors > 5
    assert some.num_postselected == 3 and plain.num_postselected == 0
    assert allp.num_instructions == plain.num_instructions and allp.k_max == plain.k_max
    assert some.postselected == [0, 3, 5]
    with pytest.raises(pk.ClifftError) as e:
        pk.Program(text, postselect=[plain.num_detectors])
    assert e.value.status == 4
    assert allp.resolve_launch(1 << 16, pk.make_launch("f32"))["split"] == 0
    with pytest.raises(pk.ClifftError):
        allp.resolve_launch(1 << 16, pk.make_launch("f32", split=2))
    k0 = circuits.surface_code_memory(d=3, rounds=2, p=0.01)
    spec = pk.Program(k0, postselect=[0])
    with pytest.raises(pk.ClifftError):
        spec.resolve_launch(1 << 16, pk.make_launch("f32", threads_per_shot=-32, specialize=1))


@pytest.mark.parametrize("name", ["surface_d5_r5_t10", "large_active_k20"])
def test_fault_count_pmf_matches_oracle(name):
    """The library's stratum weights (host Poisson-binomial, accumulated in
    odds) against the oracle's probability recurrence."""
    import numpy as np
    text = circuits.workload(name)["texts"][0]
    p, o = pk.Program(text), oracle.Program(text)
    a = np.array(p.fault_count_pmf(25))
    b = o.fault_pmf(25)
    # both sums of non-negative terms over N sites: relative error within a
    # few N ulps each
    tol = 4 * o.nsites * 2.0 ** -53
    assert np.all(np.abs(a - b) <= tol * b + 1e-300), np.max(np.abs(a - b) / b)
    assert abs(a.sum() - 1.0) < 1e-6 or a.sum() < 1.0


def test_stratified_argument_checks_host_only():
    text = circuits.surface_code_memory(d=3, rounds=2, p=0.01)
    p = pk.Program(text)
    for bad in (-1, p.num_noise_sites + 1):
        with pytest.raises(pk.ClifftError) as e:  # checked before any device work
            pk._check(pk.lib().clifft_sample_stratified(p._h, 64, 0, 0, bad, None, None, 0, None, None, None, None))
        assert e.value.status == 4
    with pytest.raises(pk.ClifftError) as e:
        pk.Program("X_ERROR(1) 0\nM 0\n").fault_count_pmf(2)
    assert e.value.status == 2


def _enum(order, q):
    j = q >> order["nv"]
    for p in order["pos"]:
        j = ((j >> p) << (p + 1)) | (j & ((1 << p) - 1))
    for i, v in enumerate(order["v"]):
        if (q >> i) & 1:
            j ^= v
    return j


@pytest.mark.parametrize("name", ["large_active_k20", "surface_d5_r5_t10", "batched64"])
def test_pair_orders_are_permutations(name):
    """The compiler's item orders for the paired measurement passes (Appendix
    B.2 on two measurements; clifft_pair_orders) map the items q < 2^n onto
    themselves one to one in both element sizes: directions in reduced
    echelon form with their pivots among the zero-insertion positions, all
    below 2^n, and a brute-force check of the whole map up to n = 16."""
    texts = circuits.workload(name)["texts"]
    kinds = set()
    for text in texts[:24]:
        for e in pk.Program(text).pair_orders():
            kinds.add(e["kind"])
            assert 1 <= e["kind"] <= 5 and e["n"] >= 0
            n = e["n"]
            for prec in ("f32", "f64"):
                o = e[prec]
                assert 0 <= o["nv"] <= 4 and len(o["pos"]) == o["nv"] == len(o["v"])
                assert list(o["pos"]) == sorted(o["pos"]) and all(p < n for p in o["pos"])
                for i, v in enumerate(o["v"]):
                    assert 0 < v < (1 << n)
                    assert v.bit_length() - 1 in o["pos"]
                    for jj, w in enumerate(o["v"]):
                        if jj != i:
                            assert not (w >> (v.bit_length() - 1)) & 1
                if n <= 16:
                    img = sorted(_enum(o, q) for q in range(1 << n))
                    assert img == list(range(1 << n))
    assert kinds, "no paired passes"


def test_pairs_follow_the_precision_rule():
    """Paired collapses (Appendix B.2 on two measurements): FP64 pairs every
    eligible measurement; FP32 only on vectors of 2^17 amplitudes or more
    whose moved slots lie above the line bits, so of these workloads only
    k = 20 pairs in FP32.  The group byte model counts the pairs it prices."""
    k20 = pk.Program(circuits.workload("large_active_k20")["texts"][0])
    b3 = pk.Program(circuits.workload("batched64")["texts"][3])
    d5 = pk.Program(circuits.workload("surface_d5_r5_t10")["texts"][0])
    assert k20.cost_model("f32")["paired_measurements"] > 0
    assert k20.cost_model("f64")["paired_measurements"] >= k20.cost_model("f32")["paired_measurements"]
    assert b3.k_max == 16 and b3.cost_model("f32")["paired_measurements"] == 0
    assert b3.cost_model("f64")["paired_measurements"] > 0
    assert d5.cost_model("f32")["paired_measurements"] == 0
    for p in (k20, b3, d5):
        for prec in ("f32", "f64"):
            c = p.cost_model(prec)
            if c["paired_measurements"] == 0:
                assert c["vector_bytes_fused_group"] == c["vector_bytes_fused_batch"]
            else:
                assert c["vector_bytes_fused_group"] < c["vector_bytes_fused_batch"]


@pytest.mark.parametrize("name", ["large_active_k20", "surface_d5_r5_t10", "batched64"])
def test_pair_orders_agree_with_the_byte_model(name):
    """The compiler's two walks over the kernels' pairing decisions (the
    item orders and the byte model) agree in FP64, where every eligible
    measurement pairs: one second-measurement pass (kinds 3-5) per pair
    start, and a first measurement's read pass (kind 1) only where no joint
    sums were carried to it (so never more read passes than pairs)."""
    for text in circuits.workload(name)["texts"][:24]:
        p = pk.Program(text)
        kinds = [e["kind"] for e in p.pair_orders()]
        starts = p.cost_model("f64")["paired_measurements"]
        assert sum(k in (3, 4, 5) for k in kinds) == starts
        assert kinds.count(1) <= starts
