"""Pins of the FP64 oracle against things other than itself.

* Philox4x32-10 known-answer vectors (Random123 / SC'11), rocRAND's
  independent header implementation, chi-square uniformity of its words.
* The paper's worked example (Section 3.1, Figs. 3-4): structure and closed
  form statistics.
* Closed forms: T-state expectations (Appendix C), R_Z rotation angles.
* Record-by-record and amplitude-by-amplitude agreement with an independent
  dense state-vector brute force (tests/dense_ref.py) on random circuits.
* Gap sampler: exact inversion rule, per-site rates, and the
  Poisson-binomial law of the fault count per shot.
* Lemma 1: every localization takes at most 2N virtual gates.
* Noiseless surface codes (detectors all zero), mirror circuits (records all
  zero), single-fault propagation versus GF(2) Pauli propagation.
"""
import json
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import dense_ref
import oracle
from paper_2604_27058_amd import circuits
from stats import popcount_rows, two_sample_ok, within_sigma

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox
KAT = [  # Random123 known-answer vectors for philox4x32-10
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_kat(ctr, key, want):
    assert tuple(oracle.philox(ctr, key)) == want
    assert tuple(dense_ref.philox(ctr, key)) == want


def test_philox_oracle_equals_dense_random_inputs():
    rng = np.random.default_rng(1)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**32, 4)]
        key = [int(v) for v in rng.integers(0, 2**32, 2)]
        assert tuple(oracle.philox(ctr, key)) == tuple(dense_ref.philox(ctr, key))


ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned long long seeds[3] = {0ull, 0x0123456789abcdefull, 0xffffffffffffffffull};
  for (int s = 0; s < 3; s++)
    for (unsigned long long sub = 0; sub < 3; sub++) {
      rocrand_device::philox4x32_10_engine e(seeds[s], sub, 0);
      uint4 v = e.next4();
      printf("%llu %llu %u %u %u %u\n", seeds[s], sub, v.x, v.y, v.z, v.w);
    }
}
"""


def test_philox_matches_rocrand_header(tmp_path):
    """rocRAND's Philox4x32-10 is an independent implementation of the same
    published generator: its engine seeded with (seed, subsequence) returns
    philox(ctr = (0, 0, sub_lo, sub_hi), key = (seed_lo, seed_hi)) first."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "probe.cpp"
    src.write_text(ROCRAND_PROBE)
    exe = tmp_path / "probe"
    r = subprocess.run([hipcc, "-O1", "-o", str(exe), str(src)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not build the rocRAND probe: " + r.stderr[-300:])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    n = 0
    for line in out:
        if not line.strip():
            continue
        seed, sub, a, b, c, d = [int(t) for t in line.split()]
        want = oracle.philox([0, 0, sub & 0xFFFFFFFF, sub >> 32], [seed & 0xFFFFFFFF, seed >> 32])
        assert (a, b, c, d) == tuple(want)
        n += 1
    assert n == 9


# ---------------------------------------------------------------- worked example
def _mirror_text():
    return open(os.path.join(GOLD, "mirror_example.stim")).read()


def test_worked_example_structure():
    g = json.load(open(os.path.join(GOLD, "mirror_example.json")))
    p = oracle.Program(_mirror_text())
    assert p.kmax == g["kmax"]
    assert p.nsites == g["noise_sites"]
    cls = p.event_classes()
    names = {0: "static", 1: "random", 2: "active"}
    assert names[int(cls[0])] == g["event_classes_by_record"]["0"]
    assert names[int(cls[1])] == g["event_classes_by_record"]["1"]
    ops = [oracle.OP_NAMES[o] for o in p.ops()[:, 0]]
    assert ops.count("EXPAND") == 1 and ops.count("MACTIVE_X") == 1 and ops.count("MSTATIC") == 1
    kp = p.k_profile()
    assert kp.max() == 1 and kp[-1] == 0


def test_worked_example_statistics():
    g = json.load(open(os.path.join(GOLD, "mirror_example.json")))
    # noiseless: exact probabilities
    t = oracle.Program(_mirror_text().replace("DEPOLARIZE1(0.001) 0 1", "")).trace(0, 0)
    assert abs(t["probs"][0] - g["noiseless_p_rec0"]) < 1e-15
    assert t["probs"][1] == g["noiseless_p_rec1"]
    # noisy: sample and compare with the closed forms
    p = 1e-3
    q = 2 * p / 3
    prog = oracle.Program(_mirror_text())
    shots = 400_000
    meas, _, _ = prog.sample(shots, seed=7, threads=8)
    c = popcount_rows(meas, shots)
    assert within_sigma(c[1], shots, 2 * q * (1 - q))
    assert within_sigma(c[0], shots, 0.5)
    both = popcount_rows(meas[0:1] & meas[1:2], shots)[0]
    assert within_sigma(both, shots, 0.5 * 2 * q * (1 - q))


# ---------------------------------------------------------------- closed forms
def test_t_state_expectations():
    g = json.load(open(os.path.join(GOLD, "t_state.json")))
    px = oracle.Program("H 0\nT 0\nMX 0\n").trace()["probs"][0]
    py = oracle.Program("H 0\nT 0\nS_DAG 0\nH 0\nM 0\n").trace()["probs"][0]
    pz = oracle.Program("H 0\nT 0\nM 0\n").trace()["probs"][0]
    assert abs(px - g["p1_mx_after_H_T"]) < 1e-15
    assert abs(py - g["p1_my_after_H_T"]) < 1e-15
    assert abs(pz - g["p1_mz_after_H_T"]) < 1e-15
    # T_DAG flips the sign of <Y>
    pyd = oracle.Program("H 0\nT_DAG 0\nS_DAG 0\nH 0\nM 0\n").trace()["probs"][0]
    assert abs(pyd - (1 + 1 / math.sqrt(2)) / 2) < 1e-15


@pytest.mark.parametrize("theta", [0.02, 0.3, 1.0, 2.5, -0.7, math.pi])
def test_rz_closed_form(theta):
    pr = oracle.Program("H 0\nR_Z(%r) 0\nH 0\nM 0\n" % theta).trace()["probs"][0]
    assert abs(pr - math.sin(theta / 2) ** 2) < 1e-14
    # the same rotation reached through a Clifford-entangled generator
    pr2 = oracle.Program("H 0\nCX 0 1\nCX 0 2\nR_Z(%r) 2\nCX 0 2\nCX 0 1\nH 0\nM 0\n" % theta).trace()["probs"][0]
    assert abs(pr2 - math.sin(theta / 2) ** 2) < 1e-14


# ---------------------------------------------------------------- dense brute force
ONEQ = ["H", "S", "S_DAG", "X", "Y", "Z"]


def random_small_circuit(rng, n, nops, p_noise=0.08, rotations=True, repeat=True):
    out = []
    nrec = 0
    body = []

    def emit(line, recs=0):
        body.append(line)
        return recs

    for _ in range(nops):
        r = rng.random()
        q = int(rng.integers(0, n))
        if r < 0.25:
            emit("%s %d" % (ONEQ[int(rng.integers(0, 6))], q))
        elif r < 0.45:
            a, b = [int(v) for v in rng.choice(n, 2, replace=False)]
            emit("%s %d %d" % (["CX", "CZ", "SWAP", "CX"][int(rng.integers(0, 4))], a, b))
        elif r < 0.60 and rotations:
            k = int(rng.integers(0, 3))
            emit(["T %d" % q, "T_DAG %d" % q, "R_Z(%r) %d" % (float(rng.uniform(-3, 3)), q)][k])
        elif r < 0.75:
            kind = ["M", "MX", "MR", "R"][int(rng.integers(0, 4))]
            emit("%s %d" % (kind, q))
            if kind != "R":
                nrec += 1
                if nrec >= 2 and rng.random() < 0.5:
                    emit("DETECTOR rec[-1] rec[-2]")
                if rng.random() < 0.3:
                    emit("OBSERVABLE_INCLUDE(%d) rec[-1]" % int(rng.integers(0, 2)))
        elif p_noise:
            kind = int(rng.integers(0, 5))
            pp = float(rng.uniform(0.02, p_noise))
            if kind == 1:
                a, b = [int(v) for v in rng.choice(n, 2, replace=False)]
                emit("DEPOLARIZE2(%r) %d %d" % (pp, a, b))
            else:
                emit("%s(%r) %d" % (["DEPOLARIZE1", "", "X_ERROR", "Y_ERROR", "Z_ERROR"][kind], pp, q))
    if repeat and len(body) > 6 and rng.random() < 0.5:
        # wrap a measurement-free middle slice in a REPEAT block
        i = len(body) // 3
        j = i + 3
        mid = body[i:j]
        if not any(l.split()[0].split("(")[0] in ("M", "MX", "MR", "R", "DETECTOR", "OBSERVABLE_INCLUDE")
                   for l in mid):
            body = body[:i] + ["REPEAT 2 {"] + mid + ["}"] + body[j:]
    out.extend(body)
    out.append("M " + " ".join(map(str, range(n))))
    return "\n".join(out) + "\n"


def _product(rng, n):
    k = int(rng.integers(1, min(n, 3) + 1))
    qs = [int(v) for v in rng.choice(n, k, replace=False)]
    return "*".join("%s%d" % ("XYZ"[int(rng.integers(0, 3))], q) for q in qs)


def random_wide_circuit(rng, n, nops, p_noise=0.08, probes=False):
    """random_small_circuit's operations plus the wider gate set: R_X, R_Y,
    U3, rotations about Pauli products, product measurements (MPP) and
    record-controlled Paulis; with probes, expectation-value probes of
    random Pauli products (EXP_VAL) between them."""
    body = []
    nrec = 0
    for _ in range(nops):
        if probes and rng.random() < 0.15:
            body.append("EXP_VAL %s" % _product(rng, n))
        r = rng.random()
        q = int(rng.integers(0, n))
        if r < 0.2:
            body.append("%s %d" % (ONEQ[int(rng.integers(0, 6))], q))
        elif r < 0.32:
            a, b = [int(v) for v in rng.choice(n, 2, replace=False)]
            body.append("%s %d %d" % (["CX", "CZ", "SWAP"][int(rng.integers(0, 3))], a, b))
        elif r < 0.52:
            k = int(rng.integers(0, 5))
            ang = float(rng.uniform(-3, 3))
            if k == 0:
                body.append("R_X(%r) %d" % (ang, q))
            elif k == 1:
                body.append("R_Y(%r) %d" % (ang, q))
            elif k == 2:
                body.append("U3(%r, %r, %r) %d" % (ang, float(rng.uniform(-3, 3)), float(rng.uniform(-3, 3)), q))
            elif k == 3:
                body.append("R_PAULI(%r) %s" % (ang, _product(rng, n)))
            else:
                body.append("T %d" % q)
        elif r < 0.7:
            k = int(rng.integers(0, 4))
            if k == 0:
                body.append("MPP %s" % _product(rng, n))
            else:
                body.append("%s %d" % (["M", "MX", "MR"][k - 1], q))
            nrec += 1
            if nrec >= 2 and rng.random() < 0.4:
                body.append("DETECTOR rec[-1] rec[-2]")
            if rng.random() < 0.5:
                body.append("%s rec[-%d] %d" % (["CX", "CY", "CZ"][int(rng.integers(0, 3))],
                                                int(rng.integers(1, nrec + 1)), int(rng.integers(0, n))))
        elif p_noise:
            kind = int(rng.integers(0, 5))
            pp = float(rng.uniform(0.02, p_noise))
            if kind == 1:
                a, b = [int(v) for v in rng.choice(n, 2, replace=False)]
                body.append("DEPOLARIZE2(%r) %d %d" % (pp, a, b))
            else:
                body.append("%s(%r) %d" % (["DEPOLARIZE1", "", "X_ERROR", "Y_ERROR", "Z_ERROR"][kind], pp, q))
    body.append("M " + " ".join(map(str, range(n))))
    return "\n".join(body) + "\n"


@pytest.mark.parametrize("theta", [0.3, 1.0, 2.5, -0.7])
def test_wide_gate_closed_forms(theta):
    """R_X(t)|0>, R_Y(t)|0> and U3(t, p, l)|0> measured in Z give
    sin^2(t/2); a rotation about X0*X1 from |00> gives the same for Z0;
    U3(t, p, l) = e^{i(p+l)/2} R_Z(p) R_Y(t) R_Z(l) is checked through the
    global scalar of the oracle's state against the dense matrix."""
    s2 = math.sin(theta / 2) ** 2
    for text in ("R_X(%r) 0\nM 0\n" % theta, "R_Y(%r) 0\nM 0\n" % theta, "U3(%r, 0.4, -1.1) 0\nM 0\n" % theta,
                 "R_PAULI(%r) X0*X1\nM 0\n" % theta, "R_PAULI(%r) Y0*Z2\nM 0\n" % theta):
        pr = oracle.Program(text).trace()["probs"][0]
        assert abs(pr - s2) < 1e-14, text
    _compare_shot("U3(%r, 0.4, -1.1) 0\nH 1\nCX 1 0\n" % theta, seed=0, shot=0)


def test_product_measurements_and_feed_forward():
    # Bell pair: X0X1 = +1, Z0Z1 = +1, Y0Y1 = -1, all deterministic
    p = oracle.Program("H 0\nCX 0 1\nMPP X0*X1 Z0*Z1 Y0*Y1\n")
    t = p.trace()
    assert list(t["recs"]) == [0, 0, 1] and list(p.event_classes()) == [0, 0, 0]
    # measuring one half of a Bell pair and correcting the other with the
    # record leaves it in |0>: its measurement always reads 0
    m, _, _ = oracle.Program("H 0\nCX 0 1\nM 0\nCX rec[-1] 1\nM 1\n").sample(4096, seed=3)
    assert popcount_rows(m[0:1], 4096)[0] > 1500 and popcount_rows(m[1:2], 4096)[0] == 0
    # a Z correction after an X-basis measurement, CZ with the record second
    m, _, _ = oracle.Program("H 0\nCX 0 1\nMX 0\nCZ 1 rec[-1]\nH 1\nM 1\n").sample(4096, seed=4)
    assert popcount_rows(m[1:2], 4096)[0] == 0


def test_expectation_probes_t_state():
    """Appendix C: for |T> = T H |0>, <X> = <Y> = 1/sqrt(2) and <Z> = 0;
    the probes read the state without changing it (the measurement after
    them still sees P(X = -1) of the T state)."""
    t = oracle.Program("H 0\nT 0\nEXP_VAL X0 Y0 Z0\nMX 0\n").trace()
    r = 1 / math.sqrt(2)
    np.testing.assert_allclose(t["expvals"], [r, r, 0.0], atol=1e-15)
    assert abs(t["probs"][0] - (1 - r) / 2) < 1e-15
    # a probe behind a Clifford frame and a Pauli frame: X on the T state
    # conjugated by CX into a two-qubit observable, and a frame flip by X
    t = oracle.Program("H 0\nT 0\nCX 0 1\nX 1\nEXP_VAL X0*X1 Y0*X1 Z0*Z1 Z1\n").trace()
    np.testing.assert_allclose(t["expvals"], [r, r, -1.0, 0.0], atol=1e-15)


@pytest.mark.parametrize("case", range(20))
def test_oracle_matches_dense_probes(case):
    rng = np.random.default_rng(8600 + case)
    text = random_wide_circuit(rng, int(rng.integers(2, 6)), int(rng.integers(10, 40)), probes=True)
    for shot in range(3):
        _compare_shot(text, seed=case, shot=shot, check_state=(shot == 0))


@pytest.mark.parametrize("case", range(30))
def test_oracle_matches_dense_wide_gate_set(case):
    rng = np.random.default_rng(8100 + case)
    text = random_wide_circuit(rng, int(rng.integers(2, 6)), int(rng.integers(10, 40)))
    for shot in range(3):
        _compare_shot(text, seed=case, shot=shot, check_state=(shot == 0))


@pytest.mark.parametrize("case", range(10))
def test_oracle_matches_dense_wide_gate_set_forced(case):
    rng = np.random.default_rng(8200 + case)
    text = random_wide_circuit(rng, int(rng.integers(2, 6)), int(rng.integers(10, 40)))
    _compare_shot(text, seed=case, shot=0, forced=True, rng=rng)


def _compare_shot(text, seed, shot, check_state=True, forced=False, rng=None):
    prog = oracle.Program(text)
    dn = dense_ref.Dense(text)
    if forced:
        # forced faults: any outcome at a random subset of sites; forced
        # outcomes: chosen along the dense trajectory with nonzero probability
        ff = [int(rng.integers(0, dense_ref.NOISE_OUT[s[0]])) if rng.random() < 0.3 else -1 for s in dn.sites]
        d0 = dn.run(seed, shot, forced_faults=ff)
        fm = d0["m"].copy()
        t = prog.trace(seed, shot, forced_m=fm, forced_faults=np.array(ff, np.int32))
        d = dn.run(seed, shot, forced_m=fm, forced_faults=ff)
    else:
        t = prog.trace(seed, shot)
        d = dn.run(seed, shot)
    assert t["error"] == 0
    cls = {0: "static", 1: "random", 2: "active"}
    assert [cls[int(c)] for c in prog.event_classes()] == d["classes"]
    assert prog.kmax == d["kmax"]
    assert list(t["faults"]) == list(d["faults"])
    assert np.array_equal(t["m"], d["m"])
    assert np.array_equal(t["recs"], d["recs"])
    assert np.array_equal(t["dets"], d["dets"])
    assert np.array_equal(t["obs"], d["obs"][: len(t["obs"])])
    np.testing.assert_allclose(t["probs"], d["probs"], atol=1e-12)
    np.testing.assert_allclose(t["expvals"], d["expvals"], atol=1e-12)
    if check_state:
        fr = t["frame"]
        psi_o = dense_ref.oracle_state_to_dense(prog.nq, prog.uclog(), fr[0], fr[1], t["phi"], t["slots"],
                                                t["gamma"])
        np.testing.assert_allclose(psi_o, d["psi"], atol=1e-10)


@pytest.mark.parametrize("case", range(40))
def test_oracle_matches_dense_random_circuits(case):
    rng = np.random.default_rng(100 + case)
    n = int(rng.integers(2, 6))
    text = random_small_circuit(rng, n, int(rng.integers(10, 45)))
    for shot in range(3):
        _compare_shot(text, seed=case, shot=shot)


@pytest.mark.parametrize("case", range(20))
def test_oracle_matches_dense_forced(case):
    rng = np.random.default_rng(500 + case)
    n = int(rng.integers(2, 6))
    text = random_small_circuit(rng, n, int(rng.integers(10, 40)))
    _compare_shot(text, seed=case, shot=0, forced=True, rng=rng)


def test_oracle_matches_dense_mirror_example_many_shots():
    text = _mirror_text().replace("0.001", "0.2")
    for shot in range(30):
        _compare_shot(text, seed=3, shot=shot, check_state=(shot < 3))


@pytest.mark.parametrize("name", ["clifford_t_small", "surface_d2"])
def test_oracle_matches_dense_structured(name):
    if name == "clifford_t_small":
        text = circuits.random_clifford_t(n=6, layers=8, n_t=3, p=0.02, seed=11)
    else:
        text = circuits.surface_code_memory(d=2, rounds=2, p=0.02)
    for shot in range(4):
        _compare_shot(text, seed=1, shot=shot, check_state=(shot == 0))


@pytest.mark.parametrize("name", ["surface_d2_t1", "register_n10_k4", "register_n9_k6"])
def test_oracle_matches_dense_workload_recipes(name):
    """Small-N versions of the benchmark recipes through the dense brute
    force: the surface code with a T layer between rounds (the d = 5 + 10 T
    recipe at d = 2) and the magic-register recipe of the batched and
    large-k workloads (register expanded by H + T / R_Z, Clifford layers,
    mid-circuit MR of register qubits and re-expansion, final measurement),
    at noise high enough that most shots carry faults."""
    if name == "surface_d2_t1":
        text = circuits.surface_code_memory(d=2, rounds=3, p=0.02, t_rotations=1, t_after_round=1)
        kmax = 1
    elif name == "register_n10_k4":
        text = circuits.register_circuit(10, 12, 4, 6, 0.02, seed=7, mid_measure_every=8, mid_measure_count=2)
        kmax = 4
    else:
        text = circuits.register_circuit(9, 10, 6, 9, 0.03, seed=8, mid_measure_every=4, mid_measure_count=3)
        kmax = 6
    assert oracle.Program(text).kmax == kmax
    for shot in range(6):
        _compare_shot(text, seed=2, shot=shot, check_state=(shot == 0))


@pytest.mark.parametrize("name", ["register_n9_k6", "surface_d2_t1"])
def test_oracle_matches_dense_workload_recipes_forced(name):
    """The same recipes on forced faults and outcomes (every branch
    probability and the final state along the forced trajectory)."""
    if name == "surface_d2_t1":
        text = circuits.surface_code_memory(d=2, rounds=3, p=0.02, t_rotations=1, t_after_round=1)
    else:
        text = circuits.register_circuit(9, 10, 6, 9, 0.03, seed=8, mid_measure_every=4, mid_measure_count=3)
    rng = np.random.default_rng(31)
    for shot in range(3):
        _compare_shot(text, seed=4, shot=shot, forced=True, rng=rng, check_state=(shot == 0))


def test_impossible_forced_outcome_flagged():
    p = oracle.Program("H 0\nT 0\nH 0\nT 0\nM 0\nM 0\n")
    t = p.trace(0, 0, forced_m=np.array([1, 0], np.uint8))
    assert t["error"] == 2  # second measurement must repeat the first


# ---------------------------------------------------------------- gap sampler
def test_gap_inversion_rule_exact():
    rng = np.random.default_rng(3)
    ps = rng.uniform(0, 0.3, 12)
    S = [1.0]
    for p in ps:
        S.append(S[-1] * (1.0 - p))
    S = np.array(S)
    for cur in range(len(ps)):
        for u in np.linspace(0, 1, 4001, endpoint=False):
            j = oracle.gap_next(S, cur, u)
            tau = u * S[cur]
            if j < 0:
                assert all(S[i + 1] > tau for i in range(cur, len(ps)))
            else:
                assert S[j + 1] <= tau and all(S[i + 1] > tau for i in range(cur, j))
    # the measure of u mapping to j is (S_j - S_{j+1}) / S_cur
    for cur in (0, 5):
        us = np.linspace(0, 1, 200001, endpoint=False)
        js = np.array([oracle.gap_next(S, cur, u) for u in us])
        for j in range(cur, len(ps)):
            frac = np.mean(js == j)
            assert abs(frac - (S[j] - S[j + 1]) / S[cur]) < 2e-5


def test_fault_sites_rates_and_outcomes():
    text = "\n".join(["DEPOLARIZE1(0.05) 0", "X_ERROR(0.2) 1", "DEPOLARIZE2(0.1) 0 1", "Z_ERROR(0.01) 2"]) + "\n"
    text += "M 0 1 2\n"
    p = oracle.Program(text)
    counts = np.zeros((4, 16))
    shots = 20000
    for s in range(shots):
        f = p.faults(5, s)
        for i, v in enumerate(f):
            if v >= 0:
                counts[i, v] += 1
    for i, (pp, nout) in enumerate([(0.05, 3), (0.2, 1), (0.1, 15), (0.01, 1)]):
        assert within_sigma(counts[i].sum(), shots, pp)
        for o in range(nout):
            assert within_sigma(counts[i, o], shots, pp / nout)


def test_faults_oracle_equals_dense_many_chunks():
    # more than one 4096-site chunk
    text = "DEPOLARIZE1(0.002) 0\n" * 9000 + "M 0\n"
    p = oracle.Program(text)
    d = dense_ref.Dense(text)
    assert p.nchunks == 3
    for shot in range(5):
        assert list(p.faults(9, shot)) == d.faults(9, shot)


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("d,rounds", [(3, 3), (5, 5)])
def test_noiseless_surface_code_detectors_zero(d, rounds):
    p = oracle.Program(circuits.surface_code_memory(d, rounds, p=0.0, noise=False))
    assert p.kmax == 0
    shots = 2048
    meas, det, obs = p.sample(shots, seed=2, threads=8)
    assert not det.any() and not obs.any()
    # the random X-stabilizer outcomes are really random
    assert meas.any()


def test_noiseless_surface_code_with_t_rotations_k10():
    p = oracle.Program(circuits.surface_code_memory(5, 5, 5e-4, t_rotations=10, t_after_round=2, seed=3000))
    assert p.kmax == 10
    assert int(np.sum(p.event_classes() == 2)) == 10


@pytest.mark.parametrize("seed", range(6))
def test_mirror_circuits_return_to_zero(seed):
    rng = np.random.default_rng(seed)
    n = 6
    fwd = []
    for _ in range(30):
        r = rng.random()
        if r < 0.3:
            fwd.append(("H", [int(rng.integers(0, n))]))
        elif r < 0.5:
            fwd.append(("S", [int(rng.integers(0, n))]))
        elif r < 0.75:
            fwd.append(("CX", [int(v) for v in rng.choice(n, 2, replace=False)]))
        else:
            fwd.append(("T", [int(rng.integers(0, n))]))
    inv = {"H": "H", "S": "S_DAG", "CX": "CX", "T": "T_DAG"}
    lines = ["%s %s" % (g, " ".join(map(str, t))) for g, t in fwd]
    lines += ["%s %s" % (inv[g], " ".join(map(str, t))) for g, t in reversed(fwd)]
    lines.append("M " + " ".join(map(str, range(n))))
    p = oracle.Program("\n".join(lines) + "\n")
    assert p.kmax >= 1
    meas, _, _ = p.sample(512, seed=seed, threads=4)
    assert not meas.any()
    t = p.trace(seed, 0)
    assert np.all(t["probs"] < 1e-12)


def test_single_fault_propagation_surface_d3():
    """Forcing one fault must flip exactly the detectors predicted by
    propagating the physical Pauli through the Clifford circuit (GF(2))."""
    text = circuits.surface_code_memory(3, 3, 1e-3)
    p = oracle.Program(text)
    ops = dense_ref.parse(text)
    n = p.nq
    # physical noise sites in order with their targets
    sites = []
    for name, arg, tg in ops:
        if name in dense_ref.NOISE_OUT:
            ar = 2 if name == "DEPOLARIZE2" else 1
            for i in range(0, len(tg), ar):
                sites.append((name, tg[i:i + ar]))
    base = p.trace(4, 0, forced_faults=np.full(p.nsites, -1, np.int32))
    assert not base["dets"].any()
    checked = 0
    for s, (name, tg) in enumerate(sites):
        for o in range(dense_ref.NOISE_OUT[name]):
            ff = np.full(p.nsites, -1, np.int32)
            ff[s] = o
            t = p.trace(4, 0, forced_faults=ff)
            want = _propagate_single_fault(ops, s, o, n)
            assert list(t["dets"]) == want[0], (s, name, o)
            assert list(t["obs"]) == want[1]
            checked += 1
    assert checked > 300


def _propagate_single_fault(ops, site, outcome, n):
    """GF(2) propagation of one physical Pauli fault; returns detector and
    observable flips."""
    x = np.zeros(n, np.uint8)
    z = np.zeros(n, np.uint8)
    flips = []
    dets = []
    obs = {}
    s = 0
    for name, arg, tg in ops:
        if name in ("H", "S", "S_DAG"):
            for q in tg:
                dense_ref.conj_bits(x, z, name, q)
        elif name in ("CX", "CZ", "SWAP"):
            for i in range(0, len(tg), 2):
                dense_ref.conj_bits(x, z, name, tg[i], tg[i + 1])
        elif name in dense_ref.NOISE_OUT:
            ar = 2 if name == "DEPOLARIZE2" else 1
            for i in range(0, len(tg), ar):
                if s == site:
                    la, lb = dense_ref.noise_letters(name, outcome)
                    for q, L in zip(tg[i:i + ar], (la, lb)):
                        x[q] ^= L in (1, 2)
                        z[q] ^= L in (2, 3)
                s += 1
        elif name in ("M", "MR", "R", "MX"):
            for q in tg:
                f = int(z[q] if name == "MX" else x[q])
                if name != "R":
                    flips.append(f)
                if name in ("MR", "R"):
                    x[q] = 0
        elif name == "DETECTOR":
            dets.append(int(np.bitwise_xor.reduce([flips[len(flips) + k] for _, k in tg])))
        elif name == "OBSERVABLE_INCLUDE":
            o = int(arg)
            obs[o] = obs.get(o, 0) ^ int(np.bitwise_xor.reduce([flips[len(flips) + k] for _, k in tg]))
    return dets, [obs.get(i, 0) for i in range(len(obs))]


@pytest.mark.parametrize("name", ["random_clifford_t_n8", "surface_d3_r3", "surface_d5_r5_t10"])
def test_classification_matches_stabilizer_group(name):
    """k(t) = N - rank(G_t) and the random/static/active classes are physical
    (basis independent); an independent stabilizer-group tracker must agree."""
    text = circuits.workload(name)["texts"][0]
    p = oracle.Program(text)
    assert p.kmax == circuits.workload(name)["kmax"]
    G = dense_ref.Stabilizers(p.nq)
    classes = []
    kmax = 0
    n = p.nq
    for nm, arg, tg in dense_ref.parse(text):
        if nm in ("H", "S", "S_DAG"):
            for q in tg:
                G.conj(nm, q)
        elif nm in ("CX", "CZ", "SWAP"):
            for i in range(0, len(tg), 2):
                G.conj(nm, tg[i], tg[i + 1])
        elif nm in ("T", "T_DAG", "R_Z"):
            for q in tg:
                pz = np.zeros(n, np.uint8)
                pz[q] = 1
                G.rotation(np.zeros(n, np.uint8), pz)
        elif nm in ("M", "MX", "MR", "R"):
            for q in tg:
                px = np.zeros(n, np.uint8)
                pz = np.zeros(n, np.uint8)
                (px if nm == "MX" else pz)[q] = 1
                classes.append(G.measure(px, pz))
        kmax = max(kmax, G.k())
    names = {0: "static", 1: "random", 2: "active"}
    assert [names[int(c)] for c in p.event_classes()] == classes
    assert kmax == p.kmax


def test_shard_resume_bit_identical():
    p = oracle.Program(circuits.surface_code_memory(3, 3, 1e-2))
    a = p.sample(1024, seed=5, offset=0, threads=3)
    b = p.sample(512, seed=5, offset=0, threads=1)
    c = p.sample(512, seed=5, offset=512, threads=2)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, np.concatenate([y, z], axis=1))


def test_unit_norm_all_workloads():
    for name in ["random_clifford_t_n8", "surface_d5_r5_t10"]:
        p = oracle.Program(circuits.workload(name)["texts"][0])
        p.sample(256, seed=1, threads=8)  # raises on a unit-norm violation
    for c in circuits.batched_set()[:6]:
        oracle.Program(c["text"]).sample(64, seed=1, threads=8)


def test_parse_errors():
    with pytest.raises(oracle.OracleError):
        oracle.Program("FOO 1\n")
    with pytest.raises(oracle.OracleError):
        oracle.Program("REPEAT 2 {\nH 0\n")
    with pytest.raises(oracle.OracleError):
        oracle.Program("DETECTOR rec[-1]\n")


def test_consecutive_shots_equal_single_shot_traces():
    """Each shot of a multi-shot sample equals a fresh single-shot trace
    (no state carried between shots)."""
    text = circuits.surface_code_memory(3, 2, 2e-2)
    p = oracle.Program(text)
    shots = 130
    meas, det, obs = p.sample(shots, seed=8, threads=1)
    for s in range(shots):
        t = p.trace(8, s)
        assert [(int(meas[r, s // 64]) >> (s % 64)) & 1 for r in range(p.nrec)] == list(t["recs"])
        assert [(int(det[r, s // 64]) >> (s % 64)) & 1 for r in range(p.ndet)] == list(t["dets"])
        assert [(int(obs[r, s // 64]) >> (s % 64)) & 1 for r in range(p.nobs)] == list(t["obs"])


# ---------------------------------------------------------------- more pins
def test_philox_words_uniform_chi_square():
    """Each output word's top 4 bits are uniform over 16 bins (chi-square,
    15 degrees of freedom, fixed counters; the bound is the 1e-6 quantile)."""
    counts = np.zeros(16, dtype=np.int64)
    n = 8000
    for i in range(n):
        w = oracle.philox((i, 0x4E000000, i * 2654435761 & 0xFFFFFFFF, 7), (12345, 678))
        for x in w:
            counts[x >> 28] += 1
    expect = 4 * n / 16
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    assert chi2 < 50.0, chi2


def _poisson_binomial(ps):
    pmf = np.zeros(len(ps) + 1)
    pmf[0] = 1.0
    for p in ps:
        pmf[1:] = pmf[1:] * (1 - p) + pmf[:-1] * p
        pmf[0] *= 1 - p
    return pmf


def test_fault_count_is_poisson_binomial():
    """The number of realized faults per shot follows the Poisson-binomial
    law of the site probabilities (Section 3.2: every site fires
    independently with its own p), checked bin by bin within 5 sigma."""
    ps = [0.02, 0.05, 0.1, 0.15, 0.2, 0.03, 0.08, 0.12, 0.25, 0.01, 0.3, 0.06]
    text = "".join("X_ERROR(%r) %d\n" % (p, i) for i, p in enumerate(ps))
    text += "".join("M %d\n" % i for i in range(len(ps)))
    prog = oracle.Program(text)
    shots = 12000
    hist = np.zeros(len(ps) + 1, dtype=np.int64)
    for s in range(shots):
        hist[int((prog.faults(seed=3, shot=s) >= 0).sum())] += 1
    pmf = _poisson_binomial(ps)
    for c, p in zip(hist, pmf):
        assert within_sigma(c, shots, p, 5.0), (hist, pmf * shots)


@pytest.mark.parametrize("case", range(10))
def test_localization_gate_count_lemma1(case):
    """Lemma 1: localizing a Pauli takes at most N - 1 CNOTs from the pivot,
    N - 1 CZs, one S and one H, so every run of virtual Clifford gates that
    precedes a rotation or measurement has at most 2N gates."""
    rng = np.random.default_rng(2100 + case)
    n = int(rng.integers(2, 9))
    prog = oracle.Program(random_small_circuit(rng, n, 80))
    vg = {oracle.OP_NAMES.index(k) for k in ("VCX", "VCZ", "VS", "VH")}
    run = longest = 0
    for kind, _, _, _ in prog.ops():
        if kind in vg:
            run += 1
            longest = max(longest, run)
        else:
            run = 0
    assert longest <= 2 * n, (longest, n)
