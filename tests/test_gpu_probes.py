"""Expectation-value probes on the GPU (clifft_sample_expval): per shot the
value <psi|P|psi> at the probe, against the oracle's on the same shots
(same seed, so the same trajectory when the records agree): within 1e-12 in
FP64 and 2e-5 in FP32; the T-state values of Appendix C exactly; and with
the HIR passes the probes' means within 5 standard errors of the
oracle's."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_2604_27058_amd as pk
from test_gpu_parity import u64
from test_oracle_pins import random_wide_circuit

pytestmark = pytest.mark.gpu

TIERS = [(0, 0), (1, -1), (1, 1), (64, -1), (64, 1), (256, -1), (256, 1)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    yield


def gpu_probes(p, shots, seed, precision, G=0, hbm=0):
    L = pk.make_launch(precision, threads_per_shot=G, vector_in_hbm=hbm)
    (m, d, o), ev = p.sample_expval(shots, seed=seed, launch=L)
    torch.cuda.synchronize()
    return (u64(m), u64(d), u64(o)), ev.cpu().numpy()


def test_probes_t_state_exact():
    text = "H 0\nT 0\nEXP_VAL X0 Y0 Z0\nH 1\nT_DAG 1\nCX 1 2\nEXP_VAL Y1*X2 Z1*Z2\n"
    p = pk.Program(text)
    assert p.num_probes == 5
    r = 1 / math.sqrt(2)
    for prec, tol in (("f64", 1e-15), ("f32", 1e-7)):
        _, ev = gpu_probes(p, 1000, 0, prec)
        want = np.array([r, r, 0.0, -r, 1.0])[:, None]
        assert np.max(np.abs(ev - want)) <= tol, prec


@pytest.mark.parametrize("G,hbm", TIERS)
def test_probes_match_oracle_per_shot_fp64(G, hbm):
    worst = 0.0
    for case in range(8):
        rng = np.random.default_rng(8700 + case)
        text = random_wide_circuit(rng, int(rng.integers(2, 6)), int(rng.integers(15, 40)), probes=True)
        op = oracle.Program(text)
        if op.nprobes == 0:
            continue
        shots = 700
        om, od, oo, oev = op.sample(shots, seed=case, threads=8, expvals=True)
        (gm, gd, go), gev = gpu_probes(pk.Program(text), shots, case, "f64", G, hbm)
        assert np.array_equal(gm, om), case
        worst = max(worst, float(np.max(np.abs(gev - oev))))
    print("worst probe difference %.3g" % worst)
    assert worst <= 1e-12


def test_probes_match_oracle_fp32():
    worst = 0.0
    for case in range(8):
        rng = np.random.default_rng(8800 + case)
        text = random_wide_circuit(rng, int(rng.integers(2, 6)), int(rng.integers(15, 40)), probes=True)
        op = oracle.Program(text)
        if op.nprobes == 0:
            continue
        shots = 2000
        om, _, _, oev = op.sample(shots, seed=case, threads=8, expvals=True)
        (gm, _, _), gev = gpu_probes(pk.Program(text), shots, case, "f32")
        # shots whose records agree followed the same trajectory
        same = np.ones(shots, bool)
        if om.size:
            diff = np.bitwise_or.reduce(om ^ gm, axis=0)
            bits = np.unpackbits(diff.view(np.uint8), bitorder="little")[:shots].astype(bool)
            same &= ~bits
        worst = max(worst, float(np.max(np.abs(gev[:, same] - oev[:, same]))))
    print("worst FP32 probe difference %.3g" % worst)
    assert worst <= 2e-5


@pytest.mark.parametrize("passes", [1, 3])
def test_probe_means_with_hir_passes(passes):
    shots = 100_000
    for case in range(4):
        rng = np.random.default_rng(8900 + case)
        text = random_wide_circuit(rng, 4, 30, probes=True)
        op = oracle.Program(text)
        if op.nprobes == 0:
            continue
        _, _, _, oev = op.sample(shots, seed=2, threads=8, expvals=True)
        _, gev = gpu_probes(pk.Program(text, hir_passes=passes), shots, 1, "f64")
        for i in range(op.nprobes):
            se = math.sqrt((np.var(oev[i]) + np.var(gev[i])) / shots) + 1e-12
            assert abs(np.mean(gev[i]) - np.mean(oev[i])) <= 5 * se + 1e-9, (case, i)
