"""The wider gate set on the GPU (R_X, R_Y, U3, rotations about Pauli
products, product measurements MPP, record-controlled Paulis): records equal
the oracle's bit for bit in FP64 on every tier and in the split form, within
the derived near-threshold bound in FP32, and forced shots give the oracle's
branch probabilities and gamma * phi."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_2604_27058_amd as pk
from test_gpu_parity import _forced_check, fp32_mismatch_bound, gpu_sample, mismatched_shots
from test_gpu_rates import failing_rows, host_threads
from test_oracle_pins import random_wide_circuit

pytestmark = pytest.mark.gpu

TIERS = [(1, -1), (1, 1), (64, -1), (64, 1), (256, -1), (256, 1)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    yield


def _case(case):
    rng = np.random.default_rng(8400 + case)
    return random_wide_circuit(rng, int(rng.integers(2, 6)), int(rng.integers(15, 45)))


@pytest.mark.parametrize("G,hbm", TIERS)
def test_wide_records_fp64_every_tier(G, hbm):
    for case in range(8):
        text = _case(case)
        shots = 900 + 11 * case
        om, od, oo = oracle.Program(text).sample(shots, seed=case, threads=8)
        gm, gd, go = gpu_sample(text, shots, seed=case, precision="f64", threads_per_shot=G, vector_in_hbm=hbm)
        assert np.array_equal(gm, om) and np.array_equal(gd, od) and np.array_equal(go, oo), case


def test_wide_records_split_and_fp32():
    for case in range(8):
        text = _case(case)
        shots = 2000
        om, od, oo = oracle.Program(text).sample(shots, seed=case, threads=8)
        if pk.Program(text).k_max > 0:
            gm, gd, go = gpu_sample(text, shots, seed=case, precision="f64", split=1)
            assert np.array_equal(gm, om) and np.array_equal(gd, od), case
        gm, gd, go = gpu_sample(text, shots, seed=case, precision="f32")
        ref = np.vstack([x for x in (om, od, oo) if x.size])
        got = np.vstack([x for x in (gm, gd, go) if x.size])
        assert mismatched_shots(ref, got, shots) <= fp32_mismatch_bound(text, shots, seed=case), case


@pytest.mark.parametrize("case", range(6))
@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-5)])
@pytest.mark.parametrize("tier", [None, (1, 1), (256, 1)], ids=["auto", "lane-hbm", "group-hbm"])
def test_wide_forced_probabilities_and_state(case, precision, tol, tier):
    rng = np.random.default_rng(8500 + case)
    text = _case(case + 20).rsplit("M ", 1)[0]  # keep the final vector
    _forced_check(text, case, precision, tol, tier, rng)


def test_wide_hir_passes_rates():
    shots = 200_000
    bad = []
    for case in range(5):
        text = _case(case + 40)
        g = gpu_sample(pk.Program(text, hir_passes=3), shots, seed=1, precision="f64")
        o = oracle.Program(text).sample(shots, seed=2, threads=host_threads())
        bad += [(case,) + b for b in failing_rows(g, shots, o, shots)]
    print("rows failing 5 sigma:", bad)
    assert not bad
