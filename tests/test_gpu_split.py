"""The split form on the GPU: the Pauli frames of every shot run bit-sliced
with the active outcomes taken as 0, then the vector instructions alone, then
a fix-up XORs the outcomes into the records that depend on them (records and
the frame bits the vector reads are affine over GF(2) in the outcomes).
Records must equal the oracle's: bit for bit with FP64 amplitudes, up to the
derived near-threshold bound with FP32."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_2604_27058_amd as pk
from paper_2604_27058_amd import circuits
from test_gpu_parity import fp32_mismatch_bound, gpu_sample, mismatched_shots
from test_oracle_pins import random_small_circuit

pytestmark = pytest.mark.gpu

TIERS = [(1, -1), (1, 1), (64, -1), (64, 1), (256, -1), (256, 1)]  # vector pass: (threads per shot, in HBM)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    yield


def split_sample(text, shots, seed=0, offset=0, precision="f64", G=0, hbm=0, grid=0):
    return gpu_sample(text, shots, seed=seed, offset=offset, precision=precision, threads_per_shot=G,
                      vector_in_hbm=hbm, grid=grid, split=1)


@pytest.mark.parametrize("G,hbm", TIERS)
def test_split_random_circuits_fp64_bit_exact(G, hbm):
    """Random circuits with every gate, noise type, reset, detector, MX and
    rotations (active Z and X measurements, dormant random ones, resets of
    active qubits), split form on each vector-pass tier."""
    for case in range(8):
        rng = np.random.default_rng(2100 + case)
        text = random_small_circuit(rng, int(rng.integers(2, 6)), int(rng.integers(15, 50)))
        if pk.Program(text).k_max == 0:
            continue
        shots = 1000 + 7 * case
        print("case", case, flush=True)
        om, od, oo = oracle.Program(text).sample(shots, seed=case, threads=8)
        gm, gd, go = split_sample(text, shots, seed=case, G=G, hbm=hbm)
        assert np.array_equal(gm, om) and np.array_equal(gd, od) and np.array_equal(go, oo), case


@pytest.mark.parametrize("G,hbm", [(0, 0), (1, -1), (64, -1), (64, 1), (256, 1)])
def test_split_clifford_t_n8_fp64(G, hbm):
    w = circuits.workload("random_clifford_t_n8")
    text = w["texts"][0]
    om, od, oo = oracle.Program(text).sample(w["shots"], seed=0, threads=8)
    gm, gd, go = split_sample(text, w["shots"], seed=0, G=G, hbm=hbm)
    assert np.array_equal(gm, om)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("G,hbm", [(0, 0), (64, -1), (64, 1), (256, 1)])
def test_split_surface_d5_t10(precision, G, hbm):
    """The d = 5 + 10 T workload: 120 detectors and the observable depend on
    the active outcomes of the round after the T layer through the fix-up."""
    text = circuits.workload("surface_d5_r5_t10")["texts"][0]
    shots = 8192 + 5
    om, od, oo = oracle.Program(text).sample(shots, seed=3, threads=8)
    gm, gd, go = split_sample(text, shots, seed=3, precision=precision, G=G, hbm=hbm)
    bad = mismatched_shots(np.vstack([om, od, oo]), np.vstack([gm, gd, go]), shots)
    bound = 0 if precision == "f64" else fp32_mismatch_bound(text, shots, seed=3)
    print("split d5 %s G=%d: %d shots differ (bound %d)" % (precision, G, bad, bound))
    assert bad <= bound


def test_split_batched_set_programs_fp64():
    """Programs of the batched set (k_max 4..16, W = 1 and 2, mid-circuit
    resets of active qubits), default split tier, against the oracle."""
    specs = circuits.batched_set(count=10, seed=4200)
    for i, c in enumerate(specs):
        n = 512 if c["k"] <= 12 else 64
        om, od, oo = oracle.Program(c["text"]).sample(n, seed=i, threads=8)
        gm, gd, go = split_sample(c["text"], n, seed=i)
        assert np.array_equal(gm, om), (i, c["k"])


def test_split_shards_join():
    text = circuits.workload("surface_d5_r5_t10")["texts"][0]
    a = split_sample(text, 4096, seed=5)
    b = split_sample(text, 2048, seed=5, offset=0)
    c = split_sample(text, 2048, seed=5, offset=2048)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, np.concatenate([y, z], axis=1))


def test_split_k20_fp64_few_shots():
    text = circuits.workload("large_active_k20")["texts"][0]
    shots = 4
    om, _, _ = oracle.Program(text).sample(shots, seed=0, threads=4)
    gm, _, _ = split_sample(text, shots, seed=0, G=256, hbm=1)
    assert mismatched_shots(om, gm, shots) == 0


def test_split_equals_whole_program_large():
    """At the benchmark's shot count the split form's FP64 records equal the
    whole-program interpreter's word for word."""
    text = circuits.workload("surface_d5_r5_t10")["texts"][0]
    shots = 1_000_000
    p = pk.Program(text)
    a = gpu_sample(p, shots, seed=7, precision="f64", split=-1)
    b = gpu_sample(p, shots, seed=7, precision="f64", split=1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
