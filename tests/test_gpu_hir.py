"""The optimisation passes on the Heisenberg representation (Section 3.1,
middle end) validated against the unoptimized oracle: rates of every record
within 5 sigma (two samples of different seeds), and along forced
trajectories the probabilities of the forced outcomes -- event by event for
the peephole pass (which keeps the order of measurements), and as the joint
probability of the whole outcome sequence once measurements are reordered."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_2604_27058_amd as pk
from paper_2604_27058_amd import circuits
from test_gpu_parity import gpu_sample
from test_gpu_rates import failing_rows, host_threads
from test_hir_cpu import _mirror
from test_oracle_pins import random_small_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    yield


def _cases():
    out = []
    for case in range(5):
        rng = np.random.default_rng(7700 + case)
        out.append(random_small_circuit(rng, int(rng.integers(3, 6)), int(rng.integers(20, 50))))
    for case in range(3):
        rng = np.random.default_rng(7800 + case)
        t = _mirror(rng, 4, 14).splitlines()
        # noise in the middle of the mirror keeps it non-Clifford
        mid = len(t) // 2
        t = t[:mid] + ["DEPOLARIZE1(0.05) 0 1 2 3"] + t[mid:]
        out.append("\n".join(t) + "\n")
    out.append(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                 "mirror_example.stim")).read().replace("0.001", "0.05"))
    return out


@pytest.mark.parametrize("passes", [1, 2, 3])
def test_hir_rates_match_unoptimized_oracle(passes):
    shots = 200_000
    bad = []
    for i, text in enumerate(_cases()):
        p = pk.Program(text, hir_passes=passes)
        g = gpu_sample(p, shots, seed=1, precision="f64")
        o = oracle.Program(text).sample(shots, seed=2, threads=host_threads())
        bad += [(i,) + b for b in failing_rows(g, shots, o, shots)]
    print("rows failing 5 sigma:", bad)
    assert not bad


def test_hir_rates_batched_programs():
    shots = 100_000
    pre = 4096
    bad = []
    for i, c in enumerate(circuits.batched_set(count=6, seed=4300)):
        p = pk.Program(c["text"], hir_passes=3)
        g = gpu_sample(p, shots, seed=i, precision="f32")
        o = oracle.Program(c["text"]).sample(pre, seed=i, threads=host_threads())
        bad += [(i,) + b for b in failing_rows(g, shots - pre, o, pre, gpu_first=pre)]
    print("rows failing 5 sigma:", bad)
    assert not bad


@pytest.mark.parametrize("passes", [1, 3])
def test_hir_forced_probabilities(passes):
    """Forced faults and outcomes of oracle shots (of the unoptimized
    circuit) replayed on the optimized program in FP64."""
    worst = 0.0
    for i, text in enumerate(_cases()):
        op = oracle.Program(text)
        gp = pk.Program(text, hir_passes=passes)
        if op.nevents == 0:
            continue
        shots = 8
        fm = np.zeros((shots, op.nevents), np.uint32)
        ff = np.full((shots, max(op.nsites, 1)), -1, np.int32)
        po = np.zeros((shots, op.nevents))
        for s in range(shots):
            faults = op.faults(i, s)
            t = op.trace(i, s, forced_faults=faults)
            fm[s], ff[s, : op.nsites], po[s] = t["m"], faults, t["probs"]
        res = gp.sample_trace(shots, seed=i, launch=pk.make_launch("f64"), forced_m=torch.from_numpy(fm),
                              forced_faults=torch.from_numpy(ff[:, : op.nsites]), want_phi=False)
        torch.cuda.synchronize()
        pg = res["probs"].cpu().numpy()
        m = fm.astype(bool)
        qg = np.where(m, pg, 1 - pg)
        qo = np.where(m, po, 1 - po)
        if passes == 1:
            err = float(np.max(np.abs(qg - qo)))
        else:
            jg, jo = qg.prod(axis=1), qo.prod(axis=1)
            err = float(np.max(np.abs(jg - jo) / jo))
        worst = max(worst, err)
    print("worst error %.3g" % worst)
    assert worst <= 1e-10
