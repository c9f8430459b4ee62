"""Sampling calls captured in a HIP graph (torch.cuda.CUDAGraph over the
library's stream argument) and replayed: every replay must write the records
of the eager call.  The program upload and the one-time kernel attributes
happen in an eager warm-up, so the captured call holds kernel nodes only
(record zero-fill is a kernel, never a memset node)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2604_27058_amd as pk
from paper_2604_27058_amd import circuits
from test_oracle_pins import random_small_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    yield


def snapshot(outs, sizes=None):
    """Host copies of the outputs (only the first sizes[i] words of each, if
    given: a batch with no detectors still gets a one-word placeholder)."""
    got = [o.cpu().numpy().reshape(-1).copy() for o in outs]
    return got if sizes is None else [g[:n] for g, n in zip(got, sizes)]


def capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()  # warm-up on a side stream (upload, kernel attributes)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def replay_and_check(g, outs, ref, replays=3, sizes=None):
    for r in range(replays):
        for o in outs:
            o.fill_(-1)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = snapshot(outs, sizes)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), "replay %d differs from the eager call" % r


CASES = [
    ("surface d3 bit-sliced", lambda: circuits.surface_code_memory(3, 3, 1e-3), dict(threads_per_shot=-32), 50000),
    ("surface d3 specialized", lambda: circuits.surface_code_memory(3, 3, 1e-3),
     dict(threads_per_shot=-32, specialize=1), 50000),
    ("surface d3 shot per workgroup", lambda: circuits.surface_code_memory(3, 2, 1e-3), dict(threads_per_shot=256),
     3000),
    ("random k<=4 shot per lane FP64", lambda: random_small_circuit(np.random.default_rng(77), 7, 60),
     dict(precision="f64", threads_per_shot=1), 5000),
    ("surface d5 + 10 T, HBM vectors", lambda: circuits.workload("surface_d5_r5_t10")["texts"][0],
     dict(threads_per_shot=1, vector_in_hbm=1), 4096),
]


@pytest.mark.parametrize("name,make,launch,shots", CASES, ids=[c[0] for c in CASES])
def test_sample_graph_replay(name, make, launch, shots):
    print("graph case:", name, flush=True)
    p = pk.Program(make())
    L = pk.make_launch(**launch)
    outs = tuple(o.fill_(-1) for o in p.alloc_outputs(shots))
    ws = p.alloc_workspace(L, shots=shots)
    p.sample(shots, seed=9, launch=L, outputs=outs, workspace=ws)
    torch.cuda.synchronize()
    ref = snapshot(outs)
    g = capture(lambda: p.sample(shots, seed=9, launch=L, outputs=outs, workspace=ws))
    replay_and_check(g, outs, ref)


def test_batch_graph_replay():
    print("graph case: batched launch", flush=True)
    cs = circuits.batched_set(count=6, seed=4100)
    progs = [pk.Program(c["text"]) for c in cs]
    shots = [700 + 61 * i for i in range(len(progs))]
    seeds = [3 + i for i in range(len(progs))]
    B = pk.Batch(progs, shots, seeds, precision="f32")
    outs, ws = B.alloc()
    for o in outs:
        o.fill_(-1)
    B.sample(outs, ws)
    torch.cuda.synchronize()
    sizes = (B.meas_words, B.det_words, B.obs_words)
    ref = snapshot(outs, sizes)
    g = capture(lambda: B.sample(outs, ws))
    replay_and_check(g, outs, ref, sizes=sizes)
