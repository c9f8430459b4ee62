"""Post-selection and stratified fault sampling on the GPU (Section 3.2).

Post-selected programs (OP_POSTSELECT: a shot whose detector reads 1 ends
there) and stratified calls (clifft_sample_stratified: exactly r faults per
shot) against the oracle on the same shots: records bit for bit in FP64 on
every tier (shot per lane, wave and workgroup, vectors in LDS and HBM, the
bit-sliced kernel with its fault list, its per-shot cursors and its
list-overflow path, the batched launch), probes of rejected shots 0, and in
FP32 the rates within 5 sigma.  At any size: the stratified estimate
sum_r pmf(r) rate_r of a logical observable agrees with plain sampling
within 5 combined standard errors.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
import paper_2604_27058_amd as pk
from paper_2604_27058_amd import circuits
from stats import popcount_rows, two_sample_ok
from test_gpu_parity import u64

pytestmark = pytest.mark.gpu

# (threads_per_shot, vector_in_hbm)
TIERS_K = [(0, 0), (1, -1), (1, 1), (64, -1), (64, 1), (256, -1), (256, 1)]
TIERS_0 = [(-32, 0), (1, 0), (64, 0), (256, 0)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    yield


def _text_t(p=0.02):
    return circuits.surface_code_memory(d=3, rounds=3, p=p, t_rotations=2, seed=1)


def _text_0(p=0.02):
    return circuits.surface_code_memory(d=3, rounds=3, p=p)


def _gpu(p, shots, seed, precision="f64", G=0, hbm=0, faults=None):
    L = pk.make_launch(precision, threads_per_shot=G, vector_in_hbm=hbm)
    if faults is None:
        outs = p.sample(shots, seed=seed, launch=L)
    else:
        outs = p.sample_stratified(shots, faults, seed=seed, launch=L)
    torch.cuda.synchronize()
    return [u64(x) for x in outs]


def _assert_same(g, o, what):
    for name, a, b in zip(("meas", "det", "obs"), g, o):
        assert a.shape == b.shape, (what, name)
        bad = np.nonzero((a != b).any(axis=1))[0]
        assert bad.size == 0, "%s: %s rows differ: %s" % (what, name, bad[:8])


@pytest.mark.parametrize("which", ["all", "even"])
@pytest.mark.parametrize("G,hbm", TIERS_K)
def test_postselect_records_equal_oracle_active(which, G, hbm):
    text = _text_t()
    op0 = oracle.Program(text)
    ps = "all" if which == "all" else list(range(0, op0.ndet, 2))
    shots = 4096 + 37
    o = oracle.Program(text, postselect=ps).sample(shots, seed=3, threads=8)
    p = pk.Program(text, postselect=ps)
    assert p.k_max > 0 and p.num_postselected == (op0.ndet if which == "all" else len(ps))
    g = _gpu(p, shots, 3, "f64", G, hbm)
    _assert_same(g, o, "post %s G=%d hbm=%d" % (which, G, hbm))
    kept = popcount_rows(u64(p.kept(torch.from_numpy(g[1].view(np.int64)).cuda()).cpu()[None, :]), shots)[0]
    print("kept %d of %d" % (kept, shots))
    assert 0 < kept < shots


@pytest.mark.parametrize("G,hbm", TIERS_0)
def test_postselect_records_equal_oracle_frames(G, hbm):
    text = _text_0()
    shots = 3 * 2048 + 101
    o = oracle.Program(text, postselect="all").sample(shots, seed=5, threads=8)
    p = pk.Program(text, postselect="all")
    g = _gpu(p, shots, 5, "f64", G, hbm)
    _assert_same(g, o, "post k=0 G=%d" % G)


def test_postselect_probes_of_rejected_shots_are_zero():
    text = "H 0\nT 0\nX_ERROR(0.3) 1\nM 1\nDETECTOR rec[-1]\nEXP_VAL X0 Z0\nM 0\n"
    shots = 3000
    om, od, oo, oev = oracle.Program(text, postselect="all").sample(shots, seed=2, expvals=True)
    p = pk.Program(text, postselect="all")
    for G in (1, 64, 256):
        (m, d, b), ev = p.sample_expval(shots, seed=2, launch=pk.make_launch("f64", threads_per_shot=G))
        torch.cuda.synchronize()
        _assert_same([u64(m), u64(d), u64(b)], [om, od, oo], "probes G=%d" % G)
        ev = ev.cpu().numpy()
        assert np.max(np.abs(ev - oev)) <= 1e-15
        rejected = np.unpackbits(od.view(np.uint8), bitorder="little")[:shots].astype(bool)
        assert rejected.any() and not ev[:, rejected].any()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_postselect_batched_launch(precision):
    texts = [_text_t(), _text_0(), _text_t(0.01)]
    progs = [pk.Program(t, postselect="all") for t in texts]
    shots = [2048 + 17, 4096, 1000]
    seeds = [7, 8, 9]
    B = pk.Batch(progs, shots, seeds, precision=precision)
    outs = B.sample()
    torch.cuda.synchronize()
    for i, t in enumerate(texts):
        o = oracle.Program(t, postselect="all").sample(shots[i], seed=seeds[i], threads=8)
        g = [u64(x) for x in B.records(outs, i)]
        if precision == "f64" or progs[i].k_max == 0:
            _assert_same(g, o, "batch %d" % i)
        else:
            for a, b in zip(g, o):
                for r in range(a.shape[0]):
                    ka = popcount_rows(a[r:r + 1], shots[i])[0]
                    kb = popcount_rows(b[r:r + 1], shots[i])[0]
                    assert two_sample_ok(int(ka), shots[i], int(kb), shots[i])


@pytest.mark.parametrize("r", [0, 1, 3, 7])
@pytest.mark.parametrize("G,hbm", TIERS_K)
def test_stratified_records_equal_oracle_active(r, G, hbm):
    text = _text_t(0.01)
    shots = 2048 + 45
    o = oracle.Program(text).sample(shots, seed=11, threads=8, faults=r)
    g = _gpu(pk.Program(text), shots, 11, "f64", G, hbm, faults=r)
    _assert_same(g, o, "strat r=%d G=%d hbm=%d" % (r, G, hbm))


@pytest.mark.parametrize("r", [0, 2, 5, 20])
@pytest.mark.parametrize("G,hbm", TIERS_0)
def test_stratified_records_equal_oracle_frames(r, G, hbm):
    text = _text_0(0.01)
    shots = 2 * 2048 + 77
    o = oracle.Program(text).sample(shots, seed=12, threads=8, faults=r)
    g = _gpu(pk.Program(text), shots, 12, "f64", G, hbm, faults=r)
    _assert_same(g, o, "strat k=0 r=%d G=%d" % (r, G))


def test_stratified_bitsliced_list_overflow(monkeypatch):
    """The bit-sliced kernel's fault-list overflow path (capacity forced to
    8 entries per lane) re-draws the stratified faults statelessly."""
    text = _text_0(0.01)
    shots = 2048 + 5
    o = oracle.Program(text).sample(shots, seed=13, threads=8, faults=6)
    monkeypatch.setenv("CLIFFT_FRAMES_LIST_CAP", "8")
    g = _gpu(pk.Program(text), shots, 13, "f64", -32, 0, faults=6)
    _assert_same(g, o, "strat overflow")


def test_stratified_with_postselect():
    text = _text_t(0.01)
    shots = 4096
    for r in (1, 4):
        o = oracle.Program(text, postselect="all").sample(shots, seed=14, threads=8, faults=r)
        for G in (1, 256):
            g = _gpu(pk.Program(text, postselect="all"), shots, 14, "f64", G, 0, faults=r)
            _assert_same(g, o, "strat+post r=%d G=%d" % (r, G))


def test_stratified_full_size_d5_t10():
    """1e6 stratified shots (r = 4) of the d = 5 + 10 T workload: the FP64
    first 2048 shots equal the oracle's, and the FP32 rates of every record
    row are within 5 sigma of 20000 oracle shots of another seed."""
    text = circuits.workload("surface_d5_r5_t10")["texts"][0]
    p = pk.Program(text)
    pre = 2048
    g64 = _gpu(p, pre, 21, "f64", faults=4)
    _assert_same(g64, oracle.Program(text).sample(pre, seed=21, threads=16, faults=4), "d5 prefix")
    n = 1_000_000
    g32 = _gpu(p, n, 22, "f32", faults=4)
    no = 20000
    o = oracle.Program(text).sample(no, seed=23, threads=16, faults=4)
    bad = []
    for a, b in zip(g32, o):
        ka, kb = popcount_rows(a, n), popcount_rows(b, no)
        bad += [r for r in range(len(ka)) if not two_sample_ok(int(ka[r]), n, int(kb[r]), no)]
    assert not bad


def test_stratified_estimate_matches_plain_sampling():
    """sum_r pmf(r) P(obs = 1 | r) over the strata r <= R (pmf mass beyond R
    below 1e-9) against plain sampling of the same program: within 5
    combined standard errors (bit-sliced tier, k_max = 0, p = 0.02)."""
    text = _text_0(0.02)
    p = pk.Program(text)
    pmf = np.array(p.fault_count_pmf(80))
    R = int(np.nonzero(np.cumsum(pmf) > 1 - 1e-9)[0][0])
    n_r = 200_000
    est, var = 0.0, 0.0
    for r in range(R + 1):
        _, _, obs = _gpu(p, n_r, 100 + r, "f32", faults=r)
        k = popcount_rows(obs, n_r)[0]
        q = k / n_r
        est += pmf[r] * q
        var += pmf[r] ** 2 * max(q * (1 - q), 1.0 / n_r) / n_r
    n = 4_000_000
    _, _, obs = _gpu(p, n, 99, "f32")
    q = popcount_rows(obs, n)[0] / n
    se = np.sqrt(var + q * (1 - q) / n)
    print("strata 0..%d: stratified %.6f, plain %.6f, se %.2e" % (R, est, q, se))
    assert abs(est - q) <= 5 * se
