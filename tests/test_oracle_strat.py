"""Pins of the oracle's stratified fault sampling and post-selection.

Section 3.2 (rare-event sampling): shots are conditioned on a fixed number r
of realized faults and weighted by the Poisson-binomial probability of that
count; (post-selection): a shot whose post-selected detector fires ends at
once.  The oracle is checked against exhaustive enumeration of fault
configurations on small circuits, against the binomial closed forms when
every site has the same probability, and against a brute-force Python
implementation of the same inverse-transform draws (its own Philox and
survival function by enumeration).
"""
import itertools
import math

import numpy as np
import pytest

import dense_ref
import oracle
from paper_2604_27058_amd import circuits
from stats import popcount_rows, within_sigma

# Seven noise sites of different probabilities and channels; every
# measurement is deterministic given the faults.
TINY = """R 0 1 2
X_ERROR(0.1) 0
X_ERROR(0.25) 1
DEPOLARIZE1(0.2) 2
CX 0 1
X_ERROR(0.05) 1
DEPOLARIZE2(0.3) 1 2
Z_ERROR(0.15) 0
X_ERROR(0.4) 2
M 0 1 2
DETECTOR rec[-3]
DETECTOR rec[-2] rec[-3]
OBSERVABLE_INCLUDE(0) rec[-1]
"""
TINY_P = [0.1, 0.25, 0.2, 0.05, 0.3, 0.15, 0.4]
TINY_NOUT = [1, 1, 3, 1, 15, 1, 1]
PURPOSE_STRAT = 0x53000000


def _subsets_prob(ps, lo=0):
    """{frozenset of fired sites in [lo, N): probability} over all subsets."""
    n = len(ps)
    out = {}
    for bits in itertools.product((0, 1), repeat=n - lo):
        pr = 1.0
        for i, b in enumerate(bits):
            pr *= ps[lo + i] if b else 1.0 - ps[lo + i]
        out[frozenset(lo + i for i, b in enumerate(bits) if b)] = pr
    return out


def _surv_bf(ps, s, j, t):
    """P(no fault in [j, t) | exactly s faults in [j, N)) by enumeration."""
    sub = _subsets_prob(ps, j)
    tot = sum(pr for f, pr in sub.items() if len(f) == s)
    good = sum(pr for f, pr in sub.items() if len(f) == s and (not f or min(f) >= t))
    return good / tot


def test_tiny_site_probabilities():
    o = oracle.Program(TINY)
    assert o.nsites == len(TINY_P)
    S = o.survival(0)
    np.testing.assert_allclose(1.0 - S[1:] / S[:-1], TINY_P, rtol=1e-12)


def test_fault_pmf_matches_enumeration():
    """Poisson-binomial pmf of the fault count: exhaustive sum over subsets."""
    o = oracle.Program(TINY)
    pmf = o.fault_pmf(len(TINY_P) + 2)
    sub = _subsets_prob(TINY_P)
    for r in range(len(TINY_P) + 3):
        exact = sum(pr for f, pr in sub.items() if len(f) == r)
        assert abs(pmf[r] - exact) <= 1e-15 + 1e-13 * exact
    assert abs(pmf.sum() - 1.0) < 1e-13
    assert abs(float(np.dot(np.arange(len(pmf)), pmf)) - sum(TINY_P)) < 1e-13


def test_fault_pmf_equal_p_is_binomial():
    n, p = 40, 0.01
    o = oracle.Program("X_ERROR(%r) %s\nM %s\n" % (p, " ".join(map(str, range(n))), " ".join(map(str, range(n)))))
    pmf = o.fault_pmf(12)
    for r in range(13):
        b = math.comb(n, r) * p ** r * (1 - p) ** (n - r)
        assert abs(pmf[r] - b) <= 1e-13 * b + 1e-300


def test_strat_survival_matches_enumeration():
    o = oracle.Program(TINY)
    n = len(TINY_P)
    for s in (1, 2, 3):
        for j in range(n - s + 1):
            for t in range(j, n + 1):
                got = o.strat_survival(s, j, t)
                want = _surv_bf(TINY_P, s, j, t)
                assert abs(got - want) < 1e-13, (s, j, t, got, want)


def test_strat_survival_equal_p_closed_form():
    """Equal probabilities: the conditioned fault set is a uniform s-subset,
    so P(next fault >= t) = C(N - t, s) / C(N - j, s)."""
    n = 12
    o = oracle.Program("X_ERROR(0.03) %s\nM %s\n" % (" ".join(map(str, range(n))), " ".join(map(str, range(n)))))
    for s in (1, 2, 4):
        for j in (0, 3, 7):
            if n - j < s:
                continue
            for t in range(j, n + 1):
                want = math.comb(n - t, s) / math.comb(n - j, s)
                assert abs(o.strat_survival(s, j, t) - want) < 1e-13


def _faults_strat_bf(ps, nout, r, seed, shot):
    """The draw contract written out by brute force: fault i from draw i
    (purpose STRAT); next site = smallest t >= j with survival(t + 1) <= u;
    fired Pauli = floor(word64 * nout / 2^64) of the same draw."""
    n = len(ps)
    out = [-1] * n
    j = 0
    for i in range(r):
        w = dense_ref.draw(i, PURPOSE_STRAT, shot, seed)
        u = dense_ref.u53(w)
        left = r - i
        t = j
        while t < n - 1 and _surv_bf(ps, left, j, t + 1) > u:
            t += 1
        w64 = (int(w[3]) << 32) | int(w[2])
        out[t] = (w64 * nout[t]) >> 64
        j = t + 1
    return out


@pytest.mark.parametrize("r", [1, 2, 3])
def test_strat_draws_equal_brute_force(r):
    o = oracle.Program(TINY)
    for shot in range(120):
        got = list(o.faults_strat(r, seed=11, shot=shot))
        assert got == _faults_strat_bf(TINY_P, TINY_NOUT, r, 11, shot), shot


def test_strat_fault_set_distribution():
    """20000 shots of r = 2: each has exactly two faults, every fault set
    occurs at its conditional probability (5 sigma), and the fired Pauli of
    a depolarizing site is uniform over its outcomes."""
    o = oracle.Program(TINY)
    r, n_shots = 2, 20000
    counts = {}
    outs = {2: np.zeros(3), 4: np.zeros(15)}
    for shot in range(n_shots):
        f = o.faults_strat(r, seed=5, shot=shot)
        fired = frozenset(int(i) for i in np.nonzero(f >= 0)[0])
        assert len(fired) == r
        counts[fired] = counts.get(fired, 0) + 1
        for s in (2, 4):
            if f[s] >= 0:
                outs[s][f[s]] += 1
    sub = _subsets_prob(TINY_P)
    tot = sum(pr for f, pr in sub.items() if len(f) == r)
    for f, pr in sub.items():
        if len(f) == r:
            assert within_sigma(counts.get(f, 0), n_shots, pr / tot), (sorted(f), counts.get(f, 0), pr / tot)
    for s, c in outs.items():
        m = int(c.sum())
        for k in c:
            assert within_sigma(int(k), m, 1.0 / len(c))


def _enumerate_records(text, ps, nout):
    """Every fault configuration (site -> outcome or -1) with its
    probability and the oracle's deterministic detector / observable values
    under it (forced faults)."""
    o = oracle.Program(text)
    rows = []
    choices = [[-1] + list(range(k)) for k in nout]
    for cfg in itertools.product(*choices):
        pr = 1.0
        for s, c in enumerate(cfg):
            pr *= (1.0 - ps[s]) if c < 0 else ps[s] / nout[s]
        t = o.trace(seed=0, shot=0, forced_faults=np.array(cfg, np.int32))
        assert t["error"] == 0
        rows.append((pr, sum(c >= 0 for c in cfg), np.array(t["dets"]), np.array(t["obs"])))
    return rows


@pytest.mark.parametrize("r", [1, 2, 3])
def test_strat_record_rates_match_enumeration(r):
    """Detector and observable rates of 20000 stratified shots within 5 sigma
    of E[record | r faults] computed over all 1024 fault configurations."""
    rows = _enumerate_records(TINY, TINY_P, TINY_NOUT)
    tot = sum(pr for pr, k, _, _ in rows if k == r)
    det_p = sum(pr * d for pr, k, d, _ in rows if k == r) / tot
    obs_p = sum(pr * b for pr, k, _, b in rows if k == r) / tot
    n = 20000
    o = oracle.Program(TINY)
    _, det, obs = o.sample(n, seed=9, threads=4, faults=r)
    for row, p in zip(popcount_rows(det, n), det_p):
        assert within_sigma(int(row), n, float(p))
    for row, p in zip(popcount_rows(obs, n), obs_p):
        assert within_sigma(int(row), n, float(p))


def test_strat_impossible_stratum():
    o = oracle.Program(TINY)
    with pytest.raises(oracle.OracleError):
        o.sample(64, seed=1, faults=len(TINY_P) + 1)
    with pytest.raises(oracle.OracleError):
        o.faults_strat(len(TINY_P) + 1, 0, 0)
    z = oracle.Program("X_ERROR(1e-300) 0\nX_ERROR(0.5) 1\nM 0 1\n")
    assert z.nsites == 2 and abs(z.fault_pmf(2)[2]) < 1e-299
    for shot in range(50):
        assert list(z.faults_strat(1, 3, shot)) == [-1, 0]  # a (nearly) impossible site does not fire


def test_strat_zero_faults_is_noiseless():
    text = circuits.surface_code_memory(d=3, rounds=2, p=0.01)
    o = oracle.Program(text)
    _, det, obs = o.sample(256, seed=4, threads=2, faults=0)
    assert not det.any() and not obs.any()


# ---------------------------------------------------------------- post-selection
def _records_before_detectors(text):
    """Number of measurement records created before each DETECTOR."""
    nrec, out = 0, []
    for name, _arg, tg in dense_ref.parse(text):
        if name in ("M", "MX", "MY", "MR", "MPP"):
            nrec += len(tg)
        elif name == "DETECTOR":
            out.append(nrec)
    return out


def _bits(words, n):
    return np.unpackbits(words.view(np.uint8), axis=1, bitorder="little")[:, :n]


@pytest.mark.parametrize("which", ["all", "even"])
def test_postselect_truncates_shots(which):
    """Post-selection changes no draw: a shot whose post-selected detectors
    all read 0 keeps every record of the plain run; otherwise the records
    up to the first firing post-selected detector (inclusive) are those of
    the plain run and everything after, observables included, is 0."""
    text = circuits.surface_code_memory(d=3, rounds=3, p=0.02, t_rotations=2, seed=1)
    plain = oracle.Program(text)
    ps_idx = list(range(plain.ndet)) if which == "all" else list(range(0, plain.ndet, 2))
    post = oracle.Program(text, postselect=which if which == "all" else ps_idx)
    n = 4096
    a = [_bits(x, n) for x in plain.sample(n, seed=21, threads=4)]
    b = [_bits(x, n) for x in post.sample(n, seed=21, threads=4)]
    before = _records_before_detectors(text)
    kept = 0
    for s in range(n):
        fired = [d for d in ps_idx if a[1][d, s]]
        if not fired:
            kept += 1
            for x, y in zip(a, b):
                assert np.array_equal(x[:, s], y[:, s])
            continue
        d0 = fired[0]
        assert np.array_equal(b[1][: d0 + 1, s], a[1][: d0 + 1, s]) and not b[1][d0 + 1:, s].any()
        m0 = before[d0]
        assert np.array_equal(b[0][:m0, s], a[0][:m0, s]) and not b[0][m0:, s].any()
        assert not b[2][:, s].any()
    assert 0 < kept < n


# the observable accumulated before the post-selected detectors
TINY_OBS_FIRST = TINY.replace("OBSERVABLE_INCLUDE(0) rec[-1]\n", "").replace(
    "M 0 1 2\n", "M 0 1 2\nOBSERVABLE_INCLUDE(0) rec[-1]\n")


@pytest.mark.parametrize("text", [TINY, TINY_OBS_FIRST], ids=["obs_last", "obs_first"])
def test_postselect_kept_rate_matches_enumeration(text):
    """P(kept) and the observable rate among kept shots, post-selecting on
    detector 0 of the tiny circuit: exact over all fault configurations.
    Rejected shots read 0 on the later detector and on the observable, also
    when the observable was accumulated before the rejecting detector."""
    rows = _enumerate_records(text, TINY_P, TINY_NOUT)
    p_keep = sum(pr for pr, _, d, _ in rows if d[0] == 0)
    p_obs_keep = sum(pr * b[0] for pr, _, d, b in rows if d[0] == 0) / p_keep
    n = 40000
    o = oracle.Program(text, postselect=[0])
    _, det, obs = o.sample(n, seed=13, threads=4)
    d = _bits(det, n)
    b = _bits(obs, n)
    keep = d[0] == 0
    assert within_sigma(int(keep.sum()), n, p_keep)
    assert within_sigma(int(b[0][keep].sum()), int(keep.sum()), p_obs_keep)
    assert not b[0][~keep].any() and not d[1][~keep].any()


def test_postselect_mask_checked():
    with pytest.raises(oracle.OracleError):
        oracle.Program(TINY, postselect=[5])
