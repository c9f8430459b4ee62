"""Host checks of the optimisation passes on the Heisenberg representation
(Section 3.1, middle end): lowering through the representation without
passes gives the one-sweep program; the peephole pass fuses rotations about
one generator and absorbs their Clifford part (noiseless mirror circuits
U U^dagger become Clifford, k_max = 0); the reorder pass moves measurements
ahead of the rotations they commute with (the worked example of Figure 4);
neither pass raises k_max."""
import os

import numpy as np
import pytest

import paper_2604_27058_amd as pk
from paper_2604_27058_amd import circuits
from test_oracle_pins import random_small_circuit

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fingerprint(p):
    return (p.info, p.k_profile(), p.event_classes(), p.final_slots(), p.cost_model("f32"))


@pytest.mark.parametrize("case", range(20))
def test_lowering_through_the_representation_is_the_plain_program(case):
    rng = np.random.default_rng(7100 + case)
    text = random_small_circuit(rng, int(rng.integers(2, 7)), int(rng.integers(10, 60)))
    assert _fingerprint(pk.Program(text, hir_passes=4)) == _fingerprint(pk.Program(text))


def test_lowering_through_the_representation_workloads():
    for name in ("random_clifford_t_n8", "surface_d5_r5_t10"):
        text = circuits.workload(name)["texts"][0]
        assert _fingerprint(pk.Program(text, hir_passes=4)) == _fingerprint(pk.Program(text))


def _mirror(rng, n, layers):
    """U then U^dagger for a random Clifford+T+R_Z circuit U."""
    ops = []
    for _ in range(layers):
        q = int(rng.integers(0, n))
        r = rng.random()
        if r < 0.25:
            ops.append(("H", q))
        elif r < 0.4:
            ops.append(("S", q))
        elif r < 0.6 and n > 1:
            a, b = [int(x) for x in rng.choice(n, 2, replace=False)]
            ops.append(("CX", a, b))
        elif r < 0.85:
            ops.append(("T", q))
        else:
            ops.append(("R_Z", q, float(rng.uniform(-3, 3))))
    inv = {"H": "H", "S": "S_DAG", "T": "T_DAG", "CX": "CX"}
    lines = []
    for o in ops:
        lines.append("R_Z(%r) %d" % (o[2], o[1]) if o[0] == "R_Z" else "%s %s" % (o[0], " ".join(map(str, o[1:]))))
    for o in reversed(ops):
        lines.append("R_Z(%r) %d" % (-o[2], o[1]) if o[0] == "R_Z" else "%s %s" % (inv[o[0]], " ".join(map(str, o[1:]))))
    lines.append("M " + " ".join(map(str, range(n))))
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("case", range(12))
def test_peephole_makes_noiseless_mirror_circuits_clifford(case):
    rng = np.random.default_rng(7300 + case)
    text = _mirror(rng, int(rng.integers(2, 6)), int(rng.integers(5, 25)))
    p = pk.Program(text, hir_passes=1)
    assert p.k_max == 0
    assert p.event_classes() == [0] * p.num_events  # every outcome determined


def test_figure4_example():
    """The worked example: T T T on one generator fuse into one T rotation
    and an absorbed Clifford (the interfering measurement then carries an S
    pass), and the measurement of qubit 1 moves ahead of the T_DAG rotation
    and of the measurement of qubit 0."""
    text = open(os.path.join(GOLDEN, "mirror_example.stim")).read()
    plain = pk.Program(text)
    opt = pk.Program(text, hir_passes=3)
    assert plain.k_max == opt.k_max == 1
    assert opt.event_classes() == plain.event_classes() == [2, 0]
    assert opt.cost_model("f64")["flops"] < plain.cost_model("f64")["flops"]
    # the dormant static measurement (event 1) now runs while the active
    # qubit is still expanded
    kp = opt.k_profile()
    assert kp == [1, 1, 1, 1, 1, 1, 0, 0]
    assert pk.Program(text, hir_passes=1).k_profile() == [1, 1, 1, 1, 1, 0, 0, 0]


@pytest.mark.parametrize("passes", [1, 2, 3])
def test_passes_never_raise_k_max(passes):
    for case in range(120):
        rng = np.random.default_rng(7500 + case)
        text = random_small_circuit(rng, int(rng.integers(2, 7)), int(rng.integers(10, 60)))
        assert pk.Program(text, hir_passes=passes).k_max <= pk.Program(text).k_max
