"""Seeded synthetic circuit generators (Stim-subset text).

These stand in for the paper's benchmark families (surface-code memory,
coherent / near-Clifford circuits, the large-k end of Table 1), whose circuit
files are not available here.  The module only writes circuit text: it holds
none of the simulation method's arithmetic, so both the oracle and the HIP
path may consume its output.

Conventions of the text format:
  T = exp(-i pi/8 Z), T_DAG = exp(+i pi/8 Z), R_Z(phi) = exp(-i phi Z / 2).
Noise model ("uniform circuit-level"): DEPOLARIZE1(p) after every one-qubit
unitary, DEPOLARIZE2(p) after every two-qubit gate, X_ERROR(p) before every
measurement; resets are noiseless.
"""
import math

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _fmt(p):
    return repr(float(p))


# --------------------------------------------------------------------------
# Rotated surface code, memory-Z experiment.
# --------------------------------------------------------------------------
class SurfaceLayout:
    """d x d data qubits at (r, c) -> index r*d + c; one ancilla per face.

    Face (i, j), 0 <= i, j <= d, touches data (i-1, j-1), (i-1, j), (i, j-1),
    (i, j) when in range.  Bulk faces have type X when (i + j) is even and Z
    otherwise; weight-2 faces are kept on the top/bottom edges when they are
    X-type and on the left/right edges when they are Z-type.  Logical Z_L is Z
    on data row 0.
    """

    def __init__(self, d):
        self.d = d
        faces = []
        for i in range(d + 1):
            for j in range(d + 1):
                typ = "X" if (i + j) % 2 == 0 else "Z"
                nw = (i - 1, j - 1)
                ne = (i - 1, j)
                sw = (i, j - 1)
                se = (i, j)
                inside = [q for q in (nw, ne, sw, se) if 0 <= q[0] < d and 0 <= q[1] < d]
                if len(inside) == 4:
                    pass
                elif len(inside) == 2:
                    top_bottom = i in (0, d)
                    if top_bottom and typ != "X":
                        continue
                    if not top_bottom and typ != "Z":
                        continue
                else:
                    continue
                # CNOT order: X faces NW, NE, SW, SE ("Z" shape); Z faces NW, SW, NE, SE ("N" shape)
                order = [nw, ne, sw, se] if typ == "X" else [nw, sw, ne, se]
                slots = [(q[0] * d + q[1]) if (0 <= q[0] < d and 0 <= q[1] < d) else None for q in order]
                faces.append((typ, slots))
        self.faces = faces
        self.ndata = d * d
        self.nq = d * d + len(faces)
        self.anc = [d * d + f for f in range(len(faces))]
        self.xfaces = [f for f, (t, _) in enumerate(faces) if t == "X"]
        self.zfaces = [f for f, (t, _) in enumerate(faces) if t == "Z"]
        self.logical_z = [c for c in range(d)]  # row 0
        self._check()

    def support(self, f):
        return [q for q in self.faces[f][1] if q is not None]

    def _check(self):
        d = self.d
        assert len(self.faces) == d * d - 1
        for f in self.xfaces:
            assert len(set(self.support(f)) & set(self.logical_z)) % 2 == 0
        for f in self.xfaces:
            for g in self.zfaces:
                assert len(set(self.support(f)) & set(self.support(g))) % 2 == 0

    def x_syndrome(self, q):
        return [1 if q in self.support(f) else 0 for f in self.xfaces]


def surface_code_memory(d=3, rounds=3, p=1e-3, t_rotations=0, t_after_round=2, seed=0, noise=True):
    """Memory-Z experiment; optionally `t_rotations` alternating T / T_DAG on
    distinct data qubits between rounds `t_after_round` and the next, chosen
    so their X-syndrome vectors are independent over GF(2)."""
    L = SurfaceLayout(d)
    out = []
    P = _fmt(p)
    nz = noise and p > 0

    def dep1(qs):
        if nz and qs:
            out.append("DEPOLARIZE1(%s) %s" % (P, " ".join(map(str, qs))))

    t_qubits = []
    if t_rotations:
        rng = _rng(seed)
        order = list(rng.permutation(L.ndata))
        basis = []
        for q in order:
            v = np.array(L.x_syndrome(int(q)), np.uint8)
            cand = basis + [v]
            if _gf2_rank(np.array(cand)) == len(cand):
                basis.append(v)
                t_qubits.append(int(q))
            if len(t_qubits) == t_rotations:
                break
        if len(t_qubits) < t_rotations:
            raise ValueError("not enough independent data qubits for %d rotations" % t_rotations)

    out.append("R " + " ".join(map(str, range(L.nq))))
    xa = [L.anc[f] for f in L.xfaces]
    prev = {}
    nmeas = 0
    for r in range(rounds):
        out.append("TICK")
        out.append("H " + " ".join(map(str, xa)))
        dep1(xa)
        for layer in range(4):
            pairs = []
            for f, (typ, slots) in enumerate(L.faces):
                q = slots[layer]
                if q is None:
                    continue
                a = L.anc[f]
                pairs += [a, q] if typ == "X" else [q, a]
            out.append("CX " + " ".join(map(str, pairs)))
            if nz:
                out.append("DEPOLARIZE2(%s) %s" % (P, " ".join(map(str, pairs))))
        out.append("H " + " ".join(map(str, xa)))
        dep1(xa)
        if nz:
            out.append("X_ERROR(%s) %s" % (P, " ".join(map(str, L.anc))))
        out.append("MR " + " ".join(map(str, L.anc)))
        na = len(L.anc)
        cur = {f: nmeas + i for i, f in enumerate(range(na))}
        nmeas += na
        for f in range(na):
            typ = L.faces[f][0]
            if r == 0:
                if typ == "Z":
                    out.append("DETECTOR rec[%d]" % (cur[f] - nmeas))
            else:
                out.append("DETECTOR rec[%d] rec[%d]" % (cur[f] - nmeas, prev[f] - nmeas))
        prev = cur
        if t_qubits and r + 1 == t_after_round:
            for i, q in enumerate(t_qubits):
                out.append(("T %d" if i % 2 == 0 else "T_DAG %d") % q)
                dep1([q])
    data = list(range(L.ndata))
    if nz:
        out.append("X_ERROR(%s) %s" % (P, " ".join(map(str, data))))
    out.append("M " + " ".join(map(str, data)))
    base = nmeas
    nmeas += L.ndata
    for f in L.zfaces:
        refs = ["rec[%d]" % (base + q - nmeas) for q in L.support(f)]
        refs.append("rec[%d]" % (prev[f] - nmeas))
        out.append("DETECTOR " + " ".join(refs))
    out.append("OBSERVABLE_INCLUDE(0) " + " ".join("rec[%d]" % (base + q - nmeas) for q in L.logical_z))
    return "\n".join(out) + "\n"


def _gf2_rank(M):
    M = np.array(M, np.uint8) % 2
    r = 0
    rows, cols = M.shape
    for c in range(cols):
        piv = next((i for i in range(r, rows) if M[i, c]), None)
        if piv is None:
            continue
        M[[r, piv]] = M[[piv, r]]
        for i in range(rows):
            if i != r and M[i, c]:
                M[i] ^= M[r]
        r += 1
        if r == rows:
            break
    return r


# --------------------------------------------------------------------------
# Random Clifford+T circuit (small correctness workload).
# --------------------------------------------------------------------------
def random_clifford_t(n=8, layers=40, n_t=4, p=1e-3, seed=0):
    """Each layer shuffles the qubits and gives every qubit one gate from
    {H, S, CNOT} (a CNOT consumes a partner).  `n_t` T gates sit on seeded
    (layer, qubit) slots after layer 1 (each placed right after an H on its
    qubit).  Noise after every gate; Z-basis measurement of all qubits."""
    rng = _rng(seed)
    P = _fmt(p)
    out = []
    slots = set()
    while len(slots) < n_t:
        slots.add((int(rng.integers(1, layers)), int(rng.integers(0, n))))
    for layer in range(layers):
        perm = list(rng.permutation(n))
        i = 0
        while i < n:
            q = int(perm[i])
            g = int(rng.integers(0, 3))
            if g == 2 and i + 1 < n:
                q2 = int(perm[i + 1])
                out.append("CX %d %d" % (q, q2))
                if p:
                    out.append("DEPOLARIZE2(%s) %d %d" % (P, q, q2))
                i += 2
                continue
            name = "H" if g == 0 or (g == 2) else "S"
            out.append("%s %d" % (name, q))
            if p:
                out.append("DEPOLARIZE1(%s) %d" % (P, q))
            i += 1
        for (l, q) in sorted(slots):
            if l == layer:
                out.append("H %d" % q)
                out.append("T %d" % q)
                if p:
                    out.append("DEPOLARIZE1(%s) %d %d" % (P, q, q))
    if p:
        out.append("X_ERROR(%s) %s" % (P, " ".join(map(str, range(n)))))
    out.append("M " + " ".join(map(str, range(n))))
    return "\n".join(out) + "\n"


# --------------------------------------------------------------------------
# Near-Clifford "magic register" circuits (batched set and large-k stress).
# --------------------------------------------------------------------------
def _clifford_layer(out, rng, qubits, P):
    perm = list(rng.permutation(qubits))
    i = 0
    while i < len(perm):
        q = int(perm[i])
        g = int(rng.integers(0, 3))
        if g == 2 and i + 1 < len(perm):
            q2 = int(perm[i + 1])
            out.append("CX %d %d" % (q, q2))
            if P:
                out.append("DEPOLARIZE2(%s) %d %d" % (P, q, q2))
            i += 2
            continue
        out.append("%s %d" % ("H" if g != 1 else "S", q))
        if P:
            out.append("DEPOLARIZE1(%s) %d" % (P, q))
        i += 1


def _nonclifford(out, rng, q, P, rz_frac):
    if rng.random() < rz_frac:
        out.append("R_Z(%r) %d" % (float(rng.uniform(0, 2 * math.pi)), q))
    else:
        out.append(("T %d" if rng.random() < 0.5 else "T_DAG %d") % q)
    if P:
        out.append("DEPOLARIZE1(%s) %d" % (P, q))


def register_circuit(n, depth, k_target, n_nonclifford, p, seed, rz_frac=0.5, mid_measure_every=0,
                     mid_measure_count=0):
    """The first `k_target` qubits form a magic register: H then a non-Clifford
    rotation on each of them (each one expands the active set), random
    Clifford layers on the register and on the rest (the two never interact),
    the remaining rotations on register qubits (inside the active set), and a
    final measurement of everything.  With `mid_measure_every` > 0, every that
    many layers `mid_measure_count` register qubits are measured and reset
    (contracting k) and re-expanded by H + T."""
    rng = _rng(seed)
    P = _fmt(p) if p else None
    reg = list(range(k_target))
    bulk = list(range(k_target, n))
    out = []
    used = 0
    for q in reg:
        out.append("H %d" % q)
        if P:
            out.append("DEPOLARIZE1(%s) %d" % (P, q))
        _nonclifford(out, rng, q, P, rz_frac)
        used += 1
    extra_slots = set()
    remaining = max(0, n_nonclifford - used)
    if mid_measure_every and mid_measure_count:
        remaining -= (depth - 1) // mid_measure_every * mid_measure_count
    remaining = max(0, remaining)
    while len(extra_slots) < remaining:
        extra_slots.add((int(rng.integers(0, depth)), int(rng.integers(0, k_target))))
    for layer in range(depth):
        _clifford_layer(out, rng, reg, P)
        if bulk:
            _clifford_layer(out, rng, bulk, P)
        for (l, q) in sorted(extra_slots):
            if l == layer:
                _nonclifford(out, rng, q, P, rz_frac)
        if mid_measure_every and layer > 0 and layer % mid_measure_every == 0 and layer < depth - 1:
            qs = [int(q) for q in rng.choice(reg, size=mid_measure_count, replace=False)]
            if P:
                out.append("X_ERROR(%s) %s" % (P, " ".join(map(str, qs))))
            out.append("MR " + " ".join(map(str, qs)))
            for q in qs:
                out.append("H %d" % q)
                if P:
                    out.append("DEPOLARIZE1(%s) %d" % (P, q))
                out.append("T %d" % q)
                if P:
                    out.append("DEPOLARIZE1(%s) %d" % (P, q))
    if P:
        out.append("X_ERROR(%s) %s" % (P, " ".join(map(str, range(n)))))
    out.append("M " + " ".join(map(str, range(n))))
    return "\n".join(out) + "\n"


def batched_set(count=64, seed=4000, n_range=(20, 100), depth_range=(50, 200), k_range=(4, 16),
                p_range=(1e-4, 1e-3)):
    """Heterogeneous batch: circuit i draws N, depth, k_target, the number of
    non-Clifford rotations (about half R_Z with uniform angles) and p."""
    out = []
    for i in range(count):
        rng = _rng(seed + i)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        k = min(k, n)
        nnc = int(rng.integers(max(2, k), 17))
        p = float(rng.uniform(p_range[0], p_range[1]))
        out.append(dict(n=n, depth=depth, k=k, nonclifford=nnc, p=p,
                        text=register_circuit(n, depth, k, nnc, p, seed=seed + 1000 + i,
                                              mid_measure_every=max(1, (2 * depth) // 3),
                                              mid_measure_count=max(1, k // 2))))
    return out


def large_active(n=200, depth=300, k_target=20, n_t=40, p=1e-4, seed=5000):
    """Large-k stress: a 20-qubit register reaching k = 20, register
    measurements every 30 layers (contract, then re-expand), 40 T total."""
    return register_circuit(n, depth, k_target, n_t, p, seed, rz_frac=0.0, mid_measure_every=30,
                            mid_measure_count=2)


# --------------------------------------------------------------------------
# The five benchmark workloads and their shot counts.
# --------------------------------------------------------------------------
def workload(name):
    """Returns dict(texts=[...], shots=int, precision='f64'|'f32', kmax=int|None).
    "batched64[i]" is circuit i of the batched set alone (its 1e5 shots)."""
    if name.startswith("batched64[") and name.endswith("]"):
        c = batched_set()[int(name[len("batched64["):-1])]
        return dict(texts=[c["text"]], shots=100_000, precision="f32", kmax=c["k"])
    if name == "random_clifford_t_n8":
        return dict(texts=[random_clifford_t(8, 40, 4, 1e-3, seed=1000)], shots=10_000, precision="f64", kmax=4)
    if name == "surface_d3_r3":
        return dict(texts=[surface_code_memory(3, 3, 1e-3)], shots=10_000_000, precision="f32", kmax=0)
    if name == "surface_d5_r5_t10":
        return dict(texts=[surface_code_memory(5, 5, 5e-4, t_rotations=10, t_after_round=2, seed=3000)],
                    shots=1_000_000, precision="f32", kmax=10)
    if name == "batched64":
        return dict(texts=[c["text"] for c in batched_set()], shots=100_000, precision="f32", kmax=None)
    if name == "large_active_k20":
        return dict(texts=[large_active()], shots=10_000, precision="f32", kmax=20)
    raise KeyError(name)


WORKLOADS = ["random_clifford_t_n8", "surface_d3_r3", "surface_d5_r5_t10", "batched64", "large_active_k20"]
