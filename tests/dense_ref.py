"""Dense state-vector brute force used to pin the oracle (N <= ~12 qubits).

Independent of oracle/ and of the HIP path: its own parser, its own Philox,
its own survival products, plain 2^N state vectors and explicit gate
matrices.  It simulates the *physical* circuit directly and applies the same
stochastic contract in physical terms:

  * the noise-only Pauli frame E is the product of all fired noise Paulis,
    propagated through the physical Clifford gates (and corrected by resets);
  * pn = [E anticommutes with the measured observable];
  * a measurement is classified by a stabilizer-group tracker (the group G of
    Paulis that stabilize the state for any amplitudes): anticommutes with G
    -> random, in G -> static, otherwise -> active;
  * m_ref = deterministic value / Philox bit r_j / [u_j < P(m_ref = 1)];
    recorded m = m_ref XOR pn.
"""
import math

import numpy as np

M64 = (1 << 64) - 1
CHUNK = 4096


# ---------------------------------------------------------------- Philox
def philox(ctr, key):
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
            k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
        p0 = 0xD2511F53 * c0
        p1 = 0xCD9E8D57 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF, ((p0 >> 32) ^ c3 ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF
    return c0, c1, c2, c3


def draw(index, purpose, shot, seed):
    return philox((index & 0xFFFFFFFF, purpose, shot & 0xFFFFFFFF, shot >> 32), (seed & 0xFFFFFFFF, seed >> 32))


def u53(w):
    return ((((w[1] << 32) | w[0]) >> 11)) * (1.0 / 9007199254740992.0)


NOISE, RBIT, AMEAS = 0x4E000000, 0x52000000, 0x41000000


# ---------------------------------------------------------------- parser
def parse(text):
    """Flat list of (name, arg, targets) with REPEAT unrolled; rec targets as ('rec', k)."""
    lines = []
    for raw in text.splitlines():
        s = raw.split("#")[0].strip()
        if s:
            lines.append(s)

    def block(i):
        out = []
        while i < len(lines):
            s = lines[i]
            if s == "}":
                return out, i + 1
            if s.upper().startswith("REPEAT"):
                n = int(s.split()[1])
                body, j = block(i + 1)
                out.extend(body * n)
                i = j
                continue
            arg = None
            if "(" in s.split()[0] or (len(s.split()) > 1 and s.split()[1].startswith("(")):
                head, _, tail = s.partition("(")
                a, _, rest = tail.partition(")")
                vals = [float(v) for v in a.split(",")]
                arg = vals[0] if len(vals) == 1 else tuple(vals)
                head = head.strip()
            else:
                head, _, rest = s.partition(" ")
            tg = []
            for t in rest.split():
                if t.startswith("rec["):
                    tg.append(("rec", int(t[4:-1])))
                elif t[0] in "XYZxyz":
                    tg.append(("prod", [(int(f[1:]), "XYZ".index(f[0].upper()) + 1) for f in t.split("*")]))
                else:
                    tg.append(int(t))
            out.append((head.upper(), arg, tg))
            i += 1
        return out, i

    ops, _ = block(0)
    return ops


# ---------------------------------------------------------------- matrices
SQ2 = 1 / math.sqrt(2)
MAT1 = {
    "H": np.array([[SQ2, SQ2], [SQ2, -SQ2]], complex),
    "S": np.array([[1, 0], [0, 1j]], complex),
    "S_DAG": np.array([[1, 0], [0, -1j]], complex),
    "X": np.array([[0, 1], [1, 0]], complex),
    "Y": np.array([[0, -1j], [1j, 0]], complex),
    "Z": np.array([[1, 0], [0, -1]], complex),
    "I": np.eye(2, dtype=complex),
}


def rotz(theta):
    """exp(-i theta Z)."""
    return np.array([[np.exp(-1j * theta), 0], [0, np.exp(1j * theta)]], complex)


def apply1(psi, n, q, U):
    v = psi.reshape(1 << (n - q - 1), 2, 1 << q)
    return np.einsum("ab,xby->xay", U, v).reshape(-1)


def apply_cx(psi, n, c, t):
    idx = np.arange(1 << n)
    src = np.where((idx >> c) & 1, idx ^ (1 << t), idx)
    return psi[src]


def apply_cz(psi, n, a, b):
    idx = np.arange(1 << n)
    sgn = np.where(((idx >> a) & 1) & ((idx >> b) & 1), -1.0, 1.0)
    return psi * sgn


def apply_swap(psi, n, a, b):
    idx = np.arange(1 << n)
    ba, bb = (idx >> a) & 1, (idx >> b) & 1
    src = idx ^ ((ba ^ bb) << a) ^ ((ba ^ bb) << b)
    return psi[src]


def pauli_bits(n, letters):
    """x and z bit vectors of a product of letters (1 X, 2 Y, 3 Z)."""
    px = np.zeros(n, np.uint8)
    pz = np.zeros(n, np.uint8)
    for q, L in letters:
        px[q] = L in (1, 2)
        pz[q] = L in (2, 3)
    return px, pz


def u3(theta, phi, lam):
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -np.exp(1j * lam) * s], [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]], complex)


def apply_pauli_letters(psi, n, letters):
    for q, L in letters:
        if L:
            psi = apply1(psi, n, q, MAT1["IXYZ"[L]])
    return psi


# ---------------------------------------------------------------- Pauli bookkeeping
def conj_bits(x, z, gate, a, b=None):
    """Propagate the (x, z) bits of a Pauli through a physical Clifford gate (signs dropped)."""
    if gate == "H":
        x[a], z[a] = z[a], x[a]
    elif gate in ("S", "S_DAG"):
        z[a] ^= x[a]
    elif gate == "CX":
        x[b] ^= x[a]
        z[a] ^= z[b]
    elif gate == "CZ":
        z[b] ^= x[a]
        z[a] ^= x[b]
    elif gate == "SWAP":
        x[a], x[b] = x[b], x[a]
        z[a], z[b] = z[b], z[a]


def anticommute(x1, z1, x2, z2):
    return int((np.sum(x1 & z2) + np.sum(z1 & x2)) & 1)


class Stabilizers:
    """Generators (x, z rows over GF(2)) of the group G that stabilises the state
    for every value of its amplitudes; rank(G) = N - k."""

    def __init__(self, n):
        self.n = n
        self.x = np.zeros((n, n), np.uint8)
        self.z = np.eye(n, dtype=np.uint8)

    def k(self):
        return self.n - self.x.shape[0]

    def conj(self, gate, a, b=None):
        for r in range(self.x.shape[0]):
            conj_bits(self.x[r], self.z[r], gate, a, b)

    def _anti(self, px, pz):
        return [(int(np.sum(self.x[r] & pz) + np.sum(self.z[r] & px)) & 1) for r in range(self.x.shape[0])]

    def rotation(self, px, pz):
        a = [r for r, v in enumerate(self._anti(px, pz)) if v]
        if a:
            r0 = a[0]
            for r in a[1:]:
                self.x[r] ^= self.x[r0]
                self.z[r] ^= self.z[r0]
            self.x = np.delete(self.x, r0, 0)
            self.z = np.delete(self.z, r0, 0)

    def in_span(self, px, pz):
        if self.x.shape[0] == 0:
            return False
        M = np.concatenate([self.x, self.z], axis=1).astype(np.uint8)
        v = np.concatenate([px, pz]).astype(np.uint8)
        return _rank(np.vstack([M, v])) == _rank(M)

    def measure(self, px, pz):
        """Returns 'random', 'static' or 'active' and updates G."""
        a = [r for r, v in enumerate(self._anti(px, pz)) if v]
        if a:
            r0 = a[0]
            for r in a[1:]:
                self.x[r] ^= self.x[r0]
                self.z[r] ^= self.z[r0]
            self.x[r0] = px
            self.z[r0] = pz
            return "random"
        if self.in_span(px, pz):
            return "static"
        self.x = np.vstack([self.x, px[None]])
        self.z = np.vstack([self.z, pz[None]])
        return "active"


def _rank(M):
    M = M.copy() % 2
    r = 0
    rows, cols = M.shape
    for c in range(cols):
        piv = None
        for i in range(r, rows):
            if M[i, c]:
                piv = i
                break
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


# ---------------------------------------------------------------- simulator
NOISE_OUT = {"DEPOLARIZE1": 3, "DEPOLARIZE2": 15, "X_ERROR": 1, "Y_ERROR": 1, "Z_ERROR": 1}
GATES1 = ("H", "S", "S_DAG", "X", "Y", "Z")


def noise_letters(name, idx):
    if name == "DEPOLARIZE1":
        return idx + 1, 0
    if name == "DEPOLARIZE2":
        return (idx + 1) >> 2, (idx + 1) & 3
    return {"X_ERROR": 1, "Y_ERROR": 2, "Z_ERROR": 3}[name], 0


class Dense:
    def __init__(self, text):
        self.ops = parse(text)
        n = 0
        self.sites = []
        for name, arg, tg in self.ops:
            for t in tg:
                if not isinstance(t, tuple):
                    n = max(n, t + 1)
                elif t[0] == "prod":
                    n = max(n, max(q for q, _ in t[1]) + 1)
            if name in NOISE_OUT and arg:
                ar = 2 if name == "DEPOLARIZE2" else 1
                for i in range(0, len(tg), ar):
                    self.sites.append((name, arg))
        self.n = n
        # survival products per chunk, FP64, same order as the contract
        self.surv = []
        for c0 in range(0, len(self.sites), CHUNK):
            S = [1.0]
            for name, p in self.sites[c0:c0 + CHUNK]:
                S.append(S[-1] * (1.0 - p))
            self.surv.append(S)

    def faults(self, seed, shot):
        out = [-1] * len(self.sites)
        for c, S in enumerate(self.surv):
            cur, ordinal, L = 0, 0, len(S) - 1
            while True:
                w = draw(ordinal, NOISE | c, shot, seed)
                ordinal += 1
                tau = u53(w) * S[cur]
                j = next((j for j in range(cur, L) if S[j + 1] <= tau), None)
                if j is None:
                    break
                site = c * CHUNK + j
                out[site] = ((((w[3] << 32) | w[2]) * NOISE_OUT[self.sites[site][0]]) >> 64)
                cur = j + 1
        return out

    def run(self, seed=0, shot=0, forced_m=None, forced_faults=None):
        n = self.n
        psi = np.zeros(1 << n, complex)
        psi[0] = 1
        ex = np.zeros(n, np.uint8)
        ez = np.zeros(n, np.uint8)
        G = Stabilizers(n)
        faults = forced_faults if forced_faults is not None else self.faults(seed, shot)
        recs, ms, probs, classes, ks, dets, obs, exps = [], [], [], [], [], [], {}, []
        site = 0
        j = 0
        rbits = {}

        def measure(q, basis, record):
            nonlocal psi, j
            px = np.zeros(n, np.uint8)
            pz = np.zeros(n, np.uint8)
            (px if basis == "X" else pz)[q] = 1
            pn = anticommute(ex, ez, px, pz)
            cls = G.measure(px, pz)
            if basis == "X":
                psi = apply1(psi, n, q, MAT1["H"])
            idx = np.arange(1 << n)
            one = ((idx >> q) & 1).astype(bool)
            nrm = np.vdot(psi, psi).real
            p1 = float(np.sum(np.abs(psi[one]) ** 2) / nrm)
            if forced_m is not None:
                m = int(forced_m[j])
            elif cls == "static":
                m = int(p1 > 0.5)
            elif cls == "random":
                blk = j >> 7
                if blk not in rbits:
                    w = draw(blk, RBIT, shot, seed)
                    rbits[blk] = w[0] | (w[1] << 32) | (w[2] << 64) | (w[3] << 96)
                m = ((rbits[blk] >> (j & 127)) & 1) ^ pn
            else:
                pref1 = p1 if pn == 0 else 1.0 - p1
                m = int(u53(draw(j, AMEAS, shot, seed)) < pref1) ^ pn
            keep = one if m else ~one
            psi = np.where(keep, psi, 0)
            psi = psi / np.sqrt(np.vdot(psi, psi).real)
            if basis == "X":
                psi = apply1(psi, n, q, MAT1["H"])
            probs.append(p1)
            ms.append(m)
            classes.append(cls)
            j += 1
            if record:
                recs.append(m)
            return m, pn

        def measure_product(letters):
            """Measurement of a Pauli product (eigenvalue (-1)^m): projector
            (I + (-1)^m P) / 2 applied directly."""
            nonlocal psi, j
            px, pz = pauli_bits(n, letters)
            pn = anticommute(ex, ez, px, pz)
            cls = G.measure(px, pz)
            ppsi = apply_pauli_letters(psi, n, letters)
            nrm = np.vdot(psi, psi).real
            p1 = float(max(0.0, (nrm - np.vdot(psi, ppsi).real) / 2) / nrm)
            if forced_m is not None:
                m = int(forced_m[j])
            elif cls == "static":
                m = int(p1 > 0.5)
            elif cls == "random":
                blk = j >> 7
                if blk not in rbits:
                    w = draw(blk, RBIT, shot, seed)
                    rbits[blk] = w[0] | (w[1] << 32) | (w[2] << 64) | (w[3] << 96)
                m = ((rbits[blk] >> (j & 127)) & 1) ^ pn
            else:
                pref1 = p1 if pn == 0 else 1.0 - p1
                m = int(u53(draw(j, AMEAS, shot, seed)) < pref1) ^ pn
            psi = (psi + (-1) ** m * ppsi) / 2
            psi = psi / np.sqrt(np.vdot(psi, psi).real)
            probs.append(p1)
            ms.append(m)
            classes.append(cls)
            j += 1
            recs.append(m)

        def rotate(letters, theta):
            """exp(-i theta P) = cos(theta) I - i sin(theta) P."""
            nonlocal psi
            psi = math.cos(theta) * psi - 1j * math.sin(theta) * apply_pauli_letters(psi, n, letters)
            G.rotation(*pauli_bits(n, letters))

        for name, arg, tg in self.ops:
            if name in GATES1:
                for q in tg:
                    psi = apply1(psi, n, q, MAT1[name])
                    if name in ("H", "S", "S_DAG"):
                        conj_bits(ex, ez, name, q)
                        G.conj(name, q)
            elif name in ("CX", "CNOT", "CY", "CZ") and any(isinstance(t, tuple) for t in tg):
                # feed-forward: Pauli on the qubit if the record is 1 (the
                # noise frame only follows physical faults)
                L = {"CX": 1, "CNOT": 1, "CY": 2, "CZ": 3}[name]
                for i in range(0, len(tg), 2):
                    r, q = (tg[i], tg[i + 1]) if isinstance(tg[i], tuple) else (tg[i + 1], tg[i])
                    if recs[len(recs) + r[1]]:
                        psi = apply_pauli_letters(psi, n, [(q, L)])
            elif name in ("R_X", "R_Y"):
                for q in tg:
                    rotate([(q, 1 if name == "R_X" else 2)], arg / 2)
            elif name == "R_PAULI":
                for t in tg:
                    rotate(t[1], arg / 2)
            elif name == "U3":
                th, ph, la = arg
                for q in tg:
                    psi = apply1(psi, n, q, u3(th, ph, la))
                    # as R_Z(phi) R_Y(theta) R_Z(lambda) for the active-set tracker
                    for L in (3, 2, 3):
                        G.rotation(*pauli_bits(n, [(q, L)]))
            elif name == "MPP":
                for t in tg:
                    measure_product(t[1])
            elif name == "EXP_VAL":
                for t in tg:
                    nrm = np.vdot(psi, psi).real
                    exps.append(float(np.vdot(psi, apply_pauli_letters(psi, n, t[1])).real / nrm))
            elif name in ("CX", "CNOT", "CZ", "SWAP"):
                g = "CX" if name == "CNOT" else name
                for i in range(0, len(tg), 2):
                    a, b = tg[i], tg[i + 1]
                    psi = {"CX": apply_cx, "CZ": apply_cz, "SWAP": apply_swap}[g](psi, n, a, b)
                    conj_bits(ex, ez, g, a, b)
                    G.conj(g, a, b)
            elif name in ("T", "T_DAG", "R_Z"):
                th = math.pi / 8 if name == "T" else -math.pi / 8 if name == "T_DAG" else arg / 2
                for q in tg:
                    psi = apply1(psi, n, q, rotz(th))
                    pz = np.zeros(n, np.uint8)
                    pz[q] = 1
                    G.rotation(np.zeros(n, np.uint8), pz)
            elif name in ("M", "MX", "MR", "R"):
                for q in tg:
                    m, pn = measure(q, "X" if name == "MX" else "Z", name != "R")
                    if name in ("MR", "R"):
                        if m:
                            psi = apply1(psi, n, q, MAT1["X"])
                        ex[q] ^= pn
            elif name in NOISE_OUT:
                if not arg:
                    continue
                ar = 2 if name == "DEPOLARIZE2" else 1
                for i in range(0, len(tg), ar):
                    f = faults[site]
                    if f >= 0:
                        la, lb = noise_letters(name, f)
                        lets = [(tg[i], la)] + ([(tg[i + 1], lb)] if ar == 2 else [])
                        psi = apply_pauli_letters(psi, n, lets)
                        for q, L in lets:
                            ex[q] ^= L in (1, 2)
                            ez[q] ^= L in (2, 3)
                    site += 1
            elif name == "DETECTOR":
                dets.append(int(np.bitwise_xor.reduce([recs[len(recs) + k] for _, k in tg] or [0])))
            elif name == "OBSERVABLE_INCLUDE":
                o = int(arg)
                obs[o] = obs.get(o, 0) ^ int(np.bitwise_xor.reduce([recs[len(recs) + k] for _, k in tg] or [0]))
            elif name in ("TICK", "QUBIT_COORDS", "SHIFT_COORDS"):
                pass
            else:
                raise ValueError("dense_ref: unsupported " + name)
            ks.append(G.k())
        nobs = max(obs) + 1 if obs else 0
        return dict(psi=psi, recs=np.array(recs, np.uint8), m=np.array(ms, np.uint8), probs=np.array(probs),
                    classes=classes, kmax=max(ks) if ks else 0, dets=np.array(dets, np.uint8),
                    obs=np.array([obs.get(i, 0) for i in range(nobs)], np.uint8), faults=faults,
                    expvals=np.array(exps))


# ---------------------------------------------------------------- oracle state -> dense vector
def _gate_matrix_full(n, gate, a, b, dagger=False):
    """Dense 2^n x 2^n matrix of a gate (used to rebuild U_C from the oracle's log)."""
    dim = 1 << n
    eye = np.eye(dim, dtype=complex)
    cols = []
    names = ["H", "S", "S_DAG", "X", "Y", "Z", "CX", "CZ", "SWAP"]
    g = names[gate]
    if dagger and g == "S":
        g = "S_DAG"
    elif dagger and g == "S_DAG":
        g = "S"
    for c in range(dim):
        v = eye[:, c]
        if g in GATES1:
            v = apply1(v, n, a, MAT1[g])
        elif g == "CX":
            v = apply_cx(v, n, a, b)
        elif g == "CZ":
            v = apply_cz(v, n, a, b)
        else:
            v = apply_swap(v, n, a, b)
        cols.append(v)
    return np.stack(cols, axis=1)


def oracle_state_to_dense(n, uclog, frame_x, frame_z, phi, slots, gamma):
    """gamma * U_C * P~ * (phi_A (x) |0>_D) as a dense vector (Definition 2, Eq. 2)."""
    dim = 1 << n
    U = np.eye(dim, dtype=complex)
    for side, gate, a, b in uclog:
        M = _gate_matrix_full(n, gate, a, b, dagger=(side == 1))
        U = M @ U if side == 0 else U @ M
    v = np.zeros(dim, complex)
    for i, amp in enumerate(phi):
        idx = 0
        for s, q in enumerate(slots):
            if (i >> s) & 1:
                idx |= 1 << q
        v[idx] = amp
    for q in range(n):
        if frame_z[q]:
            v = apply1(v, n, q, MAT1["Z"])
    for q in range(n):
        if frame_x[q]:
            v = apply1(v, n, q, MAT1["X"])
    return gamma * (U @ v)
