// Host-side compiler: circuit text -> flat wave-uniform instruction stream.
//
// Follows the paper's compile-once pipeline (Section 3.1): physical Clifford
// gates are absorbed into the Clifford frame U_C (Definition 1, Eq. 1); each
// active operation's generator is mapped to the virtual basis and localized
// to one virtual qubit (Lemma 1, Appendix A) with sequences that respect
// dormant invariance (Lemma 2); the result is classified into the update
// cases of Appendix B.  Because of Theorem 1 all of this is shot independent,
// so the GPU only runs the resulting stream.
//
// Differences from a gate-by-gate lowering: the fan of CNOTs (or CZs) that
// shares one pivot is emitted as one frame instruction acting on W 64-bit
// words, and its array part (if any) as one pass; expansion and the first
// rotation on the new axis are one instruction (the paper's fused
// expand+rotation); consecutive noise sites form one block (the paper's
// noise coalescing); a demoted slot is refilled by the top slot instead of
// shifting all slots above it down.
#include "compiler.h"

#include <cctype>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace clifft {

namespace {

// ---------------------------------------------------------------- parsing
enum PK {
  K_H, K_S, K_SDAG, K_X, K_Y, K_Z, K_CX, K_CZ, K_SWAP, K_ROTZ, K_M, K_MX, K_MR, K_R, K_NOISE, K_DET, K_OBS,
  K_PROT,    // exp(-i theta P) for the Pauli product `prod`
  K_MPP,     // measurement of the Pauli product `prod`
  K_CFEED,   // Pauli prod[0] if record refs[0] is 1 (feed-forward)
  K_GPHASE,  // global phase exp(-i theta)
  K_EXPVAL   // expectation value of the Pauli product `prod` (probe obs)
};

struct PhysOp {
  int kind;
  int a, b;
  double arg;  // rotation angle theta of exp(-i theta P), or probability
  int ntype;
  int obs;
  std::vector<int> refs;  // absolute record indices
  std::vector<std::pair<int, char>> prod;  // Pauli product: (qubit, 'X' / 'Y' / 'Z')
};

struct Parsed {
  std::vector<PhysOp> ops;
  int nq = 0;
  int nrec = 0;
  int ndet = 0;
  int nobs = 0;
  int nprobes = 0;
};

struct Lines {
  std::vector<std::string> v;
  std::vector<int> lineno;
};

static std::string strip(const std::string& s) {
  size_t a = 0, b = s.size();
  while (a < b && isspace((unsigned char)s[a])) a++;
  while (b > a && isspace((unsigned char)s[b - 1])) b--;
  return s.substr(a, b - a);
}

static bool parse_range(const Lines& L, size_t& i, Parsed& P, int depth, std::string& err, int& code);

static bool fail(std::string& err, int& code, int c, int line, const std::string& msg) {
  char buf[64];
  snprintf(buf, sizeof buf, "line %d: ", line);
  err = buf + msg;
  code = c;
  return false;
}

static bool parse_line(const std::string& raw, int line, Parsed& P, std::string& err, int& code) {
  size_t i = 0;
  std::string name;
  while (i < raw.size() && !isspace((unsigned char)raw[i]) && raw[i] != '(') name += (char)toupper((unsigned char)raw[i++]);
  while (i < raw.size() && isspace((unsigned char)raw[i])) i++;
  double arg = 0;
  std::vector<double> args;
  bool has_arg = false;
  if (i < raw.size() && raw[i] == '(') {
    size_t e = raw.find(')', i);
    if (e == std::string::npos) return fail(err, code, 1, line, "missing ')'");
    const char* a = raw.c_str() + i + 1;
    const char* stop = raw.c_str() + e;
    while (a < stop && args.size() < 3) {
      char* end = nullptr;
      double v = strtod(a, &end);
      if (end == a) break;
      args.push_back(v);
      while (end < stop && isspace((unsigned char)*end)) end++;
      if (end >= stop || *end != ',') break;
      a = end + 1;
    }
    has_arg = !args.empty();
    arg = has_arg ? args[0] : 0.0;
    i = e + 1;
  }
  std::vector<long> tg;
  std::vector<bool> isrec;
  std::vector<std::vector<std::pair<int, char>>> prods;  // Pauli product targets (X0*Y3*Z5)
  while (i < raw.size()) {
    while (i < raw.size() && isspace((unsigned char)raw[i])) i++;
    if (i >= raw.size()) break;
    size_t j = i;
    while (j < raw.size() && !isspace((unsigned char)raw[j])) j++;
    std::string t = raw.substr(i, j - i);
    i = j;
    if (strchr("XYZxyz", t[0])) {
      std::vector<std::pair<int, char>> pr;
      size_t k = 0;
      while (k < t.size()) {
        const char letter = (char)toupper((unsigned char)t[k]);
        if (!strchr("XYZ", letter)) return fail(err, code, 1, line, "bad Pauli product '" + t + "'");
        char* end = nullptr;
        long v = strtol(t.c_str() + k + 1, &end, 10);
        if (end == t.c_str() + k + 1 || v < 0 || v >= 65535 || (*end && *end != '*'))
          return fail(err, code, 1, line, "bad Pauli product '" + t + "'");
        for (auto& f : pr)
          if (f.first == (int)v) return fail(err, code, 1, line, "repeated qubit in a product");
        pr.push_back({(int)v, letter});
        if (v + 1 > P.nq) P.nq = (int)v + 1;
        k = (size_t)(end - t.c_str()) + (*end ? 1 : 0);
      }
      prods.push_back(pr);
      continue;
    }
    if (t.compare(0, 4, "rec[") == 0) {
      tg.push_back(strtol(t.c_str() + 4, nullptr, 10));
      isrec.push_back(true);
    } else {
      char* end = nullptr;
      long v = strtol(t.c_str(), &end, 10);
      if (end == t.c_str() || *end || v < 0 || v >= 65535) return fail(err, code, 1, line, "bad target '" + t + "'");
      tg.push_back(v);
      isrec.push_back(false);
      if (v + 1 > P.nq) P.nq = (int)v + 1;
    }
  }
  if (name == "TICK" || name == "QUBIT_COORDS" || name == "SHIFT_COORDS") return true;
  const bool prod_gate = name == "MPP" || name == "R_PAULI" || name == "EXP_VAL";
  if (!prods.empty() && !prod_gate) return fail(err, code, 1, line, "Pauli product target on " + name);
  if (prod_gate) {
    // MPP P...: one measurement per product; R_PAULI(phi) P...: exp(-i phi P / 2)
    if (!tg.empty()) return fail(err, code, 1, line, name + " takes Pauli products");
    if (name == "R_PAULI" && !has_arg) return fail(err, code, 1, line, "R_PAULI needs an angle");
    for (auto& pr : prods) {
      PhysOp o{};
      o.kind = name == "MPP" ? K_MPP : name == "EXP_VAL" ? K_EXPVAL : K_PROT;
      o.arg = arg / 2;
      o.prod = pr;
      if (o.kind == K_EXPVAL) o.obs = P.nprobes++;
      P.ops.push_back(o);
      if (o.kind == K_MPP) P.nrec++;
    }
    return true;
  }
  // a Pauli on a qubit controlled by a measurement record (feed-forward):
  // CX / CY / CZ rec[-k] q (CZ also q rec[-k])
  if (name == "CX" || name == "CNOT" || name == "ZCX" || name == "CY" || name == "ZCY" || name == "CZ" || name == "ZCZ") {
    bool anyrec = false;
    for (bool r : isrec) anyrec = anyrec || r;
    if (anyrec) {
      const char letter = (name == "CY" || name == "ZCY") ? 'Y' : (name == "CZ" || name == "ZCZ") ? 'Z' : 'X';
      if (tg.size() % 2) return fail(err, code, 1, line, name + " needs target pairs");
      for (size_t t = 0; t < tg.size(); t += 2) {
        size_t r = t, q = t + 1;
        if (letter == 'Z' && !isrec[t] && isrec[t + 1]) std::swap(r, q);
        if (!isrec[r] || isrec[q]) return fail(err, code, 1, line, "feed-forward needs rec[-k] then a qubit");
        if (tg[r] >= 0 || P.nrec + tg[r] < 0) return fail(err, code, 1, line, "bad record target");
        PhysOp o{};
        o.kind = K_CFEED;
        o.a = (int)tg[q];
        o.refs.push_back((int)(P.nrec + tg[r]));
        o.prod.push_back({(int)tg[q], letter});
        P.ops.push_back(o);
      }
      return true;
    }
  }
  if (name == "R_X" || name == "R_Y") {
    // R_X(phi) = exp(-i phi X / 2), R_Y(phi) = exp(-i phi Y / 2)
    if (!has_arg) return fail(err, code, 1, line, name + " needs an angle");
    for (long t : tg) {
      PhysOp o{};
      o.kind = K_PROT;
      o.arg = arg / 2;
      o.prod.push_back({(int)t, name[2]});
      P.ops.push_back(o);
    }
    return true;
  }
  if (name == "U3") {
    // U3(theta, phi, lambda) = e^{i (phi + lambda) / 2} R_Z(phi) R_Y(theta) R_Z(lambda)
    if (args.size() != 3) return fail(err, code, 1, line, "U3 needs three angles");
    for (long t : tg) {
      PhysOp z1{}, y{}, z2{}, g{};
      z1.kind = K_ROTZ; z1.a = (int)t; z1.b = -1; z1.arg = args[2] / 2;
      y.kind = K_PROT; y.arg = args[0] / 2; y.prod.push_back({(int)t, 'Y'});
      z2.kind = K_ROTZ; z2.a = (int)t; z2.b = -1; z2.arg = args[1] / 2;
      g.kind = K_GPHASE; g.arg = -(args[1] + args[2]) / 2;
      P.ops.push_back(z1);
      P.ops.push_back(y);
      P.ops.push_back(z2);
      P.ops.push_back(g);
    }
    return true;
  }
  struct G { const char* nm; int kind, arity; };
  static const G gates[] = {{"H", K_H, 1},    {"S", K_S, 1},     {"S_DAG", K_SDAG, 1}, {"X", K_X, 1},   {"Y", K_Y, 1},
                            {"Z", K_Z, 1},    {"CX", K_CX, 2},   {"CNOT", K_CX, 2},    {"ZCX", K_CX, 2}, {"CZ", K_CZ, 2},
                            {"SWAP", K_SWAP, 2}, {"M", K_M, 1},  {"MZ", K_M, 1},       {"MX", K_MX, 1}, {"MR", K_MR, 1},
                            {"MRZ", K_MR, 1}, {"R", K_R, 1},     {"RZ", K_R, 1}};
  for (const G& g : gates) {
    if (name != g.nm) continue;
    if (tg.size() % g.arity) return fail(err, code, 1, line, name + " needs target pairs");
    for (size_t t = 0; t < tg.size(); t += g.arity) {
      if (isrec[t]) return fail(err, code, 1, line, "record target on a gate");
      PhysOp o{};
      o.kind = g.kind;
      o.a = (int)tg[t];
      o.b = g.arity == 2 ? (int)tg[t + 1] : -1;
      if (o.a == o.b) return fail(err, code, 1, line, "repeated qubit");
      P.ops.push_back(o);
      if (g.kind == K_M || g.kind == K_MX || g.kind == K_MR) P.nrec++;
    }
    return true;
  }
  if (name == "T" || name == "T_DAG" || name == "R_Z") {
    double th;
    if (name == "T") th = M_PI / 8;
    else if (name == "T_DAG") th = -M_PI / 8;
    else {
      if (!has_arg) return fail(err, code, 1, line, "R_Z needs an angle");
      th = arg / 2;  // R_Z(phi) = exp(-i phi Z / 2)
    }
    for (long t : tg) {
      PhysOp o{};
      o.kind = K_ROTZ;
      o.a = (int)t;
      o.b = -1;
      o.arg = th;
      P.ops.push_back(o);
    }
    return true;
  }
  struct N { const char* nm; int type, arity; };
  static const N noises[] = {{"DEPOLARIZE1", S_DEP1, 1}, {"DEPOLARIZE2", S_DEP2, 2}, {"X_ERROR", S_XERR, 1},
                             {"Y_ERROR", S_YERR, 1},     {"Z_ERROR", S_ZERR, 1}};
  for (const N& nn : noises) {
    if (name != nn.nm) continue;
    if (!has_arg || !(arg >= 0 && arg <= 1)) return fail(err, code, 1, line, "bad probability");
    if (tg.size() % nn.arity) return fail(err, code, 1, line, "noise needs target pairs");
    if (arg == 0) return true;
    for (size_t t = 0; t < tg.size(); t += nn.arity) {
      PhysOp o{};
      o.kind = K_NOISE;
      o.ntype = nn.type;
      o.a = (int)tg[t];
      o.b = nn.arity == 2 ? (int)tg[t + 1] : -1;
      o.arg = arg;
      if (o.a == o.b) return fail(err, code, 1, line, "repeated qubit");
      P.ops.push_back(o);
    }
    return true;
  }
  if (name == "DETECTOR" || name == "OBSERVABLE_INCLUDE") {
    PhysOp o{};
    o.kind = name == "DETECTOR" ? K_DET : K_OBS;
    o.obs = (int)arg;
    for (size_t t = 0; t < tg.size(); t++) {
      if (!isrec[t] || tg[t] >= 0 || P.nrec + tg[t] < 0) return fail(err, code, 1, line, "bad record target");
      o.refs.push_back((int)(P.nrec + tg[t]));
    }
    if (o.kind == K_DET) P.ndet++;
    else if (o.obs + 1 > P.nobs) P.nobs = o.obs + 1;
    P.ops.push_back(o);
    return true;
  }
  return fail(err, code, 2, line, "unsupported instruction '" + name + "'");
}

static bool parse_range(const Lines& L, size_t& i, Parsed& P, int depth, std::string& err, int& code) {
  while (i < L.v.size()) {
    const std::string& s = L.v[i];
    int line = L.lineno[i];
    if (s == "}") {
      if (depth == 0) return fail(err, code, 1, line, "unmatched '}'");
      i++;
      return true;
    }
    std::string up;
    for (char c : s.substr(0, 6)) up += (char)toupper((unsigned char)c);
    if (up == "REPEAT") {
      char* end = nullptr;
      long n = strtol(s.c_str() + 6, &end, 10);
      std::string rest = strip(end ? end : "");
      if (rest != "{" || n < 0) return fail(err, code, 1, line, "bad REPEAT");
      size_t start = i + 1;
      size_t after = start;
      if (n == 0) {
        Parsed dummy;
        size_t j = start;
        if (!parse_range(L, j, dummy, depth + 1, err, code)) return false;
        after = j;
      }
      for (long r = 0; r < n; r++) {
        size_t j = start;
        if (!parse_range(L, j, P, depth + 1, err, code)) return false;
        after = j;
      }
      i = after;
      continue;
    }
    if (!parse_line(s, line, P, err, code)) return false;
    i++;
  }
  if (depth > 0) return fail(err, code, 1, (int)L.v.size(), "missing '}'");
  return true;
}

// ---------------------------------------------------------------- Paulis on W words
struct Pauli {
  std::vector<uint64_t> x, z;
  int r = 0;  // sign bit; letters sigma(1,0)=X sigma(0,1)=Z sigma(1,1)=Y
  Pauli() {}
  explicit Pauli(int W) : x(W, 0), z(W, 0) {}
  bool getx(int q) const { return (x[q >> 6] >> (q & 63)) & 1; }
  bool getz(int q) const { return (z[q >> 6] >> (q & 63)) & 1; }
  void flipx(int q) { x[q >> 6] ^= 1ull << (q & 63); }
  void flipz(int q) { z[q >> 6] ^= 1ull << (q & 63); }
  void setx(int q, bool v) { if (getx(q) != v) flipx(q); }
  void setz(int q, bool v) { if (getz(q) != v) flipz(q); }
};

// a <- i^extra * a * b for Hermitian Paulis whose product (times i^extra) is
// Hermitian; the power of i is computed word-parallel: with the cyclic order
// X -> Y -> Z, a "forward" pair contributes +1 and a "backward" pair -1.
static void mul_into(Pauli& a, const Pauli& b, int extra) {
  int e = extra + 2 * a.r + 2 * b.r;
  for (size_t w = 0; w < a.x.size(); w++) {
    uint64_t X1 = a.x[w] & ~a.z[w], Y1 = a.x[w] & a.z[w], Z1 = ~a.x[w] & a.z[w];
    uint64_t X2 = b.x[w] & ~b.z[w], Y2 = b.x[w] & b.z[w], Z2 = ~b.x[w] & b.z[w];
    uint64_t fwd = (X1 & Y2) | (Y1 & Z2) | (Z1 & X2);
    uint64_t bwd = (X1 & Z2) | (Y1 & X2) | (Z1 & Y2);
    e += __builtin_popcountll(fwd) - __builtin_popcountll(bwd);
    a.x[w] ^= b.x[w];
    a.z[w] ^= b.z[w];
  }
  e = ((e % 4) + 4) % 4;
  if (e & 1) abort();  // product is not Hermitian: caller error
  a.r = e >> 1;
}

// Conjugation P -> G P G^dagger by the virtual gates of the localization
// sequences (Aaronson-Gottesman update rules).
static void cj_cx(Pauli& p, int c, int t) {
  int xc = p.getx(c), zc = p.getz(c), xt = p.getx(t), zt = p.getz(t);
  p.r ^= xc & zt & (xt ^ zc ^ 1);
  p.setx(t, xt ^ xc);
  p.setz(c, zc ^ zt);
}
static void cj_cz(Pauli& p, int a, int b) {
  int xa = p.getx(a), za = p.getz(a), xb = p.getx(b), zb = p.getz(b);
  p.r ^= xa & xb & (za ^ zb);
  p.setz(a, za ^ xb);
  p.setz(b, zb ^ xa);
}
static void cj_s(Pauli& p, int a) {
  int xa = p.getx(a), za = p.getz(a);
  p.r ^= xa & za;
  p.setz(a, za ^ xa);
}
static void cj_h(Pauli& p, int a) {
  int xa = p.getx(a), za = p.getz(a);
  p.r ^= xa & za;
  p.setx(a, za);
  p.setz(a, xa);
}

enum VG { V_CX, V_CZ, V_S, V_H };

// ---------------------------------------------------------------- compiler state
struct Compiler {
  int n, W;
  std::vector<Pauli> ix, iz;  // U_C^dagger X_q U_C, U_C^dagger Z_q U_C
  std::vector<int> slot_of;   // virtual qubit -> slot or -1
  std::vector<int> q_at;      // slot -> virtual qubit
  int k = 0;
  CompiledProgram* out;
  bool drop_phases = false;

  Compiler(int n_, CompiledProgram* o) : n(n_), W((n_ + 63) / 64), out(o) {
    ix.assign(n, Pauli(W));
    iz.assign(n, Pauli(W));
    for (int q = 0; q < n; q++) {
      ix[q].flipx(q);
      iz[q].flipz(q);
    }
    slot_of.assign(n, -1);
  }
  bool active(int q) const { return slot_of[q] >= 0; }

  Pauli image(int q, char letter) const {
    if (letter == 'X') return ix[q];
    if (letter == 'Z') return iz[q];
    Pauli y = ix[q];
    mul_into(y, iz[q], 1);  // Y = i X Z
    return y;
  }

  // U_C <- G U_C (Definition 1 on the new frame): images of G^dagger P G.
  void phys(int kind, int a, int b) {
    switch (kind) {
      case K_H: std::swap(ix[a], iz[a]); break;
      case K_S: { Pauli y = image(a, 'Y'); y.r ^= 1; ix[a] = y; break; }  // S^dag X S = -Y
      case K_SDAG: ix[a] = image(a, 'Y'); break;                          // S X S^dag = Y
      case K_X: iz[a].r ^= 1; break;
      case K_Z: ix[a].r ^= 1; break;
      case K_Y: ix[a].r ^= 1; iz[a].r ^= 1; break;
      case K_CX: mul_into(ix[a], ix[b], 0); mul_into(iz[b], iz[a], 0); break;
      case K_CZ: mul_into(ix[a], iz[b], 0); mul_into(ix[b], iz[a], 0); break;
      case K_SWAP: std::swap(ix[a], ix[b]); std::swap(iz[a], iz[b]); break;
    }
  }

  // U_C <- U_C V^dagger: every image becomes V P~ V^dagger.
  void virt(int g, int a, int b) {
    for (int q = 0; q < n; q++)
      for (Pauli* p : {&ix[q], &iz[q]}) {
        if (g == V_CX) cj_cx(*p, a, b);
        else if (g == V_CZ) cj_cz(*p, a, b);
        else if (g == V_S) cj_s(*p, a);
        else cj_h(*p, a);
      }
  }

  uint32_t push_mask(const std::vector<uint64_t>& w) {
    uint32_t off = (uint32_t)out->masks.size();
    out->masks.insert(out->masks.end(), w.begin(), w.end());
    return off;
  }
  uint32_t push_pauli(const Pauli& p) {
    uint32_t off = push_mask(p.x);
    push_mask(p.z);
    return off;
  }
  // A rotation exp(-i theta Z) on an axis acts as diag(e^{-i theta},
  // e^{i theta}); the kernels apply e^{2 i theta} to the upper half and put
  // the common factor e^{-i theta} into the global scalar.
  uint32_t push_angle(double theta) {
    uint32_t idx = (uint32_t)(out->consts.size() / 4);
    out->consts.push_back(cos(2 * theta));
    out->consts.push_back(sin(2 * theta));
    out->consts.push_back(cos(theta));
    out->consts.push_back(sin(theta));
    return idx;
  }
  void emit(uint8_t op, uint8_t flags, int v, int s, uint32_t a, uint32_t b, int u = 0) {
    GInstr in{};
    in.op = op;
    in.flags = flags;
    in.v = (uint16_t)(v < 0 ? 0 : v);
    in.s = (uint16_t)(s < 0 ? 0 : s);
    in.u = (uint16_t)u;
    in.a = a;
    in.b = b;
    out->code.push_back(in);
    out->k_after.push_back(k);
    if (k > out->kmax) out->kmax = k;
  }
  uint32_t slot_mask(const std::vector<int>& qs) const {
    uint32_t m = 0;
    for (int q : qs)
      if (active(q)) m |= 1u << slot_of[q];
    return m;
  }

  // Lemma 1 / Appendix A, case 1: pivot v with x_v = 1.  CNOT v->q fan over
  // the rest of x, CZ v,q fan over the remaining z, S_v if a Y is left.
  void localize_case1(Pauli& g, int v) {
    std::vector<int> qs;
    std::vector<uint64_t> m(W, 0);
    for (int q = 0; q < n; q++)
      if (q != v && g.getx(q)) { qs.push_back(q); m[q >> 6] |= 1ull << (q & 63); }
    if (!qs.empty()) {
      for (int q : qs) { cj_cx(g, v, q); virt(V_CX, v, q); }
      emit(OP_FANCX, 0, v, 0, push_mask(m), 0);
      if (active(v)) emit(OP_APERM, 0, v, slot_of[v], slot_mask(qs), 0);  // all of qs are active here
    }
    qs.clear();
    m.assign(W, 0);
    for (int q = 0; q < n; q++)
      if (q != v && g.getz(q)) { qs.push_back(q); m[q >> 6] |= 1ull << (q & 63); }
    if (!qs.empty()) {
      for (int q : qs) { cj_cz(g, v, q); virt(V_CZ, v, q); }
      emit(OP_FANCZ, 0, v, 0, push_mask(m), 0);
      uint32_t sm = slot_mask(qs);
      if (active(v) && sm) emit(OP_ASIGN, 0, v, slot_of[v], sm, 0);
    }
    if (g.getz(v)) {
      cj_s(g, v);
      virt(V_S, v, -1);
      emit(OP_FS, 0, v, 0, 0, 0);
      if (active(v)) emit(OP_AS, 0, v, slot_of[v], 0, 0);
    }
  }

  // Lemma 1 / Appendix A, case 2: x = 0, pivot v with z_v = 1; CNOT q->v.
  void localize_case2(Pauli& g, int v) {
    std::vector<int> qs;
    std::vector<uint64_t> m(W, 0);
    for (int q = 0; q < n; q++)
      if (q != v && g.getz(q)) { qs.push_back(q); m[q >> 6] |= 1ull << (q & 63); }
    if (qs.empty()) return;
    for (int q : qs) { cj_cx(g, q, v); virt(V_CX, q, v); }
    emit(OP_FAN2, 0, v, 0, push_mask(m), 0);
    uint32_t sm = slot_mask(qs);
    if (sm) emit(OP_APERM2, 0, v, slot_of[v], sm, 0);
  }

  int lowest(const std::vector<uint64_t>& bits, bool want_active) const {
    for (int q = 0; q < n; q++)
      if (((bits[q >> 6] >> (q & 63)) & 1) && active(q) == want_active) return q;
    return -1;
  }
  static bool nonzero(const std::vector<uint64_t>& b) {
    for (uint64_t w : b)
      if (w) return true;
    return false;
  }

  // U_C^dagger P U_C for a Pauli P given in the basis the images refer to
  // (the product of its letters' images; letters of different qubits commute).
  Pauli map(const Pauli& p) const {
    Pauli r(W);
    r.r = p.r;
    for (int q = 0; q < n; q++) {
      const bool x = p.getx(q), z = p.getz(q);
      if (x || z) mul_into(r, image(q, x && z ? 'Y' : x ? 'X' : 'Z'), 0);
    }
    return r;
  }

  // U_C^dagger P U_C for a physical Pauli product (letters on different qubits)
  Pauli product(const std::vector<std::pair<int, char>>& pr) const {
    Pauli r(W);
    for (auto& f : pr) mul_into(r, image(f.first, f.second), 0);
    return r;
  }

  // feed-forward Pauli with virtual image e if record `rec` is 1 (Appendix B.3)
  void feed(const Pauli& e, int rec) { emit(OP_CFEED, e.r ? F_SIGN : 0, 0, 0, push_pauli(e), (uint32_t)rec); }

  // expectation-value probe of the virtual observable g: its W-word image,
  // then the slot masks of its X and Z letters on active qubits; F_ZERO when
  // it has X support on a dormant qubit (the value is then 0)
  void probe(const Pauli& g, int idx) {
    uint32_t xm = 0, zm = 0;
    bool dormant_x = false;
    for (int q = 0; q < n; q++) {
      if (g.getx(q)) {
        if (active(q)) xm |= 1u << slot_of[q];
        else dormant_x = true;
      }
      if (g.getz(q) && active(q)) zm |= 1u << slot_of[q];
    }
    const uint32_t off = push_pauli(g);
    push_mask(std::vector<uint64_t>{xm, zm});
    emit(OP_EXPVAL, (uint8_t)((g.r ? F_SIGN : 0) | (dormant_x ? F_ZERO : 0)), 0, 0, off, (uint32_t)idx);
  }

  // a phase exp(-i theta) of the global scalar only
  void global_phase(double theta) {
    if (!drop_phases) emit(OP_PHASE, 0, 0, 0, push_mask(std::vector<uint64_t>(W, 0)), push_angle(theta));
  }

  // Appendix B.1: rotation exp(-i theta g) about the virtual generator g.
  void rotation(Pauli g, double theta) {
    int vd = lowest(g.x, false);
    int va = lowest(g.x, true);
    if (vd >= 0) {
      localize_case1(g, vd);  // -> +-X_v, v dormant
      cj_h(g, vd);            // H_v promotes v: |0> -> |+>
      virt(V_H, vd, -1);
      int s = k;
      slot_of[vd] = s;
      q_at.push_back(vd);
      k++;
      emit(OP_EXPAND, 0, vd, s, push_angle(g.r ? -theta : theta), 0);
    } else if (va >= 0) {
      localize_case1(g, va);  // -> +-X_v, v active
      cj_h(g, va);
      virt(V_H, va, -1);
      emit(OP_FH, 0, va, 0, 0, 0);
      emit(OP_AH, 0, va, slot_of[va], 0, 0);
      emit(OP_AROT, 0, va, slot_of[va], push_angle(g.r ? -theta : theta), 0);
    } else {
      int vz = lowest(g.z, true);
      if (vz >= 0) {
        localize_case2(g, vz);
        emit(OP_AROT, 0, vz, slot_of[vz], push_angle(g.r ? -theta : theta), 0);
      }
      else if (!drop_phases)  // a Z string on dormant qubits: a phase of the global scalar only
        emit(OP_PHASE, 0, 0, 0, push_mask(g.z), push_angle(g.r ? -theta : theta));
    }
  }

  void demote(int v) {
    int s = slot_of[v];
    int top = k - 1;
    if (s != top) {
      int qt = q_at[top];
      q_at[s] = qt;
      slot_of[qt] = s;
    }
    q_at.pop_back();
    slot_of[v] = -1;
    k--;
  }

  // Appendix B.2: measurement of the virtual observable g as event j (the
  // next ordinal when j < 0), recorded as record `rec` (-1: not recorded).
  int measure(Pauli g, int rec, int j = -1) {
    if (j < 0) j = out->nevents;
    out->nevents = std::max(out->nevents, j + 1);
    if ((int)out->ev_rec.size() <= j) {
      out->ev_rec.resize(j + 1, -1);
      out->ev_class.resize(j + 1, 0);
    }
    out->ev_rec[j] = rec;
    bool anyx = nonzero(g.x);
    int xd = lowest(g.x, false);
    if (!anyx && lowest(g.z, true) < 0) {
      out->ev_class[j] = 0;
      emit(OP_MSTATIC, g.r ? F_SIGN : 0, 0, 0, push_mask(g.z), (uint32_t)j);
    } else if (xd >= 0) {
      localize_case1(g, xd);
      virt(V_H, xd, -1);  // H_v absorbed after the outcome
      out->ev_class[j] = 1;
      emit(OP_MRANDOM, g.r ? F_SIGN : 0, xd, 0, 0, (uint32_t)j);
    } else {
      int v;
      uint8_t op;
      if (anyx) {
        v = lowest(g.x, true);
        localize_case1(g, v);
        virt(V_H, v, -1);
        op = OP_MACTX;
      } else {
        v = lowest(g.z, true);
        localize_case2(g, v);
        op = OP_MACTZ;
      }
      int s = slot_of[v];
      out->ev_class[j] = 2;
      demote(v);
      emit(op, g.r ? F_SIGN : 0, v, s, 0, (uint32_t)j);
    }
    return j;
  }

  // reset correction X^m of event j; xq is the virtual image of X on the qubit
  void reset_fix(const Pauli& xq, int j) {
    emit(OP_CPAULI, xq.r ? F_SIGN : 0, 0, 0, push_pauli(xq), (uint32_t)j);
  }

  // noise site: img holds the virtual images of X and Z on its qubit (and
  // on its second qubit for DEPOLARIZE2)
  void noise(const PhysOp& o, const Pauli* img) {
    uint32_t site = (uint32_t)out->site_type.size();
    out->site_type.push_back((uint8_t)o.ntype);
    out->site_p.push_back(o.arg);
    out->site_img.push_back((uint32_t)out->masks.size());
    push_pauli(img[0]);
    push_pauli(img[1]);
    uint8_t sg = (uint8_t)(img[0].r | (img[1].r << 1));
    if (o.ntype == S_DEP2) {
      push_pauli(img[2]);
      push_pauli(img[3]);
      sg |= (uint8_t)((img[2].r << 2) | (img[3].r << 3));
    }
    out->site_sign.push_back(sg);
    if (!out->code.empty() && out->code.back().op == OP_NOISE && out->code.back().b == site) {
      out->code.back().b = site + 1;  // extend the current block
    } else {
      emit(OP_NOISE, 0, 0, 0, site, site + 1);
    }
  }
};

// ---------------------------------------------------------------- Heisenberg representation
// A node of the Heisenberg intermediate representation (Section 3.1): an
// active operation whose generator is mapped through the physical Cliffords
// only (the virtual basis before any localization), in program order.
struct HNode {
  enum Kind { ROT, MEAS, NOISE, CPAULI, DET, OBS, CFEED, GPHASE, PROBE } kind;
  Pauli g;          // ROT: exp(-i theta g); MEAS: the measured observable;
                    // CPAULI: image of X on the reset qubit
  double theta = 0;
  int event = -1;   // MEAS, CPAULI: measurement event ordinal
  int rec = -1;     // MEAS: record index or -1
  const PhysOp* op = nullptr;  // NOISE, DET, OBS: the parsed operation
  Pauli img[4];     // NOISE: images of X, Z on its qubits
};

static bool commutes(const Pauli& a, const Pauli& b) {
  int par = 0;
  for (size_t w = 0; w < a.x.size(); w++)
    par ^= __builtin_popcountll((a.x[w] & b.z[w]) ^ (a.z[w] & b.x[w])) & 1;
  return par == 0;
}

static bool same_axis(const Pauli& a, const Pauli& b) { return a.x == b.x && a.z == b.z; }

// every fault outcome of a noise node commutes with g
static bool noise_commutes(const HNode& n, const Pauli& g) {
  const int t = n.op->ntype, nq = t == S_DEP2 ? 2 : 1;
  for (int q = 0; q < nq; q++) {
    const bool cx = commutes(n.img[2 * q], g), cz = commutes(n.img[2 * q + 1], g);
    if (t == S_XERR && !cx) return false;
    if (t == S_ZERR && !cz) return false;
    if (t == S_YERR && cx != cz) return false;
    if ((t == S_DEP1 || t == S_DEP2) && !(cx && cz)) return false;
  }
  return true;
}

// whether node n commutes with the operator exp(-i theta g) or a measurement of g
static bool node_commutes(const HNode& n, const Pauli& g) {
  switch (n.kind) {
    case HNode::ROT: case HNode::MEAS: case HNode::CPAULI: case HNode::CFEED: case HNode::PROBE:
      return commutes(n.g, g);
    case HNode::NOISE: return noise_commutes(n, g);
    default: return true;  // detectors and observables are classical
  }
}

// q <- C^dagger q C for the Clifford C = exp(-i c pi/4 g)
static void conj_clifford(Pauli& q, const Pauli& g, int c) {
  c &= 3;
  if (c == 0 || commutes(q, g)) return;
  if (c == 2) { q.r ^= 1; return; }  // exp(-i pi/2 g) = -i g
  Pauli t = g;
  mul_into(t, q, c == 1 ? 1 : 3);    // +i g q (c = 1), -i g q (c = 3)
  q = t;
}

// Middle end (Section 3.1), peephole pass: rotations about one generator
// that meet through operations commuting with it are fused into one; the
// Clifford part of every rotation (the multiple of pi/4 nearest its angle,
// so that the rest lies in (-pi/8, pi/8]) is absorbed into the frame, that
// is, conjugated into every later generator, and a rotation left with angle
// 0 disappears (inverse pairs cancel).
static void hir_peephole(std::vector<HNode>& h) {
  const double q4 = M_PI / 4;
  for (bool changed = true; changed;) {
    changed = false;
    for (size_t i = 0; i < h.size(); i++) {
      if (h[i].kind != HNode::ROT) continue;
      for (size_t j = i + 1; j < h.size();) {
        if (h[j].kind == HNode::ROT && same_axis(h[j].g, h[i].g)) {
          h[i].theta += h[j].g.r == h[i].g.r ? h[j].theta : -h[j].theta;
          h.erase(h.begin() + (long)j);
          changed = true;
          continue;
        }
        if (!node_commutes(h[j], h[i].g)) break;
        j++;
      }
    }
    for (size_t i = 0; i < h.size();) {
      if (h[i].kind != HNode::ROT) { i++; continue; }
      // the multiple of pi/4 nearest the angle, ties towards 0 (|rest| <= pi/8)
      const double th = h[i].theta;
      const long cl = (th >= 0 ? 1 : -1) * (long)std::ceil((std::fabs(th) - M_PI / 8) / q4 - 1e-9);
      const double rest = th - (double)cl * q4;
      const int c = (int)(((cl % 4) + 4) % 4);
      const Pauli g = h[i].g;
      const bool drop = std::fabs(rest) < 1e-12;
      if (c != 0) {
        for (size_t j = i + 1; j < h.size(); j++) {
          conj_clifford(h[j].g, g, c);
          if (h[j].kind == HNode::NOISE)
            for (int k = 0; k < (h[j].op->ntype == S_DEP2 ? 4 : 2); k++) conj_clifford(h[j].img[k], g, c);
        }
        changed = true;
      }
      if (drop) {
        h.erase(h.begin() + (long)i);
        changed = true;
        continue;
      }
      h[i].theta = rest;
      i++;
    }
  }
}

// Middle end, commuting reorder: each measurement (with its reset
// correction, if it has one), taken once in program order, moves earlier past
// every rotation, noise site, measurement and detector that commutes with it
// (with both, for a reset), so that measurements come before the
// non-Clifford rotations they commute with.  A measurement keeps its event
// ordinal (its random draws) and its record index wherever it lands.
static void hir_reorder(std::vector<HNode>& h) {
  std::vector<int> order;  // events in program order
  for (const HNode& n : h)
    if (n.kind == HNode::MEAS) order.push_back(n.event);
  for (int ev : order) {
    size_t j = 0;
    while (!(h[j].kind == HNode::MEAS && h[j].event == ev)) j++;
    const bool reset = j + 1 < h.size() && h[j + 1].kind == HNode::CPAULI && h[j + 1].event == ev;
    const size_t len = reset ? 2 : 1;
    while (j > 0) {
      const HNode& p = h[j - 1];
      // a reset's correction stays with its measurement; a probe's value
      // would change if a measurement moved before it
      if (p.kind == HNode::CPAULI || p.kind == HNode::PROBE) break;
      if (!node_commutes(p, h[j].g) || (reset && !node_commutes(p, h[j + 1].g))) break;
      // a measurement passed over must not be separated from its correction
      std::rotate(h.begin() + (long)(j - 1), h.begin() + (long)j, h.begin() + (long)(j + len));
      j--;
    }
  }
}

}  // namespace

// Survival products of the cumulative hazard (Section 3.2) per chunk:
// S[0] = 1, S[i+1] = S[i] * (1 - p_i) in FP64 with no contraction.
// Paired collapses (PairLine in program.h): the pass each active
// measurement runs on the cooperative HBM tiers, decided as the kernel
// decides it (deferred expansions, carried sums), and the line-complete
// item order of that pass for lines of 2^LB elements (LB = 4 in FP32, 3 in
// FP64).  A pass's items q touch, in each array, L(q) ^ span(offsets), L a
// chain of bit moves and zero insertions; a lane group whose items span
// the directions D reads whole lines when L(D) + span(offsets) holds every
// line bit, so for each line bit the candidate direction is the preimage of
// the bit reduced by the offsets (triangular: offset i has a bit, its
// pivot, that no later offset and no image of L has).
namespace {
struct BitMove {
  int s, top;  // bit s moves to top (top == s: none); top < 0: a zero is inserted at s
};
uint32_t move_fwd(uint32_t x, BitMove t) {
  if (t.top < 0) return ((x >> t.s) << (t.s + 1)) | (x & ((1u << t.s) - 1u));
  if (t.s == t.top) return x;
  return (x & ~(1u << t.s)) | (((x >> t.s) & 1u) << t.top);
}
uint32_t move_inv(uint32_t y, BitMove t) {
  if (t.top < 0) return (((y >> t.s) >> 1) << t.s) | (y & ((1u << t.s) - 1u));
  if (t.s == t.top) return y;
  return (y & ~(1u << t.top)) | (((y >> t.top) & 1u) << t.s);
}
int move_pos(int p, BitMove t) { return t.top < 0 ? (p >= t.s ? p + 1 : p) : (p == t.s ? t.top : p); }
struct PassArray {
  std::vector<BitMove> moves;                   // from the item index outwards
  std::vector<std::pair<uint32_t, int>> offs;  // member offsets and their pivots, triangular
  int width = 0;                                // index bits of the array
};
void line_candidates(const PassArray& a, int LB, std::vector<uint32_t>& out) {
  for (int b = 0; b < LB; b++) {
    uint32_t y = b < a.width ? 1u << b : 0u;
    for (const auto& o : a.offs)
      if ((y >> o.second) & 1u) y ^= o.first;
    for (size_t i = a.moves.size(); i-- > 0;) y = move_inv(y, a.moves[i]);
    out.push_back(y);
  }
}
// the LineEnum of the kernels: up to four spanning directions in reduced
// echelon form (pivot: the highest bit), kept in the order of the candidates
// (items: q < 2^n; a direction outside them is dropped, so that the order
// stays a permutation of the items whatever the offsets)
PairLine pair_line(int kind, const PassArray& first, const PassArray& second, int LB, int n) {
  std::vector<uint32_t> cand;
  line_candidates(first, LB, cand);
  line_candidates(second, LB, cand);
  for (uint32_t& x : cand)
    if (n < 32 && (x >> n) != 0) x = 0;
  PairLine L{};
  uint32_t v[4] = {0, 0, 0, 0};
  int piv[4] = {0, 0, 0, 0}, nv = 0;
  for (uint32_t x : cand) {
    for (int i = 0; i < nv; i++)
      if ((x >> piv[i]) & 1u) x ^= v[i];
    if (!x || nv == 4) continue;
    const int pb = 31 - __builtin_clz(x);
    for (int i = 0; i < nv; i++)
      if ((v[i] >> pb) & 1u) v[i] ^= x;
    v[nv] = x;
    piv[nv++] = pb;
  }
  std::vector<int> pos(piv, piv + nv);
  std::sort(pos.begin(), pos.end());
  for (int i = 0; i < 4; i++) L.v[i] = v[i];
  for (int i = 0; i < 5; i++) L.pos[i] = (int8_t)(i < nv ? pos[i] : 64);
  L.nv = (int8_t)nv;
  L.npos = (int8_t)nv;
  L.kind = (int8_t)kind;
  return L;
}
}  // namespace

static void pair_lines(CompiledProgram& P) {
  P.pline.assign(2, PairLine{});
  P.pline_items.assign(1, 0);
  std::vector<GInstr>& C = P.code;
  auto is_meas = [](uint8_t op) { return op == OP_MACTZ || op == OP_MACTX; };
  auto next_meas = [&](size_t i) -> long {
    for (size_t q = i + 1; q < C.size(); q++)
      if (is_meas(C[q].op)) return (long)q;
    return -1;
  };
  // the folded localization pass that permutes a measurement's pairs
  auto fold_tm = [&](size_t m) -> uint32_t {
    for (size_t q = m; q-- > 0;) {
      const uint8_t op = C[q].op;
      if (op == OP_APERM && (C[q].flags & F_FOLD_NEXT)) return C[q].a;
      if ((op == OP_ASIGN || op == OP_AS) && (C[q].flags & F_FOLD_NEXT)) continue;
      if ((op >= OP_APERM && op <= OP_AROT) || is_meas(op) || op == OP_EXPVAL) return 0;
    }
    return 0;
  };
  int carried = 0, dfr = 0;  // carried: 1 the next measurement's sums, 2 the next two's joint sums
  bool pend = false;
  size_t pa = 0;
  for (size_t i = 0; i < C.size(); i++) {
    const GInstr in = C[i];
    const int k = i == 0 ? 0 : P.k_after[i - 1];
    switch (in.op) {
      case OP_APERM: case OP_ASIGN: case OP_AS:
        if (!(in.flags & F_FOLD_NEXT)) { dfr = 0; carried = 0; }
        break;
      case OP_AROT: case OP_APERM2: case OP_AH: case OP_EXPVAL: dfr = 0; carried = 0; break;
      case OP_EXPAND:
        if (dfr == kDeferMax) dfr--;
        dfr++;
        carried = 0;
        break;
      case OP_MACTZ: case OP_MACTX: {
        const bool fuse = (in.flags & F_FUSE_NEXT) && k >= 2;
        const long nx = fuse ? next_meas(i) : -1;
        const bool joint = fuse && !dfr && k - 1 >= 3 && nx >= 0 && (C[nx].flags & F_FUSE_NEXT);
        const long nnx = joint ? next_meas((size_t)nx) : -1;
        int kind = PP_NONE, nitems = 0;  // the pass's items: q < 2^nitems
        PassArray a1, a2;
        auto bit = [](int s) { return 1u << s; };
        if (pend) {
          // B (this) of the pair with A: the vector has k + 1 slots, the result k - 1
          const int kv = k + 1, kw = k - 1;
          const int sA = C[pa].s, sB = in.s;
          const BitMove mb{sB, kv - 2}, ma{sA, kv - 1};
          const uint32_t dA = bit(sA) ^ fold_tm(pa), dB = move_fwd(bit(sB) ^ fold_tm(i), ma);
          a1.moves = {mb, ma};
          a1.offs = {{dA, sA}, {dB, move_pos(sB, ma)}};
          a1.width = kv;
          a2.width = kw;
          auto up = [&](uint32_t x) { return move_fwd(move_fwd(x, mb), ma); };
          auto upp = [&](int p) { return move_pos(move_pos(p, mb), ma); };
          if (joint) {
            kind = PP_PAIR_JOINT;
            nitems = kw - 2;
            const int sC = C[nx].s, sD = C[nnx].s;
            const BitMove mc{sC, kw - 1}, md{sD, kw - 2};
            const uint32_t oc = bit(sC) ^ fold_tm(nx), od = move_fwd(bit(sD) ^ fold_tm(nnx), mc);
            const int pc = sC, pd = move_pos(sD, mc);
            a2.moves = {md, mc};
            a2.offs = {{oc, pc}, {od, pd}};
            a1.moves = {md, mc, mb, ma};
            a1.offs.push_back({up(oc), upp(pc)});
            a1.offs.push_back({up(od), upp(pd)});
          } else if (fuse) {
            kind = PP_PAIR_NEXT;
            nitems = kw - 1;
            const int sC = C[nx].s;
            const BitMove mc{sC, -1};
            const uint32_t oc = bit(sC) ^ fold_tm(nx);
            a2.moves = {mc};
            a2.offs = {{oc, sC}};
            a1.moves = {mc, mb, ma};
            a1.offs.push_back({up(oc), upp(sC)});
          } else {
            kind = PP_PAIR;
            nitems = kw;
          }
          pend = false;
          carried = joint ? 2 : fuse ? 1 : 0;
        } else if ((in.flags & F_FUSE_NEXT) && k >= 3 && !dfr && carried != 1) {
          // A of a pair with the next measurement: a read pass for the joint
          // sums unless they are carried
          if (!carried) {
            kind = PP_JOINT_READ;
            nitems = k - 2;
            const long b = next_meas(i);
            const int sA = in.s, sB = C[b].s;
            const BitMove mb{sB, k - 2}, ma{sA, k - 1};
            a1.moves = {mb, ma};
            a1.offs = {{bit(sA) ^ fold_tm(i), sA}, {move_fwd(bit(sB) ^ fold_tm((size_t)b), ma), move_pos(sB, ma)}};
            a1.width = k;
          }
          pend = true;
          pa = i;
          carried = 0;
        } else if (dfr) {
          carried = 0;  // the cooperative tiers carry nothing out of a deferred collapse
        } else {
          if (joint) {
            // a single collapse (k slots to k - 1) taking the joint sums of C, D
            kind = PP_SINGLE_JOINT;
            nitems = k - 3;
            const int s = in.s, sC = C[nx].s, sD = C[nnx].s;
            const BitMove mc{sC, k - 2}, md{sD, k - 3}, ms{s, k - 1};
            const uint32_t oc = bit(sC) ^ fold_tm(nx), od = move_fwd(bit(sD) ^ fold_tm(nnx), mc);
            const int pc = sC, pd = move_pos(sD, mc);
            a2.moves = {md, mc};
            a2.offs = {{oc, pc}, {od, pd}};
            a2.width = k - 1;
            a1.moves = {md, mc, ms};
            a1.offs = {{bit(s) ^ fold_tm(i), s}, {move_fwd(oc, ms), move_pos(pc, ms)}, {move_fwd(od, ms), move_pos(pd, ms)}};
            a1.width = k;
          }
          carried = joint ? 2 : fuse ? 1 : 0;
        }
        dfr = 0;
        if (kind != PP_NONE && P.pline.size() / 2 < 65536) {
          C[i].u = (uint16_t)(P.pline.size() / 2);
          P.pline.push_back(pair_line(kind, a1, a2, 4, nitems));
          P.pline.push_back(pair_line(kind, a1, a2, 3, nitems));
          P.pline_items.push_back(nitems);
        }
        break;
      }
      default: break;
    }
  }
}

static void survival_tables(CompiledProgram& P) {
  int ns = (int)P.site_p.size();
  P.nchunks = (ns + kChunk - 1) / kChunk;
  P.surv.assign((size_t)P.nchunks * (kChunk + 1), 0.0);
  for (int c = 0; c < P.nchunks; c++) {
    volatile double s = 1.0;
    double* S = &P.surv[(size_t)c * (kChunk + 1)];
    S[0] = s;
    int lo = c * kChunk, hi = std::min(ns, lo + kChunk);
    for (int i = lo; i < hi; i++) {
      volatile double q = 1.0 - P.site_p[i];
      s = s * q;
      S[i - lo + 1] = s;
    }
    for (int i = hi - lo + 1; i <= kChunk; i++) S[i] = 0.0;  // beyond the chunk: never fires
  }
}

// Per-shot algorithmic work, summed over the compiled stream with the k in
// force at each instruction (A = 2^k amplitudes before the instruction, a =
// bytes per amplitude, W = frame words; a 64-bit word operation counts as two
// 32-bit lane operations; both Pauli frames are updated by frame operations).
//   fan (CX / CZ / target fan)   16W + 12 int ops
//   frame S or H                 12 int ops
//   deterministic measurement    8W + 8 int ops
//   dormant random measurement   22 int ops
//   reset correction             16W int ops
//   noise block                  2 int ops, + 158 + 24W per expected fault
//                                (draw, search, apply), + 158 per chunk
//   detector / observable        2/64 int op per reference (word XOR)
//   EXPAND        6A flops,  2A a bytes     AROT   3A flops,  A a bytes
//   AH            4A flops,  2A a bytes     AS / ASIGN / APERM / APERM2: A a bytes
//   active Z meas 5A flops,  2A a bytes     active X meas 8A flops, 2.5A a bytes
//                 (+ 110 int ops: draw and bookkeeping)
CostModel cost_model(const CompiledProgram& P, bool fp64) {
  CostModel c;
  const double W = P.W, a = fp64 ? 16.0 : 8.0;
  for (size_t i = 0; i < P.code.size(); i++) {
    const GInstr& in = P.code[i];
    int kb = (int)(i == 0 ? 0 : P.k_after[i - 1]);
    double A = std::ldexp(1.0, kb);
    c.instructions += 1;
    switch (in.op) {
      case OP_FANCX: case OP_FANCZ: case OP_FAN2: c.int_ops += 16 * W + 12; break;
      case OP_FS: case OP_FH: c.int_ops += 12; break;
      case OP_APERM: case OP_APERM2: case OP_ASIGN: case OP_AS: c.vector_bytes += A * a; c.int_ops += 4; break;
      case OP_AH: c.flops += 4 * A; c.vector_bytes += 2 * A * a; break;
      case OP_EXPAND: c.flops += 6 * A; c.vector_bytes += 2 * A * a; c.int_ops += 12; break;
      case OP_AROT: c.flops += 3 * A; c.vector_bytes += A * a; c.int_ops += 4; break;
      case OP_MSTATIC: c.int_ops += 8 * W + 8; break;
      case OP_MRANDOM: c.int_ops += 22; break;
      case OP_MACTZ: c.flops += 5 * A; c.vector_bytes += 2 * A * a; c.int_ops += 110; break;
      case OP_MACTX: c.flops += 8 * A; c.vector_bytes += 2.5 * A * a; c.int_ops += 110; break;
      case OP_CPAULI: case OP_CFEED: c.int_ops += 16 * W; break;
      case OP_EXPVAL: if (!(in.flags & F_ZERO)) { c.flops += 8 * A; c.vector_bytes += 2 * A * a; } break;
      case OP_NOISE: {
        double f = 0;
        for (uint32_t s = in.a; s < in.b; s++) f += P.site_p[s];
        c.expected_faults += f;
        c.int_ops += 2 + f * (158 + 24 * W);
        break;
      }
      case OP_DET: case OP_POSTSELECT: case OP_OBS: c.int_ops += in.u * 2.0 / 64.0; break;
      default: break;
    }
  }
  c.int_ops += 158.0 * P.nchunks;
  c.record_bytes = (P.nrec + P.ndet + P.nobs) / 8.0;

  // Fused passes of the HBM tiers: localization passes folded into the next
  // measurement or H pass move nothing (that pass reads through them, the H
  // pass out of place and through deferred expansions, and also applies a
  // rotation on its slot that directly follows it); up to kDeferMax
  // trailing expansions move
  // nothing until the next active measurement reads the stored 2^(k-d)
  // elements (once for its branch sums, once for its collapse, which writes
  // all 2^(k-1) outputs, and on the lane tier carries the next
  // measurement's branch sums), an expansion beyond them
  // applies the oldest one (reads and writes 2^(k-d) elements), and any
  // other vector instruction first writes the deferred part; a collapse
  // reads the vector and writes half of it; its reduction pass is skipped
  // when the previous measurement's collapse carried its branch sums.  On
  // the cooperative tiers (no carry out of a collapse that reads deferred
  // expansions) two consecutive measurements A and B with only frame work
  // between them collapse together: A moves nothing (its joint branch sums
  // with B carried by the previous collapse, else one read pass), B reads
  // the 2^(k+1) elements and writes 2^(k-1).
  auto next_fused = [&](size_t i) -> const GInstr* {
    for (size_t q = i + 1; q < P.code.size(); q++)
      if (P.code[q].op == OP_MACTZ || P.code[q].op == OP_MACTX) return &P.code[q];
    return nullptr;
  };
  for (int tier = 0; tier < 3; tier++) {  // lane, group, group of the batched launch
    const bool lane_tier = tier == 0, pairs = tier == 1;
    double& bytes = tier == 0 ? c.vector_bytes_fused : tier == 1 ? c.vector_bytes_fused_group : c.vector_bytes_fused_batch;
    int carried = 0;  // 1: the next measurement's sums, 2: the next two's joint sums
    bool pend = false;
    int dfr = 0;
    for (size_t i = 0; i < P.code.size(); i++) {
      const GInstr& in = P.code[i];
      const int k = i == 0 ? 0 : P.k_after[i - 1];
      const double A = std::ldexp(1.0, k);
      const double stored = std::ldexp(1.0, k - dfr);
      auto materialize = [&]() {
        if (dfr) bytes += (stored + (A - stored)) * a;
        dfr = 0;
      };
      switch (in.op) {
        case OP_APERM: case OP_ASIGN: case OP_AS:
          if (!(in.flags & F_FOLD_NEXT)) { materialize(); bytes += A * a; carried = 0; }
          break;
        case OP_AROT:
          // directly after an H on its slot, the H pass applies it
          if (i > 0 && P.code[i - 1].op == OP_AH && P.code[i - 1].s == in.s) break;
          materialize();
          bytes += A * a;
          carried = 0;
          break;
        case OP_APERM2: materialize(); bytes += A * a; carried = 0; break;
        case OP_AH: bytes += 2 * A * a; dfr = 0; carried = 0; break;  // reads through deferred factors
        case OP_EXPAND:
          if (dfr == kDeferMax) {
            bytes += 2 * stored * a;
            dfr--;
          }
          dfr++;
          carried = 0;
          break;
        case OP_MACTZ: case OP_MACTX: {
          const bool fuse = (in.flags & F_FUSE_NEXT) && k >= 2;
          const GInstr* nx = fuse ? next_fused(i) : nullptr;
          const GInstr* nnx = nx && (nx->flags & F_FUSE_NEXT) ? next_fused((size_t)(nx - P.code.data())) : nullptr;
          // FP32 pairs only measurements whose slots lie above the line bits
          // (the kernels' rule; FP64 walks line-complete orders instead)
          auto slot_ok = [&](const GInstr* g) { return g && (fp64 || g->s >= 4); };
          const int min_k = fp64 ? 3 : 17;  // and FP32 pairs vectors of 2^17 amplitudes or more
          const int carry = !fuse || (!lane_tier && dfr) ? 0
                            : (pairs && !dfr && k - 1 >= min_k && nx && (nx->flags & F_FUSE_NEXT) &&
                               (pend || slot_ok(&in)) && slot_ok(nx) && slot_ok(nnx)) ? 2 : 1;
          if (pend) {
            bytes += 2.5 * A * a;
            pend = false;
          } else if (pairs && (in.flags & F_FUSE_NEXT) && k >= min_k && !dfr && carried != 1 && slot_ok(&in) &&
                     slot_ok(next_fused(i))) {
            if (!carried) bytes += A * a;
            pend = true;
            carried = 0;
            c.pair_starts++;
            break;
          } else if (dfr) {
            bytes += 2 * stored * a + 0.5 * A * a;
          } else {
            bytes += (carried ? 0.0 : A * a) + 1.5 * A * a;
          }
          carried = carry;
          dfr = 0;
          break;
        }
        default: break;
      }
    }
  }

  // Bit-sliced form (k_max = 0): a frame word holds one bit of 32 shots, so
  // frame, parity, accumulator and record work is shared by 32 shots, while
  // the per-shot draws (first gap-sampler draw of every chunk, one draw per
  // fault, one draw per 128-event block of dormant random outcomes) and the
  // per-shot bit of each dormant random outcome are not.
  {
    auto bits = [&](uint32_t off, int words) {
      double t = 0;
      for (int w = 0; w < words; w++) t += __builtin_popcountll(P.masks[off + w]);
      return t;
    };
    double shared = 0, per_shot = 158.0 * P.nchunks;
    std::vector<char> block_seen;
    for (const GInstr& in : P.code) {
      switch (in.op) {
        case OP_FANCX: case OP_FANCZ: case OP_FAN2: shared += 4 * bits(in.a, P.W) + 4; break;
        case OP_FS: shared += 2; break;
        case OP_MSTATIC: case OP_MRANDOM: {
          const int r = P.ev_rec[in.b];
          const double tg = r >= 0 ? (double)(P.rec_tgt_off[r + 1] - P.rec_tgt_off[r]) : 0.0;
          if (in.op == OP_MSTATIC) shared += 2 * bits(in.a, P.W) + 2 + tg + 1;
          else {
            shared += 5 + tg + 1;
            per_shot += 4;
            const uint32_t blk = in.b >> 7;
            if (block_seen.size() <= blk) block_seen.resize(blk + 1, 0);
            if (!block_seen[blk]) per_shot += 100;
            block_seen[blk] = 1;
          }
          break;
        }
        case OP_CPAULI: shared += 2 * bits(in.a, 2 * P.W); break;
        case OP_NOISE: {
          double f = 0;
          for (uint32_t s = in.a; s < in.b; s++) f += P.site_p[s];
          shared += 3;
          per_shot += f * 166;
          break;
        }
        case OP_DET: case OP_POSTSELECT: shared += 1; break;
        default: break;
      }
    }
    c.int_ops_bitsliced = per_shot + shared / 32.0;
  }
  return c;
}

// Split form (program.h): the frame-only and vector-only streams, and the
// GF(2) dependency of the needed bits and of every output row on the active
// measurement outcomes, found by running the frame instructions on masks:
// each full-frame bit carries the set of active outcomes it depends on
// (the frames' other inputs, faults and dormant random bits, are sampled by
// the frame stream itself).  An active measurement leaves x_v = m ^ sign; a
// reset's correction X^m adds the dependency of m to the bits it flips; a
// dormant random measurement leaves x_v = m ^ sign with m independent of
// the active outcomes.
static void build_split(CompiledProgram& P) {
  const int n = P.nq, W = P.W;
  int nact = 0;
  for (int cl : P.ev_class) nact += cl == 2;
  P.nactive = nact;
  P.split_ok = P.kmax > 0 && nact <= kSplitMaxActive && P.nprobes == 0;
  if (!P.split_ok) return;
  const int DW = std::max(1, (nact + 63) / 64);
  P.dep_words = DW;
  using Dep = std::vector<uint64_t>;
  const Dep zero(DW, 0);
  auto xr = [&](Dep& a, const Dep& b) {
    for (int w = 0; w < DW; w++) a[w] ^= b[w];
  };
  auto each_bit = [&](uint32_t off, auto fn) {
    for (int w = 0; w < W; w++) {
      uint64_t m = P.masks[off + w];
      while (m) {
        fn(w * 64 + __builtin_ctzll(m));
        m &= m - 1;
      }
    }
  };
  std::vector<Dep> dx(n, zero), dz(n, zero), ev_dep(std::max(P.nevents, 1), zero);
  std::vector<Dep> rows(P.nrec + P.ndet + P.nobs, zero);  // meas, det, obs rows
  P.vev_rec.assign(std::max(P.nevents, 1), -1);
  int nb = 0, act = 0;
  auto need = [&](const Dep& d) {
    P.vdep.insert(P.vdep.end(), d.begin(), d.end());
    return nb++;
  };
  auto vpush = [&](GInstr g, size_t i) {
    P.vcode.push_back(g);
    P.vk_after.push_back(P.k_after[i]);
  };
  for (size_t i = 0; i < P.code.size(); i++) {
    GInstr in = P.code[i];
    const int v = in.v;
    switch (in.op) {
      case OP_FANCX: {
        Dep par = zero;
        each_bit(in.a, [&](int q) { xr(dx[q], dx[v]); xr(par, dz[q]); });
        xr(dz[v], par);
        P.fcode.push_back(in);
        break;
      }
      case OP_FANCZ: {
        Dep par = zero;
        each_bit(in.a, [&](int q) { xr(dz[q], dx[v]); xr(par, dx[q]); });
        xr(dz[v], par);
        P.fcode.push_back(in);
        break;
      }
      case OP_FAN2: {
        Dep par = zero;
        each_bit(in.a, [&](int q) { xr(dz[q], dz[v]); xr(par, dx[q]); });
        xr(dx[v], par);
        P.fcode.push_back(in);
        break;
      }
      case OP_FS: xr(dz[v], dx[v]); P.fcode.push_back(in); break;
      case OP_FH: std::swap(dx[v], dz[v]); P.fcode.push_back(in); break;
      case OP_EXPAND: {
        std::swap(dx[v], dz[v]);
        GInstr h{};
        h.op = OP_FH;
        h.v = (uint16_t)v;
        P.fcode.push_back(h);
        GInstr e{};
        e.op = OP_EMIT;
        e.v = (uint16_t)v;
        e.u = (uint16_t)nb;
        P.fcode.push_back(e);
        in.v = (uint16_t)need(dx[v]);
        vpush(in, i);
        break;
      }
      case OP_AROT: {
        GInstr e{};
        e.op = OP_EMIT;
        e.v = (uint16_t)v;
        e.u = (uint16_t)nb;
        P.fcode.push_back(e);
        in.v = (uint16_t)need(dx[v]);
        vpush(in, i);
        break;
      }
      case OP_APERM: case OP_ASIGN: case OP_APERM2: case OP_AS: case OP_AH:
        vpush(in, i);
        break;
      case OP_MSTATIC: {
        Dep d = zero;
        each_bit(in.a, [&](int q) { xr(d, dx[q]); });
        ev_dep[in.b] = d;
        if (P.ev_rec[in.b] >= 0) rows[P.ev_rec[in.b]] = d;
        P.fcode.push_back(in);
        break;
      }
      case OP_MRANDOM: {
        // the outcome is independent of the active outcomes; x_v = m ^ sign
        const Dep ox = dx[v];
        dx[v] = zero;
        dz[v] = ox;
        ev_dep[in.b] = zero;
        P.fcode.push_back(in);
        break;
      }
      case OP_MACTZ: case OP_MACTX: {
        const bool isx = in.op == OP_MACTX;
        GInstr f{};
        f.op = OP_MACTF;
        f.flags = (uint8_t)((in.flags & F_SIGN) | (isx ? F_XMEAS : 0));
        f.v = (uint16_t)v;
        f.u = (uint16_t)nb;
        f.b = in.b;
        P.fcode.push_back(f);
        const int row = need(isx ? dz[v] : dx[v]);  // p
        need(zero);                                 // pn: noise frame only
        in.v = (uint16_t)row;
        in.a = (uint32_t)act;
        vpush(in, i);
        if (isx) std::swap(dx[v], dz[v]);
        Dep e = zero;
        e[act >> 6] |= 1ull << (act & 63);
        dx[v] = e;
        ev_dep[in.b] = e;
        if (P.ev_rec[in.b] >= 0) rows[P.ev_rec[in.b]] = e;
        P.vev_rec[in.b] = act++;
        break;
      }
      case OP_CPAULI: case OP_CFEED: {
        // X^m of a reset (the event's outcome) or a feed-forward Pauli (a record)
        const Dep d = in.op == OP_CPAULI ? ev_dep[in.b] : rows[in.b];
        each_bit(in.a, [&](int q) { xr(dx[q], d); });
        each_bit(in.a + W, [&](int q) { xr(dz[q], d); });
        P.fcode.push_back(in);
        break;
      }
      case OP_DET: {
        Dep d = zero;
        for (uint32_t k = 0; k < in.u; k++) xr(d, rows[P.refs[in.a + k]]);
        rows[P.nrec + in.b] = d;
        P.fcode.push_back(in);
        break;
      }
      case OP_OBS: {
        for (uint32_t k = 0; k < in.u; k++) xr(rows[P.nrec + P.ndet + in.b], rows[P.refs[in.a + k]]);
        P.fcode.push_back(in);
        break;
      }
      case OP_END:
        P.fcode.push_back(in);
        vpush(in, i);
        break;
      default:  // noise blocks, phase-only instructions
        P.fcode.push_back(in);
        break;
    }
  }
  P.nbits = nb;
  if (P.vdep.empty()) P.vdep.assign(DW, 0);
  P.xdep_off.assign(1, 0);
  for (const Dep& d : rows) {
    for (int a = 0; a < nact; a++)
      if ((d[a >> 6] >> (a & 63)) & 1) P.xdep.push_back((uint32_t)a);
    P.xdep_off.push_back((uint32_t)P.xdep.size());
  }
  if (P.xdep.empty()) P.xdep.push_back(0);
}

int compile_text(const char* text, size_t len, const CompileOptions& opts, CompiledProgram& P, std::string& err) {
  Lines L;
  {
    std::string all(text, len);
    size_t pos = 0;
    int line = 0;
    while (pos <= all.size()) {
      size_t e = all.find('\n', pos);
      if (e == std::string::npos) e = all.size();
      std::string s = all.substr(pos, e - pos);
      line++;
      size_t h = s.find('#');
      if (h != std::string::npos) s = s.substr(0, h);
      s = strip(s);
      if (!s.empty()) {
        L.v.push_back(s);
        L.lineno.push_back(line);
      }
      if (e == all.size()) break;
      pos = e + 1;
    }
  }
  Parsed ps;
  size_t i = 0;
  int code = 0;
  if (!parse_range(L, i, ps, 0, err, code)) return code;
  int n = ps.nq > 0 ? ps.nq : 1;
  if (n > 64 * kMaxWords) {
    err = "more than 256 qubits";
    return 3;
  }
  P = CompiledProgram();
  P.nq = n;
  P.W = (n + 63) / 64;
  Compiler C(n, &P);
  C.drop_phases = opts.drop_phases;
  const int k_limit = opts.k_limit > 0 && opts.k_limit < kMaxK ? opts.k_limit : kMaxK;
  int rec = 0;
  auto classical = [&](const PhysOp& o) {
    uint32_t off = (uint32_t)P.refs.size();
    for (int r : o.refs) P.refs.push_back((uint32_t)r);
    if (o.refs.size() > 65535) { err = "too many detector references"; return false; }
    uint32_t idx = o.kind == K_DET ? (uint32_t)P.ndet++ : (uint32_t)o.obs;
    C.emit(o.kind == K_DET ? OP_DET : OP_OBS, 0, 0, 0, off, idx, (int)o.refs.size());
    return true;
  };
  auto over_limit = [&]() {
    if (P.kmax <= k_limit) return false;
    err = k_limit == kMaxK ? "active dimension exceeds the format limit" : "active dimension exceeds k_limit";
    return true;
  };
  if (opts.hir_passes == 0) {
    // operations as written: Heisenberg mapping and localization in one sweep
    for (const PhysOp& o : ps.ops) {
      switch (o.kind) {
        case K_H: case K_S: case K_SDAG: case K_X: case K_Y: case K_Z: case K_CX: case K_CZ: case K_SWAP:
          C.phys(o.kind, o.a, o.b);
          break;
        case K_ROTZ: C.rotation(C.iz[o.a], o.arg); break;
        case K_PROT: C.rotation(C.product(o.prod), o.arg); break;
        case K_MPP: C.measure(C.product(o.prod), rec++); break;
        case K_CFEED: C.feed(C.image(o.a, o.prod[0].second), o.refs[0]); break;
        case K_GPHASE: C.global_phase(o.arg); break;
        case K_EXPVAL: C.probe(C.product(o.prod), o.obs); break;
        case K_M: C.measure(C.image(o.a, 'Z'), rec++); break;
        case K_MX: C.measure(C.image(o.a, 'X'), rec++); break;
        case K_MR: { int j = C.measure(C.image(o.a, 'Z'), rec++); C.reset_fix(C.ix[o.a], j); break; }
        case K_R: { int j = C.measure(C.image(o.a, 'Z'), -1); C.reset_fix(C.ix[o.a], j); break; }
        case K_NOISE: {
          const Pauli img[4] = {C.ix[o.a], C.iz[o.a], o.ntype == S_DEP2 ? C.ix[o.b] : Pauli(), o.ntype == S_DEP2 ? C.iz[o.b] : Pauli()};
          C.noise(o, img);
          break;
        }
        case K_DET:
        case K_OBS:
          if (!classical(o)) return 3;
          break;
      }
      if (over_limit()) return 3;
    }
  } else {
    // front end: the Heisenberg representation (physical Cliffords only)
    Compiler F(n, &P);
    std::vector<HNode> h;
    int nev = 0;
    for (const PhysOp& o : ps.ops) {
      HNode nd{};
      switch (o.kind) {
        case K_H: case K_S: case K_SDAG: case K_X: case K_Y: case K_Z: case K_CX: case K_CZ: case K_SWAP:
          F.phys(o.kind, o.a, o.b);
          continue;
        case K_ROTZ: nd.kind = HNode::ROT; nd.g = F.iz[o.a]; nd.theta = o.arg; break;
        case K_PROT: nd.kind = HNode::ROT; nd.g = F.product(o.prod); nd.theta = o.arg; break;
        case K_CFEED: nd.kind = HNode::CFEED; nd.g = F.image(o.a, o.prod[0].second); nd.rec = o.refs[0]; break;
        case K_GPHASE: nd.kind = HNode::GPHASE; nd.g = Pauli(P.W); nd.theta = o.arg; break;
        case K_EXPVAL: nd.kind = HNode::PROBE; nd.g = F.product(o.prod); nd.rec = o.obs; break;
        case K_MPP:
          nd.kind = HNode::MEAS;
          nd.g = F.product(o.prod);
          nd.event = nev++;
          nd.rec = rec++;
          h.push_back(nd);
          continue;
        case K_M: case K_MX: case K_MR: case K_R:
          nd.kind = HNode::MEAS;
          nd.g = F.image(o.a, o.kind == K_MX ? 'X' : 'Z');
          nd.event = nev++;
          nd.rec = o.kind == K_R ? -1 : rec++;
          h.push_back(nd);
          if (o.kind == K_MR || o.kind == K_R) {
            HNode cp{};
            cp.kind = HNode::CPAULI;
            cp.g = F.ix[o.a];
            cp.event = nd.event;
            h.push_back(cp);
          }
          continue;
        case K_NOISE:
          nd.kind = HNode::NOISE;
          nd.op = &o;
          nd.g = Pauli(P.W);
          nd.img[0] = F.ix[o.a];
          nd.img[1] = F.iz[o.a];
          if (o.ntype == S_DEP2) { nd.img[2] = F.ix[o.b]; nd.img[3] = F.iz[o.b]; }
          break;
        case K_DET: case K_OBS:
          nd.kind = o.kind == K_DET ? HNode::DET : HNode::OBS;
          nd.op = &o;
          nd.g = Pauli(P.W);
          break;
      }
      h.push_back(nd);
    }
    P.ev_rec.assign(nev, -1);
    P.ev_class.assign(nev, 0);
    // middle end
    if (opts.hir_passes & 1) hir_peephole(h);
    if (opts.hir_passes & 2) hir_reorder(h);
    if (opts.hir_passes & 1) hir_peephole(h);
    // back end: localization of the optimized representation
    for (const HNode& nd : h) {
      switch (nd.kind) {
        case HNode::ROT: C.rotation(C.map(nd.g), nd.theta); break;
        case HNode::MEAS: C.measure(C.map(nd.g), nd.rec, nd.event); break;
        case HNode::CPAULI: C.reset_fix(C.map(nd.g), nd.event); break;
        case HNode::CFEED: C.feed(C.map(nd.g), nd.rec); break;
        case HNode::GPHASE: C.global_phase(nd.theta); break;
        case HNode::PROBE: C.probe(C.map(nd.g), nd.rec); break;
        case HNode::NOISE: {
          const int m = nd.op->ntype == S_DEP2 ? 4 : 2;
          Pauli img[4];
          for (int k = 0; k < m; k++) img[k] = C.map(nd.img[k]);
          C.noise(*nd.op, img);
          break;
        }
        case HNode::DET: case HNode::OBS:
          if (!classical(*nd.op)) return 3;
          break;
      }
      if (over_limit()) return 3;
    }
    P.nevents = nev;
  }
  C.emit(OP_END, 0, 0, 0, 0, 0);
  P.nrec = rec;
  P.nobs = ps.nobs;
  P.final_slots = C.q_at;
  // Accumulator rows for kernels that XOR detectors and observables
  // incrementally: a detector's row is live from its first record to its
  // DETECTOR instruction, so rows are allocated like registers over those
  // intervals (the DET instruction carries its row in `s` and the kernel
  // clears the row after emitting it); observables keep rows to the end.
  // rec_tgt lists the rows each record feeds (a record counted twice cancels).
  {
    std::vector<int> rec_at(P.nrec, 0);  // instruction producing each record
    for (size_t i = 0; i < P.code.size(); i++) {
      const GInstr& in = P.code[i];
      if (in.op == OP_MSTATIC || in.op == OP_MRANDOM || in.op == OP_MACTZ || in.op == OP_MACTX) {
        int r = P.ev_rec[in.b];
        if (r >= 0) rec_at[r] = (int)i;
      }
    }
    struct Iv { int start, end; size_t instr; };
    std::vector<Iv> ivs;
    for (size_t i = 0; i < P.code.size(); i++) {
      const GInstr& in = P.code[i];
      if (in.op != OP_DET) continue;
      int start = (int)i;
      for (uint32_t k = 0; k < in.u; k++) start = std::min(start, rec_at[P.refs[in.a + k]]);
      ivs.push_back(Iv{start, (int)i, i});
    }
    std::vector<Iv> by_start = ivs;
    std::stable_sort(by_start.begin(), by_start.end(), [](const Iv& x, const Iv& y) { return x.start < y.start; });
    std::vector<int> slot_end;  // per slot: end of its current interval (-1 free)
    std::vector<uint32_t> det_row(P.ndet, 0);
    for (const Iv& iv : by_start) {
      int s = -1;
      for (size_t k = 0; k < slot_end.size(); k++)
        if (slot_end[k] < iv.start) { s = (int)k; break; }
      if (s < 0) { s = (int)slot_end.size(); slot_end.push_back(0); }
      slot_end[s] = iv.end;
      P.code[iv.instr].s = (uint16_t)s;
      det_row[P.code[iv.instr].b] = (uint32_t)s;
    }
    P.ndet_rows = (int)slot_end.size();
    std::vector<std::vector<uint32_t>> tg(P.nrec);
    auto toggle = [&](uint32_t r, uint32_t t) {
      auto& v = tg[r];
      auto it = std::find(v.begin(), v.end(), t);
      if (it == v.end()) v.push_back(t);
      else v.erase(it);
    };
    for (const GInstr& in : P.code) {
      if (in.op != OP_DET && in.op != OP_OBS) continue;
      uint32_t t = in.op == OP_DET ? det_row[in.b] : (uint32_t)P.ndet_rows + in.b;
      for (uint32_t i = 0; i < in.u; i++) toggle(P.refs[in.a + i], t);
    }
    P.rec_tgt_off.assign(1, 0);
    for (int r = 0; r < P.nrec; r++) {
      for (uint32_t t : tg[r]) P.rec_tgt.push_back(t);
      P.rec_tgt_off.push_back((uint32_t)P.rec_tgt.size());
    }
    if (P.rec_tgt.empty()) P.rec_tgt.push_back(0);
  }
  // Dormant random events per 128-event block; each MRANDOM learns its index.
  {
    int nblocks = (P.nevents + 127) / 128;
    std::vector<std::vector<int>> blk(nblocks > 0 ? nblocks : 1);
    for (GInstr& in : P.code) {
      if (in.op != OP_MRANDOM) continue;
      auto& v = blk[in.b >> 7];
      in.u = (uint16_t)v.size();
      v.push_back((int)(in.b & 127));
    }
    P.rblk_off.assign(1, 0);
    for (auto& v : blk) {
      for (int e : v) P.rblk_ev.push_back((uint8_t)e);
      P.rblk_off.push_back((uint32_t)P.rblk_ev.size());
      P.rblk_max = std::max<int>(P.rblk_max, (int)v.size());
    }
    if (P.rblk_ev.empty()) P.rblk_ev.push_back(0);
  }
  // Fusion marks for the active-vector passes (see program.h): the
  // localization passes of an active measurement that can be read through,
  // and measurements whose successor's branch sums their collapse computes.
  {
    auto touches_vector = [](uint8_t op) {
      return (op >= OP_APERM && op <= OP_AROT) || op == OP_MACTZ || op == OP_MACTX || op == OP_EXPVAL;
    };
    auto is_meas = [](uint8_t op) { return op == OP_MACTZ || op == OP_MACTX; };
    std::vector<size_t> vecops;
    for (size_t i = 0; i < P.code.size(); i++)
      if (touches_vector(P.code[i].op)) vecops.push_back(i);
    for (size_t n = 0; n < vecops.size(); n++) {
      const GInstr& m = P.code[vecops[n]];
      if (!is_meas(m.op) && m.op != OP_AH) continue;  // an H pass on the slot reads through them too
      size_t j = n;
      const uint8_t order[3] = {OP_AS, OP_ASIGN, OP_APERM};  // backwards from the measurement
      for (uint8_t want : order) {
        if (j == 0) break;
        GInstr& g = P.code[vecops[j - 1]];
        if (g.op == want && g.s == m.s) {
          g.flags |= F_FOLD_NEXT;
          j--;
        }
      }
    }
    for (size_t n = 0; n < vecops.size(); n++) {
      GInstr& in = P.code[vecops[n]];
      if (!is_meas(in.op)) continue;
      size_t j = n + 1;
      while (j < vecops.size() && (P.code[vecops[j]].flags & F_FOLD_NEXT)) j++;
      if (j < vecops.size() && is_meas(P.code[vecops[j]].op)) in.flags |= F_FUSE_NEXT;
    }
  }
  pair_lines(P);
  survival_tables(P);
  if (P.masks.empty()) P.masks.push_back(0);
  for (const GInstr& in : P.code) P.has_cfeed = P.has_cfeed || in.op == OP_CFEED;
  P.nprobes = ps.nprobes;
  build_split(P);
  // Post-selected detectors (Section 3.2, post-selection): their OP_DET
  // becomes OP_POSTSELECT, which ends a shot that reads 1.  The split form's
  // frame pass cannot end shots, so such programs do not use it.
  for (size_t w = 0; w < opts.postselect.size(); w++)
    for (int b = 0; b < 64; b++)
      if (((opts.postselect[w] >> b) & 1u) && (int64_t)w * 64 + b >= P.ndet) {
        err = "post-selected detector " + std::to_string(w * 64 + b) + " does not exist (the circuit has " +
              std::to_string(P.ndet) + ")";
        return 4;
      }
  for (GInstr& in : P.code)
    if (in.op == OP_DET && (opts.postselect_all || (in.b / 64 < opts.postselect.size() &&
                                                    ((opts.postselect[in.b / 64] >> (in.b % 64)) & 1u)))) {
      in.op = OP_POSTSELECT;
      P.npost++;
    }
  if (P.npost) {
    P.split_ok = false;
    P.fcode.clear();
    P.vcode.clear();
  }
  if (P.consts.empty()) P.consts = {1.0, 0.0, 1.0, 0.0};
  if (P.refs.empty()) P.refs.push_back(0);
  if (P.ev_rec.empty()) P.ev_rec.push_back(-1);
  if (P.site_type.empty()) { P.site_type.push_back(0); P.site_img.push_back(0); P.site_sign.push_back(0); }
  if (P.surv.empty()) P.surv.assign(kChunk + 1, 0.0);
  return 0;
}

}  // namespace clifft
