// Generator and run-time compiler of the program-specialized bit-sliced
// kernels (see specialize.h).  The generated body follows the compiled
// stream instruction by instruction with the same semantics as the
// interpreter k_frames:
//   fans (Lemma 1, App. A)      rows of the targets ^= the pivot word, pivot
//                                ^= parity of the other rows, in both frames;
//   deterministic measurement   m = sign ^ parity of the full frame's x rows
//   (App. B.2)                   over the measured Z-string, pn the same over
//                                the noise frame;
//   dormant random measurement  m = Philox bit ^ pn, then H absorbed and the
//                                correction X^b;
//   reset correction (App. B.3) X^m on the full frame, X^pn on the noise frame;
//   noise block (Section 3.2)   the lane's faults at sites of the block;
//   detector / observable       accumulator rows fed by their records.
#include "specialize.h"

#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <sstream>

namespace clifft {
namespace {

// philox.h, spec_args.h and spec_prelude.h, concatenated by the build
const char kPrelude[] =
#include "spec_prelude.inc"
    ;

constexpr int kSpecMaxRegs = 200;      // frame, accumulator and random-bit rows held in registers
constexpr size_t kSpecMaxCode = 600;  // instructions (run-time compilation grows faster than linearly)
constexpr unsigned kSpecListCap = 24;  // must equal kListCap of the prelude

struct Gen {
  const CompiledProgram& P;
  int N, W;
  std::ostringstream o;

  explicit Gen(const CompiledProgram& p) : P(p), N(p.nq), W(p.W) {}

  static std::string f(int row) { return "f[" + std::to_string(row) + "]"; }

  std::vector<int> bits(uint32_t off, int words) const {
    std::vector<int> q;
    for (int w = 0; w < words; w++)
      for (uint64_t m = P.masks[off + w]; m; m &= m - 1) q.push_back(w * 64 + __builtin_ctzll(m));
    return q;
  }

  // XOR of rows base + q over the qubits q of a mask ("0u" when empty)
  std::string parity(const std::vector<int>& qs, int base) const {
    if (qs.empty()) return "0u";
    std::string s;
    for (size_t i = 0; i < qs.size(); i++) s += (i ? " ^ " : "") + f(base + qs[i]);
    return s;
  }

  // The Pauli of outcome o (variable `o`) at site s, on the shot bit `bit`,
  // XORed into both frames.
  void site_body(int s) {
    const int t = P.site_type[s];
    const uint32_t img = P.site_img[s];
    const int ncomp = t == S_DEP2 ? 2 : 1;
    o << "        {";
    if (t == S_DEP1)
      o << " const unsigned int x0 = o < 2u ? bit : 0u, z0 = o >= 1u ? bit : 0u;";
    else if (t == S_DEP2)
      o << " const unsigned int la = (o + 1u) >> 2, lb = (o + 1u) & 3u;"
        << " const unsigned int x0 = (la - 1u) < 2u ? bit : 0u, z0 = la >= 2u ? bit : 0u;"
        << " const unsigned int x1 = (lb - 1u) < 2u ? bit : 0u, z1 = lb >= 2u ? bit : 0u;";
    else if (t == S_XERR)
      o << " const unsigned int x0 = bit, z0 = 0u;";
    else if (t == S_YERR)
      o << " const unsigned int x0 = bit, z0 = bit;";
    else
      o << " const unsigned int x0 = 0u, z0 = bit;";
    std::vector<std::string> tx(N), tz(N);
    auto add = [](std::string& a, const std::string& v) { a += (a.empty() ? "" : " ^ ") + v; };
    for (int c = 0; c < ncomp; c++) {
      const uint32_t ix = img + (uint32_t)(c * 4 * W), iz = ix + (uint32_t)(2 * W);
      const std::string xs = "x" + std::to_string(c), zs = "z" + std::to_string(c);
      for (int q : bits(ix, W)) add(tx[q], xs);
      for (int q : bits(iz, W)) add(tx[q], zs);
      for (int q : bits(ix + W, W)) add(tz[q], xs);
      for (int q : bits(iz + W, W)) add(tz[q], zs);
    }
    for (int q = 0; q < N; q++) {
      if (!tx[q].empty())
        o << " { const unsigned int t = " << tx[q] << "; " << f(q) << " ^= t; " << f(2 * N + q) << " ^= t; }";
      if (!tz[q].empty())
        o << " { const unsigned int t = " << tz[q] << "; " << f(N + q) << " ^= t; " << f(3 * N + q) << " ^= t; }";
    }
    o << " }\n";
  }

  // Faults of sites [lo, hi).  Each lane's next unapplied fault is kept in
  // `e` (its key, 0xFFFFFFFF when none).  The block sweeps its sites in
  // order; a lane applies its entry for a site when the sweep reaches it
  // (keys are ascending, so sites come in order).  The sweep repeats while a
  // lane still holds an entry of the block (a second fault at a site
  // already passed) or ran out of list while more faults remain (it then
  // rebuilds the list above its last applied key).
  void noise(uint32_t lo, uint32_t hi, uint32_t nsites, uint32_t nchunks) {
    o << "    // noise sites [" << lo << ", " << hi << ")\n"
      << "    for (;;) {\n";
    for (uint32_t s = lo; s < hi; s++) {
      o << "      if ((e >> 9) == " << s << "u) {\n"
        << "        const unsigned int bit = 1u << ((e >> 4) & 31u), o = e & 15u;\n";
      site_body((int)s);
      o << "        last = e; lhead++;\n"
        << "        e = lhead < lim ? L[lhead * 64 + lane] : 0xFFFFFFFFu;\n"
        << "      }\n";
    }
    // another sweep for a second fault of the lane at a site already passed
    // (two of its shots at one site) or after a refill
    o << "      const bool rf = lhead == lim && more;\n"
      << "      if (__ballot(rf || (e >> 9) < " << hi << "u) == 0) break;\n"
      << "      if (rf) {\n"
      << "        const unsigned int n = build_list(A, sl, SEND, " << nsites << "u, " << nchunks
      << "u, s0, L, lane, cap, last + 1);\n"
      << "        lim = n < cap ? n : cap; more = n > cap; lhead = 0; e = L[lane];\n"
      << "      }\n"
      << "    }\n";
  }

  void record(const GInstr& in) {
    const int r = P.ev_rec[in.b];
    if (r < 0) return;
    o << "      if (A.meas32 && st) A.meas32[" << r << "ull * 2 * A.words64 + col] = m & valid;\n";
    for (uint32_t t = P.rec_tgt_off[r]; t < P.rec_tgt_off[r + 1]; t++)
      o << "      a[" << P.rec_tgt[t] << "] ^= m;\n";
  }

  std::string source() {
    const uint32_t nsites = (uint32_t)P.site_p.size();
    const bool surv_lds = P.nchunks == 1 && nsites < 2048;
    const int nacc = P.ndet_rows + P.nobs;
    o << kPrelude;
    o << "\nextern \"C\" __global__ __launch_bounds__(64) void " << kSpecEntry << "(clifft_spec::SpecArgs A) {\n"
      << "  using namespace clifft_spec;\n"
      << "  __shared__ unsigned int L[" << kSpecListCap * 64 << "];\n";
    if (surv_lds) o << "  __shared__ double SL[" << nsites + 1 << "];\n";
    o << "  const int lane = threadIdx.x;\n";
    // survival product at the end of the only chunk, as an exact literal
    if (P.nchunks == 1 && nsites > 0) {
      char lit[64];
      snprintf(lit, sizeof lit, "%a", P.surv[nsites]);
      o << "  const double SEND = " << lit << ";\n";
    } else {
      o << "  const double SEND = -1.0;\n";
    }
    if (surv_lds)
      o << "  for (unsigned int i = lane; i <= " << nsites << "u; i += 64) SL[i] = A.surv[i];\n"
        << "  __syncthreads();\n"
        << "  const double* sl = SL;\n";
    else
      o << "  const double* sl = nullptr;\n";
    o << "  const unsigned long long tiles = (A.shots + 2047) / 2048;\n"
      << "  const unsigned int cap = A.list_cap < 1 ? 1u : A.list_cap < kListCap ? A.list_cap : kListCap;\n"
      << "  for (unsigned long long tile = blockIdx.x; tile < tiles; tile += gridDim.x) {\n"
      << "    const unsigned long long s0 = tile * 2048 + (unsigned long long)lane * 32;\n"
      << "    const unsigned int valid = s0 >= A.shots ? 0u : (A.shots - s0 >= 32 ? ~0u : ((1u << (A.shots - s0)) - "
         "1u));\n"
      << "    const unsigned long long col = s0 >> 5;\n"
      << "    const bool st = col < 2 * A.words64;\n";
    if (nsites)
      o << "    const unsigned int n0 = build_list(A, sl, SEND, " << nsites << "u, " << P.nchunks
        << "u, s0, L, lane, cap, 0u);\n";
    else
      o << "    const unsigned int n0 = 0;\n";
    o << "    unsigned int lim = n0 < cap ? n0 : cap, lhead = 0, last = 0;\n"
      << "    bool more = n0 > cap;\n"
      << "    unsigned int e = lim ? L[lane] : 0xFFFFFFFFu;\n"
      << "    (void)lim; (void)lhead; (void)last; (void)more; (void)e;\n"
      << "    unsigned int f[" << 4 * N << "];\n"
      << "#pragma unroll\n"
      << "    for (int i = 0; i < " << 4 * N << "; i++) f[i] = 0;\n"
      << "    unsigned int a[" << std::max(nacc, 1) << "];\n"
      << "#pragma unroll\n"
      << "    for (int i = 0; i < " << std::max(nacc, 1) << "; i++) a[i] = 0;\n"
      << "    unsigned int r[" << std::max(P.rblk_max, 1) << "];\n"
      << "    unsigned int lm = 0, lp = 0;\n"
      << "    (void)lm; (void)lp; (void)r;\n";
    uint32_t rblk = 0xFFFFFFFFu;
    for (const GInstr& in : P.code) {
      const int v = in.v;
      switch (in.op) {
        case OP_FANCX:
        case OP_FANCZ:
        case OP_FAN2: {
          const std::vector<int> qs = bits(in.a, W);
          for (int c = 0; c < 4 * N; c += 2 * N) {
            const int X = c, Z = c + N;
            o << "    {\n";
            if (in.op == OP_FANCX) {
              o << "      const unsigned int s = " << f(X + v) << ";\n";
              for (int q : qs) o << "      " << f(X + q) << " ^= s;\n";
              o << "      " << f(Z + v) << " ^= " << parity(qs, Z) << ";\n";
            } else if (in.op == OP_FANCZ) {
              o << "      const unsigned int s = " << f(X + v) << ";\n";
              for (int q : qs) o << "      " << f(Z + q) << " ^= s;\n";
              o << "      " << f(Z + v) << " ^= " << parity(qs, X) << ";\n";
            } else {
              o << "      const unsigned int s = " << f(Z + v) << ";\n";
              for (int q : qs) o << "      " << f(Z + q) << " ^= s;\n";
              o << "      " << f(X + v) << " ^= " << parity(qs, X) << ";\n";
            }
            o << "    }\n";
          }
          break;
        }
        case OP_FS:
          o << "    " << f(N + v) << " ^= " << f(v) << "; " << f(3 * N + v) << " ^= " << f(2 * N + v) << ";\n";
          break;
        case OP_FH:
          o << "    { unsigned int t = " << f(v) << "; " << f(v) << " = " << f(N + v) << "; " << f(N + v)
            << " = t; t = " << f(2 * N + v) << "; " << f(2 * N + v) << " = " << f(3 * N + v) << "; "
            << f(3 * N + v) << " = t; }\n";
          break;
        case OP_MSTATIC: {
          const std::vector<int> qs = bits(in.a, W);
          o << "    {\n"
            << "      const unsigned int m = " << ((in.flags & F_SIGN) ? "~0u" : "0u") << " ^ " << parity(qs, 0)
            << ";\n"
            << "      const unsigned int p = " << parity(qs, 2 * N) << ";\n";
          record(in);
          o << "      lm = m; lp = p;\n"
            << "    }\n";
          break;
        }
        case OP_MRANDOM: {
          const uint32_t blk = in.b >> 7;
          if (blk != rblk) {
            const uint32_t o0 = P.rblk_off[blk], o1 = P.rblk_off[blk + 1];
            o << "    // dormant random outcomes of event block " << blk << "\n";
            for (uint32_t k = o0; k < o1; k++) o << "    r[" << k - o0 << "] = 0;\n";
            o << "    for (unsigned int s = 0; s < kShotsPerLane; s++) {\n"
              << "      const U4 w = draw(" << blk << "u, kPurposeRbit, A.offset + s0 + s, A.seed);\n";
            for (uint32_t k = o0; k < o1; k++) {
              const int e = P.rblk_ev[k];
              o << "      r[" << k - o0 << "] |= ((w.w" << (e >> 5) << " >> " << (e & 31) << ") & 1u) << s;\n";
            }
            o << "    }\n";
            rblk = blk;
          }
          o << "    {\n"
            << "      const unsigned int x = " << f(v) << ", z = " << f(N + v) << ", nx = " << f(2 * N + v)
            << ", nz = " << f(3 * N + v) << ";\n"
            << "      const unsigned int m = r[" << in.u << "] ^ nz;\n"
            << "      const unsigned int b = m ^ z" << ((in.flags & F_SIGN) ? " ^ ~0u" : "") << ";\n"
            << "      " << f(v) << " = z ^ b; " << f(N + v) << " = x; " << f(2 * N + v) << " = nz; "
            << f(3 * N + v) << " = nx;\n";
          record(in);
          o << "      lm = m; lp = nz;\n"
            << "    }\n";
          break;
        }
        case OP_CPAULI: {
          o << "    {\n";
          for (int q : bits(in.a, W)) o << "      " << f(q) << " ^= lm; " << f(2 * N + q) << " ^= lp;\n";
          for (int q : bits(in.a + W, W)) o << "      " << f(N + q) << " ^= lm; " << f(3 * N + q) << " ^= lp;\n";
          o << "    }\n";
          break;
        }
        case OP_NOISE:
          noise(in.a, in.b, nsites, (uint32_t)P.nchunks);
          break;
        case OP_DET:
          o << "    if (A.det32 && st) A.det32[" << in.b << "ull * 2 * A.words64 + col] = a[" << in.s
            << "] & valid;\n"
            << "    a[" << in.s << "] = 0;\n";
          break;
        default:  // OP_OBS (accumulated from its records), OP_END
          break;
      }
    }
    for (int ob = 0; ob < P.nobs; ob++)
      o << "    if (A.obs32 && st) A.obs32[" << ob << "ull * 2 * A.words64 + col] = a[" << P.ndet_rows + ob
        << "] & valid;\n";
    o << "  }\n}\n";
    return o.str();
  }
};

}  // namespace

bool spec_supported(const CompiledProgram& P, std::string* why) {
  auto no = [&](const char* m) {
    if (why) *why = m;
    return false;
  };
  if (P.kmax != 0) return no("specialized kernels need k_max = 0");
  if (P.has_cfeed) return no("feed-forward Paulis need per-shot record bits");
  if (P.nprobes) return no("expectation-value probes need the interpreter");
  if (P.npost) return no("post-selection ends shots early: interpreter tiers only");
  if (4 * P.nq + P.ndet_rows + P.nobs + P.rblk_max > kSpecMaxRegs) return no("too many frame and accumulator rows");
  if (P.code.size() > kSpecMaxCode) return no("program too long to specialize");
  double f = 0;
  for (double q : P.site_p) f += q;
  if (P.site_p.size() >= (1u << 23) || f * 32 > kSpecListCap / 4) return no("noise too dense for the fault list");
  for (const GInstr& in : P.code)
    if ((in.op >= OP_APERM && in.op <= OP_AROT) || in.op == OP_MACTZ || in.op == OP_MACTX)
      return no("active-vector instruction");
  return true;
}

std::string spec_source(const CompiledProgram& P) {
  Gen g(P);
  return g.source();
}

bool spec_compile(const std::string& src, std::vector<char>* code, std::string* log) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "clifft_frames_spec.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    *log = "hiprtcCreateProgram failed";
    return false;
  }
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-ffp-contract=off", "-std=c++17",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  size_t n = 0;
  if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
    log->assign(n, '\0');
    hiprtcGetProgramLog(prog, &(*log)[0]);
  }
  bool ok = r == HIPRTC_SUCCESS;
  if (ok) {
    size_t cs = 0;
    ok = hiprtcGetCodeSize(prog, &cs) == HIPRTC_SUCCESS && cs > 0;
    if (ok) {
      code->assign(cs, 0);
      ok = hiprtcGetCode(prog, code->data()) == HIPRTC_SUCCESS;
    }
  }
  hiprtcDestroyProgram(&prog);
  return ok;
}

}  // namespace clifft
