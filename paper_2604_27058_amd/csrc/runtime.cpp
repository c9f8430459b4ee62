// C-ABI implementation: program handles, device upload, launch-shape
// selection and the sampling entry points declared in include/clifft.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/clifft.h"
#include "compiler.h"
#include "kernels.h"
#include "spec_args.h"
#include "specialize.h"
#include "probe.h"

using namespace clifft;

namespace {

thread_local std::string g_err;

clifft_status fail(clifft_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

struct DeviceCopy {
  DevProgram view{};
  // split form: the frame-only view (bit-sliced kernel), the vector-only view,
  // and the fix-up tables (output rows with a dependency, their entries)
  bool has_split = false;
  DevProgram fview{}, vview{};
  const uint32_t* xrows = nullptr;
  uint32_t nxrows = 0;
  const uint32_t* xdep_off = nullptr;
  const uint32_t* xdep = nullptr;
  std::vector<void*> allocs;
  // stratified sampling tables (DevProgram::strat), uploaded by the first
  // stratified call and grown when a call needs more rows
  const double* strat = nullptr;
  int strat_rows = 0;
  hipModule_t spec_mod = nullptr;  // specialized kernel, loaded at its first launch
  hipFunction_t spec_fn = nullptr;
};

}  // namespace

struct clifft_program {
  CompiledProgram host;
  std::mutex mu;
  std::map<int, DeviceCopy> dev;
  std::map<std::pair<int, int>, clifft_launch> tuned;  // (device, precision) -> autotuned launch
  int spec_state = 0;          // specialized kernel: 0 not built, 1 code object ready, -1 unavailable
  std::vector<char> spec_code;  // gfx950 code object
  std::string spec_log;         // reason or compiler log when unavailable
};

namespace {

template <typename T>
hipError_t upload_vec(const std::vector<T>& v, const T** dst, std::vector<void*>& allocs) {
  void* d = nullptr;
  size_t bytes = v.size() * sizeof(T);
  hipError_t e = hipMalloc(&d, bytes ? bytes : 16);
  if (e != hipSuccess) return e;
  allocs.push_back(d);
  if (bytes) {
    e = hipMemcpy(d, v.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
  }
  *dst = (const T*)d;
  return hipSuccess;
}

clifft_status ensure_device(const clifft_program* cp, const DevProgram** out, const DeviceCopy** copy = nullptr) {
  clifft_program* p = const_cast<clifft_program*>(cp);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CLIFFT_E_DEVICE, "no HIP device");
  std::lock_guard<std::mutex> lock(p->mu);
  auto it = p->dev.find(dev);
  if (it != p->dev.end()) {
    *out = &it->second.view;
    if (copy) *copy = &it->second;
    return CLIFFT_OK;
  }
  DeviceCopy dc;
  const CompiledProgram& H = p->host;
  DevProgram& v = dc.view;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload_vec(H.code, &v.code, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.masks, &v.masks, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.consts, &v.consts, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.refs, &v.refs, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.ev_rec, &v.ev_rec, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.site_type, &v.site_type, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.site_img, &v.site_img, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.site_sign, &v.site_sign, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.surv, &v.surv, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.rec_tgt_off, &v.rec_tgt_off, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.rec_tgt, &v.rec_tgt, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.rblk_off, &v.rblk_off, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.rblk_ev, &v.rblk_ev, dc.allocs);
  if (e == hipSuccess) e = upload_vec(H.pline, &v.pline, dc.allocs);
  if (e != hipSuccess) {
    for (void* a : dc.allocs) (void)hipFree(a);
    return fail(CLIFFT_E_DEVICE, std::string("program upload failed: ") + hipGetErrorString(e));
  }
  v.nq = H.nq;
  v.W = H.W;
  v.kmax = H.kmax;
  v.ncode = (int)H.code.size();
  v.nevents = H.nevents;
  v.nrec = H.nrec;
  v.ndet = H.ndet;
  v.nobs = H.nobs;
  v.nprobes = H.nprobes;
  v.nsites = (int)H.site_p.size();
  v.nchunks = H.nchunks;
  v.rblk_max = H.rblk_max;
  v.ndet_rows = H.ndet_rows;
  v.has_post = H.npost > 0;
  v.has_pairs[0] = cost_model(H, false).pair_starts > 0;
  v.has_pairs[1] = cost_model(H, true).pair_starts > 0;
  {
    double f = 0;
    for (double q : H.site_p) f += q;
    v.exp_faults = (float)f;
  }
  if (H.split_ok) {
    DevProgram f = v, g = v;
    std::vector<uint32_t> xrows;
    for (size_t i = 0; i + 1 < H.xdep_off.size(); i++)
      if (H.xdep_off[i + 1] > H.xdep_off[i]) xrows.push_back((uint32_t)i);
    if (xrows.empty()) xrows.push_back(0);
    if (e == hipSuccess) e = upload_vec(H.fcode, &f.code, dc.allocs);
    if (e == hipSuccess) e = upload_vec(H.vcode, &g.code, dc.allocs);
    if (e == hipSuccess) e = upload_vec(H.vdep, &g.vdep, dc.allocs);
    if (e == hipSuccess) e = upload_vec(H.vev_rec, &g.ev_rec, dc.allocs);
    if (e == hipSuccess) e = upload_vec(xrows, &dc.xrows, dc.allocs);
    if (e == hipSuccess) e = upload_vec(H.xdep_off, &dc.xdep_off, dc.allocs);
    if (e == hipSuccess) e = upload_vec(H.xdep, &dc.xdep, dc.allocs);
    if (e != hipSuccess) {
      for (void* a : dc.allocs) (void)hipFree(a);
      return fail(CLIFFT_E_DEVICE, std::string("program upload failed: ") + hipGetErrorString(e));
    }
    f.ncode = (int)H.fcode.size();
    f.kmax = 0;
    g.ncode = (int)H.vcode.size();
    g.W = 1;
    g.nrec = H.nactive;
    g.ndet = g.nobs = 0;
    g.nsites = g.nchunks = 0;
    g.rblk_max = 0;
    g.ndet_rows = 0;
    g.exp_faults = 0;
    g.nbits = H.nbits;
    g.dep_words = H.dep_words;
    dc.fview = f;
    dc.vview = g;
    dc.nxrows = H.xdep_off.back() > 0 ? (uint32_t)(xrows.size()) : 0u;
    dc.has_split = true;
  }
  auto res = p->dev.emplace(dev, std::move(dc));
  *out = &res.first->second.view;
  if (copy) *copy = &res.first->second;
  return CLIFFT_OK;
}

// Builds the specialized kernel's code object once (host only).
clifft_status ensure_spec(clifft_program* p) {
  std::lock_guard<std::mutex> lock(p->mu);
  if (p->spec_state == 1) return CLIFFT_OK;
  if (p->spec_state == -1) return fail(CLIFFT_E_UNSUPPORTED, p->spec_log);
  std::string why;
  if (!spec_supported(p->host, &why)) {
    p->spec_state = -1;
    p->spec_log = why;
    return fail(CLIFFT_E_UNSUPPORTED, why);
  }
  std::string log;
  if (!spec_compile(spec_source(p->host), &p->spec_code, &log)) {
    p->spec_state = -1;
    p->spec_log = "run-time compilation failed: " + log;
    return fail(CLIFFT_E_DEVICE, p->spec_log);
  }
  p->spec_state = 1;
  return CLIFFT_OK;
}

// The specialized kernel's function on the current device (module loaded on
// first use).
clifft_status spec_function(clifft_program* p, hipFunction_t* fn) {
  clifft_status st = ensure_spec(p);
  if (st != CLIFFT_OK) return st;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CLIFFT_E_DEVICE, "no HIP device");
  std::lock_guard<std::mutex> lock(p->mu);
  auto it = p->dev.find(dev);
  if (it == p->dev.end()) return fail(CLIFFT_E_DEVICE, "program not on this device");
  DeviceCopy& dc = it->second;
  if (!dc.spec_fn) {
    hipError_t e = hipModuleLoadData(&dc.spec_mod, p->spec_code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&dc.spec_fn, dc.spec_mod, kSpecEntry);
    if (e != hipSuccess) {
      if (dc.spec_mod) (void)hipModuleUnload(dc.spec_mod);
      dc.spec_mod = nullptr;
      dc.spec_fn = nullptr;
      return fail(CLIFFT_E_DEVICE, std::string("loading the specialized kernel failed: ") + hipGetErrorString(e));
    }
  }
  *fn = dc.spec_fn;
  return CLIFFT_OK;
}

hipError_t launch_spec(hipFunction_t fn, const DevProgram& D, const KArgs& A, int grid, hipStream_t s) {
  clifft_spec::SpecArgs S{};
  S.shots = A.shots;
  S.seed = A.seed;
  S.offset = A.offset;
  S.words64 = (A.shots + 63) / 64;
  S.meas32 = (unsigned int*)A.meas;
  S.det32 = (unsigned int*)A.det;
  S.obs32 = (unsigned int*)A.obs;
  S.surv = D.surv;
  S.site_type = D.site_type;
  S.list_cap = A.list_cap;
  void* args[] = {&S};
  return hipModuleLaunchKernel(fn, grid, 1, 1, 64, 1, 1, 0, s, args, nullptr);
}

constexpr size_t kLdsLimit = 160 * 1024;
constexpr int kLaneMaxK = 12;                              // shot-per-lane tier up to this k_max
constexpr int kBatchLaneMaxK = 10;                         // the same inside a batched launch
constexpr int kWaveMaxK = 15;                              // shot-per-wave tier up to this k_max
constexpr int kBitSliced = -32;                            // 32 shots per lane, bit-sliced frames
constexpr size_t kWorkspaceBudget = (size_t)4 << 30;       // default global vector workspace

int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

// Launch shape: the tier follows the active-vector size (threads per shot
// and storage), the grid fills the device with persistent workgroups.
clifft_status choose_shape(const CompiledProgram& H, const DevProgram* D, const clifft_launch* cfg, uint64_t shots,
                           LaunchShape* L, bool* fp64,
                           const std::map<std::pair<int, int>, clifft_launch>* tuned = nullptr, bool trace = false,
                           int strat_r = -1) {
  const bool strat = strat_r >= 0;
  clifft_launch c{};
  if (cfg) c = *cfg;
  if (c.precision != CLIFFT_FP32 && c.precision != CLIFFT_FP64) return fail(CLIFFT_E_INVALID_ARG, "bad precision");
  *fp64 = c.precision == CLIFFT_FP64;
  if (tuned && c.threads_per_shot == 0 && c.grid == 0 && c.vector_in_hbm == 0 && c.specialize == 0 && c.split == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto it = tuned->find({dev, c.precision});
    // a stratum with faults runs faster shot per lane than bit-sliced (whose
    // per-shot fault cursors serialise on dependent LDS reads)
    if (it != tuned->end() && !(trace && (it->second.threads_per_shot == kBitSliced || it->second.split >= 1)) &&
        !(strat && (it->second.split >= 1 || it->second.specialize == 1 ||
                    (strat_r > 0 && it->second.threads_per_shot == kBitSliced))))
      c = it->second;
  }
  if (strat && (c.split >= 1 || c.specialize == 1))
    return fail(CLIFFT_E_INVALID_ARG, "stratified sampling runs on the interpreter tiers (no split form, no specialized kernel)");
  const size_t amp = *fp64 ? 16 : 8;
  const size_t vec = (size_t)1 << H.kmax;
  if (c.split < -1 || c.split > 3) return fail(CLIFFT_E_INVALID_ARG, "split must be -1, 0, 1, 2 or 3");
  if (c.split >= 1) {
    if (trace) return fail(CLIFFT_E_INVALID_ARG, "the split form has no trace mode");
    if (!H.split_ok)
      return fail(CLIFFT_E_UNSUPPORTED, "the split form needs an active vector and at most 256 active measurements");
    if (c.specialize == 1) return fail(CLIFFT_E_INVALID_ARG, "specialize applies to the bit-sliced tier only");
    // frame pass: the bit-sliced kernel over the frame-only stream
    DevProgram tmp{};
    tmp.nq = H.nq;
    tmp.ndet = H.ndet;
    tmp.nobs = H.nobs;
    tmp.rblk_max = H.rblk_max;
    tmp.ndet_rows = H.ndet_rows;
    tmp.nsites = (int)H.site_p.size();
    tmp.nchunks = H.nchunks;
    {
      double f = 0;
      for (double q : H.site_p) f += q;
      tmp.exp_faults = (float)f;
    }
    const size_t rows_bytes = frames_lds_rows(tmp) * 64 * 4;
    // frame pass: bit-sliced (2), shot per lane with frames in VGPRs (3), or
    // (1) bit-sliced when its rows fit in LDS and its 2048-shot tiles fill
    // the device twice over
    const bool fits = rows_bytes <= kLdsLimit && !H.has_cfeed;  // feed-forward needs per-shot record bits
    if (c.split == 2 && !fits)
      return fail(CLIFFT_E_CAPACITY, "the bit-sliced frame pass needs LDS rows and no feed-forward Paulis");
    const bool flane = c.split == 3 || !fits || (c.split == 1 && (shots + 2047) / 2048 < 2 * (uint64_t)device_cus());
    int fgrid;
    if (!flane) {
      const uint64_t tiles = (shots + 2047) / 2048;
      fgrid = device_cus() * (int)std::max<size_t>(1, std::min<size_t>(16, kLdsLimit / rows_bytes));
      if ((uint64_t)fgrid > tiles) fgrid = (int)std::max<uint64_t>(1, tiles);
    } else {
      const uint64_t blocks = ((shots + 63) / 64 + 3) / 4;
      fgrid = device_cus() * 8;
      if ((uint64_t)fgrid > blocks) fgrid = (int)std::max<uint64_t>(1, blocks);
    }
    // vector pass: the vector-only stream, no frames
    int G = c.threads_per_shot;
    if (G == 0) G = H.kmax <= 6 ? 1 : H.kmax <= 13 ? 64 : 256;
    if (G != 1 && G != 64 && G != 256) return fail(CLIFFT_E_INVALID_ARG, "the split form's threads_per_shot is 1, 64 or 256");
    const size_t need = (G == 256 ? 1 : 4) * vec * amp * (G == 1 ? 64 : 1);
    bool global_vec = c.vector_in_hbm == 1 ||
                      (c.vector_in_hbm == 0 && need > (G == 256 ? (size_t)32 * 1024 : kLdsLimit - 16 * 1024));
    DevProgram tv{};
    tv.nrec = H.nactive;
    tv.kmax = H.kmax;
    const size_t lds = lds_bytes_for(tv, G, global_vec, *fp64);
    if (lds > kLdsLimit) return fail(CLIFFT_E_CAPACITY, "active vectors exceed LDS; use the HBM workspace");
    const uint64_t blocks_needed = G == 256 ? shots : G == 64 ? (shots + 3) / 4 : ((shots + 63) / 64 + 3) / 4;
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, kLdsLimit / std::max<size_t>(lds, 1)));
    int grid = c.grid > 0 ? c.grid : device_cus() * per_cu;
    if (global_vec && c.grid <= 0) {
      const size_t per_block = 2 * (size_t)(G == 256 ? 1 : 4) * vec * amp * (G == 1 ? 64 : 1);
      const size_t cap = std::max<size_t>(1, kWorkspaceBudget / per_block);
      if ((size_t)grid > cap) grid = (int)cap;
    }
    if ((uint64_t)grid > blocks_needed) grid = (int)std::max<uint64_t>(1, blocks_needed);
    L->G = G;
    L->grid = grid;
    L->lds_bytes = lds;
    L->global_vec = global_vec;
    L->spec = false;
    L->split = true;
    L->fgrid = fgrid;
    L->flane = flane;
    L->G = G;
    return CLIFFT_OK;
  }
  L->split = false;
  L->fgrid = 0;
  L->flane = false;
  int G = c.threads_per_shot;
  if (G != 0 && G != 1 && G != 64 && G != 256 && G != kBitSliced)
    return fail(CLIFFT_E_INVALID_ARG, "threads_per_shot must be 0, 1, 64, 256 or -32");
  {
    // bit-sliced Pauli frames: k_max = 0 programs whose rows fit in LDS
    DevProgram tmp{};
    tmp.nq = H.nq;
    tmp.ndet = H.ndet;
    tmp.nobs = H.nobs;
    tmp.rblk_max = H.rblk_max;
    tmp.ndet_rows = H.ndet_rows;
    tmp.nsites = (int)H.site_p.size();
    tmp.nchunks = H.nchunks;
    {
      double f = 0;
      for (double q : H.site_p) f += q;
      tmp.exp_faults = (float)f;
    }
    const size_t rows_bytes = frames_lds_rows(tmp, strat_r) * 64 * 4;
    const bool spec = c.specialize == 1;
    const bool bs_ok = H.kmax == 0 && !trace && !H.has_cfeed && H.nprobes == 0 && (spec || rows_bytes <= kLdsLimit);
    if (c.specialize == 1 && G != 0 && G != kBitSliced)
      return fail(CLIFFT_E_INVALID_ARG, "specialize applies to the bit-sliced tier only");
    if ((G == kBitSliced || spec) && !bs_ok)
      return fail(CLIFFT_E_CAPACITY, "bit-sliced frames need k_max = 0 and rows in LDS (not in trace mode)");
    if (spec && !spec_supported(H, nullptr)) {
      std::string why;
      spec_supported(H, &why);
      return fail(CLIFFT_E_UNSUPPORTED, why);
    }
    if (G == 0 && bs_ok && strat_r <= 0) G = kBitSliced;
    if (G == kBitSliced) {
      const uint64_t tiles = (shots + 2047) / 2048;
      // the specialized kernel keeps its rows in registers (about 8 waves per
      // CU fit); the interpreter is bounded by LDS
      int per_cu = spec ? 8 : (int)std::max<size_t>(1, std::min<size_t>(16, kLdsLimit / rows_bytes));
      int grid = c.grid > 0 ? c.grid : device_cus() * per_cu;
      if ((uint64_t)grid > tiles) grid = (int)std::max<uint64_t>(1, tiles);
      L->G = kBitSliced;
      L->grid = grid;
      L->lds_bytes = spec ? 0 : rows_bytes;
      L->global_vec = false;
      L->spec = spec;
      return CLIFFT_OK;
    }
  }
  // Tiers: frames shot-per-lane whenever the vectors of 64 shots fit the
  // global budget (k <= 12), else one shot per workgroup.  Shot-per-lane
  // vectors go to LDS when they fit.  A shot-per-workgroup vector stays in
  // LDS only while four workgroups per CU fit (32 KB); beyond that the HBM
  // workspace serves it faster, with more workgroups streaming per CU.
  if (G == 0) G = H.kmax <= kLaneMaxK ? 1 : H.kmax <= kWaveMaxK ? 64 : 256;
  bool global_vec = false;
  if (H.kmax > 0) {
    size_t need = (G == 256 ? 1 : 4) * vec * amp * (G == 1 ? 64 : 1);
    if (c.vector_in_hbm == 1) global_vec = true;
    else if (c.vector_in_hbm == -1) global_vec = false;
    else global_vec = need > (G == 256 ? (size_t)32 * 1024 : kLdsLimit - 16 * 1024);
  }
  DevProgram tmp{};
  tmp.nrec = H.nrec;
  tmp.ndet = H.ndet;
  tmp.nobs = H.nobs;
  tmp.kmax = H.kmax;
  size_t lds = lds_bytes_for(D ? *D : tmp, G, global_vec, *fp64);
  if (lds > kLdsLimit) return fail(CLIFFT_E_CAPACITY, "records and active vectors exceed LDS; use a larger tier");
  // work items: 64-shot tiles per wave (G = 1), single shots per wave (G = 64)
  // or per workgroup (G = 256)
  uint64_t blocks_needed = G == 256 ? shots : G == 64 ? (shots + 3) / 4 : ((shots + 63) / 64 + 3) / 4;
  int per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, kLdsLimit / std::max<size_t>(lds, 1)));
  int grid = c.grid > 0 ? c.grid : device_cus() * per_cu;
  if (global_vec && c.grid <= 0) {
    // keep the default workspace within budget
    size_t per_block = 2 * (size_t)(G == 256 ? 1 : 4) * vec * amp * (G == 1 ? 64 : 1);
    size_t cap = std::max<size_t>(1, kWorkspaceBudget / per_block);
    if ((size_t)grid > cap) grid = (int)cap;
  }
  if ((uint64_t)grid > blocks_needed) grid = (int)std::max<uint64_t>(1, blocks_needed);
  L->G = G;
  L->grid = grid;
  L->lds_bytes = lds;
  L->global_vec = global_vec;
  return CLIFFT_OK;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Split form: needed-bit rows, then active-outcome rows (bit-packed).
size_t split_rows_bytes(const CompiledProgram& H, uint64_t shots) {
  const size_t words = (shots + 63) / 64;
  return align256((size_t)H.nbits * words * 8) + align256((size_t)H.nactive * words * 8);
}

// Workspace layout: [split rows][active vectors in HBM]
size_t workspace_bytes(const CompiledProgram& H, const LaunchShape& L, bool fp64, uint64_t shots) {
  size_t bytes = L.split ? split_rows_bytes(H, shots) : 0;
  if (!L.global_vec) return bytes;
  size_t amp = fp64 ? 16 : 8;
  size_t units = (size_t)L.grid * (L.G == 256 ? 1 : 4);
  // two buffers per unit: active measurements collapse from one into the other
  return bytes + 2 * units * ((size_t)1 << H.kmax) * amp * (L.G == 1 ? 64 : 1);
}

// One sampling launch sequence on `s`: the whole-program kernel, or the
// split form's frame pass, vector pass and record fix-up.
hipError_t launch_plan(const CompiledProgram& H, const DeviceCopy& dc, const LaunchShape& L, const KArgs& A,
                       bool fp64, bool trace, hipStream_t s, const DevProgram* view = nullptr) {
  if (!L.split) return launch_sample(view ? *view : dc.view, A, L, fp64, trace, s);
  const uint64_t words = (A.shots + 63) / 64;
  unsigned char* ws = (unsigned char*)A.workspace;
  uint64_t* bits = (uint64_t*)ws;
  uint64_t* mrows = (uint64_t*)(ws + align256((size_t)H.nbits * words * 8));
  void* vws = ws + split_rows_bytes(H, A.shots);
  KArgs AF = A;
  AF.nbits = bits;
  AF.workspace = nullptr;
  hipError_t e;
  if (L.flane) {
    LaunchShape LF{};
    LF.G = 1;
    LF.grid = L.fgrid;
    LF.lds_bytes = lds_bytes_for(dc.fview, 1, false, fp64);
    e = launch_sample(dc.fview, AF, LF, fp64, false, s);
  } else {
    e = launch_frames(dc.fview, AF, L.fgrid, s);
  }
  if (e != hipSuccess) return e;
  KArgs AV{};
  AV.shots = A.shots;
  AV.seed = A.seed;
  AV.offset = A.offset;
  AV.meas = H.nactive ? mrows : nullptr;
  AV.workspace = L.global_vec ? vws : nullptr;
  AV.nbits = bits;
  AV.list_cap = A.list_cap;
  e = launch_vector_pass(dc.vview, AV, L, fp64, s);
  if (e != hipSuccess) return e;
  FixupArgs X{};
  X.meas = A.meas;
  X.det = A.det;
  X.obs = A.obs;
  X.nrec = H.nrec;
  X.ndet = H.ndet;
  X.nobs = H.nobs;
  X.rows = dc.xrows;
  X.nrows = dc.nxrows;
  X.xdep_off = dc.xdep_off;
  X.xdep = dc.xdep;
  X.mrows = mrows;
  X.words = words;
  return launch_fixup(X, s);
}

// Stratified sampling tables (Section 3.2, rare-event sampling).  With odds
// w_l = p_l / (1 - p_l), e_s(t) = sum over s-subsets of the sites t .. N-1 of
// the product of their odds; P(exactly s of them fire) = e_s(t) prod(1 - p),
// so given s faults from site j on, the next one lies at or after t with
// probability e_s(t) / e_s(j).  Recurrence: e_0 = 1, e_s(N) = 0 for s >= 1,
// e_s(t) = e_s(t+1) + w_t e_{s-1}(t+1) (site t fires or not).  Every term is
// non-negative, so the relative rounding error stays within N ulps.
clifft_status strat_check(const CompiledProgram& H, int32_t r) {
  const int N = (int)H.site_p.size();
  if (r < 0) return fail(CLIFFT_E_INVALID_ARG, "the fault count must be >= 0");
  if (r > N) return fail(CLIFFT_E_INVALID_ARG, "more faults than noise sites");
  for (double q : H.site_p)
    if (!(q < 1.0)) return fail(CLIFFT_E_UNSUPPORTED, "stratified sampling needs every site probability below 1");
  return CLIFFT_OK;
}

std::vector<double> strat_rows(const CompiledProgram& H, int rows) {
  const size_t N = H.site_p.size();
  std::vector<double> E((size_t)rows * (N + 1));
  std::vector<double> prev(N + 1, 1.0), cur(N + 1);
  for (int s = 1; s <= rows; s++) {
    cur[N] = 0.0;
    for (size_t t = N; t-- > 0;) {
      const double w = H.site_p[t] / (1.0 - H.site_p[t]);
      cur[t] = cur[t + 1] + w * prev[t + 1];
    }
    std::copy(cur.begin(), cur.end(), E.begin() + (size_t)(s - 1) * (N + 1));
    prev.swap(cur);
  }
  return E;
}

clifft_status ensure_strat(const clifft_program* cp, const DeviceCopy* dc, int32_t r) {
  clifft_program* p = const_cast<clifft_program*>(cp);
  const CompiledProgram& H = p->host;
  clifft_status st = strat_check(H, r);
  if (st != CLIFFT_OK) return st;
  std::lock_guard<std::mutex> lock(p->mu);
  DeviceCopy* d = const_cast<DeviceCopy*>(dc);
  if (r == 0 || d->strat_rows >= r) return CLIFFT_OK;
  const size_t N = H.site_p.size();
  int rows = std::min<int>((int)N, std::max<int>(r, 2 * d->strat_rows));
  if ((size_t)rows * (N + 1) * sizeof(double) > ((size_t)1 << 30)) rows = r;
  if ((size_t)rows * (N + 1) * sizeof(double) > ((size_t)1 << 30))
    return fail(CLIFFT_E_CAPACITY, "stratified tables (faults x noise sites) exceed 1 GiB");
  std::vector<double> E = strat_rows(H, rows);
  const double er = E[(size_t)(r - 1) * (N + 1)];
  if (!(er > 0.0)) return fail(CLIFFT_E_INVALID_ARG, "the stratum has probability zero");
  if (!std::isfinite(er)) return fail(CLIFFT_E_CAPACITY, "stratified tables overflow for this fault count");
  // the previous (smaller) table stays allocated until the program is
  // freed: launches already queued may still read it
  const double* dst = nullptr;
  hipError_t e = upload_vec(E, &dst, d->allocs);
  if (e != hipSuccess) return fail(CLIFFT_E_DEVICE, std::string("stratified table upload failed: ") + hipGetErrorString(e));
  d->strat = dst;
  d->strat_rows = rows;
  return CLIFFT_OK;
}

clifft_status do_sample(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t offset,
                        const clifft_launch* cfg, void* ws, size_t ws_bytes, uint64_t* meas, uint64_t* det,
                        uint64_t* obs, void* stream, const uint32_t* forced_m, const int32_t* forced_faults,
                        double* probs, double* phi, double* gamma, bool trace, double* expval = nullptr,
                        int32_t strat_r = -1) {
  if (!p) return fail(CLIFFT_E_INVALID_ARG, "null program");
  if (shots == 0) return CLIFFT_OK;
  const DevProgram* D = nullptr;
  const DeviceCopy* DC = nullptr;
  clifft_status st = ensure_device(p, &D, &DC);
  if (st != CLIFFT_OK) return st;
  DevProgram V = *D;
  if (strat_r >= 0) {
    st = ensure_strat(p, DC, strat_r);
    if (st != CLIFFT_OK) return st;
    V.strat = DC->strat;
    V.strat_rows = DC->strat_rows;
  }
  LaunchShape L{};
  bool fp64 = false;
  st = choose_shape(p->host, D, cfg, shots, &L, &fp64, &p->tuned, trace, strat_r);
  if (st != CLIFFT_OK) return st;
  size_t need = workspace_bytes(p->host, L, fp64, shots);
  if (need > 0 && (ws == nullptr || ws_bytes < need)) {
    char buf[128];
    snprintf(buf, sizeof buf, "workspace of %zu bytes needed", need);
    return fail(CLIFFT_E_CAPACITY, buf);
  }
  KArgs A{};
  A.shots = shots;
  A.seed = seed;
  A.offset = offset;
  A.meas = meas;
  A.det = det;
  A.obs = obs;
  A.workspace = ws;
  A.expval = expval;
  A.strat_r = strat_r;
  A.list_cap = 0xFFFFFFFFu;
  if (const char* cap = getenv("CLIFFT_FRAMES_LIST_CAP")) A.list_cap = (uint32_t)strtoul(cap, nullptr, 10);
  hipStream_t s = (hipStream_t)stream;
  int* dflag = nullptr;
  if (trace) {
    A.forced_m = forced_m;
    A.forced_faults = forced_faults;
    A.probs = probs;
    A.phi_out = phi;
    A.gamma_out = gamma;
    if (hipMalloc(&dflag, sizeof(int)) != hipSuccess) return fail(CLIFFT_E_DEVICE, "flag allocation failed");
    (void)hipMemsetAsync(dflag, 0, sizeof(int), s);
    A.error = dflag;
  }
  hipError_t e = hipSuccess;
  if (L.spec) {
    hipFunction_t fn = nullptr;
    st = spec_function(const_cast<clifft_program*>(p), &fn);
    if (st != CLIFFT_OK) return st;
    e = launch_spec(fn, *D, A, L.grid, s);
  } else {
    e = launch_plan(p->host, *DC, L, A, fp64, trace, s, &V);
  }
  if (e != hipSuccess) {
    if (dflag) (void)hipFree(dflag);
    return fail(CLIFFT_E_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  }
  if (trace) {
    int h = 0;
    e = hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dflag);
    if (e != hipSuccess) return fail(CLIFFT_E_DEVICE, std::string("trace failed: ") + hipGetErrorString(e));
    if (h & 2) return fail(CLIFFT_E_IMPOSSIBLE_OUTCOME, "a forced outcome has probability zero");
  }
  return CLIFFT_OK;
}

}  // namespace

struct clifft_batch {
  std::vector<const clifft_program*> progs;
  std::vector<BatchProgram> table;  // device pointers of each program's upload
  // three queues: single shots of shot-per-workgroup programs, groups of
  // four shots of shot-per-wave programs, and 64-shot tile groups of
  // shot-per-lane programs; each sorted longest first
  std::vector<BatchItem> items_g, items_w, items_l;
  uint64_t wstart_g[5] = {}, wstart_w[5] = {}, wstart_l[5] = {};  // per-width item ranges
  bool fp64 = false;
  int device = 0;
  int grid_g = 0, grid_w = 0, grid_l = 0;
  size_t lds = 0;
  uint64_t slot_g = 0, slot_w = 0, slot_l = 0;  // workspace bytes per workgroup of each queue
  uint32_t rec_words = 0;
  uint64_t meas_words = 0, det_words = 0, obs_words = 0;
  BatchProgram* d_table = nullptr;
  BatchItem* d_items_g = nullptr;
  BatchItem* d_items_w = nullptr;
  BatchItem* d_items_l = nullptr;
  uint64_t* d_counter = nullptr;

  size_t workspace_bytes() const {
    return std::max({(size_t)grid_g * slot_g, (size_t)grid_w * slot_w, (size_t)grid_l * slot_l});
  }
};

extern "C" {

clifft_status clifft_compile(const char* text, size_t len, const clifft_compile_opts* opts, clifft_program** out) {
  if (!text || !out) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  *out = nullptr;
  CompileOptions co;
  if (opts) {
    if (opts->hir_passes & ~7) return fail(CLIFFT_E_INVALID_ARG, "hir_passes: unknown pass bits");
    if (opts->k_limit < 0) return fail(CLIFFT_E_INVALID_ARG, "k_limit must be >= 0");
    if (opts->drop_phases != 0 && opts->drop_phases != 1) return fail(CLIFFT_E_INVALID_ARG, "drop_phases must be 0 or 1");
    co.hir_passes = opts->hir_passes;
    co.k_limit = opts->k_limit;
    co.drop_phases = opts->drop_phases == 1;
    if (opts->postselect_words < -1 || (opts->postselect_words > 0 && !opts->postselect))
      return fail(CLIFFT_E_INVALID_ARG, "postselect: bad mask");
    if (opts->postselect_words == -1) co.postselect_all = true;
    else if (opts->postselect_words > 0) co.postselect.assign(opts->postselect, opts->postselect + opts->postselect_words);
  }
  clifft_program* p = new clifft_program();
  std::string err;
  int rc = compile_text(text, len, co, p->host, err);
  if (rc != 0) {
    delete p;
    return fail(rc == 1   ? CLIFFT_E_PARSE
                : rc == 2 ? CLIFFT_E_UNSUPPORTED
                : rc == 4 ? CLIFFT_E_INVALID_ARG
                          : CLIFFT_E_CAPACITY,
                err);
  }
  *out = p;
  return CLIFFT_OK;
}

clifft_status clifft_program_info(const clifft_program* p, clifft_info* o) {
  if (!p || !o) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  const CompiledProgram& H = p->host;
  o->num_qubits = H.nq;
  o->frame_words = H.W;
  o->k_max = H.kmax;
  o->num_events = H.nevents;
  o->num_measurements = H.nrec;
  o->num_detectors = H.ndet;
  o->num_observables = H.nobs;
  o->num_noise_sites = (int32_t)H.site_p.size();
  o->num_instructions = (int32_t)H.code.size();
  int nr = 0, na = 0;
  for (int c : H.ev_class) { nr += c == 1; na += c == 2; }
  o->num_random_events = nr;
  o->num_active_events = na;
  o->num_probes = H.nprobes;
  o->num_postselected = H.npost;
  return CLIFFT_OK;
}

clifft_status clifft_k_profile(const clifft_program* p, int32_t* out, size_t cap, size_t* n) {
  if (!p || !n) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  const auto& v = p->host.k_after;
  *n = v.size();
  for (size_t i = 0; out && i < v.size() && i < cap; i++) out[i] = v[i];
  return CLIFFT_OK;
}

clifft_status clifft_pair_orders(const clifft_program* p, int32_t* out, size_t cap, size_t* n) {
  if (!p || !n) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  const CompiledProgram& H = p->host;
  std::vector<int32_t> v;
  for (size_t i = 0; i < H.code.size(); i++) {
    const GInstr& in = H.code[i];
    if ((in.op != OP_MACTZ && in.op != OP_MACTX) || in.u == 0) continue;
    v.push_back((int32_t)i);
    v.push_back(H.pline[2u * in.u].kind);
    v.push_back(H.pline_items[in.u]);
    for (int e = 0; e < 2; e++) {
      const PairLine& L = H.pline[2u * in.u + e];
      v.push_back(L.nv);
      v.push_back(L.npos);
      for (int j = 0; j < 5; j++) v.push_back(L.pos[j]);
      for (int j = 0; j < 4; j++) v.push_back((int32_t)L.v[j]);
    }
  }
  *n = v.size();
  for (size_t i = 0; out && i < v.size() && i < cap; i++) out[i] = v[i];
  return CLIFFT_OK;
}

clifft_status clifft_event_classes(const clifft_program* p, int32_t* out, size_t cap, size_t* n) {
  if (!p || !n) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  const auto& v = p->host.ev_class;
  *n = v.size();
  for (size_t i = 0; out && i < v.size() && i < cap; i++) out[i] = v[i];
  return CLIFFT_OK;
}

clifft_status clifft_final_slots(const clifft_program* p, int32_t* slots, int32_t* k) {
  if (!p || !k) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  const auto& v = p->host.final_slots;
  *k = (int32_t)v.size();
  for (size_t i = 0; slots && i < v.size(); i++) slots[i] = v[i];
  return CLIFFT_OK;
}

clifft_status clifft_cost_model(const clifft_program* p, int32_t precision, clifft_cost* out) {
  if (!p || !out) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  if (precision != CLIFFT_FP32 && precision != CLIFFT_FP64) return fail(CLIFFT_E_INVALID_ARG, "bad precision");
  CostModel c = cost_model(p->host, precision == CLIFFT_FP64);
  out->int_ops = c.int_ops;
  out->flops = c.flops;
  out->vector_bytes = c.vector_bytes;
  out->record_bytes = c.record_bytes;
  out->expected_faults = c.expected_faults;
  out->instructions = c.instructions;
  out->int_ops_bitsliced = c.int_ops_bitsliced;
  out->vector_bytes_fused = c.vector_bytes_fused;
  out->vector_bytes_fused_group = c.vector_bytes_fused_group;
  out->vector_bytes_fused_batch = c.vector_bytes_fused_batch;
  out->paired_measurements = c.pair_starts;
  return CLIFFT_OK;
}

clifft_status clifft_resolve_launch(const clifft_program* p, const clifft_launch* cfg, uint64_t shots,
                                    clifft_launch* out) {
  if (!p || !out) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  LaunchShape L{};
  bool fp64 = false;
  clifft_status st = choose_shape(p->host, nullptr, cfg, shots ? shots : 1, &L, &fp64, &p->tuned);
  if (st != CLIFFT_OK) return st;
  out->precision = fp64 ? CLIFFT_FP64 : CLIFFT_FP32;
  out->threads_per_shot = L.G;
  out->grid = L.grid;
  out->vector_in_hbm = L.global_vec ? 1 : -1;
  out->specialize = L.G == kBitSliced ? (L.spec ? 1 : -1) : 0;
  out->split = L.split ? (L.flane ? 3 : 2) : (p->host.split_ok ? -1 : 0);
  return CLIFFT_OK;
}

clifft_status clifft_specialize(clifft_program* p, char* log, size_t cap) {
  if (!p) return fail(CLIFFT_E_INVALID_ARG, "null program");
  clifft_status st = ensure_spec(p);
  if (log && cap) {
    const std::string& m = p->spec_log;
    size_t n = std::min(cap - 1, m.size());
    memcpy(log, m.data(), n);
    log[n] = '\0';
  }
  return st;
}

clifft_status clifft_workspace_size(const clifft_program* p, const clifft_launch* cfg, uint64_t shots, size_t* bytes) {
  if (!p || !bytes) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  LaunchShape L{};
  bool fp64 = false;
  // the grid is sized for the largest shot count (so the workspace covers any call)
  clifft_status st = choose_shape(p->host, nullptr, cfg, ~0ull >> 8, &L, &fp64, &p->tuned);
  if (st != CLIFFT_OK) return st;
  *bytes = workspace_bytes(p->host, L, fp64, shots);
  return CLIFFT_OK;
}

clifft_status clifft_sample(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                            const clifft_launch* cfg, void* workspace, size_t workspace_bytes, uint64_t* meas,
                            uint64_t* det, uint64_t* obs, void* stream) {
  return do_sample(p, shots, seed, shot_offset, cfg, workspace, workspace_bytes, meas, det, obs, stream, nullptr,
                   nullptr, nullptr, nullptr, nullptr, false);
}

clifft_status clifft_sample_expval(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                                   const clifft_launch* cfg, void* workspace, size_t workspace_bytes, uint64_t* meas,
                                   uint64_t* det, uint64_t* obs, double* expval, void* stream) {
  return do_sample(p, shots, seed, shot_offset, cfg, workspace, workspace_bytes, meas, det, obs, stream, nullptr,
                   nullptr, nullptr, nullptr, nullptr, false, expval);
}

clifft_status clifft_sample_stratified(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                                       int32_t faults, const clifft_launch* cfg, void* workspace,
                                       size_t workspace_bytes, uint64_t* meas, uint64_t* det, uint64_t* obs,
                                       void* stream) {
  if (!p) return fail(CLIFFT_E_INVALID_ARG, "null program");
  clifft_status st = strat_check(p->host, faults);
  if (st != CLIFFT_OK) return st;
  return do_sample(p, shots, seed, shot_offset, cfg, workspace, workspace_bytes, meas, det, obs, stream, nullptr,
                   nullptr, nullptr, nullptr, nullptr, false, nullptr, faults);
}

clifft_status clifft_fault_count_pmf(const clifft_program* p, int32_t rmax, double* pmf) {
  if (!p || !pmf || rmax < 0) return fail(CLIFFT_E_INVALID_ARG, "null argument or rmax < 0");
  const CompiledProgram& H = p->host;
  for (double q : H.site_p)
    if (!(q < 1.0)) return fail(CLIFFT_E_UNSUPPORTED, "the fault-count weights need every site probability below 1");
  // pmf[r] = prod(1 - p) e_r over all sites: the log of the product, and
  // e_r accumulated site by site (e_r += w e_{r-1}, highest degree first)
  double lp0 = 0.0;
  std::vector<double> e((size_t)rmax + 1, 0.0);
  e[0] = 1.0;
  for (double q : H.site_p) {
    lp0 += std::log1p(-q);
    const double w = q / (1.0 - q);
    for (int r = rmax; r >= 1; r--) e[r] += w * e[r - 1];
  }
  for (int r = 0; r <= rmax; r++) {
    if (!std::isfinite(e[r])) return fail(CLIFFT_E_CAPACITY, "fault-count weights overflow");
    pmf[r] = e[r] > 0.0 ? std::exp(lp0 + std::log(e[r])) : 0.0;
  }
  return CLIFFT_OK;
}

clifft_status clifft_sample_noalloc(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                                    const clifft_launch* cfg, uint64_t* meas, uint64_t* det, uint64_t* obs,
                                    void* stream) {
  if (!p) return fail(CLIFFT_E_INVALID_ARG, "null program");
  if (shots == 0) return CLIFFT_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CLIFFT_E_DEVICE, "no HIP device");
  const DevProgram* D = nullptr;
  const DeviceCopy* DC = nullptr;
  hipFunction_t spec_fn = nullptr;
  {
    // the program must already be resident: uploading it would allocate
    clifft_program* mp = const_cast<clifft_program*>(p);
    std::lock_guard<std::mutex> lock(mp->mu);
    auto it = mp->dev.find(dev);
    if (it == mp->dev.end())
      return fail(CLIFFT_E_INVALID_ARG,
                  "program is not resident on this device (a clifft_sample call on the device uploads it)");
    D = &it->second.view;
    DC = &it->second;
    spec_fn = it->second.spec_fn;
  }
  LaunchShape L{};
  bool fp64 = false;
  clifft_status st = choose_shape(p->host, D, cfg, shots, &L, &fp64, &p->tuned, false);
  if (st != CLIFFT_OK) return st;
  if (L.spec && !spec_fn) {
    // loading the specialized code object would allocate: the bit-sliced
    // interpreter writes the same records
    if (cfg && cfg->specialize == 1)
      return fail(CLIFFT_E_INVALID_ARG, "the specialized kernel is not loaded on this device yet");
    clifft_launch c = cfg ? *cfg : clifft_launch{};
    c.precision = fp64 ? CLIFFT_FP64 : CLIFFT_FP32;
    c.threads_per_shot = kBitSliced;
    c.grid = L.grid;
    c.specialize = -1;
    st = choose_shape(p->host, D, &c, shots, &L, &fp64, nullptr, false);
    if (st != CLIFFT_OK) return st;
  }
  void* ws = nullptr;
  size_t need = workspace_bytes(p->host, L, fp64, shots);
  if (need > 0) {
    if (need > kScratchBytes) {
      // keep the workspace inside the fixed scratch: fewer persistent
      // workgroups (records do not depend on the grid); the split form's
      // rows do not shrink with the grid
      const size_t fixed = L.split ? split_rows_bytes(p->host, shots) : 0;
      const size_t per_block = L.global_vec ? (need - fixed) / (size_t)L.grid : 0;
      const size_t fit = per_block && fixed < kScratchBytes ? (kScratchBytes - fixed) / per_block : 0;
      if ((cfg && cfg->grid > 0) || fit == 0) {
        char buf[160];
        snprintf(buf, sizeof buf, "workspace of %zu bytes exceeds the %zu-byte scratch of the allocation-free call",
                 need, kScratchBytes);
        return fail(CLIFFT_E_CAPACITY, buf);
      }
      L.grid = (int)fit;
    }
    hipError_t e = scratch_region(&ws);
    if (e != hipSuccess) return fail(CLIFFT_E_DEVICE, std::string("scratch lookup failed: ") + hipGetErrorString(e));
  }
  KArgs A{};
  A.shots = shots;
  A.seed = seed;
  A.offset = shot_offset;
  A.meas = meas;
  A.det = det;
  A.obs = obs;
  A.workspace = ws;
  A.list_cap = 0xFFFFFFFFu;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = L.spec ? launch_spec(spec_fn, *D, A, L.grid, s) : launch_plan(p->host, *DC, L, A, fp64, false, s);
  if (e != hipSuccess) return fail(CLIFFT_E_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return CLIFFT_OK;
}

clifft_status clifft_sample_trace(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                                  const clifft_launch* cfg, const uint32_t* forced_m, const int32_t* forced_faults,
                                  double* probs, double* phi, double* gamma, void* workspace, size_t workspace_bytes,
                                  uint64_t* meas, uint64_t* det, uint64_t* obs, void* stream) {
  return do_sample(p, shots, seed, shot_offset, cfg, workspace, workspace_bytes, meas, det, obs, stream, forced_m,
                   forced_faults, probs, phi, gamma, true);
}

clifft_status clifft_batch_create(const clifft_program* const* progs, int32_t n, const uint64_t* shots,
                                  const uint64_t* seeds, const clifft_launch* cfg, clifft_batch** out) {
  if (!progs || !shots || !seeds || !out || n <= 0) return fail(CLIFFT_E_INVALID_ARG, "bad batch arguments");
  *out = nullptr;
  clifft_launch c{};
  if (cfg) c = *cfg;
  if (c.precision != CLIFFT_FP32 && c.precision != CLIFFT_FP64) return fail(CLIFFT_E_INVALID_ARG, "bad precision");
  clifft_batch* b = new clifft_batch();
  b->fp64 = c.precision == CLIFFT_FP64;
  (void)hipGetDevice(&b->device);
  const size_t amp = b->fp64 ? 16 : 8;
  std::vector<double> cost_g, cost_w, cost_l;
  for (int i = 0; i < n; i++) {
    if (!progs[i]) { delete b; return fail(CLIFFT_E_INVALID_ARG, "null program in batch"); }
    const DevProgram* D = nullptr;
    clifft_status st = ensure_device(progs[i], &D);
    if (st != CLIFFT_OK) { delete b; return st; }
    const CompiledProgram& H = progs[i]->host;
    BatchProgram bp{};
    bp.P = *D;
    bp.shots = shots[i];
    bp.seed = seeds[i];
    bp.offset = 0;
    const uint64_t words = (shots[i] + 63) / 64;
    bp.meas_off = b->meas_words;
    bp.det_off = b->det_words;
    bp.obs_off = b->obs_words;
    b->meas_words += (uint64_t)H.nrec * words;
    b->det_words += (uint64_t)H.ndet * words;
    b->obs_words += (uint64_t)H.nobs * words;
    // tier: frames shot-per-lane while 64 vectors per wave stay small, a
    // shot per wave up to kWaveMaxK, else one shot per workgroup
    int G = c.threads_per_shot == 256 || c.threads_per_shot == 64 || c.threads_per_shot == 1
                ? c.threads_per_shot
                : (H.kmax <= kBatchLaneMaxK ? 1 : H.kmax <= kWaveMaxK ? 64 : 256);
    // (an autotuned program's standalone tier is not used here: the queue
    // kernels' costs differ, and on the batched set the k_max rule above
    // ran the step faster than the standalone choices)
    bp.G = G;
    const uint64_t vec = (uint64_t)1 << H.kmax;
    // two buffers per shot vector (out-of-place collapses)
    if (G == 1) b->slot_l = std::max<uint64_t>(b->slot_l, 2 * 4 * 64 * vec * amp);
    else if (G == 64) b->slot_w = std::max<uint64_t>(b->slot_w, 2 * 4 * vec * amp);
    else b->slot_g = std::max<uint64_t>(b->slot_g, 2 * vec * amp);
    b->rec_words = std::max<uint32_t>(b->rec_words, (uint32_t)(H.nrec + H.ndet + H.nobs));
    b->progs.push_back(progs[i]);
    b->table.push_back(bp);
    // per-shot cost estimate (only used to order the items, longest first)
    CostModel cm = cost_model(H, b->fp64);
    // rough item durations: a lane item runs one shot per lane (its time is
    // one shot's per-lane work), a workgroup item spreads one shot over 256
    // threads
    const double lane_item = 20.0 * cm.instructions + cm.int_ops + cm.vector_bytes;
    const double block_item = 20.0 * cm.instructions + (cm.vector_bytes + cm.flops) / 64.0;
    const double wave_item = 20.0 * cm.instructions + (cm.vector_bytes + cm.flops) / 16.0;
    if (G == 1) {
      for (uint64_t t = 0; t < words; t += 4) {
        b->items_l.push_back(BatchItem{(uint32_t)i, 1u, t});
        cost_l.push_back(lane_item);
      }
    } else if (G == 64) {
      for (uint64_t s = 0; s < shots[i]; s += 4) {
        b->items_w.push_back(BatchItem{(uint32_t)i, 64u, s});
        cost_w.push_back(wave_item);
      }
    } else {
      for (uint64_t s = 0; s < shots[i]; s++) {
        b->items_g.push_back(BatchItem{(uint32_t)i, 256u, s});
        cost_g.push_back(block_item);
      }
    }
  }
  auto longest_first = [](std::vector<BatchItem>& items, const std::vector<double>& cost) {
    std::vector<size_t> order(items.size());
    for (size_t i = 0; i < order.size(); i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c2) { return cost[a] > cost[c2]; });
    std::vector<BatchItem> sorted(order.size());
    for (size_t i = 0; i < order.size(); i++) sorted[i] = items[order[i]];
    items.swap(sorted);
  };
  longest_first(b->items_g, cost_g);
  longest_first(b->items_w, cost_w);
  longest_first(b->items_l, cost_l);
  // each queue runs one kernel per frame width: group its items by width
  // (stable, so each group stays longest first)
  auto by_width = [&](std::vector<BatchItem>& items, uint64_t* ws) {
    std::stable_sort(items.begin(), items.end(), [&](const BatchItem& x, const BatchItem& y) {
      return b->table[x.prog].P.W < b->table[y.prog].P.W;
    });
    ws[0] = 0;
    for (int w = 1; w <= 4; w++) {
      ws[w] = ws[w - 1];
      while (ws[w] < items.size() && b->table[items[ws[w]].prog].P.W == w) ws[w]++;
    }
  };
  by_width(b->items_g, b->wstart_g);
  by_width(b->items_w, b->wstart_w);
  by_width(b->items_l, b->wstart_l);
  b->rec_words = (b->rec_words + 1) & ~1u;
  b->lds = (size_t)4 * b->rec_words * 8 + 64 + 64;
  if (b->lds > kLdsLimit) { delete b; return fail(CLIFFT_E_CAPACITY, "too many records for the batched launch"); }
  const int cus = device_cus();
  auto grid_for = [&](int per_cu, uint64_t slot, size_t nitems) {
    int g = c.grid > 0 ? c.grid : cus * per_cu;
    const size_t cap = std::max<size_t>(1, kWorkspaceBudget / std::max<uint64_t>(slot, 1));
    if (c.grid <= 0 && (size_t)g > cap) g = (int)cap;
    if ((size_t)g > nitems) g = (int)std::max<size_t>(1, nitems);
    return g;
  };
  // the workgroup queue is bounded by registers (about two workgroups per
  // CU resident), the lane queue by LDS
  b->grid_g = grid_for(4, b->slot_g, b->items_g.size());
  b->grid_w = grid_for(4, b->slot_w, b->items_w.size());
  b->grid_l = grid_for((int)std::max<size_t>(1, std::min<size_t>(8, kLdsLimit / b->lds)), b->slot_l, b->items_l.size());
  hipError_t e = hipMalloc((void**)&b->d_table, sizeof(BatchProgram) * b->table.size());
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_items_g, sizeof(BatchItem) * std::max<size_t>(1, b->items_g.size()));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_items_w, sizeof(BatchItem) * std::max<size_t>(1, b->items_w.size()));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_items_l, sizeof(BatchItem) * std::max<size_t>(1, b->items_l.size()));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_counter, 128);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_table, b->table.data(), sizeof(BatchProgram) * b->table.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !b->items_g.empty())
    e = hipMemcpy(b->d_items_g, b->items_g.data(), sizeof(BatchItem) * b->items_g.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !b->items_w.empty())
    e = hipMemcpy(b->d_items_w, b->items_w.data(), sizeof(BatchItem) * b->items_w.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !b->items_l.empty())
    e = hipMemcpy(b->d_items_l, b->items_l.data(), sizeof(BatchItem) * b->items_l.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    clifft_batch_free(b);
    return fail(CLIFFT_E_DEVICE, std::string("batch upload failed: ") + hipGetErrorString(e));
  }
  *out = b;
  return CLIFFT_OK;
}

clifft_status clifft_batch_layout(const clifft_batch* b, int32_t i, uint64_t* meas_off, uint64_t* det_off,
                                  uint64_t* obs_off) {
  if (!b || i < 0 || (size_t)i >= b->table.size()) return fail(CLIFFT_E_INVALID_ARG, "bad batch index");
  if (meas_off) *meas_off = b->table[i].meas_off;
  if (det_off) *det_off = b->table[i].det_off;
  if (obs_off) *obs_off = b->table[i].obs_off;
  return CLIFFT_OK;
}

clifft_status clifft_batch_sizes(const clifft_batch* b, uint64_t* meas_words, uint64_t* det_words,
                                 uint64_t* obs_words, size_t* workspace_bytes, int32_t* threads_per_shot) {
  if (!b) return fail(CLIFFT_E_INVALID_ARG, "null batch");
  if (meas_words) *meas_words = b->meas_words;
  if (det_words) *det_words = b->det_words;
  if (obs_words) *obs_words = b->obs_words;
  if (workspace_bytes) *workspace_bytes = b->workspace_bytes();
  if (threads_per_shot)
    for (size_t i = 0; i < b->table.size(); i++) threads_per_shot[i] = b->table[i].G;
  return CLIFFT_OK;
}

clifft_status clifft_batch_sample(const clifft_batch* b, void* workspace, size_t workspace_bytes, uint64_t* meas,
                                  uint64_t* det, uint64_t* obs, void* stream) {
  if (!b) return fail(CLIFFT_E_INVALID_ARG, "null batch");
  const size_t need = b->workspace_bytes();
  if (need > 0 && (!workspace || workspace_bytes < need)) {
    char buf[128];
    snprintf(buf, sizeof buf, "workspace of %zu bytes needed", need);
    return fail(CLIFFT_E_CAPACITY, buf);
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev != b->device) return fail(CLIFFT_E_INVALID_ARG, "batch belongs to another device");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_zero(meas, b->meas_words, s);
  if (e == hipSuccess) e = launch_zero(det, b->det_words, s);
  if (e == hipSuccess) e = launch_zero(obs, b->obs_words, s);
  BatchArgs G{};
  G.progs = b->d_table;
  G.items = b->d_items_g;
  G.nitems = b->items_g.size();
  std::copy(b->wstart_g, b->wstart_g + 5, G.wstart);
  G.counter = (uint32_t*)b->d_counter;
  G.meas = meas;
  G.det = det;
  G.obs = obs;
  G.workspace = workspace;
  G.slot_bytes = b->slot_g;
  G.rec_words = b->rec_words;
  BatchArgs Wv = G;
  Wv.items = b->d_items_w;
  Wv.nitems = b->items_w.size();
  std::copy(b->wstart_w, b->wstart_w + 5, Wv.wstart);
  Wv.counter = (uint32_t*)b->d_counter + 8;
  Wv.slot_bytes = b->slot_w;
  BatchArgs L = G;
  L.items = b->d_items_l;
  L.nitems = b->items_l.size();
  std::copy(b->wstart_l, b->wstart_l + 5, L.wstart);
  L.counter = (uint32_t*)b->d_counter + 16;
  L.slot_bytes = b->slot_l;
  if (e == hipSuccess) {
    // batches holding post-selected programs take the kernels with that path
    bool ext = false;
    for (const clifft_program* q : b->progs) ext = ext || q->host.npost > 0;
    e = ext ? launch_batch_ext(G, b->grid_g, Wv, b->grid_w, L, b->grid_l, b->lds, b->fp64, s)
            : launch_batch(G, b->grid_g, Wv, b->grid_w, L, b->grid_l, b->lds, b->fp64, s);
  }
  if (e != hipSuccess) return fail(CLIFFT_E_DEVICE, std::string("batch launch failed: ") + hipGetErrorString(e));
  return CLIFFT_OK;
}

void clifft_batch_free(clifft_batch* b) {
  if (!b) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b->device);
  if (b->d_table) (void)hipFree(b->d_table);
  if (b->d_items_g) (void)hipFree(b->d_items_g);
  if (b->d_items_w) (void)hipFree(b->d_items_w);
  if (b->d_items_l) (void)hipFree(b->d_items_l);
  if (b->d_counter) (void)hipFree(b->d_counter);
  (void)hipSetDevice(cur);
  delete b;
}

}  // extern "C"

namespace {

// Autotuner results by program signature (the compiled stream and side
// tables, the precision, the trial size and the device), so that a program
// compiled again in the same process is not timed again.
struct TuneKey {
  uint64_t sig;
  int precision;
  uint64_t trial;
  int device;
  bool operator<(const TuneKey& o) const {
    return std::tie(sig, precision, trial, device) < std::tie(o.sig, o.precision, o.trial, o.device);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, clifft_launch> g_tune_cache;

uint64_t program_signature(const CompiledProgram& H) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a, 64 bit
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; i++) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(&H.nq, sizeof H.nq);
  mix(H.code.data(), H.code.size() * sizeof(GInstr));
  mix(H.masks.data(), H.masks.size() * sizeof(uint64_t));
  mix(H.consts.data(), H.consts.size() * sizeof(double));
  mix(H.site_p.data(), H.site_p.size() * sizeof(double));
  mix(H.site_type.data(), H.site_type.size());
  return h;
}

}  // namespace

extern "C" {

clifft_status clifft_autotune(clifft_program* p, uint64_t shots, int32_t precision, void* stream, clifft_launch* out) {
  if (!p) return fail(CLIFFT_E_INVALID_ARG, "null program");
  if (precision != CLIFFT_FP32 && precision != CLIFFT_FP64) return fail(CLIFFT_E_INVALID_ARG, "bad precision");
  const CompiledProgram& H = p->host;
  const int cus = device_cus();
  // trial size: enough work to fill the device a few times over
  // (Pauli-frame programs take the workload itself up to 2^24 shots: their
  // best grid depends on the number of 2048-shot tiles)
  uint64_t trial = H.kmax == 0 ? ((uint64_t)1 << 24) : H.kmax <= 12 ? ((uint64_t)1 << 18) : (uint64_t)cus * 8;
  if (shots > 0 && shots < trial) trial = shots;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const TuneKey key{program_signature(H), precision, trial, dev};
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      std::lock_guard<std::mutex> lock2(p->mu);
      p->tuned[{dev, precision}] = it->second;
      if (out) *out = it->second;
      return CLIFFT_OK;
    }
  }
  // Stage 1: every tier at its default grid.  Stage 2: grids from one to
  // eight workgroups per CU for the two fastest tiers.
  std::vector<clifft_launch> tiers;
  if (H.kmax == 0 && !H.has_cfeed) {
    tiers.push_back(clifft_launch{precision, kBitSliced, 0, 0, -1, 0});
    if (spec_supported(H, nullptr) && ensure_spec(p) == CLIFFT_OK)
      tiers.push_back(clifft_launch{precision, kBitSliced, 0, 0, 1, 0});
    tiers.push_back(clifft_launch{precision, 1, 0, 0, 0, -1});
  } else if (H.kmax == 0) {
    tiers.push_back(clifft_launch{precision, 1, 0, 0, 0, -1});
  } else {
    for (int G : {1, 64, 256}) {
      if (G == 1 && H.kmax > kLaneMaxK) continue;
      if (G == 64 && H.kmax < 7) continue;
      if (G == 256 && H.kmax < 11) continue;
      for (int hbm : {-1, 1}) tiers.push_back(clifft_launch{precision, G, 0, hbm, 0, -1});
    }
    // split form: frame pass bit-sliced (2) or shot per lane (3), vector
    // pass shot per lane (the shot-granular vector passes are latency bound
    // without frame work to hide it)
    if (H.split_ok && H.kmax <= kLaneMaxK)
      for (int fp : {2, 3})
        for (int hbm : {-1, 1})
          if (fp == 3 || !H.has_cfeed) tiers.push_back(clifft_launch{precision, 1, 0, hbm, 0, fp});
  }
  const DevProgram* D = nullptr;
  const DeviceCopy* DC = nullptr;
  clifft_status st = ensure_device(p, &D, &DC);
  if (st != CLIFFT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const uint64_t words = (trial + 63) / 64;
  uint64_t *meas = nullptr, *det = nullptr, *obs = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void**)&meas, (H.nrec + 1) * words * 8);
  if (e == hipSuccess) e = hipMalloc((void**)&det, (H.ndet + 1) * words * 8);
  if (e == hipSuccess) e = hipMalloc((void**)&obs, (H.nobs + 1) * words * 8);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // time one candidate (the faster of two launches); < 0 when it does not fit
  auto time_one = [&](const clifft_launch& c, clifft_launch* resolved) -> float {
    LaunchShape L{};
    bool fp64 = false;
    if (e != hipSuccess || choose_shape(H, D, &c, trial, &L, &fp64) != CLIFFT_OK) return -1.0f;
    size_t wsb = workspace_bytes(H, L, fp64, trial);
    void* ws = nullptr;
    if (wsb && hipMalloc(&ws, wsb) != hipSuccess) {
      (void)hipGetLastError();
      return -1.0f;
    }
    KArgs A{};
    A.shots = trial;
    A.seed = 0;
    A.meas = meas;
    A.det = det;
    A.obs = obs;
    A.workspace = ws;
    A.list_cap = 0xFFFFFFFFu;
    hipFunction_t fn = nullptr;
    if (L.spec && spec_function(p, &fn) != CLIFFT_OK) {
      if (ws) (void)hipFree(ws);
      return -1.0f;
    }
    float best = 1e30f;
    for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {
      float ms = 0;
      e = hipEventRecord(e0, s);
      if (e == hipSuccess) e = L.spec ? launch_spec(fn, *D, A, L.grid, s) : launch_plan(H, *DC, L, A, fp64, false, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      best = std::min(best, ms);
    }
    if (ws) (void)hipFree(ws);
    *resolved = clifft_launch{precision, L.G, L.grid, L.global_vec ? 1 : -1,
                              L.G == kBitSliced ? (L.spec ? 1 : -1) : 0,
                              L.split ? (L.flane ? 3 : 2) : (H.split_ok ? -1 : 0)};
    return e == hipSuccess ? best : -1.0f;
  };
  std::vector<std::pair<float, clifft_launch>> ranked;  // (ms, tier as requested)
  float best_ms = 1e30f;
  clifft_launch best{};
  bool found = false;
  for (const clifft_launch& c : tiers) {
    clifft_launch r{};
    const float ms = time_one(c, &r);
    if (ms < 0) continue;
    ranked.push_back({ms, c});
    if (ms < best_ms) { best_ms = ms; best = r; found = true; }
  }
  std::sort(ranked.begin(), ranked.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  const std::vector<int> mults = H.kmax == 0 ? std::vector<int>{1, 2, 4, 5, 8, 16} : std::vector<int>{1, 2, 4, 8};
  for (size_t t = 0; t < ranked.size() && t < 2 && e == hipSuccess; t++)
    for (int m : mults) {
      clifft_launch c = ranked[t].second;
      c.grid = cus * (c.specialize == 1 ? 2 * m : m);
      clifft_launch r{};
      const float ms = time_one(c, &r);
      if (ms >= 0 && ms < best_ms) { best_ms = ms; best = r; found = true; }
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (meas) (void)hipFree(meas);
  if (det) (void)hipFree(det);
  if (obs) (void)hipFree(obs);
  if (e != hipSuccess) return fail(CLIFFT_E_DEVICE, std::string("autotune failed: ") + hipGetErrorString(e));
  if (!found) return fail(CLIFFT_E_CAPACITY, "no launch shape fits this program");
  {
    std::lock_guard<std::mutex> lock(p->mu);
    p->tuned[{dev, precision}] = best;
  }
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = best;
  }
  if (out) *out = best;
  return CLIFFT_OK;
}

void clifft_program_free(clifft_program* p) {
  if (!p) return;
  for (auto& kv : p->dev) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(kv.first);
    for (void* a : kv.second.allocs) (void)hipFree(a);
    if (kv.second.spec_mod) (void)hipModuleUnload(kv.second.spec_mod);
    (void)hipSetDevice(cur);
  }
  delete p;
}

clifft_status clifft_probe(int32_t kind, void* dst, const void* src, uint64_t n, int32_t grid, void* stream) {
  if (!dst || grid <= 0 || kind < 0 || kind > 2) return fail(CLIFFT_E_INVALID_ARG, "bad probe arguments");
  if (kind != 1 && (!src || n % 16 != 0))
    return fail(CLIFFT_E_INVALID_ARG, "copy and read probes need src and a multiple of 16 bytes");
  if (kind == 1 && n > 0xFFFFFFFFull) return fail(CLIFFT_E_INVALID_ARG, "too many probe iterations");
  hipError_t e = launch_probe(kind, dst, src, n, grid, (hipStream_t)stream);
  if (e != hipSuccess) return fail(CLIFFT_E_DEVICE, std::string("probe launch failed: ") + hipGetErrorString(e));
  return CLIFFT_OK;
}

const char* clifft_last_error(void) { return g_err.c_str(); }

}  // extern "C"
