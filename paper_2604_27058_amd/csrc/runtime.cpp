// C-ABI implementation: program handles, device upload, launch-shape
// selection and the sampling entry points declared in include/clifft.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
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
  std::vector<void*> allocs;
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

clifft_status ensure_device(const clifft_program* cp, const DevProgram** out) {
  clifft_program* p = const_cast<clifft_program*>(cp);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CLIFFT_E_DEVICE, "no HIP device");
  std::lock_guard<std::mutex> lock(p->mu);
  auto it = p->dev.find(dev);
  if (it != p->dev.end()) {
    *out = &it->second.view;
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
  v.nsites = (int)H.site_p.size();
  v.nchunks = H.nchunks;
  v.rblk_max = H.rblk_max;
  v.ndet_rows = H.ndet_rows;
  {
    double f = 0;
    for (double q : H.site_p) f += q;
    v.exp_faults = (float)f;
  }
  auto res = p->dev.emplace(dev, std::move(dc));
  *out = &res.first->second.view;
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
                           const std::map<std::pair<int, int>, clifft_launch>* tuned = nullptr, bool trace = false) {
  clifft_launch c{};
  if (cfg) c = *cfg;
  if (c.precision != CLIFFT_FP32 && c.precision != CLIFFT_FP64) return fail(CLIFFT_E_INVALID_ARG, "bad precision");
  *fp64 = c.precision == CLIFFT_FP64;
  if (tuned && c.threads_per_shot == 0 && c.grid == 0 && c.vector_in_hbm == 0 && c.specialize == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto it = tuned->find({dev, c.precision});
    if (it != tuned->end() && !(trace && it->second.threads_per_shot == kBitSliced)) c = it->second;
  }
  const size_t amp = *fp64 ? 16 : 8;
  const size_t vec = (size_t)1 << H.kmax;
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
    const size_t rows_bytes = frames_lds_rows(tmp) * 64 * 4;
    const bool spec = c.specialize == 1;
    const bool bs_ok = H.kmax == 0 && !trace && (spec || rows_bytes <= kLdsLimit);
    if (c.specialize == 1 && G != 0 && G != kBitSliced)
      return fail(CLIFFT_E_INVALID_ARG, "specialize applies to the bit-sliced tier only");
    if ((G == kBitSliced || spec) && !bs_ok)
      return fail(CLIFFT_E_CAPACITY, "bit-sliced frames need k_max = 0 and rows in LDS (not in trace mode)");
    if (spec && !spec_supported(H, nullptr)) {
      std::string why;
      spec_supported(H, &why);
      return fail(CLIFFT_E_UNSUPPORTED, why);
    }
    if (G == 0 && bs_ok) G = kBitSliced;
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

size_t workspace_bytes(const CompiledProgram& H, const LaunchShape& L, bool fp64) {
  if (!L.global_vec) return 0;
  size_t amp = fp64 ? 16 : 8;
  size_t units = (size_t)L.grid * (L.G == 256 ? 1 : 4);
  // two buffers per unit: active measurements collapse from one into the other
  return 2 * units * ((size_t)1 << H.kmax) * amp * (L.G == 1 ? 64 : 1);
}

clifft_status do_sample(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t offset,
                        const clifft_launch* cfg, void* ws, size_t ws_bytes, uint64_t* meas, uint64_t* det,
                        uint64_t* obs, void* stream, const uint32_t* forced_m, const int32_t* forced_faults,
                        double* probs, double* phi, double* gamma, bool trace) {
  if (!p) return fail(CLIFFT_E_INVALID_ARG, "null program");
  if (shots == 0) return CLIFFT_OK;
  const DevProgram* D = nullptr;
  clifft_status st = ensure_device(p, &D);
  if (st != CLIFFT_OK) return st;
  LaunchShape L{};
  bool fp64 = false;
  st = choose_shape(p->host, D, cfg, shots, &L, &fp64, &p->tuned, trace);
  if (st != CLIFFT_OK) return st;
  size_t need = workspace_bytes(p->host, L, fp64);
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
    e = launch_sample(*D, A, L, fp64, trace, s);
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
    if (opts->hir_passes & ~3) return fail(CLIFFT_E_INVALID_ARG, "hir_passes: unknown pass bits");
    if (opts->k_limit < 0) return fail(CLIFFT_E_INVALID_ARG, "k_limit must be >= 0");
    if (opts->drop_phases != 0 && opts->drop_phases != 1) return fail(CLIFFT_E_INVALID_ARG, "drop_phases must be 0 or 1");
    co.hir_passes = opts->hir_passes;
    co.k_limit = opts->k_limit;
    co.drop_phases = opts->drop_phases == 1;
  }
  clifft_program* p = new clifft_program();
  std::string err;
  int rc = compile_text(text, len, co, p->host, err);
  if (rc != 0) {
    delete p;
    return fail(rc == 1 ? CLIFFT_E_PARSE : rc == 2 ? CLIFFT_E_UNSUPPORTED : CLIFFT_E_CAPACITY, err);
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
  return CLIFFT_OK;
}

clifft_status clifft_k_profile(const clifft_program* p, int32_t* out, size_t cap, size_t* n) {
  if (!p || !n) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  const auto& v = p->host.k_after;
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

clifft_status clifft_workspace_size(const clifft_program* p, const clifft_launch* cfg, size_t* bytes) {
  if (!p || !bytes) return fail(CLIFFT_E_INVALID_ARG, "null argument");
  LaunchShape L{};
  bool fp64 = false;
  clifft_status st = choose_shape(p->host, nullptr, cfg, ~0ull >> 8, &L, &fp64, &p->tuned);
  if (st != CLIFFT_OK) return st;
  *bytes = workspace_bytes(p->host, L, fp64);
  return CLIFFT_OK;
}

clifft_status clifft_sample(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                            const clifft_launch* cfg, void* workspace, size_t workspace_bytes, uint64_t* meas,
                            uint64_t* det, uint64_t* obs, void* stream) {
  return do_sample(p, shots, seed, shot_offset, cfg, workspace, workspace_bytes, meas, det, obs, stream, nullptr,
                   nullptr, nullptr, nullptr, nullptr, false);
}

clifft_status clifft_sample_noalloc(const clifft_program* p, uint64_t shots, uint64_t seed, uint64_t shot_offset,
                                    const clifft_launch* cfg, uint64_t* meas, uint64_t* det, uint64_t* obs,
                                    void* stream) {
  if (!p) return fail(CLIFFT_E_INVALID_ARG, "null program");
  if (shots == 0) return CLIFFT_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CLIFFT_E_DEVICE, "no HIP device");
  const DevProgram* D = nullptr;
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
  size_t need = workspace_bytes(p->host, L, fp64);
  if (need > 0) {
    if (need > kScratchBytes) {
      // keep the workspace inside the fixed scratch: fewer persistent
      // workgroups (records do not depend on the grid)
      const size_t per_block = need / (size_t)L.grid;
      const size_t fit = kScratchBytes / per_block;
      if ((cfg && cfg->grid > 0) || fit == 0) {
        char buf[160];
        snprintf(buf, sizeof buf, "workspace of %zu bytes exceeds the %zu-byte scratch of the allocation-free call",
                 cfg && cfg->grid > 0 ? need : per_block, kScratchBytes);
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
  hipError_t e = L.spec ? launch_spec(spec_fn, *D, A, L.grid, s) : launch_sample(*D, A, L, fp64, false, s);
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
    if (c.threads_per_shot == 0) {
      // an autotuned program keeps its tier inside the batch
      auto it = progs[i]->tuned.find({b->device, c.precision});
      if (it != progs[i]->tuned.end() && it->second.threads_per_shot > 0 &&
          (H.kmax <= kLaneMaxK || it->second.threads_per_shot != 1))
        G = it->second.threads_per_shot;
    }
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
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_counter, 64);
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
  Wv.counter = (uint32_t*)b->d_counter + 2;
  Wv.slot_bytes = b->slot_w;
  BatchArgs L = G;
  L.items = b->d_items_l;
  L.nitems = b->items_l.size();
  L.counter = (uint32_t*)b->d_counter + 4;
  L.slot_bytes = b->slot_l;
  if (e == hipSuccess) e = launch_batch(G, b->grid_g, Wv, b->grid_w, L, b->grid_l, b->lds, b->fp64, s);
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
  std::vector<clifft_launch> cands;
  const int mult[4] = {1, 2, 4, 8};
  if (H.kmax == 0) {
    for (int m : {1, 2, 4, 5, 8, 16}) cands.push_back(clifft_launch{precision, kBitSliced, cus * m, 0, -1});
    if (spec_supported(H, nullptr) && ensure_spec(p) == CLIFFT_OK)
      for (int m : {4, 8, 12, 16, 24, 32}) cands.push_back(clifft_launch{precision, kBitSliced, cus * m, 0, 1});
  }
  for (int G : {1, 64, 256}) {
    if (H.kmax == 0 && G != 1) continue;
    for (int hbm : {-1, 1}) {
      if (H.kmax == 0 && hbm == 1) continue;
      if (G == 1 && H.kmax > kLaneMaxK) continue;
      for (int m : mult) cands.push_back(clifft_launch{precision, G, cus * m, H.kmax == 0 ? 0 : hbm});
    }
  }
  const DevProgram* D = nullptr;
  clifft_status st = ensure_device(p, &D);
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
  float best_ms = 1e30f;
  clifft_launch best{};
  bool found = false;
  for (const clifft_launch& c : cands) {
    if (e != hipSuccess) break;
    LaunchShape L{};
    bool fp64 = false;
    if (choose_shape(H, D, &c, trial, &L, &fp64) != CLIFFT_OK) continue;
    size_t wsb = workspace_bytes(H, L, fp64);
    void* ws = nullptr;
    if (wsb && hipMalloc(&ws, wsb) != hipSuccess) { (void)hipGetLastError(); continue; }
    KArgs A{};
    A.shots = trial;
    A.seed = 0;
    A.meas = meas;
    A.det = det;
    A.obs = obs;
    A.workspace = ws;
    hipFunction_t fn = nullptr;
    if (L.spec && spec_function(p, &fn) != CLIFFT_OK) {
      if (ws) (void)hipFree(ws);
      continue;
    }
    float ms = 0;
    for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {
      e = hipEventRecord(e0, s);
      if (e == hipSuccess) e = L.spec ? launch_spec(fn, *D, A, L.grid, s) : launch_sample(*D, A, L, fp64, false, s);
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (ws) (void)hipFree(ws);
    if (e == hipSuccess && ms < best_ms) {
      best_ms = ms;
      best = clifft_launch{precision, L.G, L.grid, L.global_vec ? 1 : -1, L.G == kBitSliced ? (L.spec ? 1 : -1) : 0};
      found = true;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (meas) (void)hipFree(meas);
  if (det) (void)hipFree(det);
  if (obs) (void)hipFree(obs);
  if (e != hipSuccess) return fail(CLIFFT_E_DEVICE, std::string("autotune failed: ") + hipGetErrorString(e));
  if (!found) return fail(CLIFFT_E_CAPACITY, "no launch shape fits this program");
  int dev = 0;
  (void)hipGetDevice(&dev);
  {
    std::lock_guard<std::mutex> lock(p->mu);
    p->tuned[{dev, precision}] = best;
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
