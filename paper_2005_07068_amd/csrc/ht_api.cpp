// Host side of the C ABI: context, validation, device copies of the model and observations,
// workspace management and kernel launches.  Every entry point validates its arguments before
// enqueuing anything and reports failures through ht_status + ht_last_error().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "handtrack.h"
#include "ht_device.h"

// Scratch of ht_eval_particles_noalloc: the evaluation workspace of one call, carved out of a
// file-scope device array (each GPU that loads the library holds its own copy until the
// process ends).  In host code `scratch` only names the symbol: its device address on each
// GPU comes from hipGetSymbolAddress with that GPU current (scratch_address below) and is the
// only form in which the array is handed to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

ht_status fail(ht_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HT_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? HT_ERR_OOM : HT_ERR_HIP, "%s: %s", #call,  \
                  hipGetErrorString(e_));                                                  \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device `dev`, looked up once per device.
hipError_t scratch_address(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

struct SlotHost {
  bool set = false;
  int W = 0, H = 0, TW = 0, TH = 0;
  size_t cap_tiles = 0, cap_px = 0;
  uint32_t* words = nullptr;
  float* tile_td = nullptr;
  int* tile_skin = nullptr;
  double* totals = nullptr;
  uint16_t* stage_depth = nullptr;
  uint8_t* stage_skin = nullptr;
  uint8_t* mask = nullptr;       // gradient pixel mask (ht_set_pixel_mask)
  size_t cap_mask = 0;
  ht::FrameSlot entry{};
};

struct GraphKey {
  ht_swarm sw;
  ht_pso_params p;
  int gens;
  bool operator<(const GraphKey& o) const { return std::memcmp(this, &o, sizeof *this) < 0; }
};

}  // namespace

struct ht_ctx {
  int device = 0;
  int n_cu = 256;
  bool has_model = false;
  int n_dof = 0, n_seg = 0, n_prim = 0;
  ht::TypeMasks tmask{};
  ht::DevModel* d_model = nullptr;
  ht::DevModel h_model{};
  ht::FrameSlot* d_slots = nullptr;
  SlotHost slots[HT_MAX_SLOTS];
  // evaluation workspace
  ht::Workspace ws{};
  int cap_particles = 0;
  int cap_items = 0;
  int cap_tiles = 0;
  bool cap_wrench = false;
  ht_launch_config lc{16, 4, 1};
  // swarm refinement scratch
  float* r_x = nullptr;       // [cap_ref][n_dof] current positions of the refined particles
  float* r_cost = nullptr;    // [cap_ref]
  float* r_grad = nullptr;    // [cap_ref][n_dof]
  float* r_cand = nullptr;    // [4 * cap_ref][n_dof]
  float* r_ccost = nullptr;   // [4 * cap_ref]
  float* r_cgrad = nullptr;   // [4 * cap_ref][n_dof] gradients of the candidates
  int* r_sel = nullptr;       // [cap_ref]
  int* r_active = nullptr;    // [cap_ref]
  int* r_slots = nullptr;     // [4 * cap_ref] frame slot of each refined particle
  int cap_ref = 0;
  int* pso_flags = nullptr;   // [cap_flags] per-particle improved / mutated flags
  int cap_flags = 0;
  int* seg_partial = nullptr; // [cap_seg] per-block minima of the preprocessing
  int cap_seg = 0;
  std::map<GraphKey, hipGraphExec_t> graphs;
  void* scratch = nullptr;    // this device's address of the no-allocation scratch array
  unsigned long long* d_eval_count = nullptr;   // [2] forward / gradient evaluations
  unsigned int* d_errors = nullptr;              // HT_DEVERR_* flags
  // tracing of eager launches
  struct ProfRec {
    int kind;
    int particles;
    hipEvent_t e0, e1;
  };
  bool prof = false;
  std::vector<ProfRec> prof_recs;

  int max_tiles() const {
    int m = 0;
    for (const auto& s : slots)
      if (s.set) m = std::max(m, s.TW * s.TH);
    return m;
  }
};

namespace {

using ht::kMinTilesPerItem;

constexpr size_t kMaxCachedGraphs = 32;

// Drop every cached graph (they hold buffers, launch shapes and sizes captured earlier); the
// device is synchronised first, so no launch of them is still running.
void invalidate_graphs(ht_ctx* c) {
  if (c->graphs.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

void free_workspace(ht_ctx* c) {
  invalidate_graphs(c);
  dfree(c->ws.recs);
  dfree(c->ws.boxes);
  dfree(c->ws.caps);
  dfree(c->ws.capr);
  dfree(c->ws.pinfo);
  dfree(c->ws.dof_frame);
  dfree(c->ws.seg_org);
  dfree(c->ws.tiles);
  dfree(c->ws.item_off);
  dfree(c->ws.item_map);
  dfree(c->ws.partial);
  dfree(c->ws.wrench);
  dfree(c->ws.counters);
  c->cap_particles = c->cap_items = c->cap_tiles = 0;
  c->cap_wrench = false;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

// Whether the workspace already holds n_total particles over observations of max_tiles tiles.
bool workspace_fits(const ht_ctx* c, int n_total, int max_tiles, bool grad) {
  const long long items =
      std::max<long long>((long long)n_total * ((max_tiles + kMinTilesPerItem - 1) / kMinTilesPerItem), 1);
  return n_total <= c->cap_particles && items <= c->cap_items && max_tiles <= c->cap_tiles &&
         (!grad || c->cap_wrench);
}

// Make sure the workspace holds n_total particles over observations of max_tiles tiles.
ht_status ensure_workspace(ht_ctx* c, int n_total, int max_tiles, bool grad, hipStream_t s) {
  const long long items_ll =
      (long long)n_total * ((max_tiles + kMinTilesPerItem - 1) / kMinTilesPerItem);
  if (items_ll > (1ll << 30)) return fail(HT_ERR_ARG, "workload too large: %lld work items", items_ll);
  const int items = (int)std::max<long long>(items_ll, 1);
  if (workspace_fits(c, n_total, max_tiles, grad)) return HT_OK;
  if (capturing(s))
    return fail(HT_ERR_STATE, "workspace too small during graph capture; call ht_reserve first");
  HT_HIP(hipDeviceSynchronize());
  const int np = std::max(n_total, c->cap_particles);
  const int nt = std::max(max_tiles, c->cap_tiles);
  const int ni = std::max<long long>(items, (long long)np * ((nt + kMinTilesPerItem - 1) / kMinTilesPerItem));
  const bool wr = grad || c->cap_wrench;
  free_workspace(c);
  auto& w = c->ws;
  HT_HIP(hipMalloc(&w.recs, (size_t)np * c->n_prim * ht::kRec * sizeof(float)));
  HT_HIP(hipMalloc(&w.boxes, (size_t)np * c->n_prim * sizeof(int4)));
  HT_HIP(hipMalloc(&w.caps, (size_t)np * c->n_prim * sizeof(float4)));
  HT_HIP(hipMalloc(&w.capr, (size_t)np * c->n_prim * sizeof(float2)));
  HT_HIP(hipMalloc(&w.pinfo, (size_t)np * sizeof(ht::PInfo)));
  HT_HIP(hipMalloc(&w.dof_frame, (size_t)np * c->n_dof * 8 * sizeof(float)));
  HT_HIP(hipMalloc(&w.seg_org, (size_t)np * c->n_seg * 4 * sizeof(float)));
  HT_HIP(hipMalloc(&w.tiles, (size_t)np * sizeof(int)));
  HT_HIP(hipMalloc(&w.item_off, (size_t)(np + 1) * sizeof(int)));
  HT_HIP(hipMalloc(&w.item_map, (size_t)ni * sizeof(int)));
  HT_HIP(hipMalloc(&w.partial, (size_t)ni * sizeof(ht::Partial)));
  if (wr) HT_HIP(hipMalloc(&w.wrench, (size_t)ni * c->n_seg * 6 * sizeof(float)));
  HT_HIP(hipMalloc(&w.counters, 4 * sizeof(int)));
  HT_HIP(hipMemset(w.counters, 0, 4 * sizeof(int)));
  w.max_items = ni;
  c->cap_tiles = nt;
  c->cap_particles = np;
  c->cap_items = ni;
  c->cap_wrench = wr;
  return HT_OK;
}

// Work items that a call over n_total particles and observations of max_tiles tiles can
// produce (items are never shorter than kMinTilesPerItem tiles).
long long item_bound(int n_total, int max_tiles) {
  return std::max<long long>(
      (long long)n_total * ((max_tiles + kMinTilesPerItem - 1) / kMinTilesPerItem), 1);
}

// Lays the forward-evaluation workspace of np particles and ni work items out from base in
// 256-byte aligned pieces (no wrench buffer) and returns the bytes it spans; base == nullptr
// computes the size only.
size_t carve_workspace(unsigned char* base, long long np, long long ni, int n_prim, int n_dof,
                       int n_seg, ht::Workspace* w) {
  size_t off = 0;
  auto take = [&](auto*& ptr, size_t bytes) {
    off = (off + 255) / 256 * 256;
    ptr = base ? reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(base + off) : nullptr;
    off += bytes;
  };
  ht::Workspace t{};
  take(t.recs, (size_t)np * n_prim * ht::kRec * sizeof(float));
  take(t.boxes, (size_t)np * n_prim * sizeof(int4));
  take(t.caps, (size_t)np * n_prim * sizeof(float4));
  take(t.capr, (size_t)np * n_prim * sizeof(float2));
  take(t.pinfo, (size_t)np * sizeof(ht::PInfo));
  take(t.dof_frame, (size_t)np * n_dof * 8 * sizeof(float));
  take(t.seg_org, (size_t)np * n_seg * 4 * sizeof(float));
  take(t.tiles, (size_t)np * sizeof(int));
  take(t.item_off, (size_t)(np + 1) * sizeof(int));
  take(t.item_map, (size_t)ni * sizeof(int));
  take(t.partial, (size_t)ni * sizeof(ht::Partial));
  take(t.counters, 4 * sizeof(int));
  t.wrench = nullptr;
  t.max_items = (int)ni;
  if (w) *w = t;
  return off;
}

// Run `launch` on stream s, bracketed by HIP events when tracing (and not capturing).
template <class F>
hipError_t traced(ht_ctx* c, int kind, int particles, hipStream_t s, F&& launch) {
  if (!c->prof || capturing(s)) return launch();
  ht_ctx::ProfRec r{kind, particles, nullptr, nullptr};
  hipError_t e = hipEventCreate(&r.e0);
  if (e == hipSuccess) e = hipEventCreate(&r.e1);
  if (e == hipSuccess) e = hipEventRecord(r.e0, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(r.e1, s);
  c->prof_recs.push_back(r);
  return e;
}

ht_status check_ctx(ht_ctx* c, bool need_model = true) {
  if (!c) return fail(HT_ERR_ARG, "context is NULL");
  if (need_model && !c->has_model) return fail(HT_ERR_STATE, "no model: call ht_set_model first");
  return HT_OK;
}

ht_status check_slots_set(ht_ctx* c) {
  for (const auto& s : c->slots)
    if (s.set) return HT_OK;
  return fail(HT_ERR_STATE, "no observation: call ht_set_observation first");
}

}  // namespace

namespace ht {

// Evaluation shared by ht_eval_particles, ht_eval_particles_grad and the swarm step.
// With src, particle r of frame f reuses the kinematics that the previous evaluation (of
// src_stride particles per frame) left for its particle src[r] of frame f: poses must equal
// those, and the kinematics stage is skipped.
// With `fixed` (forward only), that workspace is used as it is: nothing is allocated and the
// launches are not traced.
ht_status eval_impl(ht_ctx* c, int n_frames, const int32_t* frame_slots, int n_particles,
                    const float* poses, float* cost, float* grad, const uint8_t* pixel_mask,
                    const ht_debug* dbg, hipStream_t s, const int32_t* frame_stop = nullptr,
                    const int32_t* src = nullptr, int src_stride = 0,
                    const Workspace* fixed = nullptr, const int32_t* active = nullptr,
                    int active_div = 1, bool assemble = true, EvalArgs* args_out = nullptr) {
  const int n_total = n_frames * n_particles;
  if (n_total == 0) return HT_OK;
  if (!fixed) {
    // reused kinematics would not survive a reallocation of the workspace: compute them again
    if (src && !workspace_fits(c, n_total, c->max_tiles(), grad != nullptr)) src = nullptr;
    ht_status st = ensure_workspace(c, n_total, c->max_tiles(), grad != nullptr, s);
    if (st != HT_OK) return st;
  }
  const Workspace& ws = fixed ? *fixed : c->ws;
  EvalArgs a{};
  a.model = c->d_model;
  a.slots = c->d_slots;
  a.frame_slots = frame_slots;
  a.n_frames = n_frames;
  a.n_particles = n_particles;
  a.poses = poses;
  a.cost = cost;
  a.grad = grad;
  a.pixel_mask = pixel_mask;
  a.frame_stop = frame_stop;
  a.src = src;
  a.src_stride = src_stride;
  a.active = active;
  a.active_div = active_div;
  a.eval_count = c->d_eval_count;
  a.dev_errors = c->d_errors;
  if (dbg) {
    a.dbg = *dbg;
    const SlotHost& sh = c->slots[dbg->slot];
    a.dbg_W = sh.W;
    a.dbg_H = sh.H;
    a.dbg_bg = sh.entry.bg;
  }
  a.type_masks = c->tmask;
  // the work-list kernel shortens work items for launches with few tiles (tiles_per_item is
  // their maximum); never more persistent workgroups than there can be items
  a.tiles_per_item = c->lc.tiles_per_item;
  a.cull = c->lc.cull;
  const long long bound = (long long)n_total *
                          ((c->max_tiles() + kMinTilesPerItem - 1) / kMinTilesPerItem);
  const bool dbg_on = a.dbg.depth || a.dbg.hit || a.dbg.rm || a.dbg.winner || a.dbg.margin;
  const bool all_types = (c->tmask.m[HT_CONE][0] | c->tmask.m[HT_CONE][1] |
                          c->tmask.m[HT_ECYLINDER][0] | c->tmask.m[HT_ECYLINDER][1]) != 0ull;
  // launches of at most kSelfSchedMax particles without debug images build their work list
  // in the ray cast (no work-list launch)
  a.self_sched = n_total <= ht::kSelfSchedMax && !dbg_on ? 1 : 0;
  int gpc = std::min(c->lc.groups_per_cu,
                     ht::raycast_groups_per_cu(grad != nullptr, dbg_on, all_types,
                                               a.self_sched != 0));
  if (a.self_sched) gpc = std::min(gpc, ht::kSelfGroupsPerCu);
  a.grid = (int)std::max<long long>(1, std::min<long long>((long long)c->n_cu * gpc, bound));
  a.n_prim = c->n_prim;
  a.n_seg = c->n_seg;
  a.n_dof = c->n_dof;
  const int kinds[kNumStages] = {HT_K_FK, HT_K_SCHED, grad ? HT_K_RAYCAST_GRAD : HT_K_RAYCAST,
                                 HT_K_FINALIZE};
  if (args_out) *args_out = a;
  for (int stage = 0; stage < kNumStages; ++stage) {
    if (stage == kStageFk && src) continue;   // reused from the previous evaluation
    if (stage == kStageFinalize && !assemble) continue;   // assembled by the next kernel
    if (stage == kStageSched && a.self_sched) continue;   // built by the ray cast
    if (fixed)
      HT_HIP(launch_eval_stage(stage, a, ws, s));
    else
      HT_HIP(traced(c, kinds[stage], n_total, s,
                    [&] { return launch_eval_stage(stage, a, ws, s); }));
  }
  return HT_OK;
}

}  // namespace ht

extern "C" {

const char* ht_last_error(void) { return g_err.c_str(); }

const char* ht_version(void) { return "handtrack 0.1 (gfx950)"; }

ht_status ht_create(ht_ctx** out, int hip_device) {
  g_err.clear();
  if (!out) return fail(HT_ERR_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  HT_HIP(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n)
    return fail(HT_ERR_ARG, "device %d out of range (%d devices)", hip_device, n);
  DeviceGuard g(hip_device);
  hipDeviceProp_t prop;
  HT_HIP(hipGetDeviceProperties(&prop, hip_device));
  ht_ctx* c = new ht_ctx();
  c->device = hip_device;
  c->n_cu = prop.multiProcessorCount;
  hipError_t e = hipMalloc(&c->d_slots, HT_MAX_SLOTS * sizeof(ht::FrameSlot));
  if (e == hipSuccess) e = hipMemset(c->d_slots, 0, HT_MAX_SLOTS * sizeof(ht::FrameSlot));
  if (e == hipSuccess) e = hipMalloc(&c->d_model, sizeof(ht::DevModel));
  if (e == hipSuccess) e = hipMalloc(&c->d_eval_count, 2 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(c->d_eval_count, 0, 2 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(&c->d_errors, sizeof(unsigned int));
  if (e == hipSuccess) e = hipMemset(c->d_errors, 0, sizeof(unsigned int));
  if (e != hipSuccess) {
    ht_destroy(c);
    return fail(HT_ERR_OOM, "context allocation failed: %s", hipGetErrorString(e));
  }
  // the no-allocation entry point's scratch on this device (the device is current here)
  e = scratch_address(hip_device, &c->scratch);
  if (e != hipSuccess) {
    ht_destroy(c);
    return fail(HT_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  }
  *out = c;
  return HT_OK;
}

void ht_destroy(ht_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  free_workspace(c);
  for (auto& s : c->slots) {
    dfree(s.words);
    dfree(s.tile_td);
    dfree(s.tile_skin);
    dfree(s.totals);
    dfree(s.stage_depth);
    dfree(s.stage_skin);
    dfree(s.mask);
  }
  dfree(c->r_x);
  dfree(c->r_cost);
  dfree(c->r_grad);
  dfree(c->r_cand);
  dfree(c->r_ccost);
  dfree(c->r_cgrad);
  dfree(c->r_sel);
  dfree(c->r_active);
  dfree(c->r_slots);
  dfree(c->pso_flags);
  dfree(c->seg_partial);
  dfree(c->d_slots);
  dfree(c->d_model);
  dfree(c->d_eval_count);
  dfree(c->d_errors);
  delete c;
}

}  // extern "C"

namespace {

// Validate the host model tables and lay them out for the device.
ht_status build_model(const ht_model* m, ht::DevModel& d, ht::TypeMasks& tm) {
  if (!m) return fail(HT_ERR_ARG, "model is NULL");
  if (m->n_dof <= 0 || m->n_dof > HT_MAX_DOF) return fail(HT_ERR_ARG, "n_dof %d out of 1..%d", m->n_dof, HT_MAX_DOF);
  if (m->n_seg <= 0 || m->n_seg > HT_MAX_SEG) return fail(HT_ERR_ARG, "n_seg %d out of 1..%d", m->n_seg, HT_MAX_SEG);
  if (m->n_prim <= 0 || m->n_prim > HT_MAX_PRIM) return fail(HT_ERR_ARG, "n_prim %d out of 1..%d", m->n_prim, HT_MAX_PRIM);
  if (m->n_kc < 0 || m->n_kc > HT_MAX_KC) return fail(HT_ERR_ARG, "n_kc %d out of 0..%d", m->n_kc, HT_MAX_KC);
  if (!m->seg_parent || !m->seg_root_dof || !m->seg_offset || !m->seg_joint_axis ||
      !m->seg_joint_dof || !m->prim_type || !m->prim_seg || !m->prim_frame || !m->prim_size ||
      !m->bounds_lo || !m->bounds_hi || !m->mutate_mask || (m->n_kc && !m->kc_pairs))
    return fail(HT_ERR_ARG, "model table pointer is NULL");
  std::memset(&d, 0, sizeof d);
  d.n_dof = m->n_dof;
  d.n_seg = m->n_seg;
  d.n_prim = m->n_prim;
  d.n_kc = m->n_kc;
  std::vector<int> used(m->n_dof, 0);
  for (int s = 0; s < m->n_seg; ++s) {
    const int par = m->seg_parent[s];
    if (par >= s || par < -1) return fail(HT_ERR_ARG, "segment %d: parent %d must precede it", s, par);
    d.seg_parent[s] = par;
    d.seg_depth[s] = par < 0 ? 0 : d.seg_depth[par] + 1;
    d.max_depth = std::max(d.max_depth, d.seg_depth[s]);
    if (par < 0) {
      const int b = m->seg_root_dof[s];
      if (b < 0 || b + 6 > m->n_dof) return fail(HT_ERR_ARG, "segment %d: root dof %d out of range", s, b);
      d.seg_root_dof[s] = b;
      for (int i = 0; i < 6; ++i) used[b + i]++;
      for (int i = 0; i < 3; ++i) d.dof_trans[b + i] = 1;
    } else {
      d.seg_root_dof[s] = -1;
    }
    for (int i = 0; i < 12; ++i) d.seg_off[s][i] = m->seg_offset[s * 12 + i];
    for (int j = 0; j < 2; ++j) {
      const int dof = m->seg_joint_dof[s * 2 + j];
      if (dof < -1 || dof >= m->n_dof) return fail(HT_ERR_ARG, "segment %d: joint dof %d out of range", s, dof);
      d.seg_dof[s][j] = dof;
      double n2 = 0.0;
      for (int i = 0; i < 3; ++i) {
        d.seg_axis[s][j][i] = m->seg_joint_axis[(s * 2 + j) * 3 + i];
        n2 += d.seg_axis[s][j][i] * d.seg_axis[s][j][i];
      }
      if (dof >= 0) {
        if (std::fabs(n2 - 1.0) > 1e-9) return fail(HT_ERR_ARG, "segment %d: joint axis %d is not a unit vector", s, j);
        used[dof]++;
      }
    }
  }
  for (int j = 0; j < m->n_dof; ++j)
    if (used[j] > 1) return fail(HT_ERR_ARG, "pose parameter %d drives more than one joint", j);
  // kinematic trees (hands): trees beyond kMaxRects share the last tile rectangle
  std::vector<int> tree(m->n_seg, 0);
  d.n_roots = 0;
  for (int s = 0; s < m->n_seg; ++s)
    tree[s] = d.seg_parent[s] < 0 ? std::min(d.n_roots++, ht::kMaxRects - 1) : tree[d.seg_parent[s]];
  d.n_roots = std::min(d.n_roots, ht::kMaxRects);
  // segments moved by each pose parameter: the driven segment and its descendants
  for (int s = 0; s < m->n_seg; ++s) {
    for (int q = s; q >= 0; q = d.seg_parent[q]) {
      for (int j = 0; j < 2; ++j)
        if (d.seg_dof[q][j] >= 0) d.dof_desc[d.seg_dof[q][j]] |= 1u << s;
      if (d.seg_parent[q] < 0)
        for (int i = 0; i < 6; ++i) d.dof_desc[d.seg_root_dof[q] + i] |= 1u << s;
    }
  }
  tm = ht::TypeMasks{};
  for (int k = 0; k < m->n_prim; ++k) {
    const int t = m->prim_type[k], s = m->prim_seg[k];
    if (t < HT_SPHERE || t > HT_ECYLINDER) return fail(HT_ERR_ARG, "primitive %d: bad type %d", k, t);
    if (s < 0 || s >= m->n_seg) return fail(HT_ERR_ARG, "primitive %d: segment %d out of range", k, s);
    d.prim_type[k] = t;
    d.prim_seg[k] = s;
    d.prim_root[k] = tree[s];
    for (int i = 0; i < 3; ++i) {
      const double z = m->prim_size[k * 3 + i];
      d.prim_inv2[k][i] = z > 0.0 ? 1.0 / (z * z) : 0.0;
    }
    for (int i = 0; i < 12; ++i) d.prim_frame[k][i] = m->prim_frame[k * 12 + i];
    const int need = t == HT_SPHERE ? 1 : (t == HT_CYLINDER ? 2 : 3);   // sizes that must be > 0
    for (int i = 0; i < 3; ++i) {
      d.prim_size[k][i] = m->prim_size[k * 3 + i];
      if (i < need && !(d.prim_size[k][i] > 0.0)) return fail(HT_ERR_ARG, "primitive %d: size %d must be > 0", k, i);
    }
    tm.m[t][k / 64] |= 1ull << (k % 64);
  }
  {
    int n = 0;
    for (int t = HT_SPHERE; t <= HT_ECYLINDER; ++t)
      for (int k = 0; k < m->n_prim; ++k)
        if (m->prim_type[k] == t) d.prim_order[n++] = k;
  }
  for (int j = 0; j < m->n_dof; ++j) {
    if (!(m->bounds_lo[j] <= m->bounds_hi[j])) return fail(HT_ERR_ARG, "bounds of dof %d: lo > hi", j);
    d.lo[j] = (float)m->bounds_lo[j];
    d.hi[j] = (float)m->bounds_hi[j];
    d.mutate[j] = m->mutate_mask[j] ? 1 : 0;
  }
  for (int i = 0; i < m->n_kc; ++i) {
    const int a = m->kc_pairs[2 * i], b = m->kc_pairs[2 * i + 1];
    if (a < 0 || a >= m->n_dof || b < 0 || b >= m->n_dof) return fail(HT_ERR_ARG, "kc pair %d out of range", i);
    d.kc_a[i] = a;
    d.kc_b[i] = b;
  }
  return HT_OK;
}

}  // namespace

extern "C" {

ht_status ht_check_model(const ht_model* m) {
  g_err.clear();
  ht::DevModel d;
  ht::TypeMasks tm;
  return build_model(m, d, tm);
}

ht_status ht_set_model(ht_ctx* c, const ht_model* m) {
  g_err.clear();
  ht_status st = check_ctx(c, false);
  if (st != HT_OK) return st;
  ht::DevModel d;
  ht::TypeMasks tm;
  if ((st = build_model(m, d, tm)) != HT_OK) return st;
  DeviceGuard g(c->device);
  HT_HIP(hipDeviceSynchronize());
  invalidate_graphs(c);
  HT_HIP(hipMemcpy(c->d_model, &d, sizeof d, hipMemcpyHostToDevice));
  c->h_model = d;
  c->tmask = tm;
  if (c->has_model && (c->n_dof != m->n_dof || c->n_seg != m->n_seg || c->n_prim != m->n_prim)) {
    free_workspace(c);
    c->cap_ref = 0;
  }
  c->n_dof = m->n_dof;
  c->n_seg = m->n_seg;
  c->n_prim = m->n_prim;
  c->has_model = true;
  return HT_OK;
}


ht_status ht_set_observation(ht_ctx* c, int slot, int W, int H, const uint16_t* depth_mm,
                             const uint8_t* skin, ht_camera cam, float bg, int ptr_kind,
                             void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c, false);
  if (st != HT_OK) return st;
  if (slot < 0 || slot >= HT_MAX_SLOTS) return fail(HT_ERR_ARG, "frame slot %d out of 0..%d", slot, HT_MAX_SLOTS - 1);
  if (W < 1 || H < 1 || W > HT_MAX_ROI || H > HT_MAX_ROI) return fail(HT_ERR_ARG, "ROI %dx%d out of 1..%d", W, H, HT_MAX_ROI);
  if (!depth_mm || !skin) return fail(HT_ERR_ARG, "observation pointer is NULL");
  if (!(cam.fx > 0.0f) || !(cam.fy > 0.0f) || !std::isfinite(cam.cx) || !std::isfinite(cam.cy))
    return fail(HT_ERR_ARG, "camera needs fx, fy > 0 and finite cx, cy");
  if (!std::isfinite(bg)) return fail(HT_ERR_ARG, "background depth must be finite");
  if (ptr_kind != HT_PTR_HOST && ptr_kind != HT_PTR_DEVICE) return fail(HT_ERR_ARG, "bad ptr_kind %d", ptr_kind);
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  SlotHost& sh = c->slots[slot];
  const int TW = (W + ht::kTile - 1) / ht::kTile, TH = (H + ht::kTile - 1) / ht::kTile;
  const size_t n_tiles = (size_t)TW * TH, n_px = (size_t)W * H;
  // graphs captured for smaller observations would overrun their work lists
  if ((int)n_tiles > c->cap_tiles) invalidate_graphs(c);
  if (n_tiles > sh.cap_tiles) {
    HT_HIP(hipDeviceSynchronize());
    dfree(sh.words);
    dfree(sh.tile_td);
    dfree(sh.tile_skin);
    HT_HIP(hipMalloc(&sh.words, n_tiles * ht::kTilePx * sizeof(uint32_t)));
    HT_HIP(hipMalloc(&sh.tile_td, n_tiles * sizeof(float)));
    HT_HIP(hipMalloc(&sh.tile_skin, n_tiles * sizeof(int)));
    if (!sh.totals) HT_HIP(hipMalloc(&sh.totals, 2 * sizeof(double)));
    sh.cap_tiles = n_tiles;
  }
  const uint16_t* dsrc = depth_mm;
  const uint8_t* ssrc = skin;
  if (ptr_kind == HT_PTR_HOST) {
    if (n_px > sh.cap_px) {
      HT_HIP(hipDeviceSynchronize());
      dfree(sh.stage_depth);
      dfree(sh.stage_skin);
      HT_HIP(hipMalloc(&sh.stage_depth, n_px * sizeof(uint16_t)));
      HT_HIP(hipMalloc(&sh.stage_skin, n_px));
      sh.cap_px = n_px;
    }
    HT_HIP(hipMemcpyAsync(sh.stage_depth, depth_mm, n_px * sizeof(uint16_t), hipMemcpyHostToDevice, s));
    HT_HIP(hipMemcpyAsync(sh.stage_skin, skin, n_px, hipMemcpyHostToDevice, s));
    dsrc = sh.stage_depth;
    ssrc = sh.stage_skin;
  }
  HT_HIP(ht::launch_pack_observation(dsrc, ssrc, W, H, TW, TH, sh.words, sh.tile_td,
                                     sh.tile_skin, sh.totals, bg, s));
  ht::FrameSlot& e = sh.entry;
  e.W = W;
  e.H = H;
  e.TW = TW;
  e.TH = TH;
  if (cam.fx == cam.fy) {
    e.sx = 1.0f;
    e.sy = 1.0f;
    e.sz = cam.fx;
  } else {
    e.sx = cam.fy;
    e.sy = cam.fx;
    e.sz = cam.fx * cam.fy;
  }
  e.cx = cam.cx;
  e.cy = cam.cy;
  e.fx = cam.fx;
  e.fy = cam.fy;
  e.bg = bg;
  e.set = 1;
  e.words = sh.words;
  e.tile_td = sh.tile_td;
  e.tile_skin = sh.tile_skin;
  e.totals = sh.totals;
  e.grad_mask = nullptr;   // a new observation clears the slot's gradient mask
  HT_HIP(hipMemcpyAsync(&c->d_slots[slot], &e, sizeof e, hipMemcpyHostToDevice, s));
  HT_HIP(hipStreamSynchronize(s));
  sh.set = true;
  sh.W = W;
  sh.H = H;
  sh.TW = TW;
  sh.TH = TH;
  return HT_OK;
}

ht_status ht_reserve(ht_ctx* c, int max_particles, int max_pixels) {
  g_err.clear();
  ht_status st = check_ctx(c);
  if (st != HT_OK) return st;
  if (max_particles < 0 || max_pixels < 0) return fail(HT_ERR_ARG, "negative reservation");
  const int side = (int)std::ceil(std::sqrt((double)max_pixels)) + ht::kTile;
  const int tiles = std::max(c->max_tiles(), (side / ht::kTile + 1) * (side / ht::kTile + 1));
  DeviceGuard g(c->device);
  return ensure_workspace(c, std::max(max_particles, 1), tiles, true, nullptr);
}

ht_status ht_eval_particles(ht_ctx* c, int n_frames, const int32_t* frame_slots, int n_particles,
                            const float* poses, float* cost, const ht_debug* dbg, void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c);
  if (st != HT_OK) return st;
  if (n_frames < 0 || n_particles < 0) return fail(HT_ERR_ARG, "negative counts");
  if ((long long)n_frames * n_particles > (1 << 24)) return fail(HT_ERR_ARG, "too many particles");
  if (n_frames * n_particles == 0) return HT_OK;
  if (!frame_slots || !poses || !cost) return fail(HT_ERR_ARG, "NULL device pointer");
  if ((st = check_slots_set(c)) != HT_OK) return st;
  if (dbg && (dbg->depth || dbg->hit || dbg->rm || dbg->winner || dbg->margin)) {
    if (n_frames != 1) return fail(HT_ERR_UNSUPPORTED, "debug images need n_frames == 1");
    if (dbg->slot < 0 || dbg->slot >= HT_MAX_SLOTS || !c->slots[dbg->slot].set)
      return fail(HT_ERR_STATE, "debug slot %d is not set", dbg->slot);
  } else {
    dbg = nullptr;
  }
  DeviceGuard g(c->device);
  return ht::eval_impl(c, n_frames, frame_slots, n_particles, poses, cost, nullptr, nullptr, dbg,
                       (hipStream_t)stream);
}

ht_status ht_eval_particles_grad(ht_ctx* c, int n_frames, const int32_t* frame_slots,
                                 int n_particles, const float* poses, float* cost, float* grad,
                                 const uint8_t* pixel_mask, void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c);
  if (st != HT_OK) return st;
  if (n_frames < 0 || n_particles < 0) return fail(HT_ERR_ARG, "negative counts");
  if ((long long)n_frames * n_particles > (1 << 24)) return fail(HT_ERR_ARG, "too many particles");
  if (n_frames * n_particles == 0) return HT_OK;
  if (!frame_slots || !poses || !cost || !grad) return fail(HT_ERR_ARG, "NULL device pointer");
  if (pixel_mask && n_frames != 1) return fail(HT_ERR_UNSUPPORTED, "pixel_mask needs n_frames == 1");
  if ((st = check_slots_set(c)) != HT_OK) return st;
  DeviceGuard g(c->device);
  return ht::eval_impl(c, n_frames, frame_slots, n_particles, poses, cost, grad, pixel_mask,
                       nullptr, (hipStream_t)stream);
}

ht_status ht_eval_particles_noalloc(ht_ctx* c, int n_frames, const int32_t* frame_slots,
                                    int n_particles, const float* poses, float* cost,
                                    void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c);
  if (st != HT_OK) return st;
  if (n_frames < 0 || n_particles < 0) return fail(HT_ERR_ARG, "negative counts");
  if ((long long)n_frames * n_particles > (1 << 24)) return fail(HT_ERR_ARG, "too many particles");
  if (n_frames * n_particles == 0) return HT_OK;
  if (!frame_slots || !poses || !cost) return fail(HT_ERR_ARG, "NULL device pointer");
  if ((st = check_slots_set(c)) != HT_OK) return st;
  if (!c->scratch) return fail(HT_ERR_STATE, "no scratch address on device %d", c->device);
  const int n_total = n_frames * n_particles;
  const long long ni = item_bound(n_total, c->max_tiles());
  const size_t need = carve_workspace(nullptr, n_total, ni, c->n_prim, c->n_dof, c->n_seg, nullptr);
  if (need > kScratchBytes)
    return fail(HT_ERR_ARG,
                "%d particles over observations of up to %d tiles need %zu bytes of scratch; "
                "ht_eval_particles_noalloc has %zu: evaluate fewer particles per call",
                n_total, c->max_tiles(), need, kScratchBytes);
  ht::Workspace w{};
  carve_workspace(static_cast<unsigned char*>(c->scratch), n_total, ni, c->n_prim, c->n_dof,
                  c->n_seg, &w);
  DeviceGuard g(c->device);
  return ht::eval_impl(c, n_frames, frame_slots, n_particles, poses, cost, nullptr, nullptr,
                       nullptr, (hipStream_t)stream, nullptr, nullptr, 0, &w);
}

}  // extern "C"

namespace {

ht_status check_swarm(ht_ctx* c, const ht_swarm* sw) {
  if (!sw) return fail(HT_ERR_ARG, "swarm is NULL");
  if (sw->n_frames < 0 || sw->n_particles < 0) return fail(HT_ERR_ARG, "negative swarm counts");
  if (sw->n_frames > HT_MAX_SLOTS) return fail(HT_ERR_ARG, "too many frames");
  if (sw->n_particles > 4096) return fail(HT_ERR_ARG, "at most 4096 particles per frame");
  if ((long long)sw->n_frames * sw->n_particles > (1 << 22)) return fail(HT_ERR_ARG, "swarm too large");
  if (sw->n_frames * sw->n_particles == 0) return HT_OK;
  if (!sw->frame_slots || !sw->x || !sw->v || !sw->pbest_x || !sw->pbest_cost || !sw->gbest_x ||
      !sw->gbest_cost || !sw->cost || !sw->gen || !sw->init_lo || !sw->init_hi)
    return fail(HT_ERR_ARG, "swarm buffer is NULL");
  (void)c;
  return HT_OK;
}

ht_status check_params(const ht_swarm* sw, const ht_pso_params* p) {
  if (!p) return fail(HT_ERR_ARG, "params is NULL");
  if (!std::isfinite(p->w) || !std::isfinite(p->c1) || !std::isfinite(p->c2))
    return fail(HT_ERR_ARG, "w, c1, c2 must be finite");
  if (p->mutate_every < 0) return fail(HT_ERR_ARG, "mutate_every must be >= 0");
  if (!(p->mutate_frac >= 0.0f && p->mutate_frac <= 1.0f)) return fail(HT_ERR_ARG, "mutate_frac out of [0, 1]");
  if (p->refine_topk < 0 || p->refine_steps < 0) return fail(HT_ERR_ARG, "negative refinement counts");
  if (p->refine_topk > sw->n_particles) return fail(HT_ERR_ARG, "refine_topk exceeds n_particles");
  if (p->refine_topk > 0 && p->refine_steps > 0 &&
      !(p->eta_rot > 0.0f && p->eta_trans > 0.0f && std::isfinite(p->eta_rot) && std::isfinite(p->eta_trans)))
    return fail(HT_ERR_ARG, "eta_rot and eta_trans must be positive");
  if (!(p->stop_cost >= 0.0f && std::isfinite(p->stop_cost)))
    return fail(HT_ERR_ARG, "stop_cost must be finite and >= 0");
  if (p->stop_cost > 0.0f && !sw->stop_gen && sw->n_frames * sw->n_particles > 0)
    return fail(HT_ERR_ARG, "stop_cost > 0 needs the swarm's stop_gen buffer");
  return HT_OK;
}

ht_status ensure_refine(ht_ctx* c, int n_ref, hipStream_t s) {
  if (n_ref <= c->cap_ref) return HT_OK;
  if (capturing(s)) return fail(HT_ERR_STATE, "refinement buffers too small during capture");
  HT_HIP(hipDeviceSynchronize());
  invalidate_graphs(c);   // captured graphs hold the old buffers
  dfree(c->r_x);
  dfree(c->r_cost);
  dfree(c->r_grad);
  dfree(c->r_cand);
  dfree(c->r_ccost);
  dfree(c->r_cgrad);
  dfree(c->r_sel);
  dfree(c->r_active);
  const size_t D = c->n_dof;
  HT_HIP(hipMalloc(&c->r_x, (size_t)n_ref * D * sizeof(float)));
  HT_HIP(hipMalloc(&c->r_cost, (size_t)n_ref * sizeof(float)));
  HT_HIP(hipMalloc(&c->r_grad, (size_t)n_ref * D * sizeof(float)));
  HT_HIP(hipMalloc(&c->r_cand, (size_t)4 * n_ref * D * sizeof(float)));
  HT_HIP(hipMalloc(&c->r_ccost, (size_t)4 * n_ref * sizeof(float)));
  HT_HIP(hipMalloc(&c->r_cgrad, (size_t)4 * n_ref * D * sizeof(float)));
  HT_HIP(hipMalloc(&c->r_sel, (size_t)n_ref * sizeof(int)));
  HT_HIP(hipMalloc(&c->r_active, (size_t)n_ref * sizeof(int)));
  c->cap_ref = n_ref;
  return HT_OK;
}

// One generation on stream s (arguments already validated).
ht_status pso_step_impl(ht_ctx* c, const ht_swarm& sw, const ht_pso_params& p, hipStream_t s) {
  const int F = sw.n_frames, P = sw.n_particles, D = c->n_dof;
  if (F * P == 0) return HT_OK;
  ht_status st = ht::eval_impl(c, F, sw.frame_slots, P, sw.x, sw.cost, nullptr, nullptr, nullptr, s,
                               sw.stop_gen);
  if (st != HT_OK) return st;
  const int K = p.refine_topk;
  if (K > 0 && p.refine_steps > 0) {
    const int n_ref = F * K;
    if ((st = ensure_refine(c, n_ref, s)) != HT_OK) return st;
    HT_HIP(traced(c, HT_K_REFINE, n_ref, s, [&] { return ht::launch_refine_select(sw, K, D, c->r_sel, c->r_x, c->r_cost, c->r_active, s); }));
    // the gradient at the start (the selected particles' kinematics are the swarm
    // evaluation's, still in the workspace); afterwards each step's candidates are evaluated
    // with their gradients (except in the last step), so the accepted candidate brings its own.
    // No evaluation of the chain is assembled by a finalize kernel: each update kernel
    // assembles the evaluation before it (the particle's own, then its four candidates').
    ht::EvalArgs prev{};
    st = ht::eval_impl(c, F, sw.frame_slots, K, c->r_x, c->r_cost, c->r_grad, nullptr, nullptr, s,
                       sw.stop_gen, c->r_sel, P, nullptr, nullptr, 1, false, &prev);
    if (st != HT_OK) return st;
    bool prev_grad = true;
    // step s: accept the previous step's best candidate (after the first), propose four new
    // ones and evaluate them; after the last step the accept is fused with writing the
    // refined particles back into the swarm
    for (int step = 0; step <= p.refine_steps; ++step) {
      const bool accept = step > 0, propose = step < p.refine_steps;
      const bool gather = step == p.refine_steps;
      ht::RefineArgs ra{};
      ra.n_ref = n_ref;
      ra.K = K;
      ra.n_dof = D;
      ra.eta_rot = p.eta_rot;
      ra.eta_trans = p.eta_trans;
      ra.op = ht::RefineOp{accept ? 1 : 0, propose ? 1 : 0, gather ? 1 : 0};
      ra.eval_grad = prev_grad ? 1 : 0;
      ra.sw = sw;
      ra.sel = c->r_sel;
      ra.rx = c->r_x;
      ra.rcost = c->r_cost;
      ra.active = c->r_active;
      ra.cand = c->r_cand;
      ra.grad = c->r_grad;
      HT_HIP(traced(c, HT_K_REFINE, n_ref, s,
                    [&] { return ht::launch_refine_update(prev, c->ws, ra, s); }));
      if (!propose) break;
      const bool g = step + 1 < p.refine_steps;
      // the four candidates of a particle that has stopped refining are not evaluated
      st = ht::eval_impl(c, F, sw.frame_slots, 4 * K, c->r_cand, c->r_ccost,
                         g ? c->r_cgrad : nullptr, nullptr, nullptr, s, sw.stop_gen, nullptr, 0,
                         nullptr, c->r_active, 4, false, &prev);
      if (st != HT_OK) return st;
      prev_grad = g;
    }
  }
  if (F * P > c->cap_flags) {
    if (capturing(s)) return fail(HT_ERR_STATE, "swarm flags too small during capture");
    HT_HIP(hipDeviceSynchronize());
    invalidate_graphs(c);   // captured graphs hold the old buffers
    dfree(c->pso_flags);
    HT_HIP(hipMalloc(&c->pso_flags, (size_t)F * P * sizeof(int)));
    c->cap_flags = F * P;
  }
  HT_HIP(traced(c, HT_K_PSO, F * P, s,
                [&] { return ht::launch_pso_update(c->d_model, sw, p, D, c->pso_flags, s); }));
  return HT_OK;
}

}  // namespace

extern "C" {

ht_status ht_pso_init(ht_ctx* c, const ht_swarm* sw, void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c);
  if (st != HT_OK) return st;
  if ((st = check_swarm(c, sw)) != HT_OK) return st;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  HT_HIP(traced(c, HT_K_PSO, sw->n_frames * sw->n_particles, s,
                [&] { return ht::launch_pso_init(c->d_model, *sw, c->n_dof, s); }));
  return HT_OK;
}

ht_status ht_set_pixel_mask(ht_ctx* c, int slot, const uint8_t* mask, int ptr_kind,
                            void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c, false);
  if (st != HT_OK) return st;
  if (slot < 0 || slot >= HT_MAX_SLOTS) return fail(HT_ERR_ARG, "frame slot %d out of 0..%d", slot, HT_MAX_SLOTS - 1);
  if (ptr_kind != HT_PTR_HOST && ptr_kind != HT_PTR_DEVICE) return fail(HT_ERR_ARG, "bad ptr_kind %d", ptr_kind);
  SlotHost& sh = c->slots[slot];
  if (!sh.set) return fail(HT_ERR_STATE, "frame slot %d has no observation", slot);
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  ht::FrameSlot& e = sh.entry;
  if (mask) {
    const size_t n_px = (size_t)e.W * e.H;
    if (n_px > sh.cap_mask) {
      HT_HIP(hipDeviceSynchronize());
      dfree(sh.mask);
      HT_HIP(hipMalloc(&sh.mask, n_px));
      sh.cap_mask = n_px;
    }
    HT_HIP(hipMemcpyAsync(sh.mask, mask, n_px,
                          ptr_kind == HT_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                          s));
    e.grad_mask = sh.mask;
  } else {
    e.grad_mask = nullptr;
  }
  HT_HIP(hipMemcpyAsync(&c->d_slots[slot], &e, sizeof e, hipMemcpyHostToDevice, s));
  HT_HIP(hipStreamSynchronize(s));
  return HT_OK;
}

ht_status ht_preprocess_rgbd(ht_ctx* c, int W, int H, const uint8_t* rgb, const uint16_t* depth,
                             const ht_seg_params* p, uint16_t* depth_out, uint8_t* skin_out,
                             void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c, false);
  if (st != HT_OK) return st;
  if (W < 1 || H < 1 || W > HT_MAX_ROI || H > HT_MAX_ROI)
    return fail(HT_ERR_ARG, "W, H = %d, %d out of 1..%d", W, H, HT_MAX_ROI);
  if (!rgb || !depth || !p || !depth_out || !skin_out) return fail(HT_ERR_ARG, "NULL buffer");
  if (p->cb_lo > p->cb_hi || p->cr_lo > p->cr_hi || p->band_mm < 0 ||
      !(p->bg_depth_mm >= 0.0f && p->bg_depth_mm <= 65535.0f))
    return fail(HT_ERR_ARG, "bad segmentation parameters");
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  const int nb = ht::preprocess_partials(W, H);
  if (nb > c->cap_seg) {
    if (capturing(s)) return fail(HT_ERR_STATE, "preprocessing scratch too small during capture");
    HT_HIP(hipDeviceSynchronize());
    dfree(c->seg_partial);
    HT_HIP(hipMalloc(&c->seg_partial, (size_t)nb * sizeof(int)));
    c->cap_seg = nb;
  }
  HT_HIP(ht::launch_preprocess(W, H, rgb, depth, *p, c->seg_partial, depth_out, skin_out, s));
  return HT_OK;
}

ht_status ht_pso_box_around(ht_ctx* c, int n_frames, const float* center, const float* halfwidth,
                            float* lo, float* hi, void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c);
  if (st != HT_OK) return st;
  if (n_frames < 0 || n_frames > (1 << 22)) return fail(HT_ERR_ARG, "n_frames %d out of range", n_frames);
  if (n_frames == 0) return HT_OK;
  if (!center || !halfwidth || !lo || !hi) return fail(HT_ERR_ARG, "box buffer is NULL");
  DeviceGuard g(c->device);
  HT_HIP(ht::launch_box_around(c->d_model, n_frames, c->n_dof, center, halfwidth, lo, hi,
                               (hipStream_t)stream));
  return HT_OK;
}

ht_status ht_pso_step(ht_ctx* c, const ht_swarm* sw, const ht_pso_params* p, void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c);
  if (st != HT_OK) return st;
  if ((st = check_swarm(c, sw)) != HT_OK) return st;
  if ((st = check_params(sw, p)) != HT_OK) return st;
  if (sw->n_frames * sw->n_particles == 0) return HT_OK;
  if ((st = check_slots_set(c)) != HT_OK) return st;
  DeviceGuard g(c->device);
  return pso_step_impl(c, *sw, *p, (hipStream_t)stream);
}

ht_status ht_pso_run_graph(ht_ctx* c, const ht_swarm* sw, const ht_pso_params* p, int n_gen,
                           void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c);
  if (st != HT_OK) return st;
  if ((st = check_swarm(c, sw)) != HT_OK) return st;
  if ((st = check_params(sw, p)) != HT_OK) return st;
  if (n_gen < 0 || n_gen > 100000) return fail(HT_ERR_ARG, "n_generations %d out of range", n_gen);
  if (sw->n_frames * sw->n_particles == 0 || n_gen == 0) return HT_OK;
  if ((st = check_slots_set(c)) != HT_OK) return st;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  GraphKey key;
  std::memset(&key, 0, sizeof key);
  key.sw = *sw;
  key.p = *p;
  key.gens = n_gen;
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    // the cache is keyed by the whole swarm (buffers and seed): bounded, it is emptied when
    // full rather than growing with every new swarm
    if (c->graphs.size() >= kMaxCachedGraphs) invalidate_graphs(c);
    // size every buffer before capture: nothing may be allocated while capturing
    const int F = sw->n_frames, P = sw->n_particles, K = p->refine_topk;
    const bool refine = K > 0 && p->refine_steps > 0;
    const int most = std::max(F * P, refine ? F * 4 * K : 0);
    if ((st = ensure_workspace(c, most, c->max_tiles(), refine, s)) != HT_OK) return st;
    if (refine && (st = ensure_refine(c, F * K, s)) != HT_OK) return st;
    if (F * P > c->cap_flags) {
      HT_HIP(hipDeviceSynchronize());
      invalidate_graphs(c);   // captured graphs hold the old buffers
      dfree(c->pso_flags);
      HT_HIP(hipMalloc(&c->pso_flags, (size_t)F * P * sizeof(int)));
      c->cap_flags = F * P;
    }
    hipStream_t cs;
    HT_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return fail(HT_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    st = HT_OK;
    e = ht::launch_pso_init(c->d_model, *sw, c->n_dof, cs);
    if (e != hipSuccess) st = fail(HT_ERR_HIP, "init launch: %s", hipGetErrorString(e));
    for (int i = 0; i < n_gen && st == HT_OK; ++i) st = pso_step_impl(c, *sw, *p, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (st != HT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail(HT_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(HT_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    it = c->graphs.emplace(key, exec).first;
  }
  HT_HIP(hipGraphLaunch(it->second, s));
  return HT_OK;
}

ht_status ht_autotune(ht_ctx* c, int n_frames, const int32_t* frame_slots, int n_particles,
                      const float* poses, float* cost, int repeats, ht_launch_config* out,
                      void* stream) {
  g_err.clear();
  ht_status st = check_ctx(c);
  if (st != HT_OK) return st;
  if (n_frames <= 0 || n_particles <= 0 || !frame_slots || !poses || !cost || repeats < 1 || !out)
    return fail(HT_ERR_ARG, "bad autotune arguments");
  if ((st = check_slots_set(c)) != HT_OK) return st;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  if (capturing(s)) return fail(HT_ERR_STATE, "autotune cannot run during graph capture");
  const ht_launch_config saved = c->lc;
  hipEvent_t e0, e1;
  HT_HIP(hipEventCreate(&e0));
  HT_HIP(hipEventCreate(&e1));
  float best = INFINITY;
  ht_launch_config best_cfg = saved;
  // a candidate replaces the best so far only if it is faster by more than 1 %, so that
  // timing noise does not pick among near-equal shapes; culling is tried first (it is what the
  // gradient launches, which are not timed here, gain most from)
  const int tpis[] = {64, 32, 16, 8, 4};
  const int gpcs[] = {8, 4, 2, 1};
  for (int cull = 1; cull >= 0 && st == HT_OK; --cull) {
    for (int tpi : tpis) {
      for (int gpc : gpcs) {
        c->lc = ht_launch_config{tpi, gpc, cull};
        st = ht::eval_impl(c, n_frames, frame_slots, n_particles, poses, cost, nullptr, nullptr,
                           nullptr, s);
        if (st != HT_OK) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < repeats && st == HT_OK; ++r)
          st = ht::eval_impl(c, n_frames, frame_slots, n_particles, poses, cost, nullptr,
                             nullptr, nullptr, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (st == HT_OK && ms < 0.99f * best) {
          best = ms;
          best_cfg = c->lc;
        }
      }
      if (st != HT_OK) break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != HT_OK) {
    c->lc = saved;
    return st;
  }
  // captured graphs hold the launch shape they were captured with
  if (std::memcmp(&best_cfg, &saved, sizeof saved) != 0) invalidate_graphs(c);
  c->lc = best_cfg;
  *out = best_cfg;
  return HT_OK;
}

ht_status ht_profile_begin(ht_ctx* c) {
  g_err.clear();
  if (!c) return fail(HT_ERR_ARG, "context is NULL");
  DeviceGuard g(c->device);
  for (auto& r : c->prof_recs) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  c->prof_recs.clear();
  c->prof = true;
  return HT_OK;
}

ht_status ht_profile_end(ht_ctx* c, ht_kernel_stat* stats) {
  g_err.clear();
  if (!c || !stats) return fail(HT_ERR_ARG, "NULL argument");
  DeviceGuard g(c->device);
  for (int k = 0; k < HT_K_COUNT; ++k) stats[k] = ht_kernel_stat{0, 0, 0.0};
  ht_status st = HT_OK;
  for (auto& r : c->prof_recs) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(r.e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.e0, r.e1);
    if (e != hipSuccess && st == HT_OK) st = fail(HT_ERR_HIP, "event timing: %s", hipGetErrorString(e));
    stats[r.kind].launches += 1;
    stats[r.kind].particles += r.particles;
    stats[r.kind].total_ms += ms;
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  c->prof_recs.clear();
  c->prof = false;
  return st;
}

ht_status ht_eval_counts(ht_ctx* c, int64_t* forward, int64_t* gradient, int reset) {
  g_err.clear();
  if (!c || !forward || !gradient) return fail(HT_ERR_ARG, "NULL argument");
  DeviceGuard g(c->device);
  unsigned long long v[2] = {0, 0};
  HT_HIP(hipDeviceSynchronize());
  HT_HIP(hipMemcpy(v, c->d_eval_count, sizeof v, hipMemcpyDeviceToHost));
  if (reset) HT_HIP(hipMemset(c->d_eval_count, 0, sizeof v));
  *forward = (int64_t)v[0];
  *gradient = (int64_t)v[1];
  return HT_OK;
}

ht_status ht_device_errors(ht_ctx* c, uint32_t* flags, int reset) {
  g_err.clear();
  if (!c || !flags) return fail(HT_ERR_ARG, "NULL argument");
  DeviceGuard g(c->device);
  unsigned int v = 0;
  HT_HIP(hipDeviceSynchronize());
  HT_HIP(hipMemcpy(&v, c->d_errors, sizeof v, hipMemcpyDeviceToHost));
  if (reset) HT_HIP(hipMemset(c->d_errors, 0, sizeof v));
  *flags = v;
  return HT_OK;
}

ht_status ht_get_launch_config(ht_ctx* c, ht_launch_config* out) {
  g_err.clear();
  if (!c || !out) return fail(HT_ERR_ARG, "NULL argument");
  *out = c->lc;
  return HT_OK;
}

ht_status ht_set_launch_config(ht_ctx* c, const ht_launch_config* cfg) {
  g_err.clear();
  if (!c || !cfg) return fail(HT_ERR_ARG, "NULL argument");
  if (cfg->tiles_per_item < kMinTilesPerItem || cfg->tiles_per_item > 1024)
    return fail(HT_ERR_ARG, "tiles_per_item %d out of %d..1024", cfg->tiles_per_item, kMinTilesPerItem);
  if (cfg->cull != 0 && cfg->cull != 1) return fail(HT_ERR_ARG, "cull must be 0 or 1");
  if (cfg->groups_per_cu < 1 || cfg->groups_per_cu > 64)
    return fail(HT_ERR_ARG, "groups_per_cu %d out of 1..64", cfg->groups_per_cu);
  if (std::memcmp(cfg, &c->lc, sizeof c->lc) != 0) {
    // captured graphs hold the launch shape they were captured with
    DeviceGuard g(c->device);
    invalidate_graphs(c);
  }
  c->lc = *cfg;
  return HT_OK;
}

}  // extern "C"
