// api.hip -- the C ABI of libcm: validation, workspace sizing, launch planning.
//
// Read-only model parameters are copied from the caller's host array into
// kernel arguments at launch time; per-run read-write state never exists
// outside the kernels' registers (the read-only/read-write split and
// flat-array inputs/outputs of the Distill paper, Sec. 3.3).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "internal.hpp"

struct cm_handle {
  int device;
  int cu_count;
  size_t lds_per_block;
  cm_tuning tune[4][3];  // [kind][precision]
  // kernel timing: event pairs recorded around simulation kernels
  uint32_t* host_count = nullptr;  // pinned, for the unfused step loop
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t used = 0;
  // serving queue: one stream, completion event and input hand-off event per slot
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr, handoff = nullptr;
    uint64_t ticket = 0;
    bool busy = false;
  };
  std::vector<Slot> slots;
  uint64_t next_ticket = 1;
  // graph cache of cm_launch_graph: instantiated graphs keyed by the whole
  // argument set (see graph_signature), least recently used dropped first
  struct Graph {
    std::vector<uint64_t> sig;
    hipGraphExec_t exec = nullptr;
    uint64_t last = 0;
  };
  std::vector<Graph> graphs;
  uint64_t graph_clock = 0;
  hipStream_t capture = nullptr;  // the library's own stream for captures
};

static void clear_graphs(cm_handle* h) {
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
}

// The device work queue: pinned host memory the host publishes into
// (header, done words, request ring, request descriptors), device memory the
// persistent kernel claims and counts with (claim word, copy count, pull
// lock, per-slot counters, copies of the ring and descriptors), and the
// host's view of the requests in flight.
struct cm_queue {
  cm_handle* h = nullptr;
  uint32_t kind = 0, prec = 0, cap_slots = 0, cap_ring = 0, groups = 0;
  uint64_t idle_ticks = 0;
  size_t lds = 0;
  char* host = nullptr;  // pinned: [tail, stop, pad...][done][ring][desc]
  uint32_t* tail = nullptr;
  uint32_t* stop = nullptr;
  uint32_t* done = nullptr;
  cm::QueueReq* ring = nullptr;
  cm::QueueDesc* desc = nullptr;
  char* dev = nullptr;  // device: claim word, dev_tail, pull_lock, dev_stop, prep_done[cap_slots],
                        // chunk_done[cap_slots], then the ring and descriptor copies
  size_t o_dring = 0, o_ddesc = 0;
  hipStream_t run = nullptr;
  hipEvent_t run_done = nullptr;
  hipEvent_t handoff = nullptr;  // the producer stream's work before a submit
  bool launched = false;
  uint32_t published = 0;  // requests published (== *tail)
  uint64_t next_ticket = 1;
  std::vector<uint64_t> slot_prep, slot_chunks;  // pieces and chunks ever assigned to each slot
  std::vector<uint64_t> slot_ticket;  // 0: free
  hipStream_t copy = nullptr;            // result copies into host buffers
  std::vector<hipEvent_t> copied;        // per slot: the copies of its request are finished
  struct Copy {
    void* dst;
    const void* src;
    uint64_t bytes;
  };
  struct Req {
    uint64_t ticket;
    uint32_t slot, number;  // number: publication order
    bool copying;           // the device is done; the host copies are enqueued
    Copy cp[4];             // hist, stats, score, best (dst NULL: none)
  };
  std::vector<Req> reqs;  // in publication order
};

// Workspace of cm_launch_scratch: one array per device, living as long as
// the process.  In host code `scratch` names a host-side stand-in, not the
// device array: its device address comes from hipGetSymbolAddress (taken once
// per device when the first handle on it is created) and only that address
// is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[CM_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

// Device address of `scratch` per device ordinal (NULL until looked up).
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;

cm_status fail(cm_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
cm_status fail(cm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

cm_status ok() {
  g_err.clear();
  return CM_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

constexpr uint64_t kMaxChunk = 1u << 20;
constexpr size_t kWorkspaceAlign = 256;
constexpr size_t kLdsBudget = 32 * 1024;  // histogram window per workgroup

uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// Workspace layout (offsets in bytes from the workspace base).
struct Layout {
  uint64_t drive, correct, norm2, wfrag, total;
};

Layout layout(const cm_model* m, const cm_sweep* s) {
  Layout L{};
  uint64_t off = 0;
  L.correct = off;
  off = align_up(off + 16 * sizeof(int32_t), kWorkspaceAlign);
  L.drive = off;
  if (m->kind == CM_CONFLICT_LCA) off = align_up(off + s->n_settings * 9u * 2u * sizeof(double), kWorkspaceAlign);
  if (m->kind == CM_CONFLICT_LOOP) {
    const uint64_t lv = (uint64_t)m->params[CM_LOOP_LEVELS];  // validated before any layout is used
    L.norm2 = off + lv * lv * 9u * 2u * sizeof(double);  // after the drive table
    off = align_up(L.norm2 + lv * lv * sizeof(double), kWorkspaceAlign);
  }
  L.wfrag = off;
  if (m->kind == CM_RATE_RNN) {
    const uint64_t elem = m->precision == CM_FP64 ? sizeof(double) : 2u;
    off = align_up(off + (uint64_t)m->n_units * m->n_units * elem, kWorkspaceAlign);
  }
  L.total = std::max<uint64_t>(off, kWorkspaceAlign);
  return L;
}

struct UnfusedLayout {
  Layout base;
  uint64_t x, z, n, flag, choice, active, count, total;
};

UnfusedLayout unfused_layout(const cm_model* m, const cm_sweep* s) {
  UnfusedLayout U{};
  U.base = layout(m, s);
  const uint64_t runs = s->n_settings * s->trials;
  uint64_t off = U.base.total;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = off;
    off = align_up(off + bytes, kWorkspaceAlign);
    return at;
  };
  U.x = take(runs * 16u);
  U.z = take(runs * 16u);
  U.n = take(runs * 4u);
  U.flag = take(runs);
  U.choice = take(runs);
  U.active = take(runs * 8u);
  U.count = take(8u);
  U.total = off;
  return U;
}

cm_status check_model_sweep(const cm_model* m, const cm_sweep* s) {
  if (!m || !s) return fail(CM_E_INVALID, "model and sweep must not be NULL");
  if (m->abi_version != CM_ABI_VERSION)
    return fail(CM_E_INVALID, "abi_version %u, library speaks %u", m->abi_version, CM_ABI_VERSION);
  if (!m->params) return fail(CM_E_INVALID, "params must not be NULL");
  if (s->n_settings < 1 || s->n_settings >= 0xFFFFFFFFull)
    return fail(CM_E_INVALID, "n_settings must be in [1, 2^32-2]");
  if (s->trials < 1 || s->trials >= (1ull << 31)) return fail(CM_E_INVALID, "trials must be in [1, 2^31)");
  if (s->n_settings > (1ull << 62) / s->trials) return fail(CM_E_INVALID, "too many runs");
  if (s->max_steps < 1) return fail(CM_E_INVALID, "max_steps must be >= 1");
  if (s->n_bins < 1 || s->n_bins > s->max_steps) return fail(CM_E_INVALID, "n_bins must be in [1, max_steps]");
  if ((uint64_t)s->n_bins * s->max_steps >= (1ull << 32))
    return fail(CM_E_INVALID, "n_bins * max_steps must be < 2^32");
  if (!(s->flag_eps >= 0.0) || !isfinite(s->flag_eps)) return fail(CM_E_INVALID, "flag_eps must be finite and >= 0");
  if (!isfinite(s->reward) || !isfinite(s->cost)) return fail(CM_E_INVALID, "reward and cost must be finite");
  if (m->n_signals > 0 && !s->grid) return fail(CM_E_INVALID, "grid must not be NULL when n_signals > 0");
  if (s->grid && !aligned(s->grid, 8)) return fail(CM_E_INVALID, "grid must be 8-byte aligned");
  const double* p = m->params;
  switch (m->kind) {
    case CM_DDM:
      if (m->n_params < CM_DDM_NPARAM) return fail(CM_E_INVALID, "DDM needs %d params", CM_DDM_NPARAM);
      if (m->n_units != 1 || m->n_stimuli != 1 || m->n_signals > 1)
        return fail(CM_E_INVALID, "DDM: n_units 1, n_stimuli 1, n_signals 0 or 1");
      if (!(p[CM_DDM_DT] > 0) || !isfinite(p[CM_DDM_DT])) return fail(CM_E_INVALID, "dt must be > 0");
      if (!(p[CM_DDM_NOISE] >= 0) || !isfinite(p[CM_DDM_NOISE])) return fail(CM_E_INVALID, "noise must be >= 0");
      if (!(p[CM_DDM_THRESH] > 0)) return fail(CM_E_INVALID, "threshold must be > 0");
      if (!(fabs(p[CM_DDM_START]) < p[CM_DDM_THRESH])) return fail(CM_E_INVALID, "|start| must be < threshold");
      if (!isfinite(p[CM_DDM_DRIFT])) return fail(CM_E_INVALID, "drift must be finite");
      if (m->precision == CM_BF16_PROJ) return fail(CM_E_UNSUPPORTED, "bf16 projection applies to the rate network only");
      break;
    case CM_CONFLICT_LCA:
      if (m->n_params < CM_LCA_NPARAM) return fail(CM_E_INVALID, "LCA needs %d params", CM_LCA_NPARAM);
      if (m->n_units != 2 || m->n_stimuli != 9 || (m->n_signals != 0 && m->n_signals != 2))
        return fail(CM_E_INVALID, "conflict LCA: n_units 2, n_stimuli 9, n_signals 0 or 2");
      if (!m->weights || m->n_weights < 40) return fail(CM_E_INVALID, "conflict LCA needs 40 weights");
      if (!aligned(m->weights, 8)) return fail(CM_E_INVALID, "weights must be 8-byte aligned");
      if (!(p[CM_LCA_DT] > 0) || !isfinite(p[CM_LCA_DT])) return fail(CM_E_INVALID, "dt must be > 0");
      if (!(p[CM_LCA_NOISE] >= 0) || !isfinite(p[CM_LCA_NOISE])) return fail(CM_E_INVALID, "noise must be >= 0");
      if (!(p[CM_LCA_THRESH] > 0)) return fail(CM_E_INVALID, "threshold must be > 0");
      for (int i : {CM_LCA_LEAK, CM_LCA_COMP, CM_LCA_OFFSET, CM_LCA_HID_GAIN, CM_LCA_HID_BIAS})
        if (!isfinite(p[i])) return fail(CM_E_INVALID, "LCA parameter %d must be finite", i);
      if (m->precision == CM_BF16_PROJ) return fail(CM_E_UNSUPPORTED, "bf16 projection applies to the rate network only");
      break;
    case CM_RATE_RNN:
      if (m->n_params < CM_RNN_NPARAM) return fail(CM_E_INVALID, "rate network needs %d params", CM_RNN_NPARAM);
      if (m->n_units < 64 || m->n_units > 256 || m->n_units % 64 || m->n_stimuli != 1 || m->n_signals > 1)
        return fail(CM_E_INVALID, "rate network: n_units in {64,128,192,256}, n_stimuli 1, n_signals 0 or 1");
      if (!m->weights || m->n_weights < (uint64_t)m->n_units * m->n_units + 2u * m->n_units)
        return fail(CM_E_INVALID, "rate network needs n*n + 2n weights");
      if (!aligned(m->weights, 8)) return fail(CM_E_INVALID, "weights must be 8-byte aligned");
      if (!(p[CM_RNN_DT] > 0) || !isfinite(p[CM_RNN_DT])) return fail(CM_E_INVALID, "dt must be > 0");
      if (!(p[CM_RNN_NOISE] >= 0) || !isfinite(p[CM_RNN_NOISE])) return fail(CM_E_INVALID, "noise must be >= 0");
      if (!(p[CM_RNN_THRESH] > 0)) return fail(CM_E_INVALID, "threshold must be > 0");
      if (!isfinite(p[CM_RNN_INPUT_GAIN])) return fail(CM_E_INVALID, "input gain must be finite");
      if (m->precision == CM_FP32_STEP)
        return fail(CM_E_UNSUPPORTED, "rate network: use CM_FP64 or CM_BF16_PROJ");
      break;
    case CM_CONFLICT_LOOP: {
      if (m->n_params < CM_LOOP_NPARAM) return fail(CM_E_INVALID, "closed loop needs %d params", CM_LOOP_NPARAM);
      if (m->n_units != 2 || m->n_stimuli != 9 || m->n_signals > 1)
        return fail(CM_E_INVALID, "closed loop: n_units 2, n_stimuli 9, n_signals 0 or 1");
      if (!m->weights || m->n_weights < 40) return fail(CM_E_INVALID, "closed loop needs 40 weights");
      if (!aligned(m->weights, 8)) return fail(CM_E_INVALID, "weights must be 8-byte aligned");
      if (!(p[CM_LCA_DT] > 0) || !isfinite(p[CM_LCA_DT])) return fail(CM_E_INVALID, "dt must be > 0");
      if (!(p[CM_LCA_NOISE] >= 0) || !isfinite(p[CM_LCA_NOISE])) return fail(CM_E_INVALID, "noise must be >= 0");
      if (!(p[CM_LCA_THRESH] > 0)) return fail(CM_E_INVALID, "threshold must be > 0");
      for (int i : {(int)CM_LCA_LEAK, (int)CM_LCA_COMP, (int)CM_LCA_OFFSET, (int)CM_LCA_HID_GAIN,
                    (int)CM_LCA_HID_BIAS, (int)CM_LOOP_COST})
        if (!isfinite(p[i])) return fail(CM_E_INVALID, "closed-loop parameter %d must be finite", i);
      const double L = p[CM_LOOP_LEVELS], M = p[CM_LOOP_SAMPLES];
      if (!(L >= 1 && L <= 4096 && L == floor(L)) || !(M >= 1 && M <= 4096 && M == floor(M)))
        return fail(CM_E_INVALID, "levels and samples must be integers in [1, 4096]");
      if (L * L * M >= 1073741824.0) return fail(CM_E_INVALID, "levels^2 * samples must be < 2^30");
      if (!(p[CM_LOOP_AMAX] >= 0) || !isfinite(p[CM_LOOP_AMAX])) return fail(CM_E_INVALID, "A_max must be finite and >= 0");
      if (m->precision == CM_BF16_PROJ) return fail(CM_E_UNSUPPORTED, "bf16 projection applies to the rate network only");
      break;
    }
    default:
      return fail(CM_E_INVALID, "unknown kind %u", m->kind);
  }
  if (m->precision > CM_BF16_PROJ) return fail(CM_E_INVALID, "unknown precision %u", m->precision);
  return ok();
}

cm_status check_result(const cm_model* m, const cm_sweep* s, const cm_result* r) {
  if (!r || !r->hist || !r->stats) return fail(CM_E_INVALID, "hist and stats must not be NULL");
  if (!aligned(r->hist, 8) || !aligned(r->stats, 8)) return fail(CM_E_INVALID, "hist/stats must be 8-byte aligned");
  const bool scored = s->reward != 0.0 || s->cost != 0.0;
  if (scored && !r->score) return fail(CM_E_INVALID, "score must not be NULL when reward or cost is set");
  if (r->score && !aligned(r->score, 8)) return fail(CM_E_INVALID, "score must be 8-byte aligned");
  if (r->best && !scored) return fail(CM_E_INVALID, "best requires reward or cost");
  if (r->best && !aligned(r->best, 8)) return fail(CM_E_INVALID, "best must be 8-byte aligned");
  const bool any_dump = r->run_choice || r->run_step || r->run_flag || r->run_state;
  if (any_dump && !(r->run_choice && r->run_step && r->run_flag))
    return fail(CM_E_INVALID, "run_choice, run_step and run_flag are dumped together");
  if (r->run_step && !aligned(r->run_step, 4)) return fail(CM_E_INVALID, "run_step must be 4-byte aligned");
  if (r->run_state && !aligned(r->run_state, 8)) return fail(CM_E_INVALID, "run_state must be 8-byte aligned");
  (void)m;
  return ok();
}

// runs_per_lane 0 = chosen per launch from the sweep size (see plan_lane).
cm_tuning default_tuning(uint32_t kind, uint32_t prec) {
  cm_tuning t{};
  t.block = 256;
  t.runs_per_lane = 0;
  t.steps_per_sync = kind == CM_DDM ? 8 : 16;  // DDM counts step pairs
  t.tile_rows = 16;
  t.lanes_per_run = 0;  // DDM: chosen per launch (see plan_lane)
  (void)prec;
  return t;
}

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

cm_status hip_fail(hipError_t e, const char* what) {
  return fail(CM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Look up the device address of `scratch` on device `dev`, once per device;
// the device must be current.
cm_status scratch_setup(int dev, int n_devices) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr.size() < (size_t)n_devices) g_scratch_ptr.resize((size_t)n_devices, nullptr);
  if (g_scratch_ptr[(size_t)dev]) return ok();
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (!p || !aligned(p, kWorkspaceAlign)) return fail(CM_E_DEVICE, "scratch array has no aligned device address");
  g_scratch_ptr[(size_t)dev] = p;
  return ok();
}

void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (size_t)dev < g_scratch_ptr.size() ? g_scratch_ptr[(size_t)dev] : nullptr;
}

// Serving slots.  A busy slot becomes free once its completion event has fired.
cm_status refresh_slot(cm_handle::Slot& sl) {
  if (!sl.busy) return CM_OK;
  const hipError_t e = hipEventQuery(sl.done);
  if (e == hipSuccess) {
    sl.busy = false;
    return CM_OK;
  }
  if (e == hipErrorNotReady) return CM_OK;
  return hip_fail(e, "hipEventQuery");
}

void release_slots(cm_handle* h) {
  for (auto& sl : h->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.handoff) (void)hipEventDestroy(sl.handoff);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  h->slots.clear();
}

cm_status make_slots(cm_handle* h, uint32_t n) {
  release_slots(h);
  h->slots.resize(n);
  for (auto& sl : h->slots) {
    hipError_t e;
    // default priority (no priority argument), non-blocking w.r.t. the null stream
    if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.handoff, hipEventDisableTiming)) != hipSuccess) {
      release_slots(h);
      return hip_fail(e, "serving slot");
    }
  }
  return CM_OK;
}

// Events around the simulation kernel when profiling is on.
struct ProfScope {
  cm_handle* h;
  hipStream_t st;
  bool on = true;  // false: never time (creates no events)
  std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
  hipError_t begin() {
    if (!on || !h->prof) return hipSuccess;
    hipError_t e;
    if (h->used == h->events.size()) {
      std::pair<hipEvent_t, hipEvent_t> p{};
      if ((e = hipEventCreate(&p.first)) != hipSuccess) return e;
      if ((e = hipEventCreate(&p.second)) != hipSuccess) {
        (void)hipEventDestroy(p.first);
        return e;
      }
      h->events.push_back(p);
    }
    ev = &h->events[h->used++];
    return hipEventRecord(ev->first, st);
  }
  hipError_t end() { return ev ? hipEventRecord(ev->second, st) : hipSuccess; }
};

cm_status check_launch(const cm_model* m, const cm_sweep* s, const cm_result* r, void* workspace,
                       uint64_t workspace_bytes, Layout& L) {
  cm_status st = check_model_sweep(m, s);
  if (st != CM_OK) return st;
  st = check_result(m, s, r);
  if (st != CM_OK) return st;
  L = layout(m, s);
  if (!workspace || !aligned(workspace, kWorkspaceAlign))
    return fail(CM_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
  if (workspace_bytes < L.total)
    return fail(CM_E_BUDGET, "workspace has %llu bytes, needs %llu",
                (unsigned long long)workspace_bytes, (unsigned long long)L.total);
  return ok();
}

// The DDM's wavefront-per-run scan cuts a run's latency 64-fold at similar
// work per step; it wins while the sweep is too small to fill the GPU with
// lanes (measured on MI355X: 16x faster at 10^4 runs, 1.4x slower at 10^7).
bool scan_ddm(const cm_tuning& t, uint64_t runs) {
  if (t.lanes_per_run == 64) return true;
  if (t.lanes_per_run == 1) return false;
  return runs <= (1ull << 20);
}

// Time course requested with a launch: output [settings][K][6] and the
// sample spacing (every = 0: none).
struct TcSpec {
  int64_t* out = nullptr;
  uint32_t every = 0;
};

// Kernel arguments and launch shape of one lane-kernel sweep.
// launch_runs: runs of every sweep in the same launch (sets the automatic
// runs per lane, which trades GPU fill against the tail of each chunk).

// Threads per workgroup of a lane-kernel launch: the tuned block; the
// time-course variant is built for 256 only.
uint32_t lane_block(const cm_tuning& t, bool timecourse) { return timecourse ? 256u : t.block; }

cm_status plan_lane(cm_handle* h, const cm_model* m, const cm_sweep* s, const cm_result* r, char* ws,
                    const Layout& L, uint32_t scan_block, uint64_t launch_runs, const TcSpec& tc,
                    cm::SimArgs& a, uint64_t& groups, size_t& lds, uint32_t force_block = 0) {
  const bool scan = scan_block != 0;
  const cm_tuning& tune = h->tune[m->kind][m->precision];
  const uint32_t block = force_block ? force_block : lane_block(tune, tc.every != 0);
  const double* p = m->params;
  const uint64_t S = s->n_settings, T = s->trials, runs = S * T;
  const uint32_t B = s->n_bins;
  a = cm::SimArgs{};
  a.trials = T;
  a.n_settings = S;
  a.total_runs = runs;
  a.seed = s->seed;
  a.max_steps = s->max_steps;
  a.n_bins = B;
  a.trials_magic = cm::udiv_magic_for((uint32_t)T);
  a.steps_magic = cm::udiv_magic_for(s->max_steps);
  a.n_signals = m->n_signals;
  a.flag_eps = s->flag_eps;
  a.grid = s->grid;
  a.hist = r->hist;
  a.stats = r->stats;
  a.run_choice = r->run_choice;
  a.run_step = r->run_step;
  a.run_flag = r->run_flag;
  a.run_state = r->run_state;
  a.steps_per_sync = tune.steps_per_sync;
  a.correct = (const int32_t*)(ws + L.correct);
  if (m->kind == CM_DDM) {
    a.dt = p[CM_DDM_DT];
    a.drift = p[CM_DDM_DRIFT];
    a.b = p[CM_DDM_NOISE] * sqrt(p[CM_DDM_DT]);
    a.thresh = p[CM_DDM_THRESH];
    a.start = p[CM_DDM_START];
  } else {
    a.dt = p[CM_LCA_DT];
    a.leak = p[CM_LCA_LEAK];
    a.comp = p[CM_LCA_COMP];
    a.b = p[CM_LCA_NOISE] * sqrt(p[CM_LCA_DT]);
    a.thresh = p[CM_LCA_THRESH];
    a.nonneg = p[CM_LCA_NONNEG] != 0.0;
    a.drive = (const double*)(ws + L.drive);
  }
  // the FP32 steps' constants, rounded once here as the kernels would
  a.pf = cm::lca_f32(a.leak, a.comp, a.dt, a.b);
  a.bf = (float)a.b;
  a.guard_f = (float)(a.thresh - 2.0 * a.flag_eps);
  // Few runs per lane keep every SIMD busy when the launch is small (the tail
  // of long runs dominates); more runs per lane amortise the end of each
  // workgroup's chunk when the launch is large, until too few workgroups are
  // left to balance the GPU.  Measured on MI355X: 2 for ~10^5-10^6 runs, 6-8
  // for ~10^7.
  uint64_t rpl = tune.runs_per_lane;
  uint64_t chunk;
  if (scan) {
    // One wavefront per run: a workgroup of W wavefronts takes W runs per
    // round.  More runs per wavefront lengthen each wavefront's serial chain;
    // fewer mean more workgroups, each flushing its histogram window with
    // atomics into the same few global counters.  The two costs balance near
    // a chunk of 4 sqrt(runs / 600) runs (measured on MI355X with 4
    // wavefronts: 2 runs per wavefront at 2,000 runs, 4 at 10^4, 4-8 at
    // 5x10^4); 8 wavefronts per workgroup keep that chunk with half the
    // serial chain.
    const uint32_t waves = scan_block / 64u;
    if (!rpl)
      rpl = std::max<uint64_t>(
          1, std::min<uint64_t>(64, (uint64_t)llround(4.0 * sqrt((double)runs / 600.0) / waves)));
    chunk = (uint64_t)waves * rpl;
  } else {
    if (!rpl) rpl = std::max<uint64_t>(2, std::min<uint64_t>(8, launch_runs / (4096ull * h->cu_count)));
    chunk = (uint64_t)block * rpl;
  }
  chunk = std::min<uint64_t>(chunk, kMaxChunk);
  if (tc.every) {
    a.tc = tc.out;
    a.tc_every = tc.every;
    a.tc_k = s->max_steps / tc.every;
    // Runs start at the lane loop's sync points, so when the steps between
    // sync points are a multiple of the sampling interval every run of a
    // wavefront samples at the same steps and the wavefront takes the
    // sampling branch once per interval instead of at several phases of it.
    // The DDM advances in step pairs.
    const uint32_t unit = m->kind == CM_DDM ? (tc.every % 2u ? tc.every : tc.every / 2u) : tc.every;
    if (unit <= 64u) {
      const uint32_t mult = std::max<uint32_t>(1u, (a.steps_per_sync + unit / 2u) / unit);
      a.steps_per_sync = unit * std::min<uint32_t>(mult, 64u / unit);
    }
  }
  const size_t rec_bytes = 4u * (cm::rec_words(B) + (tc.every ? cm::tc_words(a.tc_k) : 0u));
  // the lane kernel also stages its drain through LDS after the window
  const size_t stage = scan ? 0 : cm::lane_stage_bytes((int)m->kind, (int)m->precision, block);
  const uint64_t wmax =
      std::min<size_t>(kLdsBudget, h->lds_per_block > stage ? h->lds_per_block - stage : 0) / rec_bytes;
  bool direct = false;
  // settings touched by one chunk: at most floor((chunk-1)/T) + 2
  if (wmax < 2 || (chunk - 1) / T + 2 > wmax) {
    const uint64_t fit = wmax >= 2 ? (wmax - 1) * T : 0;
    if (fit >= std::min<uint64_t>(chunk, block)) chunk = fit;
    else direct = true;
  }
  a.chunk = chunk;
  a.direct = direct ? 1u : 0u;
  a.window = direct ? 0 : (uint32_t)std::min<uint64_t>((chunk - 1) / T + 2, S);
  groups = (runs + chunk - 1) / chunk;
  lds = direct ? 0 : (size_t)a.window * rec_bytes;
  lds += stage;
  if (lds > h->lds_per_block) return fail(CM_E_UNSUPPORTED, "lane kernel: LDS stage too large for this block size");
  return ok();
}

// Output zero-fill and the per-sweep tables the simulation reads.
// Preparation of one sweep as item k of a batched prep launch.
void fill_prep(const cm_model* m, const cm_sweep* s, const cm_result* r, char* ws, const Layout& L,
               cm::PrepBatch& b, const TcSpec& tc = TcSpec{}) {
  cm::PrepItem& it = b.it[b.n];
  const uint64_t S = s->n_settings;
  const double* p = m->params;
  it = cm::PrepItem{};
  it.hist = r->hist;
  it.n_hist = S * 2u * s->n_bins;
  it.stats = r->stats;
  it.n_stats = S * CM_NSTAT;
  it.kind = (uint32_t)m->kind;
  if (tc.every) {
    it.extra = (uint64_t*)tc.out;
    it.n_extra = S * (uint64_t)(s->max_steps / tc.every) * cm::kTcWords;
  }
  uint64_t tables = 0;
  if (m->kind == CM_DDM) {
    it.d.correct = (int32_t*)(ws + L.correct);
    tables = 1;
  } else if (m->kind == CM_CONFLICT_LCA) {
    it.d.n_settings = S;
    it.d.n_signals = m->n_signals;
    it.d.gain = p[CM_LCA_HID_GAIN];
    it.d.bias = p[CM_LCA_HID_BIAS];
    it.d.offset = p[CM_LCA_OFFSET];
    it.d.weights = m->weights;
    it.d.grid = s->grid;
    it.d.drive = (double*)(ws + L.drive);
    it.d.correct = (int32_t*)(ws + L.correct);
    tables = 9 + S * 9u;
  } else if (m->kind == CM_CONFLICT_LOOP) {
    const uint32_t lv = (uint32_t)p[CM_LOOP_LEVELS];
    it.kind = CM_CONFLICT_LCA;  // the same tables, one drive row per allocation
    it.d.n_settings = (uint64_t)lv * lv;
    it.d.levels = lv;
    it.d.amax = p[CM_LOOP_AMAX];
    it.d.gain = p[CM_LCA_HID_GAIN];
    it.d.bias = p[CM_LCA_HID_BIAS];
    it.d.offset = p[CM_LCA_OFFSET];
    it.d.weights = m->weights;
    it.d.drive = (double*)(ws + L.drive);
    it.d.correct = (int32_t*)(ws + L.correct);
    it.d.norm2 = (double*)(ws + L.norm2);
    tables = 9 + it.d.n_settings * 9u;
  }
  it.end = (b.n ? b.it[b.n - 1].end : 0) + it.n_hist + it.n_stats + it.n_extra + tables;
  ++b.n;
}

cm_status enqueue_prep(const cm_model* m, const cm_sweep* s, const cm_result* r, char* ws, const Layout& L,
                       hipStream_t stream) {
  cm::PrepBatch b{};
  fill_prep(m, s, r, ws, L, b);
  hipError_t e = cm::launch_prep(b, stream);
  return e == hipSuccess ? ok() : hip_fail(e, "sweep preparation");
}

// Score of one sweep as the next entry of a batched score launch (unscored
// sweeps add nothing).
void fill_score(const cm_model* m, const cm_sweep* s, const cm_result* r, cm::ScoreBatch& b) {
  if (s->reward == 0.0 && s->cost == 0.0) return;
  cm::ScoreArgs& sa = b.a[b.n++];
  sa = cm::ScoreArgs{};
  sa.n_settings = s->n_settings;
  sa.trials = s->trials;
  sa.seed = s->seed;
  sa.n_signals = m->n_signals;
  sa.reward = s->reward;
  sa.cost = s->cost;
  sa.grid = s->grid;
  sa.stats = r->stats;
  sa.score = r->score;
  sa.best = r->best;
}

cm_status enqueue_score(const cm_model* m, const cm_sweep* s, const cm_result* r, hipStream_t stream) {
  cm::ScoreBatch b{};
  fill_score(m, s, r, b);
  hipError_t e = cm::launch_score(b, stream);
  return e == hipSuccess ? ok() : hip_fail(e, "score kernel");
}

cm_status launch_rnn_sweep(cm_handle* h, const cm_model* m, const cm_sweep* s, const cm_result* r,
                           char* ws, const Layout& L, hipStream_t stream, bool timed = true) {
  const double* p = m->params;
  const uint64_t S = s->n_settings, T = s->trials, runs = S * T;
  const uint32_t n = m->n_units;
  cm::RnnArgs a{};
  a.trials = T;
  a.n_settings = S;
  a.total_runs = runs;
  a.seed = s->seed;
  a.max_steps = s->max_steps;
  a.n_bins = s->n_bins;
  a.n_signals = m->n_signals;
  a.n_units = n;
  a.thresh = p[CM_RNN_THRESH];
  a.flag_eps = s->flag_eps;
  a.dt = p[CM_RNN_DT];
  a.b = p[CM_RNN_NOISE] * sqrt(p[CM_RNN_DT]);
  a.gain = p[CM_RNN_INPUT_GAIN];
  a.grid = s->grid;
  a.wfrag = ws + L.wfrag;
  a.R = m->weights + (uint64_t)n * n;
  a.hist = r->hist;
  a.stats = r->stats;
  a.run_choice = r->run_choice;
  a.run_step = r->run_step;
  a.run_flag = r->run_flag;
  a.run_state = r->run_state;
  // 16 run slots per workgroup, two workgroups per CU
  const uint64_t want = (runs + 15) / 16;
  const uint32_t groups = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, 2ull * h->cu_count));
  cm_status st = enqueue_prep(m, s, r, ws, L, stream);
  if (st != CM_OK) return st;
  hipError_t e;
  if ((e = cm::launch_rnn_prep(m->weights, n, ws + L.wfrag, m->precision != CM_FP64, stream)) != hipSuccess)
    return hip_fail(e, "weight fragments");
  ProfScope prof{h, stream, timed};
  if ((e = prof.begin()) != hipSuccess) return hip_fail(e, "hipEventRecord");
  if ((e = cm::launch_rnn(m->precision, a, groups, stream)) != hipSuccess) return hip_fail(e, "rate-network kernel");
  if ((e = prof.end()) != hipSuccess) return hip_fail(e, "hipEventRecord");
  return enqueue_score(m, s, r, stream);
}

cm_status launch_loop_sweep(cm_handle* h, const cm_model* m, const cm_sweep* s, const cm_result* r,
                            char* ws, const Layout& L, hipStream_t stream, bool timed = true) {
  const double* p = m->params;
  cm::LoopArgs a{};
  a.trials = s->trials;
  a.n_settings = s->n_settings;
  a.total_runs = s->n_settings * s->trials;
  a.seed = s->seed;
  a.max_steps = s->max_steps;
  a.n_bins = s->n_bins;
  a.steps_magic = cm::udiv_magic_for(s->max_steps);
  a.n_signals = m->n_signals;
  a.L = (uint32_t)p[CM_LOOP_LEVELS];
  a.J = a.L * a.L;
  a.M = (uint32_t)p[CM_LOOP_SAMPLES];
  a.nonneg = p[CM_LCA_NONNEG] != 0.0;
  a.thresh = p[CM_LCA_THRESH];
  a.flag_eps = s->flag_eps;
  a.dt = p[CM_LCA_DT];
  a.b = p[CM_LCA_NOISE] * sqrt(p[CM_LCA_DT]);
  a.leak = p[CM_LCA_LEAK];
  a.comp = p[CM_LCA_COMP];
  a.cost = p[CM_LOOP_COST];
  a.grid = s->grid;
  a.drive = (const double*)(ws + L.drive);
  a.norm2 = (const double*)(ws + L.norm2);
  a.correct = (const int32_t*)(ws + L.correct);
  a.hist = r->hist;
  a.stats = r->stats;
  a.run_choice = r->run_choice;
  a.run_step = r->run_step;
  a.run_flag = r->run_flag;
  a.run_state = r->run_state;
  cm_status st = enqueue_prep(m, s, r, ws, L, stream);
  if (st != CM_OK) return st;
  const uint32_t team = cm::loop_team_lanes(a.J, a.total_runs, (uint32_t)h->cu_count);
  const uint64_t teams_per_block = 256u / team;
  const uint64_t want = (a.total_runs + teams_per_block - 1) / teams_per_block;
  // Teams take runs in a fixed stride, so a workgroup's work varies with its
  // runs' lengths; with several rounds of workgroups the dispatcher refills
  // freed slots and evens that out (measured on MI355X: wavefront teams 10 %
  // faster at 32 workgroups per CU than at 8, one run per team slower;
  // workgroup teams best at 8)
  const uint64_t per_cu = team == 256u ? 8u : 32u;
  const uint32_t blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, per_cu * h->cu_count));
  hipError_t e;
  ProfScope prof{h, stream, timed};
  if ((e = prof.begin()) != hipSuccess) return hip_fail(e, "hipEventRecord");
  if ((e = cm::launch_loop(m->precision, a, team, blocks, stream)) != hipSuccess)
    return hip_fail(e, "closed-loop kernel");
  if ((e = prof.end()) != hipSuccess) return hip_fail(e, "hipEventRecord");
  return enqueue_score(m, s, r, stream);
}

// One launch of the lane kernel over the sweeps idx[0..n) (same kind and precision).
cm_status launch_lane_group(cm_handle* h, uint32_t kind, uint32_t prec, const cm_model* ms, const cm_sweep* ss,
                            const cm_result* rs, void* const* wss, const Layout* Ls, const uint32_t* idx,
                            uint32_t n, hipStream_t stream, const TcSpec& tc = TcSpec{},
                            bool timed = true) {
  // one form per launch: the DDM scan form when the sweeps of the group are
  // small (cm_launch_batch groups DDM sweeps by form; the time course needs
  // the lane form)
  bool scan = kind == CM_DDM && !tc.every;
  for (uint32_t k = 0; k < n && scan; ++k) {
    const uint32_t i = idx[k];
    scan = scan_ddm(h->tune[kind][prec], ss[i].n_settings * ss[i].trials);
  }
  uint64_t launch_runs = 0;
  for (uint32_t k = 0; k < n; ++k) launch_runs += ss[idx[k]].n_settings * ss[idx[k]].trials;
  // the scan form: 8 wavefronts per workgroup while the launch is small (more
  // wavefronts in flight for the same number of histogram flushes; measured
  // on MI355X: 10-12 % faster at 10^4 runs, even at 10^5, slower at 10^6)
  const uint32_t scan_block = scan ? (launch_runs <= (1ull << 17) ? 512u : 256u) : 0u;
  cm::LaneBatch b{};
  b.n = n;
  size_t lds = 0;
  uint64_t base = 0;
  for (uint32_t k = 0; k < n; ++k) {
    const uint32_t i = idx[k];
    uint64_t groups = 0;
    size_t l = 0;
    cm_status st =
        plan_lane(h, &ms[i], &ss[i], &rs[i], (char*)wss[i], Ls[i], scan_block, launch_runs, tc, b.a[k], groups, l);
    if (st != CM_OK) return st;
    // the launch's last tail_sweeps sweeps: chunks of half the runs, so
    // that the last workgroups of the launch end closer together (the
    // window of the smaller chunk is no wider, so the LDS plan holds)
    const cm_tuning& tu = h->tune[kind][prec];
    if (!scan && !tc.every && k + tu.tail_sweeps >= n && !b.a[k].direct && b.a[k].chunk >= 2u) {
      cm::SimArgs& sa = b.a[k];
      const uint64_t runs = ss[i].n_settings * ss[i].trials;
      sa.chunk = (sa.chunk + 1u) / 2u;
      sa.window = (uint32_t)std::min<uint64_t>((sa.chunk - 1u) / sa.trials + 2u, sa.n_settings);
      groups = (runs + sa.chunk - 1u) / sa.chunk;
    }
    b.base[k] = base;
    base += groups;
    lds = std::max(lds, l);
  }
  b.base[n] = base;
  if (base > 0x7FFFFFFFull) return fail(CM_E_INVALID, "batch too large for one launch");
  cm::PrepBatch pb{};
  cm::ScoreBatch sb{};
  for (uint32_t k = 0; k < n; ++k) {
    const uint32_t i = idx[k];
    fill_prep(&ms[i], &ss[i], &rs[i], (char*)wss[i], Ls[i], pb, tc);
    fill_score(&ms[i], &ss[i], &rs[i], sb);
  }
  hipError_t e;
  if ((e = cm::launch_prep(pb, stream)) != hipSuccess) return hip_fail(e, "sweep preparation");
  ProfScope prof{h, stream, timed};
  if ((e = prof.begin()) != hipSuccess) return hip_fail(e, "hipEventRecord");
  if ((e = cm::launch_sim_lane((int)kind, (int)prec, scan_block, tc.every != 0,
                               h->tune[kind][prec].waves_per_simd,
                               lane_block(h->tune[kind][prec], tc.every != 0), b, lds, stream)) != hipSuccess)
    return hip_fail(e, "simulation kernel");
  if ((e = prof.end()) != hipSuccess) return hip_fail(e, "hipEventRecord");
  if ((e = cm::launch_score(sb, stream)) != hipSuccess) return hip_fail(e, "score kernel");
  return ok();
}

}  // namespace

extern "C" {

const char* cm_last_error(void) { return g_err.c_str(); }

cm_status cm_validate(const cm_model* model, const cm_sweep* sweep) {
  return check_model_sweep(model, sweep);
}

cm_status cm_workspace_bytes(const cm_model* model, const cm_sweep* sweep, uint64_t* bytes) {
  if (!bytes) return fail(CM_E_INVALID, "bytes must not be NULL");
  cm_status st = check_model_sweep(model, sweep);
  if (st != CM_OK) return st;
  *bytes = layout(model, sweep).total;
  return ok();
}

cm_status cm_create(int device_ordinal, cm_handle** out) {
  if (!out) return fail(CM_E_INVALID, "out must not be NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device_ordinal < 0 || device_ordinal >= n)
    return fail(CM_E_INVALID, "device %d out of range (%d devices)", device_ordinal, n);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device_ordinal);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  {
    DeviceGuard guard(device_ordinal);
    cm_status st = scratch_setup(device_ordinal, n);
    if (st != CM_OK) return st;
  }
  cm_handle* h = new (std::nothrow) cm_handle();
  if (!h) return fail(CM_E_DEVICE, "out of host memory");
  h->device = device_ordinal;
  h->cu_count = prop.multiProcessorCount;
  h->lds_per_block = prop.sharedMemPerBlock;
  for (uint32_t k = 0; k < 4; ++k)
    for (uint32_t p = 0; p < 3; ++p) h->tune[k][p] = default_tuning(k, p);
  *out = h;
  return ok();
}

cm_status cm_destroy(cm_handle* h) {
  if (h) {
    DeviceGuard guard(h->device);
    release_slots(h);
    clear_graphs(h);
    if (h->capture) (void)hipStreamDestroy(h->capture);
  }
  if (h && h->host_count) (void)hipHostFree(h->host_count);
  if (h) {
    for (auto& ev : h->events) {
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
  }
  delete h;
  return ok();
}

cm_status cm_serve_config(cm_handle* h, uint32_t n_slots) {
  if (!h) return fail(CM_E_INVALID, "handle must not be NULL");
  if (n_slots < 1 || n_slots > 64) return fail(CM_E_INVALID, "n_slots must be in [1, 64]");
  DeviceGuard guard(h->device);
  for (auto& sl : h->slots) {
    cm_status st = refresh_slot(sl);
    if (st != CM_OK) return st;
    if (sl.busy) return fail(CM_E_BUSY, "a slot still holds unfinished work");
  }
  return make_slots(h, n_slots);
}

cm_status cm_submit(cm_handle* h, uint32_t n, const cm_model* models, const cm_sweep* sweeps,
                    const cm_result* results, void* const* workspaces, const uint64_t* workspace_bytes,
                    const cm_host_result* host, void* producer_stream, uint64_t* ticket) {
  if (!h || !ticket) return fail(CM_E_INVALID, "handle and ticket must not be NULL");
  if (n < 1 || !models || !sweeps || !results || !workspaces || !workspace_bytes)
    return fail(CM_E_INVALID, "batch needs n >= 1 and non-NULL arrays");
  // validate everything before touching a slot: no partial enqueue
  for (uint32_t i = 0; i < n; ++i) {
    Layout L;
    cm_status st = check_launch(&models[i], &sweeps[i], &results[i], workspaces[i], workspace_bytes[i], L);
    if (st != CM_OK) {
      if (n > 1) g_err = "batch entry " + std::to_string(i) + ": " + g_err;
      return st;
    }
  }
  DeviceGuard guard(h->device);
  if (h->slots.empty()) {
    cm_status st = make_slots(h, 4);
    if (st != CM_OK) return st;
  }
  cm_handle::Slot* slot = nullptr;
  for (auto& sl : h->slots) {
    cm_status st = refresh_slot(sl);
    if (st != CM_OK) return st;
    if (!sl.busy) {
      slot = &sl;
      break;
    }
  }
  if (!slot) return fail(CM_E_BUSY, "all %zu slots hold unfinished work", h->slots.size());
  hipError_t e;
  if (producer_stream) {
    if ((e = hipEventRecord(slot->handoff, (hipStream_t)producer_stream)) != hipSuccess)
      return hip_fail(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(slot->stream, slot->handoff, 0)) != hipSuccess)
      return hip_fail(e, "hipStreamWaitEvent");
  }
  cm_status st = cm_launch_batch(h, n, models, sweeps, results, workspaces, workspace_bytes, slot->stream);
  if (st != CM_OK) return st;
  if (host) {
    for (uint32_t i = 0; i < n; ++i) {
      const uint64_t S = sweeps[i].n_settings;
      const struct {
        void* dst;
        const void* src;
        uint64_t bytes;
      } cp[4] = {{host[i].hist, results[i].hist, S * 2u * sweeps[i].n_bins * 8u},
                 {host[i].stats, results[i].stats, S * CM_NSTAT * 8u},
                 {host[i].score, results[i].score, S * 8u},
                 {host[i].best, results[i].best, 16u}};
      for (const auto& c : cp) {
        if (!c.dst || !c.src) continue;
        if ((e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToHost, slot->stream)) != hipSuccess)
          return hip_fail(e, "result copy");
      }
    }
  }
  if ((e = hipEventRecord(slot->done, slot->stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  slot->ticket = h->next_ticket++;
  slot->busy = true;
  *ticket = slot->ticket;
  return ok();
}

cm_status cm_poll(cm_handle* h, uint64_t ticket, int* done) {
  if (!h || !done) return fail(CM_E_INVALID, "handle and done must not be NULL");
  if (ticket == 0 || ticket >= h->next_ticket) return fail(CM_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  DeviceGuard guard(h->device);
  *done = 1;  // a ticket no slot holds any more has finished (slots are reused only when done)
  for (auto& sl : h->slots) {
    if (sl.ticket != ticket) continue;
    cm_status st = refresh_slot(sl);
    if (st != CM_OK) return st;
    *done = sl.busy ? 0 : 1;
  }
  return ok();
}

cm_status cm_profile(cm_handle* h, int enable) {
  if (!h) return fail(CM_E_INVALID, "handle must not be NULL");
  h->prof = enable != 0;
  h->used = 0;
  return ok();
}

cm_status cm_profile_read(cm_handle* h, double* sim_ms, uint64_t* launches) {
  if (!h || !sim_ms || !launches) return fail(CM_E_INVALID, "NULL argument");
  double total = 0.0;
  for (size_t i = 0; i < h->used; ++i) {
    hipError_t e = hipEventSynchronize(h->events[i].second);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, h->events[i].first, h->events[i].second);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    total += ms;
  }
  *sim_ms = total;
  *launches = h->used;
  return ok();
}

cm_status cm_set_tuning(cm_handle* h, uint32_t kind, uint32_t precision, const cm_tuning* t) {
  if (!h || !t || kind > 3 || precision > 2) return fail(CM_E_INVALID, "bad tuning arguments");
  cm_tuning v = *t;
  const cm_tuning d = default_tuning(kind, precision);
  if (!v.block) v.block = d.block;
  if (!v.steps_per_sync) v.steps_per_sync = d.steps_per_sync;
  if (!v.tile_rows) v.tile_rows = d.tile_rows;
  if (v.lanes_per_run != 0 && v.lanes_per_run != 1 && !(kind == CM_DDM && v.lanes_per_run == 64))
    return fail(CM_E_INVALID, "lanes_per_run must be 0, 1 (or 64 for the DDM)");
  if (v.block != 256 && !((kind == CM_DDM || kind == CM_CONFLICT_LCA) && (v.block == 512 || v.block == 1024)))
    return fail(CM_E_UNSUPPORTED, "block must be 256, or 512 or 1024 for the DDM and conflict-LCA lane kernels");
  if (v.runs_per_lane > 4096) return fail(CM_E_INVALID, "runs_per_lane must be <= 4096");
  if (v.steps_per_sync < 1 || v.steps_per_sync > 64) return fail(CM_E_INVALID, "steps_per_sync must be in [1, 64]");
  if (v.tile_rows != 16) return fail(CM_E_UNSUPPORTED, "tile_rows must be 16");
  if (v.waves_per_simd != 0 && v.waves_per_simd != 4 && v.waves_per_simd != 8)
    return fail(CM_E_UNSUPPORTED, "waves_per_simd must be 0, 4 or 8");
  if (v.waves_per_simd && kind != CM_DDM && kind != CM_CONFLICT_LCA)
    return fail(CM_E_UNSUPPORTED, "waves_per_simd applies to the DDM and conflict-LCA lane kernels");
  if (v.tail_sweeps > cm::kMaxBatch) return fail(CM_E_INVALID, "tail_sweeps must be <= %u", cm::kMaxBatch);
  if (v.tail_sweeps && kind != CM_DDM && kind != CM_CONFLICT_LCA)
    return fail(CM_E_UNSUPPORTED, "tail_sweeps applies to the DDM and conflict-LCA lane kernels");
  h->tune[kind][precision] = v;
  return ok();
}

cm_status cm_get_tuning(cm_handle* h, uint32_t kind, uint32_t precision, cm_tuning* t) {
  if (!h || !t || kind > 3 || precision > 2) return fail(CM_E_INVALID, "bad tuning arguments");
  *t = h->tune[kind][precision];
  return ok();
}

cm_status cm_launch(cm_handle* h, const cm_model* m, const cm_sweep* s, const cm_result* r,
                    void* workspace, uint64_t workspace_bytes, void* hip_stream) {
  return cm_launch_batch(h, 1, m, s, r, &workspace, &workspace_bytes, hip_stream);
}

// cm_launch over the device's scratch array: the same kernels on one sweep,
// with no allocation of any kind on the way (no vectors, no events).
cm_status cm_launch_scratch(cm_handle* h, const cm_model* m, const cm_sweep* s, const cm_result* r,
                            void* hip_stream) {
  if (!h) return fail(CM_E_INVALID, "handle must not be NULL");
  cm_status st = check_model_sweep(m, s);
  if (st != CM_OK) return st;
  const uint64_t need = layout(m, s).total;
  if (need > CM_SCRATCH_BYTES)
    return fail(CM_E_BUDGET, "sweep needs %llu workspace bytes, the scratch array holds %llu",
                (unsigned long long)need, (unsigned long long)CM_SCRATCH_BYTES);
  void* ws = scratch_ptr(h->device);
  if (!ws) return fail(CM_E_DEVICE, "no scratch address for device %d", h->device);
  Layout L;
  st = check_launch(m, s, r, ws, CM_SCRATCH_BYTES, L);
  if (st != CM_OK) return st;
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceGuard guard(h->device);
  if (m->kind == CM_RATE_RNN) return launch_rnn_sweep(h, m, s, r, (char*)ws, L, stream, false);
  if (m->kind == CM_CONFLICT_LOOP) return launch_loop_sweep(h, m, s, r, (char*)ws, L, stream, false);
  const uint32_t idx = 0;
  return launch_lane_group(h, m->kind, m->precision, m, s, r, &ws, &L, &idx, 1, stream, TcSpec{}, false);
}

cm_status cm_launch_timecourse(cm_handle* h, const cm_model* m, const cm_sweep* s, const cm_result* r,
                               uint32_t every, int64_t* timecourse, void* workspace,
                               uint64_t workspace_bytes, void* hip_stream) {
  if (!h) return fail(CM_E_INVALID, "handle must not be NULL");
  Layout L;
  cm_status st = check_launch(m, s, r, workspace, workspace_bytes, L);
  if (st != CM_OK) return st;
  if (m->kind != CM_DDM && m->kind != CM_CONFLICT_LCA)
    return fail(CM_E_UNSUPPORTED, "the time course covers the DDM and the conflict LCA");
  if (every < 1 || every > s->max_steps) return fail(CM_E_INVALID, "every must be in [1, max_steps]");
  if (!timecourse || !aligned(timecourse, 8)) return fail(CM_E_INVALID, "timecourse must be non-NULL and 8-byte aligned");
  DeviceGuard guard(h->device);
  const uint32_t idx = 0;
  TcSpec tc;
  tc.out = timecourse;
  tc.every = every;
  return launch_lane_group(h, (uint32_t)m->kind, (uint32_t)m->precision, m, s, r, &workspace, &L, &idx, 1,
                           (hipStream_t)hip_stream, tc);
}

cm_status cm_ceiling(cm_handle* h, const cm_model* m, uint32_t steps, uint64_t lanes, double* out,
                     void* hip_stream) {
  if (!h || !m || !out) return fail(CM_E_INVALID, "handle, model and out must not be NULL");
  if (m->abi_version != CM_ABI_VERSION) return fail(CM_E_INVALID, "abi_version mismatch");
  if (m->kind != CM_DDM && m->kind != CM_CONFLICT_LCA)
    return fail(CM_E_UNSUPPORTED, "the ceiling kernel covers the DDM and the conflict LCA");
  if (m->precision != CM_FP64 && m->precision != CM_FP32_STEP)
    return fail(CM_E_UNSUPPORTED, "precision must be CM_FP64 or CM_FP32_STEP");
  const uint32_t need = m->kind == CM_DDM ? CM_DDM_NPARAM : CM_LCA_NPARAM;
  if (!m->params || m->n_params < need) return fail(CM_E_INVALID, "params missing");
  if (steps < 1 || steps > 1000000) return fail(CM_E_INVALID, "steps must be in [1, 10^6]");
  if (lanes < 256 || lanes % 256 || lanes > (1ull << 32))
    return fail(CM_E_INVALID, "lanes must be a multiple of 256 in [256, 2^32]");
  if (!aligned(out, 8)) return fail(CM_E_INVALID, "out must be 8-byte aligned");
  const double* p = m->params;
  cm::SimArgs a{};
  a.seed = 1;
  if (m->kind == CM_DDM) {
    a.dt = p[CM_DDM_DT];
    a.drift = p[CM_DDM_DRIFT];
    a.b = p[CM_DDM_NOISE] * sqrt(p[CM_DDM_DT]);
    a.start = p[CM_DDM_START];
  } else {
    a.dt = p[CM_LCA_DT];
    a.leak = p[CM_LCA_LEAK];
    a.comp = p[CM_LCA_COMP];
    a.b = p[CM_LCA_NOISE] * sqrt(p[CM_LCA_DT]);
  }
  a.pf = cm::lca_f32(a.leak, a.comp, a.dt, a.b);
  a.bf = (float)a.b;
  DeviceGuard guard(h->device);
  const hipError_t e = cm::launch_ceiling((int)m->kind, (int)m->precision, a, steps, lanes, out,
                                          (hipStream_t)hip_stream);
  return e == hipSuccess ? ok() : hip_fail(e, "ceiling kernel");
}

}  // extern "C"

namespace {

cm_status check_batch(uint32_t n, const cm_model* models, const cm_sweep* sweeps, const cm_result* results,
                      void* const* workspaces, const uint64_t* workspace_bytes, std::vector<Layout>& L) {
  if (n < 1 || !models || !sweeps || !results || !workspaces || !workspace_bytes)
    return fail(CM_E_INVALID, "batch needs n >= 1 and non-NULL arrays");
  L.assign(n, Layout{});
  for (uint32_t i = 0; i < n; ++i) {
    cm_status st = check_launch(&models[i], &sweeps[i], &results[i], workspaces[i], workspace_bytes[i], L[i]);
    if (st != CM_OK) {
      if (n > 1) g_err = "batch entry " + std::to_string(i) + ": " + g_err;
      return st;
    }
  }
  return ok();
}

// The launches of a checked batch, enqueued on `stream` (current device set).
cm_status enqueue_batch(cm_handle* h, uint32_t n, const cm_model* models, const cm_sweep* sweeps,
                        const cm_result* results, void* const* workspaces, const std::vector<Layout>& L,
                        hipStream_t stream) {
  // rate-network sweeps launch one by one; lane-kernel sweeps of one kind and
  // precision share launches of up to kMaxBatch sweeps
  std::vector<uint32_t> group;
  for (uint32_t kind = 0; kind < 4; ++kind)
    for (uint32_t prec = 0; prec < 3; ++prec) {
      group.clear();
      for (uint32_t i = 0; i < n; ++i)
        if (models[i].kind == kind && models[i].precision == prec) group.push_back(i);
      if (group.empty()) continue;
      if (kind == CM_RATE_RNN || kind == CM_CONFLICT_LOOP) {
        for (uint32_t i : group) {
          cm_status st = kind == CM_RATE_RNN
                             ? launch_rnn_sweep(h, &models[i], &sweeps[i], &results[i], (char*)workspaces[i], L[i], stream)
                             : launch_loop_sweep(h, &models[i], &sweeps[i], &results[i], (char*)workspaces[i], L[i], stream);
          if (st != CM_OK) return st;
        }
        continue;
      }
      // A DDM sweep runs in the scan form or the lane form by its own size
      // alone (the two sum a run's increments in different orders), so the
      // group splits by form: a sweep's states never depend on what it is
      // batched with.
      for (int form = 0; form < 2; ++form) {
        std::vector<uint32_t> sub;
        for (uint32_t i : group) {
          const bool scan = kind == CM_DDM && scan_ddm(h->tune[kind][prec], sweeps[i].n_settings * sweeps[i].trials);
          if ((int)scan == form) sub.push_back(i);
        }
        for (size_t g0 = 0; g0 < sub.size(); g0 += cm::kMaxBatch) {
          const size_t g1 = std::min(sub.size(), g0 + (size_t)cm::kMaxBatch);
          cm_status st = launch_lane_group(h, kind, prec, models, sweeps, results, workspaces, L.data(),
                                           sub.data() + g0, (uint32_t)(g1 - g0), stream);
          if (st != CM_OK) return st;
        }
      }
    }
  return ok();
}

// Everything a batched launch reads on the host: every field of every entry
// (pointers as addresses), the parameter values behind `params`, the
// handle's tuning and its device.  Two calls with equal signatures enqueue
// the same kernels with the same arguments.
std::vector<uint64_t> graph_signature(const cm_handle* h, uint32_t n, const cm_model* models,
                                      const cm_sweep* sweeps, const cm_result* results,
                                      void* const* workspaces, const uint64_t* workspace_bytes) {
  std::vector<uint64_t> v;
  auto put = [&](uint64_t x) { v.push_back(x); };
  auto putd = [&](double x) {
    uint64_t u;
    memcpy(&u, &x, sizeof u);
    v.push_back(u);
  };
  put((uint64_t)h->device);
  for (uint32_t k = 0; k < 4; ++k)
    for (uint32_t p = 0; p < 3; ++p) {
      const cm_tuning& t = h->tune[k][p];
      put(((uint64_t)t.block << 32) | t.runs_per_lane);
      put(((uint64_t)t.steps_per_sync << 32) | t.tile_rows);
      put(((uint64_t)t.lanes_per_run << 32) | t.waves_per_simd);
      put(t.tail_sweeps);
    }
  put(n);
  for (uint32_t i = 0; i < n; ++i) {
    const cm_model& m = models[i];
    put(((uint64_t)m.abi_version << 32) | m.kind);
    put(((uint64_t)m.precision << 32) | m.n_units);
    put(((uint64_t)m.n_stimuli << 32) | m.n_signals);
    put(m.n_params);
    for (uint32_t k = 0; k < m.n_params; ++k) putd(m.params[k]);
    put((uint64_t)(uintptr_t)m.weights);
    put(m.n_weights);
    const cm_sweep& sw = sweeps[i];
    put((uint64_t)(uintptr_t)sw.grid);
    put(sw.n_settings);
    put(sw.trials);
    put(sw.seed);
    put(((uint64_t)sw.max_steps << 32) | sw.n_bins);
    putd(sw.reward);
    putd(sw.cost);
    putd(sw.flag_eps);
    const cm_result& r = results[i];
    for (const void* q : {(const void*)r.hist, (const void*)r.stats, (const void*)r.score, (const void*)r.best,
                          (const void*)r.run_choice, (const void*)r.run_step, (const void*)r.run_flag,
                          (const void*)r.run_state})
      put((uint64_t)(uintptr_t)q);
    put((uint64_t)(uintptr_t)workspaces[i]);
    put(workspace_bytes[i]);
  }
  return v;
}

}  // namespace

extern "C" {

cm_status cm_launch_batch(cm_handle* h, uint32_t n, const cm_model* models, const cm_sweep* sweeps,
                          const cm_result* results, void* const* workspaces,
                          const uint64_t* workspace_bytes, void* hip_stream) {
  if (!h) return fail(CM_E_INVALID, "handle must not be NULL");
  std::vector<Layout> L;
  cm_status st = check_batch(n, models, sweeps, results, workspaces, workspace_bytes, L);
  if (st != CM_OK) return st;
  DeviceGuard guard(h->device);
  return enqueue_batch(h, n, models, sweeps, results, workspaces, L, (hipStream_t)hip_stream);
}

cm_status cm_launch_graph(cm_handle* h, uint32_t n, const cm_model* models, const cm_sweep* sweeps,
                          const cm_result* results, void* const* workspaces,
                          const uint64_t* workspace_bytes, void* hip_stream) {
  if (!h) return fail(CM_E_INVALID, "handle must not be NULL");
  std::vector<Layout> L;
  cm_status st = check_batch(n, models, sweeps, results, workspaces, workspace_bytes, L);
  if (st != CM_OK) return st;
  DeviceGuard guard(h->device);
  hipStream_t stream = (hipStream_t)hip_stream;
  std::vector<uint64_t> sig = graph_signature(h, n, models, sweeps, results, workspaces, workspace_bytes);
  hipError_t e;
  for (auto& g : h->graphs)
    if (g.sig == sig) {
      g.last = ++h->graph_clock;
      if ((e = hipGraphLaunch(g.exec, stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
      return ok();
    }
  // capture the batch's launches on the library's own stream (untimed: no
  // events enter the graph) and keep the instantiated graph
  if (!h->capture && (e = hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(e, "hipStreamCreateWithFlags");
  if ((e = hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return hip_fail(e, "hipStreamBeginCapture");
  const bool prof = h->prof;
  h->prof = false;
  st = enqueue_batch(h, n, models, sweeps, results, workspaces, L, h->capture);
  h->prof = prof;
  const std::string err = g_err;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(h->capture, &graph);
  if (st != CM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    g_err = err;
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  if (h->graphs.size() >= CM_GRAPH_CACHE) {
    size_t lru = 0;
    for (size_t i = 1; i < h->graphs.size(); ++i)
      if (h->graphs[i].last < h->graphs[lru].last) lru = i;
    (void)hipGraphExecDestroy(h->graphs[lru].exec);
    h->graphs.erase(h->graphs.begin() + (ptrdiff_t)lru);
  }
  h->graphs.push_back(cm_handle::Graph{std::move(sig), exec, ++h->graph_clock});
  if ((e = hipGraphLaunch(exec, stream)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ok();
}

cm_status cm_graph_clear(cm_handle* h) {
  if (!h) return fail(CM_E_INVALID, "handle must not be NULL");
  DeviceGuard guard(h->device);
  clear_graphs(h);
  return ok();
}

}  // extern "C"

namespace {

// Launch the queue's persistent kernel unless it is still running (it ends
// by itself after idle_ticks without an item).
cm_status queue_ensure_running(cm_queue* q) {
  if (q->launched) {
    const hipError_t e = hipEventQuery(q->run_done);
    if (e == hipErrorNotReady) return ok();
    if (e != hipSuccess) return hip_fail(e, "queue kernel");
  }
  cm::QueueArgs a{};
  a.tail = q->tail;
  a.stop = q->stop;
  a.done = q->done;
  a.ring = q->ring;
  a.desc = q->desc;
  a.cap_ring = q->cap_ring;
  a.word = (unsigned long long*)q->dev;
  a.dev_tail = (uint32_t*)(q->dev + 64);
  a.pull_lock = (uint32_t*)(q->dev + 128);
  a.dev_stop = (uint32_t*)(q->dev + 192);
  a.prep_done = (unsigned long long*)(q->dev + 256);
  a.chunk_done = a.prep_done + q->cap_slots;
  a.dring = (cm::QueueReq*)(q->dev + q->o_dring);
  a.ddesc = (cm::QueueDesc*)(q->dev + q->o_ddesc);
  a.idle_ticks = q->idle_ticks;
  hipError_t e;
  if ((e = cm::launch_queue((int)q->kind, (int)q->prec, a, q->groups, q->lds, q->run)) != hipSuccess)
    return hip_fail(e, "queue kernel");
  if ((e = hipEventRecord(q->run_done, q->run)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  q->launched = true;
  return ok();
}

void queue_free(cm_queue* q) {
  if (q->run) {
    if (q->stop) __atomic_store_n(q->stop, 1u, __ATOMIC_RELEASE);
    (void)hipStreamSynchronize(q->run);
    (void)hipStreamDestroy(q->run);
  }
  if (q->run_done) (void)hipEventDestroy(q->run_done);
  if (q->handoff) (void)hipEventDestroy(q->handoff);
  if (q->copy) {
    (void)hipStreamSynchronize(q->copy);
    (void)hipStreamDestroy(q->copy);
  }
  for (hipEvent_t ev : q->copied) (void)hipEventDestroy(ev);
  if (q->host) (void)hipHostFree(q->host);
  if (q->dev) (void)hipFree(q->dev);
  delete q;
}

}  // namespace

extern "C" {

cm_status cm_queue_create(cm_handle* h, uint32_t kind, uint32_t precision, uint32_t slots, uint32_t groups_per_cu,
                          uint32_t idle_us, cm_queue** out) {
  if (!h || !out) return fail(CM_E_INVALID, "handle and out must not be NULL");
  *out = nullptr;
  if (kind != CM_CONFLICT_LCA || (precision != CM_FP64 && precision != CM_FP32_STEP))
    return fail(CM_E_UNSUPPORTED, "the device queue runs conflict-LCA sweeps in FP64 or FP32 steps");
  if (slots < 1 || slots > 4096) return fail(CM_E_INVALID, "slots in [1, 4096]");
  if (groups_per_cu < 1 || groups_per_cu > 4) return fail(CM_E_INVALID, "groups_per_cu in [1, 4]");
  if (idle_us < 100 || idle_us > 10000000) return fail(CM_E_INVALID, "idle_us in [100, 10^7]");
  DeviceGuard guard(h->device);
  cm_queue* q = new (std::nothrow) cm_queue();
  if (!q) return fail(CM_E_DEVICE, "out of host memory");
  q->h = h;
  q->kind = kind;
  q->prec = precision;
  q->cap_slots = slots;
  q->cap_ring = std::max<uint32_t>(512u, 4u * slots);  // requests between the oldest unfinished one and the newest
  q->groups = groups_per_cu * (uint32_t)h->cu_count;
  q->idle_ticks = (uint64_t)idle_us * 100u;  // the real-time clock runs at 100 MHz
  q->lds = cm::lane_stage_bytes((int)kind, (int)precision, 256) + kLdsBudget;
  if (q->lds > h->lds_per_block) {
    delete q;
    return fail(CM_E_UNSUPPORTED, "queue kernel: LDS too small on this device");
  }
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t o_done = 256, o_ring = up(o_done + 4u * (size_t)slots),
               o_desc = up(o_ring + sizeof(cm::QueueReq) * (size_t)q->cap_ring),
               bytes = o_desc + sizeof(cm::QueueDesc) * (size_t)slots;
  hipError_t e;
  if ((e = hipHostMalloc((void**)&q->host, bytes, hipHostMallocCoherent)) != hipSuccess) {
    delete q;
    return hip_fail(e, "hipHostMalloc");
  }
  memset(q->host, 0, bytes);
  q->tail = (uint32_t*)q->host;
  q->stop = (uint32_t*)(q->host + 64);
  q->done = (uint32_t*)(q->host + o_done);
  q->ring = (cm::QueueReq*)(q->host + o_ring);
  q->desc = (cm::QueueDesc*)(q->host + o_desc);
  q->o_dring = up(256 + 16u * (size_t)slots);
  q->o_ddesc = up(q->o_dring + sizeof(cm::QueueReq) * (size_t)q->cap_ring);
  const size_t dbytes = q->o_ddesc + sizeof(cm::QueueDesc) * (size_t)slots;
  if ((e = hipMalloc((void**)&q->dev, dbytes)) != hipSuccess || (e = hipMemset(q->dev, 0, dbytes)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&q->run, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&q->run_done, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&q->handoff, hipEventDisableTiming)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&q->copy, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    queue_free(q);
    return hip_fail(e, "queue set-up");
  }
  q->copied.assign(slots, nullptr);
  for (uint32_t i = 0; i < slots; ++i)
    if ((e = hipEventCreateWithFlags(&q->copied[i], hipEventDisableTiming)) != hipSuccess) {
      queue_free(q);
      return hip_fail(e, "queue set-up");
    }
  q->slot_prep.assign(slots, 0);
  q->slot_chunks.assign(slots, 0);
  q->slot_ticket.assign(slots, 0);
  *out = q;
  return ok();
}

cm_status cm_queue_submit(cm_queue* q, const cm_model* m, const cm_sweep* s, const cm_result* r, void* workspace,
                          uint64_t workspace_bytes, const cm_host_result* host, void* producer_stream,
                          uint64_t* ticket) {
  if (!q || !ticket) return fail(CM_E_INVALID, "queue and ticket must not be NULL");
  Layout L;
  cm_status st = check_launch(m, s, r, workspace, workspace_bytes, L);
  if (st != CM_OK) return st;
  if (m->kind != q->kind || m->precision != q->prec)
    return fail(CM_E_UNSUPPORTED, "the queue runs one kind and precision");
  cm_handle* h = q->h;
  DeviceGuard guard(h->device);
  cm::SimArgs a;
  uint64_t groups = 0;
  size_t lds = 0;
  if ((st = plan_lane(h, m, s, r, (char*)workspace, L, 0, s->n_settings * s->trials, TcSpec{}, a, groups, lds,
                      256)) != CM_OK)
    return st;
  if (lds > q->lds) return fail(CM_E_UNSUPPORTED, "request needs more LDS than the queue kernel has");
  cm::PrepBatch pb{};
  fill_prep(m, s, r, (char*)workspace, L, pb);
  cm::ScoreBatch sb{};
  fill_score(m, s, r, sb);
  const uint64_t pieces = (pb.it[0].end + cm::kQueuePrepSpan - 1) / cm::kQueuePrepSpan;
  const uint64_t n_items = pieces + groups;
  if (n_items >= 0xFFFFFFFFull) return fail(CM_E_UNSUPPORTED, "the sweep is too large for the queue");
  if (q->published == 0xFFFFFFFFu) return fail(CM_E_UNSUPPORTED, "the queue has published 2^32 - 1 requests");
  // room: a free slot, and ring space behind the oldest unfinished request
  uint32_t slot = q->cap_slots;
  for (uint32_t i = 0; i < q->cap_slots; ++i)
    if (!q->slot_ticket[i]) {
      slot = i;
      break;
    }
  const uint32_t oldest = q->reqs.empty() ? q->published : q->reqs.front().number;
  if (slot == q->cap_slots || q->published - oldest >= q->cap_ring) return fail(CM_E_BUSY, "queue full");
  // host copies, enqueued by cm_queue_poll once the device is done: pinned
  // buffers, so that the copies run asynchronously
  cm_queue::Copy cp[4] = {};
  if (host) {
    const uint64_t S = s->n_settings;
    const cm_queue::Copy want[4] = {{host->hist, r->hist, S * 2u * s->n_bins * 8u},
                                    {host->stats, r->stats, S * CM_NSTAT * 8u},
                                    {host->score, r->score, S * 8u},
                                    {host->best, r->best, 16u}};
    for (int i = 0; i < 4; ++i) {
      if (!want[i].dst || !want[i].src) continue;
      hipPointerAttribute_t at{};
      if (hipPointerGetAttributes(&at, want[i].dst) != hipSuccess || at.type != hipMemoryTypeHost) {
        (void)hipGetLastError();
        return fail(CM_E_INVALID, "host result buffers must be pinned host memory (hipHostMalloc)");
      }
      cp[i] = want[i];
    }
  }
  // the producer's work on the buffers (their uploads) is finished before any
  // item can run
  hipError_t e;
  if (producer_stream) {
    if ((e = hipEventRecord(q->handoff, (hipStream_t)producer_stream)) != hipSuccess ||
        (e = hipEventSynchronize(q->handoff)) != hipSuccess)
      return hip_fail(e, "producer hand-off");
  }
  const uint64_t t = q->next_ticket++;
  cm::QueueDesc& d = q->desc[slot];
  d.a = a;
  d.prep = pb.it[0];
  d.score = sb.n ? sb.a[0] : cm::ScoreArgs{};
  d.scored = sb.n ? 1u : 0u;
  d.prep_target = q->slot_prep[slot] + pieces;
  d.chunk_target = q->slot_chunks[slot] + groups;
  d.pieces = (uint32_t)pieces;
  d.ticket = (uint32_t)t;
  d.pad = 0;
  cm::QueueReq& ent = q->ring[q->published % q->cap_ring];
  ent.num_items = ((unsigned long long)q->published << 32) | n_items;
  ent.slot = slot;
  ent.pad = 0;
  q->slot_prep[slot] += pieces;
  q->slot_chunks[slot] += groups;
  q->slot_ticket[slot] = t;
  q->reqs.push_back(cm_queue::Req{t, slot, q->published, false, {cp[0], cp[1], cp[2], cp[3]}});
  q->published += 1u;
  __atomic_store_n(q->tail, q->published, __ATOMIC_RELEASE);  // publish after the entry and descriptor
  *ticket = t;
  return queue_ensure_running(q);
}

cm_status cm_queue_poll(cm_queue* q, uint64_t ticket, int* done) {
  if (!q || !done) return fail(CM_E_INVALID, "queue and done must not be NULL");
  *done = 0;
  size_t k = 0;
  while (k < q->reqs.size() && q->reqs[k].ticket != ticket) ++k;
  if (k == q->reqs.size()) return fail(CM_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  DeviceGuard guard(q->h->device);
  cm_queue::Req& rq = q->reqs[k];
  hipError_t e;
  if (!rq.copying) {
    if (__atomic_load_n(&q->done[rq.slot], __ATOMIC_ACQUIRE) != (uint32_t)ticket)
      return queue_ensure_running(q);  // relaunch if the kernel went idle before this request's items
    bool any = false;
    for (const auto& c : rq.cp) {
      if (!c.dst) continue;
      if ((e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToHost, q->copy)) != hipSuccess)
        return hip_fail(e, "result copy");
      any = true;
    }
    rq.copying = true;
    if (any && (e = hipEventRecord(q->copied[rq.slot], q->copy)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if (!any) {
      q->slot_ticket[rq.slot] = 0;
      q->reqs.erase(q->reqs.begin() + (ptrdiff_t)k);
      *done = 1;
      return ok();
    }
  }
  e = hipEventQuery(q->copied[rq.slot]);
  if (e == hipErrorNotReady) return ok();
  if (e != hipSuccess) return hip_fail(e, "result copy");
  q->slot_ticket[rq.slot] = 0;
  q->reqs.erase(q->reqs.begin() + (ptrdiff_t)k);
  *done = 1;
  return ok();
}

cm_status cm_queue_destroy(cm_queue* q) {
  if (!q) return ok();
  DeviceGuard guard(q->h->device);
  queue_free(q);
  return ok();
}

// The node-by-node kernels index runs with 32-bit integers.
static cm_status check_unfused(const cm_model* m, const cm_sweep* s) {
  cm_status st = check_model_sweep(m, s);
  if (st != CM_OK) return st;
  if (m->kind != CM_DDM && m->kind != CM_CONFLICT_LCA)
    return fail(CM_E_UNSUPPORTED, "unfused execution: DDM and conflict LCA only");
  if (s->n_settings * s->trials > 0xFFFFFFFFull)
    return fail(CM_E_INVALID, "unfused execution: at most 2^32 - 1 runs (n_settings x trials)");
  return ok();
}

cm_status cm_unfused_workspace_bytes(const cm_model* m, const cm_sweep* s, uint64_t* bytes) {
  if (!bytes) return fail(CM_E_INVALID, "bytes must not be NULL");
  cm_status st = check_unfused(m, s);
  if (st != CM_OK) return st;
  *bytes = unfused_layout(m, s).total;
  return ok();
}

cm_status cm_launch_unfused(cm_handle* h, const cm_model* m, const cm_sweep* s, const cm_result* r,
                            void* workspace, uint64_t workspace_bytes, void* hip_stream) {
  if (!h) return fail(CM_E_INVALID, "handle must not be NULL");
  cm_status st = check_unfused(m, s);
  if (st != CM_OK) return st;
  if ((st = check_result(m, s, r)) != CM_OK) return st;
  const UnfusedLayout U = unfused_layout(m, s);
  if (!workspace || !aligned(workspace, kWorkspaceAlign))
    return fail(CM_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
  if (workspace_bytes < U.total)
    return fail(CM_E_BUDGET, "workspace has %llu bytes, needs %llu", (unsigned long long)workspace_bytes,
                (unsigned long long)U.total);
  hipStream_t stream = (hipStream_t)hip_stream;
  DeviceGuard guard(h->device);
  hipError_t e;
  if (!h->host_count && (e = hipHostMalloc((void**)&h->host_count, sizeof(uint32_t))) != hipSuccess)
    return hip_fail(e, "hipHostMalloc");
  char* ws = (char*)workspace;
  if ((st = enqueue_prep(m, s, r, ws, U.base, stream)) != CM_OK) return st;
  const double* p = m->params;
  cm::UnfusedArgs a{};
  a.trials = s->trials;
  a.n_settings = s->n_settings;
  a.total_runs = s->n_settings * s->trials;
  a.seed = s->seed;
  a.max_steps = s->max_steps;
  a.n_bins = s->n_bins;
  a.n_signals = m->n_signals;
  a.kind = m->kind;
  a.flag_eps = s->flag_eps;
  a.grid = s->grid;
  a.correct = (const int32_t*)(ws + U.base.correct);
  if (m->kind == CM_DDM) {
    a.dt = p[CM_DDM_DT];
    a.drift = p[CM_DDM_DRIFT];
    a.b = p[CM_DDM_NOISE] * sqrt(p[CM_DDM_DT]);
    a.thresh = p[CM_DDM_THRESH];
    a.start = p[CM_DDM_START];
  } else {
    a.dt = p[CM_LCA_DT];
    a.leak = p[CM_LCA_LEAK];
    a.comp = p[CM_LCA_COMP];
    a.b = p[CM_LCA_NOISE] * sqrt(p[CM_LCA_DT]);
    a.thresh = p[CM_LCA_THRESH];
    a.nonneg = p[CM_LCA_NONNEG] != 0.0;
    a.drive = (const double*)(ws + U.base.drive);
  }
  a.x = (double*)(ws + U.x);
  a.z = (double*)(ws + U.z);
  a.n = (uint32_t*)(ws + U.n);
  a.flag = (uint8_t*)(ws + U.flag);
  a.choice = (int8_t*)(ws + U.choice);
  a.active = (uint32_t*)(ws + U.active);
  a.count = (uint32_t*)(ws + U.count);
  a.hist = r->hist;
  a.stats = r->stats;
  a.run_choice = r->run_choice;
  a.run_step = r->run_step;
  a.run_flag = r->run_flag;
  a.run_state = r->run_state;
  ProfScope prof{h, stream};
  if ((e = prof.begin()) != hipSuccess) return hip_fail(e, "hipEventRecord");
  if ((e = cm::launch_uf_init(a, stream)) != hipSuccess) return hip_fail(e, "unfused init");
  uint64_t bound = a.total_runs;
  for (uint32_t n = 1; n <= s->max_steps; ++n) {
    const int cur = (int)((n - 1u) & 1u);
    if ((e = cm::launch_uf_step(a, (int)m->precision, n, cur, bound, stream)) != hipSuccess)
      return hip_fail(e, "unfused step");
    if (n % 16u == 0 && n < s->max_steps) {  // the host-side scheduler looks at the active count
      if ((e = hipMemcpyAsync(h->host_count, a.count + (1 - cur), sizeof(uint32_t), hipMemcpyDeviceToHost,
                              stream)) != hipSuccess)
        return hip_fail(e, "active count");
      if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
      bound = *h->host_count;
      if (!bound) break;
    }
  }
  if ((e = cm::launch_uf_reduce(a, stream)) != hipSuccess) return hip_fail(e, "unfused reduce");
  if ((e = prof.end()) != hipSuccess) return hip_fail(e, "hipEventRecord");
  return enqueue_score(m, s, r, stream);
}

cm_status cm_ddm_density(cm_handle* h, const cm_model* m, const cm_sweep* s, uint32_t n_cells, double tol,
                         double* first_passage, void* hip_stream) {
  if (!h) return fail(CM_E_INVALID, "handle must not be NULL");
  cm_status st = check_model_sweep(m, s);
  if (st != CM_OK) return st;
  if (m->kind != CM_DDM) return fail(CM_E_UNSUPPORTED, "density propagation applies to the DDM only");
  if (!(m->params[CM_DDM_NOISE] > 0)) return fail(CM_E_INVALID, "density propagation needs noise > 0");
  if (n_cells < 16 || n_cells > 1300) return fail(CM_E_INVALID, "n_cells must be in [16, 1300]");
  if (s->n_settings > 0x7FFFFFFFull) return fail(CM_E_INVALID, "too many settings for one launch");
  if (!(tol >= 0) || !isfinite(tol)) return fail(CM_E_INVALID, "tol must be finite and >= 0");
  if (!first_passage || !aligned(first_passage, 8)) return fail(CM_E_INVALID, "first_passage must be 8-byte aligned");
  const double* p = m->params;
  cm::DensityArgs a{};
  a.n_settings = s->n_settings;
  a.max_steps = s->max_steps;
  a.cells = n_cells;
  a.n_signals = m->n_signals;
  a.dt = p[CM_DDM_DT];
  a.drift = p[CM_DDM_DRIFT];
  a.b = p[CM_DDM_NOISE] * sqrt(p[CM_DDM_DT]);
  a.thresh = p[CM_DDM_THRESH];
  a.start = p[CM_DDM_START];
  a.tol = tol;
  a.grid = s->grid;
  a.out = first_passage;
  if (cm::density_lds_bytes(n_cells) > h->lds_per_block)
    return fail(CM_E_INVALID, "n_cells %u needs more LDS than a workgroup has", n_cells);
  DeviceGuard guard(h->device);
  hipStream_t stream = (hipStream_t)hip_stream;
  ProfScope prof{h, stream};
  hipError_t e;
  if ((e = prof.begin()) != hipSuccess) return hip_fail(e, "hipEventRecord");
  if ((e = cm::launch_ddm_density(a, stream)) != hipSuccess) return hip_fail(e, "density kernel");
  if ((e = prof.end()) != hipSuccess) return hip_fail(e, "hipEventRecord");
  return ok();
}

}  // extern "C"
