// Host side of the C ABI declared in include/msgpm.h: parameter validation,
// workspace layout and the launch sequence of the pipeline.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <deque>
#include <map>
#include <thread>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "common.h"

using namespace msgpm;

// The binding mirrors these structures field by field.
static_assert(sizeof(msgpm_params) == 136, "msgpm_params layout");
static_assert(sizeof(msgpm_plane) == 144, "msgpm_plane layout");

namespace {

thread_local std::string g_err;
thread_local bool g_capturing = false;  // launches are being captured into a graph: no timing events
thread_local bool g_no_events = false;  // a call that must not create HIP objects: no timing events

msgpm_status fail(msgpm_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
msgpm_status fail(msgpm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

msgpm_status check(hipError_t e, const char* what) {
  if (e == hipSuccess) return MSGPM_OK;
  return fail(e == hipErrorOutOfMemory ? MSGPM_E_OOM : MSGPM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Allocations the library makes itself (pinned staging, events of the batched
// and serving forms) go through these two, so that a test can make them fail.
std::atomic<int> g_fail_allocs{0};

bool injected_failure() {
  int n = g_fail_allocs.load();
  while (n > 0)
    if (g_fail_allocs.compare_exchange_weak(n, n - 1)) return true;
  return false;
}

hipError_t host_alloc(void** p, size_t bytes) {
  if (injected_failure()) return hipErrorOutOfMemory;
  return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

hipError_t event_create(hipEvent_t* e) {
  if (injected_failure()) return hipErrorOutOfMemory;
  return hipEventCreateWithFlags(e, hipEventDisableTiming);
}

int block_count(int n, int B) {
  if (n <= B) return 1;
  const int S = B / 2;
  int m = (n - B) / S + 1;
  if ((n - B) % S) ++m;
  return m;
}

uint64_t align256(uint64_t v) { return (v + 255) & ~(uint64_t)255; }

// One direction's list of restricted half-sweep pixels (all pixels of one colour).
uint64_t active_list_bytes(const DevParams& d) { return align256((uint64_t)((d.W + 1) / 2) * d.H * sizeof(int32_t)); }

// Optional per-kind kernel timing with reusable HIP events.
struct Timer {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> pool;  // events created so far, reused after each read
  size_t used = 0;
  std::vector<int> kinds;        // kind of each recorded (start, stop) pair
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};
Timer g_timer;

// roctx range of a phase, visible to rocprofv3 --marker-trace; host-side
// markers only (none in calls that must not create objects).
const char* const kPhaseNames[MSGPM_TIMER_KINDS] = {
    "msgpm features", "msgpm init", "msgpm eval_cost", "msgpm pm initial pass", "msgpm pm restricted (distorted)",
    "msgpm ransac", "msgpm assign", "msgpm symmetry", "msgpm fb", "msgpm nnf_update", "msgpm finalize",
    "msgpm pm lists", "msgpm pm restricted (identity)", "msgpm fill"};

struct Range {
  bool on;
  explicit Range(const char* name) : on(!g_no_events) {
    if (on) roctxRangePushA(name);
  }
  ~Range() {
    if (on) roctxRangePop();
  }
};

template <class F>
hipError_t timed(int kind, hipStream_t s, F&& launch) {
  Range range(kPhaseNames[kind]);
  if (!g_timer.on || g_capturing || g_no_events) return launch();
  std::lock_guard<std::mutex> lk(g_timer.mu);
  hipEvent_t a = g_timer.get(), b = g_timer.get();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  if (e == hipSuccess) g_timer.kinds.push_back(kind);
  return e;
}

// Validates *p and derives the kernel parameters and the workspace layout.
msgpm_status prepare(const msgpm_params* p, DevParams* P, msgpm_layout* L) {
  if (!p) return fail(MSGPM_E_INVALID, "params is NULL");
  if (p->width < 2 || p->height < 2 || p->width > 32767 || p->height > 32767)
    return fail(MSGPM_E_INVALID, "frame size %dx%d outside 2..32767", p->width, p->height);
  if (p->channels != 3 && p->channels != 5) return fail(MSGPM_E_INVALID, "channels must be 3 or 5");
  if (p->patch_radius < 1 || p->patch_radius > 4)
    return fail(MSGPM_E_UNSUPPORTED, "patch_radius %d outside 1..4", p->patch_radius);
  if (p->n_levels < 0 || p->n_levels > MSGPM_MAX_LEVELS) return fail(MSGPM_E_INVALID, "n_levels outside 0..8");
  for (int l = 0; l < p->n_levels; ++l)
    if (p->block[l] < 4 || p->block[l] > 128) return fail(MSGPM_E_INVALID, "block[%d] = %d outside 4..128", l, p->block[l]);
  if (p->pm_iters < 0 || p->pm_iters > 1000) return fail(MSGPM_E_INVALID, "pm_iters outside 0..1000");
  if (p->ransac_hyps < 1 || p->ransac_hyps > 1024) return fail(MSGPM_E_INVALID, "ransac_hyps outside 1..1024");
  if (p->search_radius0 < 0 || p->search_radius0 > 32767) return fail(MSGPM_E_INVALID, "search_radius0 outside 0..32767");
  if (p->min_support_abs < 0) return fail(MSGPM_E_INVALID, "min_support_abs < 0");
  if (p->eta_den <= 0 || p->eta_num < 0) return fail(MSGPM_E_INVALID, "eta must be num >= 0, den > 0");
  if (!(p->inlier_px > 0) || !(p->eps_color > 0) || !(p->fb_px > 0) || !(p->min_support_frac >= 0) ||
      !(p->grad_weight >= 0))
    return fail(MSGPM_E_INVALID, "thresholds must be positive and finite");
  if (p->flags & ~(MSGPM_FLAG_FP16 | MSGPM_FLAG_CUE_OVERLAP | MSGPM_FLAG_CUE_UNIQUE | MSGPM_FLAG_HISTEQ |
                   MSGPM_FLAG_MERGE_STRICT | MSGPM_FLAG_ONE_STREAM))
    return fail(MSGPM_E_INVALID, "unknown flags 0x%x", p->flags);
  if (p->fill_sweeps < 0 || p->fill_sweeps > 65536) return fail(MSGPM_E_INVALID, "fill_sweeps outside 0..65536");
  {
    // kernels address one frame's features with 32-bit byte offsets, including
    // the unclamped offsets of patch rows up to r rows beyond the last
    const uint64_t px_bytes = (p->flags & MSGPM_FLAG_FP16) ? (p->channels == 3 ? 8 : 12) : 4 * (uint64_t)p->channels;
    if (((uint64_t)p->width * ((uint64_t)p->height + p->patch_radius) + 1) * px_bytes > 0x7fffffffull)
      return fail(MSGPM_E_UNSUPPORTED, "frame %dx%d: features exceed 2 GiB", p->width, p->height);
  }

  DevParams d;
  memset(&d, 0, sizeof d);
  d.W = p->width;
  d.H = p->height;
  d.C = p->channels;
  d.r = p->patch_radius;
  d.iters = p->pm_iters;
  d.hyps = p->ransac_hyps;
  d.R0 = p->search_radius0 > 0 ? p->search_radius0 : (p->width > p->height ? p->width : p->height);
  d.nk = 0;
  while ((d.R0 >> d.nk) >= 1) ++d.nk;
  d.m_min_abs = p->min_support_abs;
  d.eta_num = p->eta_num;
  d.eta_den = p->eta_den;
  d.fp16 = (p->flags & MSGPM_FLAG_FP16) ? 1 : 0;
  d.cues = (int)(p->flags & (MSGPM_FLAG_CUE_OVERLAP | MSGPM_FLAG_CUE_UNIQUE));
  d.fill_sweeps = p->fill_sweeps;
  d.histeq = (p->flags & MSGPM_FLAG_HISTEQ) ? 1 : 0;
  d.merge_strict = (p->flags & MSGPM_FLAG_MERGE_STRICT) ? 1 : 0;
  d.n_levels = p->n_levels;
  int off = 0;
  for (int l = 0; l < p->n_levels; ++l) {
    d.block[l] = p->block[l];
    d.nbx[l] = block_count(d.W, d.block[l]);
    d.nby[l] = block_count(d.H, d.block[l]);
    d.plane_off[l] = off;
    off += 2 * d.nbx[l] * d.nby[l];
  }
  d.planes_per_dir = off;
  d.gw = (float)p->grad_weight;
  d.tau2 = p->inlier_px * p->inlier_px;
  d.eps2 = p->eps_color * p->eps_color;
  d.fb2 = p->fb_px * p->fb_px;
  d.mu = p->min_support_frac;
  d.seed = p->seed;
  if (P) *P = d;

  if (L) {
    msgpm_layout o;
    memset(&o, 0, sizeof o);
    const uint64_t n = (uint64_t)d.W * d.H;
    uint64_t cur = 0;
    o.feat_bytes = (n + 1) * (d.fp16 ? (d.C == 3 ? 8 : 12) : 4 * (uint64_t)d.C);
    for (int f = 0; f < 2; ++f) {
      o.feat[f] = cur;
      cur = align256(cur + o.feat_bytes);
    }
    for (int k = 0; k < 2; ++k) {
      o.nnf[k] = cur;
      cur = align256(cur + 4 * n);
      o.cost[k] = cur;
      cur = align256(cur + 4 * n);
      o.win[k] = cur;
      cur = align256(cur + 4 * n);
      o.loss[k] = cur;
      cur = align256(cur + 8 * n);
      o.hlabel[k] = cur;
      cur = align256(cur + 4 * n);
      o.twin[k] = cur;
      cur = align256(cur + 4 * n);
      o.tloss[k] = cur;
      cur = align256(cur + 8 * n);
    }
    o.planes = cur;
    o.n_planes = 2 * d.planes_per_dir;
    cur = align256(cur + (uint64_t)o.n_planes * sizeof(msgpm_plane));
    o.counters = cur;
    cur = align256(cur + (uint64_t)kCounterKinds * kCounterStripes * sizeof(uint64_t));
    o.histeq = cur;
    cur = align256(cur + (2 * 256 + 2 * 256 + 2) * sizeof(uint32_t));
    o.active = cur;
    cur = align256(cur + 4 * active_list_bytes(d) + 16 * sizeof(uint32_t));
    o.total_bytes = cur;
    o.n_levels = d.n_levels;
    for (int l = 0; l < d.n_levels; ++l) {
      o.level_blocks[l] = d.nbx[l] * d.nby[l];
      o.level_nbx[l] = d.nbx[l];
    }
    *L = o;
  }
  return MSGPM_OK;
}

Ws make_ws(const DevParams& P, const msgpm_layout& L, void* base) {
  char* b = static_cast<char*>(base);
  Ws w;
  for (int k = 0; k < 2; ++k) {
    w.feat[k] = b + L.feat[k];
    w.nnf[k] = reinterpret_cast<int32_t*>(b + L.nnf[k]);
    w.cost[k] = reinterpret_cast<float*>(b + L.cost[k]);
    w.win[k] = reinterpret_cast<int32_t*>(b + L.win[k]);
    w.loss[k] = reinterpret_cast<double*>(b + L.loss[k]);
    w.hlabel[k] = reinterpret_cast<int32_t*>(b + L.hlabel[k]);
    w.twin[k] = reinterpret_cast<int32_t*>(b + L.twin[k]);
    w.tloss[k] = reinterpret_cast<double*>(b + L.tloss[k]);
  }
  w.planes = reinterpret_cast<msgpm_plane*>(b + L.planes);
  w.counters = reinterpret_cast<unsigned long long*>(b + L.counters);
  w.heq = reinterpret_cast<unsigned*>(b + L.histeq);
  const uint64_t lb = active_list_bytes(P);
  for (int k = 0; k < 4; ++k) w.act[k] = reinterpret_cast<int32_t*>(b + L.active + k * lb);
  w.act_count = reinterpret_cast<unsigned*>(b + L.active + 4 * lb);
  return w;
}

struct Ctx {
  DevParams P;
  msgpm_layout L;
  Ws w;
  hipStream_t s;
  bool one_stream = false;  // restricted half-sweeps: both launches on s, one after the other
};

msgpm_status open_ctx(const msgpm_params* p, void* ws, void* stream, Ctx* c) {
  msgpm_status st = prepare(p, &c->P, &c->L);
  if (st != MSGPM_OK) return st;
  if (!ws) return fail(MSGPM_E_INVALID, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(MSGPM_E_INVALID, "workspace not 256-byte aligned");
  c->w = make_ws(c->P, c->L, ws);
  c->s = static_cast<hipStream_t>(stream);
  c->one_stream = (p->flags & MSGPM_FLAG_ONE_STREAM) != 0;
  return MSGPM_OK;
}

msgpm_status check_level(const Ctx& c, int level, int stage) {
  if (level < 0 || level >= c.P.n_levels) return fail(MSGPM_E_INVALID, "level %d outside 0..%d", level, c.P.n_levels - 1);
  if (stage != 1 && stage != 2) return fail(MSGPM_E_INVALID, "stage must be 1 or 2");
  return MSGPM_OK;
}

// A second stream of the calling thread (one per device), on which the
// identity-patch launch of a restricted half-sweep runs beside the
// distorted-patch launch: the two update disjoint pixels of one colour and
// only read the other colour.  Created on first use and kept for the life of
// the thread; default priority.
struct Aux {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
thread_local std::map<int, Aux> t_aux;

hipError_t aux_stream(Aux** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  Aux& a = t_aux[dev];
  if (!a.s) {
    if ((e = hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&a.fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&a.join, hipEventDisableTiming)) != hipSuccess) return e;
  }
  *out = &a;
  return hipSuccess;
}

// Runs on_second on the calling thread's second stream beside on_caller on s:
// forked from s and joined back into it by events, also when a launch fails.
template <class A, class B>
msgpm_status side_by_side(hipStream_t s, A&& on_caller, B&& on_second) {
  Aux* a = nullptr;
  msgpm_status st;
  if ((st = check(aux_stream(&a), "second stream")) != MSGPM_OK) return st;
  if ((st = check(hipEventRecord(a->fork, s), "fork")) != MSGPM_OK) return st;
  if ((st = check(hipStreamWaitEvent(a->s, a->fork, 0), "fork")) != MSGPM_OK) return st;
  const msgpm_status st1 = on_second(a->s);
  const msgpm_status st0 = on_caller(s);
  if ((st = check(hipEventRecord(a->join, a->s), "join")) != MSGPM_OK) return st;
  if ((st = check(hipStreamWaitEvent(s, a->join, 0), "join")) != MSGPM_OK) return st;
  return st1 != MSGPM_OK ? st1 : st0;
}

msgpm_status run_lists(const Ctx& c) {
  return check(timed(MSGPM_T_PM_LIST, c.s, [&] { return launch_pm_lists(c.P, c.w, c.s); }), "pm_list");
}

// One half-sweep; a restricted one reads the lists run_lists built.  fresh:
// the swept pixels' current costs are computed in the sweep (the cost refresh
// of the pass) instead of being read.
msgpm_status run_halfsweep(const Ctx& c, int colour, int it, int slot, int restricted, int fresh) {
  if (!restricted)
    return check(timed(MSGPM_T_PM_INIT, c.s, [&] { return launch_pm_halfsweep(c.P, c.w, colour, it, slot, fresh, c.s); }), "pm_halfsweep");
  if (c.one_stream) {
    // the two launches update disjoint pixels and read only the other colour:
    // in sequence they give the same result as side by side
    msgpm_status st = check(timed(MSGPM_T_PM_RESTRICTED, c.s, [&] {
      return launch_pm_restricted(c.P, c.w, colour, it, slot, 0, fresh, c.s);
    }), "pm_restricted");
    if (st != MSGPM_OK) return st;
    return check(timed(MSGPM_T_PM_RESTRICTED_IDENT, c.s, [&] {
      return launch_pm_restricted(c.P, c.w, colour, it, slot, 1, fresh, c.s);
    }), "pm_restricted");
  }
  // distorted patches on the caller's stream, identity patches on the second one
  return side_by_side(
      c.s,
      [&](hipStream_t s) {
        return check(timed(MSGPM_T_PM_RESTRICTED, s, [&] { return launch_pm_restricted(c.P, c.w, colour, it, slot, 0, fresh, s); }), "pm_restricted");
      },
      [&](hipStream_t s) {
        return check(timed(MSGPM_T_PM_RESTRICTED_IDENT, s, [&] { return launch_pm_restricted(c.P, c.w, colour, it, slot, 1, fresh, s); }), "pm_restricted");
      });
}

// A pass of half-sweeps; a restricted pass reads the lists built before it.
// The cost refresh that opens the pass (mode 0, or mode 1 for a restricted
// one) is folded into the first half-sweep of each colour, which computes its
// pixels' costs before their candidates; a pass without half-sweeps runs it
// on its own.
msgpm_status run_pm_pass(const Ctx& c, int slot, int restricted) {
  if (c.P.iters == 0)
    return check(timed(MSGPM_T_EVAL_COST, c.s, [&] { return launch_eval_cost(c.P, c.w, restricted, c.s); }), "eval_cost");
  for (int it = 0; it < c.P.iters; ++it)
    for (int colour = 0; colour < 2; ++colour) {
      msgpm_status st = run_halfsweep(c, colour, it, slot, restricted, it == 0);
      if (st != MSGPM_OK) return st;
    }
  return MSGPM_OK;
}

}  // namespace

extern "C" {

const char* msgpm_last_error(void) { return g_err.c_str(); }

msgpm_status msgpm_layout_query(const msgpm_params* p, msgpm_layout* out) {
  if (!out) return fail(MSGPM_E_INVALID, "layout pointer is NULL");
  return prepare(p, nullptr, out);
}

msgpm_status msgpm_features(const msgpm_params* p, const float* d_rgb1, const float* d_rgb2, void* d_ws,
                            void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  if (!d_rgb1 || !d_rgb2) return fail(MSGPM_E_INVALID, "frame pointer is NULL");
  if (c.P.histeq) {
    st = check(timed(MSGPM_T_FEATURES, c.s, [&] { return launch_histeq(c.P, c.w, d_rgb1, d_rgb2, c.s); }), "histeq");
    if (st != MSGPM_OK) return st;
  }
  st = check(timed(MSGPM_T_FEATURES, c.s, [&] { return launch_features(c.P, c.w, d_rgb1, 0, c.s); }), "features");
  if (st != MSGPM_OK) return st;
  return check(timed(MSGPM_T_FEATURES, c.s, [&] { return launch_features(c.P, c.w, d_rgb2, 1, c.s); }), "features");
}

msgpm_status msgpm_init_state(const msgpm_params* p, const int32_t* d_init_nnf0, const int32_t* d_init_nnf1,
                              void* d_ws, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  return check(timed(MSGPM_T_INIT, c.s, [&] { return launch_init_state(c.P, c.w, d_init_nnf0, d_init_nnf1, c.s); }), "init_state");
}

msgpm_status msgpm_eval_cost(const msgpm_params* p, void* d_ws, int mode, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  if (mode < 0 || mode > 2) return fail(MSGPM_E_INVALID, "mode must be 0, 1 or 2");
  if (mode == 1 && (st = run_lists(c)) != MSGPM_OK) return st;  // mode 1 reads the unassigned pixels' lists
  return check(timed(MSGPM_T_EVAL_COST, c.s, [&] { return launch_eval_cost(c.P, c.w, mode, c.s); }), "eval_cost");
}

msgpm_status msgpm_pm_halfsweep(const msgpm_params* p, void* d_ws, int colour, int iter, int slot, int restricted,
                                void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  if (colour != 0 && colour != 1) return fail(MSGPM_E_INVALID, "colour must be 0 or 1");
  if (iter < 0 || slot < 0 || slot > 255) return fail(MSGPM_E_INVALID, "iter or slot out of range");
  if (restricted < 0 || restricted > (1 | MSGPM_PM_FRESH))
    return fail(MSGPM_E_INVALID, "restricted must be 0 or 1, optionally with MSGPM_PM_FRESH");
  if ((restricted & 1) && (st = run_lists(c)) != MSGPM_OK) return st;
  return run_halfsweep(c, colour, iter, slot, restricted & 1, (restricted & MSGPM_PM_FRESH) ? 1 : 0);
}

msgpm_status msgpm_ransac(const msgpm_params* p, void* d_ws, int level, int stage, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  if ((st = check_level(c, level, stage)) != MSGPM_OK) return st;
  return check(timed(MSGPM_T_RANSAC, c.s, [&] { return launch_ransac(c.P, c.w, level, stage, c.s); }), "ransac");
}

msgpm_status msgpm_assign(const msgpm_params* p, void* d_ws, int level, int stage, int tentative, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  if ((st = check_level(c, level, stage)) != MSGPM_OK) return st;
  return check(timed(MSGPM_T_ASSIGN, c.s, [&] { return launch_assign(c.P, c.w, level, stage, tentative ? 1 : 0, c.s); }), "assign");
}

msgpm_status msgpm_symmetry(const msgpm_params* p, void* d_ws, int level, int stage, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  if ((st = check_level(c, level, stage)) != MSGPM_OK) return st;
  return check(timed(MSGPM_T_SYMMETRY, c.s, [&] { return launch_symmetry(c.P, c.w, level, stage, c.s); }), "symmetry");
}

msgpm_status msgpm_fb_unassign(const msgpm_params* p, void* d_ws, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  return check(timed(MSGPM_T_FB, c.s, [&] { return launch_fb_unassign(c.P, c.w, c.s); }), "fb_unassign");
}

msgpm_status msgpm_unique(const msgpm_params* p, void* d_ws, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  return check(timed(MSGPM_T_FB, c.s, [&] { return launch_unique(c.P, c.w, c.s); }), "unique");
}

msgpm_status msgpm_fill(const msgpm_params* p, void* d_ws, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  return check(timed(MSGPM_T_FILL, c.s, [&] { return launch_fill(c.P, c.w, c.s); }), "fill");
}

msgpm_status msgpm_nnf_update(const msgpm_params* p, void* d_ws, int level, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  if ((st = check_level(c, level, 1)) != MSGPM_OK) return st;
  return check(timed(MSGPM_T_NNF_UPDATE, c.s, [&] { return launch_nnf_update(c.P, c.w, level, c.s); }), "nnf_update");
}

msgpm_status msgpm_finalize(const msgpm_params* p, void* d_ws, float* d_flow0, float* d_flow1, uint8_t* d_occ0,
                            uint8_t* d_occ1, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  st = check(timed(MSGPM_T_EVAL_COST, c.s, [&] { return launch_eval_cost(c.P, c.w, 2, c.s); }), "eval_cost");
  if (st != MSGPM_OK) return st;
  return check(timed(MSGPM_T_FINALIZE, c.s, [&] { return launch_finalize(c.P, c.w, d_flow0, d_flow1, d_occ0, d_occ1, c.s); }), "finalize");
}

}  // extern "C"

namespace {

msgpm_status solve_sequence(const Ctx& c, const float* d_rgb1, const float* d_rgb2, const int32_t* d_init_nnf0,
                            const int32_t* d_init_nnf1, float* d_flow0, float* d_flow1, uint8_t* d_occ0,
                            uint8_t* d_occ1) {
  msgpm_status st;
  Range whole("msgpm solve");
#define RUN(expr, what)                          \
  do {                                           \
    msgpm_status s_ = check((expr), what);       \
    if (s_ != MSGPM_OK) return s_;               \
  } while (0)
  if (c.P.histeq) RUN(timed(MSGPM_T_FEATURES, c.s, [&] { return launch_histeq(c.P, c.w, d_rgb1, d_rgb2, c.s); }), "histeq");
  RUN(timed(MSGPM_T_FEATURES, c.s, [&] { return launch_features(c.P, c.w, d_rgb1, 0, c.s); }), "features");
  RUN(timed(MSGPM_T_FEATURES, c.s, [&] { return launch_features(c.P, c.w, d_rgb2, 1, c.s); }), "features");
  RUN(timed(MSGPM_T_INIT, c.s, [&] { return launch_init_state(c.P, c.w, d_init_nnf0, d_init_nnf1, c.s); }), "init_state");
  // the initial pass, its cost refresh folded into it
  if ((st = run_pm_pass(c, 0, 0)) != MSGPM_OK) return st;
  for (int l = 0; l < c.P.n_levels; ++l) {
    for (int stage = 1; stage <= 2; ++stage) {
      RUN(timed(MSGPM_T_RANSAC, c.s, [&] { return launch_ransac(c.P, c.w, l, stage, c.s); }), "ransac");
      RUN(timed(MSGPM_T_ASSIGN, c.s, [&] { return launch_assign(c.P, c.w, l, stage, 1, c.s); }), "assign");
      RUN(timed(MSGPM_T_SYMMETRY, c.s, [&] { return launch_symmetry(c.P, c.w, l, stage, c.s); }), "symmetry");
      RUN(timed(MSGPM_T_ASSIGN, c.s, [&] { return launch_assign(c.P, c.w, l, stage, 0, c.s); }), "assign");
    }
    RUN(timed(MSGPM_T_FB, c.s, [&] { return launch_fb_unassign(c.P, c.w, c.s); }), "fb_unassign");
    if (c.P.cues & MSGPM_FLAG_CUE_UNIQUE) RUN(timed(MSGPM_T_FB, c.s, [&] { return launch_unique(c.P, c.w, c.s); }), "unique");
    RUN(timed(MSGPM_T_NNF_UPDATE, c.s, [&] { return launch_nnf_update(c.P, c.w, l, c.s); }), "nnf_update");
    // the unassigned pixels' lists serve the whole restricted pass (its cost
    // refresh folded into it)
    if ((st = run_lists(c)) != MSGPM_OK) return st;
    if ((st = run_pm_pass(c, l + 1, 1)) != MSGPM_OK) return st;
  }
  if (c.P.fill_sweeps > 0) RUN(timed(MSGPM_T_FILL, c.s, [&] { return launch_fill(c.P, c.w, c.s); }), "fill");
  RUN(timed(MSGPM_T_EVAL_COST, c.s, [&] { return launch_eval_cost(c.P, c.w, 2, c.s); }), "eval_cost");
  RUN(timed(MSGPM_T_FINALIZE, c.s, [&] { return launch_finalize(c.P, c.w, d_flow0, d_flow1, d_occ0, d_occ1, c.s); }), "finalize");
#undef RUN
  return MSGPM_OK;
}

// Instantiated graphs, keyed by everything their launches depend on (the
// parameters and buffer addresses of a whole pipeline, or the launch sequence
// and table address of a batched one); the oldest is dropped beyond
// kGraphCache.
constexpr size_t kGraphCache = 64;
struct GraphCache {
  std::mutex mu;
  std::vector<std::pair<std::string, hipGraphExec_t>> entries;
  hipStream_t capture = nullptr;
};
GraphCache g_graphs;

// Launches the graph cached under `key` on s; on a miss, record(stream)
// enqueues the launches on the library's capture stream, which are captured
// into the graph first.
template <class F>
msgpm_status cached_graph_launch(const std::string& key, hipStream_t s, F&& record) {
  std::lock_guard<std::mutex> lk(g_graphs.mu);
  hipGraphExec_t exec = nullptr;
  for (auto& e : g_graphs.entries)
    if (e.first == key) exec = e.second;
  if (!exec) {
    msgpm_status st;
    if (!g_graphs.capture &&
        (st = check(hipStreamCreateWithFlags(&g_graphs.capture, hipStreamNonBlocking), "graph stream")) != MSGPM_OK)
      return st;
    if ((st = check(hipStreamBeginCapture(g_graphs.capture, hipStreamCaptureModeThreadLocal), "graph capture")) !=
        MSGPM_OK)
      return st;
    g_capturing = true;
    const msgpm_status run = record(g_graphs.capture);
    g_capturing = false;
    hipGraph_t graph = nullptr;
    st = check(hipStreamEndCapture(g_graphs.capture, &graph), "graph capture");
    if (run != MSGPM_OK || st != MSGPM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return run != MSGPM_OK ? run : st;
    }
    st = check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
    (void)hipGraphDestroy(graph);
    if (st != MSGPM_OK) return st;
    if (g_graphs.entries.size() >= kGraphCache) {
      (void)hipGraphExecDestroy(g_graphs.entries.front().second);
      g_graphs.entries.erase(g_graphs.entries.begin());
    }
    g_graphs.entries.emplace_back(key, exec);
  }
  return check(hipGraphLaunch(exec, s), "graph launch");
}

}  // namespace

extern "C" {

msgpm_status msgpm_solve(const msgpm_params* p, const float* d_rgb1, const float* d_rgb2,
                         const int32_t* d_init_nnf0, const int32_t* d_init_nnf1, void* d_ws, float* d_flow0,
                         float* d_flow1, uint8_t* d_occ0, uint8_t* d_occ1, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  if (!d_rgb1 || !d_rgb2) return fail(MSGPM_E_INVALID, "frame pointer is NULL");
  return solve_sequence(c, d_rgb1, d_rgb2, d_init_nnf0, d_init_nnf1, d_flow0, d_flow1, d_occ0, d_occ1);
}

msgpm_status msgpm_solve_graph(const msgpm_params* p, const float* d_rgb1, const float* d_rgb2,
                               const int32_t* d_init_nnf0, const int32_t* d_init_nnf1, void* d_ws,
                               float* d_flow0, float* d_flow1, uint8_t* d_occ0, uint8_t* d_occ1, void* stream) {
  Ctx c;
  msgpm_status st = open_ctx(p, d_ws, stream, &c);
  if (st != MSGPM_OK) return st;
  if (!d_rgb1 || !d_rgb2) return fail(MSGPM_E_INVALID, "frame pointer is NULL");
  const void* ptrs[] = {d_rgb1, d_rgb2, d_init_nnf0, d_init_nnf1, d_ws, d_flow0, d_flow1, d_occ0, d_occ1};
  std::string key(reinterpret_cast<const char*>(p), sizeof *p);
  key.append(reinterpret_cast<const char*>(ptrs), sizeof ptrs);
  Aux* aux = nullptr;  // created outside the capture; joins it through the fork event
  if (!c.one_stream && (st = check(aux_stream(&aux), "second stream")) != MSGPM_OK) return st;
  return cached_graph_launch(key, c.s, [&](hipStream_t cs) {
    Ctx cc = c;
    cc.s = cs;
    return solve_sequence(cc, d_rgb1, d_rgb2, d_init_nnf0, d_init_nnf1, d_flow0, d_flow1, d_occ0, d_occ1);
  });
}

msgpm_status msgpm_graph_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_graphs.mu);
  for (auto& e : g_graphs.entries) (void)hipGraphExecDestroy(e.second);
  g_graphs.entries.clear();
  return MSGPM_OK;
}

}  // extern "C"

// ---- the whole pipeline without allocation ---------------------------------
// The workspace of msgpm_solve_static: one array per device, part of the
// library's device code object, so it exists on every GPU the library runs on
// until the process ends.  Host code never uses its name as an address: the
// array's device address is read once per device (hipGetSymbolAddress, with
// that device current) and kept in g_scratch_ptr.
static_assert(MSGPM_STATIC_WS_BYTES % 256 == 0, "static workspace size");
static __device__ __align__(256) unsigned char scratch[MSGPM_STATIC_WS_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // per device, nullptr until looked up

// Device address of the current device's copy of `scratch`.
msgpm_status scratch_address(void** out) {
  int dev = -1;
  msgpm_status st = check(hipGetDevice(&dev), "current device");
  if (st != MSGPM_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) return fail(MSGPM_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    st = check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "static workspace address");
    if (st != MSGPM_OK) return st;
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255))
      return fail(MSGPM_E_DEVICE, "static workspace address %p not 256-byte aligned", ptr);
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MSGPM_OK;
}

struct NoEvents {
  NoEvents() { g_no_events = true; }
  ~NoEvents() { g_no_events = false; }
};
}  // namespace

extern "C" msgpm_status msgpm_solve_static(const msgpm_params* p, const float* d_rgb1, const float* d_rgb2,
                                           const int32_t* d_init_nnf0, const int32_t* d_init_nnf1,
                                           float* d_flow0, float* d_flow1, uint8_t* d_occ0, uint8_t* d_occ1,
                                           msgpm_plane* d_planes, void* stream) {
  Ctx c;
  msgpm_status st = prepare(p, &c.P, &c.L);
  if (st != MSGPM_OK) return st;
  if (c.L.total_bytes > MSGPM_STATIC_WS_BYTES)
    return fail(MSGPM_E_INVALID, "workspace of %llu bytes for %dx%d exceeds the static workspace of %llu bytes",
                (unsigned long long)c.L.total_bytes, p->width, p->height, (unsigned long long)MSGPM_STATIC_WS_BYTES);
  if (!d_rgb1 || !d_rgb2 || !d_flow0 || !d_flow1 || !d_occ0 || !d_occ1)
    return fail(MSGPM_E_INVALID, "frame or output pointer is NULL");
  void* base = nullptr;
  if ((st = scratch_address(&base)) != MSGPM_OK) return st;
  c.w = make_ws(c.P, c.L, base);
  c.s = static_cast<hipStream_t>(stream);
  c.one_stream = true;  // no second stream: nothing is created
  NoEvents quiet;       // no timing events either
  // every array the pipeline reads is written by it first (features with their
  // pad pixel, initial state, plane records, counters, lists), so what earlier
  // calls left in the array does not matter
  if ((st = solve_sequence(c, d_rgb1, d_rgb2, d_init_nnf0, d_init_nnf1, d_flow0, d_flow1, d_occ0, d_occ1)) !=
      MSGPM_OK)
    return st;
  if (!d_planes) return MSGPM_OK;
  return check(hipMemcpyAsync(d_planes, static_cast<char*>(base) + c.L.planes,
                              (size_t)c.L.n_planes * sizeof(msgpm_plane), hipMemcpyDeviceToDevice, c.s),
               "plane table copy");
}

namespace {

// ---- batched solves ----------------------------------------------------------
struct BatchStep {
  int kind, timer;
  int a[5];
};

// The launch sequence of msgpm_solve, as batched kernel kinds.
std::vector<BatchStep> batch_schedule(const DevParams& P) {
  std::vector<BatchStep> v;
  auto add = [&](int kind, int timer, int a0 = 0, int a1 = 0, int a2 = 0, int a3 = 0) {
    v.push_back(BatchStep{kind, timer, {a0, a1, a2, a3, 0}});
  };
  if (P.histeq) {
    add(BK_HEQ_CLEAR, MSGPM_T_FEATURES);
    add(BK_HEQ_HIST, MSGPM_T_FEATURES);
    add(BK_HEQ_MAP, MSGPM_T_FEATURES);
  }
  add(BK_FEATURES, MSGPM_T_FEATURES);
  add(BK_INIT_PIXELS, MSGPM_T_INIT);
  add(BK_INIT_PLANES, MSGPM_T_INIT);
  // cost refreshes are folded into the first half-sweep of each colour (run
  // alone when a pass has none)
  if (P.iters == 0) add(BK_EVAL_COST_IDENT, MSGPM_T_EVAL_COST, 0);
  for (int it = 0; it < P.iters; ++it)
    for (int colour = 0; colour < 2; ++colour) add(BK_PM_INIT, MSGPM_T_PM_INIT, colour, it, 0, it == 0 ? 2 : 0);
  for (int l = 0; l < P.n_levels; ++l) {
    for (int stage = 1; stage <= 2; ++stage) {
      add(BK_RANSAC, MSGPM_T_RANSAC, l, stage);
      add(BK_ASSIGN, MSGPM_T_ASSIGN, l, stage, 1);
      add(BK_SYMMETRY, MSGPM_T_SYMMETRY, l, stage);
      add(BK_ASSIGN, MSGPM_T_ASSIGN, l, stage, 0);
    }
    add(BK_FB, MSGPM_T_FB);
    add(BK_COMMIT, MSGPM_T_FB);
    if (P.cues & MSGPM_FLAG_CUE_UNIQUE)
      for (int phase = 0; phase < 4; ++phase) add(BK_UNIQUE, MSGPM_T_FB, phase);
    add(BK_NNF_UPDATE, MSGPM_T_NNF_UPDATE, l);
    add(BK_ZERO_ACTIVE, MSGPM_T_PM_LIST);
    for (int colour = 0; colour < 2; ++colour) add(BK_ACTIVE_LIST, MSGPM_T_PM_LIST, colour);
    if (P.iters == 0) {
      add(BK_EVAL_COST_IDENT, MSGPM_T_EVAL_COST, 1);
      add(BK_EVAL_COST_PLANE, MSGPM_T_EVAL_COST, 1);
    }
    for (int it = 0; it < P.iters; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        const int mode = it == 0 ? 3 : 1;
        add(BK_PM_RESTRICTED, MSGPM_T_PM_RESTRICTED, colour, it, l + 1, mode);
        add(BK_PM_RESTRICTED_IDENT, MSGPM_T_PM_RESTRICTED_IDENT, colour, it, l + 1, mode);
      }
  }
  if (P.fill_sweeps > 0) {
    add(BK_FILL_CLEAR, MSGPM_T_FILL);
    for (int t = 0; t < P.fill_sweeps; ++t) add(BK_FILL, MSGPM_T_FILL, t);
  }
  add(BK_EVAL_COST_PLANE, MSGPM_T_EVAL_COST, 2);
  add(BK_FINALIZE, MSGPM_T_FINALIZE);
  return v;
}

// What the pairs of one batched launch sequence must share.
bool same_schedule(const DevParams& a, const DevParams& b) {
  return b.r == a.r && b.C == a.C && b.fp16 == a.fp16 && b.iters == a.iters && b.n_levels == a.n_levels &&
         b.cues == a.cues && b.fill_sweeps == a.fill_sweeps && b.histeq == a.histeq;
}

// Validates a batch and derives each pair's kernel parameters.
msgpm_status batch_prepare(int n, const msgpm_params* params, std::vector<DevParams>& P,
                           std::vector<msgpm_layout>& L) {
  if (n < 1 || n > 4096) return fail(MSGPM_E_INVALID, "batch size %d outside 1..4096", n);
  if (!params) return fail(MSGPM_E_INVALID, "params is NULL");
  P.resize(n);
  L.resize(n);
  for (int i = 0; i < n; ++i) {
    msgpm_status st = prepare(&params[i], &P[i], &L[i]);
    if (st != MSGPM_OK) return fail(st, "pair %d: %s", i, g_err.c_str());
    if (!same_schedule(P[0], P[i]))
      return fail(MSGPM_E_INVALID,
                  "pair %d: a batch needs one patch radius, channel count, storage, iteration count, level count, "
                  "set of occlusion cues, filling length and equalisation setting",
                  i);
  }
  return MSGPM_OK;
}

// Resident workgroups per compute unit of the persistent batched launches, per
// class of kernel and kernel instantiation (msgpm_tuning); entry 0 is the
// default for every instantiation.
std::mutex g_tune_mu;
std::vector<msgpm_tuning> g_tune = {msgpm_tuning{0, 0, -1, {0, 0, 0, 16}}};

bool tune_key_valid(const msgpm_tuning& t) {
  return (t.patch_radius == 0 || (t.patch_radius >= 1 && t.patch_radius <= 4)) &&
         (t.channels == 0 || t.channels == 3 || t.channels == 5) && (t.fp16 >= -1 && t.fp16 <= 1);
}

// The shape for instantiation (r, C, fp16): the most specific stored entry.
msgpm_tuning tune_for(int r, int C, int fp16) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const msgpm_tuning* best = &g_tune[0];
  int score = -1;
  for (const msgpm_tuning& t : g_tune) {
    if ((t.patch_radius && t.patch_radius != r) || (t.channels && t.channels != C) || (t.fp16 >= 0 && t.fp16 != fp16))
      continue;
    const int sc = (t.patch_radius != 0) + (t.channels != 0) + (t.fp16 >= 0);
    if (sc > score) {
      score = sc;
      best = &t;
    }
  }
  return *best;
}

int tune_class(int kind) {
  switch (kind) {
    case BK_PM_INIT:
    case BK_PM_RESTRICTED_IDENT:
    case BK_EVAL_COST_IDENT:
      return MSGPM_TUNE_PM_IDENTITY;
    case BK_PM_RESTRICTED:
    case BK_EVAL_COST_PLANE:
      return MSGPM_TUNE_PM_DISTORTED;
    case BK_RANSAC:
      return MSGPM_TUNE_RANSAC;
    default:
      return MSGPM_TUNE_PIXEL;
  }
}

// Compute units of the current device (cached per device; 256 if unknown).
int device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cache[dev].load();
  if (v > 0) return v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
  cache[dev].store(v);
  return v;
}

// One launch of a plan: its kind and arguments, its item list, its number of
// virtual workgroups and its grid (independent of the pairs: the resident
// workgroups of its class).
struct Launch {
  int kind, timer;
  BArgs A;
  int list, total, grid;
  bool persist;  // loop over the virtual workgroups (else one each, grid = total)
  size_t lds;
};

struct Plan {
  int n = 0;
  std::vector<Launch> launches;
  std::vector<std::vector<Item>> lists;  // distinct item lists, shared by launches
  std::vector<uint64_t> list_off;
  uint64_t desc_off = 0, bytes = 0;
};

Plan make_plan(int n, const std::vector<DevParams>& P, const msgpm_tuning& t, int cus) {
  Plan pl;
  pl.n = n;
  for (const BatchStep& st : batch_schedule(P[0])) {
    std::vector<Item> items(n);
    int start = 0;
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
      Item& it = items[i];
      it.pair = i;
      it.nb = batch_blocks(st.kind, P[i], st.a);
      it.start = start;
      start += (it.nb + kXcds - 1) / kXcds * kXcds;
      if (st.kind == BK_RANSAC) {
        const size_t m = ransac_smem_bytes_window(P[i].block[st.a[0]]);
        lds = m > lds ? m : lds;
      }
    }
    int list = -1;
    for (size_t j = 0; j < pl.lists.size() && list < 0; ++j)
      if (memcmp(pl.lists[j].data(), items.data(), (size_t)n * sizeof(Item)) == 0) list = (int)j;
    if (list < 0) {
      list = (int)pl.lists.size();
      pl.lists.push_back(items);
    }
    Launch L;
    L.kind = st.kind;
    L.timer = st.timer;
    for (int k = 0; k < 5; ++k) L.A.a[k] = st.a[k];
    L.list = list;
    L.total = start;
    L.lds = lds;
    const int w = t.wg_per_cu[tune_class(st.kind)];
    L.persist = true;
    if (st.kind == BK_ZERO_ACTIVE) {
      L.grid = kXcds;
    } else if (w == 0) {
      L.grid = start;  // one workgroup per virtual workgroup
      L.persist = false;
    } else {
      const long g = (long)w * cus;
      L.grid = (int)((g + kXcds - 1) / kXcds * kXcds);
    }
    pl.launches.push_back(L);
  }
  uint64_t off = align256(sizeof(BatchHead) + pl.launches.size() * sizeof(LaunchTab));
  pl.desc_off = off;
  off = align256(off + (uint64_t)n * sizeof(PairDesc));
  for (const auto& l : pl.lists) {
    pl.list_off.push_back(off);
    off += (uint64_t)l.size() * sizeof(Item);
  }
  pl.bytes = align256(off);
  return pl;
}

// The plan's table (header, launch entries, descriptors, item lists) at h.
void write_tables(const Plan& pl, const PairDesc* desc, char* h) {
  BatchHead hd;
  hd.n_launches = (int)pl.launches.size();
  hd.n_pairs = pl.n;
  hd.desc_off = (uint32_t)pl.desc_off;
  hd.pad = 0;
  memcpy(h, &hd, sizeof hd);
  LaunchTab* L = reinterpret_cast<LaunchTab*>(h + sizeof(BatchHead));
  for (size_t k = 0; k < pl.launches.size(); ++k) {
    L[k].total = pl.launches[k].total;
    L[k].items = (uint32_t)pl.list_off[pl.launches[k].list];
  }
  memcpy(h + pl.desc_off, desc, (size_t)pl.n * sizeof(PairDesc));
  for (size_t j = 0; j < pl.lists.size(); ++j)
    memcpy(h + pl.list_off[j], pl.lists[j].data(), pl.lists[j].size() * sizeof(Item));
}

// The plan's launches on s, reading the table at dev.
msgpm_status run_plan(const Plan& pl, const DevParams& P0, const uint8_t* dev, hipStream_t s) {
  for (size_t k = 0; k < pl.launches.size(); ++k) {
    const Launch& L = pl.launches[k];
    msgpm_status st = check(
        timed(L.timer, s, [&] { return launch_batched(L.kind, P0, dev, (int)k, L.grid, L.lds, L.A, L.persist, s); }),
        "batched launch");
    if (st != MSGPM_OK) return st;
  }
  return MSGPM_OK;
}

// The plan's launches as one graph launch on s: the graph depends only on the
// launch sequence, the kernel instantiation and the table's address, so it is
// captured once and serves any set of pairs with that schedule.
msgpm_status run_plan_graph(const Plan& pl, const DevParams& P0, const uint8_t* dev, hipStream_t s) {
  std::string key("batch");
  const int inst[3] = {P0.r, P0.C, P0.fp16};
  key.append(reinterpret_cast<const char*>(inst), sizeof inst);
  key.append(reinterpret_cast<const char*>(&dev), sizeof dev);
  for (const Launch& L : pl.launches) {
    const int64_t rec[9] = {L.kind, L.A.a[0], L.A.a[1], L.A.a[2], L.A.a[3], L.A.a[4], L.grid, (int64_t)L.lds,
                            L.persist};
    key.append(reinterpret_cast<const char*>(rec), sizeof rec);
  }
  return cached_graph_launch(key, s, [&](hipStream_t cs) { return run_plan(pl, P0, dev, cs); });
}

// Pinned staging buffer for the table upload of msgpm_solve_batch; reused
// once the previous upload (recorded by `done`) has completed.
struct Staging {
  std::mutex mu;
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
};
Staging g_staging;

msgpm_status batch_run(int n, const msgpm_params* params, const float* const* d_rgb1, const float* const* d_rgb2,
                       const int32_t* const* d_init_nnf0, const int32_t* const* d_init_nnf1, void* const* d_ws,
                       float* const* d_flow0, float* const* d_flow1, uint8_t* const* d_occ0, uint8_t* const* d_occ1,
                       void* d_scratch, void* stream, bool graph) {
  std::vector<DevParams> P;
  std::vector<msgpm_layout> L;
  msgpm_status st = batch_prepare(n, params, P, L);
  if (st != MSGPM_OK) return st;
  if (!d_rgb1 || !d_rgb2 || !d_ws || !d_flow0 || !d_flow1 || !d_occ0 || !d_occ1)
    return fail(MSGPM_E_INVALID, "pointer array is NULL");
  if (!d_scratch || (reinterpret_cast<uintptr_t>(d_scratch) & 255))
    return fail(MSGPM_E_INVALID, "scratch is NULL or not 256-byte aligned");
  std::vector<PairDesc> desc(n);
  for (int i = 0; i < n; ++i) {
    if (!d_ws[i] || (reinterpret_cast<uintptr_t>(d_ws[i]) & 255))
      return fail(MSGPM_E_INVALID, "pair %d: workspace is NULL or not 256-byte aligned", i);
    if (!d_rgb1[i] || !d_rgb2[i] || !d_flow0[i] || !d_flow1[i] || !d_occ0[i] || !d_occ1[i])
      return fail(MSGPM_E_INVALID, "pair %d: frame or output pointer is NULL", i);
    memset(&desc[i], 0, sizeof(PairDesc));
    desc[i].P = P[i];
    desc[i].w = make_ws(P[i], L[i], d_ws[i]);
    desc[i].rgb[0] = d_rgb1[i];
    desc[i].rgb[1] = d_rgb2[i];
    desc[i].init[0] = d_init_nnf0 ? d_init_nnf0[i] : nullptr;
    desc[i].init[1] = d_init_nnf1 ? d_init_nnf1[i] : nullptr;
    desc[i].flow[0] = d_flow0[i];
    desc[i].flow[1] = d_flow1[i];
    desc[i].occ[0] = d_occ0[i];
    desc[i].occ[1] = d_occ1[i];
  }
  const msgpm_tuning t = tune_for(P[0].r, P[0].C, P[0].fp16);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* dev = static_cast<char*>(d_scratch);
  {
    std::lock_guard<std::mutex> lk(g_staging.mu);
    const Plan plan = make_plan(n, P, t, 256);  // the table's size does not depend on the grids
    if (g_staging.done && (st = check(hipEventSynchronize(g_staging.done), "staging")) != MSGPM_OK) return st;
    if (g_staging.cap < plan.bytes) {
      if (g_staging.host) (void)hipHostFree(g_staging.host);
      g_staging.host = nullptr;
      g_staging.cap = 0;
      if ((st = check(host_alloc(&g_staging.host, plan.bytes), "staging")) != MSGPM_OK) return st;
      g_staging.cap = plan.bytes;
    }
    if (!g_staging.done && (st = check(event_create(&g_staging.done), "staging")) != MSGPM_OK) return st;
    const Plan run = make_plan(n, P, t, device_cus());
    write_tables(run, desc.data(), static_cast<char*>(g_staging.host));
    if ((st = check(hipMemcpyAsync(dev, g_staging.host, run.bytes, hipMemcpyHostToDevice, s), "upload")) != MSGPM_OK)
      return st;
    if ((st = check(hipEventRecord(g_staging.done, s), "staging")) != MSGPM_OK) return st;
    const uint8_t* tab = reinterpret_cast<const uint8_t*>(dev);
    return graph ? run_plan_graph(run, P[0], tab, s) : run_plan(run, P[0], tab, s);
  }
}

}  // namespace

extern "C" {

msgpm_status msgpm_batch_query(int n, const msgpm_params* params, uint64_t* scratch_bytes) {
  if (!scratch_bytes) return fail(MSGPM_E_INVALID, "scratch_bytes is NULL");
  std::vector<DevParams> P;
  std::vector<msgpm_layout> L;
  msgpm_status st = batch_prepare(n, params, P, L);
  if (st != MSGPM_OK) return st;
  *scratch_bytes = make_plan(n, P, tune_for(P[0].r, P[0].C, P[0].fp16), 256).bytes;
  return MSGPM_OK;
}

msgpm_status msgpm_solve_batch(int n, const msgpm_params* params, const float* const* d_rgb1,
                               const float* const* d_rgb2, const int32_t* const* d_init_nnf0,
                               const int32_t* const* d_init_nnf1, void* const* d_ws, float* const* d_flow0,
                               float* const* d_flow1, uint8_t* const* d_occ0, uint8_t* const* d_occ1,
                               void* d_scratch, void* stream) {
  return batch_run(n, params, d_rgb1, d_rgb2, d_init_nnf0, d_init_nnf1, d_ws, d_flow0, d_flow1, d_occ0, d_occ1,
                   d_scratch, stream, false);
}

msgpm_status msgpm_solve_batch_graph(int n, const msgpm_params* params, const float* const* d_rgb1,
                                     const float* const* d_rgb2, const int32_t* const* d_init_nnf0,
                                     const int32_t* const* d_init_nnf1, void* const* d_ws, float* const* d_flow0,
                                     float* const* d_flow1, uint8_t* const* d_occ0, uint8_t* const* d_occ1,
                                     void* d_scratch, void* stream) {
  return batch_run(n, params, d_rgb1, d_rgb2, d_init_nnf0, d_init_nnf1, d_ws, d_flow0, d_flow1, d_occ0, d_occ1,
                   d_scratch, stream, true);
}

msgpm_status msgpm_tuning_set(const msgpm_tuning* t) {
  if (!t) return fail(MSGPM_E_INVALID, "tuning is NULL");
  if (!tune_key_valid(*t)) return fail(MSGPM_E_INVALID, "tuning instantiation (r, C, fp16) invalid");
  for (int c = 0; c < MSGPM_TUNE_CLASSES; ++c)
    if (t->wg_per_cu[c] < 0 || t->wg_per_cu[c] > 64)
      return fail(MSGPM_E_INVALID, "wg_per_cu[%d] = %d outside 0..64", c, t->wg_per_cu[c]);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (msgpm_tuning& e : g_tune)
    if (e.patch_radius == t->patch_radius && e.channels == t->channels && e.fp16 == t->fp16) {
      e = *t;
      return MSGPM_OK;
    }
  if (g_tune.size() >= 64) return fail(MSGPM_E_INVALID, "too many tuning entries");
  g_tune.push_back(*t);
  return MSGPM_OK;
}

msgpm_status msgpm_tuning_get(msgpm_tuning* t) {
  if (!t) return fail(MSGPM_E_INVALID, "tuning is NULL");
  if (!tune_key_valid(*t)) return fail(MSGPM_E_INVALID, "tuning instantiation (r, C, fp16) invalid");
  const msgpm_tuning f = tune_for(t->patch_radius, t->channels, t->fp16);
  for (int c = 0; c < MSGPM_TUNE_CLASSES; ++c) t->wg_per_cu[c] = f.wg_per_cu[c];
  return MSGPM_OK;
}

msgpm_status msgpm_check_fp16_arith(int32_t rounds, uint64_t* d_mismatches, void* stream) {
  if (rounds < 1 || rounds > 4096 || !d_mismatches) return fail(MSGPM_E_INVALID, "rounds outside 1..4096 or NULL output");
  if (reinterpret_cast<uintptr_t>(d_mismatches) & 7) return fail(MSGPM_E_INVALID, "output not 8-byte aligned");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(MSGPM_E_DEVICE, "no device");
  return check(launch_check_fp16_arith(rounds, reinterpret_cast<unsigned long long*>(d_mismatches),
                                       static_cast<hipStream_t>(stream)),
               "check_fp16_arith");
}

msgpm_status msgpm_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  g_timer.on = on != 0;
  return MSGPM_OK;
}

msgpm_status msgpm_timing_read(double* ms, int64_t* launches) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  double t[MSGPM_TIMER_KINDS] = {0};
  int64_t n[MSGPM_TIMER_KINDS] = {0};
  for (size_t i = 0; i < g_timer.kinds.size(); ++i) {
    hipEvent_t a = g_timer.pool[2 * i], b = g_timer.pool[2 * i + 1];
    hipError_t e = hipEventSynchronize(b);
    float dt = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&dt, a, b);
    if (e != hipSuccess) {
      g_timer.kinds.clear();
      g_timer.used = 0;
      return check(e, "timing_read");
    }
    t[g_timer.kinds[i]] += dt;
    n[g_timer.kinds[i]] += 1;
  }
  g_timer.kinds.clear();
  g_timer.used = 0;
  for (int k = 0; k < MSGPM_TIMER_KINDS; ++k) {
    if (ms) ms[k] = t[k];
    if (launches) launches[k] = n[k];
  }
  return MSGPM_OK;
}

}  // extern "C"

// ---- serving: continuous batching in cohorts ----------------------------------
// Each msgpm_server_step admits the queued pairs that fit (first come, first
// served, one schedule per cohort) as one cohort and enqueues its whole
// pipeline as one batched graph launch on one of the server's streams; up to
// max_cohorts (at most kCohorts) cohorts run on the device side by side, each with its own region
// of the caller's scratch for its table.
namespace {

constexpr int kCohorts = MSGPM_SERVER_MAX_COHORTS;  // cohorts in flight at most (and server streams)
constexpr int kMaxLaunches = 4096;   // launches of one pipeline a region holds
constexpr int kMaxLists = 48;        // distinct item lists of one pipeline

struct Slot {
  uint64_t ticket = 0;
  DevParams P;
  PairDesc desc;
  uint64_t bytes = 0;     // workspace footprint counted against the budget
  int state = 0;          // 0 queued, 1 in flight, 3 finished
  int cohort = -1;        // while in flight
  bool cancelled = false; // reported as cancelled when finished
};

struct Cohort {
  bool busy = false;
  std::vector<Slot*> pairs;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, done = nullptr;
  void* host = nullptr;  // pinned staging of its table
};

uint64_t region_bytes(int max_active) {
  return align256(sizeof(BatchHead) + (uint64_t)kMaxLaunches * sizeof(LaunchTab)) +
         align256((uint64_t)max_active * sizeof(PairDesc)) + align256((uint64_t)kMaxLists * max_active * sizeof(Item));
}

}  // namespace

struct msgpm_server {
  std::mutex mu;
  uint64_t budget = 0;
  int max_active = 0;
  int max_queued = 0;  // 0 = no limit
  int max_cohorts = kCohorts;  // cohorts in flight at most
  uint64_t next_ticket = 1;
  uint64_t in_use = 0;
  int in_flight = 0;
  bool shape_set = false;
  int r = 0, C = 0, fp16 = 0;
  std::deque<Slot*> queue;
  std::map<uint64_t, Slot*> slots;
  Cohort cohorts[kCohorts];
  int next = 0;  // cohort region tried first
};

namespace {

// Finishes the cohorts whose work has completed: their pairs are done and
// their budget is free.
void server_retire(msgpm_server* sv) {
  for (Cohort& c : sv->cohorts) {
    if (!c.busy || hipEventQuery(c.done) != hipSuccess) continue;
    for (Slot* q : c.pairs) {
      q->state = 3;
      q->cohort = -1;
      sv->in_use -= q->bytes;
      --sv->in_flight;
    }
    c.pairs.clear();
    c.busy = false;
  }
}

// The cohort's objects, created on its first use (so that a failure leaves
// nothing enqueued): pinned staging, events, stream.
msgpm_status cohort_objects(msgpm_server* sv, Cohort& c) {
  msgpm_status st;
  if (!c.host && (st = check(host_alloc(&c.host, region_bytes(sv->max_active)), "staging")) != MSGPM_OK) return st;
  if (!c.fork && (st = check(event_create(&c.fork), "event")) != MSGPM_OK) return st;
  if (!c.done && (st = check(event_create(&c.done), "event")) != MSGPM_OK) return st;
  if (!c.s && (st = check(hipStreamCreateWithFlags(&c.s, hipStreamNonBlocking), "server stream")) != MSGPM_OK)
    return st;
  return MSGPM_OK;
}

// Retires a finished ticket; true if it was cancelled.
bool server_forget(msgpm_server* sv, std::map<uint64_t, Slot*>::iterator f) {
  const bool cancelled = f->second->cancelled;
  delete f->second;
  sv->slots.erase(f);
  return cancelled;
}

}  // namespace

extern "C" {

msgpm_status msgpm_server_create(uint64_t hbm_budget, int max_active, msgpm_server** out) {
  if (!out) return fail(MSGPM_E_INVALID, "out is NULL");
  if (max_active < 1 || max_active > 4096) return fail(MSGPM_E_INVALID, "max_active outside 1..4096");
  msgpm_server* sv = new msgpm_server;
  sv->budget = hbm_budget;
  sv->max_active = max_active;
  *out = sv;
  return MSGPM_OK;
}

msgpm_status msgpm_server_destroy(msgpm_server* sv) {
  if (!sv) return MSGPM_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (Cohort& c : sv->cohorts) {
      if (c.busy) (void)hipEventSynchronize(c.done);
      if (c.done) (void)hipEventDestroy(c.done);
      if (c.fork) (void)hipEventDestroy(c.fork);
      if (c.s) (void)hipStreamDestroy(c.s);
      if (c.host) (void)hipHostFree(c.host);
    }
    for (auto& kv : sv->slots) delete kv.second;
  }
  delete sv;
  return MSGPM_OK;
}

msgpm_status msgpm_server_scratch_bytes(int max_active, uint64_t* bytes) {
  if (!bytes || max_active < 1 || max_active > 4096) return fail(MSGPM_E_INVALID, "bad arguments");
  *bytes = kCohorts * region_bytes(max_active);
  return MSGPM_OK;
}

msgpm_status msgpm_server_submit(msgpm_server* sv, const msgpm_params* p, const float* d_rgb1, const float* d_rgb2,
                                 const int32_t* d_init_nnf0, const int32_t* d_init_nnf1, void* d_ws,
                                 float* d_flow0, float* d_flow1, uint8_t* d_occ0, uint8_t* d_occ1,
                                 uint64_t* ticket) {
  if (!sv || !ticket) return fail(MSGPM_E_INVALID, "server or ticket is NULL");
  Slot* q = new Slot;
  msgpm_layout L;
  msgpm_status st = prepare(p, &q->P, &L);
  if (st != MSGPM_OK) {
    delete q;
    return st;
  }
  if (!d_ws || (reinterpret_cast<uintptr_t>(d_ws) & 255) || !d_rgb1 || !d_rgb2 || !d_flow0 || !d_flow1 || !d_occ0 ||
      !d_occ1) {
    delete q;
    return fail(MSGPM_E_INVALID, "NULL or misaligned buffer");
  }
  const size_t steps = batch_schedule(q->P).size();
  if (steps > (size_t)kMaxLaunches) {
    delete q;
    return fail(MSGPM_E_UNSUPPORTED, "a served pipeline has at most %d launches (these parameters give %zu)",
                kMaxLaunches, steps);
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  if (!sv->shape_set) {
    sv->r = q->P.r;
    sv->C = q->P.C;
    sv->fp16 = q->P.fp16;
    sv->shape_set = true;
  } else if (q->P.r != sv->r || q->P.C != sv->C || q->P.fp16 != sv->fp16) {
    delete q;
    return fail(MSGPM_E_INVALID, "a server serves one patch radius, channel count and storage");
  }
  q->bytes = L.total_bytes;
  if (q->bytes > sv->budget) {
    delete q;
    return fail(MSGPM_E_OOM, "workspace of %llu bytes exceeds the budget of %llu", (unsigned long long)L.total_bytes,
                (unsigned long long)sv->budget);
  }
  if (sv->max_queued > 0 && (int)sv->queue.size() >= sv->max_queued) {
    delete q;
    return fail(MSGPM_E_BUSY, "queue full (%d pairs waiting)", (int)sv->queue.size());
  }
  memset(&q->desc, 0, sizeof q->desc);
  q->desc.P = q->P;
  q->desc.w = make_ws(q->P, L, d_ws);
  q->desc.rgb[0] = d_rgb1;
  q->desc.rgb[1] = d_rgb2;
  q->desc.init[0] = d_init_nnf0;
  q->desc.init[1] = d_init_nnf1;
  q->desc.flow[0] = d_flow0;
  q->desc.flow[1] = d_flow1;
  q->desc.occ[0] = d_occ0;
  q->desc.occ[1] = d_occ1;
  q->ticket = sv->next_ticket++;
  sv->queue.push_back(q);
  sv->slots[q->ticket] = q;
  *ticket = q->ticket;
  return MSGPM_OK;
}

msgpm_status msgpm_server_step(msgpm_server* sv, void* d_scratch, void* stream, int* pending) {
  if (!sv || !d_scratch || (reinterpret_cast<uintptr_t>(d_scratch) & 255))
    return fail(MSGPM_E_INVALID, "server NULL or scratch NULL / misaligned");
  std::lock_guard<std::mutex> lk(sv->mu);
  msgpm_status st = MSGPM_OK;
  server_retire(sv);
  if (pending) *pending = (int)sv->queue.size() + sv->in_flight;
  if (sv->queue.empty()) return MSGPM_OK;
  int ci = -1, busy = 0;
  for (int k = 0; k < kCohorts; ++k) {
    const int c = (sv->next + k) % kCohorts;
    if (sv->cohorts[c].busy)
      ++busy;
    else if (ci < 0)
      ci = c;
  }
  // every region in use, or the cohort limit reached: admitted at a later step
  if (ci < 0 || busy >= sv->max_cohorts) return MSGPM_OK;
  // the cohort: queued pairs with the head's schedule, first come first served,
  // while the budget and the in-flight limit allow
  std::vector<Slot*> take;
  uint64_t bytes = 0;
  const DevParams head = sv->queue.front()->P;
  for (Slot* q : sv->queue) {
    if (!same_schedule(head, q->P)) continue;
    if (sv->in_flight + (int)take.size() >= sv->max_active || sv->in_use + bytes + q->bytes > sv->budget) break;
    take.push_back(q);
    bytes += q->bytes;
  }
  if (take.empty()) return MSGPM_OK;
  Cohort& c = sv->cohorts[ci];
  if ((st = cohort_objects(sv, c)) != MSGPM_OK) return st;
  const msgpm_tuning t = tune_for(head.r, head.C, head.fp16);
  const int n = (int)take.size();
  std::vector<DevParams> P(n);
  std::vector<PairDesc> desc(n);
  for (int i = 0; i < n; ++i) {
    P[i] = take[i]->P;
    desc[i] = take[i]->desc;
  }
  const Plan plan = make_plan(n, P, t, device_cus());
  if ((int)plan.lists.size() > kMaxLists || plan.bytes > region_bytes(sv->max_active))
    return fail(MSGPM_E_UNSUPPORTED, "cohort table of %llu bytes does not fit its region",
                (unsigned long long)plan.bytes);
  write_tables(plan, desc.data(), static_cast<char*>(c.host));
  uint8_t* dev = static_cast<uint8_t*>(d_scratch) + (uint64_t)ci * region_bytes(sv->max_active);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // ordered after the caller's work so far (its frames), then on its own stream
  if ((st = check(hipEventRecord(c.fork, s), "fork")) != MSGPM_OK) return st;
  if ((st = check(hipStreamWaitEvent(c.s, c.fork, 0), "fork")) != MSGPM_OK) return st;
  if ((st = check(hipMemcpyAsync(dev, c.host, plan.bytes, hipMemcpyHostToDevice, c.s), "upload")) != MSGPM_OK)
    return st;
  if ((st = run_plan_graph(plan, P[0], dev, c.s)) != MSGPM_OK) return st;
  if ((st = check(hipEventRecord(c.done, c.s), "event")) != MSGPM_OK) return st;
  for (Slot* q : take) {
    q->state = 1;
    q->cohort = ci;
    c.pairs.push_back(q);
    for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it)
      if (*it == q) {
        sv->queue.erase(it);
        break;
      }
  }
  c.busy = true;
  sv->in_use += bytes;
  sv->in_flight += n;
  sv->next = (ci + 1) % kCohorts;
  if (pending) *pending = (int)sv->queue.size() + sv->in_flight;
  return MSGPM_OK;
}

msgpm_status msgpm_server_cancel(msgpm_server* sv, uint64_t ticket, int* retired) {
  if (!sv) return fail(MSGPM_E_INVALID, "server is NULL");
  if (retired) *retired = 0;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto f = sv->slots.find(ticket);
  if (f == sv->slots.end()) return fail(MSGPM_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  Slot* q = f->second;
  if (q->state == 0) {  // still queued: nothing was enqueued for it
    for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it)
      if (*it == q) {
        sv->queue.erase(it);
        break;
      }
    server_forget(sv, f);
    if (retired) *retired = 1;
  } else if (q->state == 1) {
    q->cancelled = true;
  }
  return MSGPM_OK;
}

msgpm_status msgpm_server_set_queue_limit(msgpm_server* sv, int max_queued) {
  if (!sv || max_queued < 0) return fail(MSGPM_E_INVALID, "server is NULL or limit negative");
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->max_queued = max_queued;
  return MSGPM_OK;
}

msgpm_status msgpm_server_set_cohorts(msgpm_server* sv, int cohorts) {
  if (!sv || cohorts < 1 || cohorts > kCohorts)
    return fail(MSGPM_E_INVALID, "server is NULL or cohorts outside 1..%d", kCohorts);
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->max_cohorts = cohorts;
  return MSGPM_OK;
}

msgpm_status msgpm_server_wait(msgpm_server* sv, uint64_t ticket, int64_t timeout_us) {
  if (!sv) return fail(MSGPM_E_INVALID, "server is NULL");
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      auto f = sv->slots.find(ticket);
      if (f == sv->slots.end()) return fail(MSGPM_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
      if (f->second->state == 1) server_retire(sv);
      if (f->second->state == 3) {
        if (server_forget(sv, f)) return fail(MSGPM_E_CANCELLED, "ticket %llu was cancelled", (unsigned long long)ticket);
        return MSGPM_OK;
      }
    }
    const int64_t waited =
        std::chrono::duration_cast<std::chrono::microseconds>(std::chrono::steady_clock::now() - t0).count();
    if (timeout_us >= 0 && waited >= timeout_us)
      return fail(MSGPM_E_TIMEOUT, "ticket %llu not done after %lld us", (unsigned long long)ticket,
                  (long long)waited);
    int64_t nap = 50;
    if (timeout_us >= 0 && timeout_us - waited < nap) nap = timeout_us - waited;
    std::this_thread::sleep_for(std::chrono::microseconds(nap));
  }
}

msgpm_status msgpm_debug_fail_allocations(int n) {
  g_fail_allocs.store(n > 0 ? n : 0);
  return MSGPM_OK;
}

msgpm_status msgpm_server_poll(msgpm_server* sv, uint64_t ticket, int* done) {
  if (!sv || !done) return fail(MSGPM_E_INVALID, "server or done is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto f = sv->slots.find(ticket);
  if (f == sv->slots.end()) return fail(MSGPM_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  if (f->second->state == 1) server_retire(sv);
  *done = f->second->state == 3;
  if (*done) server_forget(sv, f);
  return MSGPM_OK;
}

}  // extern "C"
