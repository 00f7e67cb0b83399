// Host runtime and C ABI of lpgpu (declared in include/lpgpu.h).
//
// The handle owns the device state of one LP.  An iteration is the kernel chain
// k_price -> k_update -> k_finish (k_price32 -> k_shortlist -> k_update -> k_finish in the
// mixed form); lp_solve captures iters_per_sync such chains once into a HIP graph and
// replays it, reading back only the small control block after each replay
// (the status scalar plus counters).  The kernels themselves stop doing work once the
// status leaves RUNNING, so a replay that overshoots the end of the solve is harmless.
// Near a pivot cap, shorter graphs of 1, 2, 4, ... iterations are replayed instead, so
// that no replay runs iterations past the cap.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lp_device.h"
#include "lp_reinv.h"
#include "lpgpu.h"

using namespace lpgpu;

// Device memory of lp_solve_device_noalloc: one array per GPU, alive until the process
// ends.  Host code never passes this name to a kernel or a copy (on the host it is only a
// stand-in for the symbol): it uses the address hipGetSymbolAddress returns for the
// current device.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_msg;
thread_local int g_code = 0;

int fail(int code, const std::string& msg) {
  g_code = code;
  g_msg = msg;
  return code;
}

}  // namespace

namespace lpgpu {
int record_error(int code, const std::string& msg) { return fail(code, msg); }

// Called from a catch-all handler: an exception of host code (an allocation that failed, a
// thread that could not start) becomes LP_ERR_NOMEM, since nothing may unwind through the
// C ABI.
int host_exception() noexcept {
  try {
    try {
      throw;
    } catch (const std::bad_alloc&) {
      return fail(LP_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception& e) {
      return fail(LP_ERR_NOMEM, std::string("host resources exhausted: ") + e.what());
    } catch (...) {
      return fail(LP_ERR_NOMEM, "unexpected host exception");
    }
  } catch (...) {  // the message itself could not be stored
    g_code = LP_ERR_NOMEM;
    g_msg.clear();
    return LP_ERR_NOMEM;
  }
}
}  // namespace lpgpu

namespace {

int fail_hip(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(LP_ERR_NOMEM, std::string(what) + ": " + hipGetErrorString(e));
  return fail(LP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Transfers between pageable host memory and the device: the stream is drained, then a
// blocking copy runs, so the copy follows the stream's earlier work and is complete on
// return, whatever kind of stream the caller gave.  (Pinned control-block traffic and
// device-to-device copies stay asynchronous on the stream.)
hipError_t pageable_copy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s) {
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess && bytes > 0) e = hipMemcpy(dst, src, bytes, kind);
  return e;
}

// Order-independent 64-bit hash of the bit patterns of `count` doubles whose first one sits
// at element `base` of an array: the wrapping sum of a SplitMix64 finaliser of (bits,
// index), so a device kernel can form it in any order and compare it with this value.
uint64_t hash_doubles(const double* x, size_t count, uint64_t base) {
  uint64_t h = 0;
  for (size_t k = 0; k < count; ++k) {
    uint64_t bits;
    std::memcpy(&bits, &x[k], sizeof(bits));
    h += hash_word(bits, base + k);
  }
  return h;
}

#define HIP_TRY(expr, what)                   \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return fail_hip(e_, what); \
  } while (0)

int64_t round_up(int64_t x, int64_t k) { return (x + k - 1) / k * k; }

// Runs f when the scope ends, by a return or by an exception.
template <class F>
struct ScopeExit {
  F f;
  ~ScopeExit() { f(); }
};
template <class F>
ScopeExit<F> on_scope_exit(F f) {
  return {f};
}

}  // namespace

struct lp_problem {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  lp_options opt{};
  int32_t m = 0, n = 0, ld = 0;
  DevLP d{};
  std::vector<void*> allocs;
  double* b0 = nullptr;  // device copies of b and c, kept for lp_reset
  double* c0 = nullptr;
  std::vector<double> hc;  // host copy of c for the reported objective
  Ctrl* h_ctrl = nullptr;  // pinned mirror of the control block
  Ctrl* h_stage = nullptr; // pinned staging for host -> device control writes
  int num_cu = 0;
  int price_grid = 1, update_grid = 1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_k = 0;
  // tail graphs: 2^k iterations each, for the last replays before a pivot cap
  hipGraph_t tail_graph[12] = {};
  hipGraphExec_t tail_exec[12] = {};
  std::vector<hipEvent_t> events;
  lp_stats stats{};
  int price32_grid = 0;    // mixed form
  int reinv_period = 0;    // resolved opt.reinv_period
  int64_t last_reinv_t = 0;
  ReinvState* rv = nullptr;
  hipEvent_t rv_ev[2] = {nullptr, nullptr};
  bool rv_timing = false;  // a reinversion's events are waiting to be read
  // Two-phase start (lp_create_general); n_user == n and phase == 0 otherwise.
  int32_t n_user = 0;       // the caller's columns; n_user..n-1 are surplus columns
  int phase = 0;            // 0: one phase; 1: phase 1 running; 2: phase 2
  bool two_phase = false;   // phase 1 is needed (some row has an artificial variable)
  std::vector<double> rsign;     // -1 for rows multiplied by -1
  std::vector<int8_t> art_h;     // art_h[i]: the unit column of row i is artificial
  double eps_f = 0.0;
  double* chat1 = nullptr;  // phase-1 costs (device)
  double* chat2 = nullptr;  // the LP's own costs (device)
  double* tab_t = nullptr;  // drive-out scratch: per-workgroup tableau-row candidates
  int32_t* tab_j = nullptr;
  int32_t* drive = nullptr;
  int64_t phase1_t = -1;
  int64_t drive_outs = 0;
  double switch_ms = 0.0;
  // Out-of-core panel mode (Section 3, Case 2): B^-1 in pinned host memory, streamed in
  // panels of panel_rows rows; the last panel (rows res_lo..m-1) stays on the device.
  bool panel = false;
  int panel_rows = 0, npanels = 0, res_lo = 0;
  double* binv_host = nullptr;      // m x ld, pinned
  double* binv_host_dev = nullptr;  // its address for kernels
  double* pbuf[2] = {nullptr, nullptr};
  double* res = nullptr;
  double* rowbuf = nullptr;  // row r of B^-1 for the pricing kernel
};

namespace {

template <class T>
hipError_t dalloc(lp_problem* p, T** out, size_t count) {
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    *out = nullptr;
    return e;
  }
  p->allocs.push_back(ptr);
  *out = static_cast<T*>(ptr);
  return hipSuccess;
}

void dfree(lp_problem* p, void* ptr) {
  if (!ptr) return;
  auto it = std::find(p->allocs.begin(), p->allocs.end(), ptr);
  if (it != p->allocs.end()) p->allocs.erase(it);
  (void)hipFree(ptr);
}

void drop_graph(lp_problem* p) {
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
  p->graph_k = 0;
  for (int k = 0; k < 12; ++k) {
    if (p->tail_exec[k]) (void)hipGraphExecDestroy(p->tail_exec[k]);
    if (p->tail_graph[k]) (void)hipGraphDestroy(p->tail_graph[k]);
    p->tail_exec[k] = nullptr;
    p->tail_graph[k] = nullptr;
  }
  for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
  p->events.clear();
}

void release(lp_problem* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  drop_graph(p);
  for (void* ptr : p->allocs) (void)hipFree(ptr);
  p->allocs.clear();
  if (p->h_ctrl) (void)hipHostFree(p->h_ctrl);
  if (p->h_stage) (void)hipHostFree(p->h_stage);
  if (p->binv_host) (void)hipHostFree(p->binv_host);
  reinv_free(p->rv);
  for (hipEvent_t e : p->rv_ev)
    if (e) (void)hipEventDestroy(e);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

int check_options(const lp_options* o) {
  if (o->sense != LP_MIN && o->sense != LP_MAX) return fail(LP_ERR_ARG, "options.sense must be LP_MIN or LP_MAX");
  if (o->tabu_tenure < 0) return fail(LP_ERR_ARG, "options.tabu_tenure must be >= 0");
  if (o->iters_per_sync < 1 || o->iters_per_sync > 4096)
    return fail(LP_ERR_ARG, "options.iters_per_sync must be in [1, 4096]");
  if (o->max_iter < 0) return fail(LP_ERR_ARG, "options.max_iter must be >= 0");
  if (o->profile < 0 || o->profile > 2) return fail(LP_ERR_ARG, "options.profile must be 0, 1 or 2");
  if (o->precision != LP_FP64 && o->precision != LP_MIXED)
    return fail(LP_ERR_ARG, "options.precision must be LP_FP64 or LP_MIXED");
  if (o->shortlist_k < 1 || o->shortlist_k > kShortlist) return fail(LP_ERR_ARG, "options.shortlist_k must be in [1, 16]");
  if (o->reinv_period < -1) return fail(LP_ERR_ARG, "options.reinv_period must be >= -1");
  if (o->device_budget < 0) return fail(LP_ERR_ARG, "options.device_budget must be >= 0");
  if (!(o->eps_d >= 0.0) || !(o->eps_p >= 0.0) || !(o->eps_z >= 0.0) || !(o->eps_t >= 0.0) ||
      !std::isfinite(o->eps_d) || !std::isfinite(o->eps_p) || !std::isfinite(o->eps_z) || !std::isfinite(o->eps_t))
    return fail(LP_ERR_ARG, "options.eps_* must be finite and >= 0");
  return LP_OK;
}

// Pivot log and tabu-list storage sized for `cap` pivots; keeps existing entries.
int ensure_capacity(lp_problem* p, int64_t cap) {
  cap = std::max<int64_t>(cap, 1);
  if (cap <= p->d.log_cap && cap <= p->d.Lcap) return LP_OK;
  if (cap > INT32_MAX) return fail(LP_ERR_ARG, "pivot limit above 2^31-1");
  const int64_t keep_log = std::min<int64_t>(p->h_ctrl ? p->h_ctrl->t : 0, p->d.log_cap);
  const int64_t keep_L = p->h_ctrl ? std::min<int64_t>(p->h_ctrl->nL, p->d.Lcap) : 0;
  int32_t* arrs[7] = {nullptr};
  for (int k = 0; k < 7; ++k) HIP_TRY(dalloc(p, &arrs[k], (size_t)cap), "allocating the pivot log");
  int32_t* old[7] = {p->d.log_enter, p->d.log_row, p->d.log_leave, p->d.log_flags, p->d.Lq, p->d.Ll, p->d.Lgen};
  for (int k = 0; k < 7; ++k) {
    const int64_t keep = k < 4 ? keep_log : keep_L;
    if (old[k] && keep > 0)
      HIP_TRY(hipMemcpyAsync(arrs[k], old[k], keep * sizeof(int32_t), hipMemcpyDeviceToDevice, p->stream),
              "copying the pivot log");
  }
  HIP_TRY(hipStreamSynchronize(p->stream), "copying the pivot log");
  for (int k = 0; k < 7; ++k) dfree(p, old[k]);
  p->d.log_enter = arrs[0];
  p->d.log_row = arrs[1];
  p->d.log_leave = arrs[2];
  p->d.log_flags = arrs[3];
  p->d.Lq = arrs[4];
  p->d.Ll = arrs[5];
  p->d.Lgen = arrs[6];
  p->d.log_cap = cap;
  p->d.Lcap = (int32_t)cap;
  drop_graph(p);  // kernels captured the old pointers
  return LP_OK;
}

int read_ctrl(lp_problem* p) {
  HIP_TRY(hipMemcpyAsync(p->h_ctrl, p->d.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, p->stream), "reading status");
  HIP_TRY(hipStreamSynchronize(p->stream), "reading status");
  return LP_OK;
}

// Reinversion between two replays, bracketed by events whose elapsed time is collected
// at the next read-back (no extra host wait).
int run_reinversion(lp_problem* p) {
  for (auto& e : p->rv_ev)
    if (!e) HIP_TRY(hipEventCreate(&e), "creating reinversion events");
  HIP_TRY(hipEventRecord(p->rv_ev[0], p->stream), "recording an event");
  // compact columns: Binv up to date first (a reinversion abandoned on a zero pivot keeps it)
  if (p->d.cmode) HIP_TRY(launch_materialize(p->d, p->stream), "writing B^-1 out");
  int k = 0;
  int rc = reinvert(p->d, p->b0, &p->rv, p->stream, p->h_ctrl->nsb, p->h_ctrl->nD, &k);
  if (rc != LP_OK) return rc;
  // The reinversion forms W from the structural basic variables' costs; in phase 1 the
  // artificial variables cost 1, so W and z are recomputed from their definitions.
  if (p->phase == 1) HIP_TRY(launch_reprice(p->d, p->stream), "pricing the phase-1 basis");
  if (p->d.cmode) HIP_TRY(launch_rebuild_compact(p->d, p->h_ctrl->nD, p->stream), "compacting B^-1");
  HIP_TRY(hipEventRecord(p->rv_ev[1], p->stream), "recording an event");
  p->rv_timing = true;
  p->last_reinv_t = p->h_ctrl->t;
  return LP_OK;
}

int collect_reinv_time(lp_problem* p) {
  if (!p->rv_timing) return LP_OK;
  float ms = 0.f;
  HIP_TRY(hipEventSynchronize(p->rv_ev[1]), "waiting for the reinversion");
  HIP_TRY(hipEventElapsedTime(&ms, p->rv_ev[0], p->rv_ev[1]), "timing the reinversion");
  p->stats.reinv_ms += ms;
  p->rv_timing = false;
  return LP_OK;
}

// The kernels of K iterations, in launch order.  FP64 form: k_price -> k_update, then
// (k_price_fin -> k_update) for each further iteration, and k_finish last: k_price_fin
// finishes the previous iteration's ratio test and prices the next one in one launch, so
// K iterations take 2K + 1 launches.  Mixed form: K times k_price32 -> k_shortlist ->
// k_update -> k_finish (k_price32 runs the FP64 pass in the iteration after a fallback
// verdict).  kind: what each launch is counted as in the profile (kinds below).
enum { kKindPrice = 0, kKindShortlist = 1, kKindUpdate = 2, kKindFinish = 3, kKindPriceFin = 4 };
struct IterKernel {
  const void* fn;
  int grid, block;
  size_t lds;
  int kind;
};

std::vector<IterKernel> iteration_kernels(const lp_problem* p, int K) {
  std::vector<IterKernel> out;
  const IterKernel upd{update_kernel_for(p->d), p->update_grid, std::abs(p->d.upd_block),
                       p->d.cmode ? compact_lds_bytes(p->ld) : update_lds_for_block(p->d.upd_block, p->ld),
                       kKindUpdate};
  const IterKernel fin{finish_kernel(), 1, kFinishBlock, 0, kKindFinish};
  if (p->d.mixed) {
    for (int k = 0; k < K; ++k) {
      out.push_back({price32_kernel(), p->price32_grid, kPrice32Block, price32_lds_bytes(p->ld), kKindPrice});
      out.push_back({shortlist_kernel(), p->d.sl_k, shortlist_block(), 0, kKindShortlist});
      out.push_back(upd);
      out.push_back(fin);
    }
    return out;
  }
  for (int k = 0; k < K; ++k) {
    const bool nt = p->d.a_nt != 0;
    out.push_back({k == 0 ? price_kernel(nt) : price_fin_kernel(nt), p->price_grid, kPriceBlock, price_lds_bytes(p->ld),
                   k == 0 ? kKindPrice : kKindPriceFin});
    out.push_back(upd);
  }
  out.push_back(fin);
  return out;
}

// An iteration graph: K iterations as a linear chain of kernel nodes.  With events (the
// main graph under profile = 1) an event-record node sits before every kernel and at the end.
int build_chain(lp_problem* p, int K, bool prof, hipGraph_t* graph, hipGraphExec_t* gexec) {
  const std::vector<IterKernel> ks = iteration_kernels(p, K);
  const int E = (int)ks.size();
  if (prof) {
    p->events.resize(E + 1, nullptr);
    for (auto& e : p->events) HIP_TRY(hipEventCreate(&e), "creating profiling events");
  }
  HIP_TRY(hipGraphCreate(graph, 0), "creating the iteration graph");
  hipGraphNode_t prev = nullptr;
  auto add_event = [&](hipEvent_t ev) -> hipError_t {
    hipGraphNode_t node;
    hipError_t e = hipGraphAddEventRecordNode(&node, *graph, prev ? &prev : nullptr, prev ? 1 : 0, ev);
    if (e == hipSuccess) prev = node;
    return e;
  };
  void* args[] = {&p->d};
  auto add_kernel = [&](const IterKernel& ik) -> hipError_t {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(ik.fn);
    kp.gridDim = dim3(ik.grid);
    kp.blockDim = dim3(ik.block);
    kp.sharedMemBytes = (unsigned)ik.lds;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, *graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (e == hipSuccess) prev = node;
    return e;
  };
  for (int i = 0; i < E; ++i) {
    if (prof) HIP_TRY(add_event(p->events[i]), "adding a profiling event");
    HIP_TRY(add_kernel(ks[i]), "adding a kernel node");
  }
  if (prof) HIP_TRY(add_event(p->events[E]), "adding a profiling event");
  HIP_TRY(hipGraphInstantiate(gexec, *graph, nullptr, nullptr, 0), "instantiating the iteration graph");
  return LP_OK;
}

int build_graph(lp_problem* p) {
  drop_graph(p);
  const int rc = build_chain(p, p->opt.iters_per_sync, p->opt.profile == 1, &p->graph, &p->gexec);
  if (rc == LP_OK) p->graph_k = p->opt.iters_per_sync;
  return rc;
}

// profile = 2: the same K iterations launched directly on the stream (no graph), each
// kernel with a start and a stop event bound to its own dispatch, so that the elapsed
// time between them is the kernel's execution alone (no launch gap).
int launch_direct(lp_problem* p, int K) {
  const std::vector<IterKernel> ks = iteration_kernels(p, K);
  const int E = (int)ks.size();
  if ((int)p->events.size() < 2 * E) {
    for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
    p->events.assign(2 * E, nullptr);
    for (auto& e : p->events) HIP_TRY(hipEventCreate(&e), "creating profiling events");
  }
  for (int i = 0; i < E; ++i) {
    void* args[] = {&p->d};
    HIP_TRY(hipExtLaunchKernel(ks[i].fn, dim3(ks[i].grid), dim3(ks[i].block), args, ks[i].lds, p->stream,
                               p->events[2 * i], p->events[2 * i + 1], 0),
            "launching an iteration kernel");
  }
  return LP_OK;
}

// Out-of-core panel mode (Section 3, Case 2).  Switched off: it has not run on the device
// yet, so an LP that does not fit the device memory budget is rejected instead (the code
// below is kept for its validation).
constexpr bool kPanelModeEnabled = false;

// Out-of-core panel mode: B^-1 = I in the pinned host copy (after the stream has drained)
// and in the device-resident last panel.
int init_panels(lp_problem* p) {
  if (!p->panel) return LP_OK;
  const int m = p->m, ld = p->ld;
  HIP_TRY(hipStreamSynchronize(p->stream), "initialising B^-1");
  std::memset(p->binv_host, 0, sizeof(double) * (size_t)m * ld);
  for (int i = 0; i < m; ++i) p->binv_host[(size_t)i * ld + i] = 1.0;
  HIP_TRY(hipMemcpyAsync(p->res, p->binv_host + (size_t)p->res_lo * ld, sizeof(double) * (size_t)(m - p->res_lo) * ld,
                         hipMemcpyHostToDevice, p->stream),
          "initialising B^-1");
  HIP_TRY(hipStreamSynchronize(p->stream), "initialising B^-1");
  return LP_OK;
}

// Out-of-core panel mode: k iterations launched directly.  Each runs the pricing kernel,
// then for every panel (in row order) a copy to the device, the update kernel on its rows
// (partials in its own slice) and a copy back, except for the resident last panel; then the
// finishing kernel over every panel's partials and the fetch of row r for the next pricing.
int launch_panel_iters(lp_problem* p, int k) {
  hipStream_t s = p->stream;
  const int ld = p->ld, P = p->panel_rows, np = p->npanels, g = p->update_grid;
  const size_t row_bytes = sizeof(double) * ld;
  DevLP fin = p->d;
  fin.update_grid = g * np;
  for (int it = 0; it < k; ++it) {
    HIP_TRY(launch_price(p->d, p->price_grid, s), "launching the pricing kernel");
    for (int pi = 0; pi < np; ++pi) {
      const int lo = pi * P, hi = std::min(p->m, lo + P);
      const bool resident = pi == np - 1;
      double* dev = resident ? p->res : p->pbuf[pi & 1];
      if (!resident)
        HIP_TRY(hipMemcpyAsync(dev, p->binv_host + (size_t)lo * ld, (hi - lo) * row_bytes, hipMemcpyHostToDevice, s),
                "streaming a panel of B^-1 to the device");
      DevLP dp = p->d;
      dp.Binv = dev;
      dp.row_lo = lo;
      dp.row_hi = hi;
      const size_t off = (size_t)pi * g;
      dp.part_th += off;
      dp.part_low += off;
      dp.part_t1 += off;
      dp.part_t2 += off;
      dp.part_al += off;
      dp.part_bv += off;
      HIP_TRY(launch_update(dp, g, s), "launching the update kernel");
      if (!resident)
        HIP_TRY(hipMemcpyAsync(p->binv_host + (size_t)lo * ld, dev, (hi - lo) * row_bytes, hipMemcpyDeviceToHost, s),
                "streaming a panel of B^-1 back");
    }
    HIP_TRY(launch_finish(fin, s), "launching the finishing kernel");
    HIP_TRY(launch_fetch_row(p->d.ctrl, p->binv_host_dev, p->res, p->res_lo, ld, p->rowbuf, s),
            "fetching the pivot row");
  }
  return LP_OK;
}

// Workgroup counts of the iteration kernels for an m x n LP (FP64 form) on a device with
// num_cu compute units, from the occupancy the kernels' LDS allows.
int iteration_grids(int32_t m, int32_t n, int num_cu, bool cmode, int* price_grid, int* update_grid,
                    int* upd_block) {
  const int ld = (int)round_up(m, 8);
  int price_per_cu = 0, update_per_cu = 0;
  hipError_t e = kernel_occupancy(&price_per_cu, &update_per_cu, ld, cmode);
  if (e != hipSuccess) return fail_hip(e, "querying kernel occupancy");
  if (price_per_cu < 1 || update_per_cu < 1) return fail(LP_ERR_ARG, "m too large for the kernels' LDS");
  *upd_block = cmode ? kUpdateBlock : update_block(ld);  // (k_update_c runs kUpdateBlock threads)
  const int pw = kPriceBlock / 64, uw = std::abs(*upd_block) / 64;
  *price_grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)price_per_cu * num_cu, (n + pw - 1) / pw));
  *update_grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)update_per_cu * num_cu, (m + uw - 1) / uw));
  if ((m + (int64_t)*update_grid * uw - 1) / ((int64_t)*update_grid * uw) > kMaxRowsPerWave)
    return fail(LP_ERR_ARG, "m too large for this device: more than kMaxRowsPerWave rows per wavefront");
  return LP_OK;
}

int create_common(lp_problem** out, int32_t m, int32_t n, const double* A, const double* b, const double* c,
                  const lp_options* opt, bool device_inputs) {
  if (!out) return fail(LP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (m <= 0 || n < 0) return fail(LP_ERR_ARG, "need m > 0 and n >= 0");
  if (m > LP_MAX_ROWS) return fail(LP_ERR_ARG, "m exceeds LP_MAX_ROWS");
  if ((int64_t)n + m > INT32_MAX / 2) return fail(LP_ERR_ARG, "n + m too large");
  if (!b || (n > 0 && (!A || !c))) return fail(LP_ERR_ARG, "NULL data pointer");
  lp_options o;
  lp_default_options(&o);
  if (opt) o = *opt;
  if (int rc = check_options(&o)) return rc;
  if (o.max_iter == 0) o.max_iter = 10 * ((int64_t)m + n);
  const bool mixed = o.precision == LP_MIXED;

  std::vector<double> hb(m), hc(n);
  if (!device_inputs) {
    const size_t cnt = (size_t)m * n;
    for (size_t k = 0; k < cnt; ++k) {
      if (!std::isfinite(A[k])) return fail(LP_ERR_ARG, "A contains a non-finite value");
      if (mixed && std::fabs(A[k]) > (double)FLT_MAX)
        return fail(LP_ERR_ARG, "A has an entry beyond the FP32 range, which the mixed form cannot screen");
    }
    for (int32_t i = 0; i < m; ++i) {
      if (!std::isfinite(b[i])) return fail(LP_ERR_ARG, "b contains a non-finite value");
      if (b[i] < 0.0) return fail(LP_ERR_NEG_RHS, "b_i < 0: the slack basis is infeasible");
    }
    for (int32_t j = 0; j < n; ++j)
      if (!std::isfinite(c[j])) return fail(LP_ERR_ARG, "c contains a non-finite value");
    std::memcpy(hb.data(), b, sizeof(double) * m);
    if (n) std::memcpy(hc.data(), c, sizeof(double) * n);
  }

  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "selecting the device");
  lp_problem* p = new (std::nothrow) lp_problem();
  if (!p) return fail(LP_ERR_NOMEM, "host allocation failed");
  int rc = LP_OK;
  auto bail = [&](int code) {
    release(p);
    p = nullptr;
    return code;
  };
  const auto drop = on_scope_exit([&] {  // an exception before the hand-over releases it too
    if (p) release(p);
  });
  p->device = dev;
  p->opt = o;
  p->m = m;
  p->n = n;
  p->n_user = n;
  p->ld = (int32_t)round_up(m, 8);
  const int ld = p->ld;
  const int N = n + m;
  if (o.stream) {
    p->stream = static_cast<hipStream_t>(o.stream);
  } else {
    // A blocking stream: ordered after work the caller left on the legacy default stream.
    hipError_t e = hipStreamCreate(&p->stream);
    if (e != hipSuccess) return bail(fail_hip(e, "creating a stream"));
    p->own_stream = true;
  }
  {
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return bail(fail_hip(e, "querying the device"));
    p->num_cu = prop.multiProcessorCount;
  }
  int upd_block = 0;
  // Compact columns on rows long enough for the sparse-column update.
  bool cmode = compact_columns(ld);
  if ((rc = iteration_grids(m, n, p->num_cu, cmode, &p->price_grid, &p->update_grid, &upd_block)) != LP_OK)
    return bail(rc);
  p->reinv_period = o.reinv_period >= 0 ? o.reinv_period : (mixed ? 64 : 0);
  if (mixed) {
    int per_cu = 0;
    hipError_t e = price32_occupancy(&per_cu, ld);
    if (e != hipSuccess) return bail(fail_hip(e, "querying kernel occupancy"));
    if (per_cu < 1) return bail(fail(LP_ERR_ARG, "m too large for the FP32 pricing kernel's LDS"));
    const int w32 = kPrice32Block / 64;
    p->price32_grid = (int)std::max<int64_t>(
        1, std::min<int64_t>(std::min<int64_t>((int64_t)per_cu * p->num_cu, max_price32_grid()), (N + w32 - 1) / w32));
    // The FP64 pass runs inside k_price32's grid: its partials are k_price32's.
    p->price_grid = p->price32_grid;
  }

  // Device memory (Section 3, Figure 2): A' (ld x n) + B^-1 (m x ld) dominate.  Against the
  // free memory, or the caller's budget: the whole tableau (Case 1), or B^-1 in row panels
  // streamed from host memory (Case 2).
  {
    size_t freeb = 0, totalb = 0;
    hipError_t e = hipMemGetInfo(&freeb, &totalb);
    if (e != hipSuccess) return bail(fail_hip(e, "querying device memory"));
    const double budget = o.device_budget > 0 ? std::min((double)o.device_budget, (double)freeb) : (double)freeb;
    const double rest = (mixed ? 12.0 : 8.0) * ld * (double)n + 64.0 * N + 64.0 * ld + 64.0 * o.max_iter +
                        16.0 * (p->update_grid + p->price_grid) * 8.0;
    const double binv = (cmode ? 16.0 : 8.0) * m * (double)ld;  // B^-1 (and Bc)
    if (rest + binv > budget && !kPanelModeEnabled)
      return bail(fail(LP_ERR_NOMEM, "LP does not fit in the device memory budget (the out-of-core panel mode "
                                     "is switched off in this build)"));
    if (rest + binv > budget) {
      // three panel buffers: two streamed alternately and the resident last panel
      const double rows = std::floor((budget - rest) / (3.0 * 8.0 * ld));
      if (rows < 8) return bail(fail(LP_ERR_NOMEM, "LP does not fit in the device memory budget"));
      if (mixed || p->reinv_period > 0 || o.profile != 0)
        return bail(fail(LP_ERR_ARG, "B^-1 does not fit the device memory budget; the out-of-core panel mode runs "
                                     "the FP64 form without reinversion or profiling"));
      p->panel = true;
      p->panel_rows = (int)std::min<double>(rows, m);
      // the panel mode streams rows of Binv itself: no compact columns
      cmode = false;
      if ((rc = iteration_grids(m, n, p->num_cu, false, &p->price_grid, &p->update_grid, &upd_block)) != LP_OK)
        return bail(rc);
      p->npanels = (m + p->panel_rows - 1) / p->panel_rows;
      p->res_lo = (p->npanels - 1) * p->panel_rows;
    }
  }
  double* dA = nullptr;
  double* chat = nullptr;
#define ALLOC(ptr, cnt)                                                    \
  do {                                                                     \
    hipError_t e_ = dalloc(p, &(ptr), (cnt));                              \
    if (e_ != hipSuccess) return bail(fail_hip(e_, "allocating " #ptr)); \
  } while (0)
  ALLOC(dA, (size_t)ld * std::max(n, 1));
  ALLOC(chat, (size_t)N);
  const size_t nparts_u = (size_t)p->update_grid * (p->panel ? p->npanels : 1);
  if (p->panel) {
    ALLOC(p->pbuf[0], (size_t)p->panel_rows * ld);
    ALLOC(p->pbuf[1], (size_t)p->panel_rows * ld);
    ALLOC(p->res, (size_t)(m - p->res_lo) * ld);
    ALLOC(p->rowbuf, (size_t)ld);
  } else {
    ALLOC(p->d.Binv, (size_t)m * ld);
  }
  if (cmode) {
    ALLOC(p->d.Bc, (size_t)m * ld);
    ALLOC(p->d.rho_c, (size_t)ld);
  }
  ALLOC(p->d.xB, (size_t)m);
  ALLOC(p->d.W0, (size_t)ld);
  ALLOC(p->d.W1, (size_t)ld);
  ALLOC(p->d.rho, (size_t)ld);
  ALLOC(p->d.alpha0, (size_t)m);
  ALLOC(p->d.alpha1, (size_t)m);
  ALLOC(p->d.basis, (size_t)m);
  ALLOC(p->d.dlist, (size_t)m);
  ALLOC(p->d.inD, (size_t)m);
  ALLOC(p->d.pos, (size_t)N);
  ALLOC(p->d.tabu_until, (size_t)N);
  ALLOC(p->d.gen, (size_t)N);
  ALLOC(p->d.excl, (size_t)N);
  ALLOC(p->d.part_d, 2 * (size_t)p->price_grid);
  ALLOC(p->d.part_j, 2 * (size_t)p->price_grid);
  ALLOC(p->d.part_th, nparts_u);
  ALLOC(p->d.part_low, nparts_u);
  ALLOC(p->d.part_t1, nparts_u);
  ALLOC(p->d.part_t2, nparts_u);
  ALLOC(p->d.part_al, nparts_u);
  ALLOC(p->d.part_bv, nparts_u);
  ALLOC(p->d.ctrl, 1);
  ALLOC(p->b0, (size_t)m);
  ALLOC(p->c0, (size_t)std::max(n, 1));
  float* dA32 = nullptr;
  if (mixed) {
    ALLOC(dA32, (size_t)ld * std::max(n, 1));
    ALLOC(p->d.part32, (size_t)p->price32_grid * kShortlist);
    ALLOC(p->d.sl_d, (size_t)kShortlist);
    ALLOC(p->d.sl_j, (size_t)kShortlist);
  }
#undef ALLOC
  p->d.m = m;
  p->d.n = n;
  p->d.cmode = cmode ? 1 : 0;
  p->d.a_nt = price_nt(ld, n) ? 1 : 0;
  p->d.upd_block = upd_block;
  p->d.price_grid = p->price_grid;
  p->d.update_grid = p->update_grid;
  p->d.ld = ld;
  p->d.A = dA;
  p->d.chat = chat;
  p->d.tenure = o.tabu_tenure;
  p->d.use_llist = o.leaving_list ? 1 : 0;
  p->d.eps_d = o.eps_d;
  p->d.eps_p = o.eps_p;
  p->d.eps_z = o.eps_z;
  p->d.eps_t = o.eps_t;
  p->d.mixed = mixed ? 1 : 0;
  p->d.sl_k = o.shortlist_k;
  p->d.A32 = dA32;
  p->d.price32_grid = p->price32_grid;
  p->d.row_lo = 0;
  p->d.row_hi = m;
  p->d.rowsrc = p->panel ? p->rowbuf : nullptr;
  if (p->panel) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p->binv_host), sizeof(double) * (size_t)m * ld,
                                 hipHostMallocDefault);
    if (e != hipSuccess) return bail(fail_hip(e, "allocating pinned memory for B^-1"));
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&p->binv_host_dev), p->binv_host, 0);
    if (e != hipSuccess) return bail(fail_hip(e, "mapping the host copy of B^-1"));
  }
  {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p->h_ctrl), sizeof(Ctrl), hipHostMallocDefault);
    if (e != hipSuccess) return bail(fail_hip(e, "allocating pinned memory"));
    std::memset(p->h_ctrl, 0, sizeof(Ctrl));
    e = hipHostMalloc(reinterpret_cast<void**>(&p->h_stage), sizeof(Ctrl), hipHostMallocDefault);
    if (e != hipSuccess) return bail(fail_hip(e, "allocating pinned memory"));
    std::memset(p->h_stage, 0, sizeof(Ctrl));
  }
  if ((rc = ensure_capacity(p, o.max_iter)) != LP_OK) return bail(rc);

  hipStream_t s = p->stream;
  hipError_t e = hipSuccess;
  // Device scratch of the upload: a flag word and a hash word.
  int32_t* flag = nullptr;
  unsigned long long* dhash = nullptr;
  if ((e = dalloc(p, &flag, 1)) != hipSuccess || (e = dalloc(p, &dhash, 1)) != hipSuccess)
    return bail(fail_hip(e, "allocating the upload check"));
  if (device_inputs) {
    // Packed into the padded layout and validated on the device, then b and c come to
    // the host for the reported objective.
    if ((e = launch_clear_flag(flag, s)) != hipSuccess ||
        (e = launch_pack_lp(dA, ld, A, m, n, p->b0, b, p->c0, c, flag, s)) != hipSuccess)
      return bail(fail_hip(e, "copying the LP"));
    // (the mixed form keeps an FP32 copy of A', so there every entry must be in the FP32 range)
    if (mixed && (e = launch_check_finite(dA, (int64_t)ld * n, (double)FLT_MAX, flag, s)) != hipSuccess)
      return bail(fail_hip(e, "validating A"));
    int32_t hflag = 0;
    if ((e = pageable_copy(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = pageable_copy(hb.data(), p->b0, sizeof(double) * m, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = pageable_copy(hc.data(), p->c0, sizeof(double) * n, hipMemcpyDeviceToHost, s)) != hipSuccess)
      return bail(fail_hip(e, "reading the LP data"));
    if (hflag & 2) return bail(fail(LP_ERR_NEG_RHS, "b_i < 0: the slack basis is infeasible"));
    if (hflag)
      return bail(fail(LP_ERR_ARG, mixed ? "A, b or c contains a non-finite value, or A one beyond the FP32 range "
                                           "(mixed form)"
                                         : "A, b or c contains a non-finite value"));
  } else {
    // One contiguous copy of A' in the padded layout (packed on the host unless ld = m),
    // then an order-independent hash of what arrived, formed on the device, against the
    // same hash of what was sent: a copy that moved nothing, or not all of it, is an error.
    std::vector<double> packed;
    const double* src = A;
    if (ld != m && n > 0) {
      packed.assign((size_t)ld * n, 0.0);
      for (int32_t j = 0; j < n; ++j) std::memcpy(&packed[(size_t)j * ld], A + (size_t)j * m, sizeof(double) * m);
      src = packed.data();
    }
    const size_t na = (size_t)ld * n;
    const uint64_t want = hash_doubles(src, na, 0) + hash_doubles(hb.data(), m, na) + hash_doubles(hc.data(), n, na + m);
    if ((n > 0 && ((e = pageable_copy(dA, src, sizeof(double) * na, hipMemcpyHostToDevice, s)) != hipSuccess ||
                   (e = pageable_copy(p->c0, hc.data(), sizeof(double) * n, hipMemcpyHostToDevice, s)) != hipSuccess)) ||
        (e = pageable_copy(p->b0, hb.data(), sizeof(double) * m, hipMemcpyHostToDevice, s)) != hipSuccess)
      return bail(fail_hip(e, "copying the LP"));
    uint64_t got = 0;
    if ((e = launch_hash(dA, na, 0, p->b0, m, p->c0, n, dhash, s)) != hipSuccess ||
        (e = pageable_copy(&got, dhash, sizeof(got), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return bail(fail_hip(e, "checking the upload"));
    if (got != want) return bail(fail(LP_ERR_DEVICE, "the LP data on the device differ from the host's after the copy"));
  }
  dfree(p, flag);
  dfree(p, dhash);
  if (mixed) {
    // FP32 copy of A' with the same padding (round to nearest).
    e = launch_convert32(dA, dA32, (size_t)ld * n, s);
    if (e != hipSuccess) return bail(fail_hip(e, "converting A to FP32"));
  }
  e = launch_init(p->d, p->b0, p->c0, o.sense == LP_MAX ? -1.0 : 1.0, s);
  if (e != hipSuccess) return bail(fail_hip(e, "initialising the slack basis"));
  if ((rc = init_panels(p)) != LP_OK) return bail(rc);
  if ((rc = read_ctrl(p)) != LP_OK) return bail(rc);
  if (p->reinv_period > 0 && (rc = reinv_prepare(&p->rv, m, ld)) != LP_OK) return bail(rc);
  p->hc = std::move(hc);
  *out = p;
  p = nullptr;  // handed over
  return LP_OK;
}

// Phase 1 from the basis of unit columns: its costs into chat, W and z from them.
int start_phase1(lp_problem* p) {
  HIP_TRY(hipMemcpyAsync(const_cast<double*>(p->d.chat), p->chat1, sizeof(double) * ((size_t)p->n + p->m),
                         hipMemcpyDeviceToDevice, p->stream),
          "setting the phase-1 costs");
  HIP_TRY(launch_reprice(p->d, p->stream), "pricing the phase-1 basis");
  p->phase = 1;
  p->phase1_t = -1;
  p->drive_outs = 0;
  p->switch_ms = 0.0;
  return read_ctrl(p);
}

// Section 3.4 / the two-phase method: phase 1 has priced out optimal (no pivot pending).
// Either the LP is infeasible, or the artificial variables left basic at zero are driven
// out and phase 2 starts from this basis with the LP's own costs.
int phase_switch(lp_problem* p) {
  const auto t0 = std::chrono::steady_clock::now();
  const int m = p->m, n = p->n;
  p->phase1_t = p->h_ctrl->t;
  if (p->h_ctrl->z > p->eps_f) {
    p->h_stage->status = LP_INFEASIBLE;
    HIP_TRY(hipMemcpyAsync(&p->d.ctrl->status, &p->h_stage->status, sizeof(int32_t), hipMemcpyHostToDevice,
                           p->stream),
            "setting the status");
    p->phase = 2;
    int rc = read_ctrl(p);
    p->switch_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
  }
  std::vector<int32_t> bas(m);
  HIP_TRY(pageable_copy(bas.data(), p->d.basis, sizeof(int32_t) * m, hipMemcpyDeviceToHost, p->stream),
          "reading the basis");
  // the switch reads and pivots B^-1 by its own columns: compact columns written out first
  if (p->d.cmode) HIP_TRY(launch_materialize(p->d, p->stream), "writing B^-1 out");
  for (int r = 0; r < m; ++r) {
    // A drive-out changes only its own row of the basis: this list stays valid.
    if (bas[r] < n || !p->art_h[bas[r] - n]) continue;
    HIP_TRY(launch_drive_out(p->d, r, p->tab_t, p->tab_j, p->drive, p->stream), "driving out an artificial variable");
  }
  HIP_TRY(hipMemcpyAsync(const_cast<double*>(p->d.chat), p->chat2, sizeof(double) * ((size_t)n + m),
                         hipMemcpyDeviceToDevice, p->stream),
          "restoring the costs");
  HIP_TRY(launch_reprice(p->d, p->stream), "pricing the phase-2 basis");
  if (p->d.cmode) HIP_TRY(launch_rebuild_compact(p->d, p->h_ctrl->nD, p->stream), "compacting B^-1");
  p->h_stage->status = LP_RUNNING;
  HIP_TRY(hipMemcpyAsync(&p->d.ctrl->status, &p->h_stage->status, sizeof(int32_t), hipMemcpyHostToDevice, p->stream),
          "setting the status");
  int rc = read_ctrl(p);
  if (rc != LP_OK) return rc;
  p->drive_outs = p->h_ctrl->t - p->phase1_t;
  p->phase = 2;
  p->switch_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return LP_OK;
}

// Iterates until a terminal status or until the pivot count reaches iter_cap.  decide:
// at the cap, one more pricing decides between OPTIMAL and ITER_LIMIT (lp_solve_until);
// otherwise the solve stops there still RUNNING (lp_iterate).  Replays of the main graph
// run while at least iters_per_sync pivots remain, then power-of-two tail graphs.
int run_until(lp_problem* p, int64_t iter_cap, bool decide, int32_t* status_out) {
  int rc;
  if ((p->h_ctrl->status == LP_OPTIMAL && p->phase != 1) || p->h_ctrl->status == LP_UNBOUNDED ||
      p->h_ctrl->status == LP_INFEASIBLE) {
    if (status_out) *status_out = p->h_ctrl->status;
    return LP_OK;
  }
  // (drive-out pivots of a phase switch may add up to m log entries past the limit)
  if ((rc = ensure_capacity(p, iter_cap + (p->phase == 1 ? p->m : 0))) != LP_OK) return rc;
  const bool direct = p->opt.profile == 2;
  if (!direct && !p->panel && (!p->gexec || p->graph_k != p->opt.iters_per_sync)) {
    if ((rc = build_graph(p)) != LP_OK) return rc;
  }
  if (!decide && p->h_ctrl->t >= iter_cap) {
    if (status_out) *status_out = p->h_ctrl->status == LP_ITER_LIMIT ? LP_RUNNING : p->h_ctrl->status;
    return LP_OK;
  }
  const auto t0 = std::chrono::steady_clock::now();
  // Arm the control block: new pivot limit, and RUNNING again after an ITER_LIMIT stop.
  p->h_stage->max_iter = iter_cap;
  p->h_stage->status = LP_RUNNING;
  HIP_TRY(hipMemcpyAsync(&p->d.ctrl->max_iter, &p->h_stage->max_iter, sizeof(int64_t), hipMemcpyHostToDevice,
                         p->stream),
          "arming the solve");
  HIP_TRY(hipMemcpyAsync(&p->d.ctrl->status, &p->h_stage->status, sizeof(int32_t), hipMemcpyHostToDevice, p->stream),
          "arming the solve");
  const bool prof = p->opt.profile != 0;
  const int K = p->opt.iters_per_sync;
  const bool mixed = p->d.mixed != 0;
  for (;;) {
    const int64_t left = iter_cap - p->h_ctrl->t;
    int k = K;
    if (left < K) {
      if (left <= 0 && !decide) break;
      k = 1;
      while (2 * (int64_t)k <= left) k *= 2;
    }
    const int64_t t_before = p->h_ctrl->t;
    const int64_t fb_before = p->h_ctrl->n_fallback;
    const int64_t cols_before = p->h_ctrl->price_cols;
    const int64_t nsb_before = p->h_ctrl->nsb;
    const int64_t ubytes_before = p->h_ctrl->update_bytes;
    if (p->panel) {
      if ((rc = launch_panel_iters(p, k)) != LP_OK) return rc;
    } else if (direct) {
      if ((rc = launch_direct(p, k)) != LP_OK) return rc;
    } else if (k == K) {
      HIP_TRY(hipGraphLaunch(p->gexec, p->stream), "launching the iteration graph");
    } else {
      int lg = 0;
      while ((1 << lg) < k) ++lg;
      if (!p->tail_exec[lg] &&
          (rc = build_chain(p, k, false, &p->tail_graph[lg], &p->tail_exec[lg])) != LP_OK)
        return rc;
      HIP_TRY(hipGraphLaunch(p->tail_exec[lg], p->stream), "launching a tail graph");
    }
    if ((rc = read_ctrl(p)) != LP_OK) return rc;
    p->stats.syncs += 1;
    if ((rc = collect_reinv_time(p)) != LP_OK) return rc;
    if (prof && k == K && p->h_ctrl->status == LP_RUNNING && t_before > 0 && p->h_ctrl->t == t_before + K) {
      // Steady state: every kernel of the replay did a full pass (K pivots, so in the
      // mixed form no fallback iteration and no FP64 pass).  profile = 1: the time between
      // the event nodes around a kernel (its launch gap included); profile = 2: the
      // kernel's own start and stop.
      const std::vector<IterKernel> ks = iteration_kernels(p, K);
      for (size_t i = 0; i < ks.size(); ++i) {
        float ms = 0.f;
        const int a = direct ? (int)(2 * i) : (int)i;
        HIP_TRY(hipEventElapsedTime(&ms, p->events[a], p->events[a + 1]), "reading profile events");
        switch (ks[i].kind) {
          case kKindPrice:
            if (mixed) p->stats.price32_ms += ms;
            else p->stats.price_ms += ms;
            break;
          case kKindPriceFin: p->stats.price_ms += ms; p->stats.price_fin_ms += ms; break;
          case kKindShortlist: p->stats.shortlist_ms += ms; break;
          case kKindUpdate: p->stats.update_ms += ms; break;
          default: p->stats.finish_ms += ms; break;
        }
      }
      if (!mixed) {
        p->stats.price_launches += K;
        p->stats.price_fin_launches += K - 1;
      }
      p->stats.update_launches += K;
      p->stats.finish_launches += mixed ? K : 1;
      p->stats.price_bytes += 8.0 * p->m * (double)(p->h_ctrl->price_cols - cols_before);
      // algorithmic bytes of the update passes, counted on the device
      p->stats.update_bytes += (double)(p->h_ctrl->update_bytes - ubytes_before);
      if (mixed) {
        // Nonbasic structural columns streamed by the K screening passes (the basis
        // changes by at most one structural column per pivot; the midpoint is used).
        const double nonbasic = p->n - 0.5 * (double)(nsb_before + p->h_ctrl->nsb);
        p->stats.price32_bytes += 4.0 * p->m * nonbasic * K;
      }
    }
    if (p->h_ctrl->status == LP_OPTIMAL && p->phase == 1) {
      if ((rc = phase_switch(p)) != LP_OK) return rc;
      if (p->h_ctrl->status == LP_RUNNING) continue;
    }
    if (p->h_ctrl->status != LP_RUNNING) break;
    // Every iteration of a RUNNING solve's replay must pivot, or (mixed form) end with the
    // fallback verdict; anything else is a fault of the kernels' control logic, reported
    // instead of looping.
    if (p->h_ctrl->t + p->h_ctrl->n_fallback != t_before + fb_before + k)
      return fail(LP_ERR_DEVICE, "iteration graph made no progress while RUNNING");
    // (reinversion recomputes W from the structural basic variables only: not in phase 1)
    if (p->reinv_period > 0 && p->phase != 1 && p->h_ctrl->t - p->last_reinv_t >= p->reinv_period) {
      if ((rc = run_reinversion(p)) != LP_OK) return rc;
    }
  }
  p->stats.solve_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (status_out) *status_out = p->h_ctrl->status;
  return LP_OK;
}

// ---- the entry point that allocates nothing ----

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// The address of `scratch` on the current device, looked up once per device.
int scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(LP_ERR_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail_hip(e != hipSuccess ? e : hipErrorInvalidSymbol, "locating the scratch array");
    g_scratch[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch[dev];
  return LP_OK;
}

// Carves consecutive 256-byte aligned pieces out of the scratch array (or, with base null,
// only counts the bytes they take).
struct Carver {
  unsigned char* base;
  size_t used = 0;
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
    return p;
  }
};

// Lays out every buffer of an m x n solve with pivot capacity cap; returns the bytes used.
size_t carve_lp(Carver& cv, DevLP& d, int32_t m, int32_t n, int64_t cap, double** b0, double** c0, int32_t** flag) {
  const size_t ld = (size_t)round_up(m, 8), N = (size_t)n + m;
  d.A = cv.take<double>(ld * std::max(n, 1));
  d.chat = cv.take<double>(N);
  d.Binv = cv.take<double>((size_t)m * ld);
  if (d.cmode) {
    d.Bc = cv.take<double>((size_t)m * ld);
    d.rho_c = cv.take<double>(ld);
  }
  d.xB = cv.take<double>(m);
  d.W0 = cv.take<double>(ld);
  d.W1 = cv.take<double>(ld);
  d.rho = cv.take<double>(ld);
  d.alpha0 = cv.take<double>(m);
  d.alpha1 = cv.take<double>(m);
  d.basis = cv.take<int32_t>(m);
  d.dlist = cv.take<int32_t>(m);
  d.inD = cv.take<int32_t>(m);
  d.pos = cv.take<int32_t>(N);
  d.tabu_until = cv.take<int32_t>(N);
  d.gen = cv.take<int32_t>(N);
  d.excl = cv.take<int32_t>(N);
  d.part_d = cv.take<double>(2 * (size_t)d.price_grid);
  d.part_j = cv.take<int32_t>(2 * (size_t)d.price_grid);
  d.part_th = cv.take<double>(d.update_grid);
  d.part_low = cv.take<int32_t>(d.update_grid);
  d.part_t1 = cv.take<double>(d.update_grid);
  d.part_t2 = cv.take<double>(d.update_grid);
  d.part_al = cv.take<double>(d.update_grid);
  d.part_bv = cv.take<int32_t>(d.update_grid);
  d.ctrl = cv.take<Ctrl>(1);
  d.log_enter = cv.take<int32_t>(cap);
  d.log_row = cv.take<int32_t>(cap);
  d.log_leave = cv.take<int32_t>(cap);
  d.log_flags = cv.take<int32_t>(cap);
  d.Lq = cv.take<int32_t>(cap);
  d.Ll = cv.take<int32_t>(cap);
  d.Lgen = cv.take<int32_t>(cap);
  *b0 = cv.take<double>(m);
  *c0 = cv.take<double>(std::max(n, 1));
  *flag = cv.take<int32_t>(1);
  return cv.used;
}

}  // namespace

extern "C" {

int lp_default_options(lp_options* opt) try {
  if (!opt) return fail(LP_ERR_ARG, "opt is NULL");
  std::memset(opt, 0, sizeof(*opt));
  opt->sense = LP_MAX;
  opt->tabu_tenure = 5;
  opt->leaving_list = 1;
  opt->iters_per_sync = 16;
  opt->max_iter = 0;
  opt->eps_d = 1e-9;
  opt->eps_p = 1e-9;
  opt->eps_z = 1e-9;
  opt->eps_t = 1e-9;
  opt->record_pivots = 1;
  opt->profile = 0;
  opt->batch_small_m = -1;
  opt->batch_binv_lds_m = -1;
  opt->stream = nullptr;
  opt->precision = LP_FP64;
  opt->shortlist_k = kShortlist;
  opt->reinv_period = -1;
  opt->device_budget = 0;
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_create(lp_problem** out, int32_t m, int32_t n, const double* A_colmajor, const double* b, const double* c,
              const lp_options* opt) try {
  return create_common(out, m, n, A_colmajor, b, c, opt, false);
} catch (...) {
  return host_exception();
}

int lp_create_device(lp_problem** out, int32_t m, int32_t n, const double* A_colmajor, const double* b,
                     const double* c, const lp_options* opt) try {
  return create_common(out, m, n, A_colmajor, b, c, opt, true);
} catch (...) {
  return host_exception();
}

int lp_create_general(lp_problem** out, int32_t m, int32_t n, const double* A_colmajor, const double* b,
                      const double* c, const int32_t* row_type, const lp_options* opt) try {
  if (!out) return fail(LP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (m <= 0 || n < 0) return fail(LP_ERR_ARG, "need m > 0 and n >= 0");
  if (m > LP_MAX_ROWS) return fail(LP_ERR_ARG, "m exceeds LP_MAX_ROWS");
  if (!b || (n > 0 && (!A_colmajor || !c))) return fail(LP_ERR_ARG, "NULL data pointer");
  // Normal form: b >= 0 by row sign changes; >= rows get a surplus column -e_i.
  std::vector<double> sg(m);
  std::vector<int8_t> art(m, 0), ge(m, 0);
  int32_t ns = 0, na = 0;
  double bmax = 0.0;
  for (int32_t i = 0; i < m; ++i) {
    const int32_t ty = row_type ? row_type[i] : LP_ROW_LE;
    if (ty < LP_ROW_LE || ty > LP_ROW_EQ) return fail(LP_ERR_ARG, "unknown row type");
    if (!std::isfinite(b[i])) return fail(LP_ERR_ARG, "b contains a non-finite value");
    sg[i] = b[i] < 0.0 ? -1.0 : 1.0;
    int32_t t2 = ty;
    if (sg[i] < 0.0 && ty != LP_ROW_EQ) t2 = ty == LP_ROW_LE ? LP_ROW_GE : LP_ROW_LE;
    ge[i] = t2 == LP_ROW_GE;
    art[i] = t2 != LP_ROW_LE;
    ns += ge[i];
    na += art[i];
    bmax = std::max(bmax, std::fabs(b[i]));
  }
  if ((int64_t)n + ns > INT32_MAX / 4) return fail(LP_ERR_ARG, "n too large");
  const int32_t n2 = n + ns;
  const size_t N = (size_t)n2 + m;
  std::vector<double> A2((size_t)m * std::max(n2, 1), 0.0), b2(m), c2(std::max(n2, 1), 0.0), c1(N, 0.0);
  for (int32_t j = 0; j < n; ++j)
    for (int32_t i = 0; i < m; ++i) A2[(size_t)j * m + i] = sg[i] * A_colmajor[(size_t)j * m + i];
  for (int32_t i = 0, k = n; i < m; ++i)
    if (ge[i]) A2[(size_t)(k++) * m + i] = -1.0;
  for (int32_t i = 0; i < m; ++i) b2[i] = sg[i] * b[i];
  for (int32_t j = 0; j < n; ++j) c2[j] = c[j];
  lp_problem* p = nullptr;
  int rc = create_common(&p, m, n2, A2.data(), b2.data(), c2.data(), opt, false);
  if (rc != LP_OK) return rc;
  auto bail = [&](int code) {
    release(p);
    p = nullptr;
    return code;
  };
  const auto drop = on_scope_exit([&] {  // an exception before the hand-over releases it too
    if (p) release(p);
  });
  if (p->panel) return bail(fail(LP_ERR_ARG, "the two-phase start needs the tableau in device memory (Case 1)"));
  p->n_user = n;
  p->rsign = std::move(sg);
  p->eps_f = 1e-9 * (1.0 + bmax);
  p->two_phase = na > 0;
  if (p->two_phase) {
    int8_t* dart = nullptr;
    const int g = tabrow_grid(p->d);
    hipError_t e;
    if ((e = dalloc(p, &dart, (size_t)m)) != hipSuccess || (e = dalloc(p, &p->chat1, N)) != hipSuccess ||
        (e = dalloc(p, &p->chat2, N)) != hipSuccess || (e = dalloc(p, &p->tab_t, (size_t)g)) != hipSuccess ||
        (e = dalloc(p, &p->tab_j, (size_t)g)) != hipSuccess || (e = dalloc(p, &p->drive, 4)) != hipSuccess)
      return bail(fail_hip(e, "allocating the two-phase state"));
    for (int32_t i = 0; i < m; ++i) c1[(size_t)n2 + i] = art[i] ? 1.0 : 0.0;
    if ((e = pageable_copy(dart, art.data(), (size_t)m, hipMemcpyHostToDevice, p->stream)) != hipSuccess ||
        (e = pageable_copy(p->chat1, c1.data(), sizeof(double) * N, hipMemcpyHostToDevice, p->stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(p->chat2, p->d.chat, sizeof(double) * N, hipMemcpyDeviceToDevice, p->stream)) !=
            hipSuccess)
      return bail(fail_hip(e, "uploading the two-phase state"));
    p->d.art = dart;
    p->art_h = std::move(art);
    if ((rc = ensure_capacity(p, p->opt.max_iter + m)) != LP_OK) return bail(rc);
    if ((rc = start_phase1(p)) != LP_OK) return bail(rc);
  }
  *out = p;
  p = nullptr;  // handed over
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_solve_until(lp_problem* p, int64_t iter_cap, int32_t* status_out) try {
  if (!p) return fail(LP_ERR_ARG, "p is NULL");
  if (iter_cap < 0) return fail(LP_ERR_ARG, "iter_cap must be >= 0");
  return run_until(p, iter_cap, true, status_out);
} catch (...) {
  return host_exception();
}

int lp_iterate(lp_problem* p, int64_t count, int32_t* status_out) try {
  if (!p) return fail(LP_ERR_ARG, "p is NULL");
  if (count < 0) return fail(LP_ERR_ARG, "count must be >= 0");
  if (count > INT32_MAX - p->h_ctrl->t) return fail(LP_ERR_ARG, "count too large");
  return run_until(p, p->h_ctrl->t + count, false, status_out);
} catch (...) {
  return host_exception();
}

int lp_solve(lp_problem* p, int32_t* status_out) try {
  if (!p) return fail(LP_ERR_ARG, "p is NULL");
  return lp_solve_until(p, p->opt.max_iter, status_out);
} catch (...) {
  return host_exception();
}

int lp_reset(lp_problem* p) try {
  if (!p) return fail(LP_ERR_ARG, "p is NULL");
  HIP_TRY(launch_init(p->d, p->b0, p->c0, p->opt.sense == LP_MAX ? -1.0 : 1.0, p->stream), "resetting");
  int rc = init_panels(p);
  if (rc != LP_OK) return rc;
  rc = read_ctrl(p);
  if (rc != LP_OK) return rc;
  p->rv_timing = false;
  p->last_reinv_t = 0;
  p->stats = lp_stats{};
  if (p->two_phase) return start_phase1(p);
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_get_solution(const lp_problem* pc, double* objective, double* x, double* y, int32_t* basis,
                    int64_t* iterations) try {
  if (!pc) return fail(LP_ERR_ARG, "p is NULL");
  lp_problem* p = const_cast<lp_problem*>(pc);
  const int m = p->m, n = p->n_user;
  std::vector<double> xB(m), W(m);
  std::vector<int32_t> bas(m);
  HIP_TRY(pageable_copy(xB.data(), p->d.xB, sizeof(double) * m, hipMemcpyDeviceToHost, p->stream), "reading x_B");
  const double* dW = p->h_ctrl->wcur ? p->d.W1 : p->d.W0;
  HIP_TRY(pageable_copy(W.data(), dW, sizeof(double) * m, hipMemcpyDeviceToHost, p->stream), "reading W");
  HIP_TRY(pageable_copy(bas.data(), p->d.basis, sizeof(int32_t) * m, hipMemcpyDeviceToHost, p->stream),
          "reading the basis");
  std::vector<int32_t> row_of(n, -1);
  for (int i = 0; i < m; ++i)
    if (bas[i] < n) row_of[bas[i]] = i;
  if (x)
    for (int j = 0; j < n; ++j) x[j] = row_of[j] >= 0 ? xB[row_of[j]] : 0.0;
  if (objective) {
    double s = 0.0;
    for (int j = 0; j < n; ++j)
      if (row_of[j] >= 0) s += p->hc[j] * xB[row_of[j]];
    *objective = s;
  }
  const double sgn = p->opt.sense == LP_MAX ? -1.0 : 1.0;
  if (y)
    for (int i = 0; i < m; ++i) y[i] = sgn * W[i] * (p->rsign.empty() ? 1.0 : p->rsign[i]);
  if (basis) std::memcpy(basis, bas.data(), sizeof(int32_t) * m);
  if (iterations) *iterations = p->h_ctrl->t;
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_get_pivots(const lp_problem* pc, int32_t* entering, int32_t* leaving_row, int32_t* leaving_var,
                  int32_t* flags, int64_t capacity, int64_t* count) try {
  if (!pc) return fail(LP_ERR_ARG, "p is NULL");
  if (capacity < 0) return fail(LP_ERR_ARG, "capacity must be >= 0");
  lp_problem* p = const_cast<lp_problem*>(pc);
  const int64_t have = std::min<int64_t>(p->h_ctrl->t, p->d.log_cap);
  const int64_t k = std::min<int64_t>(have, capacity);
  int32_t* dst[4] = {entering, leaving_row, leaving_var, flags};
  int32_t* src[4] = {p->d.log_enter, p->d.log_row, p->d.log_leave, p->d.log_flags};
  for (int a = 0; a < 4; ++a)
    if (dst[a] && k > 0)
      HIP_TRY(pageable_copy(dst[a], src[a], sizeof(int32_t) * k, hipMemcpyDeviceToHost, p->stream),
              "reading the pivot log");
  if (count) *count = have;
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_get_tableau(const lp_problem* pc, double* Binv, double* xB, double* W, double* z) try {
  if (!pc) return fail(LP_ERR_ARG, "p is NULL");
  lp_problem* p = const_cast<lp_problem*>(pc);
  const int m = p->m;
  if (p->h_ctrl->r >= 0) return fail(LP_ERR_STATE, "a pivot is pending; call lp_solve to completion first");
  if (Binv && p->d.cmode) HIP_TRY(launch_materialize(p->d, p->stream), "writing B^-1 out");
  if (Binv) {
    // one contiguous copy, unpacked on the host when rows are padded (ld > m); in the
    // out-of-core mode the host copy holds every row but the resident panel's
    std::vector<double> rows;
    double* dst = Binv;
    if (p->ld != m || p->panel) {
      rows.resize((size_t)m * p->ld);
      dst = rows.data();
    }
    if (p->panel) {
      HIP_TRY(hipStreamSynchronize(p->stream), "reading B^-1");
      std::memcpy(dst, p->binv_host, sizeof(double) * (size_t)p->res_lo * p->ld);
      HIP_TRY(pageable_copy(dst + (size_t)p->res_lo * p->ld, p->res, sizeof(double) * (size_t)(m - p->res_lo) * p->ld,
                            hipMemcpyDeviceToHost, p->stream),
              "reading B^-1");
    } else {
      HIP_TRY(pageable_copy(dst, p->d.Binv, sizeof(double) * (size_t)m * p->ld, hipMemcpyDeviceToHost, p->stream),
              "reading B^-1");
    }
    if (dst != Binv)
      for (int i = 0; i < m; ++i) std::memcpy(Binv + (size_t)i * m, &rows[(size_t)i * p->ld], sizeof(double) * m);
  }
  if (xB) HIP_TRY(pageable_copy(xB, p->d.xB, sizeof(double) * m, hipMemcpyDeviceToHost, p->stream), "reading x_B");
  if (W)
    HIP_TRY(pageable_copy(W, p->h_ctrl->wcur ? p->d.W1 : p->d.W0, sizeof(double) * m, hipMemcpyDeviceToHost,
                          p->stream),
            "reading W");
  HIP_TRY(hipStreamSynchronize(p->stream), "reading the tableau");
  if (z) *z = p->h_ctrl->z;
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_get_stats(const lp_problem* p, lp_stats* s) try {
  if (!p || !s) return fail(LP_ERR_ARG, "NULL argument");
  *s = p->stats;
  s->iterations = p->h_ctrl->t;
  s->degenerate = p->h_ctrl->n_degenerate;
  s->ties = p->h_ctrl->n_tie;
  s->aspirations = p->h_ctrl->n_aspiration;
  s->list_clears = p->h_ctrl->n_lclear;
  s->ray = p->h_ctrl->status == LP_UNBOUNDED ? p->h_ctrl->ray : -1;
  s->price32_launches = p->h_ctrl->price32_launches;
  s->full_prices = p->h_ctrl->full_prices;
  s->reinversions = p->h_ctrl->n_reinv;
  s->reinv_failed = p->h_ctrl->n_reinv_failed;
  s->phase1_iterations = p->phase1_t;
  s->memory_case = p->panel ? 2 : 1;
  s->panel_rows = p->panel ? p->panel_rows : 0;
  s->panels = p->panel ? p->npanels : 0;
  s->drive_outs = p->drive_outs;
  s->phase_switch_ms = p->switch_ms;
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_reinvert(lp_problem* p) try {
  if (!p) return fail(LP_ERR_ARG, "p is NULL");
  if (p->panel) return fail(LP_ERR_STATE, "no reinversion in the out-of-core panel mode");
  int rc = read_ctrl(p);  // the structural count and the list D of the current basis
  if (rc != LP_OK) return rc;
  rc = run_reinversion(p);
  if (rc != LP_OK) return rc;
  if ((rc = read_ctrl(p)) != LP_OK) return rc;
  return collect_reinv_time(p);
} catch (...) {
  return host_exception();
}

void lp_destroy(lp_problem* p) { release(p); }

int lp_solve_device_noalloc(int32_t m, int32_t n, const double* A_colmajor, const double* b, const double* c,
                            const lp_options* opt, double* x, double* y, double* objective, int32_t* status,
                            int64_t* iterations) try {
  if (m <= 0 || n < 0) return fail(LP_ERR_ARG, "need m > 0 and n >= 0");
  if (m > LP_MAX_ROWS) return fail(LP_ERR_ARG, "m exceeds LP_MAX_ROWS");
  if ((int64_t)n + m > INT32_MAX / 2) return fail(LP_ERR_ARG, "n + m too large");
  if (!b || (n > 0 && (!A_colmajor || !c))) return fail(LP_ERR_ARG, "NULL data pointer");
  lp_options o;
  lp_default_options(&o);
  if (opt) o = *opt;
  if (int rc = check_options(&o)) return rc;
  if (o.precision != LP_FP64 || o.reinv_period > 0)
    return fail(LP_ERR_ARG, "lp_solve_device_noalloc runs the FP64 form without reinversion only");
  if (o.profile != 0) return fail(LP_ERR_ARG, "lp_solve_device_noalloc does not profile");
  if (o.max_iter == 0) o.max_iter = 10 * ((int64_t)m + n);
  if (o.max_iter > INT32_MAX) return fail(LP_ERR_ARG, "pivot limit above 2^31-1");
  hipStream_t s = static_cast<hipStream_t>(o.stream);
  int dev = 0, num_cu = 0;
  HIP_TRY(hipGetDevice(&dev), "selecting the device");
  HIP_TRY(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev), "querying the device");
  DevLP d{};
  int upd_block = 0, rc = LP_OK;
  d.cmode = compact_columns((int)round_up(m, 8)) ? 1 : 0;  // as lp_create for the FP64 form
  if ((rc = iteration_grids(m, n, num_cu, d.cmode != 0, &d.price_grid, &d.update_grid, &upd_block)) != LP_OK)
    return rc;
  double *b0 = nullptr, *c0 = nullptr;
  int32_t* flag = nullptr;
  {
    Carver count{nullptr};
    const size_t need = carve_lp(count, d, m, n, o.max_iter, &b0, &c0, &flag);
    if (need > kScratchBytes)
      return fail(LP_ERR_ARG, "LP needs " + std::to_string(need) + " bytes, beyond the " +
                                  std::to_string(kScratchBytes) + "-byte array of lp_solve_device_noalloc");
  }
  unsigned char* base = nullptr;
  if ((rc = scratch_address(dev, &base)) != LP_OK) return rc;
  Carver cv{base};
  carve_lp(cv, d, m, n, o.max_iter, &b0, &c0, &flag);
  d.m = m;
  d.n = n;
  d.ld = (int32_t)round_up(m, 8);
  d.a_nt = price_nt(d.ld, n) ? 1 : 0;
  d.upd_block = upd_block;
  d.row_lo = 0;
  d.row_hi = m;
  d.rowsrc = nullptr;
  d.log_cap = o.max_iter;
  d.Lcap = (int32_t)o.max_iter;
  d.tenure = o.tabu_tenure;
  d.use_llist = o.leaving_list ? 1 : 0;
  d.eps_d = o.eps_d;
  d.eps_p = o.eps_p;
  d.eps_z = o.eps_z;
  d.eps_t = o.eps_t;
  d.sl_k = o.shortlist_k;
  // Inputs: packed into the padded layout and validated on the device.
  HIP_TRY(launch_clear_flag(flag, s), "validating the LP");
  HIP_TRY(launch_pack_lp(const_cast<double*>(d.A), d.ld, A_colmajor, m, n, b0, b, c0, c, flag, s),
          "copying the LP");
  int32_t hflag = 0;
  HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s), "validating the LP");
  HIP_TRY(hipStreamSynchronize(s), "validating the LP");
  if (hflag & 1) return fail(LP_ERR_ARG, "A, b or c contains a non-finite value");
  if (hflag & 2) return fail(LP_ERR_NEG_RHS, "b_i < 0: the slack basis is infeasible");
  HIP_TRY(launch_init(d, b0, c0, o.sense == LP_MAX ? -1.0 : 1.0, s), "initialising the slack basis");
  HIP_TRY(launch_arm(d.ctrl, o.max_iter, s), "arming the solve");
  // Iterations launched directly (a graph would be created and instantiated), iters_per_sync
  // per read-back of the control block; the kernels do nothing once the status has changed.
  Ctrl hc{};
  const int K = o.iters_per_sync;
  int64_t t_before = 0;
  for (;;) {
    for (int k = 0; k < K; ++k) {
      HIP_TRY(launch_price(d, d.price_grid, s), "launching the pricing kernel");
      HIP_TRY(launch_update(d, d.update_grid, s), "launching the update kernel");
      HIP_TRY(launch_finish(d, s), "launching the finishing kernel");
    }
    HIP_TRY(hipMemcpyAsync(&hc, d.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s), "reading status");
    HIP_TRY(hipStreamSynchronize(s), "reading status");
    if (hc.status != LP_RUNNING) break;
    if (hc.t != t_before + K) return fail(LP_ERR_DEVICE, "iterations made no progress while RUNNING");
    t_before = hc.t;
  }
  HIP_TRY(launch_solution(d, c0, o.sense == LP_MAX ? -1.0 : 1.0, x, y, objective, s), "writing the solution");
  HIP_TRY(hipStreamSynchronize(s), "writing the solution");
  if (status) *status = hc.status;
  if (iterations) *iterations = hc.t;
  return LP_OK;
} catch (...) {
  return host_exception();
}

const char* lp_error_string(int code) {
  static thread_local std::string text;
  const char* base = "unknown code";
  switch (code) {
    case LP_OK: base = "ok"; break;
    case LP_ERR_ARG: base = "invalid argument"; break;
    case LP_ERR_NEG_RHS: base = "negative right-hand side"; break;
    case LP_ERR_NOMEM: base = "out of memory"; break;
    case LP_ERR_DEVICE: base = "device error"; break;
    case LP_ERR_STATE: base = "invalid state"; break;
  }
  try {
    text = base;
    if (code != LP_OK && code == g_code && !g_msg.empty()) text += ": " + g_msg;
    return text.c_str();
  } catch (...) {  // no memory for the detail: the code's own text
    return base;
  }
}

}  // extern "C"
