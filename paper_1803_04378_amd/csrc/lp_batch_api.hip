// Host side of the batched solver: packing, work-item order, autotuner, C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "lp_batch.h"
#include "lp_device.h"
#include "lp_gen.h"
#include "lpgpu.h"

using namespace lpgpu;

namespace lpgpu {
// Shared with lp_api.hip: error recording for lp_error_string, and the conversion of a
// host exception (inside a catch-all handler) into LP_ERR_NOMEM.
int record_error(int code, const std::string& msg);
int host_exception() noexcept;
}  // namespace lpgpu

namespace {

int fail(int code, const std::string& msg) { return lpgpu::record_error(code, msg); }

int fail_hip(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? LP_ERR_NOMEM : LP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

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

// Transfers from pageable host memory: the stream is drained, then a blocking copy runs, so
// the copy follows the stream's earlier work and is complete on return.
hipError_t pageable_copy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s) {
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess && bytes > 0) e = hipMemcpy(dst, src, bytes, kind);
  return e;
}

#define HIP_TRY(expr, what)                            \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return fail_hip(e_, what);   \
  } while (0)

// m-buckets of the autotuner: (16k, 16k+16]; narrow mode is only possible while one LP
// fits a wavefront's LDS slot.
constexpr int kBucketWidth = 16;
// LDS a workgroup may take (the kernel's static LDS comes on top).
constexpr size_t kLdsLimit = 160 * 1024 - 1024;
// Thresholds tried by the autotuner for keeping B^-1 in LDS (LPs with m <= threshold).
constexpr int kBinvCandidates[] = {0, 48, 96, 128};

}  // namespace

struct lp_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  lp_options opt{};
  int32_t count = 0;
  std::vector<BatchLP> lps;        // host copy (waves set per solve)
  std::vector<std::vector<double>> c;  // host copies of c for the objective
  std::vector<void*> allocs;
  BatchDev d{};
  BatchLP* d_lps = nullptr;
  int4* d_items = nullptr;
  int32_t max_items = 0;
  size_t region = 0;  // LDS bytes per workgroup (B^-1 in HBM)
  int64_t poolA = 0, poolb = 0, poolc = 0;  // doubles in the A', b and c pools
  int grid = 0, per_cu = 0, num_cu = 0;
  int small_m = -1;   // LPs with m <= small_m are solved one per wavefront (after tuning)
  std::vector<int> bucket_narrow;  // per bucket: 1 narrow, 0 wide, -1 untuned
  int binv_opt = -1;    // option batch_binv_lds_m
  int binv_m = 0;       // wide LPs with m <= binv_m keep B^-1 in LDS (second launch)
  bool binv_tuned = false;
  size_t region_l = 0;  // LDS bytes per workgroup of that launch
  int grid_l = 0;
  bool solved = false;
  std::string arch;     // the device's architecture name, the key of the tune table
  int64_t loaded_buckets = 0;  // buckets whose mode came from a tune table
  double solve_ms = 0.0, tune_ms = 0.0;
  int64_t narrow_lps = 0, wide_lps = 0, binv_lds_lps = 0, items_last = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

template <class T>
hipError_t dalloc(lp_batch* p, T** out, size_t count) {
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

void release(lp_batch* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (void* ptr : p->allocs) (void)hipFree(ptr);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

// Relative cost of one LP for ordering work items: bytes per iteration (~8 m (n + 2m))
// times an iteration count growing with m, divided by the wavefronts on it.
double lp_cost(const BatchLP& L, int waves) {
  return (double)L.m * ((double)L.n + 2.0 * L.m) * (double)L.m / waves;
}

// Work items for the LPs in `ids` (indices into p->lps) under the current modes, largest
// first.  Narrow LPs are packed four per item in descending size.
std::vector<int4> make_items(const lp_batch* p, const std::vector<int>& ids) {
  std::vector<int> wide, narrow;
  for (int i : ids) (p->lps[i].waves == 1 ? narrow : wide).push_back(i);
  auto bigger = [&](int a, int b) {
    const double ca = lp_cost(p->lps[a], 1), cb = lp_cost(p->lps[b], 1);
    return ca != cb ? ca > cb : a < b;
  };
  std::sort(wide.begin(), wide.end(), bigger);
  std::sort(narrow.begin(), narrow.end(), bigger);
  struct Item {
    int4 ids;
    double cost;
  };
  std::vector<Item> items;
  for (int i : wide) items.push_back({make_int4(i, -1, -1, -1), lp_cost(p->lps[i], kBatchWaves)});
  for (size_t k = 0; k < narrow.size(); k += 4) {
    int4 it = make_int4(narrow[k], -1, -1, -1);
    if (k + 1 < narrow.size()) it.y = narrow[k + 1];
    if (k + 2 < narrow.size()) it.z = narrow[k + 2];
    if (k + 3 < narrow.size()) it.w = narrow[k + 3];
    items.push_back({it, lp_cost(p->lps[narrow[k]], 1)});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
  std::vector<int4> out;
  out.reserve(items.size());
  for (auto& it : items) out.push_back(it.ids);
  return out;
}

// One persistent launch over `items`: B^-1 in HBM (binv_lds false) or in LDS.
int run_items(lp_batch* p, const std::vector<int4>& items, float* ms, bool binv_lds = false) {
  if (items.empty()) {
    if (ms) *ms = 0.f;
    return LP_OK;
  }
  HIP_TRY(pageable_copy(p->d_lps, p->lps.data(), sizeof(BatchLP) * p->lps.size(), hipMemcpyHostToDevice, p->stream),
          "uploading the batch table");
  HIP_TRY(pageable_copy(p->d_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, p->stream),
          "uploading work items");
  HIP_TRY(hipMemsetAsync(p->d.queue, 0, sizeof(int32_t), p->stream), "clearing the work queue");
  BatchDev d = p->d;
  d.n_items = (int32_t)items.size();
  HIP_TRY(hipEventRecord(p->ev0, p->stream), "recording an event");
  const int grid = std::min<int>(binv_lds ? p->grid_l : p->grid, (int)items.size());
  HIP_TRY(launch_batch(d, grid, binv_lds ? p->region_l : p->region, binv_lds, p->stream),
          "launching the batched solver");
  HIP_TRY(hipEventRecord(p->ev1, p->stream), "recording an event");
  HIP_TRY(hipEventSynchronize(p->ev1), "running the batched solver");
  float t = 0.f;
  HIP_TRY(hipEventElapsedTime(&t, p->ev0, p->ev1), "timing the batched solver");
  if (ms) *ms = t;
  return LP_OK;
}

int bucket_of(int m) { return (m - 1) / kBucketWidth; }

// Chooses narrow or wide per m-bucket by timing both on the bucket's LPs.
int autotune(lp_batch* p) {
  const auto t0 = std::chrono::steady_clock::now();
  const size_t slot = p->region / kBatchWaves;
  std::vector<std::vector<int>> buckets;
  for (int i = 0; i < p->count; ++i) {
    const BatchLP& L = p->lps[i];
    if (batch_lds_bytes(L.m, L.n) > slot) continue;
    const int bk = bucket_of(L.m);
    if ((int)buckets.size() <= bk) buckets.resize(bk + 1);
    buckets[bk].push_back(i);
  }
  if (p->bucket_narrow.size() < buckets.size()) p->bucket_narrow.resize(buckets.size(), -1);
  for (size_t bk = 0; bk < buckets.size(); ++bk) {
    if (buckets[bk].empty() || p->bucket_narrow[bk] >= 0) continue;  // none, or from a tune table
    float best[2] = {0.f, 0.f};
    for (int narrow = 0; narrow < 2; ++narrow) {
      for (int i : buckets[bk]) p->lps[i].waves = narrow ? 1 : kBatchWaves;
      const std::vector<int4> items = make_items(p, buckets[bk]);
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {  // the second run is timed
        int rc = run_items(p, items, &ms);
        if (rc != LP_OK) return rc;
      }
      best[narrow] = ms;
    }
    p->bucket_narrow[bk] = best[1] < best[0] ? 1 : 0;
  }
  p->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return LP_OK;
}

// Narrow or wide per LP (the tuned buckets or small_m), then B^-1 in LDS for wide LPs
// with m <= binv_m whose vectors and B^-1 fit a workgroup's LDS, and that launch's LDS
// size and grid.
int assign_modes(lp_batch* p) {
  const size_t slot = p->region / kBatchWaves;
  p->narrow_lps = p->wide_lps = p->binv_lds_lps = 0;
  size_t need = 0;
  for (auto& L : p->lps) {
    bool narrow = false;
    if (batch_lds_bytes(L.m, L.n) <= slot) {
      if (p->small_m >= 0) {
        narrow = L.m <= p->small_m;
      } else {
        const int bk = bucket_of(L.m);
        narrow = bk < (int)p->bucket_narrow.size() && p->bucket_narrow[bk] == 1;  // -1: no LP timed it
      }
    }
    L.waves = narrow ? 1 : kBatchWaves;
    (narrow ? p->narrow_lps : p->wide_lps) += 1;
    L.binv_lds = (!narrow && L.m <= p->binv_m && batch_lds_bytes_binv(L.m, L.n) <= kLdsLimit) ? 1 : 0;
    if (L.binv_lds) {
      p->binv_lds_lps += 1;
      need = std::max(need, batch_lds_bytes_binv(L.m, L.n));
    }
  }
  p->region_l = need;
  p->grid_l = 0;
  if (need > 0) {
    int per_cu = 0;
    HIP_TRY(batch_occupancy(&per_cu, need, true), "querying occupancy");
    if (per_cu < 1) return fail(LP_ERR_DEVICE, "batched solver: no occupancy with B^-1 in LDS");
    p->grid_l = per_cu * p->num_cu;
  }
  return LP_OK;
}

// Every LP of the batch: the LPs with B^-1 in HBM in one launch, the others in a second
// one; *ms is the sum of their device times and *items their work items.
int solve_all(lp_batch* p, float* ms, int64_t* items_out) {
  std::vector<int> hbm, lds;
  for (int i = 0; i < p->count; ++i) (p->lps[i].binv_lds ? lds : hbm).push_back(i);
  const std::vector<int4> ih = make_items(p, hbm), il = make_items(p, lds);
  float m1 = 0.f, m2 = 0.f;
  int rc;
  if ((rc = run_items(p, ih, &m1, false)) != LP_OK) return rc;
  if ((rc = run_items(p, il, &m2, true)) != LP_OK) return rc;
  if (ms) *ms = m1 + m2;
  if (items_out) *items_out = (int64_t)(ih.size() + il.size());
  return LP_OK;
}

// The B^-1-in-LDS threshold: every candidate that moves some LP to LDS is timed once on
// the whole batch (modes of the tuned buckets; the bucket tuning has warmed the kernels),
// the fastest kept.  No timing at all when no candidate applies to any LP.
int tune_binv(lp_batch* p) {
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<int> cands;
  for (int cand : kBinvCandidates) {
    p->binv_m = cand;
    int rc = assign_modes(p);
    if (rc != LP_OK) return rc;
    if (cand == 0 || p->binv_lds_lps > 0) cands.push_back(cand);
  }
  float best = 0.f;
  int best_m = 0;
  for (size_t k = 0; cands.size() > 1 && k < cands.size(); ++k) {
    p->binv_m = cands[k];
    int rc = assign_modes(p);
    if (rc != LP_OK) return rc;
    float ms = 0.f;
    if ((rc = solve_all(p, &ms, nullptr)) != LP_OK) return rc;
    if (k == 0 || ms < best) {
      best = ms;
      best_m = cands[k];
    }
  }
  p->binv_m = best_m;
  p->binv_tuned = true;
  p->tune_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return LP_OK;
}

// ---- the persistent tune table ----
// A JSON array with one object per line: {"arch": A, "precision": "fp64", "bucket_width":
// 16, "bucket": k, "narrow": 0|1} for the mode of m-bucket k (m in (16k, 16k+16]) on
// architecture A, and {"arch": A, "precision": "fp64", "binv_lds_m": t} for the B^-1-in-LDS
// threshold last chosen there.
struct TuneTable {
  std::map<std::pair<std::string, int>, int> narrow;  // (arch, bucket) -> mode
  std::map<std::string, int> binv;                    // arch -> threshold
};

bool json_str(const std::string& line, const char* key, std::string* out) {
  const std::string k = std::string("\"") + key + "\": \"";
  const size_t a = line.find(k);
  if (a == std::string::npos) return false;
  const size_t b = line.find('"', a + k.size());
  if (b == std::string::npos) return false;
  *out = line.substr(a + k.size(), b - a - k.size());
  return true;
}

bool json_int(const std::string& line, const char* key, long* out) {
  const std::string k = std::string("\"") + key + "\": ";
  const size_t a = line.find(k);
  if (a == std::string::npos) return false;
  char* end = nullptr;
  const long v = std::strtol(line.c_str() + a + k.size(), &end, 10);
  if (end == line.c_str() + a + k.size()) return false;
  *out = v;
  return true;
}

// Reads the records of precision fp64 (a missing file is an empty table).
void read_table(const char* path, TuneTable* t) {
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::string arch, prec;
    long v = 0, w = 0, bk = 0;
    if (!json_str(line, "arch", &arch) || !json_str(line, "precision", &prec) || prec != "fp64") continue;
    if (json_int(line, "binv_lds_m", &v)) {
      t->binv[arch] = (int)v;
    } else if (json_int(line, "bucket", &bk) && json_int(line, "narrow", &v) && json_int(line, "bucket_width", &w) &&
               w == kBucketWidth && bk >= 0 && bk < 4096) {
      t->narrow[{arch, (int)bk}] = v ? 1 : 0;
    }
  }
}

int write_table(const char* path, const TuneTable& t) {
  std::ostringstream o;
  o << "[\n";
  bool first = true;
  for (const auto& kv : t.narrow) {
    o << (first ? "" : ",\n") << "{\"arch\": \"" << kv.first.first << "\", \"precision\": \"fp64\", \"bucket_width\": "
      << kBucketWidth << ", \"bucket\": " << kv.first.second << ", \"m_lo\": " << kv.first.second * kBucketWidth + 1
      << ", \"m_hi\": " << (kv.first.second + 1) * kBucketWidth << ", \"narrow\": " << kv.second << "}";
    first = false;
  }
  for (const auto& kv : t.binv) {
    o << (first ? "" : ",\n") << "{\"arch\": \"" << kv.first << "\", \"precision\": \"fp64\", \"binv_lds_m\": "
      << kv.second << "}";
    first = false;
  }
  o << "\n]\n";
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return fail(LP_ERR_ARG, std::string("cannot write the tune table ") + tmp);
    f << o.str();
    if (!f.good()) return fail(LP_ERR_ARG, std::string("cannot write the tune table ") + tmp);
  }
  if (std::rename(tmp.c_str(), path) != 0) return fail(LP_ERR_ARG, std::string("cannot replace ") + path);
  return LP_OK;
}

int load_table(lp_batch* p, const char* path) {
  TuneTable t;
  read_table(path, &t);
  int64_t got = 0;
  for (const auto& kv : t.narrow) {
    if (kv.first.first != p->arch) continue;
    const int bk = kv.first.second;
    if ((int)p->bucket_narrow.size() <= bk) p->bucket_narrow.resize(bk + 1, -1);
    p->bucket_narrow[bk] = kv.second;
    ++got;
  }
  p->loaded_buckets = got;
  auto it = t.binv.find(p->arch);
  if (it != t.binv.end() && p->binv_opt < 0) {
    p->binv_m = it->second;
    p->binv_tuned = true;
  }
  return LP_OK;
}

int save_table(const lp_batch* p, const char* path) {
  TuneTable t;
  read_table(path, &t);
  for (size_t bk = 0; bk < p->bucket_narrow.size(); ++bk)
    if (p->bucket_narrow[bk] >= 0) t.narrow[{p->arch, (int)bk}] = p->bucket_narrow[bk];
  if (p->binv_tuned) t.binv[p->arch] = p->binv_m;
  return write_table(path, t);
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// A batch of count LPs of sizes m[i] x n[i] with every device buffer allocated and laid
// out (A', b and c not filled yet; c_host holds no data yet).  On success *out owns it.
int batch_alloc(lp_batch** out, int32_t count, const int32_t* m, const int32_t* n, const lp_options& o) {
  size_t max_bytes = 0, max_small = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (m[i] <= 0 || n[i] < 0) return fail(LP_ERR_ARG, "LP " + std::to_string(i) + ": invalid size");
    const size_t bytes = batch_lds_bytes(m[i], n[i]);
    max_bytes = std::max(max_bytes, bytes);
    if (m[i] <= 4 * kBucketWidth) max_small = std::max(max_small, bytes);
  }
  // a multiple of 64, so that the narrow items' per-wavefront slots stay 16-byte aligned
  const size_t region = (std::max(max_bytes, kBatchWaves * max_small) + 63) / 64 * 64;
  if (region > 160 * 1024 - 1024) return fail(LP_ERR_ARG, "an LP of the batch is too large for the batched solver");

  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "selecting the device");
  lp_batch* p = new (std::nothrow) lp_batch();
  if (!p) return fail(LP_ERR_NOMEM, "host allocation failed");
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
  p->count = count;
  p->region = region;
  p->small_m = o.batch_small_m;
  p->binv_opt = o.batch_binv_lds_m;
  if (o.stream) {
    p->stream = static_cast<hipStream_t>(o.stream);
  } else {
    hipError_t e = hipStreamCreate(&p->stream);
    if (e != hipSuccess) return bail(fail_hip(e, "creating a stream"));
    p->own_stream = true;
  }
  {
    hipError_t e = hipEventCreate(&p->ev0);
    if (e == hipSuccess) e = hipEventCreate(&p->ev1);
    if (e != hipSuccess) return bail(fail_hip(e, "creating events"));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return bail(fail_hip(e, "querying the device"));
    p->num_cu = prop.multiProcessorCount;
    p->arch = prop.gcnArchName;
    e = batch_occupancy(&p->per_cu, region, false);
    if (e != hipSuccess) return bail(fail_hip(e, "querying occupancy"));
    if (p->per_cu < 1) return bail(fail(LP_ERR_ARG, "batched solver does not fit the device"));
    p->grid = p->per_cu * p->num_cu;
  }
  // Pool layout.
  p->lps.resize(count);
  p->c.resize(count);
  int64_t oA = 0, ob = 0, oc = 0, oB = 0, oI = 0, oL = 0, oO = 0;
  for (int32_t i = 0; i < count; ++i) {
    BatchLP& L = p->lps[i];
    L.m = m[i];
    L.n = n[i];
    L.ld = (m[i] + 7) / 8 * 8;
    L.waves = kBatchWaves;
    L.cap = o.max_iter > 0 ? o.max_iter : 10 * ((int64_t)m[i] + n[i]);
    L.offA = oA;
    L.offb = ob;
    L.offc = oc;
    L.offB = oB;
    L.offI = oI;
    L.offLog = oL;
    L.offOut = oO;
    oA += (int64_t)L.ld * std::max(L.n, 1);
    ob += L.m;
    oc += std::max(L.n, 1);
    oB += (int64_t)L.m * L.ld;
    oI += 2 * ((int64_t)L.n + L.m);
    oL += L.cap;
    oO += L.m;
  }
  p->poolA = oA;
  p->poolb = ob;
  p->poolc = oc;
  double* dA = nullptr;
  double* db = nullptr;
  double* dc = nullptr;
#define ALLOC(ptr, cnt)                                                    \
  do {                                                                     \
    hipError_t e_ = dalloc(p, &(ptr), (size_t)(cnt));                      \
    if (e_ != hipSuccess) return bail(fail_hip(e_, "allocating " #ptr)); \
  } while (0)
  ALLOC(dA, oA);
  ALLOC(db, ob);
  ALLOC(dc, oc);
  ALLOC(p->d.Binv, oB);
  ALLOC(p->d.iscr, oI);
  ALLOC(p->d.log_enter, oL);
  ALLOC(p->d.log_row, oL);
  ALLOC(p->d.log_leave, oL);
  ALLOC(p->d.log_flags, oL);
  ALLOC(p->d.Lq, oL);
  ALLOC(p->d.Ll, oL);
  ALLOC(p->d.Lgen, oL);
  ALLOC(p->d.xB_out, oO);
  ALLOC(p->d.basis_out, oO);
  ALLOC(p->d.status_out, count);
  ALLOC(p->d.iters_out, count);
  ALLOC(p->d.z_out, count);
  ALLOC(p->d.ray_out, count);
  ALLOC(p->d.queue, 1);
  ALLOC(p->d_lps, count);
  ALLOC(p->d_items, count);
#undef ALLOC
  p->d.A = dA;
  p->d.b = db;
  p->d.c = dc;
  p->d.lps = p->d_lps;
  p->d.items = p->d_items;
  p->d.slot_bytes = (int32_t)(region / kBatchWaves);
  p->d.sense = o.sense == LP_MAX ? -1.0 : 1.0;
  p->d.tenure = o.tabu_tenure;
  p->d.use_llist = o.leaving_list ? 1 : 0;
  p->d.eps_d = o.eps_d;
  p->d.eps_p = o.eps_p;
  p->d.eps_z = o.eps_z;
  p->d.eps_t = o.eps_t;
  *out = p;
  p = nullptr;  // handed over
  return LP_OK;
}

int batch_options(const lp_options* opt, lp_options* o) {
  lp_default_options(o);
  if (opt) *o = *opt;
  if (o->sense != LP_MIN && o->sense != LP_MAX) return fail(LP_ERR_ARG, "options.sense must be LP_MIN or LP_MAX");
  if (o->tabu_tenure < 0 || o->max_iter < 0 || o->batch_binv_lds_m < -1) return fail(LP_ERR_ARG, "invalid options");
  if (o->precision != LP_FP64 || o->reinv_period > 0)
    return fail(LP_ERR_ARG, "the batched solver runs in FP64 without reinversion (precision LP_FP64, reinv_period <= 0)");
  return LP_OK;
}

void load_table_from_env(lp_batch* p) {
  if (const char* path = std::getenv("LPGPU_BATCH_TUNE")) {
    if (*path) load_table(p, path);
  }
}

}  // namespace

extern "C" {

int lp_batch_create(lp_batch** out, int32_t count, const int32_t* m, const int32_t* n, const double* const* A,
                    const double* const* b, const double* const* c, const lp_options* opt) try {
  if (!out) return fail(LP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (count <= 0 || !m || !n || !A || !b || !c) return fail(LP_ERR_ARG, "empty batch or NULL array");
  lp_options o;
  if (int rc = batch_options(opt, &o)) return rc;
  for (int32_t i = 0; i < count; ++i) {
    if (m[i] <= 0 || n[i] < 0 || !b[i] || (n[i] > 0 && (!A[i] || !c[i])))
      return fail(LP_ERR_ARG, "LP " + std::to_string(i) + ": invalid size or NULL data");
    const size_t cnt = (size_t)m[i] * n[i];
    for (size_t k = 0; k < cnt; ++k)
      if (!std::isfinite(A[i][k])) return fail(LP_ERR_ARG, "LP " + std::to_string(i) + ": non-finite A");
    for (int32_t k = 0; k < m[i]; ++k) {
      if (!std::isfinite(b[i][k])) return fail(LP_ERR_ARG, "LP " + std::to_string(i) + ": non-finite b");
      if (b[i][k] < 0.0) return fail(LP_ERR_NEG_RHS, "LP " + std::to_string(i) + ": b_i < 0");
    }
    for (int32_t k = 0; k < n[i]; ++k)
      if (!std::isfinite(c[i][k])) return fail(LP_ERR_ARG, "LP " + std::to_string(i) + ": non-finite c");
  }
  lp_batch* p = nullptr;
  if (int rc = batch_alloc(&p, count, m, n, o)) return rc;
  auto bail = [&](int code) {
    release(p);
    p = nullptr;
    return code;
  };
  const auto drop = on_scope_exit([&] {
    if (p) release(p);
  });
  for (int32_t i = 0; i < count; ++i) p->c[i].assign(c[i], c[i] + n[i]);
  double* dA = const_cast<double*>(p->d.A);
  double* db = const_cast<double*>(p->d.b);
  double* dc = const_cast<double*>(p->d.c);
  const int64_t oA = p->poolA, ob = p->poolb, oc = p->poolc;
  // Upload.  The LPs' A' blocks are consecutive in the pool, so runs of consecutive LPs
  // are packed (columns padded to ld rows with zeros) into one of two pinned staging
  // buffers while the other one's copy is in flight.
  {
    std::vector<double> hb((size_t)ob), hc((size_t)oc, 0.0);
    for (int32_t i = 0; i < count; ++i) {
      const BatchLP& L = p->lps[i];
      std::memcpy(&hb[L.offb], b[i], sizeof(double) * L.m);
      if (L.n) std::memcpy(&hc[L.offc], c[i], sizeof(double) * L.n);
    }
    size_t largest = 0;
    for (const BatchLP& L : p->lps) largest = std::max(largest, (size_t)L.ld * std::max(L.n, 1));
    const size_t cap = std::min<size_t>((size_t)oA, std::max<size_t>((size_t)8 << 20, largest));  // doubles
    double* stage[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
      e = hipHostMalloc(reinterpret_cast<void**>(&stage[k]), sizeof(double) * cap, hipHostMallocDefault);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&done[k], hipEventDisableTiming);
    }
    int buf = 0;
    bool pending[2] = {false, false};
    size_t used = 0, run_start = 0;  // doubles packed in stage[buf]; pool offset of its first
    auto flush = [&]() -> hipError_t {
      if (used == 0) return hipSuccess;
      hipError_t f = hipMemcpyAsync(dA + run_start, stage[buf], sizeof(double) * used, hipMemcpyHostToDevice,
                                    p->stream);
      if (f == hipSuccess) f = hipEventRecord(done[buf], p->stream);
      pending[buf] = true;
      buf ^= 1;
      used = 0;
      if (f == hipSuccess && pending[buf]) f = hipEventSynchronize(done[buf]);  // the other copy is done
      pending[buf] = false;
      return f;
    };
    // Runs of LPs that fill a staging buffer; each run is packed by up to 8 threads.
    const unsigned hw = std::thread::hardware_concurrency();
    const int nthreads = (int)std::max(1u, std::min(8u, hw));
    auto pack = [&](int32_t i, double* dst) {
      const BatchLP& L = p->lps[i];
      for (int32_t j = 0; j < L.n; ++j) {
        std::memcpy(dst + (size_t)j * L.ld, A[i] + (size_t)j * L.m, sizeof(double) * L.m);
        std::memset(dst + (size_t)j * L.ld + L.m, 0, sizeof(double) * (L.ld - L.m));
      }
      if (L.n == 0) std::memset(dst, 0, sizeof(double) * L.ld);
    };
    for (int32_t i0 = 0; i0 < count && e == hipSuccess;) {
      int32_t i1 = i0;
      size_t sz = 0;
      while (i1 < count) {
        const size_t s1 = (size_t)p->lps[i1].ld * std::max(p->lps[i1].n, 1);
        if (sz + s1 > cap) break;
        sz += s1;
        ++i1;
      }
      run_start = (size_t)p->lps[i0].offA;
      double* base = stage[buf];
      auto work = [&](int tno) {
        for (int32_t i = i0 + tno; i < i1; i += nthreads) pack(i, base + ((size_t)p->lps[i].offA - run_start));
      };
      std::vector<std::thread> pool;
      int started = 1;
      try {
        pool.reserve(nthreads);
        for (; started < nthreads && i0 + started < i1; ++started) pool.emplace_back(work, started);
      } catch (...) {  // a thread that could not start: this one packs its share
      }
      for (int tno = started; tno < nthreads && i0 + tno < i1; ++tno) work(tno);
      work(0);
      for (auto& th : pool) th.join();
      used = sz;
      e = flush();
      i0 = i1;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    for (int k = 0; k < 2; ++k) {
      if (stage[k]) (void)hipHostFree(stage[k]);
      if (done[k]) (void)hipEventDestroy(done[k]);
    }
    if (e == hipSuccess) e = hipMemcpy(db, hb.data(), sizeof(double) * hb.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dc, hc.data(), sizeof(double) * hc.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(fail_hip(e, "uploading the batch"));
  }
  load_table_from_env(p);
  *out = p;
  p = nullptr;  // handed over
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_batch_create_dense(lp_batch** out, int32_t count, uint64_t seed, int32_t m_lo, int32_t m_hi,
                          const lp_options* opt) try {
  if (!out) return fail(LP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (count <= 0 || m_lo < 1 || m_hi < m_lo) return fail(LP_ERR_ARG, "need count > 0 and 1 <= m_lo <= m_hi");
  lp_options o;
  if (int rc = batch_options(opt, &o)) return rc;
  // sizes: m_i = m_lo + (h(seed, 6, i) mod (m_hi - m_lo + 1)), n_i = 2 m_i
  std::vector<int32_t> m(count), n(count);
  const uint64_t ks = gen::stream_key(seed, gen::kStreamSize), span = (uint64_t)(m_hi - m_lo) + 1;
  for (int32_t i = 0; i < count; ++i) {
    m[i] = m_lo + (int32_t)(gen::hash(ks, (uint64_t)i) % span);
    n[i] = 2 * m[i];
  }
  lp_batch* p = nullptr;
  if (int rc = batch_alloc(&p, count, m.data(), n.data(), o)) return rc;
  auto bail = [&](int code) {
    release(p);
    p = nullptr;
    return code;
  };
  const auto drop = on_scope_exit([&] {
    if (p) release(p);
  });
  hipError_t e = pageable_copy(p->d_lps, p->lps.data(), sizeof(BatchLP) * p->lps.size(), hipMemcpyHostToDevice,
                               p->stream);
  if (e == hipSuccess)
    e = launch_gen_batch(p->d_lps, count, seed, const_cast<double*>(p->d.A), const_cast<double*>(p->d.b),
                         const_cast<double*>(p->d.c), p->stream);
  // the costs on the host as well (the objective is formed there): copied back
  std::vector<double> hc((size_t)p->poolc);
  if (e == hipSuccess)
    e = pageable_copy(hc.data(), p->d.c, sizeof(double) * hc.size(), hipMemcpyDeviceToHost, p->stream);
  if (e != hipSuccess) return bail(fail_hip(e, "generating the batch"));
  for (int32_t i = 0; i < count; ++i)
    p->c[i].assign(hc.begin() + p->lps[i].offc, hc.begin() + p->lps[i].offc + n[i]);
  load_table_from_env(p);
  *out = p;
  p = nullptr;  // handed over
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_batch_solve(lp_batch* p) try {
  if (!p) return fail(LP_ERR_ARG, "p is NULL");
  int rc;
  bool tuned = false;
  if (p->small_m < 0 && !p->solved) {
    p->tune_ms = 0.0;
    if ((rc = autotune(p)) != LP_OK) return rc;  // times only buckets no table named
    tuned = true;
  }
  if (p->binv_opt >= 0) {
    p->binv_m = p->binv_opt;
  } else if (!p->binv_tuned) {
    if ((rc = tune_binv(p)) != LP_OK) return rc;
    tuned = true;
  }
  if (tuned) {
    if (const char* path = std::getenv("LPGPU_BATCH_TUNE"))
      if (*path && (rc = save_table(p, path)) != LP_OK) return rc;
  }
  if ((rc = assign_modes(p)) != LP_OK) return rc;
  float ms = 0.f;
  if ((rc = solve_all(p, &ms, &p->items_last)) != LP_OK) return rc;
  p->solve_ms = ms;
  p->solved = true;
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_batch_results(const lp_batch* pc, int32_t* status, double* objective, int64_t* iterations) try {
  if (!pc) return fail(LP_ERR_ARG, "p is NULL");
  if (!pc->solved) return fail(LP_ERR_STATE, "lp_batch_solve has not run");
  lp_batch* p = const_cast<lp_batch*>(pc);
  const int count = p->count;
  std::vector<int32_t> st(count);
  std::vector<int64_t> it(count);
  HIP_TRY(hipMemcpy(st.data(), p->d.status_out, sizeof(int32_t) * count, hipMemcpyDeviceToHost), "reading results");
  HIP_TRY(hipMemcpy(it.data(), p->d.iters_out, sizeof(int64_t) * count, hipMemcpyDeviceToHost), "reading results");
  if (status) std::memcpy(status, st.data(), sizeof(int32_t) * count);
  if (iterations) std::memcpy(iterations, it.data(), sizeof(int64_t) * count);
  if (objective) {
    const int64_t total = p->lps.back().offOut + p->lps.back().m;
    std::vector<double> xB((size_t)total);
    std::vector<int32_t> bas((size_t)total);
    HIP_TRY(hipMemcpy(xB.data(), p->d.xB_out, sizeof(double) * total, hipMemcpyDeviceToHost), "reading x_B");
    HIP_TRY(hipMemcpy(bas.data(), p->d.basis_out, sizeof(int32_t) * total, hipMemcpyDeviceToHost), "reading bases");
    for (int i = 0; i < count; ++i) {
      const BatchLP& L = p->lps[i];
      std::vector<int32_t> row_of(L.n, -1);
      for (int k = 0; k < L.m; ++k)
        if (bas[L.offOut + k] < L.n) row_of[bas[L.offOut + k]] = k;
      double s = 0.0;
      for (int j = 0; j < L.n; ++j)
        if (row_of[j] >= 0) s += p->c[i][j] * xB[L.offOut + row_of[j]];
      objective[i] = s;
    }
  }
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_batch_get(const lp_batch* pc, int32_t i, double* x, int32_t* basis, int32_t* entering, int32_t* leaving_row,
                 int32_t* flags, int64_t capacity, int64_t* count) try {
  if (!pc) return fail(LP_ERR_ARG, "p is NULL");
  if (i < 0 || i >= pc->count) return fail(LP_ERR_ARG, "LP index out of range");
  if (!pc->solved) return fail(LP_ERR_STATE, "lp_batch_solve has not run");
  lp_batch* p = const_cast<lp_batch*>(pc);
  const BatchLP& L = p->lps[i];
  std::vector<double> xB(L.m);
  std::vector<int32_t> bas(L.m);
  int64_t t = 0;
  HIP_TRY(hipMemcpy(xB.data(), p->d.xB_out + L.offOut, sizeof(double) * L.m, hipMemcpyDeviceToHost), "reading x_B");
  HIP_TRY(hipMemcpy(bas.data(), p->d.basis_out + L.offOut, sizeof(int32_t) * L.m, hipMemcpyDeviceToHost),
          "reading the basis");
  HIP_TRY(hipMemcpy(&t, p->d.iters_out + i, sizeof(int64_t), hipMemcpyDeviceToHost), "reading the pivot count");
  if (x) {
    for (int j = 0; j < L.n; ++j) x[j] = 0.0;
    for (int k = 0; k < L.m; ++k)
      if (bas[k] < L.n) x[bas[k]] = xB[k];
  }
  if (basis) std::memcpy(basis, bas.data(), sizeof(int32_t) * L.m);
  const int64_t have = std::min<int64_t>(t, L.cap);
  const int64_t k = std::max<int64_t>(0, std::min<int64_t>(have, capacity));
  int32_t* dst[3] = {entering, leaving_row, flags};
  int32_t* src[3] = {p->d.log_enter + L.offLog, p->d.log_row + L.offLog, p->d.log_flags + L.offLog};
  for (int a = 0; a < 3; ++a)
    if (dst[a] && k > 0)
      HIP_TRY(hipMemcpy(dst[a], src[a], sizeof(int32_t) * k, hipMemcpyDeviceToHost), "reading the pivot log");
  if (count) *count = have;
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_batch_get_sizes(const lp_batch* p, int32_t* m, int32_t* n) try {
  if (!p) return fail(LP_ERR_ARG, "bt is NULL");
  for (int32_t i = 0; i < p->count; ++i) {
    if (m) m[i] = p->lps[i].m;
    if (n) n[i] = p->lps[i].n;
  }
  return LP_OK;
} catch (...) {
  return host_exception();
}

int lp_batch_get_stats(const lp_batch* p, lp_batch_stats* s) try {
  if (!p || !s) return fail(LP_ERR_ARG, "NULL argument");
  std::memset(s, 0, sizeof(*s));
  s->count = p->count;
  s->solve_ms = p->solve_ms;
  s->tune_ms = p->tune_ms;
  s->narrow_lps = p->narrow_lps;
  s->wide_lps = p->wide_lps;
  s->work_items = p->items_last;
  s->workgroups = p->grid;
  s->lds_bytes = (int64_t)p->region;
  s->binv_lds_lps = p->binv_lds_lps;
  s->binv_lds_m = p->binv_m;
  s->tuned_from_table = p->loaded_buckets;
  int64_t mask = 0;
  for (size_t bk = 0; bk < p->bucket_narrow.size() && bk < 63; ++bk)
    if (p->bucket_narrow[bk] == 1) mask |= (int64_t)1 << bk;
  s->narrow_bucket_mask = mask;
  return LP_OK;
} catch (...) {
  return host_exception();
}

void lp_batch_destroy(lp_batch* p) { release(p); }

int lp_batch_tune_load(lp_batch* p, const char* path) try {
  if (!p || !path) return fail(LP_ERR_ARG, "NULL argument");
  return load_table(p, path);
} catch (...) {
  return host_exception();
}

int lp_batch_tune_save(const lp_batch* p, const char* path) try {
  if (!p || !path) return fail(LP_ERR_ARG, "NULL argument");
  return save_table(p, path);
} catch (...) {
  return host_exception();
}

int lp_solve_batch(int32_t count, const int32_t* m, const int32_t* n, const double* const* A, const double* const* b,
                   const double* const* c, const lp_options* opt, int32_t* status, double* objective,
                   int64_t* iterations) try {
  lp_batch* p = nullptr;
  int rc = lp_batch_create(&p, count, m, n, A, b, c, opt);
  if (rc != LP_OK) return rc;
  rc = lp_batch_solve(p);
  if (rc == LP_OK) rc = lp_batch_results(p, status, objective, iterations);
  lp_batch_destroy(p);
  return rc;
} catch (...) {
  return host_exception();
}

}  // extern "C"
