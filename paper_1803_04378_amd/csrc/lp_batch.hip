// Batched form: many independent small LPs solved by one persistent kernel launch.
//
// Each LP runs the same iteration as the single-LP path (Section 2.1 Steps 3-8 on the
// Figure 1 tableau, Section 3.1 update, tabu rule of Sections 2.2/3.4), with the same
// element-wise arithmetic and the same per-lane dot-product order, so every result is
// bit-identical to lp_solve on that LP alone.  What changes is the execution shape:
//
//   * 256-thread workgroups pop work items from an atomic queue until it is empty (every
//     wave reaches the exit); items are ordered largest first by the host.
//   * An item is either one LP solved by all 4 wavefronts of the workgroup ("wide",
//     block barriers between steps) or up to 4 small LPs, one per wavefront ("narrow",
//     no block barriers at all: each wavefront runs its own LP with wave-level
//     reductions).  The host picks the mode per m-bucket (autotuned by timing).
//   * The LP's vectors (W, rho, a_q, alpha x2, x_B, ratios) and its basis bookkeeping
//     live in LDS for the whole solve; A' and B^-1 stay in HBM / cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lp_batch.h"
#include "lp_device.h"
#include "lp_gen.h"
#include "lp_wave.h"

namespace lpgpu {
using namespace detail;

namespace {

// dot(x0, y) and, when `two`, dot(x1, y): both columns' loads of a round are issued before
// either is consumed.  Each is wave_dot's fma chain per lane and butterfly, so the results
// are those of two wave_dot calls.
template <bool NT, int NB>
__device__ __forceinline__ void wave_dot2(const double2* __restrict__ x0, const double2* __restrict__ x1, bool two,
                                          const double2* y, int n2, int lane, double2 (&v0)[NB], double2 (&v1)[NB],
                                          double& s0, double& s1) {
  double acc0 = 0.0, acc1 = 0.0;
  for (int k0 = lane; k0 < n2; k0 += 64 * NB) {
    if (NT) load_batch_nt(x0, k0, n2, v0);
    else load_batch(x0, k0, n2, v0);
    if (two) {
      if (NT) load_batch_nt(x1, k0, n2, v1);
      else load_batch(x1, k0, n2, v1);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int k = k0 + 64 * u;
      if (k < n2) {
        const double2 w = y[k];
        acc0 = fma(v0[u].x, w.x, acc0);
        acc0 = fma(v0[u].y, w.y, acc0);
        if (two) {
          acc1 = fma(v1[u].x, w.x, acc1);
          acc1 = fma(v1[u].y, w.y, acc1);
        }
      }
    }
  }
  s0 = wave_sum(acc0);
  s1 = wave_sum(acc1);  // (zero when not two: every lane takes part in the butterfly)
}

#ifndef LPGPU_BATCH_SMALL
#define LPGPU_BATCH_SMALL 2
#endif
constexpr int kBatchSmall = LPGPU_BATCH_SMALL;
// Pricing reads an LP's A' at every pivot.  Up to this many rows (ld) it is loaded
// normally and stays in cache between pivots (26% off a batch of LPs with m <= 64, 2% off
// the m ~ U{16..256} batch); larger LPs stream it with non-temporal loads, which measured
// faster for them (the working set of the resident LPs exceeds the caches).
#ifndef LPGPU_BATCH_CACHED_LD
#define LPGPU_BATCH_CACHED_LD 128
#endif
constexpr int kBatchCachedLd = LPGPU_BATCH_CACHED_LD;

// Group synchronisation: G == 1 is one wavefront (lockstep; the fence orders its LDS and
// global accesses), G > 1 is the whole workgroup.
template <int G>
__device__ __forceinline__ void gsync() {
  if constexpr (G == 1) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// Group reductions: every thread of the group returns the same value.
template <int G>
__device__ __forceinline__ void g_lexmin2(double& d1, int& j1, double& d2, int& j2, double* xd, int* xj) {
  // Xor butterflies through the LDS crossbar rather than the DPP reductions of
  // lp_wave.h: here one wavefront reduces alone, latency decides, and the two independent
  // butterflies overlap (measured: 4096-LP batch 33.1 ms against 36.6 ms).
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double a1 = __shfl_xor(d1, off), a2 = __shfl_xor(d2, off);
    const int b1 = __shfl_xor(j1, off), b2 = __shfl_xor(j2, off);
    if (lex_less(a1, b1, d1, j1)) {
      d1 = a1;
      j1 = b1;
    }
    if (lex_less(a2, b2, d2, j2)) {
      d2 = a2;
      j2 = b2;
    }
  }
  if constexpr (G > 1) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
      xd[wave] = d1;
      xj[wave] = j1;
      xd[G + wave] = d2;
      xj[G + wave] = j2;
    }
    __syncthreads();
    d1 = xd[0];
    j1 = xj[0];
    d2 = xd[G];
    j2 = xj[G];
    for (int w = 1; w < G; ++w) {
      if (lex_less(xd[w], xj[w], d1, j1)) {
        d1 = xd[w];
        j1 = xj[w];
      }
      if (lex_less(xd[G + w], xj[G + w], d2, j2)) {
        d2 = xd[G + w];
        j2 = xj[G + w];
      }
    }
    __syncthreads();
  }
}

template <int G>
__device__ __forceinline__ void g_cnt_min(int& cnt, int& low, int* xj) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    cnt += __shfl_xor(cnt, off);
    low = min(low, __shfl_xor(low, off));
  }
  if constexpr (G > 1) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
      xj[wave] = cnt;
      xj[G + wave] = low;
    }
    __syncthreads();
    cnt = 0;
    low = INT_MAX;
    for (int w = 0; w < G; ++w) {
      cnt += xj[w];
      low = min(low, xj[G + w]);
    }
    __syncthreads();
  }
}

}  // namespace

// One LP, solved by a group of G wavefronts; tid is the thread's index within the group.
// BLDS: B^-1 lives in LDS right after the LP's vectors (batch_lds_bytes), so the update
// and FTRAN run on LDS; otherwise in the pooled HBM array.  The arithmetic is the same.
template <int G, bool BLDS>
__device__ void solve_lp(const BatchDev& bd, int id, unsigned char* base, int tid, double* xd, int* xj) {
  constexpr int T = 64 * G;
  const BatchLP L = bd.lps[id];
  const int m = L.m, n = L.n, ld = L.ld, ld2 = ld / 2, N = n + m;
  const int lane = tid & 63, wave = tid >> 6;
  double* W = reinterpret_cast<double*>(base);
  double* rho = W + ld;
  double* av = rho + ld;
  double* al0 = av + ld;
  double* al1 = al0 + m;
  double* xB = al1 + m;
  double* ratio = xB + m;
  int* basis = reinterpret_cast<int*>(ratio + m);
  int* pos = basis + m;
  int* tabu = pos + N;
  int* dl = tabu + N;  // columns of B^-1 that may differ from unit vectors (as in k_update)
  int* inD = dl + m;
  double2* W2 = reinterpret_cast<double2*>(W);
  double2* rho2 = reinterpret_cast<double2*>(rho);
  double2* a2 = reinterpret_cast<double2*>(av);

  const double* A = bd.A + L.offA;
  const double2* A2 = reinterpret_cast<const double2*>(A);
  const double* bb = bd.b + L.offb;
  const double* cc = bd.c + L.offc;
  double* B = BLDS ? reinterpret_cast<double*>(base + batch_lds_bytes(m, n)) : bd.Binv + L.offB;
  double2* B2 = reinterpret_cast<double2*>(B);
  int* gen = bd.iscr + L.offI;
  int* excl = gen + N;
  int32_t* lg_e = bd.log_enter + L.offLog;
  int32_t* lg_r = bd.log_row + L.offLog;
  int32_t* lg_l = bd.log_leave + L.offLog;
  int32_t* lg_f = bd.log_flags + L.offLog;
  int32_t* Lq = bd.Lq + L.offLog;
  int32_t* Ll = bd.Ll + L.offLog;
  int32_t* Lg = bd.Lgen + L.offLog;
  const double sense = bd.sense;

  // Step 1: slack basis.
  for (int k = tid; k < ld; k += T) {
    W[k] = 0.0;
    rho[k] = 0.0;
  }
  for (int i = tid; i < m; i += T) {
    xB[i] = bb[i];
    inD[i] = 0;
    basis[i] = n + i;
    al0[i] = 0.0;
    al1[i] = 0.0;
  }
  for (int v = tid; v < N; v += T) {
    pos[v] = v < n ? -1 : v - n;
    tabu[v] = -1;
    gen[v] = 0;
    excl[v] = -1;
  }
  for (int i = wave; i < m; i += G)
    for (int k = lane; k < ld2; k += 64)
      B2[(size_t)i * ld2 + k] = make_double2(2 * k == i ? 1.0 : 0.0, 2 * k + 1 == i ? 1.0 : 0.0);
  gsync<G>();

  int64_t t = 0;
  int status = kStatusRunning, ray = -1, r = -1, cur = 0, nL = 0, nD = 0;
  double theta = 0.0, z = 0.0;
  const double neg_eps = -bd.eps_d;
  double2 v[kBatchSmall];  // rows here are short: a shallow batch keeps registers for occupancy
  double2 v2[kBatchSmall];
  for (;;) {
    // Steps 3-4: reduced costs with W in LDS, two nonbasic columns per wavefront at a time
    // (twice the loads in flight; the minima do not depend on the order).
    double da = __builtin_inf(), df = __builtin_inf();
    int ja = INT_MAX, jf = INT_MAX;
    const bool cached_a = ld <= kBatchCachedLd;
    auto consider = [&](int j, double s) {
      const double d = sense * cc[j] - s;
      if (d < neg_eps) {
        if (lex_less(d, j, da, ja)) {
          da = d;
          ja = j;
        }
        if (tabu[j] < t && lex_less(d, j, df, jf)) {
          df = d;
          jf = j;
        }
      }
    };
    for (int j0 = wave; j0 < n; j0 += 2 * G) {
      const int j1 = j0 + G;
      const bool u0 = pos[j0] < 0, u1 = j1 < n && pos[j1] < 0;
      if (!u0 && !u1) continue;
      const int ja0 = u0 ? j0 : j1;  // the first priced column
      const bool two = u0 && u1;
      double s0, s1;
      if (cached_a)
        wave_dot2<false>(A2 + (size_t)ja0 * ld2, A2 + (size_t)j1 * ld2, two, W2, ld2, lane, v, v2, s0, s1);
      else
        wave_dot2<kStreamA>(A2 + (size_t)ja0 * ld2, A2 + (size_t)j1 * ld2, two, W2, ld2, lane, v, v2, s0, s1);
      consider(ja0, s0);
      if (two) consider(j1, s1);
    }
    for (int i = tid; i < m; i += T) {
      const int vv = n + i;
      if (pos[vv] >= 0) continue;
      const double d = 0.0 - W[i];
      if (d < neg_eps) {
        if (lex_less(d, vv, da, ja)) {
          da = d;
          ja = vv;
        }
        if (tabu[vv] < t && lex_less(d, vv, df, jf)) {
          df = d;
          jf = vv;
        }
      }
    }
    g_lexmin2<G>(da, ja, df, jf, xd, xj);
    int q = -1, flags = 0;
    double dq = 0.0;
    if (ja == INT_MAX) {
      status = kStatusOptimal;
    } else if (t >= L.cap) {
      status = kStatusIterLimit;
    } else if (jf != INT_MAX) {
      q = jf;
      dq = df;
    } else {
      q = ja;
      dq = da;
      flags = kFlagAspiration;
    }
    if (q >= 0) {
      if (q < n) {
        for (int k = tid; k < ld2; k += T) a2[k] = A2[(size_t)q * ld2 + k];
      } else {
        const int e = q - n;
        for (int k = tid; k < ld2; k += T) a2[k] = make_double2(2 * k == e ? 1.0 : 0.0, 2 * k + 1 == e ? 1.0 : 0.0);
      }
    }
    gsync<G>();

    // Section 3.1 update of the pending pivot fused with Step 5 and the per-row ratios.
    double* al_p = cur ? al1 : al0;
    double* al_n = cur ? al0 : al1;
    // the same switch and arithmetic as the FP64 form of lp_solve (k_update_c): over D in
    // D order on rows long enough, at any |D|
    const bool sparse = compact_columns(ld);
    if ((r >= 0 || q >= 0) && sparse) {
      for (int i = wave; i < m; i += G) {
        double* rowd = B + (size_t)i * ld;
        const bool isr = i == r;
        const double na = (r >= 0 && !isr) ? -al_p[i] : 0.0;
        double acc = 0.0;
        for (int a = lane; a < nD; a += 64) {
          const int j = dl[a];
          double val;
          if (r >= 0) {
            const double rr = rho[j];
            val = isr ? rr : fma(na, rr, rowd[j]);
            if (rr != 0.0) rowd[j] = val;
          } else {
            val = rowd[j];
          }
          if (q >= 0) acc = fma(val, av[j], acc);
        }
        double x = xB[i];
        if (r >= 0) {
          x = isr ? theta : fma(na, theta, x);
          if (fabs(x) < bd.eps_z) x = 0.0;
        }
        if (q >= 0) {
          acc = wave_sum(acc);
          const int bv = basis[i];
          if (bv >= n && !inD[bv - n]) acc += av[bv - n];
        }
        if (lane == 0) {
          xB[i] = x;
          if (q >= 0) {
            al_n[i] = acc;
            ratio[i] = acc > bd.eps_p ? fmax(x, 0.0) / acc : __builtin_inf();
          }
        }
      }
    } else if (r >= 0 || q >= 0) {
      for (int i = wave; i < m; i += G) {
        double2* row = B2 + (size_t)i * ld2;
        double acc = 0.0;
        double x = xB[i];
        if (r < 0) {
          acc = wave_dot<false>(row, a2, ld2, lane, v, false);
        } else {
          if (i == r) {
            acc = q >= 0 ? wave_store_dot<true>(row, rho2, a2, ld2, lane)
                         : wave_store_dot<false>(row, rho2, a2, ld2, lane);
            x = theta;
          } else {
            const double na = -al_p[i];
            acc = q >= 0 ? wave_update_dot<true>(row, rho2, a2, na, ld2, lane, v, false)
                         : wave_update_dot<false>(row, rho2, a2, na, ld2, lane, v, false);
            x = fma(na, theta, x);
          }
          if (fabs(x) < bd.eps_z) x = 0.0;
        }
        if (lane == 0) {
          xB[i] = x;
          if (q >= 0) {
            al_n[i] = acc;
            ratio[i] = acc > bd.eps_p ? fmax(x, 0.0) / acc : __builtin_inf();
          }
        }
      }
    }
    gsync<G>();
    r = -1;
    if (q < 0) break;  // OPTIMAL or ITER_LIMIT; the pending pivot is applied

    // Step 6: minimum ratio, tolerance ties, tabu list of the entering variable.
    // (minimum ratio, lowest candidate row) and whether some alpha is not finite, in one
    // reduction; the same decisions as k_finish.
    double th = __builtin_inf(), fin = 1.0;
    int lowc = INT_MAX, fj = INT_MAX;
    for (int i = tid; i < m; i += T) {
      const double a = al_n[i];
      if (!isfinite(a)) fin = 0.0;
      if (a > bd.eps_p && lex_less(ratio[i], i, th, lowc)) {
        th = ratio[i];
        lowc = i;
      }
    }
    g_lexmin2<G>(th, lowc, fin, fj, xd, xj);
    if (fin == 0.0 || (lowc != INT_MAX && !isfinite(th))) {
      status = kStatusNumerical;
      break;
    }
    if (lowc == INT_MAX) {  // Step 5: Y_k <= 0
      status = kStatusUnbounded;
      ray = q;
      break;
    }
    // A row is tied when it reaches zero (within eps_t) at the step th.
    int cnt = 0, low = INT_MAX;
    for (int i = tid; i < m; i += T)
      if (al_n[i] > bd.eps_p && fma(-al_n[i], th, fmax(xB[i], 0.0)) <= bd.eps_t) {
        ++cnt;
        low = min(low, i);
      }
    g_cnt_min<G>(cnt, low, xj);
    int rn = low;
    if (cnt >= 2) {
      flags |= kFlagTie;
      if (bd.use_llist) {
        const int stamp = (int)t + 1;
        const int g = gen[q];
        for (int k = tid; k < nL; k += T)
          if (Lq[k] == q && Lg[k] == g) excl[Ll[k]] = stamp;
        gsync<G>();
        int fc = 0, fl = INT_MAX;
        for (int i = tid; i < m; i += T)
          if (al_n[i] > bd.eps_p && fma(-al_n[i], th, fmax(xB[i], 0.0)) <= bd.eps_t && excl[basis[i]] != stamp)
            fl = min(fl, i);
        g_cnt_min<G>(fc, fl, xj);
        int gnew = g;
        if (fl == INT_MAX) {
          flags |= kFlagLClear;
          gnew = g + 1;
        } else {
          rn = fl;
        }
        if (tid == 0) {
          if (gnew != g) gen[q] = gnew;
          if (nL < L.cap) {
            Lq[nL] = q;
            Ll[nL] = basis[rn];
            Lg[nL] = gnew;
          }
        }
        if (nL < L.cap) ++nL;
      }
    }
    // Step 8 pivots on row rn with the step th.
    const double thr = th;
    if (thr == 0.0) flags |= kFlagDegenerate;
    const int leave = basis[rn];
    const double ar = al_n[rn];
    const bool to_D = leave >= n && !inD[leave - n];  // its column stops being a unit vector
    gsync<G>();  // every thread has read basis[rn] and inD before they change
    if (tid == 0) {
      if (to_D) {
        inD[leave - n] = 1;
        dl[nD] = leave - n;
      }
      if (bd.tenure > 0) tabu[leave] = (int)(t + bd.tenure);
      basis[rn] = q;
      pos[q] = rn;
      pos[leave] = -1;
      if (t < L.cap) {
        lg_e[t] = q;
        lg_r[t] = rn;
        lg_l[t] = leave;
        lg_f[t] = flags;
      }
    }
    if (to_D) ++nD;
    z = fma(dq, thr, z);
    ++t;
    r = rn;
    theta = thr;
    cur ^= 1;
    // Top row of the tableau: rho = B^-1[r,:] / alpha_r from the not yet updated B^-1.
    for (int k = tid; k < ld2; k += T) {
      const double2 b = B2[(size_t)r * ld2 + k];
      const double2 rr = make_double2(b.x / ar, b.y / ar);
      rho2[k] = rr;
      const double2 w = W2[k];
      W2[k] = make_double2(fma(dq, rr.x, w.x), fma(dq, rr.y, w.y));
    }
    gsync<G>();
  }

  double* xo = bd.xB_out + L.offOut;
  int* bo = bd.basis_out + L.offOut;
  for (int i = tid; i < m; i += T) {
    xo[i] = xB[i];
    bo[i] = basis[i];
  }
  if (tid == 0) {
    bd.status_out[id] = status;
    bd.iters_out[id] = t;
    bd.z_out[id] = z;
    bd.ray_out[id] = ray;
  }
}

// Held to 128 VGPRs: four 256-thread workgroups per CU instead of two.  The solver is
// bound by the latency of each LP's dependent reductions, so twice the LPs in flight pay
// for the registers it then spills (4096-LP batch: 40.6 -> 30.1 ms; with 2 instead of 4
// double2 per lane per load round, fewer spills: 29.3 ms).
template <bool BLDS>
__global__ __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_batch(BatchDev bd) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ double xd[2 * kBatchWaves];
  __shared__ int xj[2 * kBatchWaves];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) s_item = __hip_atomic_fetch_add(bd.queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= bd.n_items) return;
    const int4 it = bd.items[item];
    if (bd.lps[it.x].waves > 1) {
      solve_lp<kBatchWaves, BLDS>(bd, it.x, lds, threadIdx.x, xd, xj);
    } else {
      const int id = wave == 0 ? it.x : wave == 1 ? it.y : wave == 2 ? it.z : it.w;
      if (id >= 0) solve_lp<1, BLDS>(bd, id, lds + (size_t)wave * bd.slot_bytes, lane, nullptr, nullptr);
    }
    __syncthreads();
  }
}

hipError_t launch_batch(const BatchDev& bd, int grid, size_t lds, bool binv_lds, hipStream_t s) {
  if (binv_lds) hipLaunchKernelGGL(k_batch<true>, dim3(grid), dim3(kBatchBlock), lds, s, bd);
  else hipLaunchKernelGGL(k_batch<false>, dim3(grid), dim3(kBatchBlock), lds, s, bd);
  return hipGetLastError();
}

// One workgroup per LP: its A' column by column (padding rows zero), then b and c.
__global__ __launch_bounds__(256) void k_gen_batch(const BatchLP* __restrict__ lps, uint64_t seed,
                                                    double* __restrict__ A, double* __restrict__ b,
                                                    double* __restrict__ c) {
  const BatchLP L = lps[blockIdx.x];
  const uint64_t iseed = gen::hash(gen::stream_key(seed, gen::kStreamInst), blockIdx.x);
  const uint64_t ka = gen::stream_key(iseed, gen::kStreamA), kb = gen::stream_key(iseed, gen::kStreamB),
                 kc = gen::stream_key(iseed, gen::kStreamC);
  const int m = L.m, n = L.n, ld = L.ld;
  double* a = A + L.offA;
  const size_t total = (size_t)ld * (n > 0 ? n : 1);
  for (size_t k = threadIdx.x; k < total; k += 256) {
    const int j = (int)(k / ld), r = (int)(k - (size_t)j * ld);
    a[k] = (r < m && j < n) ? gen::uniform(ka, (uint64_t)j * m + r, 0.0, 1.0) : 0.0;
  }
  for (int r = threadIdx.x; r < m; r += 256) b[L.offb + r] = gen::uniform(kb, r, 1.0, 10.0);
  for (int j = threadIdx.x; j < n; j += 256) c[L.offc + j] = gen::uniform(kc, j, 1.0, 10.0);
}

hipError_t launch_gen_batch(const BatchLP* lps, int32_t count, uint64_t seed, double* A, double* b, double* c,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_gen_batch, dim3(count), dim3(256), 0, s, lps, seed, A, b, c);
  return hipGetLastError();
}

hipError_t batch_occupancy(int* per_cu, size_t lds, bool binv_lds) {
  const void* f = binv_lds ? reinterpret_cast<const void*>(&k_batch<true>) : reinterpret_cast<const void*>(&k_batch<false>);
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return binv_lds ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch<true>, kBatchBlock, lds)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch<false>, kBatchBlock, lds);
}

}  // namespace lpgpu
