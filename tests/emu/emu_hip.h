// CPU emulation of the HIP subset used by liblpgpu: kernels run as fibers (one per GPU
// thread), blocks one after another; wave operations and barriers are resolved by a
// scheduler; device and pinned allocations sit against guard pages.
#pragma once
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <math.h>
#include <limits.h>
#include <algorithm>
#include <functional>
#include <cmath>

// ---- qualifiers ----
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))
#define __restrict__ __restrict

// ---- vector types ----
struct dim3 { unsigned x, y, z; constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {} };
struct double2 { double x, y; };
struct float4 { float x, y, z, w; };
struct int4 { int x, y, z, w; };
struct int2 { int x, y; };
inline double2 make_double2(double a, double b) { return {a, b}; }
inline float4 make_float4(float a, float b, float c, float d) { return {a, b, c, d}; }
inline int4 make_int4(int a, int b, int c, int d) { return {a, b, c, d}; }
inline int2 make_int2(int a, int b) { return {a, b}; }

inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }
inline long min(long a, long b) { return a < b ? a : b; }
inline long max(long a, long b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned long min(unsigned long a, unsigned long b) { return a < b ? a : b; }
inline unsigned long max(unsigned long a, unsigned long b) { return a > b ? a : b; }
inline unsigned long long min(unsigned long long a, unsigned long long b) { return a < b ? a : b; }

inline long long __double_as_longlong(double d) { long long v; memcpy(&v, &d, 8); return v; }
inline double __longlong_as_double(long long v) { double d; memcpy(&d, &v, 8); return d; }
inline unsigned __float_as_uint(float f) { unsigned v; memcpy(&v, &f, 4); return v; }
inline double __dadd_rn(double a, double b) { return a + b; }
inline double __dmul_rn(double a, double b) { return a * b; }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline unsigned long long wall_clock64() { return 0; }
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __hip_atomic_fetch_add(p, v, o, s) emu_fetch_add((p), (v))
template <class T, class U> inline T emu_fetch_add(T* p, U v) { T o = *p; *p = o + (T)v; return o; }
template <class T, class U> inline T atomicAdd(T* p, U v) { T o = *p; *p = o + (T)v; return o; }
template <class T, class U> inline T atomicOr(T* p, U v) { T o = *p; *p = o | (T)v; return o; }
template <class T, class U> inline T atomicMax(T* p, U v) { T o = *p; *p = o > (T)v ? o : (T)v; return o; }
template <class T, class U> inline T atomicMin(T* p, U v) { T o = *p; *p = o < (T)v ? o : (T)v; return o; }
#define __builtin_amdgcn_fence(...) ((void)0)

// ---- the fiber machine ----
namespace emu {
struct Fiber;
struct Block;
extern Fiber* g_cur;
struct Idx { unsigned x, y, z; };
struct Fiber {
  void* sp;
  int state;  // 0 run, 1 barrier, 2 wave op, 3 done
  Idx tid;
  int flat, lane, wave;
  // wave op message
  int kind;
  unsigned long long a, b;
  int ctrl, rm, bm, bc;
  double acc4[4], res4[4];
  unsigned long long res;
  const char* site;
};
void sync_block();
void wave_op(Fiber* f);
void* dyn_lds();
void launch(const std::function<void()>& body, dim3 grid, dim3 block, size_t shmem, const char* name);
enum { K_SHFL = 1, K_XOR, K_UP, K_BALLOT, K_READLANE, K_DPP, K_MFMA, K_WBAR, K_LEXMIN, K_LEXMIN_P, K_TWO, K_MIN_I, K_SUM_I, K_MIN_D, K_SUM_D };
}  // namespace emu
extern emu::Idx threadIdx, blockIdx, blockDim, gridDim;
inline void __syncthreads() { emu::sync_block(); }

inline unsigned long long emu_wave(int kind, unsigned long long a, unsigned long long b = 0, int ctrl = 0, int rm = 0,
                                   int bm = 0, int bc = 0) {
  emu::Fiber* f = emu::g_cur;
  f->kind = kind; f->a = a; f->b = b; f->ctrl = ctrl; f->rm = rm; f->bm = bm; f->bc = bc;
  emu::wave_op(f);
  return f->res;
}
template <class T> inline unsigned long long emu_bits(T v) { unsigned long long u = 0; memcpy(&u, &v, sizeof(T)); return u; }
template <class T> inline T emu_from(unsigned long long u) { T v; memcpy(&v, &u, sizeof(T)); return v; }
template <class T> inline T __shfl(T v, int src, int width = 64) { return emu_from<T>(emu_wave(emu::K_SHFL, emu_bits(v), (unsigned)src)); }
template <class T> inline T __shfl_xor(T v, int m, int width = 64) { return emu_from<T>(emu_wave(emu::K_XOR, emu_bits(v), (unsigned)m)); }
template <class T> inline T __shfl_up(T v, unsigned d, int width = 64) { return emu_from<T>(emu_wave(emu::K_UP, emu_bits(v), d)); }
inline unsigned long long __ballot(int p) { return emu_wave(emu::K_BALLOT, p ? 1 : 0); }
inline int __builtin_amdgcn_readlane(int v, int l) { return (int)emu_wave(emu::K_READLANE, (unsigned)v, (unsigned)l); }
inline int __builtin_amdgcn_update_dpp(int old, int v, int ctrl, int rm, int bm, bool bc) {
  return (int)emu_wave(emu::K_DPP, (unsigned)v, (unsigned)old, ctrl, rm, bm, bc ? 1 : 0);
}
inline void __builtin_amdgcn_wave_barrier() { emu_wave(emu::K_WBAR, 0); }
typedef double emu_v4d __attribute__((ext_vector_type(4)));
inline emu_v4d __builtin_amdgcn_mfma_f64_16x16x4f64(double a, double b, emu_v4d c, int, int, int) {
  emu::Fiber* f = emu::g_cur;
  for (int i = 0; i < 4; ++i) f->acc4[i] = c[i];
  emu_wave(emu::K_MFMA, emu_bits(a), emu_bits(b));
  emu_v4d r; for (int i = 0; i < 4; ++i) r[i] = f->res4[i];
  return r;
}
#define __builtin_amdgcn_mfma_f64_16x16x4f64 __builtin_amdgcn_mfma_f64_16x16x4f64

// ---- runtime API ----
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1, hipErrorInvalidSymbol = 13 };
typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
typedef struct emu_graph* hipGraph_t;
typedef struct emu_graph* hipGraphExec_t;
typedef struct emu_node* hipGraphNode_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum { hipHostMallocDefault = 0, hipEventDisableTiming = 2 };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 };
struct hipDeviceProp_t { char name[256]; char gcnArchName[256]; int multiProcessorCount; size_t sharedMemPerBlock; size_t totalGlobalMem; };
struct hipKernelNodeParams { dim3 blockDim; void** extra; void* func; dim3 gridDim; void** kernelParams; unsigned sharedMemBytes; };
#define HIP_SYMBOL(x) ((const void*)&(x))
hipError_t hipMalloc(void** p, size_t n);
template <class T> hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags);
template <class T> hipError_t hipHostMalloc(T** p, size_t n, unsigned flags) { return hipHostMalloc((void**)p, n, flags); }
hipError_t hipHostFree(void* p);
hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned flags);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st);
hipError_t hipMemGetInfo(size_t* f, size_t* t);
hipError_t hipStreamCreate(hipStream_t* s);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned f);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipGetDevice(int* d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int d);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute a, int v);
template <class F> hipError_t hipFuncSetAttribute(F* f, hipFuncAttribute a, int v) { return hipSuccess; }
hipError_t emu_occupancy(int* out, const char* name, int block, size_t dyn);
#define hipOccupancyMaxActiveBlocksPerMultiprocessor(out, f, bs, dyn) emu_occupancy((out), #f, (int)(bs), (size_t)(dyn))
hipError_t hipGetSymbolAddress(void** p, const void* sym);
hipError_t hipGraphCreate(hipGraph_t* g, unsigned f);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t g);
hipError_t hipGraphAddKernelNode(hipGraphNode_t* n, hipGraph_t g, const hipGraphNode_t* deps, size_t nd, const hipKernelNodeParams* p);
hipError_t hipGraphAddEventRecordNode(hipGraphNode_t* n, hipGraph_t g, const hipGraphNode_t* deps, size_t nd, hipEvent_t e);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipExtLaunchKernel(const void* f, dim3 g, dim3 b, void** args, size_t sh, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int flags);
// graph and ext launches: every such kernel takes one by-value struct argument
extern void (*emu_call_struct)(const void* fn, void* arg);
extern size_t emu_struct_size;
#define hipLaunchKernelGGL(k, g, b, sh, st, ...) \
  emu::launch([&]() { (k)(__VA_ARGS__); }, dim3(g), dim3(b), (size_t)(sh), #k)

// Whole-wave reductions of lp_wave.h as single wave operations (same results).
inline void emu_wave_lexmin(double& d, int& j) {
  emu::Fiber* f = emu::g_cur; f->acc4[0] = d; f->acc4[1] = (double)j;
  emu_wave(emu::K_LEXMIN, emu_bits(d), (unsigned)j);
  d = f->res4[0]; j = (int)f->res4[1];
}
inline void emu_wave_lexmin_payload(double& d, int& j, int& p) {
  emu::Fiber* f = emu::g_cur;
  emu_wave(emu::K_LEXMIN_P, emu_bits(d), ((unsigned long long)(unsigned)p << 32) | (unsigned)j);
  d = f->res4[0]; j = (int)f->res4[1]; p = (int)f->res4[2];
}
inline void emu_wave_two_smallest(double& t1, double& t2) {
  emu::Fiber* f = emu::g_cur;
  emu_wave(emu::K_TWO, emu_bits(t1), emu_bits(t2));
  t1 = f->res4[0]; t2 = f->res4[1];
}
inline int emu_wave_min_int(int v) { return (int)emu_wave(emu::K_MIN_I, (unsigned)v); }
inline int emu_wave_sum_int(int v) { return (int)emu_wave(emu::K_SUM_I, (unsigned)v); }
inline double emu_wave_min(double v) { return emu_from<double>(emu_wave(emu::K_MIN_D, emu_bits(v))); }
inline double emu_wave_sum(double v) { return emu_from<double>(emu_wave(emu::K_SUM_D, emu_bits(v))); }
