#include "emu_hip.h"
#include <sys/mman.h>
#include <signal.h>
#include <execinfo.h>
#include <unistd.h>
#include <stdio.h>
#include <stdlib.h>
#include <map>
#include <mutex>
#include <string>
#include <vector>
#include <chrono>
#include <unordered_map>

extern "C" void emu_swap(void** save, void* to);
asm(R"(
.text
.globl emu_swap
.type emu_swap,@function
emu_swap:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
.size emu_swap,.-emu_swap
)");

void (*emu_call_struct)(const void* fn, void* arg) = nullptr;
size_t emu_struct_size = 0;

emu::Idx threadIdx, blockIdx, blockDim, gridDim;
namespace emu {
Fiber* g_cur = nullptr;

// ---- guarded allocations ----
static std::mutex g_mu;
struct Alloc { void* base; size_t len; size_t n; };
static std::map<void*, Alloc> g_allocs;
static const size_t kPage = 4096;
static bool front_mode() { static int m = getenv("EMU_GUARD_FRONT") ? 1 : 0; return m; }
// The byte new device, pinned and LDS memory is filled with (EMU_FILL, default 0xFF: an
// uninitialised int reads as -1): runs with other fills expose reads of memory never written.
static int fill_byte() {
  static int f = getenv("EMU_FILL") ? (int)strtol(getenv("EMU_FILL"), nullptr, 0) & 0xFF : 0xFF;
  return f;
}
void* galloc(size_t n, int fill) {
  const size_t data = (std::max<size_t>(n, 1) + kPage - 1) / kPage * kPage;
  const size_t len = data + 2 * kPage;
  char* base = (char*)mmap(nullptr, len, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
  if (base == MAP_FAILED) return nullptr;
  mprotect(base, kPage, PROT_NONE);
  mprotect(base + kPage + data, kPage, PROT_NONE);
  char* p = front_mode() ? base + kPage : base + kPage + data - ((n + 15) / 16 * 16);
  if (fill >= 0) memset(p, fill, n);
  std::lock_guard<std::mutex> l(g_mu);
  g_allocs[p] = {base, len, n};
  return p;
}
int gfree(void* p) {
  if (!p) return 0;
  std::lock_guard<std::mutex> l(g_mu);
  auto it = g_allocs.find(p);
  if (it == g_allocs.end()) { fprintf(stderr, "emu: free of unknown pointer %p\n", p); abort(); }
  munmap(it->second.base, it->second.len);
  g_allocs.erase(it);
  return 0;
}

// ---- fibers ----
static const size_t kStack = 512 * 1024;
static std::vector<char*> g_stacks;
static std::vector<Fiber> g_f;
static void* g_main_sp;
static const std::function<void()>* g_body;
static void* g_dyn = nullptr;
static size_t g_dyn_n = 0;
static const char* g_kname = "";

static void fiber_entry() {
  (*g_body)();
  g_cur->state = 3;
  emu_swap(&g_cur->sp, g_main_sp);
  abort();
}
static void yield() { emu_swap(&g_cur->sp, g_main_sp); }
void sync_block() { g_cur->state = 1; yield(); }
void wave_op(Fiber* f) { f->state = 2; yield(); }
void* dyn_lds() { return g_dyn; }

static void dpp_wave(Fiber* L, int n) {
  // L: 64 lanes (n live in order; dead lanes have state 3)
  unsigned long long src[64], old[64];
  for (int l = 0; l < 64; ++l) { src[l] = L[l].a; old[l] = L[l].b; }
  for (int l = 0; l < 64; ++l) {
    if (L[l].state != 2) continue;
    const int ctrl = L[l].ctrl, rm = L[l].rm, bm = L[l].bm, bc = L[l].bc;
    const int row = l >> 4, bank = (l >> 2) & 3, k = l & 15;
    if (!((rm >> row) & 1) || !((bm >> bank) & 1)) { L[l].res = old[l]; continue; }
    int s = -1;
    if (ctrl <= 0xFF) s = (l & ~3) | ((ctrl >> (2 * (l & 3))) & 3);
    else if (ctrl >= 0x101 && ctrl <= 0x10F) { int d = ctrl - 0x100; s = k + d < 16 ? l + d : -1; }
    else if (ctrl >= 0x111 && ctrl <= 0x11F) { int d = ctrl - 0x110; s = k - d >= 0 ? l - d : -1; }
    else if (ctrl >= 0x121 && ctrl <= 0x12F) { int d = ctrl - 0x120; s = (row << 4) | ((k - d) & 15); }
    else if (ctrl == 0x140) s = (row << 4) | (15 - k);
    else if (ctrl == 0x141) s = (l & ~7) | (7 - (l & 7));
    else if (ctrl == 0x142) s = row >= 1 ? (row << 4) - 1 : -1;
    else if (ctrl == 0x143) s = row >= 2 ? 31 : -1;
    else { fprintf(stderr, "emu: dpp ctrl %#x not emulated\n", ctrl); abort(); }
    if (s >= 0 && L[s].state != 2) s = -1;
    L[l].res = s >= 0 ? src[s] : (bc ? 0ull : old[l]);
  }
}

static void resolve_wave(Fiber* L) {
  int kind = 0;
  for (int l = 0; l < 64; ++l)
    if (L[l].state == 2) {
      if (kind && L[l].kind != kind) { fprintf(stderr, "emu: %s: lanes of one wave in different wave ops\n", g_kname); abort(); }
      kind = L[l].kind;
    }
  unsigned long long a[64];
  for (int l = 0; l < 64; ++l) a[l] = L[l].state == 2 ? L[l].a : 0ull;
  switch (kind) {
    case K_SHFL: for (int l = 0; l < 64; ++l) if (L[l].state == 2) L[l].res = a[L[l].b & 63]; break;
    case K_XOR: for (int l = 0; l < 64; ++l) if (L[l].state == 2) L[l].res = a[(l ^ (int)L[l].b) & 63]; break;
    case K_UP: for (int l = 0; l < 64; ++l) if (L[l].state == 2) { int d = (int)L[l].b; L[l].res = l >= d ? a[l - d] : a[l]; } break;
    case K_BALLOT: { unsigned long long m = 0; for (int l = 0; l < 64; ++l) if (L[l].state == 2 && a[l]) m |= 1ull << l;
      for (int l = 0; l < 64; ++l) if (L[l].state == 2) L[l].res = m; } break;
    case K_READLANE: for (int l = 0; l < 64; ++l) if (L[l].state == 2) {
        int s = (int)L[l].b & 63;
        if (L[s].state != 2) { fprintf(stderr, "emu: %s: readlane of an inactive lane %d\n", g_kname, s); abort(); }
        L[l].res = (unsigned)a[s]; } break;
    case K_DPP: dpp_wave(L, 64); break;
    case K_WBAR: break;
    case K_LEXMIN: case K_LEXMIN_P: {
      int best = -1; double bd = 0; int bj = 0;
      for (int l = 0; l < 64; ++l) {
        if (L[l].state != 2) { fprintf(stderr, "emu: %s: wave reduction with an inactive lane\n", g_kname); abort(); }
        double d; memcpy(&d, &a[l], 8); const int j = (int)(unsigned)(L[l].b & 0xffffffffu);
        if (best < 0 || (d < bd) || (d == bd && j < bj)) { best = l; bd = d; bj = j; }
      }
      const int pay = (int)(L[best].b >> 32);
      for (int l = 0; l < 64; ++l) { L[l].res4[0] = bd; L[l].res4[1] = bj; L[l].res4[2] = pay; }
    } break;
    case K_TWO: {
      double t1 = __builtin_inf(), t2 = __builtin_inf();
      for (int l = 0; l < 64; ++l) {
        if (L[l].state != 2) { fprintf(stderr, "emu: wave reduction with an inactive lane\n"); abort(); }
        double x[2]; memcpy(&x[0], &a[l], 8); memcpy(&x[1], &L[l].b, 8);
        for (double v : x) { if (v < t1) { t2 = t1; t1 = v; } else if (v < t2) t2 = v; }
      }
      for (int l = 0; l < 64; ++l) { L[l].res4[0] = t1; L[l].res4[1] = t2; }
    } break;
    case K_MIN_I: case K_SUM_I: {
      long long acc = kind == K_MIN_I ? INT_MAX : 0;
      for (int l = 0; l < 64; ++l) {
        if (L[l].state != 2) { fprintf(stderr, "emu: wave reduction with an inactive lane\n"); abort(); }
        const int v = (int)(unsigned)a[l];
        acc = kind == K_MIN_I ? std::min<long long>(acc, v) : acc + v;
      }
      for (int l = 0; l < 64; ++l) L[l].res = (unsigned)(int)acc;
    } break;
    case K_MIN_D: {
      double m = __builtin_inf();
      for (int l = 0; l < 64; ++l) { double v; memcpy(&v, &a[l], 8); m = fmin(m, v); }
      for (int l = 0; l < 64; ++l) memcpy(&L[l].res, &m, 8);
    } break;
    case K_SUM_D: {
      double v[64], w[64];
      for (int l = 0; l < 64; ++l) memcpy(&v[l], &a[l], 8);
      for (int off = 32; off > 0; off >>= 1) { for (int l = 0; l < 64; ++l) w[l] = v[l] + v[l ^ off]; memcpy(v, w, sizeof v); }
      for (int l = 0; l < 64; ++l) memcpy(&L[l].res, &v[l], 8);
    } break;
    case K_MFMA: {
      double A[16][4], B[4][16];
      for (int l = 0; l < 64; ++l) {
        double av, bv; memcpy(&av, &a[l], 8); memcpy(&bv, &L[l].b, 8);
        if (L[l].state != 2) { fprintf(stderr, "emu: mfma with an inactive lane\n"); abort(); }
        A[l & 15][l >> 4] = av; B[l >> 4][l & 15] = bv;
      }
      for (int l = 0; l < 64; ++l)
        for (int r = 0; r < 4; ++r) {
          const int row = 4 * (l >> 4) + r, col = l & 15;
          double s = L[l].acc4[r];
          for (int k = 0; k < 4; ++k) s += A[row][k] * B[k][col];
          L[l].res4[r] = s;
        }
    } break;
    default: fprintf(stderr, "emu: unknown wave op\n"); abort();
  }
  for (int l = 0; l < 64; ++l) if (L[l].state == 2) L[l].state = 0;
}

static void run_block(int nt) {
  const int nwaves = (nt + 63) / 64;
  for (int t = 0; t < nwaves * 64; ++t) {
    Fiber& f = g_f[t];
    f.flat = t; f.lane = t & 63; f.wave = t >> 6;
    f.tid = {(unsigned)(t % blockDim.x), (unsigned)((t / blockDim.x) % blockDim.y), (unsigned)(t / (blockDim.x * blockDim.y))};
    if (t >= nt) { f.state = 3; continue; }
    f.state = 0;
    char* top = g_stacks[t] + kStack;
    void** sp = (void**)top;
    *--sp = nullptr;                 // fake return address of fiber_entry
    *--sp = (void*)&fiber_entry;     // popped by ret
    for (int k = 0; k < 6; ++k) *--sp = nullptr;
    f.sp = sp;
  }
  for (;;) {
    for (int w = 0; w < nwaves; ++w) {
      Fiber* L = &g_f[w * 64];
      for (;;) {
        for (int l = 0; l < 64; ++l)
          if (L[l].state == 0) { g_cur = &L[l]; threadIdx = L[l].tid; emu_swap(&g_main_sp, L[l].sp); }
        int live = 0, at = 0, bar = 0;
        for (int l = 0; l < 64; ++l) if (L[l].state != 3) { ++live; at += L[l].state == 2; bar += L[l].state == 1; }
        // every live lane at the wave op, or (divergent code) the others already at the block barrier
        if (at && at + bar == live) { resolve_wave(L); continue; }
        break;
      }
    }
    int live = 0, bar = 0;
    for (int t = 0; t < nt; ++t) if (g_f[t].state != 3) { ++live; bar += g_f[t].state == 1; }
    if (!live) break;
    if (bar == live) { for (int t = 0; t < nt; ++t) if (g_f[t].state == 1) g_f[t].state = 0; continue; }
    fprintf(stderr, "emu: %s: deadlock (block %u,%u: %d live, %d at the block barrier)\n", g_kname, blockIdx.x, blockIdx.y, live, bar);
    abort();
  }
}

static std::unordered_map<std::string, std::pair<double, long>> g_prof;
struct ProfDump { ~ProfDump() { if (!getenv("EMU_PROF")) return; for (auto& kv : g_prof) fprintf(stderr, "emu prof %-40s %8ld launches %10.3f s\n", kv.first.c_str(), kv.second.second, kv.second.first); } } g_profdump;
void launch_(const std::function<void()>& body, dim3 grid, dim3 block, size_t shmem, const char* name);
static void on_segv(int sig, siginfo_t* si, void*) {
  char* a = (char*)si->si_addr;
  fprintf(stderr, "emu: SIGSEGV at %p in %s block (%u,%u,%u) thread %d\n", (void*)a, g_kname, blockIdx.x, blockIdx.y, blockIdx.z,
          g_cur ? g_cur->flat : -1);
  for (auto& kv : g_allocs) {
    char* base = (char*)kv.second.base;
    if (a >= base && a < base + kv.second.len) {
      char* p = (char*)kv.first;
      fprintf(stderr, "emu:   inside the guarded region of allocation %p (%zu bytes): offset %td bytes from its start\n",
              (void*)p, kv.second.n, a - p);
    }
  }
  if (g_dyn) fprintf(stderr, "emu:   dynamic LDS %p (%zu bytes)\n", g_dyn, g_dyn_n);
  void* bt[64]; int n = backtrace(bt, 64); backtrace_symbols_fd(bt, n, 2);
  _exit(139);
}
struct SegvInit { SegvInit() {
  static char altstack[1 << 16]; stack_t ss{}; ss.ss_sp = altstack; ss.ss_size = sizeof altstack; sigaltstack(&ss, nullptr);
  struct sigaction sa{}; sa.sa_sigaction = on_segv; sa.sa_flags = SA_SIGINFO | SA_ONSTACK; sigaction(SIGSEGV, &sa, nullptr); } } g_segv_init;
void launch(const std::function<void()>& body, dim3 grid, dim3 block, size_t shmem, const char* name) {
  const auto t0 = std::chrono::steady_clock::now();
  launch_(body, grid, block, shmem, name);
  auto& e = g_prof[name];
  e.first += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  e.second += 1;
}
void launch_(const std::function<void()>& body, dim3 grid, dim3 block, size_t shmem, const char* name) {
  const int nt = block.x * block.y * block.z;
  if (nt <= 0 || nt > 1024) { fprintf(stderr, "emu: %s: block of %d threads\n", name, nt); abort(); }
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) { fprintf(stderr, "emu: %s: empty grid\n", name); abort(); }
  if (shmem > 163840) { fprintf(stderr, "emu: %s: %zu bytes of dynamic LDS\n", name, shmem); abort(); }
  const int nslots = (nt + 63) / 64 * 64;
  while ((int)g_stacks.size() < nslots) {
    char* s = (char*)mmap(nullptr, kStack + kPage, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    mprotect(s, kPage, PROT_NONE);
    g_stacks.push_back(s + kPage);
  }
  if ((int)g_f.size() < nslots) g_f.resize(nslots);
  void* dyn = shmem ? galloc(shmem, fill_byte()) : nullptr;
  g_dyn = dyn; g_dyn_n = shmem; g_body = &body; g_kname = name;
  gridDim = {grid.x, grid.y, grid.z};
  blockDim = {block.x, block.y, block.z};
  for (unsigned z = 0; z < grid.z; ++z)
    for (unsigned y = 0; y < grid.y; ++y)
      for (unsigned x = 0; x < grid.x; ++x) {
        blockIdx = {x, y, z};
        if (dyn) memset(dyn, fill_byte(), shmem);
        run_block(nt);
      }
  g_cur = nullptr;
  if (dyn) gfree(dyn);
  g_dyn = nullptr;
}
}  // namespace emu

using namespace emu;

hipError_t hipMalloc(void** p, size_t n) { *p = galloc(n, fill_byte()); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipFree(void* p) { return gfree(p); }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = galloc(n, fill_byte()); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipHostFree(void* p) { return gfree(p); }
hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned) { *d = h; return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { if (n) memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { if (n) memmove(d, s, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { memset(d, v, n); return hipSuccess; }
hipError_t hipMemGetInfo(size_t* f, size_t* t) { *f = (size_t)200 << 30; *t = (size_t)288 << 30; return hipSuccess; }
struct emu_stream { int x; };
struct emu_event { int x; };
hipError_t hipStreamCreate(hipStream_t* s) { *s = new emu_stream{}; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new emu_event{}; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new emu_event{}; return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.001f; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  memset(p, 0, sizeof(*p)); strcpy(p->name, "emu"); strcpy(p->gcnArchName, "gfx950:emu");
  p->multiProcessorCount = getenv("EMU_CUS") ? atoi(getenv("EMU_CUS")) : 256;
  p->sharedMemPerBlock = 163840; p->totalGlobalMem = (size_t)288 << 30; return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { hipDeviceProp_t p; hipGetDeviceProperties(&p, 0); *v = p.multiProcessorCount; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emu error"; }
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t emu_occupancy(int* out, const char* name, int block, size_t dyn) {
  struct K { const char* n; int lds, vgpr; };
  static const K t[] = {{"k_update_wide<kUpdateBlock>", 2256, 122}, {"k_update<2 * kUpdateBlock>", 4496, 107},
                        {"k_update<kUpdateBlock>", 2256, 105}, {"k_price32", 2496, 62}, {"k_price<false>", 192, 76},
                        {"k_price<true>", 192, 76}, {"k_price_fin<false>", 448, 79}, {"k_price_fin<true>", 448, 79}, {"k_update_c<kUpdateBlock>", 2248, 119},
                        {"k_batch<true>", 112, 128}, {"k_batch<false>", 112, 128}};
  const K* k = nullptr;
  for (const K& e : t) if (std::string(name) == e.n) { k = &e; break; }
  if (!k) { fprintf(stderr, "emu: occupancy of unknown kernel %s\n", name); abort(); }
  const size_t lds = k->lds + dyn;
  const int by_lds = lds > 163840 ? 0 : (int)(163840 / std::max<size_t>(lds, 1));
  const int vg = (k->vgpr + 7) / 8 * 8;
  const int wps = std::min(8, 512 / vg);
  const int waves = (block + 63) / 64, per_simd = (waves + 3) / 4;
  const int by_vgpr = wps / per_simd;
  *out = std::min(by_lds, by_vgpr);
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }

struct emu_node { int kind; const void* fn; dim3 g, b; size_t sh; std::vector<char> arg; };
struct emu_graph { std::vector<emu_node> nodes; };
hipError_t hipGraphCreate(hipGraph_t* g, unsigned) { *g = new emu_graph{}; return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t g) { delete g; return hipSuccess; }
hipError_t hipGraphAddKernelNode(hipGraphNode_t* n, hipGraph_t g, const hipGraphNode_t*, size_t, const hipKernelNodeParams* p) {
  emu_node k{1, p->func, p->gridDim, p->blockDim, p->sharedMemBytes, {}};
  k.arg.resize(emu_struct_size);
  memcpy(k.arg.data(), p->kernelParams[0], emu_struct_size);
  g->nodes.push_back(k);
  *n = nullptr;
  return hipSuccess;
}
hipError_t hipGraphAddEventRecordNode(hipGraphNode_t* n, hipGraph_t, const hipGraphNode_t*, size_t, hipEvent_t) { *n = nullptr; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t) { *e = new emu_graph(*g); return hipSuccess; }
const char* (*emu_kernel_name)(const void* fn) = nullptr;
static void run_struct(const void* fn, dim3 g, dim3 b, size_t sh, void* arg) {
  std::vector<char> copy((char*)arg, (char*)arg + emu_struct_size);
  emu::launch([&]() { emu_call_struct(fn, copy.data()); }, g, b, sh, emu_kernel_name ? emu_kernel_name(fn) : "struct-arg kernel");
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto& n : e->nodes) run_struct(n.fn, n.g, n.b, n.sh, n.arg.data());
  return hipSuccess;
}
hipError_t hipExtLaunchKernel(const void* f, dim3 g, dim3 b, void** args, size_t sh, hipStream_t, hipEvent_t, hipEvent_t, int) {
  run_struct(f, g, b, sh, args[0]);
  return hipSuccess;
}
