// CPU emulation of the small part of HIP the kernels use, for tests only.
//
// The kernel sources are compiled with g++ after this header (which
// pre-empts <hip/hip_runtime.h>).  A launch runs the blocks one after
// another; the blockDim.x threads of a block are cooperative fibers on one OS
// thread that switch at __syncthreads().  __shared__ arrays become
// thread-local function statics, shared by the threads of the (single)
// running block.  "Device" memory is host memory.  This exercises indexing,
// barriers and arithmetic of the kernels on the CPU; it says nothing about
// timing.
//
// All emulated grid state (grid and block sizes, the running block, fiber
// stacks, __shared__ arrays) belongs to the launching host thread, so host
// threads launch concurrently with no lock between them: a ThreadSanitizer
// build (fibers announced to it below) sees the library's host code exactly
// as concurrent as the library makes it.
#pragma once
#define HIP_INCLUDE_HIP_HIP_RUNTIME_H 1

#include <algorithm>
#include <cmath>
#include <ucontext.h>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>
#if defined(__SANITIZE_THREAD__)
#include <sanitizer/tsan_interface.h>
#endif

struct double2 { double x, y; };
struct float2 { float x, y; };
struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint3_ { unsigned x = 0, y = 0, z = 0; };

extern thread_local uint3_ threadIdx;
extern thread_local uint3_ blockIdx;
extern thread_local dim3 blockDim, gridDim;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
// scheduling hints of the GPU compiler have no meaning on the CPU
inline void __builtin_amdgcn_sched_barrier(int) {}
#define __shared__ static thread_local
// clang's vector extension, as GCC's (element count -> bytes, for double)
#define ext_vector_type(n) vector_size(8 * (n))
typedef double emu_f64x4 __attribute__((vector_size(32)));
#define __restrict__

typedef int hipError_t;
typedef void* hipStream_t;
enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorInvalidDevice = 101,
  hipErrorInvalidSymbol = 701,
  hipErrorCooperativeLaunchTooLarge = 720
};
#define __align__(n) __attribute__((aligned(n)))
// a __device__ variable is a host variable here: its address is the symbol's
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyHostToHost };

namespace emu {
// Cooperative fibers: every emulated thread of a block runs on one OS thread
// until it reaches __syncthreads(); when all have arrived (or finished) the
// scheduler resumes them.  Kernels call __syncthreads() uniformly.
struct Fiber {
  ucontext_t ctx;
  bool done = false;
  unsigned tid = 0;
  void* tsan = nullptr;   // ThreadSanitizer's fiber handle (sanitizer builds)
};
constexpr size_t kStack = 1 << 17;
inline char* stack_for(unsigned t) {  // one uninitialised stack per fiber slot and host thread, reused
  struct Pool {
    std::vector<char*> s;
    ~Pool() {
      for (char* p : s) delete[] p;
    }
  };
  static thread_local Pool pool;
  while (pool.s.size() <= t) pool.s.push_back(new char[kStack]);
  return pool.s[t];
}
struct Block {
  ucontext_t sched;
  void* tsan_sched = nullptr;
  std::vector<Fiber> fibers;
  std::function<void()> body;
  int current = -1;
};
extern thread_local Block* g_block;
// announce a context switch to ThreadSanitizer (it then keeps one shadow
// stack per fiber and orders the switch like a synchronization)
inline void tsan_switch(void* to) {
#if defined(__SANITIZE_THREAD__)
  __tsan_switch_to_fiber(to, 0);
#else
  (void)to;
#endif
}
inline void fiber_entry() {
  Block* b = g_block;
  Fiber& f = b->fibers[b->current];
  threadIdx.x = f.tid;
  b->body();
  f.done = true;
  tsan_switch(b->tsan_sched);
  swapcontext(&f.ctx, &b->sched);
}
template <typename K, typename... Args>
void launch(K kernel, dim3 grid, dim3 block, Args... args) {
  gridDim = grid;
  blockDim = block;
  for (unsigned bi = 0; bi < grid.x; ++bi) {
    Block b;
    g_block = &b;
    blockIdx.x = bi;
    b.body = [&]() { kernel(args...); };
    b.fibers.resize(block.x);
#if defined(__SANITIZE_THREAD__)
    b.tsan_sched = __tsan_get_current_fiber();
#endif
    for (unsigned t = 0; t < block.x; ++t) {
      Fiber& f = b.fibers[t];
      f.tid = t;
      getcontext(&f.ctx);
      f.ctx.uc_stack.ss_sp = stack_for(t);
      f.ctx.uc_stack.ss_size = kStack;
      f.ctx.uc_link = nullptr;
      makecontext(&f.ctx, (void (*)())fiber_entry, 0);
#if defined(__SANITIZE_THREAD__)
      f.tsan = __tsan_create_fiber(0);
#endif
    }
    bool any = true;
    while (any) {
      any = false;
      for (unsigned t = 0; t < block.x; ++t) {
        if (b.fibers[t].done) continue;
        b.current = (int)t;
        threadIdx.x = t;
        tsan_switch(b.fibers[t].tsan);
        swapcontext(&b.sched, &b.fibers[t].ctx);
        if (!b.fibers[t].done) any = true;
      }
    }
#if defined(__SANITIZE_THREAD__)
    for (Fiber& f : b.fibers) __tsan_destroy_fiber(f.tsan);
#endif
    g_block = nullptr;
  }
}
inline void barrier_wait() {
  Block* b = g_block;
  Fiber& f = b->fibers[b->current];
  tsan_switch(b->tsan_sched);
  swapcontext(&f.ctx, &b->sched);
  threadIdx.x = f.tid;
}

// Cooperative (co-resident) launches: every thread of every block is a fiber
// of one scheduler, each block has its own dynamic LDS and its own barrier
// (a generation count), and a fiber that spins (s_sleep) or waits at a
// barrier yields to the others, so grid-wide waits make progress.
struct CoopFiber {
  ucontext_t ctx;
  bool done = false;
  unsigned tid = 0, bid = 0;
  void* tsan = nullptr;
};
struct CoopBlock {
  unsigned arrived = 0, gen = 0;
  std::vector<double> lds;
};
struct CoopRun {
  ucontext_t sched;
  void* tsan_sched = nullptr;
  std::vector<CoopFiber> fibers;
  std::vector<CoopBlock> blocks;
  std::function<void()> body;
  int current = -1;
};
extern thread_local CoopRun* g_coop;
inline void coop_yield() {
  CoopRun* r = g_coop;
  CoopFiber& f = r->fibers[r->current];
  tsan_switch(r->tsan_sched);
  swapcontext(&f.ctx, &r->sched);
  threadIdx.x = f.tid;
  blockIdx.x = f.bid;
}
inline void coop_barrier() {
  CoopRun* r = g_coop;
  CoopBlock& b = r->blocks[r->fibers[r->current].bid];
  const unsigned my = b.gen;
  if (++b.arrived == blockDim.x) {
    b.arrived = 0;
    ++b.gen;
  } else {
    while (b.gen == my) coop_yield();
  }
}
inline void coop_entry() {
  CoopRun* r = g_coop;
  CoopFiber& f = r->fibers[r->current];
  threadIdx.x = f.tid;
  blockIdx.x = f.bid;
  r->body();
  f.done = true;
  tsan_switch(r->tsan_sched);
  swapcontext(&f.ctx, &r->sched);
}
template <typename F>
void launch_coop(F body, dim3 grid, dim3 block, size_t lds_bytes) {
  gridDim = grid;
  blockDim = block;
  CoopRun r;
  g_coop = &r;
  r.body = body;
  r.blocks.resize(grid.x);
  for (CoopBlock& b : r.blocks) b.lds.assign((std::max<size_t>(lds_bytes, 16) + 7) / 8, 0.0);
  const unsigned n = grid.x * block.x;
  r.fibers.resize(n);
#if defined(__SANITIZE_THREAD__)
  r.tsan_sched = __tsan_get_current_fiber();
#endif
  for (unsigned i = 0; i < n; ++i) {
    CoopFiber& f = r.fibers[i];
    f.bid = i / block.x;
    f.tid = i % block.x;
    getcontext(&f.ctx);
    f.ctx.uc_stack.ss_sp = stack_for(i);
    f.ctx.uc_stack.ss_size = kStack;
    f.ctx.uc_link = nullptr;
    makecontext(&f.ctx, (void (*)())coop_entry, 0);
#if defined(__SANITIZE_THREAD__)
    f.tsan = __tsan_create_fiber(0);
#endif
  }
  bool any = true;
  while (any) {
    any = false;
    for (unsigned i = 0; i < n; ++i) {
      if (r.fibers[i].done) continue;
      r.current = (int)i;
      threadIdx.x = r.fibers[i].tid;
      blockIdx.x = r.fibers[i].bid;
      tsan_switch(r.fibers[i].tsan);
      swapcontext(&r.sched, &r.fibers[i].ctx);
      if (!r.fibers[i].done) any = true;
    }
  }
#if defined(__SANITIZE_THREAD__)
  for (CoopFiber& f : r.fibers) __tsan_destroy_fiber(f.tsan);
#endif
  g_coop = nullptr;
}
// dynamic LDS: the running block's own buffer in a cooperative launch, else
// one buffer per host thread (blocks of ordinary launches run one at a time)
inline void* dyn_lds() {
  if (g_coop) return g_coop->blocks[g_coop->fibers[g_coop->current].bid].lds.data();
  static thread_local std::vector<double> buf(160 * 1024 / sizeof(double));
  return buf.data();
}
}  // namespace emu

inline void __syncthreads() {
  if (emu::g_coop) emu::coop_barrier();
  else emu::barrier_wait();
}
// scheduling and memory-model builtins of the device code
inline void __builtin_amdgcn_s_sleep(int) {
  if (emu::g_coop) emu::coop_yield();
}
inline void __builtin_amdgcn_s_waitcnt(int) {}
inline void __builtin_amdgcn_fence(int, const char*) {}
// buffer resources: the base pointer and the byte size; 16-byte loads and
// stores (cache policy bits have no meaning here)
struct __amdgpu_buffer_rsrc_t {
  char* base;
  int bytes;
};
struct emu_u32x4 {
  unsigned v[4];
};
inline __amdgpu_buffer_rsrc_t __builtin_amdgcn_make_buffer_rsrc(void* p, short, int bytes, int) {
  return __amdgpu_buffer_rsrc_t{(char*)p, bytes};
}
inline emu_u32x4 __builtin_amdgcn_raw_buffer_load_b128(__amdgpu_buffer_rsrc_t r, int off, int soff, int) {
  emu_u32x4 x{};
  if (off + soff >= 0 && off + soff + 16 <= r.bytes) std::memcpy(&x, r.base + off + soff, 16);
  else std::abort();   // an access outside the buffer is a bug in the kernel
  return x;
}
inline void __builtin_amdgcn_raw_buffer_store_b128(emu_u32x4 x, __amdgpu_buffer_rsrc_t r, int off, int soff, int) {
  if (off + soff >= 0 && off + soff + 16 <= r.bytes) std::memcpy(r.base + off + soff, &x, 16);
  else std::abort();
}
inline double atomicAdd(double* p, double v) {
  const double old = *p;
  *p = old + v;
  return old;
}
inline unsigned atomicOr(unsigned* p, unsigned v) {
  const unsigned old = *p;
  *p = old | v;
  return old;
}
using std::isfinite;
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
template <typename T>
inline T __hip_atomic_load(const T* p, int, int) { return *p; }
template <typename T>
inline void __hip_atomic_store(T* p, T v, int, int) { *p = v; }
template <typename T>
inline T __hip_atomic_fetch_add(T* p, T v, int, int) {
  const T old = *p;
  *p = old + v;
  return old;
}
// FP64 16x16x4 matrix product of one wave (gfx950 lane layout: A[i][k] in
// lane i + 16k, B[k][j] in lane j + 16k, D[q + 4r][j] in lane j + 16q,
// element r).
// Emulated with a block-wide rendezvous, so every thread of the block must
// reach each call in the same order (as the kernels that use it do).
inline emu_f64x4 __builtin_amdgcn_mfma_f64_16x16x4f64(double a, double b, emu_f64x4 c, int, int, int) {
  static thread_local double sa[1024], sb[1024];
  const unsigned t = threadIdx.x;
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
  const unsigned w0 = t & ~63u, l = t & 63u, j = l % 16, q = l / 16;
  emu_f64x4 d = c;
  for (unsigned r = 0; r < 4; ++r) {
    double s = 0.0;
    for (unsigned k = 0; k < 4; ++k) s += sa[w0 + q + 4 * r + 16 * k] * sb[w0 + j + 16 * k];
    d[r] += s;
  }
  __syncthreads();
  return d;
}
inline void sincos(double x, double* s, double* c) { *s = std::sin(x); *c = std::cos(x); }
inline void sincosf(float x, float* s, float* c) { *s = std::sin(x); *c = std::cos(x); }
using std::min;
using std::max;

#define hipLaunchKernelGGL(K, G, B, SH, S, ...) emu::launch(K, G, B, __VA_ARGS__)
#define hipExtLaunchKernelGGL(K, G, B, SH, S, E0, E1, FL, ...) emu::launch(K, G, B, __VA_ARGS__)
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "emulated"; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  std::memset(d, v, n);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
typedef struct emu_event* hipEvent_t;
typedef struct emu_graph* hipGraph_t;
typedef struct emu_graph_exec* hipGraphExec_t;
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorInvalidValue; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = nullptr; return hipErrorInvalidValue; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, void*, size_t) { return hipErrorInvalidValue; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorInvalidValue; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)new char[1]; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete[] (char*)e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
enum hipDeviceAttribute_t { hipDeviceAttributeMaxSharedMemoryPerBlock, hipDeviceAttributeMultiprocessorCount };
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
template <typename K>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, K, int, size_t) {
  *n = 1;
  return hipSuccess;
}
template <typename A>
inline hipError_t hipLaunchCooperativeKernel(void (*k)(A), dim3 grid, dim3 block, void** args, unsigned lds, hipStream_t) {
  const A arg = *(const A*)args[0];
  emu::launch_coop([&]() { k(arg); }, grid, block, lds);
  return hipSuccess;
}
inline hipError_t hipSetDevice(int) { return hipSuccess; }
constexpr unsigned hipStreamNonBlocking = 1, hipEventDisableTiming = 2;
inline hipError_t hipStreamCreateWithFlags(hipStream_t* st, unsigned) { *st = (hipStream_t)new char[1]; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t st) { delete[] (char*)st; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = (hipEvent_t)new char[1]; return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 160 * 1024;
  return hipSuccess;
}
#define HIP_DYNAMIC_SHARED(type, var) type* var = (type*)emu::dyn_lds();
