// Test harness: host-thread execution of the HIP subset used by the library's kernel sources, so
// that tests/test_hipemu_kernels.py can run the kernel code on the CPU against the oracle.  One
// host thread per GPU thread, blocks one after another, __shared__ variables are function statics
// (shared by the block's threads), __syncthreads is a std::barrier, exited threads drop out of
// later barriers, device memory is host memory.  It checks kernel logic (indexing, barriers,
// reductions, decisions); it says nothing about GPU timing, and the package never loads it.
#pragma once
#include <algorithm>
#include <atomic>
#include <barrier>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define HIP_SYMBOL(x) (&x)
#define __align__(n) alignas(n)
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt(x))  // hardware 1/sqrt estimate
#define __builtin_amdgcn_rcp(x) (1.0 / (x))  // hardware 1/x estimate
#define __builtin_amdgcn_readfirstlane(x) (x)  // callers pass wave-uniform values
#define MHD_GLOBAL_AS  // one address space on the host

// Raw buffer resources: a base and a range in bytes.  An access outside the range is a kernel
// indexing error here (on the GPU a load there would return 0), so it aborts the test process.
struct EmuBufferRsrc {
  char* base;
  unsigned long long n;
};
typedef unsigned EmuU32x2 __attribute__((vector_size(8)));
inline EmuBufferRsrc emu_make_buffer_rsrc(void* p, short, int n, int) { return {(char*)p, (unsigned)n}; }
inline char* emu_buffer_at(const EmuBufferRsrc& r, unsigned off, unsigned soff) {
  const unsigned long long a = (unsigned long long)off + soff;
  if (a + 8 > r.n) { std::fprintf(stderr, "hipemu: buffer access at byte %llu of %llu\n", a, r.n); std::abort(); }
  return r.base + a;
}
inline EmuU32x2 emu_raw_buffer_load_b64(EmuBufferRsrc r, unsigned off, unsigned soff, int) {
  EmuU32x2 v;
  std::memcpy(&v, emu_buffer_at(r, off, soff), 8);
  return v;
}
inline void emu_raw_buffer_store_b64(EmuU32x2 v, EmuBufferRsrc r, unsigned off, unsigned soff, int) {
  std::memcpy(emu_buffer_at(r, off, soff), &v, 8);
}
#define __amdgpu_buffer_rsrc_t EmuBufferRsrc
#define __builtin_amdgcn_make_buffer_rsrc emu_make_buffer_rsrc
#define __builtin_amdgcn_raw_buffer_load_b64 emu_raw_buffer_load_b64
#define __builtin_amdgcn_raw_buffer_store_b64 emu_raw_buffer_store_b64

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct EmuIdx { unsigned x, y, z; };
struct alignas(16) double2 { double x, y; };
inline thread_local EmuIdx threadIdx{0, 0, 0}, blockIdx{0, 0, 0};
inline thread_local dim3 blockDim, gridDim;

inline thread_local std::barrier<>* emu_bar = nullptr;
inline void __syncthreads() { emu_bar->arrive_and_wait(); }
// barrier that returns nonzero in every thread when pred is nonzero in any thread of the block
// (blocks run one after another, so one accumulator serves them all)
inline std::atomic<int> emu_or_acc{0};
inline int __syncthreads_or(int pred) {
  emu_bar->arrive_and_wait();
  if (pred) emu_or_acc.fetch_or(1);
  emu_bar->arrive_and_wait();
  const int r = emu_or_acc.load();
  emu_bar->arrive_and_wait();
  emu_or_acc.store(0);
  return r;
}

inline int atomicOr(int* a, int v) { return __atomic_fetch_or(a, v, __ATOMIC_SEQ_CST); }
inline unsigned long long atomicAdd(unsigned long long* a, unsigned long long v) {
  return __atomic_fetch_add(a, v, __ATOMIC_SEQ_CST);
}
inline int atomicAdd(int* a, int v) { return __atomic_fetch_add(a, v, __ATOMIC_SEQ_CST); }

template <class F, class... A>
void emu_launch(F f, dim3 g, dim3 b, A... args) {
  const unsigned nt = b.x * b.y * b.z;
  for (unsigned bz = 0; bz < g.z; ++bz)
    for (unsigned by = 0; by < g.y; ++by)
      for (unsigned bx = 0; bx < g.x; ++bx) {
        std::barrier<> bar((std::ptrdiff_t)nt);
        std::vector<std::thread> th;
        th.reserve(nt);
        for (unsigned t = 0; t < nt; ++t)
          th.emplace_back([&, t] {
            threadIdx = EmuIdx{t % b.x, (t / b.x) % b.y, t / (b.x * b.y)};
            blockIdx = EmuIdx{bx, by, bz};
            blockDim = b; gridDim = g; emu_bar = &bar;
            f(args...);
            bar.arrive_and_drop();
          });
        for (auto& x : th) x.join();
      }
}
// Stream capture: while a capture is open, launches are recorded (with their arguments) instead of
// run; a graph is that list, and launching it runs the launches in order.  Only kernel launches may
// be captured (copies and memsets made while capturing are reported by the end of the capture).
struct EmuGraph { std::vector<std::function<void()>> ops; };
inline thread_local EmuGraph* emu_capture = nullptr;
inline thread_local bool emu_capture_bad = false;
template <class F, class... A>
void emu_launch_or_record(F f, dim3 g, dim3 b, A... args) {
  if (emu_capture) emu_capture->ops.push_back([=] { emu_launch(f, g, b, args...); });
  else emu_launch(f, g, b, args...);
}
#define hipLaunchKernelGGL(F, G, B, S, STREAM, ...) emu_launch_or_record(F, dim3(G), dim3(B), __VA_ARGS__)

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 };
typedef void* hipStream_t;
struct EmuEvent { double t; };
typedef EmuEvent* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault };
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
// a device symbol's address is its host address here (device memory is host memory)
template <class T> inline hipError_t hipGetSymbolAddress(void** p, T* sym) { *p = (void*)sym; return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "emu error"; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipMalloc(void** p, size_t n) { *p = std::calloc(1, n ? n : 8); return *p ? hipSuccess : hipErrorOutOfMemory; }
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned = 0) { return hipMalloc(p, n); }
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipHostFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { if (emu_capture) emu_capture_bad = true; std::memmove(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t = nullptr) { if (emu_capture) emu_capture_bad = true; std::memmove(d, s, n); return hipSuccess; }
inline hipError_t hipMemset(void* d, int v, size_t n) { if (emu_capture) emu_capture_bad = true; std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t = nullptr) { if (emu_capture) emu_capture_bad = true; std::memset(d, v, n); return hipSuccess; }
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = nullptr; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = (hipEvent_t)std::calloc(1, 8); return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)std::calloc(1, 8); return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { std::free(e); return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
// Graph capture on one stream (see emu_launch_or_record); a second open capture, or a copy or
// memset inside one, makes the end of the capture fail.
typedef EmuGraph* hipGraph_t;
typedef EmuGraph* hipGraphExec_t;
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
enum { hipErrorNotSupported = 801, hipErrorStreamCaptureInvalidated = 901 };
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
  if (emu_capture) return hipErrorNotSupported;
  emu_capture = new EmuGraph();
  emu_capture_bad = false;
  return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  if (!emu_capture) { *g = nullptr; return hipErrorInvalidValue; }
  EmuGraph* c = emu_capture;
  emu_capture = nullptr;
  if (emu_capture_bad) { delete c; *g = nullptr; return hipErrorStreamCaptureInvalidated; }
  *g = c;
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, void*, void*, size_t) {
  *e = new EmuGraph(*g);
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto& op : e->ops) op();
  return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
