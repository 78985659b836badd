// CPU emulation of the subset of HIP that the xs21 sources use.
//
// TEST INFRASTRUCTURE ONLY: lets the unmodified kernel and host sources build
// with g++ (+ AddressSanitizer) so that indexing, bounds and synchronisation
// logic can be checked on a machine without a GPU.  Every GPU thread of a
// block runs as an OS thread; __syncthreads is a barrier over the block and
// wave intrinsics exchange values through a per-wave slot array.  Blocks run
// one after another, so __shared__ maps to function-static storage.
//
// Streams are queues of deferred operations (launches, copies, event records
// and waits).  Work runs only when the host synchronises; the scheduler then
// interleaves the streams' queues in a seeded random order that respects
// stream order and event waits (XS21_EMU_STREAMS = "random:<seed>", the
// default "random:1", or "eager" to run every operation at issue), so that a
// missing dependency between streams shows up as a wrong result.
#pragma once

#include <stdint.h>
#include <stddef.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <tuple>
#include <utility>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __constant__
#define __align__(n) alignas(n)
#define HIP_SYMBOL(x) (&(x))

typedef int hipError_t;
enum {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidSymbol = 13,
  hipErrorNotSupported = 801,
  hipErrorNoDevice = 100,
  hipErrorLaunchFailure = 719
};
typedef void* hipStream_t;
typedef struct hipemu_graph* hipGraph_t;
typedef struct hipemu_graph_exec* hipGraphExec_t;
typedef enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1,
               hipStreamCaptureModeRelaxed = 2 } hipStreamCaptureMode;
struct hipDeviceProp_t {
  char gcnArchName[256];
};
typedef struct hipemu_event* hipEvent_t;
typedef enum { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
               hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 } hipMemcpyKind;
#define hipEventDisableTiming 2u
#define hipStreamNonBlocking 1u
#define hipHostMallocDefault 0u

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace hipemu {
struct idx3 { unsigned x, y, z; };
extern thread_local idx3 tl_thread;
extern thread_local idx3 tl_block;
extern dim3 g_grid, g_block;
void syncthreads();
void wave_sync();
void wave_exchange(const void* in, void* out, size_t bytes, int src_lane);
int lane_id();
unsigned long long wave_ballot(bool pred);
int wave_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl);
void run_grid(dim3 grid, dim3 block, void (*body)(void*), void* arg);
extern unsigned char* g_dyn_shared;  // dynamic LDS of the running launch
void enqueue(hipStream_t s, std::function<void()> op);
hipError_t last_error(hipError_t set = -1);
}  // namespace hipemu

#define HIP_DYNAMIC_SHARED(type, var) type* var = reinterpret_cast<type*>(::hipemu::g_dyn_shared);

#define threadIdx (::hipemu::tl_thread)
#define blockIdx (::hipemu::tl_block)
#define gridDim (::hipemu::g_grid)
#define blockDim (::hipemu::g_block)

inline void __syncthreads() { ::hipemu::syncthreads(); }
// a wave's lanes run as threads here: the wave-level ordering point is a
// barrier over the wave's threads
inline void __builtin_amdgcn_wave_barrier() { ::hipemu::wave_sync(); }
#define __builtin_amdgcn_fence(order, scope) ((void)0)

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  (void)width;
  T r;
  ::hipemu::wave_exchange(&v, &r, sizeof(T), ::hipemu::lane_id() ^ mask);
  return r;
}

inline unsigned long long __ballot(int pred) {
  return ::hipemu::wave_ballot(pred != 0);
}
inline unsigned __lane_id() { return static_cast<unsigned>(::hipemu::lane_id()); }
inline bool __builtin_amdgcn_inverse_ballot_w64(unsigned long long m) { return (m >> __lane_id()) & 1ull; }

inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  return ::hipemu::wave_dpp(old, src, ctrl, row_mask, bank_mask, bound_ctrl);
}
inline int __builtin_amdgcn_readlane(int v, int lane) {
  int r;
  ::hipemu::wave_exchange(&v, &r, sizeof(int), lane);
  return r;
}
// every lane of the wave calls it with all lanes active: lane 0 is the first
inline int __builtin_amdgcn_readfirstlane(int v) { return __builtin_amdgcn_readlane(v, 0); }
inline int __float_as_int(float f) { return __builtin_bit_cast(int, f); }
inline float __int_as_float(int i) { return __builtin_bit_cast(float, i); }
inline float __fdividef(float a, float b) { return a / b; }
inline float __builtin_amdgcn_rcpf(float x) { return 1.0f / x; }
inline float __builtin_amdgcn_exp2f(float x) { return exp2f(x); }
inline int atomicOr(int* p, int v) { return __atomic_fetch_or(p, v, __ATOMIC_RELAXED); }
// Clang's optimiser hint; here it is checked instead
#define __builtin_assume(cond) \
  do {                         \
    if (!(cond)) std::abort(); \
  } while (0)
// Device math function without a host counterpart: the inverse of erfc on
// (0, 2), by bisection on std::erfc (strictly decreasing) and Newton polish.
inline double erfcinv(double y) {
  if (!(y > 0.0 && y < 2.0)) return y == 0.0 ? HUGE_VAL : (y == 2.0 ? -HUGE_VAL : NAN);
  double lo = -30.0, hi = 30.0;
  for (int i = 0; i < 200; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (std::erfc(mid) > y) lo = mid; else hi = mid;
  }
  double x = 0.5 * (lo + hi);
  for (int i = 0; i < 3; ++i) {
    const double df = -1.1283791670955126 * std::exp(-x * x);
    if (df == 0.0) break;
    const double nx = x - (std::erfc(x) - y) / df;
    if (!(nx >= lo - 1e-12 && nx <= hi + 1e-12)) break;
    x = nx;
  }
  return x;
}
template <typename V>
inline void __builtin_nontemporal_store(V v, V* p) { *p = v; }
template <typename V>
inline V __builtin_nontemporal_load(const V* p) { return *p; }
inline float __expf(float x) { return expf(x); }

using std::max;
using std::min;

namespace hipemu {
template <typename F, typename Tuple>
struct Launch {
  F f;
  Tuple args;
  static void body(void* p) {
    auto* self = static_cast<Launch*>(p);
    std::apply(self->f, self->args);
  }
};

template <typename... KArgs, typename... Args>
inline hipError_t launch(void (*k)(KArgs...), dim3 grid, dim3 block, size_t shmem, hipStream_t stream,
                         Args&&... args) {
  if (block.x * block.y * block.z > 1024 || block.y != 1 || block.z != 1 || grid.x == 0 || grid.y == 0 || grid.z == 0)
    return last_error(hipErrorInvalidValue);
  using Tup = std::tuple<KArgs...>;
  using L = Launch<void (*)(KArgs...), Tup>;
  auto l = std::make_shared<L>(L{k, Tup(static_cast<KArgs>(args)...)});
  enqueue(stream, [l, grid, block, shmem] {
    // exactly `shmem` bytes, so that AddressSanitizer sees overruns
    std::unique_ptr<unsigned char[]> dyn(shmem ? new unsigned char[shmem] : nullptr);
    g_dyn_shared = dyn.get();
    run_grid(grid, block, &L::body, l.get());
    g_dyn_shared = nullptr;
  });
  return hipSuccess;
}
}  // namespace hipemu

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  (void)::hipemu::launch(kernel, dim3(grid), dim3(block), shmem, stream, ##__VA_ARGS__)

extern "C++" {
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipDeviceSynchronize();
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipEventDestroy(hipEvent_t e);
// device address of a __device__ variable: the host object itself here
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
// device properties: the architecture name "emu"
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int device);
// launch graphs are not emulated: every call returns hipErrorNotSupported
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, void* node, char* log, size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t x);
hipError_t hipGraphDestroy(hipGraph_t g);
}
