// CPU emulation runtime for hip_runtime.h (test infrastructure only).
#include "hip/hip_runtime.h"

#include <barrier>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <thread>
#include <vector>

namespace hipemu {
thread_local idx3 tl_thread{0, 0, 0};
thread_local idx3 tl_block{0, 0, 0};
dim3 g_grid, g_block;

namespace {
struct Wave {
  int size = 0;
  std::unique_ptr<std::barrier<>> bar;
  unsigned char slot[64][16];
};
std::unique_ptr<std::barrier<>> g_block_bar;
std::vector<Wave> g_waves;
thread_local int tl_lane = 0;
thread_local Wave* tl_wave = nullptr;
hipError_t g_last = hipSuccess;
}  // namespace

hipError_t last_error(hipError_t set) {
  if (set >= 0) g_last = set;
  return set >= 0 ? set : g_last;
}

void syncthreads() { g_block_bar->arrive_and_wait(); }

int lane_id() { return tl_lane; }

void wave_exchange(const void* in, void* out, size_t bytes, int src_lane) {
  Wave* w = tl_wave;
  std::memcpy(w->slot[tl_lane], in, bytes);
  w->bar->arrive_and_wait();
  if (src_lane >= 0 && src_lane < w->size) std::memcpy(out, w->slot[src_lane], bytes);
  else std::memcpy(out, in, bytes);
  w->bar->arrive_and_wait();
}

unsigned long long wave_ballot(bool pred) {
  Wave* w = tl_wave;
  w->slot[tl_lane][0] = pred ? 1 : 0;
  w->bar->arrive_and_wait();
  unsigned long long m = 0;
  for (int l = 0; l < w->size; ++l)
    if (w->slot[l][0]) m |= 1ull << l;
  w->bar->arrive_and_wait();
  return m;
}

// DPP move: lane i takes src from a partner lane chosen by ctrl; lanes of rows
// (16 lanes) or banks (4 lanes within a row) disabled by the masks keep old.
int wave_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  Wave* w = tl_wave;
  std::memcpy(w->slot[tl_lane], &src, sizeof(int));
  w->bar->arrive_and_wait();
  const int i = tl_lane, row = i / 16, j = i % 16;
  int sl = -1;
  if (ctrl >= 0 && ctrl <= 0xff) sl = 4 * (i / 4) + ((ctrl >> (2 * (i % 4))) & 3);
  else if (ctrl == 0x140) sl = 16 * row + (15 - j);
  else if (ctrl == 0x141) sl = 16 * row + 8 * (j / 8) + (7 - j % 8);
  else if (ctrl == 0x142) sl = row > 0 ? 16 * row - 1 : -1;
  else if (ctrl == 0x143) sl = row > 1 ? 31 : -1;
  else { std::fprintf(stderr, "emulated DPP control %#x not supported\n", ctrl); std::abort(); }
  int r = old;
  const bool enabled = ((row_mask >> row) & 1) && ((bank_mask >> (j / 4)) & 1);
  if (enabled) {
    if (sl >= 0 && sl < w->size) std::memcpy(&r, w->slot[sl], sizeof(int));
    else if (bound_ctrl) r = 0;
  }
  w->bar->arrive_and_wait();
  return r;
}

void run_grid(dim3 grid, dim3 block, void (*body)(void*), void* arg) {
  const int nt = static_cast<int>(block.x);
  g_grid = grid;
  g_block = block;
  g_block_bar = std::make_unique<std::barrier<>>(nt);
  const int nw = (nt + 63) / 64;
  g_waves = std::vector<Wave>(nw);
  for (int w = 0; w < nw; ++w) {
    g_waves[w].size = std::min(64, nt - 64 * w);
    g_waves[w].bar = std::make_unique<std::barrier<>>(g_waves[w].size);
  }
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int t = 0; t < nt; ++t) {
    th.emplace_back([=]() {
      tl_thread = {static_cast<unsigned>(t), 0, 0};
      tl_lane = t % 64;
      tl_wave = &g_waves[t / 64];
      for (unsigned by = 0; by < grid.y; ++by)
        for (unsigned bx = 0; bx < grid.x; ++bx) {
          tl_block = {bx, by, 0};
          body(arg);
          g_block_bar->arrive_and_wait();
        }
    });
  }
  for (auto& x : th) x.join();
}
}  // namespace hipemu

struct hipemu_event { int dummy; };

hipError_t hipGetLastError() {
  hipError_t e = hipemu::last_error();
  hipemu::last_error(hipSuccess);
  return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "emulated HIP error"; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipMalloc(void** p, size_t bytes) { *p = std::malloc(bytes); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) { return hipMalloc(p, bytes); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind k) { return hipMemcpyAsync(dst, src, bytes, k, nullptr); }
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t) { std::memset(dst, v, bytes); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new hipemu_event{0}; return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
