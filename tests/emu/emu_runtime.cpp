// CPU emulation runtime for hip_runtime.h (test infrastructure only).
#include "hip/hip_runtime.h"

#include <barrier>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <memory>
#include <random>
#include <string>
#include <thread>
#include <vector>

namespace hipemu {
thread_local idx3 tl_thread{0, 0, 0};
thread_local idx3 tl_block{0, 0, 0};
dim3 g_grid, g_block;
unsigned char* g_dyn_shared = nullptr;

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

void wave_sync() { tl_wave->bar->arrive_and_wait(); }

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
      for (unsigned bz = 0; bz < grid.z; ++bz)
        for (unsigned by = 0; by < grid.y; ++by)
          for (unsigned bx = 0; bx < grid.x; ++bx) {
            tl_block = {bx, by, bz};
            body(arg);
            g_block_bar->arrive_and_wait();
          }
    });
  }
  for (auto& x : th) x.join();
}
}  // namespace hipemu

struct hipemu_event {
  long last = -1;  // id of the latest record operation issued for this event
};

namespace hipemu {
struct Op {
  enum Kind { kWork, kRecord, kWait } kind;
  std::function<void()> work;
  long id;  // record id (kRecord) or awaited record id (kWait)
};
std::map<hipStream_t, std::deque<Op>> g_queues;  // nullptr: the default stream
std::vector<char> g_done;                        // per record id: executed
std::mt19937_64 g_rng;
int g_mode = -1;  // 0: eager, 1: deferred with random interleaving

int mode() {
  if (g_mode < 0) {
    const char* e = std::getenv("XS21_EMU_STREAMS");
    std::string v = e ? e : "random:1";
    if (v == "eager") {
      g_mode = 0;
    } else {
      g_mode = 1;
      const auto colon = v.find(':');
      g_rng.seed(colon == std::string::npos ? 1 : std::stoull(v.substr(colon + 1)));
    }
  }
  return g_mode;
}

bool runnable(const std::deque<Op>& q) {
  return !q.empty() && (q.front().kind != Op::kWait || g_done[q.front().id]);
}

// Runs the head operation of one runnable queue (chosen at random); false if none is runnable.
bool step() {
  std::vector<std::deque<Op>*> ready;
  for (auto& kv : g_queues)
    if (runnable(kv.second)) ready.push_back(&kv.second);
  if (ready.empty()) return false;
  auto& q = *ready[ready.size() == 1 ? 0 : g_rng() % ready.size()];
  Op op = std::move(q.front());
  q.pop_front();
  if (op.kind == Op::kWork) op.work();
  if (op.kind == Op::kRecord) g_done[op.id] = 1;
  return true;
}

template <typename P>
void drain_until(P done) {
  while (!done())
    if (!step()) {
      std::fprintf(stderr, "emulated streams: deadlock (a wait can never be satisfied)\n");
      std::abort();
    }
}

bool all_empty() {
  for (auto& kv : g_queues)
    if (!kv.second.empty()) return false;
  return true;
}

void push(hipStream_t s, Op op) {
  g_queues[s].push_back(std::move(op));
  if (mode() == 0) drain_until(all_empty);
}

void enqueue(hipStream_t s, std::function<void()> op) { push(s, Op{Op::kWork, std::move(op), -1}); }
}  // namespace hipemu

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
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  hipemu::enqueue(s, [=] { std::memmove(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind k) {
  hipMemcpyAsync(dst, src, bytes, k, nullptr);
  return hipDeviceSynchronize();
}
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t s) {
  hipemu::enqueue(s, [=] { std::memset(dst, v, bytes); });
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  hipemu::drain_until([s] { return hipemu::g_queues[s].empty(); });
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() {
  hipemu::drain_until(hipemu::all_empty);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new char;  // a unique handle
  hipemu::g_queues[*s];
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  hipStreamSynchronize(s);
  hipemu::g_queues.erase(s);
  delete static_cast<char*>(s);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new hipemu_event; return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  e->last = static_cast<long>(hipemu::g_done.size());
  hipemu::g_done.push_back(0);
  hipemu::push(s, hipemu::Op{hipemu::Op::kRecord, nullptr, e->last});
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  // waiting for an event that was never recorded completes at once
  if (e->last >= 0) hipemu::push(s, hipemu::Op{hipemu::Op::kWait, nullptr, e->last});
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (e->last >= 0) {
    const long id = e->last;
    hipemu::drain_until([id] { return hipemu::g_done[id] != 0; });
  }
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  hipEventSynchronize(a);
  hipEventSynchronize(b);
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }

hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  if (!p || !symbol) return hipErrorInvalidValue;
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}

hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int device) {
  if (!p || device != 0) return hipErrorInvalidValue;
  std::memset(p, 0, sizeof *p);
  std::strcpy(p->gcnArchName, "emu");
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) { return hipErrorNotSupported; }
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, char*, size_t) { return hipErrorNotSupported; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipErrorNotSupported; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipErrorNotSupported; }
