// C-ABI of the xs21 library: context, boxes, workspace layout, prepare and
// evaluation drivers.  All device memory is the caller's workspace; all device
// work is issued in order to the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/xs21.h"
#include "common.hpp"
#include "internal.hpp"
#include "launch.hpp"
#include "plan.hpp"

namespace {

using xs21::cplx;
using xs21::WalkerConst;

constexpr int kNtab = 512;       // twiddle table length (largest transform)
constexpr size_t kAlign = 256;

thread_local std::string g_error;

xs21_status fail(xs21_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return s;
}

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

size_t real_size(int dtype) { return dtype == xs21::kF64 ? 8 : 4; }
size_t store_size(int storage) { return storage == xs21::kF64 ? 8 : (storage == xs21::kF32 ? 4 : 2); }

struct BoxRec {
  int n = 0;
  double box = 0, z = 0;
  int nbins = 0;
  int dtype = 0;
  std::vector<unsigned char> host;  // host copy until prepare
  const void* dev_src = nullptr;
  std::vector<double> radii;
  std::vector<long> n2max;
  std::vector<int8_t> bintab;
  std::vector<double> counts, kmean;
  int storage = 0;
  int rbatch = 1;             // radii smoothed per launch
  std::vector<long> cut;      // (n2max, kmax) per ladder radius, then one pair keeping every mode
  std::vector<int32_t> live;  // smoothing z pass: (radius << 24) | tile of the tiles inside each radius's disk
  std::vector<long> live_off; // first entry of radius j in live (nr + 1 offsets)
  std::vector<int32_t> live_y;   // smoothing y pass: (radius << 24) | tile of the kx tiles up to each kmax
  std::vector<long> live_y_off;  // first entry of radius j in live_y
  std::vector<int32_t> bins_live;   // binning pass: tiles with a column inside ny^2 + kx^2 <= (n/2)^2
  double live_yx = 0;            // (ky, kx < n/2) pairs inside that disk
  bool mock_set = false;      // xs21_set_mock has uploaded the likelihood table
  // workspace offsets
  size_t off_bintab = 0, off_counts = 0, off_cut = 0, off_delta = 0, off_od = 0, off_dR = 0, off_like = 0;
  size_t off_slots = 0;       // SlotPlan2 per radius slot, for planning from device walker parameters
  size_t off_live = 0;        // the live-tile list of the smoothing z pass
  size_t off_live_y = 0;      // the live-tile list of the smoothing y pass
  size_t off_bins_live = 0;   // the live-tile list of the binning pass
  xs21::BoxPlan bplan{};      // the box's planning scalars (kernel argument)

  size_t cells() const { return static_cast<size_t>(n) * n * n; }
  size_t half() const { return static_cast<size_t>(n / 2 + 1); }
  size_t pitch() const { return static_cast<size_t>(xs21::half_pitch(n)); }
  size_t spec_bytes() const { return static_cast<size_t>(n) * n * pitch() * 2 * real_size(dtype); }
  int nr() const { return static_cast<int>(radii.size()); }
  size_t wc_size() const { return dtype == xs21::kF64 ? sizeof(WalkerConst<double>) : sizeof(WalkerConst<float>); }
  size_t table_bytes(int walkers) const;
};

// Walker tables of one box for `cap` walkers of the two-population model:
// the host writes [WalkerConst][WalkerPlan2][SlotPlan2] (the first `host`
// bytes), the planning pass writes the thresholds thr[cap][2][stride] and the
// cell-radius efficiency tables zt[cap][kZetaPitch].
struct Tab2 {
  size_t wc = 0, wp = 0, slots = 0, host = 0, thr = 0, zt = 0, total = 0;
};

Tab2 tab2(const BoxRec& b, int cap) {
  Tab2 t;
  const size_t rs = real_size(b.dtype), stride = static_cast<size_t>(xs21::thr_stride());
  size_t off = 0;
  t.wc = off;
  off += align_up(cap * b.wc_size());
  t.wp = off;
  off += align_up(cap * sizeof(xs21::WalkerPlan2));
  t.slots = off;
  off += align_up(stride * sizeof(xs21::SlotPlan2));
  t.host = off;
  t.thr = off;
  off += align_up(static_cast<size_t>(cap) * 2 * stride * rs);
  t.zt = off;
  off += align_up(static_cast<size_t>(cap) * xs21::kZetaPitch * rs);
  t.total = off;
  return t;
}

size_t BoxRec::table_bytes(int walkers) const {
  const size_t one = align_up(walkers * wc_size()) +
                     align_up(static_cast<size_t>(walkers) * xs21::thr_stride() * real_size(dtype));
  return std::max(one, tab2(*this, walkers).total);
}

struct Layout {
  size_t tw32 = 0, tw64 = 0;
  size_t tables = 0, tables_bytes = 0;     // batched walker tables (all boxes)
  size_t one_table = 0, one_table_bytes = 0;  // single-walker table
  size_t outs = 0;                          // small device outputs (plain / debug)
  size_t samp = 0, samp_pk = 0;             // sampler: proposals, aux, chi^2; their P(k)
  size_t slot_tab = 0;                      // sorted flag-test tables of one walker group
  size_t scratch = 0, scratch_bytes = 0;    // union of smoothing / evaluation / plain scratch
  size_t total = 0;
};

}  // namespace

// Launch shapes of one box size (0 / -1: the launchers' defaults).
struct Tune {
  int ion_blocks = 0, pipe_blocks = 0, bins_blocks = 0, flag_test = -1, group = 0;
};

struct xs21_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

struct xs21_ctx {
  int device = 0;
  std::map<int, Tune> tune;   // per grid size n
  bool capturing = false;     // inside xs21_capture_begin / xs21_capture_end
  hipStream_t stream = nullptr;
  xs21_physics phys{};
  std::vector<BoxRec> boxes;
  bool prepared = false;
  bool poisoned = false;
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  int storage = 0;
  int max_walkers = 0;
  int max_plain = 0;
  int group = 0;
  Layout lay;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  // kernel timing
  struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double bytes, ops;
  };
  bool prof = false;
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> pool;
  double tot_ms[XS21_K_COUNT] = {};
  long long launches[XS21_K_COUNT] = {};
  double tot_bytes[XS21_K_COUNT] = {};
  double tot_ops[XS21_K_COUNT] = {};
};

namespace {

xs21_status hip_fail(xs21_ctx* c, hipError_t e, const char* what) {
  if (c) c->poisoned = true;
  return fail(XS21_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHECK(ctx, call)                                  \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
  } while (0)

xs21_status check_ctx(xs21_ctx* c) {
  if (!c) return fail(XS21_EINVAL, "null context");
  if (c->poisoned) return fail(XS21_ESTATE, "context poisoned by an earlier device error");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  return XS21_OK;
}

xs21_status check_box(xs21_ctx* c, xs21_box b) {
  if (b < 0 || b >= static_cast<int>(c->boxes.size())) return fail(XS21_EINVAL, "unknown box handle %d", b);
  return XS21_OK;
}

// Entry points that synchronise with the host or upload host data cannot be
// recorded into a graph.
xs21_status no_capture(xs21_ctx* c, const char* what) {
  if (c->capturing) return fail(XS21_ESTATE, "%s is not allowed during graph capture", what);
  return XS21_OK;
}

Tune tune_of(const xs21_ctx* c, int n) {
  const auto it = c->tune.find(n);
  return it == c->tune.end() ? Tune{} : it->second;
}

// Walkers per ionisation launch on boxes of size n.
int group_of(const xs21_ctx* c, int n) {
  const int g = tune_of(c, n).group;
  return g > 0 ? std::min(g, c->group) : c->group;
}

hipEvent_t pooled_event(xs21_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launches through `f` on stream s; when timing is on, brackets it with events
// on s and remembers the pair with the launch's algorithmic bytes and ops.
template <typename F>
hipError_t timed(xs21_ctx* c, hipStream_t s, int kind, double bytes, F&& f, double ops = 0.0) {
  if (!c->prof) return f();
  hipEvent_t a = pooled_event(c), b = pooled_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = f();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  if (e != hipSuccess) return e;
  c->pending.push_back({kind, a, b, bytes, ops});
  return hipSuccess;
}


bool pow2_in_range(int n) { return n >= 8 && n <= 512 && (n & (n - 1)) == 0; }

long isqrt(long v) {
  long r = static_cast<long>(std::floor(std::sqrt(static_cast<double>(v))));
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// (n2max, kmax) of a sharp-k smoothing of radius R on box b: kmax is the
// largest |kx| any kept mode can have.
void cut_pair(const BoxRec& b, double radius, long* out) {
  const long n2 = xs21::plan::n2max(radius, b.box);
  out[0] = n2;
  out[1] = std::min(isqrt(n2), static_cast<long>(b.n / 2));
}

// Radii smoothed per launch: as many as fit a 4 GiB batch of spectra (the
// environment variable XS21_RADIUS_BATCH overrides it).
int radius_batch(const BoxRec& b) {
  long rb = static_cast<long>((4ull << 30) / b.spec_bytes());
  if (const char* e = std::getenv("XS21_RADIUS_BATCH")) rb = std::atol(e);
  return static_cast<int>(std::max(1L, std::min<long>(rb, b.nr())));
}

int box_storage(const BoxRec& b, int storage) { return b.dtype == xs21::kF64 ? xs21::kF64 : storage; }

// Scratch of each phase, per box; each region is the maximum over boxes.
// Smoothing: the box spectrum + one spectrum per radius of a launch batch
// (at least two: the velocity-gradient field uses a spectrum and a real box).
size_t smooth_scratch(const BoxRec& b) {
  return (1 + static_cast<size_t>(std::max(b.rbatch, 2))) * align_up(b.spec_bytes());
}

// Evaluation: walker spectra, their Nyquist planes, bin partial sums, x_HI partial sums.
size_t nyq_bytes(const BoxRec& b) { return static_cast<size_t>(b.n) * b.n * 2 * real_size(b.dtype); }

size_t eval_scratch(const BoxRec& b, int group) {
  const long tiles = xs21::bins_tiles(b.n);
  return align_up(group * b.spec_bytes()) + align_up(group * nyq_bytes(b)) +
         align_up(static_cast<size_t>(group) * tiles * b.nbins * 8) +
         align_up(static_cast<size_t>(group) * xs21::ion_grid_max(b.n) * 8);
}

size_t plain_scratch(const BoxRec& b, int max_plain) {
  return 2 * align_up(b.spec_bytes()) + align_up(static_cast<size_t>(max_plain) * b.cells() * real_size(b.dtype)) +
         eval_scratch(b, 1);
}

Layout compute_layout(const xs21_ctx* c, int storage, int max_walkers, int max_plain, int group,
                      std::vector<BoxRec>& boxes) {
  Layout L;
  size_t off = 0;
  L.tw32 = off;
  off += align_up(kNtab * 8);
  L.tw64 = off;
  off += align_up(kNtab * 16);
  size_t tables = 0, one = 0, scratch = 0;
  for (auto& b : boxes) {
    b.storage = box_storage(b, storage);
    b.rbatch = radius_batch(b);
    b.off_bintab = off;
    off += align_up(b.bintab.size());
    b.off_counts = off;
    off += align_up(b.nbins * 8);
    b.off_cut = off;
    off += align_up(b.cut.size() * sizeof(long));
    b.off_live = off;
    off += align_up(b.live.size() * sizeof(int32_t));
    b.off_live_y = off;
    off += align_up(b.live_y.size() * sizeof(int32_t));
    b.off_bins_live = off;
    off += align_up(b.bins_live.size() * sizeof(int32_t));
    b.off_like = off;
    off += align_up(3 * static_cast<size_t>(b.nbins) * 8);
    b.off_slots = off;
    off += align_up(xs21::thr_stride() * sizeof(xs21::SlotPlan2));
    b.off_delta = off;
    off += align_up(b.cells() * real_size(b.dtype));
    b.off_od = off;
    off += align_up(b.cells() * real_size(b.dtype));
    b.off_dR = off;
    off += align_up(static_cast<size_t>(b.nr()) * b.cells() * store_size(b.storage));
    tables += b.table_bytes(max_walkers);
    one = std::max({one,
                    align_up(sizeof(WalkerConst<double>)) + align_up(xs21::thr_stride() * 8) +
                        align_up(2 * sizeof(long) * xs21::max_radii()),
                    tab2(b, 1).total});
    scratch = std::max({scratch, smooth_scratch(b), eval_scratch(b, group), plain_scratch(b, max_plain)});
  }
  (void)c;
  L.tables = off;
  L.tables_bytes = tables;
  off += align_up(tables);
  L.one_table = off;
  L.one_table_bytes = one;
  off += align_up(one);
  L.outs = off;
  off += align_up(8 * 256);
  // sampler chunk of max_walkers: proposals [5], aux [2], chi^2 [1] per walker,
  // then P(k) rows [walker][box][max_bins] over every registered box
  L.samp = off;
  off += align_up(static_cast<size_t>(max_walkers) * 8 * 8);
  L.samp_pk = off;
  off += align_up(static_cast<size_t>(max_walkers) * boxes.size() * xs21::max_bins() * 8);
  L.slot_tab = off;
  off += align_up(xs21::slot_table_bytes());
  L.scratch = off;
  L.scratch_bytes = scratch;
  off += align_up(scratch);
  L.total = off;
  return L;
}

// Walker constants and its thresholds in radius slots s = nr - 1 - j (slot 0
// is the cell radius, the last ladder entry), padded to thr_stride() slots:
// +inf for radii above the walker's R_mfp (plain lists use every radius) and
// past the ladder end.  The kernel tests the slots in groups of 8 up to the
// last group holding a used slot.
template <typename T>
void fill_walker_table(const xs21::plan::WalkerPlan& wp, bool plain, unsigned char* wc_dst, T* thr_dst,
                       double zeta) {
  const int nr = static_cast<int>(wp.thr.size());
  const int used = plain ? nr : nr - wp.first;
  WalkerConst<T> c{};
  c.zeta = static_cast<T>(zeta);
  c.a_cell = static_cast<T>(wp.a_cell);
  c.chunks = (used + 7) / 8;
  // mode 2 iff zeta > 1 (erfc^-1(1/zeta) > 0: the cell-radius threshold
  // delta_c - sqrt(2 dsig2) erfc^-1(1/zeta) lies below delta_c)
  c.partial = wp.partial ? (wp.u_star > 0.0 ? 2 : 1) : 0;
  c.ha = static_cast<float>(0.5 * wp.a_cell);
  c.a2l = static_cast<float>(wp.a_cell * wp.a_cell * 1.4426950408889634074);
  c.upper = 0;
  std::memcpy(wc_dst, &c, sizeof c);
  const T inf = std::numeric_limits<T>::infinity();
  for (int s = 0; s < xs21::thr_stride(); ++s)
    thr_dst[s] = s < used ? static_cast<T>(wp.thr[nr - 1 - s]) : inf;
}

// Writes the constants + thresholds of `walkers` for box b into host memory
// laid out as [WalkerConst x count][thr x count x nr].
void build_tables(const xs21_physics& p, const BoxRec& b, const xs21_walker* w, int count, bool plain,
                  const std::vector<double>& radii, unsigned char* dst, int capacity) {
  const size_t wcs = b.wc_size();
  unsigned char* thr_base = dst + align_up(capacity * wcs);
  const int nr = static_cast<int>(radii.size());
  for (int i = 0; i < count; ++i) {
    const auto wp = xs21::plan::walker(p, b.z, radii.data(), nr, w[i]);
    const size_t ts = static_cast<size_t>(xs21::thr_stride());
    if (b.dtype == xs21::kF64)
      fill_walker_table<double>(wp, plain, dst + i * wcs, reinterpret_cast<double*>(thr_base) + i * ts, w[i].zeta);
    else
      fill_walker_table<float>(wp, plain, dst + i * wcs, reinterpret_cast<float*>(thr_base) + i * ts, w[i].zeta);
  }
}

// Index of the first ladder radius <= r_mfp (the cell radius if none is).
int first_radius(const BoxRec& b, double r_mfp) {
  for (int j = 0; j < b.nr() - 1; ++j)
    if (b.radii[j] <= r_mfp) return j;
  return b.nr() - 1;
}

template <typename T>
void put_const(unsigned char* dst, double a_cell, int used, bool partial) {
  WalkerConst<T> c{};
  c.zeta = T(1);   // the efficiency lives in the planned thresholds and table
  c.a_cell = static_cast<T>(a_cell);
  c.chunks = (used + 7) / 8;
  c.partial = partial ? 1 : 0;
  c.upper = 0;   // set by the planning pass
  std::memcpy(dst, &c, sizeof c);
}

// Host part of the two-population tables of `count` walkers on box b (the
// shared ladder), written at dst in the Tab2 layout for `cap` walkers.
void build_tables2(const xs21_physics& p, const BoxRec& b, const xs21_walker2* w, int count, unsigned char* dst,
                   int cap) {
  const Tab2 t = tab2(b, cap);
  const auto slots = xs21::plan::slots2(p, b.z, b.radii);
  std::memset(dst + t.slots, 0, t.host - t.slots);
  std::memcpy(dst + t.slots, slots.data(), slots.size() * sizeof(xs21::SlotPlan2));
  const double ds = slots[0].ds_cool;
  const double a_cell = ds > 0.0 ? 1.0 / std::sqrt(2.0 * ds) : 0.0;
  for (int i = 0; i < count; ++i) {
    const int used = b.nr() - first_radius(b, w[i].r_mfp);
    if (b.dtype == xs21::kF64)
      put_const<double>(dst + t.wc + i * b.wc_size(), a_cell, used, ds > 0.0);
    else
      put_const<float>(dst + t.wc + i * b.wc_size(), a_cell, used, ds > 0.0);
    const xs21::WalkerPlan2 wp = xs21::plan::walker2(p, b.z, w[i], used);
    std::memcpy(dst + t.wp + i * sizeof wp, &wp, sizeof wp);
  }
}

const void* tw_ptr(const xs21_ctx* c, int dtype) {
  return c->ws + (dtype == xs21::kF64 ? c->lay.tw64 : c->lay.tw32);
}

// Forward 3D real-to-half-complex transform of a real box (in place in `spec`), on stream st.
hipError_t forward3d(xs21_ctx* c, hipStream_t st, const BoxRec& b, const void* real_in, void* spec) {
  const long n = b.n, h = static_cast<long>(b.half()), hp = static_cast<long>(b.pitch());
  const double rs = static_cast<double>(real_size(b.dtype));
  const double cells = static_cast<double>(b.cells()), modes = static_cast<double>(n * n * h);
  const void* tw = tw_ptr(c, b.dtype);
  hipError_t e = timed(c, st, XS21_K_ROWS_R2C, cells * rs + modes * 2 * rs, [&] {
    return xs21::launch_rows_r2c(b.dtype, b.n, real_in, spec, nullptr, n * n, tw, kNtab, st);
  });
  if (e != hipSuccess) return e;
  e = timed(c, st, XS21_K_AXIS_FWD, 2 * modes * 2 * rs, [&] {
    return xs21::launch_axis(b.dtype, b.n, -1, 0, spec, spec, n, hp, h, nullptr, 1, 0, 0, tw, kNtab, st);
  });
  if (e != hipSuccess) return e;
  return timed(c, st, XS21_K_AXIS_FWD, 2 * modes * 2 * rs, [&] {
    return xs21::launch_axis(b.dtype, b.n, -1, 0, spec, spec, 1, n * hp, n * hp, nullptr, 1, 0, 0, tw, kNtab, st);
  });
}

// delta_R = IDFT(mask_R * hat) / N^3 stored as `storage` for `cnt` radii at
// once: radius i uses cutoff pair cut_dev[2 i], cut_dev[2 i + 1] (device) and
// cut_host likewise, its own spectrum tmp + i * spec and output out + i * N^3.
// The three inverse passes only touch the modes the sharp-k ball can hold:
// the z pass the columns with ny^2 + kx^2 <= n2max, the y pass the columns
// kx <= kmax, the x pass the entries kx <= kmax of each row; only the delta_R
// write is full size.
// With tiles != nullptr the z pass runs over that list of ntiles live tiles
// (entries of radii r0 .. r0 + cnt - 1) instead of a block per tile and radius,
// and the y pass over ytiles likewise.
hipError_t smooth_batch(xs21_ctx* c, hipStream_t st, const BoxRec& b, const void* hat, unsigned char* tmp,
                        const long* cut_dev, const long* cut_host, int cnt, int storage, unsigned char* out,
                        const int32_t* tiles = nullptr, long ntiles = 0, int r0 = 0,
                        const int32_t* ytiles = nullptr, long nytiles = 0) {
  const long n = b.n, hp = static_cast<long>(b.pitch());
  const double rs = static_cast<double>(real_size(b.dtype));
  const double cells = static_cast<double>(b.cells());
  const void* tw = tw_ptr(c, b.dtype);
  const long sstride = static_cast<long>(align_up(b.spec_bytes()) / (2 * real_size(b.dtype)));  // complex elements
  double zb = 0, yb = 0, xb = 0;
  long kmax_all = 0;
  for (int i = 0; i < cnt; ++i) {
    const long n2max = cut_host[2 * i], kmax = cut_host[2 * i + 1];
    kmax_all = std::max(kmax_all, kmax);
    double live = 0;  // (ky, kx) columns inside the disk
    for (long kx = 0; kx <= kmax; ++kx) live += static_cast<double>(std::min(2 * isqrt(n2max - kx * kx) + 1, n));
    zb += 2 * live * n * 2 * rs;
    yb += (live + (kmax + 1) * n) * n * 2 * rs;
    xb += (kmax + 1) * n * n * 2 * rs + cells * store_size(storage);
  }
  hipError_t e = timed(c, st, XS21_K_AXIS_INV, zb, [&] {
    if (tiles)
      return xs21::launch_axis_live(b.dtype, b.n, hat, tmp, n * hp, tiles, ntiles, r0, cut_dev, sstride, tw, kNtab,
                                    st);
    return xs21::launch_axis(b.dtype, b.n, +1, 1, hat, tmp, 1, n * hp, n * hp, cut_dev, cnt, 0, sstride, tw, kNtab,
                             st);
  });
  if (e != hipSuccess) return e;
  e = timed(c, st, XS21_K_AXIS_INV, yb, [&] {
    if (ytiles)
      return xs21::launch_axis_live_y(b.dtype, b.n, tmp, hp, kmax_all + 1, ytiles, nytiles, r0, cut_dev, sstride, tw,
                                      kNtab, st);
    return xs21::launch_axis(b.dtype, b.n, +1, 2, tmp, tmp, n, hp, kmax_all + 1, cut_dev, cnt, sstride, sstride, tw,
                             kNtab, st);
  });
  if (e != hipSuccess) return e;
  const double scale = 1.0 / (static_cast<double>(n) * n * n);
  return timed(c, st, XS21_K_ROWS_C2R, xb, [&] {
    return xs21::launch_rows_c2r(b.dtype, storage, b.n, tmp, out, n * n, scale, cut_dev, cnt, sstride,
                                 static_cast<long>(b.cells()), tw, kNtab, st, tune_of(c, b.n).pipe_blocks);
  });
}

// Forward FFT and every smoothed box of the shared ladder of one box, on stream st.
hipError_t smooth_box(xs21_ctx* c, hipStream_t st, const BoxRec& b) {
  unsigned char* hat = c->ws + c->lay.scratch;
  unsigned char* tmp = hat + align_up(b.spec_bytes());
  hipError_t e = forward3d(c, st, b, c->ws + b.off_delta, hat);
  if (e != hipSuccess) return e;
  const long* cut_dev = reinterpret_cast<const long*>(c->ws + b.off_cut);
  for (int j = 0; j < b.nr(); j += b.rbatch) {
    const int cnt = std::min(b.rbatch, b.nr() - j);
    unsigned char* out = c->ws + b.off_dR + static_cast<size_t>(j) * b.cells() * store_size(b.storage);
    const long t0 = b.live_off[j], t1 = b.live_off[j + cnt];
    const long y0 = b.live_y_off[j], y1 = b.live_y_off[j + cnt];
    e = smooth_batch(c, st, b, hat, tmp, cut_dev + 2 * j, b.cut.data() + 2 * j, cnt, b.storage, out,
                     reinterpret_cast<const int32_t*>(c->ws + b.off_live) + t0, t1 - t0, j,
                     reinterpret_cast<const int32_t*>(c->ws + b.off_live_y) + y0, y1 - y0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Density factor of dT_b for box b: odens = (1 + delta) times H / (dv_r/dr + H)
// of eq. (4) when the context includes velocities, else 1 + delta.  The
// gradient is the inverse FFT of (nz^2 / |n|^2) delta_hat (linear continuity
// with growth rate 1, line of sight along the first axis); it reads the box
// spectrum smooth_box left at the start of the scratch region.
hipError_t density_factor(xs21_ctx* c, hipStream_t st, const BoxRec& b) {
  const long n = b.n, h = static_cast<long>(b.half()), hp = static_cast<long>(b.pitch());
  const double rs = static_cast<double>(real_size(b.dtype));
  const double cells = static_cast<double>(b.cells()), modes = static_cast<double>(n * n * h);
  const void* delta = c->ws + b.off_delta;
  void* od = c->ws + b.off_od;
  if (!c->phys.velocity)
    return timed(c, st, XS21_K_OTHER, 3 * cells * rs,
                 [&] { return xs21::launch_los_factor(b.dtype, delta, nullptr, od, b.cells(), 0.0, st); });
  unsigned char* hat = c->ws + c->lay.scratch;
  unsigned char* spec = hat + align_up(b.spec_bytes());
  unsigned char* g = spec + align_up(b.spec_bytes());
  const void* tw = tw_ptr(c, b.dtype);
  hipError_t e = timed(c, st, XS21_K_AXIS_INV, 2 * modes * 2 * rs, [&] {
    return xs21::launch_axis(b.dtype, b.n, +1, 4, hat, spec, 1, n * hp, n * hp, nullptr, 1, 0, 0, tw, kNtab, st);
  });
  if (e != hipSuccess) return e;
  e = timed(c, st, XS21_K_AXIS_INV, 2 * modes * 2 * rs, [&] {
    return xs21::launch_axis(b.dtype, b.n, +1, 0, spec, spec, n, hp, h, nullptr, 1, 0, 0, tw, kNtab, st);
  });
  if (e != hipSuccess) return e;
  const long* full = reinterpret_cast<const long*>(c->ws + b.off_cut) + 2 * b.nr();
  e = timed(c, st, XS21_K_ROWS_C2R, modes * 2 * rs + cells * rs, [&] {
    return xs21::launch_rows_c2r(b.dtype, b.dtype, b.n, spec, g, n * n, 1.0 / cells, full, 1, 0,
                                 static_cast<long>(b.cells()), tw, kNtab, st);
  });
  if (e != hipSuccess) return e;
  return timed(c, st, XS21_K_OTHER, 4 * cells * rs, [&] {
    return xs21::launch_los_factor(b.dtype, delta, g, od, b.cells(), c->phys.dvdr_max, st);
  });
}

// Scratch of one evaluation of `count` walkers on one box: their x-transformed
// spectra (kx < N/2), their Nyquist planes [y][z], then the binning pass's
// FP64 partial sums, then the ionisation pass's x_HI partial sums.
struct EvalSlot {
  void* spec;
  void* nyq;
  double* part;
  double* xpart;
};

EvalSlot eval_slot(const BoxRec& b, unsigned char* base, int count) {
  EvalSlot s;
  s.spec = base;
  s.nyq = base + align_up(count * b.spec_bytes());
  s.part = reinterpret_cast<double*>(static_cast<unsigned char*>(s.nyq) + align_up(count * nyq_bytes(b)));
  s.xpart = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(s.part) +
                                      align_up(static_cast<size_t>(count) * xs21::bins_tiles(b.n) * b.nbins * 8));
  return s;
}

// Ionisation + dT_b + x pass for `count` walkers whose tables are at wc/thr
// (the ALU-bound stage), on stream st.  field_walker >= 0: that walker of the
// group also writes its x_HI and dT_b boxes to fx / fd (device).
hipError_t ion_stage(xs21_ctx* c, hipStream_t st, const BoxRec& b, const EvalSlot& sl, const void* dR, int storage,
                     int nr, const void* wc, const void* thr, const void* zt, int count, double radii_used,
                     int field_walker = -1, void* fx = nullptr, void* fd = nullptr) {
  const long n = b.n, h = static_cast<long>(b.half());
  const double rs = static_cast<double>(real_size(b.dtype));
  const double cells = static_cast<double>(b.cells()), modes = static_cast<double>(n * n * h);
  const double tb = c->phys.tb0_mK * std::sqrt((1.0 + b.z) / 10.0);
  // radii_used: sum over the group's walkers of the radii each filters at
  // (negative when the walkers live on the device: operations not counted)
  const double ion_ops =
      radii_used < 0 ? 0.0 : cells * (radii_used + count * (2.5 * std::log2(static_cast<double>(n)) + 6.0));
  return timed(
      c, st, XS21_K_ION, nr * cells * store_size(storage) + cells * rs + count * modes * 2 * rs,
      [&] {
        return xs21::launch_ion(b.dtype, storage, b.n, dR, c->ws + b.off_od, nr, wc, thr, zt, count, tb,
                                c->phys.delta_c, sl.spec, sl.nyq, sl.xpart, tw_ptr(c, b.dtype), kNtab, st,
                                field_walker, fx, fd, c->ws + c->lay.slot_tab, tune_of(c, b.n).ion_blocks,
                                tune_of(c, b.n).flag_test);
      },
      ion_ops);
}

// y pass, z pass + |X|^2 bins and the final P(k) / mean x_HI of `count`
// walkers (the memory-bound stage), on stream st; pk/xhi are device outputs
// written with the given strides.
hipError_t mem_stage(xs21_ctx* c, hipStream_t st, const BoxRec& b, const EvalSlot& sl, int count, double* pk,
                     long pk_stride, int nbins_out, double* xhi, long xhi_stride) {
  const long n = b.n, h = static_cast<long>(b.half()), hp = static_cast<long>(b.pitch());
  const double rs = static_cast<double>(real_size(b.dtype));
  const double cells = static_cast<double>(b.cells()), modes = static_cast<double>(n * n * h);
  const Tune tu = tune_of(c, b.n);
  const long parts = xs21::bins_parts(b.n, count, tu.bins_blocks);
  const int ion_blocks = xs21::ion_grid(b.n, tu.ion_blocks);   // the x_HI partials of the ionisation launch
  const void* tw = tw_ptr(c, b.dtype);
  // y pass of the kx < N/2 columns, then of the Nyquist planes; only modes
  // with ny^2 + kx^2 <= (N/2)^2 are stored (no other mode is binned)
  const double ntl = static_cast<double>(b.bins_live.size());
  hipError_t e = timed(c, st, XS21_K_AXIS_FWD, count * n * (n * (n / 2) + b.live_yx) * 2 * rs, [&] {
    return xs21::launch_axis_fwd_disk(b.dtype, b.n, sl.spec, count * n, hp, n / 2, false, tw, kNtab, st,
                                      tu.pipe_blocks);
  });
  if (e != hipSuccess) return e;
  e = timed(c, st, XS21_K_AXIS_FWD, count * n * (n + 1) * 2 * rs, [&] {
    return xs21::launch_axis_fwd_disk(b.dtype, b.n, sl.nyq, count, n, n, true, tw, kNtab, st, tu.pipe_blocks);
  });
  if (e != hipSuccess) return e;
  // the binning pass reads the live tiles (TI columns x N values each)
  e = timed(c, st, XS21_K_AXIS_BINS, count * ntl * xs21::bins_tile_cols(b.n) * n * 2 * rs, [&] {
    return xs21::launch_axis_bins(b.dtype, b.n, sl.spec, sl.nyq, count, parts,
                                  reinterpret_cast<const int32_t*>(c->ws + b.off_bins_live),
                                  static_cast<long>(b.bins_live.size()),
                                  reinterpret_cast<const int8_t*>(c->ws + b.off_bintab), b.bintab.data(), b.nbins,
                                  sl.part, tw, kNtab, st);
  });
  if (e != hipSuccess) return e;
  const double L3 = b.box * b.box * b.box;
  const double n6 = std::pow(static_cast<double>(n), 6);
  const double pbytes = static_cast<double>(count) * (parts * b.nbins + ion_blocks) * 8;
  return timed(c, st, XS21_K_FINALIZE, pbytes, [&] {
    return xs21::launch_finalize(count, sl.part, parts, b.nbins, sl.xpart, ion_blocks,
                                 reinterpret_cast<const double*>(c->ws + b.off_counts), L3 / n6, 1.0 / cells, pk,
                                 pk_stride, nbins_out, xhi, xhi_stride, st);
  });
}

}  // namespace

extern "C" {

const char* xs21_last_error(void) { return g_error.c_str(); }

xs21_status xs21_physics_default(xs21_physics* p) {
  if (!p) return fail(XS21_EINVAL, "null physics");
  std::memset(p, 0, sizeof *p);
  p->delta_c = 1.686;
  p->omega_m = 0.27;
  p->omega_l = 0.73;
  p->h = 0.7;
  p->tb0_mK = 27.0;
  p->pk_amp = 1.0;
  p->pk_k0 = 0.05;
  p->z_ref = 9.0;
  p->radius_step = 1.1;
  p->ladder_top = 20.0;
  p->mu = 0.6;
  p->mmin_form = 0;
  p->velocity = 0;
  p->dvdr_max = 0.2;
  g_error.clear();
  return XS21_OK;
}

xs21_status xs21_create(xs21_ctx** out, int hip_device, void* hip_stream, const xs21_physics* phys) {
  g_error.clear();
  if (!out || !phys) return fail(XS21_EINVAL, "null argument");
  *out = nullptr;
  if (!xs21::plan::valid_physics(*phys)) return fail(XS21_EINVAL, "invalid physics constants");
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || hip_device < 0 || hip_device >= count)
    return fail(XS21_EDEVICE, "device %d unavailable (%d devices): %s", hip_device, count, hipGetErrorString(e));
  e = hipSetDevice(hip_device);
  if (e != hipSuccess) return fail(XS21_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  auto* c = new (std::nothrow) xs21_ctx;
  if (!c) return fail(XS21_ENOMEM, "host allocation failed");
  c->device = hip_device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->phys = *phys;
  e = hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete c;
    return fail(XS21_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
  }
  // the static scratch array's address on this device (once per device)
  e = xs21::static_scratch_init(hip_device);
  if (e != hipSuccess) {
    (void)hipEventDestroy(c->upload_done);
    delete c;
    return fail(XS21_EDEVICE, "static scratch lookup (hipGetSymbolAddress): %s", hipGetErrorString(e));
  }
  *out = c;
  return XS21_OK;
}

xs21_status xs21_destroy(xs21_ctx* ctx) {
  g_error.clear();
  if (!ctx) return XS21_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->upload_pending) (void)hipEventSynchronize(ctx->upload_done);
  if (ctx->upload_done) (void)hipEventDestroy(ctx->upload_done);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& r : ctx->pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
  return XS21_OK;
}

xs21_status xs21_sync(xs21_ctx* ctx) {
  g_error.clear();
  xs21_status s = check_ctx(ctx);
  if (s) return s;
  if (xs21_status s_ = no_capture(ctx, "xs21_sync")) return s_;
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  return XS21_OK;
}

xs21_status xs21_add_box(xs21_ctx* ctx, const void* delta, int on_device, xs21_dtype dtype, int n, double box_mpc,
                         double z, int n_bins, xs21_box* out) {
  g_error.clear();
  if (!ctx) return fail(XS21_EINVAL, "null context");
  if (ctx->poisoned) return fail(XS21_ESTATE, "context poisoned");
  if (ctx->prepared) return fail(XS21_ESTATE, "boxes must be added before xs21_prepare");
  if (!delta || !out) return fail(XS21_EINVAL, "null argument");
  if (dtype != XS21_F32 && dtype != XS21_F64) return fail(XS21_EINVAL, "box dtype must be F32 or F64");
  if (!pow2_in_range(n)) return fail(XS21_EINVAL, "n = %d is not a power of two in [8, 512]", n);
  if (!(std::isfinite(box_mpc) && box_mpc > 0)) return fail(XS21_EINVAL, "box side must be finite and > 0");
  if (!(std::isfinite(z) && z > -1.0)) return fail(XS21_EINVAL, "redshift must be finite and > -1");
  if (n_bins < 1 || n_bins > xs21::max_bins()) return fail(XS21_EINVAL, "n_bins must be in [1, %d]", xs21::max_bins());
  BoxRec b;
  b.n = n;
  b.box = box_mpc;
  b.z = z;
  b.nbins = n_bins;
  b.dtype = dtype;
  b.radii = xs21::plan::ladder(ctx->phys.ladder_top, box_mpc / n, ctx->phys.radius_step);
  if (b.nr() > xs21::max_radii())
    return fail(XS21_EUNSUPPORTED, "ladder of %d radii exceeds %d", b.nr(), xs21::max_radii());
  for (double r : b.radii) b.n2max.push_back(xs21::plan::n2max(r, box_mpc));
  b.cut.resize(2 * b.radii.size() + 2);
  for (size_t j = 0; j < b.radii.size(); ++j) cut_pair(b, b.radii[j], &b.cut[2 * j]);
  b.cut[2 * b.radii.size()] = 3L * (n / 2) * (n / 2) + 1;  // every mode
  b.cut[2 * b.radii.size() + 1] = n / 2;
  {
    // tiles of the smoothing z pass with a column (ky, kx) inside the disk
    // ny^2 + kx^2 <= n2max of each radius (padding columns kx > n/2 never are)
    const long hp = xs21::half_pitch(n), h = n / 2 + 1, ti = xs21::axis_tile_cols(n), cols = n * hp;
    const long ntile = (cols + ti - 1) / ti;
    if (ti < 1 || ntile >= (1L << 24) || b.nr() >= 128)
      return fail(XS21_EUNSUPPORTED, "smoothing tile list out of range (n = %d)", n);
    b.live_off.assign(1, 0);
    for (int r = 0; r < b.nr(); ++r) {
      const long n2 = b.cut[2 * r];
      for (long t = 0; t < ntile; ++t) {
        bool any = false;
        for (long i = t * ti; i < std::min(cols, (t + 1) * ti) && !any; ++i) {
          const long ky = i / hp, kx = i % hp, ny = ky < n / 2 ? ky : ky - n;
          any = kx < h && ny * ny + kx * kx <= n2;
        }
        if (any) b.live.push_back(static_cast<int32_t>((static_cast<long>(r) << 24) | t));
      }
      b.live_off.push_back(static_cast<long>(b.live.size()));
    }
    // y pass: the kx tiles t with t * ti <= kmax of each radius
    b.live_y_off.assign(1, 0);
    for (int r = 0; r < b.nr(); ++r) {
      for (long t = 0; t * ti <= b.cut[2 * r + 1]; ++t)
        b.live_y.push_back(static_cast<int32_t>((static_cast<long>(r) << 24) | t));
      b.live_y_off.push_back(static_cast<long>(b.live_y.size()));
    }
  }
  b.bins_live = xs21::bins_live_tiles(n);
  for (long kx = 0; kx < n / 2; ++kx)
    for (long ky = 0; ky < n; ++ky) {
      const long ny = ky < n / 2 ? ky : ky - n;
      b.live_yx += (ny * ny + kx * kx <= static_cast<long>(n / 2) * (n / 2)) ? 1.0 : 0.0;
    }
  b.bintab = xs21::plan::bins(n, n_bins);
  xs21::plan::bin_stats(n, n_bins, box_mpc, b.bintab, b.counts, b.kmean);
  if (on_device) {
    b.dev_src = delta;
  } else {
    const size_t bytes = b.cells() * real_size(dtype);
    try {
      b.host.resize(bytes);
    } catch (...) {
      return fail(XS21_ENOMEM, "host copy of %zu bytes failed", bytes);
    }
    std::memcpy(b.host.data(), delta, bytes);
    if (dtype == XS21_F32) {
      const float* f = static_cast<const float*>(delta);
      for (size_t i = 0; i < b.cells(); ++i)
        if (!std::isfinite(f[i])) return fail(XS21_EINVAL, "non-finite density value at %zu", i);
    } else {
      const double* f = static_cast<const double*>(delta);
      for (size_t i = 0; i < b.cells(); ++i)
        if (!std::isfinite(f[i])) return fail(XS21_EINVAL, "non-finite density value at %zu", i);
    }
  }
  ctx->boxes.push_back(std::move(b));
  *out = static_cast<xs21_box>(ctx->boxes.size() - 1);
  return XS21_OK;
}

xs21_status xs21_box_radii(xs21_ctx* ctx, xs21_box box, double* out, int cap, int* n_radii) {
  g_error.clear();
  if (!ctx || !n_radii) return fail(XS21_EINVAL, "null argument");
  if (xs21_status s = check_box(ctx, box)) return s;
  const auto& r = ctx->boxes[box].radii;
  *n_radii = static_cast<int>(r.size());
  if (out)
    for (int i = 0; i < std::min(cap, *n_radii); ++i) out[i] = r[i];
  return XS21_OK;
}

xs21_status xs21_box_bins(xs21_ctx* ctx, xs21_box box, double* k_mean, double* counts) {
  g_error.clear();
  if (!ctx) return fail(XS21_EINVAL, "null context");
  if (xs21_status s = check_box(ctx, box)) return s;
  const auto& b = ctx->boxes[box];
  if (k_mean) std::copy(b.kmean.begin(), b.kmean.end(), k_mean);
  if (counts) std::copy(b.counts.begin(), b.counts.end(), counts);
  return XS21_OK;
}

xs21_status xs21_workspace_size(xs21_ctx* ctx, xs21_dtype storage, int max_walkers, int max_plain_radii,
                                size_t* bytes) {
  g_error.clear();
  if (!ctx || !bytes) return fail(XS21_EINVAL, "null argument");
  if (ctx->boxes.empty()) return fail(XS21_ESTATE, "no boxes registered");
  if (storage != XS21_F32 && storage != XS21_BF16 && storage != XS21_F64)
    return fail(XS21_EINVAL, "unknown storage type");
  if (max_walkers < 1) return fail(XS21_EINVAL, "max_walkers must be >= 1");
  if (max_plain_radii < 1 || max_plain_radii > xs21::max_radii())
    return fail(XS21_EINVAL, "max_plain_radii must be in [1, %d]", xs21::max_radii());
  for (const auto& b : ctx->boxes)
    if (b.dtype == XS21_F32 && storage == XS21_F64)
      return fail(XS21_EINVAL, "F64 storage needs F64 boxes");
  const int group = std::min(max_walkers, xs21::max_group());
  *bytes = compute_layout(ctx, storage, max_walkers, max_plain_radii, group, ctx->boxes).total;
  return XS21_OK;
}

xs21_status xs21_prepare(xs21_ctx* ctx, void* workspace, size_t bytes, xs21_dtype storage, int max_walkers,
                         int max_plain_radii) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s_ = no_capture(ctx, "xs21_prepare")) return s_;
  if (ctx->prepared) return fail(XS21_ESTATE, "already prepared");
  size_t need = 0;
  if (xs21_status s = xs21_workspace_size(ctx, storage, max_walkers, max_plain_radii, &need)) return s;
  if (!workspace) return fail(XS21_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(XS21_EINVAL, "workspace not 256-byte aligned");
  if (bytes < need) return fail(XS21_ENOMEM, "workspace holds %zu bytes, %zu needed", bytes, need);
  ctx->ws = static_cast<unsigned char*>(workspace);
  ctx->ws_bytes = bytes;
  ctx->storage = storage;
  ctx->max_walkers = max_walkers;
  ctx->max_plain = max_plain_radii;
  ctx->group = std::min(max_walkers, xs21::max_group());
  ctx->lay = compute_layout(ctx, storage, max_walkers, max_plain_radii, ctx->group, ctx->boxes);

  // pinned staging for walker tables
  ctx->pinned_bytes = std::max<size_t>(ctx->lay.tables_bytes, ctx->lay.one_table_bytes);
  HIPCHECK(ctx, hipHostMalloc(&ctx->pinned, ctx->pinned_bytes, hipHostMallocDefault));

  const auto tw = xs21::plan::twiddles(kNtab);
  std::vector<float> tw32(tw.begin(), tw.end());
  HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + ctx->lay.tw32, tw32.data(), tw32.size() * 4, hipMemcpyHostToDevice, ctx->stream));
  HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + ctx->lay.tw64, tw.data(), tw.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  for (auto& b : ctx->boxes) {
    HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_bintab, b.bintab.data(), b.bintab.size(), hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_counts, b.counts.data(), b.nbins * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_cut, b.cut.data(), b.cut.size() * sizeof(long), hipMemcpyHostToDevice,
                                 ctx->stream));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_live, b.live.data(), b.live.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_live_y, b.live_y.data(), b.live_y.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_bins_live, b.bins_live.data(),
                                 b.bins_live.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    {
      const auto slots = xs21::plan::slots2(ctx->phys, b.z, b.radii);
      b.bplan = xs21::plan::box_plan(ctx->phys, b.z, b.nr());
      HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_slots, slots.data(), slots.size() * sizeof(xs21::SlotPlan2),
                                   hipMemcpyHostToDevice, ctx->stream));
      HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));   // `slots` is a host temporary
    }
    const size_t dbytes = b.cells() * real_size(b.dtype);
    if (b.dev_src)
      HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_delta, b.dev_src, dbytes, hipMemcpyDeviceToDevice, ctx->stream));
    else
      HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_delta, b.host.data(), dbytes, hipMemcpyHostToDevice, ctx->stream));
    HIPCHECK(ctx, smooth_box(ctx, ctx->stream, b));
    HIPCHECK(ctx, density_factor(ctx, ctx->stream, b));
  }
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& b : ctx->boxes) {
    std::vector<unsigned char>().swap(b.host);
    b.dev_src = nullptr;
  }
  ctx->prepared = true;
  return XS21_OK;
}

}  // extern "C"

namespace {

// Shared body of xs21_eval_batch (w1) and xs21_eval_batch2 (w2): exactly
// one walker array is non-null.
// field_walker >= 0: the ionisation launch of that walker on boxes[field_box]
// also writes its x_HI and dT_b boxes to fx / fd.
xs21_status eval_batch_impl(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_walker* w1,
                            const xs21_walker2* w2, int nw, double* pk, double* xhi_mean, int field_walker = -1,
                            int field_box = -1, void* fx = nullptr, void* fd = nullptr) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s_ = no_capture(ctx, "evaluation with host-planned walkers (xs21_eval_batch)")) return s_;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (!boxes || nb < 1 || !(w1 || w2) || nw < 1) return fail(XS21_EINVAL, "empty batch");
  if (nb > static_cast<int>(ctx->boxes.size())) return fail(XS21_EINVAL, "more listed boxes than registered");
  int nbmax = 0;
  for (int i = 0; i < nb; ++i) {
    if (xs21_status s = check_box(ctx, boxes[i])) return s;
    if (ctx->boxes[boxes[i]].dtype != ctx->boxes[boxes[0]].dtype)
      return fail(XS21_EINVAL, "boxes of one batch must share a dtype");
    nbmax = std::max(nbmax, ctx->boxes[boxes[i]].nbins);
    for (int k = 0; k < i; ++k)
      if (boxes[k] == boxes[i]) return fail(XS21_EINVAL, "box %d listed twice", boxes[i]);
  }
  for (int w = 0; w < nw; ++w)
    if (w1 ? !xs21::plan::valid_walker(w1[w]) : !xs21::plan::valid_walker2(w2[w]))
      return fail(XS21_EINVAL, "walker %d has invalid parameters", w);
  if (field_walker >= 0 && (field_walker >= nw || field_box < 0 || field_box >= nb || !fx || !fd))
    return fail(XS21_EINVAL, "field walker / box out of range or null field output");
  auto r_mfp = [&](long w) { return w1 ? w1[w].r_mfp : w2[w].r_mfp; };

  const hipStream_t st = ctx->stream;
  const size_t stride = static_cast<size_t>(xs21::thr_stride());
  for (int w0 = 0; w0 < nw; w0 += ctx->max_walkers) {
    const int cnt = std::min(ctx->max_walkers, nw - w0);
    if (ctx->upload_pending) HIPCHECK(ctx, hipEventSynchronize(ctx->upload_done));
    // host planning for every (walker, box) of this chunk
    size_t off = 0;
    std::vector<size_t> boff(nb);
    unsigned char* pin = static_cast<unsigned char*>(ctx->pinned);
    for (int i = 0; i < nb; ++i) {
      const BoxRec& b = ctx->boxes[boxes[i]];
      boff[i] = off;
      if (w1)
        build_tables(ctx->phys, b, w1 + w0, cnt, false, b.radii, pin + off, ctx->max_walkers);
      else
        build_tables2(ctx->phys, b, w2 + w0, cnt, pin + off, ctx->max_walkers);
      off += b.table_bytes(ctx->max_walkers);
    }
    if (w1) {
      HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + ctx->lay.tables, pin, off, hipMemcpyHostToDevice, st));
    } else {
      for (int i = 0; i < nb; ++i)   // only the host-written part of each box's tables
        HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + ctx->lay.tables + boff[i], pin + boff[i],
                                     tab2(ctx->boxes[boxes[i]], ctx->max_walkers).host, hipMemcpyHostToDevice, st));
    }
    HIPCHECK(ctx, hipEventRecord(ctx->upload_done, st));
    ctx->upload_pending = true;
    for (int i = 0; i < nb; ++i) {
      const BoxRec& b = ctx->boxes[boxes[i]];
      const size_t rs = real_size(b.dtype);
      unsigned char* base = ctx->ws + ctx->lay.tables + boff[i];
      const unsigned char* wc = base;
      const unsigned char* thr = wc + align_up(ctx->max_walkers * b.wc_size());
      const unsigned char* zt = nullptr;
      size_t thr_w = stride * rs;   // threshold bytes per walker
      if (w2) {
        const Tab2 t = tab2(b, ctx->max_walkers);
        thr = base + t.thr;
        zt = base + t.zt;
        thr_w = 2 * stride * rs;
        HIPCHECK(ctx, timed(ctx, st, XS21_K_PLAN, 0.0, [&] {
          return xs21::launch_plan2(b.dtype, reinterpret_cast<const xs21::SlotPlan2*>(base + t.slots), b.nr(),
                                    reinterpret_cast<const xs21::WalkerPlan2*>(base + t.wp), cnt, base + t.wc,
                                    base + t.thr, static_cast<int>(stride), base + t.zt, xs21::kZetaPitch,
                                    ctx->phys.delta_c, st);
        }));
      }
      const int G = group_of(ctx, b.n);
      for (int g0 = 0; g0 < cnt; g0 += G) {
        const int g = std::min(G, cnt - g0);
        const long wg = w0 + g0;
        double used = 0;
        for (int k = 0; k < g; ++k) used += b.nr() - first_radius(b, r_mfp(wg + k));
        double* pk_out = pk ? pk + (wg * nb + i) * nbmax : nullptr;
        double* xh_out = xhi_mean ? xhi_mean + wg * nb + i : nullptr;
        const EvalSlot sl = eval_slot(b, ctx->ws + ctx->lay.scratch, g);
        const int fw = (i == field_box && field_walker >= wg && field_walker < wg + g) ? field_walker - wg : -1;
        HIPCHECK(ctx, ion_stage(ctx, st, b, sl, ctx->ws + b.off_dR, b.storage, b.nr(), wc + g0 * b.wc_size(),
                                thr + static_cast<size_t>(g0) * thr_w,
                                zt ? zt + static_cast<size_t>(g0) * xs21::kZetaPitch * rs : nullptr, g, used, fw, fx,
                                fd));
        HIPCHECK(ctx, mem_stage(ctx, st, b, sl, g, pk_out, static_cast<long>(nb) * nbmax, nbmax, xh_out, nb));
      }
    }
  }
  return XS21_OK;
}

}  // namespace

extern "C" {

xs21_status xs21_eval_batch(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_walker* walkers, int nw,
                            double* pk, double* xhi_mean) {
  if (!walkers) return fail(XS21_EINVAL, "null walkers");
  return eval_batch_impl(ctx, boxes, nb, walkers, nullptr, nw, pk, xhi_mean);
}

xs21_status xs21_eval_batch2(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_walker2* walkers, int nw,
                             double* pk, double* xhi_mean) {
  if (!walkers) return fail(XS21_EINVAL, "null walkers");
  return eval_batch_impl(ctx, boxes, nb, nullptr, walkers, nw, pk, xhi_mean);
}

xs21_status xs21_eval_batch_fields(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_walker* walkers, int nw,
                                   double* pk, double* xhi_mean, int field_walker, int field_box, void* x_hi,
                                   void* dtb) {
  if (!walkers) return fail(XS21_EINVAL, "null walkers");
  if (field_walker < 0) return fail(XS21_EINVAL, "field_walker must be >= 0");
  return eval_batch_impl(ctx, boxes, nb, walkers, nullptr, nw, pk, xhi_mean, field_walker, field_box, x_hi, dtb);
}

}  // extern "C"

namespace {

// Evaluation of `cnt` (<= max_walkers) walkers whose parameters are device
// rows par[cnt][d] (d = 3: constant efficiency, d = 5: two populations) on
// the listed boxes, planned on the device: P(k) rows pk[cnt][nb][nbmax] and
// chi2[cnt] summed over the boxes (every box needs a mock).
hipError_t eval_dev(xs21_ctx* ctx, const xs21_box* boxes, int nb, int d, const double* par, int cnt, double* pk,
                    int nbmax, double* chi2) {
  const hipStream_t st = ctx->stream;
  const int stride = xs21::thr_stride();
  const int cap = ctx->max_walkers;
  size_t off = 0;
  for (int i = 0; i < nb; ++i) {
    const BoxRec& b = ctx->boxes[boxes[i]];
    const size_t rs = real_size(b.dtype);
    unsigned char* base = ctx->ws + ctx->lay.tables + off;
    off += b.table_bytes(cap);
    const auto* slots = reinterpret_cast<const xs21::SlotPlan2*>(ctx->ws + b.off_slots);
    unsigned char *wc, *thr, *zt = nullptr;
    size_t thr_w;
    hipError_t e;
    if (d == 3) {
      wc = base;
      thr = base + align_up(cap * b.wc_size());
      thr_w = stride * rs;
      e = timed(ctx, st, XS21_K_PLAN, 0.0,
                [&] { return xs21::launch_plan1(b.dtype, par, cnt, b.bplan, slots, wc, thr, stride, st); });
    } else {
      const Tab2 t = tab2(b, cap);
      wc = base + t.wc;
      thr = base + t.thr;
      zt = base + t.zt;
      thr_w = 2 * stride * rs;
      auto* wp = reinterpret_cast<xs21::WalkerPlan2*>(base + t.wp);
      e = timed(ctx, st, XS21_K_PLAN, 0.0, [&] {
        hipError_t r = xs21::launch_walker2(b.dtype, par, cnt, b.bplan, slots, wc, wp, st);
        if (r != hipSuccess) return r;
        return xs21::launch_plan2(b.dtype, slots, b.nr(), wp, cnt, wc, thr, stride, zt, xs21::kZetaPitch,
                                  ctx->phys.delta_c, st);
      });
    }
    if (e != hipSuccess) return e;
    const int G = group_of(ctx, b.n);
    for (int g0 = 0; g0 < cnt; g0 += G) {
      const int g = std::min(G, cnt - g0);
      const EvalSlot sl = eval_slot(b, ctx->ws + ctx->lay.scratch, g);
      e = ion_stage(ctx, st, b, sl, ctx->ws + b.off_dR, b.storage, b.nr(), wc + g0 * b.wc_size(),
                    thr + static_cast<size_t>(g0) * thr_w,
                    zt ? zt + static_cast<size_t>(g0) * xs21::kZetaPitch * rs : nullptr, g, -1.0);
      if (e != hipSuccess) return e;
      e = mem_stage(ctx, st, b, sl, g, pk + (static_cast<size_t>(g0) * nb + i) * nbmax, static_cast<long>(nb) * nbmax,
                    nbmax, nullptr, 0);
      if (e != hipSuccess) return e;
    }
  }
  for (int i = 0; i < nb; ++i) {
    const BoxRec& b = ctx->boxes[boxes[i]];
    hipError_t e = timed(ctx, st, XS21_K_OTHER, static_cast<double>(cnt) * b.nbins * 16, [&] {
      return xs21::launch_chi2(pk + static_cast<long>(i) * nbmax, static_cast<long>(nb) * nbmax, cnt,
                               reinterpret_cast<const double*>(ctx->ws + b.off_like), b.nbins, chi2, i == 0, st);
    });
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Checks shared by the sampler entry points; fills spec and nbmax.
xs21_status sampler_args(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_sampler* s, int nw,
                         xs21::SamplerSpec* spec, int* nbmax) {
  if (xs21_status r = check_ctx(ctx)) return r;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (!boxes || nb < 1 || !s || nw < 1) return fail(XS21_EINVAL, "empty or null argument");
  if (nb > static_cast<int>(ctx->boxes.size())) return fail(XS21_EINVAL, "more listed boxes than registered");
  *nbmax = 0;
  for (int i = 0; i < nb; ++i) {
    if (xs21_status r = check_box(ctx, boxes[i])) return r;
    if (ctx->boxes[boxes[i]].dtype != ctx->boxes[boxes[0]].dtype)
      return fail(XS21_EINVAL, "boxes of one batch must share a dtype");
    if (!ctx->boxes[boxes[i]].mock_set) return fail(XS21_ESTATE, "box %d has no mock (xs21_set_mock)", boxes[i]);
    for (int k = 0; k < i; ++k)
      if (boxes[k] == boxes[i]) return fail(XS21_EINVAL, "box %d listed twice", boxes[i]);
    *nbmax = std::max(*nbmax, ctx->boxes[boxes[i]].nbins);
  }
  if (s->dim != 3 && s->dim != 5) return fail(XS21_EINVAL, "dim must be 3 or 5");
  if (!(std::isfinite(s->a) && s->a > 1.0)) return fail(XS21_EINVAL, "stretch scale a must be > 1");
  for (int c = 0; c < s->dim; ++c)
    if (!(std::isfinite(s->lo[c]) && std::isfinite(s->hi[c]) && s->lo[c] < s->hi[c]))
      return fail(XS21_EINVAL, "prior bounds of parameter %d are not finite with lo < hi", c);
  // the prior box must lie inside the parameters' valid domain
  bool ok = s->lo[0] > 0.0 && s->lo[1] > 0.0 && s->hi[2] <= 12.0;   // third coordinate: log10 T
  if (s->dim == 5)
    ok = ok && s->hi[0] <= 1e6 && s->lo[2] >= 4.0 && s->hi[2] <= 9.0 && std::fabs(s->lo[3]) <= 10.0 &&
         std::fabs(s->hi[3]) <= 10.0 && std::fabs(s->lo[4]) <= 10.0 && std::fabs(s->hi[4]) <= 10.0;
  if (!ok) return fail(XS21_EINVAL, "prior box leaves the parameters' valid domain");
  std::memset(spec, 0, sizeof *spec);
  for (int c = 0; c < s->dim; ++c) {
    spec->lo[c] = s->lo[c];
    spec->hi[c] = s->hi[c];
  }
  spec->a = s->a;
  spec->d = s->dim;
  return XS21_OK;
}

}  // namespace

extern "C" {

xs21_status xs21_mcmc_lnprob(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_sampler* s, const double* x,
                             int nw, double* lp) {
  g_error.clear();
  xs21::SamplerSpec spec;
  int nbmax = 0;
  if (xs21_status r = sampler_args(ctx, boxes, nb, s, nw, &spec, &nbmax)) return r;
  if (!x || !lp) return fail(XS21_EINVAL, "null argument");
  double* chi2 = reinterpret_cast<double*>(ctx->ws + ctx->lay.samp) + 7 * static_cast<size_t>(ctx->max_walkers);
  double* pk = reinterpret_cast<double*>(ctx->ws + ctx->lay.samp_pk);
  for (int c0 = 0; c0 < nw; c0 += ctx->max_walkers) {
    const int cnt = std::min(ctx->max_walkers, nw - c0);
    const double* xc = x + static_cast<size_t>(c0) * spec.d;
    HIPCHECK(ctx, eval_dev(ctx, boxes, nb, spec.d, xc, cnt, pk, nbmax, chi2));
    HIPCHECK(ctx, timed(ctx, ctx->stream, XS21_K_OTHER, 0.0,
                        [&] { return xs21::launch_lnprob(xc, cnt, spec, chi2, lp + c0, ctx->stream); }));
  }
  return XS21_OK;
}

xs21_status xs21_mcmc_step(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_sampler* s, double* x, double* lp,
                           int nw, const double* u, int32_t* accepted) {
  g_error.clear();
  xs21::SamplerSpec spec;
  int nbmax = 0;
  if (xs21_status r = sampler_args(ctx, boxes, nb, s, nw, &spec, &nbmax)) return r;
  if (!x || !lp || !u) return fail(XS21_EINVAL, "null argument");
  if (nw < 4 || nw % 2) return fail(XS21_EINVAL, "the ensemble needs an even number >= 4 of walkers");
  const size_t cap = static_cast<size_t>(ctx->max_walkers);
  double* prop = reinterpret_cast<double*>(ctx->ws + ctx->lay.samp);
  double* aux = prop + 5 * cap;
  double* chi2 = aux + 2 * cap;
  double* pk = reinterpret_cast<double*>(ctx->ws + ctx->lay.samp_pk);
  const int half = nw / 2;
  for (int h = 0; h < 2; ++h) {
    const double* uh = u + static_cast<size_t>(h) * half * 3;
    for (int c0 = 0; c0 < half; c0 += ctx->max_walkers) {
      const int cnt = std::min(ctx->max_walkers, half - c0);
      const int k0 = h * half + c0;
      HIPCHECK(ctx, timed(ctx, ctx->stream, XS21_K_OTHER, 0.0, [&] {
        return xs21::launch_propose(x, k0, (1 - h) * half, half, cnt, uh + 3 * static_cast<size_t>(c0), spec, prop,
                                    aux, ctx->stream);
      }));
      HIPCHECK(ctx, eval_dev(ctx, boxes, nb, spec.d, prop, cnt, pk, nbmax, chi2));
      HIPCHECK(ctx, timed(ctx, ctx->stream, XS21_K_OTHER, 0.0, [&] {
        return xs21::launch_accept(x, lp, k0, cnt, spec.d, uh + 3 * static_cast<size_t>(c0), prop, aux, chi2,
                                   accepted, ctx->stream);
      }));
    }
  }
  return XS21_OK;
}

xs21_status xs21_eval(xs21_ctx* ctx, xs21_box box, const xs21_walker* walker, const double* radii, int n_radii,
                      void* x_hi, void* dtb, double* pk, double* k_mean, double* counts, double* xhi_mean) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s_ = no_capture(ctx, "xs21_eval")) return s_;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (xs21_status s = check_box(ctx, box)) return s;
  if (!walker || !xs21::plan::valid_walker(*walker)) return fail(XS21_EINVAL, "invalid walker");
  const BoxRec& b = ctx->boxes[box];
  std::vector<double> r;
  if (radii) {
    if (n_radii < 1) return fail(XS21_EINVAL, "n_radii must be >= 1");
    r.assign(radii, radii + n_radii);
    for (int j = 0; j < n_radii; ++j) {
      if (!(std::isfinite(r[j]) && r[j] > 0)) return fail(XS21_EINVAL, "radius %d not finite and > 0", j);
      if (j && !(r[j] < r[j - 1])) return fail(XS21_EINVAL, "radii must decrease");
    }
  } else {
    r = xs21::plan::ladder(walker->r_mfp, b.box / b.n, ctx->phys.radius_step);
  }
  const int nr = static_cast<int>(r.size());
  if (nr > ctx->max_plain) return fail(XS21_ENOMEM, "%d radii exceed max_plain_radii = %d", nr, ctx->max_plain);

  // literal per-walker method: forward FFT and every smoothed box recomputed
  unsigned char* s = ctx->ws + ctx->lay.scratch;
  unsigned char* hat = s;
  unsigned char* tmp = hat + align_up(b.spec_bytes());
  unsigned char* dR = tmp + align_up(b.spec_bytes());
  unsigned char* eval_area = dR + align_up(static_cast<size_t>(ctx->max_plain) * b.cells() * real_size(b.dtype));
  // walker table and the radius cutoffs travel in one upload
  if (ctx->upload_pending) HIPCHECK(ctx, hipEventSynchronize(ctx->upload_done));
  unsigned char* pin = static_cast<unsigned char*>(ctx->pinned);
  build_tables(ctx->phys, b, walker, 1, true, r, pin, 1);
  const size_t tb_bytes = align_up(b.wc_size()) + align_up(xs21::thr_stride() * real_size(b.dtype));
  std::vector<long> cut(2 * nr);
  for (int j = 0; j < nr; ++j) cut_pair(b, r[j], &cut[2 * j]);
  std::memcpy(pin + tb_bytes, cut.data(), cut.size() * sizeof(long));
  unsigned char* wc = ctx->ws + ctx->lay.one_table;
  HIPCHECK(ctx, hipMemcpyAsync(wc, pin, tb_bytes + cut.size() * sizeof(long), hipMemcpyHostToDevice, ctx->stream));
  HIPCHECK(ctx, hipEventRecord(ctx->upload_done, ctx->stream));
  ctx->upload_pending = true;
  const long* cut_dev = reinterpret_cast<const long*>(wc + tb_bytes);
  HIPCHECK(ctx, forward3d(ctx, ctx->stream, b, ctx->ws + b.off_delta, hat));
  for (int j = 0; j < nr; ++j)
    HIPCHECK(ctx, smooth_batch(ctx, ctx->stream, b, hat, tmp, cut_dev + 2 * j, cut.data() + 2 * j, 1, b.dtype,
                               dR + static_cast<size_t>(j) * b.cells() * real_size(b.dtype)));
  const unsigned char* thr = wc + align_up(b.wc_size());

  // the eval scratch of a plain call sits after the plain smoothed boxes; the
  // fields (when asked for) come from the same ionisation launch, staged in
  // the hat / tmp area, which the smoothing no longer needs
  double* outs = reinterpret_cast<double*>(ctx->ws + ctx->lay.outs);
  const EvalSlot sl = eval_slot(b, eval_area, 1);
  const size_t fbytes = b.cells() * real_size(b.dtype);
  if ((x_hi || dtb) && 2 * align_up(fbytes) > 2 * align_up(b.spec_bytes()))
    return fail(XS21_EUNSUPPORTED, "field staging does not fit");
  void* fx = hat;
  void* fd = hat + align_up(fbytes);
  const bool fields = x_hi || dtb;
  HIPCHECK(ctx, ion_stage(ctx, ctx->stream, b, sl, dR, b.dtype, nr, wc, thr, nullptr, 1, nr, fields ? 0 : -1,
                          fields ? fx : nullptr, fields ? fd : nullptr));
  HIPCHECK(ctx, mem_stage(ctx, ctx->stream, b, sl, 1, outs, b.nbins, b.nbins, outs + 128, 1));
  if (x_hi) HIPCHECK(ctx, hipMemcpyAsync(x_hi, fx, fbytes, hipMemcpyDeviceToHost, ctx->stream));
  if (dtb) HIPCHECK(ctx, hipMemcpyAsync(dtb, fd, fbytes, hipMemcpyDeviceToHost, ctx->stream));
  double host_out[129];
  HIPCHECK(ctx, hipMemcpyAsync(host_out, outs, 129 * 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->upload_pending = false;
  if (pk) std::copy(host_out, host_out + b.nbins, pk);
  if (xhi_mean) *xhi_mean = host_out[128];
  if (k_mean) std::copy(b.kmean.begin(), b.kmean.end(), k_mean);
  if (counts) std::copy(b.counts.begin(), b.counts.end(), counts);
  return XS21_OK;
}

xs21_status xs21_materialize(xs21_ctx* ctx, xs21_box box, const xs21_walker* walker, void* x_hi, void* dtb) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s_ = no_capture(ctx, "xs21_materialize")) return s_;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (xs21_status s = check_box(ctx, box)) return s;
  if (!walker || !xs21::plan::valid_walker(*walker)) return fail(XS21_EINVAL, "invalid walker");
  if (!x_hi || !dtb) return fail(XS21_EINVAL, "null field output");
  const BoxRec& b = ctx->boxes[box];
  if (ctx->upload_pending) HIPCHECK(ctx, hipEventSynchronize(ctx->upload_done));
  build_tables(ctx->phys, b, walker, 1, false, b.radii, static_cast<unsigned char*>(ctx->pinned), 1);
  const size_t tb_bytes = align_up(b.wc_size()) + align_up(xs21::thr_stride() * real_size(b.dtype));
  unsigned char* wc = ctx->ws + ctx->lay.one_table;
  HIPCHECK(ctx, hipMemcpyAsync(wc, ctx->pinned, tb_bytes, hipMemcpyHostToDevice, ctx->stream));
  HIPCHECK(ctx, hipEventRecord(ctx->upload_done, ctx->stream));
  ctx->upload_pending = true;
  // the batched ionisation kernel over a group of this one walker, writing its fields
  const EvalSlot sl = eval_slot(b, ctx->ws + ctx->lay.scratch, 1);
  HIPCHECK(ctx, ion_stage(ctx, ctx->stream, b, sl, ctx->ws + b.off_dR, b.storage, b.nr(), wc,
                          wc + align_up(b.wc_size()), nullptr, 1, -1.0, 0, x_hi, dtb));
  return XS21_OK;
}

xs21_status xs21_materialize2(xs21_ctx* ctx, xs21_box box, const xs21_walker2* walker, void* x_hi, void* dtb) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s_ = no_capture(ctx, "xs21_materialize2")) return s_;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (xs21_status s = check_box(ctx, box)) return s;
  if (!walker || !xs21::plan::valid_walker2(*walker)) return fail(XS21_EINVAL, "invalid walker");
  if (!x_hi || !dtb) return fail(XS21_EINVAL, "null field output");
  const BoxRec& b = ctx->boxes[box];
  if (ctx->upload_pending) HIPCHECK(ctx, hipEventSynchronize(ctx->upload_done));
  build_tables2(ctx->phys, b, walker, 1, static_cast<unsigned char*>(ctx->pinned), 1);
  const Tab2 t = tab2(b, 1);
  unsigned char* base = ctx->ws + ctx->lay.one_table;
  HIPCHECK(ctx, hipMemcpyAsync(base, ctx->pinned, t.host, hipMemcpyHostToDevice, ctx->stream));
  HIPCHECK(ctx, hipEventRecord(ctx->upload_done, ctx->stream));
  ctx->upload_pending = true;
  HIPCHECK(ctx, timed(ctx, ctx->stream, XS21_K_PLAN, 0.0, [&] {
    return xs21::launch_plan2(b.dtype, reinterpret_cast<const xs21::SlotPlan2*>(base + t.slots), b.nr(),
                              reinterpret_cast<const xs21::WalkerPlan2*>(base + t.wp), 1, base + t.wc,
                              base + t.thr, xs21::thr_stride(), base + t.zt, xs21::kZetaPitch, ctx->phys.delta_c,
                              ctx->stream);
  }));
  const EvalSlot sl = eval_slot(b, ctx->ws + ctx->lay.scratch, 1);
  HIPCHECK(ctx, ion_stage(ctx, ctx->stream, b, sl, ctx->ws + b.off_dR, b.storage, b.nr(), base + t.wc,
                          base + t.thr, base + t.zt, 1, -1.0, 0, x_hi, dtb));
  return XS21_OK;
}

xs21_status xs21_smoothed(xs21_ctx* ctx, xs21_box box, int index, void* out) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (xs21_status s = check_box(ctx, box)) return s;
  const BoxRec& b = ctx->boxes[box];
  if (index < 0 || index >= b.nr()) return fail(XS21_EINVAL, "radius index %d out of range", index);
  if (!out) return fail(XS21_EINVAL, "null output");
  const void* src = ctx->ws + b.off_dR + static_cast<size_t>(index) * b.cells() * store_size(b.storage);
  HIPCHECK(ctx, xs21::launch_cast(b.dtype, b.storage, src, out, b.cells(), ctx->stream));
  return XS21_OK;
}

}  // extern "C"

namespace {

// Scratch bytes of one P(k) of box b: a padded half spectrum, its Nyquist
// plane and the binning pass's FP64 partial sums.
size_t pk_scratch_bytes(const BoxRec& b) {
  return align_up(b.spec_bytes()) + align_up(nyq_bytes(b)) +
         align_up(static_cast<size_t>(xs21::bins_parts(b.n, 1)) * b.nbins * 8);
}

// Binned P(k) of a device field on box b's geometry into pk_dev (device,
// n_bins doubles), with `scratch` (device, pk_scratch_bytes(b)) for the
// spectrum, Nyquist plane and partial sums; asynchronous on the ctx stream.
hipError_t power_spectrum_into(xs21_ctx* ctx, const BoxRec& b, const void* field, unsigned char* scratch,
                               double* pk_dev) {
  const long n = b.n, hp = static_cast<long>(b.pitch());
  // same layout and passes as one walker's spectrum in an evaluation
  const EvalSlot sl = eval_slot(b, scratch, 1);
  const long parts = xs21::bins_parts(b.n, 1);
  const void* tw = tw_ptr(ctx, b.dtype);
  hipError_t e = xs21::launch_rows_r2c(b.dtype, b.n, field, sl.spec, sl.nyq, n * n, tw, kNtab, ctx->stream);
  if (e == hipSuccess) e = xs21::launch_axis_fwd_disk(b.dtype, b.n, sl.spec, n, hp, n / 2, false, tw, kNtab, ctx->stream);
  if (e == hipSuccess) e = xs21::launch_axis_fwd_disk(b.dtype, b.n, sl.nyq, 1, n, n, true, tw, kNtab, ctx->stream);
  if (e == hipSuccess)
    e = xs21::launch_axis_bins(b.dtype, b.n, sl.spec, sl.nyq, 1, parts,
                               reinterpret_cast<const int32_t*>(ctx->ws + b.off_bins_live),
                               static_cast<long>(b.bins_live.size()),
                               reinterpret_cast<const int8_t*>(ctx->ws + b.off_bintab), b.bintab.data(), b.nbins,
                               sl.part, tw, kNtab, ctx->stream);
  const double L3 = b.box * b.box * b.box;
  if (e == hipSuccess)
    e = xs21::launch_finalize(1, sl.part, parts, b.nbins, nullptr, 0,
                              reinterpret_cast<const double*>(ctx->ws + b.off_counts),
                              L3 / std::pow(static_cast<double>(n), 6), 1.0, pk_dev, b.nbins, b.nbins, nullptr, 0,
                              ctx->stream);
  return e;
}

}  // namespace

extern "C" {

xs21_status xs21_power_spectrum(xs21_ctx* ctx, xs21_box box, const void* field, double* pk) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s_ = no_capture(ctx, "xs21_power_spectrum")) return s_;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (xs21_status s = check_box(ctx, box)) return s;
  if (!field || !pk) return fail(XS21_EINVAL, "null argument");
  const BoxRec& b = ctx->boxes[box];
  double* outs = reinterpret_cast<double*>(ctx->ws + ctx->lay.outs);
  HIPCHECK(ctx, power_spectrum_into(ctx, b, field, ctx->ws + ctx->lay.scratch, outs));
  HIPCHECK(ctx, hipMemcpyAsync(pk, outs, b.nbins * 8, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  return XS21_OK;
}

xs21_status xs21_power_spectrum_static(xs21_ctx* ctx, xs21_box box, const void* field, double* pk_dev) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (xs21_status s = check_box(ctx, box)) return s;
  if (!field || !pk_dev) return fail(XS21_EINVAL, "null argument");
  const BoxRec& b = ctx->boxes[box];
  const size_t need = pk_scratch_bytes(b);
  if (need > xs21::static_scratch_bytes())
    return fail(XS21_EINVAL, "box of %d^3 (%s) needs %zu bytes of scratch; the static scratch holds %zu", b.n,
                b.dtype == XS21_F64 ? "F64" : "F32", need, xs21::static_scratch_bytes());
  unsigned char* scratch = static_cast<unsigned char*>(xs21::static_scratch(ctx->device));
  if (!scratch) return fail(XS21_ESTATE, "static scratch address not set for device %d", ctx->device);
  HIPCHECK(ctx, power_spectrum_into(ctx, b, field, scratch, pk_dev));
  return XS21_OK;
}

xs21_status xs21_probe_bandwidth(xs21_ctx* ctx, int kind, void* buf, size_t bytes, int reps, double* gbps,
                                 double* bytes_per_launch) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s_ = no_capture(ctx, "xs21_probe_bandwidth")) return s_;
  if (kind < 0 || kind > 3) return fail(XS21_EINVAL, "unknown probe kind %d", kind);
  if (!buf || reps < 1 || !gbps) return fail(XS21_EINVAL, "null or empty argument");
  if (reinterpret_cast<uintptr_t>(buf) % kAlign) return fail(XS21_EINVAL, "probe buffer not 256-byte aligned");
  const size_t sink = align_up(xs21::probe_sink_bytes());
  if (bytes < sink + (kind == 3 ? xs21::probe_tile_spectrum_bytes() : (1u << 20)))
    return fail(XS21_EINVAL, "probe buffer of %zu bytes is too small", bytes);
  const size_t body = (bytes - sink) / kAlign * kAlign;
  float* sk = reinterpret_cast<float*>(static_cast<unsigned char*>(buf) + body);
  double moved = 0.0;
  hipEvent_t a = pooled_event(ctx), b = pooled_event(ctx);
  if (!a || !b) return fail(XS21_EDEVICE, "event creation failed");
  HIPCHECK(ctx, xs21::launch_probe(kind, buf, body, sk, &moved, ctx->stream));   // warm-up
  HIPCHECK(ctx, hipEventRecord(a, ctx->stream));
  for (int r = 0; r < reps; ++r) HIPCHECK(ctx, xs21::launch_probe(kind, buf, body, sk, &moved, ctx->stream));
  HIPCHECK(ctx, hipEventRecord(b, ctx->stream));
  HIPCHECK(ctx, hipEventSynchronize(b));
  float ms = 0.f;
  HIPCHECK(ctx, hipEventElapsedTime(&ms, a, b));
  ctx->pool.push_back(a);
  ctx->pool.push_back(b);
  *gbps = moved * reps / (static_cast<double>(ms) * 1e-3) / 1e9;
  if (bytes_per_launch) *bytes_per_launch = moved;
  return XS21_OK;
}

xs21_status xs21_erfc_f32(xs21_ctx* ctx, const float* x, float* y, long n) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (!x || !y || n < 1) return fail(XS21_EINVAL, "null or empty argument");
  HIPCHECK(ctx, xs21::launch_erfc(x, y, static_cast<size_t>(n), ctx->stream));
  return XS21_OK;
}

xs21_status xs21_set_mock(xs21_ctx* ctx, xs21_box box, const double* delta2_mock, const double* noise_sigma,
                          double model_err, double k_lo, double k_hi) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s_ = no_capture(ctx, "xs21_set_mock")) return s_;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (xs21_status s = check_box(ctx, box)) return s;
  if (!delta2_mock) return fail(XS21_EINVAL, "null mock");
  if (!(std::isfinite(model_err) && model_err >= 0)) return fail(XS21_EINVAL, "model_err must be finite and >= 0");
  if (!(std::isfinite(k_lo) && std::isfinite(k_hi) && k_lo >= 0 && k_lo <= k_hi))
    return fail(XS21_EINVAL, "need 0 <= k_lo <= k_hi, finite");
  BoxRec& b = ctx->boxes[box];
  const int nb = b.nbins;
  std::vector<double> tab(3 * static_cast<size_t>(nb));
  for (int i = 0; i < nb; ++i) {
    const double m = delta2_mock[i], sg = noise_sigma ? noise_sigma[i] : 0.0;
    if (!std::isfinite(m) || !std::isfinite(sg)) return fail(XS21_EINVAL, "non-finite mock or noise in bin %d", i);
    const double k = b.kmean[i];
    const bool fitted = b.counts[i] > 0 && k >= k_lo && k <= k_hi;
    constexpr double kPi = 3.14159265358979323846;
    tab[i] = k * k * k / (2.0 * kPi * kPi);
    tab[nb + i] = m;
    tab[2 * nb + i] = fitted ? sg * sg + (model_err * m) * (model_err * m) : 0.0;
  }
  HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_like, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  b.mock_set = true;
  return XS21_OK;
}

xs21_status xs21_chi2(xs21_ctx* ctx, const xs21_box* boxes, int nb, const double* pk, int nw, double* chi2) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (!boxes || nb < 1 || !pk || nw < 1 || !chi2) return fail(XS21_EINVAL, "empty or null argument");
  int nbmax = 0;
  for (int i = 0; i < nb; ++i) {
    if (xs21_status s = check_box(ctx, boxes[i])) return s;
    if (!ctx->boxes[boxes[i]].mock_set) return fail(XS21_ESTATE, "box %d has no mock (xs21_set_mock)", boxes[i]);
    nbmax = std::max(nbmax, ctx->boxes[boxes[i]].nbins);
  }
  for (int i = 0; i < nb; ++i) {
    const BoxRec& b = ctx->boxes[boxes[i]];
    HIPCHECK(ctx, timed(ctx, ctx->stream, XS21_K_OTHER, static_cast<double>(nw) * b.nbins * 16, [&] {
      return xs21::launch_chi2(pk + static_cast<long>(i) * nbmax, static_cast<long>(nb) * nbmax, nw,
                               reinterpret_cast<const double*>(ctx->ws + b.off_like), b.nbins, chi2, i == 0,
                               ctx->stream);
    }));
  }
  return XS21_OK;
}

xs21_status xs21_resmooth(xs21_ctx* ctx, xs21_box box, const void* new_delta) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (xs21_status s = check_box(ctx, box)) return s;
  const BoxRec& b = ctx->boxes[box];
  if (new_delta)
    HIPCHECK(ctx, hipMemcpyAsync(ctx->ws + b.off_delta, new_delta, b.cells() * real_size(b.dtype),
                                 hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHECK(ctx, smooth_box(ctx, ctx->stream, b));
  HIPCHECK(ctx, density_factor(ctx, ctx->stream, b));
  return XS21_OK;
}

xs21_status xs21_profile(xs21_ctx* ctx, int enable) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s_ = no_capture(ctx, "xs21_profile")) return s_;
  if (enable) {
    HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto& r : ctx->pending) {
      ctx->pool.push_back(r.a);
      ctx->pool.push_back(r.b);
    }
    ctx->pending.clear();
    for (int k = 0; k < XS21_K_COUNT; ++k)
      ctx->tot_ms[k] = ctx->tot_bytes[k] = ctx->tot_ops[k] = 0.0, ctx->launches[k] = 0;
  }
  ctx->prof = enable != 0;
  return XS21_OK;
}

xs21_status xs21_profile_read(xs21_ctx* ctx, int kind, double* total_ms, long long* launches, double* bytes,
                              double* ops) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s_ = no_capture(ctx, "xs21_profile_read")) return s_;
  if (kind < 0 || kind >= XS21_K_COUNT) return fail(XS21_EINVAL, "unknown kernel class %d", kind);
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  for (auto& r : ctx->pending) {
    float ms = 0.f;
    HIPCHECK(ctx, hipEventElapsedTime(&ms, r.a, r.b));
    ctx->tot_ms[r.kind] += ms;
    ctx->launches[r.kind] += 1;
    ctx->tot_bytes[r.kind] += r.bytes;
    ctx->tot_ops[r.kind] += r.ops;
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->pending.clear();
  if (total_ms) *total_ms = ctx->tot_ms[kind];
  if (launches) *launches = ctx->launches[kind];
  if (bytes) *bytes = ctx->tot_bytes[kind];
  if (ops) *ops = ctx->tot_ops[kind];
  return XS21_OK;
}

// ------------------------------------------------------------ launch shapes

}  // extern "C"

namespace {

bool valid_tuning(const xs21_tuning& t) {
  return t.ion_blocks >= 0 && t.ion_blocks <= 16384 && t.pipe_blocks >= 0 && t.pipe_blocks <= 65535 &&
         t.bins_blocks >= 0 && t.bins_blocks <= 65535 && t.flag_test >= -1 && t.flag_test <= 1 && t.group >= 0 &&
         t.group <= xs21::max_group();
}

Tune to_tune(const xs21_tuning& t) {
  Tune u;
  u.ion_blocks = t.ion_blocks;
  u.pipe_blocks = t.pipe_blocks;
  u.bins_blocks = t.bins_blocks;
  u.flag_test = t.flag_test;
  u.group = t.group;
  return u;
}

xs21_tuning from_tune(const Tune& u) {
  xs21_tuning t;
  t.ion_blocks = u.ion_blocks;
  t.pipe_blocks = u.pipe_blocks;
  t.bins_blocks = u.bins_blocks;
  t.flag_test = u.flag_test;
  t.group = u.group;
  return t;
}

const char* dtype_name(int d) { return d == xs21::kF64 ? "f64" : (d == xs21::kBF16 ? "bf16" : "f32"); }

// Entries of a tuning cache file: one line per key, "key": {...}.
std::map<std::string, std::string> read_cache(const char* path) {
  std::map<std::string, std::string> out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  char line[1024];
  while (std::fgets(line, sizeof line, f)) {
    const char* q0 = std::strchr(line, '"');
    if (!q0) continue;
    const char* q1 = std::strchr(q0 + 1, '"');
    const char* brace = q1 ? std::strchr(q1, '{') : nullptr;
    const char* end = brace ? std::strchr(brace, '}') : nullptr;
    if (!end) continue;
    out[std::string(q0 + 1, q1)] = std::string(brace, end + 1);
  }
  std::fclose(f);
  return out;
}

bool parse_entry(const std::string& obj, Tune* t, double* ms) {
  const auto field = [&](const char* name, double* v) {
    const std::string key = std::string("\"") + name + "\":";
    const size_t at = obj.find(key);
    if (at == std::string::npos) return false;
    return std::sscanf(obj.c_str() + at + key.size(), "%lf", v) == 1;
  };
  double a, b, c, d, e, m = -1.0;
  if (!(field("ion_blocks", &a) && field("pipe_blocks", &b) && field("bins_blocks", &c) && field("flag_test", &d) &&
        field("group", &e)))
    return false;
  (void)field("ms", &m);
  t->ion_blocks = static_cast<int>(a);
  t->pipe_blocks = static_cast<int>(b);
  t->bins_blocks = static_cast<int>(c);
  t->flag_test = static_cast<int>(d);
  t->group = static_cast<int>(e);
  *ms = m;
  return true;
}

bool write_cache(const char* path, const std::map<std::string, std::string>& entries) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : entries)
    std::fprintf(f, "\"%s\": %s%s\n", kv.first.c_str(), kv.second.c_str(), ++i < entries.size() ? "," : "");
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" {

xs21_status xs21_set_tuning(xs21_ctx* ctx, int n, const xs21_tuning* t) {
  g_error.clear();
  if (!ctx) return fail(XS21_EINVAL, "null context");
  if (!pow2_in_range(n)) return fail(XS21_EINVAL, "n = %d is not a power of two in [8, 512]", n);
  if (!t) {
    ctx->tune.erase(n);
    return XS21_OK;
  }
  if (!valid_tuning(*t)) return fail(XS21_EINVAL, "tuning values out of range");
  ctx->tune[n] = to_tune(*t);
  return XS21_OK;
}

xs21_status xs21_get_tuning(xs21_ctx* ctx, int n, xs21_tuning* t) {
  g_error.clear();
  if (!ctx || !t) return fail(XS21_EINVAL, "null argument");
  if (!pow2_in_range(n)) return fail(XS21_EINVAL, "n = %d is not a power of two in [8, 512]", n);
  *t = from_tune(tune_of(ctx, n));
  return XS21_OK;
}

xs21_status xs21_autotune(xs21_ctx* ctx, const xs21_box* boxes, int nb, const xs21_walker* walkers, int nw, int reps,
                          const char* cache_path, xs21_tuning* chosen, double* best_ms, int* from_cache) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (xs21_status s = no_capture(ctx, "xs21_autotune")) return s;
  if (!ctx->prepared) return fail(XS21_ESTATE, "xs21_prepare has not run");
  if (!boxes || nb < 1 || !walkers || nw < 1 || reps < 1) return fail(XS21_EINVAL, "empty or null argument");
  int n = 0, nr = 0;
  for (int i = 0; i < nb; ++i) {
    if (xs21_status s = check_box(ctx, boxes[i])) return s;
    const BoxRec& b = ctx->boxes[boxes[i]];
    if (i && b.n != n) return fail(XS21_EINVAL, "boxes tuned together must share their grid size");
    n = b.n;
    nr = std::max(nr, b.nr());
  }
  const BoxRec& b0 = ctx->boxes[boxes[0]];
  hipDeviceProp_t prop;
  HIPCHECK(ctx, hipGetDeviceProperties(&prop, ctx->device));
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  char key[256];
  std::snprintf(key, sizeof key, "%s|n=%d|%s|%s|nr=%d|g=%d", arch.c_str(), n, dtype_name(b0.dtype),
                dtype_name(b0.storage), nr, std::min(nw, ctx->group));
  std::map<std::string, std::string> cache;
  if (cache_path) {
    cache = read_cache(cache_path);
    const auto it = cache.find(key);
    Tune t;
    double ms = -1.0;
    if (it != cache.end() && parse_entry(it->second, &t, &ms) && valid_tuning(from_tune(t))) {
      ctx->tune[n] = t;
      if (chosen) *chosen = from_tune(t);
      if (best_ms) *best_ms = ms;
      if (from_cache) *from_cache = 1;
      return XS21_OK;
    }
  }
  // time eval_batch over the listed boxes for one setting (best of reps, after a warm-up)
  hipEvent_t ea = pooled_event(ctx), eb = pooled_event(ctx);
  if (!ea || !eb) return fail(XS21_EDEVICE, "event creation failed");
  xs21_status err = XS21_OK;
  const auto time_cfg = [&](const Tune& t) {
    ctx->tune[n] = t;
    double best = 1e300;
    for (int r = 0; r <= reps && err == XS21_OK; ++r) {
      hipError_t e = hipEventRecord(ea, ctx->stream);
      if (e == hipSuccess) err = eval_batch_impl(ctx, boxes, nb, walkers, nullptr, nw, nullptr, nullptr);
      if (err != XS21_OK) break;
      if (e == hipSuccess) e = hipEventRecord(eb, ctx->stream);
      if (e == hipSuccess) e = hipEventSynchronize(eb);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ea, eb);
      if (e != hipSuccess) {
        err = hip_fail(ctx, e, "autotune timing");
        break;
      }
      if (r > 0) best = std::min(best, static_cast<double>(ms));
    }
    return best;
  };
  // coordinate descent from the defaults, one knob at a time; a change must
  // win by more than 1 % (timing noise)
  const int cells2 = n * n / 2;
  Tune best;
  best.ion_blocks = xs21::ion_grid(n);
  best.pipe_blocks = 2048;
  best.bins_blocks = 2048;
  best.flag_test = b0.dtype == xs21::kF32 ? 1 : 0;
  best.group = ctx->group;
  double best_t = time_cfg(best);
  const auto trial = [&](Tune t) {
    if (err != XS21_OK) return;
    const double ms = time_cfg(t);
    if (err == XS21_OK && ms < 0.99 * best_t) {
      best = t;
      best_t = ms;
    }
  };
  if (b0.dtype == xs21::kF32) {
    Tune t = best;
    t.flag_test = 0;
    trial(t);
  }
  for (int v : {2048, 4096, 8192, 16384}) {
    if (v == best.ion_blocks || v > cells2) continue;
    Tune t = best;
    t.ion_blocks = v;
    trial(t);
  }
  for (int v : {32, 48}) {
    if (v >= ctx->group || v >= nw) continue;
    Tune t = best;
    t.group = v;
    trial(t);
  }
  for (int v : {1024, 4096}) {
    Tune t = best;
    t.pipe_blocks = v;
    trial(t);
  }
  for (int v : {1024, 4096, 8192}) {
    Tune t = best;
    t.bins_blocks = v;
    trial(t);
  }
  ctx->pool.push_back(ea);
  ctx->pool.push_back(eb);
  if (err != XS21_OK) return err;
  ctx->tune[n] = best;
  if (chosen) *chosen = from_tune(best);
  if (best_ms) *best_ms = best_t;
  if (from_cache) *from_cache = 0;
  if (cache_path) {
    char obj[256];
    std::snprintf(obj, sizeof obj,
                  "{\"ion_blocks\": %d, \"pipe_blocks\": %d, \"bins_blocks\": %d, \"flag_test\": %d, "
                  "\"group\": %d, \"ms\": %.4f}",
                  best.ion_blocks, best.pipe_blocks, best.bins_blocks, best.flag_test, best.group, best_t);
    cache[key] = obj;
    if (!write_cache(cache_path, cache)) return fail(XS21_EINVAL, "cannot write the tuning cache %s", cache_path);
  }
  return XS21_OK;
}

// ------------------------------------------------------------ graph capture

xs21_status xs21_capture_begin(xs21_ctx* ctx) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (ctx->capturing) return fail(XS21_ESTATE, "already capturing");
  if (!ctx->stream) return fail(XS21_EINVAL, "graph capture needs a context on a created stream, not the null stream");
  if (ctx->prof) return fail(XS21_ESTATE, "kernel timing (xs21_profile) is on");
  if (ctx->upload_pending) {
    HIPCHECK(ctx, hipEventSynchronize(ctx->upload_done));
    ctx->upload_pending = false;
  }
  HIPCHECK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  ctx->capturing = true;
  return XS21_OK;
}

xs21_status xs21_capture_end(xs21_ctx* ctx, xs21_graph** out) {
  g_error.clear();
  if (!ctx || !out) return fail(XS21_EINVAL, "null argument");
  if (!ctx->capturing) return fail(XS21_ESTATE, "not capturing");
  *out = nullptr;
  (void)hipSetDevice(ctx->device);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(ctx->stream, &g);
  ctx->capturing = false;
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
  auto* gr = new (std::nothrow) xs21_graph;
  if (!gr) {
    (void)hipGraphDestroy(g);
    return fail(XS21_ENOMEM, "host allocation failed");
  }
  gr->graph = g;
  gr->device = ctx->device;
  const hipError_t e2 = hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    (void)hipGraphDestroy(g);
    delete gr;
    return hip_fail(ctx, e2, "hipGraphInstantiate");
  }
  *out = gr;
  return XS21_OK;
}

xs21_status xs21_graph_launch(xs21_ctx* ctx, const xs21_graph* g) {
  g_error.clear();
  if (xs21_status s = check_ctx(ctx)) return s;
  if (!g) return fail(XS21_EINVAL, "null graph");
  if (ctx->capturing) return fail(XS21_ESTATE, "cannot launch a graph while capturing");
  if (g->device != ctx->device) return fail(XS21_EINVAL, "graph was captured on device %d", g->device);
  HIPCHECK(ctx, hipGraphLaunch(g->exec, ctx->stream));
  return XS21_OK;
}

xs21_status xs21_graph_destroy(xs21_graph* g) {
  g_error.clear();
  if (!g) return XS21_OK;
  (void)hipSetDevice(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return XS21_OK;
}

// ------------------------------------------------------------ host planning

xs21_status xs21_plan_ladder(double r_top, double r_cell, double step, double* out, int cap, int* n_radii) {
  g_error.clear();
  if (!n_radii) return fail(XS21_EINVAL, "null argument");
  if (!(std::isfinite(r_top) && r_top > 0 && std::isfinite(r_cell) && r_cell > 0 && std::isfinite(step) && step > 1))
    return fail(XS21_EINVAL, "invalid ladder parameters");
  const auto r = xs21::plan::ladder(r_top, r_cell, step);
  *n_radii = static_cast<int>(r.size());
  if (out)
    for (int i = 0; i < std::min(cap, *n_radii); ++i) out[i] = r[i];
  return XS21_OK;
}

xs21_status xs21_plan_sigma2(const xs21_physics* phys, double radius, double z, double* out) {
  g_error.clear();
  if (!phys || !out) return fail(XS21_EINVAL, "null argument");
  if (!xs21::plan::valid_physics(*phys)) return fail(XS21_EINVAL, "invalid physics constants");
  if (!(std::isfinite(radius) && radius > 0 && std::isfinite(z) && z > -1)) return fail(XS21_EINVAL, "invalid R or z");
  *out = xs21::plan::sigma2(*phys, radius, z);
  return XS21_OK;
}

xs21_status xs21_plan_walker(const xs21_physics* phys, double z, const double* radii, int n_radii,
                             const xs21_walker* walker, double* thr, double* dsig2, int* first, double* m_min) {
  g_error.clear();
  if (!phys || !radii || !walker) return fail(XS21_EINVAL, "null argument");
  if (!xs21::plan::valid_physics(*phys)) return fail(XS21_EINVAL, "invalid physics constants");
  if (!xs21::plan::valid_walker(*walker)) return fail(XS21_EINVAL, "invalid walker");
  if (n_radii < 1 || !(std::isfinite(z) && z > -1)) return fail(XS21_EINVAL, "invalid radii count or z");
  const auto wp = xs21::plan::walker(*phys, z, radii, n_radii, *walker);
  if (thr) std::copy(wp.thr.begin(), wp.thr.end(), thr);
  if (dsig2) std::copy(wp.dsig2.begin(), wp.dsig2.end(), dsig2);
  if (first) *first = wp.first;
  if (m_min) *m_min = wp.m_min;
  return XS21_OK;
}

xs21_status xs21_plan_bins(int n, int n_bins, int8_t* out) {
  g_error.clear();
  if (!out) return fail(XS21_EINVAL, "null argument");
  if (!pow2_in_range(n)) return fail(XS21_EINVAL, "n = %d is not a power of two in [8, 512]", n);
  if (n_bins < 1 || n_bins > xs21::max_bins()) return fail(XS21_EINVAL, "n_bins out of range");
  const auto t = xs21::plan::bins(n, n_bins);
  std::copy(t.begin(), t.end(), out);
  return XS21_OK;
}

}  // extern "C"
