// gfx950 kernels of the excursion-set path and their host-side launchers.
//
// Data layout (all C order, last axis contiguous):
//   real box        [z][y][x]                       N^3
//   half spectrum   [z][y][kx], kx in [0, N/2]      N * N * HP complex, rows padded
//                   to HP = N/2 + 1 rounded up to 16 (128-byte aligned rows)
//   smoothed boxes  [radius][z][y][x]               N_R * N^3 (storage type S)
//   walker spectra  [walker][z][y][kx]
//
// A 3D real-to-complex transform is three passes: rows along x (two real rows
// packed as one complex row), then the y axis, then the z axis.  The inverse
// runs z, y, then x.  The per-cell ionisation pass is fused into the x pass of
// the forward transform of dT_b, and the |X|^2 binning into its z pass.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>
#include <utility>

#include "common.hpp"
#include "fft.hpp"
#include "launch.hpp"
#include "wave.hpp"

namespace xs21 {

constexpr int kMaxGroup = 64;   // walkers per ionisation launch (x_HI sums in LDS)
constexpr int kNrMax = 40;      // radii held in registers per cell
constexpr int kMaxBins = 64;

// Row pitch of a half spectrum: N/2 + 1 complex values padded to a multiple of
// 16 (128 bytes in FP32), so that strided passes read whole aligned lines.
template <int N>
struct Half {
  static constexpr int H = N / 2 + 1;
  static constexpr int HP = (H + 15) / 16 * 16;
};

template <int N>
struct RowShape {
  static constexpr int WB = FftShape<N>::RMAX;  // sequences per LDS batch
  static constexpr int TS = FftShape<N>::TS;
  static constexpr int NT = N;                  // threads per block
  static constexpr int H = Half<N>::H;
  static constexpr int HP = Half<N>::HP;
};

template <int N>
struct AxisShape {
  static constexpr int TS = FftShape<N>::TS;
  static constexpr int TI = (TS == 1) ? 64 : (N <= 128 ? 32 : 16);  // columns per tile
  static constexpr int NT = TI * TS;
};

__device__ __forceinline__ float erfc_t(float x) { return erfc_fast(x); }
__device__ __forceinline__ double erfc_t(double x) { return erfc(x); }

// ---------------------------------------------------------------------------
// Row packing: two real rows a, b as z = a + i b, and back.
// ---------------------------------------------------------------------------

// From Z = DFT(a + i b) recover the half spectra A[k], B[k], k in [0, N/2]:
// A = (Z[k] + conj Z[N-k]) / 2,  B = (Z[k] - conj Z[N-k]) / (2 i).
template <int N, typename T>
__device__ __forceinline__ void unpack_pair(const cplx<T>* z, int k, cplx<T>& A, cplx<T>& B) {
  const cplx<T> zk = z[k];
  const cplx<T> zm = z[(N - k) & (N - 1)];
  const T h = T(0.5);
  A = {h * (zk.x + zm.x), h * (zk.y - zm.y)};
  B = {h * (zk.y + zm.y), h * (zm.x - zk.x)};
}

// Z[k] = A[k] + i B[k] over the full length from the half spectra of two real
// rows (Hermitian extension; DC and Nyquist taken as real).
// Entries with index above kmax are known to be zero and are not read.
template <int N, typename T>
__device__ __forceinline__ cplx<T> pack_pair(const cplx<T>* __restrict__ ra, const cplx<T>* __restrict__ rb, int k,
                                             int kmax) {
  cplx<T> A = {T(0), T(0)}, B = {T(0), T(0)};
  const int idx = k <= N / 2 ? k : N - k;
  if (idx <= kmax) {
    A = ra[idx];
    B = rb[idx];
    if (k == 0 || k == N / 2) {
      A.y = T(0);
      B.y = T(0);
    } else if (k > N / 2) {
      A = cconj(A);
      B = cconj(B);
    }
  }
  return {A.x - B.y, A.y + B.x};
}

// ---------------------------------------------------------------------------
// Forward rows: real [rows][N] -> half spectra [rows][N/2+1]
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ __launch_bounds__(RowShape<N>::NT) void k_rows_r2c(const T* __restrict__ in, cplx<T>* __restrict__ out,
                                                              long npairs, const cplx<T>* __restrict__ tw,
                                                              int tstride) {
  using S = RowShape<N>;
  __shared__ cplx<T> lds[S::WB * N];
  __shared__ cplx<T> twl[N];
  const int t = threadIdx.x;
  load_twiddles<N>(twl, tw, tstride);
  for (long g = blockIdx.x; g * S::WB < npairs; g += gridDim.x) {
    const long p0 = g * S::WB;
#pragma unroll
    for (int q = 0; q < S::WB; ++q) {
      const long p = p0 + q;
      cplx<T> v = {T(0), T(0)};
      if (p < npairs) v = {in[(2 * p) * N + t], in[(2 * p + 1) * N + t]};
      lds[q * N + t] = v;
    }
    __syncthreads();
    fft_team<N, -1, T>(lds + (t / S::TS) * N, 1, t % S::TS, twl, 1);
    for (int idx = t; idx < S::WB * S::H; idx += S::NT) {
      const int q = idx / S::H, k = idx % S::H;
      const long p = p0 + q;
      if (p < npairs) {
        cplx<T> A, B;
        unpack_pair<N>(lds + q * N, k, A, B);
        out[(2 * p) * S::HP + k] = A;
        out[(2 * p + 1) * S::HP + k] = B;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Inverse rows: half spectra [rows][N/2+1] -> real [rows][N] * scale, stored as S
// ---------------------------------------------------------------------------
template <typename T, typename ST, int N>
__global__ __launch_bounds__(RowShape<N>::NT) void k_rows_c2r(const cplx<T>* __restrict__ in, ST* __restrict__ out,
                                                              long npairs, T scale, int kmax,
                                                              const cplx<T>* __restrict__ tw, int tstride) {
  using S = RowShape<N>;
  __shared__ cplx<T> lds[S::WB * N];
  __shared__ cplx<T> twl[N];
  const int t = threadIdx.x;
  load_twiddles<N>(twl, tw, tstride);
  for (long g = blockIdx.x; g * S::WB < npairs; g += gridDim.x) {
    const long p0 = g * S::WB;
#pragma unroll
    for (int q = 0; q < S::WB; ++q) {
      const long p = p0 + q;
      cplx<T> v = {T(0), T(0)};
      if (p < npairs) v = pack_pair<N>(in + (2 * p) * S::HP, in + (2 * p + 1) * S::HP, t, kmax);
      lds[q * N + t] = v;
    }
    __syncthreads();
    fft_team<N, +1, T>(lds + (t / S::TS) * N, 1, t % S::TS, twl, 1);
#pragma unroll
    for (int q = 0; q < S::WB; ++q) {
      const long p = p0 + q;
      if (p < npairs) {
        const cplx<T> v = lds[q * N + t];
        store_as(out, (2 * p) * N + t, v.x * scale);
        store_as(out, (2 * p + 1) * N + t, v.y * scale);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Strided axis: data [outer][N][inner], transform along the middle axis, for
// the columns i < ilim of each outer slice.
// MODE 0: plain.
// MODE 1: z pass of a sharp-k smoothing (inner index i = y * (N/2+1) + kx):
//   modes with |n|^2 > n2max are zeroed on load; tiles whose columns all lie
//   outside the disk ny^2 + kx^2 <= n2max are skipped, and only columns inside
//   it are stored (every other column is zero after this pass).
// MODE 2: y pass of a smoothing (inner index = kx): an entry is read only if
//   ny^2 + kx^2 <= n2max, the rest is known to be zero.
// ---------------------------------------------------------------------------
// |n|^2 without the z part of flat column i = y * HP + kx of a padded half
// spectrum; padding columns (kx > N/2) get a value above every cutoff.
template <int N>
__device__ __forceinline__ long column_n2(long i) {
  const long ky = i / Half<N>::HP, kx = i % Half<N>::HP;
  const long ny = ky < N / 2 ? ky : ky - N;
  return kx < Half<N>::H ? ny * ny + kx * kx : 0x7fffffffffffL;
}

template <typename T, int N, int DIR, int MODE>
__global__ __launch_bounds__(AxisShape<N>::NT) void k_axis(const cplx<T>* src, cplx<T>* dst, long inner, long ilim,
                                                           long n2max, const cplx<T>* __restrict__ tw, int tstride) {
  using A = AxisShape<N>;
  __shared__ cplx<T> lds[N * A::TI];
  __shared__ cplx<T> twl[N];
  const int t = threadIdx.x;
  const long base = static_cast<long>(blockIdx.y) * N * inner;
  const long i0 = static_cast<long>(blockIdx.x) * A::TI;
  if constexpr (MODE == 1) {
    bool any = false;  // block-uniform
    for (int c = 0; c < A::TI; ++c) any |= (i0 + c < ilim) && column_n2<N>(i0 + c) <= n2max;
    if (!any) return;
  }
  for (int m = t; m < N; m += A::NT) twl[m] = tw[m * tstride];
  for (int l = t; l < N * A::TI; l += A::NT) {
    const int n = l / A::TI, c = l % A::TI;
    const long i = i0 + c;
    cplx<T> v = {T(0), T(0)};
    if (i < ilim) {
      const long nn = n < N / 2 ? n : n - N;
      bool live = true;
      if constexpr (MODE == 1) live = column_n2<N>(i) + nn * nn <= n2max;
      if constexpr (MODE == 2) live = nn * nn + i * i <= n2max;
      if (live) v = src[base + n * inner + i];
    }
    lds[l] = v;
  }
  __syncthreads();
  fft_team<N, DIR, T>(lds + (t % A::TI), A::TI, t / A::TI, twl, 1);
  for (int l = t; l < N * A::TI; l += A::NT) {
    const int n = l / A::TI, c = l % A::TI;
    const long i = i0 + c;
    bool keep = i < ilim;
    if constexpr (MODE == 1) keep = keep && column_n2<N>(i) <= n2max;
    if (keep) dst[base + n * inner + i] = lds[l];
  }
}

// ---------------------------------------------------------------------------
// Forward z pass fused with |X|^2 binning.  src [outer][N][inner] holds the
// x- and y-transformed spectra (inner = y * (N/2+1) + kx); each block writes
// FP64 bin sums of w |X|^2 for its tile to part[outer][tile][nbins].
// Weights w: 1 on the kx = 0 and kx = N/2 planes, 2 elsewhere (half spectrum).
// ---------------------------------------------------------------------------
template <typename T, int N>
__global__ __launch_bounds__(AxisShape<N>::NT) void k_axis_bins(const cplx<T>* __restrict__ src, long inner,
                                                                const int8_t* __restrict__ bintab, int nbins,
                                                                double* __restrict__ part,
                                                                const cplx<T>* __restrict__ tw, int tstride) {
  using A = AxisShape<N>;
  constexpr int H = Half<N>::H, HP = Half<N>::HP;
  constexpr int M = N / A::TS;           // contiguous outputs per thread
  constexpr int NW = A::NT / 64;         // waves per block
  __shared__ cplx<T> lds[N * A::TI];
  __shared__ cplx<T> twl[N];
  __shared__ double wacc[NW][kMaxBins];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const long base = static_cast<long>(blockIdx.y) * N * inner;
  const long i0 = static_cast<long>(blockIdx.x) * A::TI;
  for (int m = t; m < N; m += A::NT) twl[m] = tw[m * tstride];
  for (int b = lane; b < nbins; b += 64) wacc[wave][b] = 0.0;
  for (int l = t; l < N * A::TI; l += A::NT) {
    const int n = l / A::TI, c = l % A::TI;
    const long i = i0 + c;
    lds[l] = (i < inner && i % HP < H) ? src[base + n * inner + i] : cplx<T>{T(0), T(0)};
  }
  __syncthreads();
  const int c = t % A::TI, j = t / A::TI;
  fft_team<N, -1, T>(lds + c, A::TI, j, twl, 1);

  const long i = i0 + c;
  int bin[M];
  T val[M];
  int bmin = kMaxBins, bmax = -1;
  {
    const int ky = static_cast<int>(i / HP), kx = static_cast<int>(i % HP);
    const long ny = ky < N / 2 ? ky : ky - N;
    const long cyx = ny * ny + static_cast<long>(kx) * kx;
    const T w = (kx == 0 || kx == N / 2) ? T(1) : T(2);
    const bool col = i < inner && kx < H;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int kz = j * M + m;
      const long nz = kz < N / 2 ? kz : kz - N;
      const cplx<T> x = lds[kz * A::TI + c];
      int b = -1;
      if (col) b = bintab[nz * nz + cyx];
      bin[m] = b;
      val[m] = w * (x.x * x.x + x.y * x.y);
      if (b >= 0) {
        bmin = min(bmin, b);
        bmax = max(bmax, b);
      }
    }
  }
  bmin = wave_min(bmin);
  bmax = wave_max(bmax);
  for (int b = bmin; b <= bmax; ++b) {
    T s = T(0);
#pragma unroll
    for (int m = 0; m < M; ++m) s += bin[m] == b ? val[m] : T(0);
    const T d = wave_sum(s);
    if (lane == 0) wacc[wave][b] += static_cast<double>(d);
  }
  __syncthreads();
  const long tile = static_cast<long>(blockIdx.y) * gridDim.x + blockIdx.x;
  for (int b = t; b < nbins; b += A::NT) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += wacc[w][b];
    part[tile * nbins + b] = s;
  }
}

// ---------------------------------------------------------------------------
// Per-cell ionisation (Section 2.1, eq. 1 and partial ionisation).
// d[j] = delta_R at radius j of the ladder (decreasing R), cell = delta at the
// cell radius.  Flag iff delta_R >= thr[j] for some j: thresholds are the
// FP64-planned exact rewrite of zeta f_coll >= 1, padded with +inf to kNrMax
// entries (radii above the walker's R_mfp and past the ladder end), so the
// test is branch-free and its uniform threshold loads batch into wide scalar
// loads.  Unflagged cells keep x_HI = 1 - zeta erfc(a_cell (delta_c - delta_cell)).
// ---------------------------------------------------------------------------
template <typename T, int NR>
__device__ __forceinline__ T cell_xhi(const T (&d)[NR], T cell, int nr, const WalkerConst<T>& c,
                                      const T* __restrict__ thr_w, T dc) {
  // OR over radii as wave-wide lane masks: one compare into a scalar mask per
  // radius.  Radii before the walker's first are skipped by uniform branches;
  // their thresholds, like those past the ladder end, are +inf, so the result
  // does not depend on the skipping.
  T th[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) th[j] = thr_w[j];
  // blocks of 8 radii that lie wholly before the walker's first radius or
  // past the ladder end are skipped (one uniform branch per block); inside a
  // block every radius is tested, the +inf thresholds making the extra ones
  // irrelevant
  unsigned long long m = 0;
  const int first = c.first;
#pragma unroll
  for (int g = 0; g < NR; g += 8) {
    if (first < g + 8 && g < nr) {
#pragma unroll
      for (int j = g; j < g + 8 && j < NR; ++j) m |= __ballot(d[j] >= th[j]);
    }
  }
  const bool flag = (m >> __lane_id()) & 1ull;
  T x = T(1);
  if (flag) {
    x = T(0);
  } else if (c.partial) {
    x = T(1) - c.zeta * erfc_t(c.a_cell * (dc - cell));
  }
  return x;
}

template <typename T, typename S, int NR>
__device__ __forceinline__ void load_radii(const S* __restrict__ dR, size_t n3, size_t cell, int nr, T (&d)[NR],
                                           T& dcell) {
  dcell = T(0);
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    d[j] = T(0);
    if (j < nr) {
      d[j] = load_as<T>(dR, j * n3 + cell);
      if (j == nr - 1) dcell = d[j];
    }
  }
}

// Threads and LDS batches of the ionisation pass: one cell per thread over a
// row pair (2N cells), FFT teams of TS threads, WB walkers per LDS batch.
template <int N>
struct IonPlan {
  using type = FftPlan<N>;
};
template <>
struct IonPlan<128> {
  using type = Radices<8, 4, 4>;
};
template <>
struct IonPlan<256> {
  using type = Radices<8, 8, 4>;
};

template <int N>
struct IonShape {
  using Plan = typename IonPlan<N>::type;
  static constexpr int NT = 2 * N;
  static constexpr int TS = FftShape<N, Plan>::TS;
  static constexpr int WB = NT / TS;
  static constexpr int H = Half<N>::H;
  static constexpr int HP = Half<N>::HP;
  static constexpr int NW = NT >= 64 ? NT / 64 : 1;   // waves per block
};

// Ionisation + brightness temperature + forward x pass for a group of walkers.
// Each block owns row pairs (rows 2p, 2p+1 of the z-y plane stack); thread t
// owns cell (row 2p + t / N, x = t % N).  The smoothed values of its cell stay
// in registers while every walker of the group is processed, so the resident
// smoothed boxes are read once per group.  Two real rows are transformed as
// one complex row.  Output: spec[w][row][kx] for w < nw, and per-block x_HI
// sums xpart[w][block].
template <typename T, typename S, int N>
__global__ __launch_bounds__(IonShape<N>::NT) void k_ion_rows(
    const S* __restrict__ dR, const T* __restrict__ delta, int nr, const WalkerConst<T>* __restrict__ wc,
    const T* __restrict__ thr, int nw, T tb, T dc, cplx<T>* __restrict__ spec, double* __restrict__ xpart,
    const cplx<T>* __restrict__ tw, int tstride) {
  using IS = IonShape<N>;
  constexpr size_t N3 = static_cast<size_t>(N) * N * N;
  constexpr size_t SPEC = static_cast<size_t>(N) * N * IS::HP;
  __shared__ cplx<T> lds[IS::WB * N];
  __shared__ cplx<T> twl[N];
  __shared__ T wsum[IS::WB][IS::NT >= 64 ? IS::NW : IS::NT];
  __shared__ double acc[kMaxGroup];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int row = t / N, x = t % N;
  T* ldsr = reinterpret_cast<T*>(lds);
  for (int w = t; w < kMaxGroup; w += IS::NT) acc[w] = 0.0;
  load_twiddles<N>(twl, tw, tstride);
  for (long p = blockIdx.x; p < static_cast<long>(N) * N / 2; p += gridDim.x) {
    const size_t cell = static_cast<size_t>(2 * p + row) * N + x;
    T d[kNrMax];
    T dcell;
    load_radii<T, S>(dR, N3, cell, nr, d, dcell);
    const T od = T(1) + delta[cell];
    for (int w0 = 0; w0 < nw; w0 += IS::WB) {
      const int qn = min(IS::WB, nw - w0);  // walkers in this batch; later slots are not written out
#pragma unroll 1
      for (int q = 0; q < qn; ++q) {
        const int w = w0 + q;
        const T xh = cell_xhi<T, kNrMax>(d, dcell, nr, wc[w], thr + static_cast<size_t>(w) * kNrMax, dc);
        ldsr[2 * (q * N + x) + row] = tb * xh * od;
        if constexpr (IS::NT >= 64) {
          const T s = wave_sum(xh);
          if (lane == 0) wsum[q][wave] = s;
        } else {
          wsum[q][t] = xh;
        }
      }
      __syncthreads();
      if (t < IS::WB && w0 + t < nw) {
        double s = 0.0;
        for (int k = 0; k < (IS::NT >= 64 ? IS::NW : IS::NT); ++k) s += static_cast<double>(wsum[t][k]);
        acc[w0 + t] += s;
      }
      fft_team<N, -1, T, typename IS::Plan>(lds + (t / IS::TS) * N, 1, t % IS::TS, twl, 1);
      for (int idx = t; idx < IS::WB * IS::H; idx += IS::NT) {
        const int q = idx / IS::H, k = idx % IS::H;
        const int w = w0 + q;
        if (w < nw) {
          cplx<T> A, B;
          unpack_pair<N>(lds + q * N, k, A, B);
          cplx<T>* o = spec + static_cast<size_t>(w) * SPEC + static_cast<size_t>(2 * p) * IS::HP;
          o[k] = A;
          o[IS::HP + k] = B;
        }
      }
      __syncthreads();
    }
  }
  for (int w = t; w < nw; w += IS::NT) xpart[static_cast<size_t>(w) * gridDim.x + blockIdx.x] = acc[w];
}

// Materialise x_HI and dT_b of one walker (same per-cell arithmetic as above).
template <typename T, typename S, int N>
__global__ __launch_bounds__(256) void k_materialize(const S* __restrict__ dR, const T* __restrict__ delta, int nr,
                                                     const WalkerConst<T>* __restrict__ wc,
                                                     const T* __restrict__ thr, T tb, T dc, T* __restrict__ xhi,
                                                     T* __restrict__ dtb) {
  constexpr size_t N3 = static_cast<size_t>(N) * N * N;
  const WalkerConst<T> c = wc[0];
  for (size_t cell = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; cell < N3;
       cell += static_cast<size_t>(gridDim.x) * 256) {
    T d[kNrMax];
    T dcell;
    load_radii<T, S>(dR, N3, cell, nr, d, dcell);
    const T x = cell_xhi<T, kNrMax>(d, dcell, nr, c, thr, dc);
    if (xhi) xhi[cell] = x;
    if (dtb) dtb[cell] = tb * x * (T(1) + delta[cell]);
  }
}

// Deterministic final reduction for one walker per block:
// pk[b] = pscale * sum_tiles part / counts[b]; xhi = inv_cells * sum xpart.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ part, long ntiles, int nbins,
                                                  const double* __restrict__ xpart, long nblk,
                                                  const double* __restrict__ counts, double pscale,
                                                  double inv_cells, double* __restrict__ pk, long pk_stride,
                                                  int nbins_out, double* __restrict__ xhi, long xhi_stride) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const long w = blockIdx.x;
  const double* pw = part + w * ntiles * nbins;
  for (int b = 0; b <= nbins; ++b) {
    double s = 0.0;
    if (b < nbins) {
      for (long i = t; i < ntiles; i += 256) s += pw[i * nbins + b];
    } else if (xpart) {
      for (long i = t; i < nblk; i += 256) s += xpart[w * nblk + i];
    }
    red[t] = s;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
      if (t < h) red[t] += red[t + h];
      __syncthreads();
    }
    if (t == 0) {
      if (b < nbins) {
        if (pk) pk[w * pk_stride + b] = counts[b] > 0.0 ? pscale * red[0] / counts[b] : 0.0;
      } else if (xhi && xpart) {
        xhi[w * xhi_stride] = red[0] * inv_cells;
      }
    }
    __syncthreads();
  }
  if (pk && t >= nbins && t < nbins_out) pk[w * pk_stride + t] = 0.0;
}

template <typename T, typename S>
__global__ __launch_bounds__(256) void k_cast(const S* __restrict__ in, T* __restrict__ out, size_t n) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += static_cast<size_t>(gridDim.x) * 256)
    out[i] = load_as<T>(in, i);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {

template <typename F>
hipError_t with_n(int n, F&& f) {
  switch (n) {
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 512: return f(std::integral_constant<int, 512>{});
    default: return hipErrorInvalidValue;
  }
}

template <typename F>
hipError_t with_real(int dtype, F&& f) {
  if (dtype == kF64) return f(double{});
  if (dtype == kF32) return f(float{});
  return hipErrorInvalidValue;
}

template <typename T, typename F>
hipError_t with_storage(int storage, F&& f) {
  if constexpr (std::is_same<T, double>::value) {
    if (storage == kF64) return f(double{});
  } else {
    if (storage == kF32) return f(float{});
    if (storage == kBF16) return f(bf16{});
  }
  return hipErrorInvalidValue;
}

unsigned grid_for(long work, long cap) { return static_cast<unsigned>(work < cap ? (work > 0 ? work : 1) : cap); }

}  // namespace

int axis_tile(int n) {
  int ti = 0;
  (void)with_n(n, [&](auto nc) {
    ti = AxisShape<decltype(nc)::value>::TI;
    return hipSuccess;
  });
  return ti;
}

long axis_tiles(int n, long inner) {
  const int ti = axis_tile(n);
  return ti > 0 ? (inner + ti - 1) / ti : 0;
}

int ion_grid(int n) { return static_cast<int>(grid_for(static_cast<long>(n) * n / 2, 4096)); }

int max_group() { return kMaxGroup; }
int max_radii() { return kNrMax; }
int thr_stride() { return kNrMax; }

int half_pitch(int n) {
  int hp = 0;
  (void)with_n(n, [&](auto nc) {
    hp = Half<decltype(nc)::value>::HP;
    return hipSuccess;
  });
  return hp;
}
int max_bins() { return kMaxBins; }

hipError_t launch_rows_r2c(int dtype, int n, const void* in, void* out, long nrows, const void* tw, int ntab,
                           hipStream_t s) {
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_n(n, [&](auto nc) {
      constexpr int N = decltype(nc)::value;
      const long npairs = nrows / 2;
      const long groups = (npairs + RowShape<N>::WB - 1) / RowShape<N>::WB;
      hipLaunchKernelGGL((k_rows_r2c<T, N>), dim3(grid_for(groups, 8192)), dim3(RowShape<N>::NT), 0, s,
                         static_cast<const T*>(in), static_cast<cplx<T>*>(out), npairs,
                         static_cast<const cplx<T>*>(tw), ntab / N);
      return hipGetLastError();
    });
  });
}

hipError_t launch_rows_c2r(int dtype, int storage, int n, const void* in, void* out, long nrows, double scale,
                           int kmax, const void* tw, int ntab, hipStream_t s) {
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_storage<T>(storage, [&](auto sv) {
      using ST = decltype(sv);
      return with_n(n, [&](auto nc) {
        constexpr int N = decltype(nc)::value;
        const long npairs = nrows / 2;
        const long groups = (npairs + RowShape<N>::WB - 1) / RowShape<N>::WB;
        hipLaunchKernelGGL((k_rows_c2r<T, ST, N>), dim3(grid_for(groups, 8192)), dim3(RowShape<N>::NT), 0, s,
                           static_cast<const cplx<T>*>(in), static_cast<ST*>(out), npairs, static_cast<T>(scale),
                           kmax, static_cast<const cplx<T>*>(tw), ntab / N);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_axis(int dtype, int n, int dir, int mode, const void* src, void* dst, long outer, long inner,
                       long ilim, long n2max, const void* tw, int ntab, hipStream_t s) {
  if (ilim < 1 || ilim > inner || mode < 0 || mode > 2) return hipErrorInvalidValue;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_n(n, [&](auto nc) {
      constexpr int N = decltype(nc)::value;
      using A = AxisShape<N>;
      const dim3 grid(static_cast<unsigned>((ilim + A::TI - 1) / A::TI), static_cast<unsigned>(outer));
      const auto* sp = static_cast<const cplx<T>*>(src);
      auto* dp = static_cast<cplx<T>*>(dst);
      const auto* tp = static_cast<const cplx<T>*>(tw);
      const int ts = ntab / N;
      if (dir < 0) {
        hipLaunchKernelGGL((k_axis<T, N, -1, 0>), grid, dim3(A::NT), 0, s, sp, dp, inner, ilim, n2max, tp, ts);
      } else if (mode == 1) {
        hipLaunchKernelGGL((k_axis<T, N, +1, 1>), grid, dim3(A::NT), 0, s, sp, dp, inner, ilim, n2max, tp, ts);
      } else if (mode == 2) {
        hipLaunchKernelGGL((k_axis<T, N, +1, 2>), grid, dim3(A::NT), 0, s, sp, dp, inner, ilim, n2max, tp, ts);
      } else {
        hipLaunchKernelGGL((k_axis<T, N, +1, 0>), grid, dim3(A::NT), 0, s, sp, dp, inner, ilim, n2max, tp, ts);
      }
      return hipGetLastError();
    });
  });
}

hipError_t launch_axis_bins(int dtype, int n, const void* src, long outer, long inner, const int8_t* bintab,
                            int nbins, double* part, const void* tw, int ntab, hipStream_t s) {
  if (nbins < 1 || nbins > kMaxBins) return hipErrorInvalidValue;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_n(n, [&](auto nc) {
      constexpr int N = decltype(nc)::value;
      using A = AxisShape<N>;
      const dim3 grid(static_cast<unsigned>((inner + A::TI - 1) / A::TI), static_cast<unsigned>(outer));
      hipLaunchKernelGGL((k_axis_bins<T, N>), grid, dim3(A::NT), 0, s, static_cast<const cplx<T>*>(src), inner,
                         bintab, nbins, part, static_cast<const cplx<T>*>(tw), ntab / N);
      return hipGetLastError();
    });
  });
}

hipError_t launch_ion(int dtype, int storage, int n, const void* dR, const void* delta, int nr, const void* wc,
                      const void* thr, int nw, double tb, double dc, void* spec, double* xpart, const void* tw,
                      int ntab, hipStream_t s) {
  if (nr < 1 || nr > kNrMax || nw < 1 || nw > kMaxGroup) return hipErrorInvalidValue;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_storage<T>(storage, [&](auto sv) {
      using ST = decltype(sv);
      return with_n(n, [&](auto nc) {
        constexpr int N = decltype(nc)::value;
        hipLaunchKernelGGL((k_ion_rows<T, ST, N>), dim3(ion_grid(N)), dim3(IonShape<N>::NT), 0, s,
                           static_cast<const ST*>(dR), static_cast<const T*>(delta), nr,
                           static_cast<const WalkerConst<T>*>(wc), static_cast<const T*>(thr), nw,
                           static_cast<T>(tb), static_cast<T>(dc), static_cast<cplx<T>*>(spec), xpart,
                           static_cast<const cplx<T>*>(tw), ntab / N);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_materialize(int dtype, int storage, int n, const void* dR, const void* delta, int nr,
                              const void* wc, const void* thr, double tb, double dc, void* xhi, void* dtb,
                              hipStream_t s) {
  if (nr < 1 || nr > kNrMax) return hipErrorInvalidValue;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_storage<T>(storage, [&](auto sv) {
      using ST = decltype(sv);
      return with_n(n, [&](auto nc) {
        constexpr int N = decltype(nc)::value;
        const long cells = static_cast<long>(N) * N * N;
        hipLaunchKernelGGL((k_materialize<T, ST, N>), dim3(grid_for((cells + 255) / 256, 16384)), dim3(256), 0, s,
                           static_cast<const ST*>(dR), static_cast<const T*>(delta), nr,
                           static_cast<const WalkerConst<T>*>(wc), static_cast<const T*>(thr),
                           static_cast<T>(tb), static_cast<T>(dc), static_cast<T*>(xhi), static_cast<T*>(dtb));
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_finalize(int nwalkers, const double* part, long ntiles, int nbins, const double* xpart, long nblk,
                           const double* counts, double pscale, double inv_cells, double* pk, long pk_stride,
                           int nbins_out, double* xhi, long xhi_stride, hipStream_t s) {
  if (nbins_out > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finalize, dim3(static_cast<unsigned>(nwalkers)), dim3(256), 0, s, part, ntiles, nbins, xpart,
                     nblk, counts, pscale, inv_cells, pk, pk_stride, nbins_out, xhi, xhi_stride);
  return hipGetLastError();
}

hipError_t launch_cast(int dtype, int storage, const void* in, void* out, size_t count, hipStream_t s) {
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_storage<T>(storage, [&](auto sv) {
      using ST = decltype(sv);
      hipLaunchKernelGGL((k_cast<T, ST>), dim3(grid_for(static_cast<long>((count + 255) / 256), 16384)), dim3(256), 0,
                         s, static_cast<const ST*>(in), static_cast<T*>(out), count);
      return hipGetLastError();
    });
  });
}

}  // namespace xs21
