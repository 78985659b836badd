// gfx950 kernels of the excursion-set path and their host-side launchers.
//
// Data layout (all C order, last axis contiguous):
//   real box        [z][y][x]                       N^3
//   half spectrum   [z][y][kx], kx in [0, N/2]      N * N * HP complex, rows padded
//                   to HP = N/2 + 1 rounded up to 16 (128-byte aligned rows)
//   smoothed boxes  [radius][z][y][x]               N_R * N^3 (storage type S)
//   walker spectra  [walker][z][y][kx], kx < N/2, rows padded to HP as above,
//                   with the Nyquist plane kx = N/2 apart as [walker][y][z]
//                   (contiguous along z, so its y pass runs over full tiles
//                   and its z pass reads whole rows)
//
// A 3D real-to-complex transform is three passes: rows along x (two real rows
// packed as one complex row), then the y axis, then the z axis.  The inverse
// runs z, y, then x.  The per-cell ionisation pass is fused into the x pass of
// the forward transform of dT_b, and the |X|^2 binning into its z pass.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <utility>
#include <vector>

#include "common.hpp"
#include "fft.hpp"
#include "launch.hpp"
#include "wave.hpp"

namespace xs21 {

constexpr int kMaxGroup = 64;   // walkers per ionisation launch (x_HI sums in LDS)
constexpr int kNrMax = 40;      // radii held in registers per cell
constexpr int kMaxBins = 64;
constexpr int kBinSlotTeams = 64;  // largest FFT team of the binning pass (N = 512)

// Slot rows of the binning pass for one launch over bins [b0, b0 + nbc):
// team index j keeps bins lo[j] .. b0 + nbc - 1 at rows base[j] ..; `rows`
// rows in all (passed by value).
struct BinSlots {
  int16_t lo[kBinSlotTeams];
  int16_t base[kBinSlotTeams];
  int32_t rows;
};

// Row pitch of a half spectrum: N/2 + 1 complex values padded to a multiple of
// 16 (128 bytes in FP32), so that strided passes read whole aligned lines.
template <int N>
struct Half {
  static constexpr int H = N / 2 + 1;
  static constexpr int HP = (H + 15) / 16 * 16;
};

// Radix plan of the contiguous row passes.  At N = 256 three stages with
// 32-thread teams (8 rows per LDS batch) need half the prefetch registers of
// two radix-16 stages in the pipelined inverse pass (measured faster).
template <int N>
struct RowPlan {
  using type = FftPlan<N>;
};
template <>
struct RowPlan<256> {
  using type = Radices<8, 8, 4>;
};

template <int N>
struct RowShape {
  using Plan = typename RowPlan<N>::type;
  static constexpr int WB = FftShape<N, Plan>::RMAX;  // sequences per LDS batch
  static constexpr int TS = FftShape<N, Plan>::TS;
  static constexpr int NT = N;                        // threads per block
  static constexpr int H = Half<N>::H;
  static constexpr int HP = Half<N>::HP;
};

// Radix plan of the strided passes (y and z axes).  At N = 256 three stages
// with 32-thread teams (512-thread blocks, 8 values per thread) keep more
// waves in flight per CU than two radix-16 stages (measured on the 256^3
// workload).
template <int N>
struct AxisPlan {
  using type = FftPlan<N>;
};
template <>
struct AxisPlan<256> {
  using type = Radices<8, 8, 4>;
};

template <int N>
struct AxisShape {
  using Plan = typename AxisPlan<N>::type;
  static constexpr int TS = FftShape<N, Plan>::TS;
  static constexpr int TI = (TS == 1) ? 64 : (N <= 128 ? 32 : 16);  // columns per tile
  static constexpr int NT = TI * TS;
};

// Radix plan of the binning pass: the strided passes' plan, except at N =
// 256, where a 16 x 16 plan (teams of 16 threads) fits 16 columns, i.e.
// whole 128-byte lines of FP32 modes, in a 256-thread block.
template <int N>
struct BinPlan {
  using type = typename AxisPlan<N>::type;
};
template <>
struct BinPlan<256> {
  using type = FftPlan<256>;
};

// Threads of the binning pass: FFT teams over as many columns per tile as
// kBinsTileCols columns of the strided passes' teams take threads (and at
// most the strided passes' TI), but never fewer than one wave per block (the
// final reduction runs one wave per bin).
template <int N>
struct BinShape {
  using Plan = typename BinPlan<N>::type;
  static constexpr int TS = FftShape<N, Plan>::TS;
  static constexpr int TIW = AxisShape<N>::TI < kBinsTileCols ? AxisShape<N>::TI : kBinsTileCols;
  static constexpr int TIS = TIW * AxisShape<N>::TS / TS;
  static constexpr int TIA = TIS < AxisShape<N>::TI ? TIS : AxisShape<N>::TI;
  static constexpr int TI = TIA * TS >= 64 ? TIA : 64 / TS;
  static constexpr int NT = TI * TS;
  // Tiles per 16-column group: with 8-column tiles, the two halves of each
  // 128-byte line of FP32 modes.  A block takes its tiles a group at a time
  // (the second half's load issues while the first is transformed), so both
  // halves of a line are read by one CU, through one XCD's L2: consecutive
  // blocks run on different XCDs, and a line read half by each of two would
  // be fetched from HBM twice.
  static constexpr int G = TI < 16 ? 16 / TI : 1;
  static_assert(NT % 64 == 0 && TI <= AxisShape<N>::TI, "binning blocks are whole waves");
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
// The same without the halving, 2A and 2B: for rows stored at half scale
// (exact: halving commutes with every rounding of the transform).
template <int N, typename T>
__device__ __forceinline__ void unpack_pair2(const cplx<T>* z, int k, cplx<T>& A, cplx<T>& B) {
  const cplx<T> zk = z[k];
  const cplx<T> zm = z[(N - k) & (N - 1)];
  A = {zk.x + zm.x, zk.y - zm.y};
  B = {zk.y + zm.y, zm.x - zk.x};
}

// ---------------------------------------------------------------------------
// Forward rows: real [rows][N] -> half spectra [rows][N/2+1]
// ---------------------------------------------------------------------------
// With nyq != nullptr the kx = N/2 entry of row r = z N + y goes to
// nyq[y N + z] instead (one N^3 field: npairs = N^2 / 2).
template <typename T, int N>
__global__ __launch_bounds__(RowShape<N>::NT) void k_rows_r2c(const T* __restrict__ in, cplx<T>* __restrict__ out,
                                                              cplx<T>* __restrict__ nyq, long npairs,
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
      if (p < npairs) v = {in[(2 * p) * N + t], in[(2 * p + 1) * N + t]};
      lds[q * N + t] = v;
    }
    __syncthreads();
    fft_team<N, -1, T, typename S::Plan, true>(lds + (t / S::TS) * N, 1, t % S::TS, twl, 1);
    __syncthreads();   // the row teams synchronised only within their waves
    for (int idx = t; idx < S::WB * S::H; idx += S::NT) {
      const int q = idx / S::H, k = idx % S::H;
      const long p = p0 + q;
      if (p < npairs) {
        cplx<T> A, B;
        unpack_pair<N>(lds + q * N, k, A, B);
        if (nyq && k == N / 2) {
          const long r = 2 * p, z = r / N, y = r % N;
          nyq[y * N + z] = A;
          nyq[(y + 1) * N + z] = B;
        } else {
          out[(2 * p) * S::HP + k] = A;
          out[(2 * p + 1) * S::HP + k] = B;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Inverse rows: half spectra [rows][N/2+1] -> real [rows][N] * scale, stored as S,
// for a batch of smoothing radii.  Items g = radius * groups + group of WB row
// pairs form a grid-stride loop.  Each row pair is packed into one complex
// row Z = A + i B and transformed by one team (TS threads within one wave):
// member j reads the entries k = j + r TS of its row (index min(k, N - k) of
// the two half spectra), which are exactly its first-stage butterfly, so that
// stage runs in registers; the remaining stages and the stores are the
// team's own (wave-level synchronisation only, no block barrier).  The loads
// of a block's next item are issued into registers right after the first
// stage.  Radius r reads in + r istride, writes out + r ostride (streaming
// stores) and only reads entries kx <= kmax(r) (the rest are zero after its
// sharp-k cut).
// ---------------------------------------------------------------------------
template <typename T, typename ST, int N>
__global__ __launch_bounds__(RowShape<N>::NT) void k_rows_c2r(const cplx<T>* __restrict__ in, ST* __restrict__ out,
                                                              long npairs, long nitems, T scale,
                                                              const long* __restrict__ cut, long istride,
                                                              long ostride, const cplx<T>* __restrict__ tw,
                                                              int tstride) {
  using S = RowShape<N>;
  constexpr int TS = S::TS, R0 = FftShape<N, typename S::Plan>::R0;
  static_assert(N / R0 == TS && S::WB * TS == S::NT, "one packed row per team");
  __shared__ cplx<T> lds[S::WB * N];
  __shared__ cplx<T> twl[N];
  const int t = threadIdx.x, q = t / TS, j = t % TS;
  const long groups = (npairs + S::WB - 1) / S::WB;
  load_twiddles<N>(twl, tw, tstride);
  cplx<T>* my = lds + q * N;   // the team's packed row
  cplx<T> pa[R0], pb[R0];
  const auto load = [&](long g) {
    const long r = g / groups;
    const long p = min((g % groups) * S::WB + q, npairs - 1);  // a valid row; rows past the end are not stored
    const long kc = cut[2 * r + 1];
    const cplx<T>* sa = in + r * istride + (2 * p) * S::HP;
#pragma unroll
    for (int e = 0; e < R0; ++e) {
      const int k = j + e * TS;
      const int idx = k <= N / 2 ? k : N - k;
      pa[e] = {T(0), T(0)};
      pb[e] = {T(0), T(0)};
      if (idx <= kc) {
        pa[e] = sa[idx];
        pb[e] = sa[S::HP + idx];
      }
    }
  };
  long g = blockIdx.x;
  if (g < nitems) load(g);
  for (; g < nitems; g += gridDim.x) {
    const long r = g / groups, p = (g % groups) * S::WB + q;
    // Z[k] = A[k] + i B[k] (Hermitian extension; DC and Nyquist taken as real)
    cplx<T> v[R0];
#pragma unroll
    for (int e = 0; e < R0; ++e) {
      const int k = j + e * TS;
      cplx<T> A = pa[e], B = pb[e];
      if (k == 0 || k == N / 2) {
        A.y = T(0);
        B.y = T(0);
      } else if (k > N / 2) {
        A = cconj(A);
        B = cconj(B);
      }
      v[e] = {A.x - B.y, A.y + B.x};
    }
    fft_first_from_regs<N, +1, T, typename S::Plan>(v, my, 1, j);
    if (g + gridDim.x < nitems) load(g + gridDim.x);
    fft_rest<N, +1, T, typename S::Plan, true>(my, 1, j, twl, 1);
    if (p < npairs) {
      ST* dst = out + r * ostride;
#pragma unroll
      for (int e = 0; e < R0; ++e) {
        const int n = j + e * TS;
        const cplx<T> z = my[n];
        store_as_stream(dst, (2 * p) * N + n, z.x * scale);
        store_as_stream(dst, (2 * p + 1) * N + n, z.y * scale);
      }
    }
    stage_sync<true>();   // the team's row is read before the next item writes it
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
// MODE 3: one column (inner index ilim - 1) of each of TI consecutive outer
//   slices per block (blockIdx.x picks the slices): the Nyquist column of a
//   forward y pass, so that the main launch only covers full aligned tiles.
// MODE 4: inverse z pass (inner index as in MODE 1) of the line-of-sight
//   velocity gradient: each mode is weighted by nz^2 / |n|^2 on load (0 for
//   the mean and the padding columns).
// MODE 5: MODE 1 over a list of live tiles: block b takes entry
//   tiles[b] = (radius << 24) | tile, radius counted from r0, so that no block
//   is launched for a tile outside its radius's disk.
// MODE 6: MODE 2 over a list of live column tiles: blockIdx.x takes entry
//   tiles[blockIdx.x] = (radius << 24) | tile as above (tiles with kx <= kmax
//   of that radius), blockIdx.y the slice.
// ---------------------------------------------------------------------------
// |n|^2 without the z part of flat column i = y * HP + kx of a padded half
// spectrum; padding columns (kx > N/2) get a value above every cutoff.
// (32-bit arithmetic: i < N * HP and |n|^2 <= N^2 / 2 fit easily.)
template <int N>
__device__ __forceinline__ int column_n2(long i) {
  const int ii = static_cast<int>(i);
  const int ky = ii / Half<N>::HP, kx = ii % Half<N>::HP;
  const int ny = ky < N / 2 ? ky : ky - N;
  return kx < Half<N>::H ? ny * ny + kx * kx : 0x3fffffff;
}

template <typename T, int N, int DIR, int MODE>
__global__ __launch_bounds__(AxisShape<N>::NT) void k_axis(const cplx<T>* src, cplx<T>* dst, long inner, long ilim,
                                                           const long* __restrict__ cut, long sstride, long dstride,
                                                           long nslices, const cplx<T>* __restrict__ tw, int tstride,
                                                           const int32_t* __restrict__ tiles, int r0) {
  using A = AxisShape<N>;
  constexpr bool DISK = MODE == 1 || MODE == 5;  // z pass of a smoothing
  constexpr bool YPASS = MODE == 2 || MODE == 6;  // y pass of a smoothing
  __shared__ cplx<T> lds[N * A::TI];
  __shared__ cplx<T> twl[N];
  const int t = threadIdx.x;
  // blockIdx.z (or the list entry) selects one smoothing radius of a batch:
  // its own cutoff (n2max, kmax) and its own slice of src / dst
  long zr = blockIdx.z, bx = blockIdx.x;
  if constexpr (MODE == 5 || MODE == 6) {
    const int32_t e = tiles[blockIdx.x];
    zr = (e >> 24) - r0;
    bx = e & 0xffffff;
  }
  long n2max = 0;
  if constexpr (DISK || YPASS) {
    n2max = cut[2 * zr];
    if constexpr (YPASS) ilim = min(ilim, cut[2 * zr + 1] + 1);
  }
  src += zr * sstride;
  dst += zr * dstride;
  if constexpr (MODE == 3) {
    // gathered single columns: column c of the tile is slice blockIdx.x * TI + c
    const long outer = nslices;
    for (int m = t; m < N; m += A::NT) twl[m] = tw[m * tstride];
    for (int l = t; l < N * A::TI; l += A::NT) {
      const int n = l / A::TI, c = l % A::TI;
      const long o = static_cast<long>(blockIdx.x) * A::TI + c;
      lds[l] = o < outer ? src[(o * N + n) * inner + ilim - 1] : cplx<T>{T(0), T(0)};
    }
    __syncthreads();
    fft_team<N, DIR, T, typename A::Plan>(lds + (t % A::TI), A::TI, t / A::TI, twl, 1);
    for (int l = t; l < N * A::TI; l += A::NT) {
      const int n = l / A::TI, c = l % A::TI;
      const long o = static_cast<long>(blockIdx.x) * A::TI + c;
      if (o < outer) dst[(o * N + n) * inner + ilim - 1] = lds[l];
    }
    return;
  }
  const long base = static_cast<long>(blockIdx.y) * N * inner;
  const long i0 = bx * A::TI;
  if (i0 >= ilim) return;  // block-uniform
  if constexpr (MODE == 1) {
    bool any = false;  // block-uniform
    for (int c = 0; c < A::TI; ++c) any |= (i0 + c < ilim) && column_n2<N>(i0 + c) <= n2max;
    if (!any) return;
  }
  for (int m = t; m < N; m += A::NT) twl[m] = tw[m * tstride];
  // every element is loaded (dead ones from the slice's first element, a valid
  // address holding a finite value) before any is used, so the loads issue
  // back to back
  constexpr int L = N * A::TI / A::NT;
  static_assert(A::NT % A::TI == 0, "a thread keeps one column");
  const int c = t % A::TI;
  const long i = i0 + c;
  cplx<T> v[L];
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const int n = t / A::TI + k * (A::NT / A::TI);
    const long nn = n < N / 2 ? n : n - N;
    bool live = i < ilim;
    T wgt = T(1);
    if constexpr (DISK) live = live && column_n2<N>(i) + nn * nn <= n2max;
    if constexpr (YPASS) live = live && nn * nn + i * i <= n2max;
    if constexpr (MODE == 4) {
      const int c2 = column_n2<N>(i);
      const long k2 = c2 + nn * nn;
      live = live && c2 < 0x3fffffff && k2 > 0;
      wgt = live ? static_cast<T>(nn * nn) / static_cast<T>(k2) : T(0);
    }
    // a product, not a select, keeps the compiler from moving the load under
    // a branch (the dead lanes' element is a finite value)
    const cplx<T> x = src[live ? base + n * inner + i : base];
    const T keep = live ? wgt : T(0);
    v[k] = {x.x * keep, x.y * keep};
  }
#pragma unroll
  for (int k = 0; k < L; ++k) lds[t + k * A::NT] = v[k];
  __syncthreads();
  fft_team<N, DIR, T, typename A::Plan>(lds + (t % A::TI), A::TI, t / A::TI, twl, 1);
  for (int l = t; l < N * A::TI; l += A::NT) {
    const int n = l / A::TI, c = l % A::TI;
    const long i = i0 + c;
    bool keep = i < ilim;
    if constexpr (DISK) keep = keep && column_n2<N>(i) <= n2max;
    if (keep) dst[base + n * inner + i] = lds[l];
  }
}

// Plain strided pass over full tiles only (columns i0 .. i0 + TI - 1 < ilim),
// as a grid-stride loop over tiles g = slice * tiles_x + column block: each
// block issues the global loads of its next tile into registers before the
// FFT of the current one, so that memory latency overlaps the transform.
// Loads and stores are streaming: each element is touched once per pass.
// DISK (forward y pass of a spectrum that is only binned): outputs whose mode
// has ny^2 + kx^2 > (N/2)^2 are never binned (|n| > N/2 for every nz), so
// they are not stored.  DISK 1: kx is the column index (the kx < N/2 rows);
// DISK 2: kx = N/2 for every column (the Nyquist plane, [ky][z]).
template <typename T, int N, int DIR, int DISK = 0>
__global__ __launch_bounds__(AxisShape<N>::NT) void k_axis_pipe(const cplx<T>* src, cplx<T>* dst, long inner,
                                                                long tiles_x, long ntiles,
                                                                const cplx<T>* __restrict__ tw, int tstride) {
  using A = AxisShape<N>;
  constexpr int L = N * A::TI / A::NT;  // elements per thread and tile
  __shared__ cplx<T> lds[N * A::TI];
  __shared__ cplx<T> twl[N];
  const int t = threadIdx.x;
  const int c = t % A::TI, n0 = t / A::TI;  // element l = t + k NT sits at row n0 + k NT / TI, column c
  constexpr int NSTEP = A::NT / A::TI;
  for (int m = t; m < N; m += A::NT) twl[m] = tw[m * tstride];
  cplx<T> pre[L];
  const auto offset = [&](long g) {
    const long o = g / tiles_x, i0 = (g % tiles_x) * A::TI;
    return (o * N + n0) * inner + i0 + c;
  };
  long g = blockIdx.x;
  if (g < ntiles) {
    const long off = offset(g);
#pragma unroll
    for (int k = 0; k < L; ++k) pre[k] = load_stream(src + off + static_cast<long>(k) * NSTEP * inner);
  }
  static_assert(L == FftShape<N, typename A::Plan>::R0, "a thread's loads are its first-stage butterfly");
  for (; g < ntiles; g += gridDim.x) {
    // the loaded rows n0 + k NSTEP are this thread's first-stage butterfly:
    // that stage runs in registers, which then take the next tile's loads
    fft_first_from_regs<N, DIR, T, typename A::Plan>(pre, lds + c, A::TI, n0);
    const long off = offset(g);
    const long gn = g + gridDim.x;
    if (gn < ntiles) {
      const long offn = offset(gn);
#pragma unroll
      for (int k = 0; k < L; ++k) pre[k] = load_stream(src + offn + static_cast<long>(k) * NSTEP * inner);
    }
    fft_rest<N, DIR, T, typename A::Plan>(lds + c, A::TI, n0, twl, 1);
    int kx2 = 0;
    if constexpr (DISK == 1) {
      const int kx = static_cast<int>((g % tiles_x) * A::TI) + c;
      kx2 = kx * kx;
    } else if constexpr (DISK == 2) {
      kx2 = (N / 2) * (N / 2);
    }
#pragma unroll
    for (int k = 0; k < L; ++k) {
      bool keep = true;
      if constexpr (DISK != 0) {
        const int ky = n0 + k * NSTEP;
        const int ny = ky < N / 2 ? ky : ky - N;
        keep = ny * ny + kx2 <= (N / 2) * (N / 2);
      }
      if (keep) store_stream(dst + off + static_cast<long>(k) * NSTEP * inner, lds[t + k * A::NT]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Forward z pass fused with |X|^2 binning.  src [outer][N][N * HP] holds the
// x- and y-transformed spectra (padded rows, kx < N/2) and nyq [outer][N][N]
// their Nyquist planes kx = N/2 as [ky][z].  Tiles cover live columns only
// and keep aligned loads: "main" tiles are TI consecutive kx < KM of one y
// (KM = the largest multiple of TI <= N/2; TI = 16 at N = 256, whole
// 128-byte lines), "rest" tiles gather the remaining columns (kx in [KM, N/2], the
// Nyquist plane for N >= 32) of TI consecutive (y, kx) pairs.  Block i of a
// spectrum's `parts` blocks takes the groups i, i + parts, i + 2 parts, ... of
// G consecutive entries of the list `tiles` (BinShape::G; blocks running
// together read neighbouring groups), accumulates its bin sums over them
// and writes FP64 sums of w |X|^2 for bins [b0, b0 + nbc) to
// part[spectrum][i][nbins].  The list holds the groups with at least one
// column ny^2 + kx^2 <= (N/2)^2: no mode of the other columns is ever binned
// (the y pass does not even store them; whatever such a column holds stays in
// its own z transform and meets only the bin entry of the dropped DC mode).
// Weights w: 1 on the kx = 0 and kx = N/2 planes, 2 elsewhere (half spectrum).
//
// Every sum is FP64: |X|^2 of a mode is formed in T, each thread adds its
// modes in double to running sums in LDS, and a fixed-order wave reduction
// adds those.  A thread outputs the kz range [j M, j M + M) of its column, so
// |n| >= min |nz| over that range and its modes never reach the bins below
// BinSlots::lo[j]: it keeps double slots only for bins lo[j] .. b0 + nbc - 1,
// at rows base[j] .. of a [rows][TI] slot array (same rows for every column
// cc of a tile).
// ---------------------------------------------------------------------------
template <int N, int TI>
struct BinTiles {
  static constexpr int H = Half<N>::H;
  static constexpr int KM = (N / 2) / TI * TI;      // kx covered by main tiles
  static constexpr int RW = H - KM;                 // rest columns per y
  static constexpr long MAIN = static_cast<long>(N) * (KM / TI);
  static constexpr long REST = (static_cast<long>(N) * RW + TI - 1) / TI;
  static constexpr long COUNT = MAIN + REST;
  // (ky, kx) of column cc of a tile, or ky = -1 past the end
  __host__ __device__ static void column(long tile, int cc, int& ky, int& kx) {
    if constexpr (KM > 0) {
      if (tile < MAIN) {
        ky = static_cast<int>(tile / (KM / TI));
        kx = static_cast<int>(tile % (KM / TI)) * TI + cc;
        return;
      }
    }
    {
      const long r = (tile - MAIN) * TI + cc;
      ky = r < static_cast<long>(N) * RW ? static_cast<int>(r / RW) : -1;
      kx = KM + static_cast<int>(r % RW);
    }
  }
};

template <typename T, int N>
__global__ __launch_bounds__(BinShape<N>::NT) void k_axis_bins(const cplx<T>* __restrict__ src,
                                                                const cplx<T>* __restrict__ nyq, long parts,
                                                                const int32_t* __restrict__ tiles, long ntiles,
                                                                const int8_t* __restrict__ bintab,
                                                                int nbins, int b0, int nbc, BinSlots bs,
                                                                double* __restrict__ part,
                                                                const cplx<T>* __restrict__ tw, int tstride) {
  using A = BinShape<N>;
  using BT = BinTiles<N, A::TI>;
  constexpr int HP = Half<N>::HP;
  constexpr long PLANE = static_cast<long>(N) * HP;  // stride between z planes
  constexpr int M = N / A::TS;                       // contiguous outputs per thread
  constexpr int NW = A::NT / 64;                     // waves per block
  constexpr int L = N * A::TI / A::NT;               // loaded elements per thread and tile
  constexpr int NSTEP = A::NT / A::TI;
  static_assert(A::TS <= kBinSlotTeams, "slot table too small for this team size");
  __shared__ cplx<T> lds[N * A::TI];
  __shared__ cplx<T> twl[N];
  // slot[(base[j] + b - lo[j]) TI + cc]: running FP64 sum of bin b of the
  // threads with team index j and column cc (bs.rows rows of TI values)
  HIP_DYNAMIC_SHARED(unsigned char, dyn_lds)
  double* slot = reinterpret_cast<double*>(dyn_lds);
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int cc = t % A::TI, j = t / A::TI;  // loads: rows j + k NSTEP; FFT: team member j of column cc
  const long spec = blockIdx.x / parts, first = blockIdx.x % parts;
  const cplx<T>* sp = src + spec * N * PLANE;
  for (int m = t; m < N; m += A::NT) twl[m] = tw[m * tstride];
  for (int e = t; e < bs.rows * A::TI; e += A::NT) slot[e] = 0.0;
  // this thread's slot of bin b0 + bb sits at slot[(brow + bb) TI + cc]
  const int brow = bs.base[j] - (bs.lo[j] - b0);
  constexpr int NB2 = (N / 2) * (N / 2) + 1;  // |n|^2 > (N/2)^2 is never binned
  // The next tile's values and the bins of this thread's outputs of it are
  // loaded together, one tile ahead: the wait for a tile's data at the top of
  // the loop then also covers its bins, and no load issued for the next tile
  // is waited on before the loop comes round.  Bins are loaded
  // unconditionally (entry 0, the dropped DC mode, stands in for modes that
  // are not binned).
  cplx<T> pre[L];
  int nbin[M];
  const cplx<T>* nq = nyq + spec * N * N;
  const auto load = [&](long tile) {
    int ky, kx;
    BT::column(tile, cc, ky, kx);
    const bool live = ky >= 0;
    const long kyv = live ? ky : 0;  // a valid address either way
    // the Nyquist column kx = N/2 sits in its own plane [ky][z]
    const bool nqc = kx == N / 2;
    const cplx<T>* base = nqc ? nq + kyv * N + j : sp + static_cast<long>(j) * PLANE + kyv * HP + kx;
    const long step = nqc ? static_cast<long>(NSTEP) : static_cast<long>(NSTEP) * PLANE;
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const cplx<T> v = base[k * step];
      pre[k] = live ? v : cplx<T>{T(0), T(0)};
    }
    // this thread's outputs of the tile: column (ky, kx), kz = j M .. j M + M - 1
    const int ny = ky < N / 2 ? ky : ky - N;
    const int cyx = ny * ny + kx * kx;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int kz = j * M + m;
      const int nz = kz < N / 2 ? kz : kz - N;
      const int n2 = nz * nz + cyx;
      nbin[m] = bintab[(live && n2 < NB2) ? n2 : 0];
    }
  };
  // list entry of this block's i-th tile: groups first, first + parts, ...
  // of A::G consecutive entries (increasing in i)
  const auto entry = [&](long i) { return (first + (i / A::G) * parts) * A::G + (i % A::G); };
  __syncthreads();  // slots cleared before any thread adds to them
  long e = entry(0);
  if (e < ntiles) load(tiles[e]);
  static_assert(L == FftShape<N, typename A::Plan>::R0, "a thread's loads are its first-stage butterfly");
  for (long i = 0; e < ntiles; ++i) {
    const long tile = tiles[e];
    // the loaded rows j + k NSTEP are this thread's first-stage butterfly:
    // that stage runs on them in registers (no LDS round trip), then the
    // registers take the next tile's loads
    int bin[M];
#pragma unroll
    for (int m = 0; m < M; ++m) bin[m] = nbin[m];
    fft_first_from_regs<N, -1, T, typename A::Plan>(pre, lds + cc, A::TI, j);
    const long en = entry(i + 1);
    if (en < ntiles) load(tiles[en]);
    int ky, kx;
    BT::column(tile, cc, ky, kx);
    fft_rest<N, -1, T, typename A::Plan>(lds + cc, A::TI, j, twl, 1);
    // |nz| is monotone along m, so equal bins come in runs, each added to the
    // thread's own slot once
    const T w = (kx == 0 || kx == N / 2) ? T(1) : T(2);
    int cur = -1;
    double run = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const cplx<T> x = lds[(j * M + m) * A::TI + cc];
      const int b = bin[m] - b0;  // negative for modes that are not binned
      const int bb = (b >= 0 && b < nbc) ? b : -1;
      if (bb != cur) {
        if (cur >= 0) slot[(brow + cur) * A::TI + cc] += run;
        run = 0.0;
        cur = bb;
      }
      run += static_cast<double>(w * (x.x * x.x + x.y * x.y));
    }
    if (cur >= 0) slot[(brow + cur) * A::TI + cc] += run;
    __syncthreads();  // the FFT buffer is read before the next tile is stored
    e = en;
  }
  // one wave per bin adds the slots of that bin over every (team index,
  // column) in a fixed order (deterministic)
  double* out = part + (spec * parts + blockIdx.x % parts) * nbins + b0;
  for (int b = wave; b < nbc; b += NW) {
    double sum = 0.0;
    for (int e = lane; e < A::TS * A::TI; e += 64) {
      const int jj = e / A::TI, c = e % A::TI;
      const int lo = bs.lo[jj] - b0;
      if (b >= lo) sum += slot[(bs.base[jj] + b - lo) * A::TI + c];
    }
    const double d = wave_sum(sum);
    if (lane == 0) out[b] = d;
  }
}

// ---------------------------------------------------------------------------
// Per-cell ionisation (Section 2.1, eq. 1 and partial ionisation).
// Radius slots run from the cell radius up: d[s] = delta_R at ladder radius
// nr - 1 - s, so slot 0 is the cell radius and a walker uses the slots below
// its count of radii with R <= R_mfp.  Flag iff delta_R >= thr[s] for some
// slot: thresholds are the FP64-planned exact rewrite of zeta f_coll >= 1,
// +inf for slots the walker does not use, tested 8 slots at a time up to the
// walker's last used group (a wave-uniform exit), so the compares follow the
// walker's own radius count and its threshold loads batch into wide scalar
// loads.  Unflagged cells keep x_HI = 1 - zeta erfc(a_cell (delta_c - delta_cell)).
//
// TWO (the two-population efficiency of Section 4, eq. 9): each slot has an
// interval, flag iff thr[s] <= delta_R <= thr[NR + s] (only the lower end is
// tested for walkers whose intervals are all open above), and unflagged cells
// keep x_HI = 1 - zeta_eff(t) erfc(t), t = max(a_cell (delta_c - delta_cell), 0),
// with zeta_eff read from the walker's cell-radius table zt.
// ---------------------------------------------------------------------------

// Effective efficiency at t >= 0 from a table of t = (k h)^2, k < kZetaTab:
// 4-point Lagrange interpolation in sqrt(t), clamped to the table's end.
template <typename T>
__device__ __forceinline__ T zeta_eff(const T* __restrict__ tab, T t) {
  const T inv_h = static_cast<T>((kZetaTab - 1) / 2.8284271247461903);   // 1 / h, h = sqrt(8) / (K - 1)
  const T u = min(sqrt(t) * inv_h, static_cast<T>(kZetaTab - 1));
  const int j = min(max(static_cast<int>(u) - 1, 0), kZetaTab - 4);
  const T x = u - static_cast<T>(j);
  const T x1 = x - T(1), x2 = x - T(2), x3 = x - T(3);
  const T p0 = tab[j], p1 = tab[j + 1], p2 = tab[j + 2], p3 = tab[j + 3];
  return (x * x1 * (p3 * x2 - T(3) * p2 * x3) + x2 * x3 * (T(3) * p1 * x - p0 * x1)) * T(1.0 / 6.0);
}

// OR over the tested radius slots as wave-wide lane masks (one compare per
// slot into a scalar mask; UP: the two-sided interval test).
template <typename T, int NR, bool UP>
__device__ __forceinline__ unsigned long long flag_mask(const T (&d)[NR], int chunks, const T* thr_w) {
  static_assert(NR % 8 == 0, "radius slots come in groups of 8");
  // the cell radius is always tested, so the first group's thresholds load
  // together with the walker constants (one scalar-load wait fewer per walker)
  __builtin_assume(chunks >= 1);
  unsigned long long m = 0;
#pragma unroll
  for (int g = 0; g < NR / 8; ++g) {
    if (g >= chunks) break;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int s = 8 * g + k;
      if constexpr (UP)
        m |= __ballot((d[s] >= thr_w[s]) & (d[s] <= thr_w[NR + s]));
      else
        m |= __ballot(d[s] >= thr_w[s]);
    }
  }
  return m;
}

// 1 - zeta erfc(a u), u = delta_c - delta_cell, for an unflagged cell of a
// walker with partial != 0.  FP32 walkers with partial == 2 have u > 0 here
// (the cell-radius threshold lies below delta_c), which takes the erfc of a
// positive argument with the cell's u and u^2 formed once for all walkers.
template <typename T>
__device__ __forceinline__ T partial_xhi_pos(const WalkerConst<T>& c, T u, T u2) {
  return T(1) - c.zeta * erfc_pos(c.ha, c.a2l, u, u2);
}
template <typename T>
__device__ __forceinline__ T partial_xhi(const WalkerConst<T>& c, T u, T u2) {
  if constexpr (sizeof(T) == 4) {
    if (c.partial == 2) return partial_xhi_pos(c, u, u2);
  }
  return T(1) - c.zeta * erfc_t(c.a_cell * u);
}

template <typename T, int NR, bool TWO>
__device__ __forceinline__ T cell_xhi(const T (&d)[NR], const WalkerConst<T>& c, const T* thr_w, const T* zt_w,
                                      T dc, T u2) {
  // two-population walkers whose intervals are all open above test one end
  unsigned long long m;
  if constexpr (TWO)
    m = c.upper ? flag_mask<T, NR, true>(d, c.chunks, thr_w) : flag_mask<T, NR, false>(d, c.chunks, thr_w);
  else
    m = flag_mask<T, NR, false>(d, c.chunks, thr_w);
  // this lane's bit of the wave mask, as a lane predicate (no per-lane shift)
  const bool flag = __builtin_amdgcn_inverse_ballot_w64(m);
  T x = T(1);
  if (flag) {
    x = T(0);
  } else if (c.partial) {
    if constexpr (TWO) {
      const T t = max(c.a_cell * (dc - d[0]), T(0));
      x = T(1) - zeta_eff(zt_w, t) * erfc_t(t);
    } else {
      x = partial_xhi(c, dc - d[0], u2);
    }
  }
  return x;
}

// Loads delta_R of one cell for every radius slot (slot s = ladder radius
// nr - 1 - s).  Slots past the ladder end repeat the largest radius (their
// thresholds are +inf), so that all loads are unconditional and issue back to
// back.
template <typename T, typename S, int NR>
__device__ __forceinline__ void load_radii(const S* __restrict__ dR, size_t n3, size_t cell, int nr, T (&d)[NR]) {
#pragma unroll
  for (int s = 0; s < NR; ++s) d[s] = load_as<T>(dR, static_cast<size_t>(s < nr ? nr - 1 - s : 0) * n3 + cell);
}

// ---------------------------------------------------------------------------
// Sorted-threshold flag test.  For one walker group (<= 64 walkers) and one
// radius slot s, the set of walkers whose flag test ionises a cell is a
// function of delta_R alone: walker w is in it iff thr[w][s] <= delta_R.  With
// the group's thresholds of slot s sorted, S_0 <= ... <= S_63 (+inf for absent
// walkers and unused slots), that set is the first k of them, k = #{j : S_j <=
// delta_R}, i.e. the bits of the prefix mask P_s[k] (walkers of sorted positions
// < k).  A cell is flagged for walker w iff bit w of OR_s P_s[k_s] is set: the
// same compares as the per-walker test (ties included), reached by one binary
// search per slot for the whole group instead of one compare per walker.
// Per slot the table holds E_s[64]: S_0..S_62 in breadth-first (Eytzinger)
// order of a complete 6-level search tree (node i has children 2i+1, 2i+2),
// then S_63; and P_s[0..64] (rows of kMaskPitch).
// ---------------------------------------------------------------------------
constexpr int kSortWidth = 64;   // walkers per sorted group (= kMaxGroup)
constexpr int kMaskPitch = 66;   // prefix masks per slot (65 used), 16-byte rows
static_assert(kSortWidth == kMaxGroup, "one sorted table covers one walker group");

// Tables of slots [0, kNrMax) for walkers [0, nw) with thresholds
// thr[w * wstride + s] (slot index as in the ionisation pass).  One block of
// 64 threads per slot; thread w ranks walker w's threshold (ties by index).
// Blocks kNrMax .. 2 kNrMax - 1 (two-population walkers, wstride = 2 kNrMax)
// build the second set, E + kNrMax * kSortWidth and P + kNrMax * kMaskPitch,
// from the upper ends thr[w * wstride + kNrMax + s], each raised to the next
// float: hi < delta_R iff nextup(hi) <= delta_R, so that the same search
// counts the walkers whose interval ends below delta_R.
template <typename T>
__global__ __launch_bounds__(kSortWidth) void k_slot_tables(const T* __restrict__ thr, int wstride, int nw,
                                                            T* __restrict__ E, uint64_t* __restrict__ P) {
  const int s = blockIdx.x % kNrMax, h = blockIdx.x / kNrMax, w = threadIdx.x;
  __shared__ T v[kSortWidth];
  __shared__ T srt[kSortWidth];
  __shared__ int id[kSortWidth];
  T mine = w < nw ? thr[static_cast<size_t>(w) * wstride + h * kNrMax + s] : static_cast<T>(INFINITY);
  if (h == 1) mine = nextafter(mine, static_cast<T>(INFINITY));
  E += static_cast<size_t>(h) * kNrMax * kSortWidth;
  P += static_cast<size_t>(h) * kNrMax * kMaskPitch;
  v[w] = mine;
  __syncthreads();
  int r = 0;
  for (int j = 0; j < kSortWidth; ++j) {
    const T o = v[j];
    r += (o < mine || (o == mine && j < w)) ? 1 : 0;
  }
  srt[r] = mine;
  id[r] = w;
  __syncthreads();
  if (w < kSortWidth - 1) {
    // node w of the search tree: level l, position p within the level; its
    // in-order index (the sorted position it splits at) is (2p + 1) 2^(5 - l) - 1
    const int l = 31 - __builtin_clz(static_cast<unsigned>(w + 1));
    const int pos = w + 1 - (1 << l);
    E[s * kSortWidth + w] = srt[((2 * pos + 1) << (5 - l)) - 1];
  } else {
    E[s * kSortWidth + w] = srt[kSortWidth - 1];
  }
  uint64_t m = 0;
  for (int j = 0; j < w; ++j) m |= 1ull << id[j];
  P[s * kMaskPitch + w] = m;
  if (w == kSortWidth - 1) P[s * kMaskPitch + kSortWidth] = m | (1ull << id[w]);
}

// An empty asm taking v in a vector register and giving it back: the value
// is then opaque to the compiler's algebra and computed in every lane.
template <typename V>
__device__ __forceinline__ void in_vgpr(V& v) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm("" : "+v"(v));
#else
  (void)v;
#endif
}

// One step of the search: 2 H + (e <= d ? s1 : s0), as compare, select and
// shift-add (three instructions; as plain code the compiler splits the
// select's group offset into a fourth).  s0 and s1 come in vector registers
// (the select's VCC read is its one scalar operand).  The device pass writes them out;
// the host pass (and the CPU build of the tests) evaluates the same formula.
__device__ __forceinline__ int heap_step(int H, float e, float d, int s0, int s1) {
#if defined(__HIP_DEVICE_COMPILE__)
  int t;
  asm("v_cmp_le_f32_e32 vcc, %[e], %[d]\n\t"
      "v_cndmask_b32_e32 %[t], %[s0], %[s1], vcc\n\t"
      "v_lshl_add_u32 %[h], %[h], 1, %[t]"
      : [h] "+v"(H), [t] "=&v"(t)
      : [e] "v"(e), [d] "v"(d), [s0] "v"(s0), [s1] "v"(s1)
      : "vcc");
  return H;
#else
  return 2 * H + (e <= d ? s1 : s0);
#endif
}
__device__ __forceinline__ int heap_step(int H, double e, double d, int s0, int s1) {
  return 2 * H + (e <= d ? s1 : s0);
}

// Walker mask of one cell from the sorted tables: E (in LDS) and P (global),
// for the slot groups that hold the ladder's nr slots.  The cell's delta_R are
// loaded four slots at a time, one group ahead; slots past the ladder hold
// only +inf thresholds and re-read the cell radius's value (a cache hit)
// instead of branching, since a branch would force the pending loads to
// complete early.  The four searches of a group run level by level, so their
// LDS reads issue together, and the mask reads of a group are consumed only
// after the next group's searches.  Loads address a slot's plane (or mask
// row) from scalars plus one 32-bit offset per lane.  TWO (two-population
// intervals): a second set of tables (E + kNrMax * kSortWidth, P + kNrMax *
// kMaskPitch) of the upper ends raised to the next float gives per slot the
// walkers whose interval ends below delta_R, which that slot does not flag:
// the slot's mask is P_lo[k_lo] & ~P_hi[k_hi].  Returns bits 0..31 in lo and
// 32..63 in hi.
template <typename T, typename S, bool TWO = false>
__device__ __forceinline__ void sorted_flags(const S* __restrict__ dR, size_t n3, size_t cell, int nr, const T* E,
                                             const uint64_t* __restrict__ P, uint32_t& lo, uint32_t& hi) {
  constexpr int GS = 4;
  constexpr int SZ = static_cast<int>(sizeof(T));
  constexpr int TREE = kSortWidth * SZ;   // bytes of one slot's tree
  static_assert(kNrMax % GS == 0, "slots come in groups of 4");
  // slots past the ladder have only +inf thresholds (prefix mask 0): the
  // groups that hold none of the ladder's slots are skipped
  const int ng = (nr + GS - 1) / GS;
  // byte offset of the cell in a plane: below 2^32 (N^3 sizeof(S) <= 2^30)
  const uint32_t cb = static_cast<uint32_t>(cell) * static_cast<uint32_t>(sizeof(S));
  const auto ld = [&](int sl) {
    const unsigned char* plane =
        reinterpret_cast<const unsigned char*>(dR + static_cast<size_t>(nr - 1 - (sl < nr ? sl : 0)) * n3);
    return load_as<T>(reinterpret_cast<const S*>(plane + cb), 0);
  };
  T dn[GS];
#pragma unroll
  for (int j = 0; j < GS; ++j) dn[j] = ld(j);
  uint64_t acc = 0, pend[GS] = {0, 0, 0, 0}, pendh[GS] = {0, 0, 0, 0};
  const unsigned char* eb = reinterpret_cast<const unsigned char*>(E);
  // a rolled loop: unrolled, the compiler keeps every slot's base address live
  // across the cell loop (and spills them)
#pragma unroll 1
  for (int g = 0; g < ng; ++g) {
    T dv[GS];
#pragma unroll
    for (int j = 0; j < GS; ++j) dv[j] = dn[j];
    const int gn = g + 1 < ng ? g + 1 : g;   // the last group re-reads itself (cache hits)
#pragma unroll
    for (int j = 0; j < GS; ++j) dn[j] = ld(gn * GS + j);
    // Node h of a slot's tree (heap order from 1: children 2h and 2h + 1)
    // sits at byte H = G + SZ (h - 1) from the group's first tree, G = the
    // group's byte offset in E.  A step to child 2h + b is H' = 2H - G +
    // SZ (1 + b): one select between two group constants and one shift-add,
    // and the address needs no further add (E's place in LDS and the slot's
    // tree offset fold into the read's constant offset).
    const int G = g * GS * TREE;
    int step0 = SZ - G, step1 = 2 * SZ - G;
    in_vgpr(step0);   // in registers: the select reads VCC, its one scalar operand
    in_vgpr(step1);
    // the search of table tb (0: the thresholds, 1: the raised upper ends of
    // two-population intervals) and its mask reads
    const auto search = [&](auto tbc, uint64_t (&cur)[GS]) {
      constexpr int TB = decltype(tbc)::value;
      const unsigned char* ebt = eb + TB * kNrMax * TREE;
      int H[GS];
#pragma unroll
      for (int j = 0; j < GS; ++j) {
        H[j] = G;
        in_vgpr(H[j]);
      }
#pragma unroll
      for (int l = 0; l < 6; ++l) {
        T e[GS];
#pragma unroll
        for (int j = 0; j < GS; ++j) e[j] = *reinterpret_cast<const T*>(ebt + j * TREE + H[j]);
#pragma unroll
        for (int j = 0; j < GS; ++j) H[j] = heap_step(H[j], e[j], dv[j], step0, step1);
      }
#pragma unroll
      for (int j = 0; j < GS; ++j) {
        // h = 64 + k, k in [0, 63], so H - G = SZ (63 + k) < GS TREE and G is a
        // multiple of GS TREE: S_63 (E[63] of the slot) is read at
        // (H & -(GS TREE)) + 63 SZ, an address computed from the search so that
        // the read stays with it (a constant LDS address would be hoisted out
        // of the cell loop into a register per slot)
        const T last = *reinterpret_cast<const T*>(ebt + j * TREE + (H[j] & -(GS * TREE)) + 63 * SZ);
        int k = static_cast<int>(static_cast<uint32_t>(H[j] - G) / SZ) - (kSortWidth - 1);
        k += static_cast<int>(k == kSortWidth - 1) & static_cast<int>(last <= dv[j]);
        const unsigned char* row =
            reinterpret_cast<const unsigned char*>(P + (TB * kNrMax + g * GS + j) * kMaskPitch);
        cur[j] = *reinterpret_cast<const uint64_t*>(row + static_cast<uint32_t>(k) * 8u);
      }
    };
    uint64_t cur[GS];
    search(std::integral_constant<int, 0>{}, cur);
    if constexpr (TWO) {
      // walkers whose interval of a slot ends below delta_R are not flagged by it
      uint64_t cuh[GS];
      search(std::integral_constant<int, 1>{}, cuh);
#pragma unroll
      for (int j = 0; j < GS; ++j) {
        acc |= pend[j] & ~pendh[j];
        pend[j] = cur[j];
        pendh[j] = cuh[j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < GS; ++j) {
        acc |= pend[j];
        pend[j] = cur[j];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < GS; ++j) acc |= TWO ? (pend[j] & ~pendh[j]) : pend[j];
  lo = static_cast<uint32_t>(acc);
  hi = static_cast<uint32_t>(acc >> 32);
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

// Waves per SIMD the compiler must leave room for in the FP32 ionisation pass
// at N = 128 and 256 (it then keeps the kernel within 512 / 6 = 85 VGPRs):
// measured on the 256^3, 64-walker workload, occupancy matters more there than
// the few spills it costs.  Other shapes are limited by LDS or block size
// before registers, and FP64 needs the registers.
template <typename T, int N>
constexpr int ion_waves_per_simd() {
  return (sizeof(T) == 4 && (N == 128 || N == 256)) ? 6 : 1;
}

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
// odens[cell] = (1 + delta) times the velocity-gradient factor of eq. (4)
// (or 1), computed once per box by k_los_factor.
// Each block owns row pairs (rows 2p, 2p+1 of the z-y plane stack); thread t
// owns cell (row 2p + t / N, x = t % N).  The smoothed values of its cell stay
// in registers while every walker of the group is processed, so the resident
// smoothed boxes are read once per group.  Two real rows are transformed as
// one complex row.  Output: spec[w][row][kx < N/2] (streaming stores), the
// Nyquist plane nyq[w][y][z], and per-block x_HI sums xpart[w][block].
// The x_HI sums are FP64 above the first level: each 16-lane row of a wave
// adds its 16 values in a 4-level pairwise FP32 tree (relative error at most
// 4 units of FP32 rounding for these non-negative terms), everything after
// that in double.
// FIELDS: walker fw of the group also writes its x_HI and dT_b boxes (fx, fd,
// N^3 values each) from the same per-cell values that enter its spectrum.
// (FP32 walkers with the sorted flag test, constant-efficiency and
// two-population, take k_ion_teams below instead.)
template <typename T, typename S, int N, bool TWO, bool FIELDS>
__global__ __launch_bounds__(IonShape<N>::NT, (ion_waves_per_simd<T, N>())) void k_ion_rows(
    const S* __restrict__ dR, const T* __restrict__ odens, int nr, const WalkerConst<T>* __restrict__ wc,
    const T* __restrict__ thr, const T* __restrict__ zt, int nw, T tb, T dc, cplx<T>* __restrict__ spec,
    cplx<T>* __restrict__ nyq, double* __restrict__ xpart, const cplx<T>* __restrict__ tw, int tstride, int fw,
    T* __restrict__ fx, T* __restrict__ fd) {
  using IS = IonShape<N>;
  constexpr size_t N3 = static_cast<size_t>(N) * N * N;
  constexpr size_t SPEC = static_cast<size_t>(N) * N * IS::HP;
  __shared__ cplx<T> lds[IS::WB * N];
  __shared__ cplx<T> twl[N];
  // x_HI partial sums of a batch: one per 16-lane row (NT >= 64) or per thread
  constexpr int NPS = IS::NT >= 64 ? IS::NT / 16 : IS::NT;
  __shared__ T wsum[IS::WB][NPS];
  __shared__ double acc[kMaxGroup];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int row = t / N, x = t % N;
  T* ldsr = reinterpret_cast<T*>(lds);
  for (int w = t; w < kMaxGroup; w += IS::NT) acc[w] = 0.0;
  load_twiddles<N>(twl, tw, tstride);
  const T tbh = T(0.5) * tb;
  for (long p = blockIdx.x; p < static_cast<long>(N) * N / 2; p += gridDim.x) {
    const size_t cell = static_cast<size_t>(2 * p + row) * N + x;
    // every slot's delta_R in registers for the walker loop
    T d[kNrMax];
    load_radii<T, S>(dR, N3, cell, nr, d);
    const T odh = tbh * odens[cell];   // dT_b per unit x_HI, at half scale
    const T u = dc - d[0];   // argument of the partial ionisation, per cell
    const T u2 = u * u;
    // Every delta_R of the cell is in its register before the walker loop:
    // otherwise the compiler, unable to see that the loads have landed after
    // the first walker, keeps one load-counter wait per radius inside the loop
    // for every walker (an empty asm taking the values, no instruction).
#pragma unroll
    for (int s = 0; s < kNrMax; ++s) asm volatile("" ::"v"(d[s]));
    for (int w0 = 0; w0 < nw; w0 += IS::WB) {
      const int qn = min(IS::WB, nw - w0);  // walkers in this batch; later slots are not written out
#pragma unroll 1
      for (int q = 0; q < qn; ++q) {
        const int w = w0 + q;
        const T xh = cell_xhi<T, kNrMax, TWO>(d, load_walker(wc + w),
                                              thr + static_cast<size_t>(w) * (TWO ? 2 : 1) * kNrMax,
                                              zt + static_cast<size_t>(w) * kZetaPitch, dc, u2);
        // dT_b at half scale (tbh = tb / 2): the unpacking after the
        // transform then needs no halving, with bitwise the same spectrum
        const T tvh = xh * odh;
        ldsr[2 * (q * N + x) + row] = tvh;
        if constexpr (FIELDS) {
          if (w == fw) {
            fx[cell] = xh;
            fd[cell] = tvh + tvh;   // dT_b at full scale (doubling is exact)
          }
        }
        if constexpr (IS::NT >= 64) {
          T s = row_sum(xh);
          in_vgpr(s);   // the last DPP step in every lane, fused with its add
          if ((lane & 15) == 0) wsum[q][t >> 4] = s;
        } else {
          wsum[q][t] = xh;
        }
      }
      __syncthreads();
      if (t < IS::WB && w0 + t < nw) {
        double s = 0.0;
        for (int k = 0; k < NPS; ++k) s += static_cast<double>(wsum[t][k]);
        acc[w0 + t] += s;
      }
      // each row's team lies within one wave: its stages synchronise only
      // there, the block before (above) and after
      fft_team<N, -1, T, typename IS::Plan, true>(lds + (t / IS::TS) * N, 1, t % IS::TS, twl, 1);
      __syncthreads();
      // kx < N/2: thread t takes kx = t mod N/2 of the batch's walkers
      // t / (N/2), + NT / (N/2), ... (a whole wave on one walker for N >= 128)
      {
        constexpr int HALF = N / 2;
        constexpr int QS = IS::NT / HALF;   // walkers per pass (4)
        static_assert(IS::NT % HALF == 0 && IS::WB % QS == 0, "unpack passes must tile the batch");
        const int k = t % HALF, q0 = t / HALF;
        cplx<T>* o = spec + static_cast<size_t>(w0 + q0) * SPEC + static_cast<size_t>(2 * p) * IS::HP + k;
#pragma unroll
        for (int i = 0; i < IS::WB / QS; ++i) {
          const int q = q0 + i * QS;
          if (w0 + q < nw) {
            cplx<T> A, B;
            unpack_pair2<N>(lds + q * N, k, A, B);
            store_stream(o + static_cast<size_t>(i) * QS * SPEC, A);
            store_stream(o + static_cast<size_t>(i) * QS * SPEC + IS::HP, B);
          }
        }
      }
      // the Nyquist column kx = N/2 of each walker, into its own plane
      if (t < IS::WB && w0 + t < nw) {
        cplx<T> A, B;
        unpack_pair2<N>(lds + t * N, N / 2, A, B);
        const size_t z = static_cast<size_t>(2 * p) / N, y = static_cast<size_t>(2 * p) % N;
        cplx<T>* o = nyq + (static_cast<size_t>(w0 + t) * N + y) * N + z;
        o[0] = A;
        o[N] = B;
      }
      __syncthreads();
    }
  }
  for (int w = t; w < nw; w += IS::NT) xpart[static_cast<size_t>(w) * gridDim.x + blockIdx.x] = acc[w];
}

// Sum over the TS lanes of each aligned team (TS a power of two <= 64), in
// every lane of the team, in a fixed order.
template <int TS, typename T>
__device__ __forceinline__ T team_sum(T v) {
  if constexpr (TS >= 16) {
    v = row_sum(v);
    if constexpr (TS >= 32) v += __shfl_xor(v, 16);
    if constexpr (TS >= 64) v += __shfl_xor(v, 32);
  } else {
#pragma unroll
    for (int o = TS / 2; o >= 1; o /= 2) v += __shfl_xor(v, o);
  }
  return v;
}

// Ionisation + dT_b + forward x pass for a group of FP32 walkers with the
// sorted flag test, organised around the x-pass FFT teams (TWO: two-population
// walkers, interval tables and the partial ionisation 1 - zeta_eff(t) erfc(t)
// from the walker's cell-radius table zt).
// Per row pair (rows 2p, 2p+1; one cell per thread) the block first finds
// each cell's walker mask (sorted_flags) and keeps it with u = delta_c -
// delta_cell and dT_b per unit x_HI in LDS.  Then for each batch of WB
// walkers, team q (TS consecutive threads, within one wave) takes walker
// w0 + q (the constants of a wave's walkers are scalar loads, one batch
// ahead): member j
// forms the packed row's elements j + r TS (r < R0) — the cells x = j + r TS
// of both rows — which are exactly its first-stage butterfly, so that stage
// runs in registers; the remaining stages, the unpacking into the half
// spectra and the stores are the team's own (wave-level synchronisation
// only), and so is the walker's x_HI sum: per thread a pairwise FP32 sum of
// its 2 R0 cells (relative error at most 4 units of FP32 rounding for these
// non-negative terms), then the team's sum in double.  Block barriers: two
// per row pair.  Results equal k_ion_rows' (same per-cell arithmetic and
// transform; the x_HI sums in another order).
template <int N, bool TWO>
constexpr int team_waves_per_simd() {
  return TWO && (N == 128 || N == 256) ? 4 : ion_waves_per_simd<float, N>();
}

template <typename S, int N, bool FIELDS, bool TWO>
__global__ __launch_bounds__(IonShape<N>::NT, (team_waves_per_simd<N, TWO>())) void k_ion_teams(
    const S* __restrict__ dR, const float* __restrict__ odens, int nr, const WalkerConst<float>* __restrict__ wc,
    int nw, float tb, float dc, cplx<float>* __restrict__ spec, cplx<float>* __restrict__ nyq,
    double* __restrict__ xpart, const cplx<float>* __restrict__ tw, int tstride, int fw, float* __restrict__ fx,
    float* __restrict__ fd, const float* __restrict__ Eg, const uint64_t* __restrict__ Pg,
    const float* __restrict__ zt) {
  using T = float;
  using IS = IonShape<N>;
  using P = FftShape<N, typename IS::Plan>;
  constexpr int TS = IS::TS, WB = IS::WB, R0 = P::R0, NT = IS::NT;
  static_assert(N / R0 == TS && WB * TS == NT && 32 % WB == 0, "teams of the x pass");
  static_assert((N / 2) % TS == 0, "the unpacking splits evenly over a team");
  constexpr size_t N3 = static_cast<size_t>(N) * N * N;
  constexpr size_t SPEC = static_cast<size_t>(N) * N * IS::HP;
  __shared__ cplx<T> lds[WB * N];
  __shared__ cplx<T> twl[N];
  __shared__ T El[(TWO ? 2 : 1) * kNrMax * kSortWidth];
  // per cell of the row pair: walker mask halves (walkers 0..31, 32..63),
  // u = delta_c - delta_cell and dT_b per unit x_HI at half scale, tb / 2
  // times (1 + delta) times the velocity factor
  __shared__ uint32_t cmask[2][NT];
  __shared__ T cu[NT], cod[NT];
  __shared__ double acc[kMaxGroup];
  const int t = threadIdx.x;
  const int row = t / N, x = t % N;   // the cell of the mask phase
  const int q = t / TS, j = t % TS;   // the team and member of the walker phase
  for (int e = t; e < (nr + 3) / 4 * 4 * kSortWidth; e += NT) {
    El[e] = Eg[e];
    if constexpr (TWO) El[kNrMax * kSortWidth + e] = Eg[kNrMax * kSortWidth + e];
  }
  for (int w = t; w < kMaxGroup; w += NT) acc[w] = 0.0;
  load_twiddles<N>(twl, tw, tstride);
  const T tbh = T(0.5) * tb;   // dT_b at half scale: the unpacking needs no halving
  cplx<T>* my = lds + q * N;   // the team's packed row
  // the team's walker in the batch starting at w0 (teams past the group's end
  // repeat its last walker)
  const auto walker_of = [&](int w0) { return min(w0 + q, nw - 1); };
  // The constants of the wave's TPW walkers are scalar loads (a wave-uniform
  // address), one batch ahead (the batch after a row pair's last is the next
  // row pair's first): their wait then counts no vector memory operation, so
  // that it does not wait for the previous batch's stores.  Each team then
  // takes its own walker's fields.
  constexpr int TPW = (NT < 64 ? NT : 64) / TS;   // teams per wave
  const int qw = __builtin_amdgcn_readfirstlane(q - q % TPW);   // the wave's first team
  const int qi = q % TPW;
  WalkerConst<T> cw[TPW];
  const auto load_wave = [&](int w0) {
#pragma unroll
    for (int i = 0; i < TPW; ++i) cw[i] = load_walker_partial(wc + min(w0 + qw + i, nw - 1));
  };
  load_wave(0);
  // the walker's dT_b at half scale of the team's cells (x = j + r TS of rows
  // 2p and 2p + 1), their packed row's entries, and its x_HI sum per thread;
  // PARTIAL: 2 when every walker of the wave takes the erfc form of the
  // partial ionisation (no per-cell branch on the form), -1 otherwise
  const auto cells = [&](auto partial, const WalkerConst<T>& cw, const uint32_t* cm, uint32_t bit, bool live,
                         int w, long p, cplx<T> (&v)[R0], T (&xs)[R0]) {
    constexpr int PARTIAL = decltype(partial)::value;
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int xx = j + r * TS;
      T xh2[2], tv2[2];
#pragma unroll
      for (int rr = 0; rr < 2; ++rr) {
        const int e = rr * N + xx;
        const T u = cu[e];
        T xh;
        if constexpr (PARTIAL == 2) {
          xh = T(0);
          if (!(cm[e] & bit)) xh = partial_xhi_pos(cw, u, u * u);
        } else if constexpr (TWO) {
          // the two-population form: 1 - zeta_eff(t) erfc(t), t = max(a u, 0)
          xh = T(1);
          if (cm[e] & bit) {
            xh = T(0);
          } else if (cw.partial) {
            const T tt = max(cw.a_cell * u, T(0));
            xh = T(1) - zeta_eff(zt + static_cast<size_t>(w) * kZetaPitch, tt) * erfc_t(tt);
          }
        } else {
          xh = T(1);
          if (cm[e] & bit)
            xh = T(0);
          else if (cw.partial)
            xh = partial_xhi(cw, u, u * u);
        }
        xh2[rr] = xh;
        tv2[rr] = xh * cod[e];
        if constexpr (FIELDS) {
          if (live && w == fw) {
            const size_t cell = static_cast<size_t>(2 * p + rr) * N + xx;
            fx[cell] = xh;
            fd[cell] = tv2[rr] + tv2[rr];   // dT_b at full scale (doubling is exact)
          }
        }
      }
      // dT_b rounded before the transform, as k_ion_rows stores it (no
      // multiply-add contraction into the first butterfly): the spectra
      // of the two kernels are bitwise equal
      in_vgpr(tv2[0]);
      in_vgpr(tv2[1]);
      v[r] = {tv2[0], tv2[1]};
      xs[r] = xh2[0] + xh2[1];
    }
  };
  for (long p = blockIdx.x; p < static_cast<long>(N) * N / 2; p += gridDim.x) {
    {
      const size_t cell = static_cast<size_t>(2 * p + row) * N + x;
      uint32_t mlo = 0, mhi = 0;
      sorted_flags<T, S, TWO>(dR, N3, cell, nr, El, Pg, mlo, mhi);
      const T d0 = load_as<T>(dR, static_cast<size_t>(nr - 1) * N3 + cell);
      cmask[0][t] = mlo;
      cmask[1][t] = mhi;
      cu[t] = dc - d0;
      cod[t] = tbh * odens[cell];
    }
    __syncthreads();
    for (int w0 = 0; w0 < nw; w0 += WB) {
      // waves whose teams all lie past the group's end skip the batch (a
      // wave-uniform branch); in a wave with a live team, teams past the end
      // repeat the group's last walker and store nothing, keeping to the
      // wave-level synchronisation
      const int wn0 = w0 + WB < nw ? w0 + WB : 0;   // the next batch
      if (w0 + qw >= nw) {
        load_wave(wn0);
        continue;
      }
      const int w = walker_of(w0);
      const bool live = w0 + q < nw;
      const uint32_t* cm = cmask[w0 < 32 ? 0 : 1];   // a batch lies within one half
      const uint32_t bit = 1u << (w & 31);
      cplx<T> v[R0];
      T xs[R0];
      WalkerConst<T> c = cw[0];
#pragma unroll
      for (int i = 1; i < TPW; ++i)
        if (qi == i) c = cw[i];
      // a wave-uniform choice of the per-cell form
      bool all2 = true;
#pragma unroll
      for (int i = 0; i < TPW; ++i) all2 = all2 && cw[i].partial == 2;
      if (!TWO && all2)
        cells(std::integral_constant<int, 2>{}, c, cm, bit, live, w, p, v, xs);
      else
        cells(std::integral_constant<int, -1>{}, c, cm, bit, live, w, p, v, xs);
      // the walker's x_HI partial sum: pairwise over the thread's values, then the team
#pragma unroll
      for (int h = R0 / 2; h >= 1; h /= 2)
#pragma unroll
        for (int r = 0; r < h; ++r) xs[r] += xs[r + h];
      const double tot = team_sum<TS>(static_cast<double>(xs[0]));
      if (live && j == 0) acc[w] += tot;
      // the packed row's transform, the team alone
      fft_first_from_regs<N, -1, T, typename IS::Plan>(v, my, 1, j);
      fft_rest<N, -1, T, typename IS::Plan, true>(my, 1, j, twl, 1);
      load_wave(wn0);   // in flight during the unpacking and stores
      if (live) {
        cplx<T>* o = spec + static_cast<size_t>(w) * SPEC + static_cast<size_t>(2 * p) * IS::HP;
#pragma unroll
        for (int i = 0; i < (N / 2) / TS; ++i) {
          const int k = j + i * TS;
          cplx<T> A, B;
          unpack_pair2<N>(my, k, A, B);
          store_stream(o + k, A);
          store_stream(o + IS::HP + k, B);
        }
        if (j == 0) {   // the Nyquist column kx = N/2, into its own plane
          cplx<T> A, B;
          unpack_pair2<N>(my, N / 2, A, B);
          const size_t z = static_cast<size_t>(2 * p) / N, y = static_cast<size_t>(2 * p) % N;
          cplx<T>* on = nyq + (static_cast<size_t>(w) * N + y) * N + z;
          on[0] = A;
          on[N] = B;
        }
      }
      stage_sync<true>();   // the team's row is read before the next batch writes it
    }
    __syncthreads();   // the cell values are read before the next row pair writes them
  }
  for (int w = t; w < nw; w += NT) xpart[static_cast<size_t>(w) * gridDim.x + blockIdx.x] = acc[w];
}

// Per-cell density factor of dT_b (Section 2.2, eq. 4): odens = (1 + delta) /
// (1 + t), t = dv_r/dr / H = -g limited to [-tmax, tmax], with g the
// line-of-sight gradient field (g == nullptr: odens = 1 + delta).
template <typename T>
__global__ __launch_bounds__(256) void k_los_factor(const T* __restrict__ delta, const T* __restrict__ g,
                                                    T* __restrict__ odens, size_t count, T tmax) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < count;
       i += static_cast<size_t>(gridDim.x) * 256) {
    T f = T(1);
    if (g) f = T(1) / (T(1) + min(max(-g[i], -tmax), tmax));
    odens[i] = (T(1) + delta[i]) * f;
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

// y[i] = erfc(x[i]) by the FP32 routine of the ionisation pass.
__global__ __launch_bounds__(256) void k_erfc(const float* __restrict__ x, float* __restrict__ y, size_t n) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += static_cast<size_t>(gridDim.x) * 256)
    y[i] = erfc_fast(x[i]);
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

// Blocks of the grid-stride pipelined passes: several resident blocks per CU,
// each working through many tiles.  (The CPU emulation used by the tests
// builds with a tiny value so that every block walks through several items.)
#ifndef XS21_PIPE_BLOCKS
#define XS21_PIPE_BLOCKS 2048
#endif
constexpr long kPipeBlocks = XS21_PIPE_BLOCKS;
constexpr long kIonBlocksMax = 16384;   // largest ionisation grid a launch may ask for

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

// Tiles of the binning pass with at least one column (ky, kx) inside the
// disk ny^2 + kx^2 <= (n/2)^2, in increasing order.
std::vector<int32_t> bins_live_tiles(int n) {
  std::vector<int32_t> out;
  (void)with_n(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    using BT = BinTiles<N, BinShape<N>::TI>;
    constexpr int G = BinShape<N>::G;
    // whole groups of G tiles (the halves of one line stay together)
    for (long t0 = 0; t0 < BT::COUNT; t0 += G) {
      bool live = false;
      for (long t = t0; t < t0 + G && t < BT::COUNT && !live; ++t)
        for (int cc = 0; cc < BinShape<N>::TI && !live; ++cc) {
          int ky, kx;
          BT::column(t, cc, ky, kx);
          const int ny = ky < N / 2 ? ky : ky - N;
          live = ky >= 0 && ny * ny + kx * kx <= (N / 2) * (N / 2);
        }
      if (live)
        for (long t = t0; t < t0 + G && t < BT::COUNT; ++t) out.push_back(static_cast<int32_t>(t));
    }
    return hipSuccess;
  });
  return out;
}

long bins_live_count(int n) {
  static long cache[10] = {};
  int l = 0;
  while ((1 << l) < n) ++l;
  if (l < 10 && cache[l] == 0) cache[l] = static_cast<long>(bins_live_tiles(n).size());
  return l < 10 ? cache[l] : 0;
}

// Blocks per spectrum of the binning pass: enough blocks over `outer`
// spectra to fill the chip, each walking every parts-th live tile.
long bins_parts(int n, long outer, long blocks) {
  const long count = bins_live_count(n);
  const long target = blocks > 0 ? blocks : kPipeBlocks;
  const long k = (target + outer - 1) / outer;
  return k < 1 ? 1 : (k > count ? count : k);
}

// LDS budget of one binning block (static tile + twiddles + FP64 slots).
// (The CPU emulation used by the tests lowers it so that FP64 at N = 16 takes
// several launches.)
#ifndef XS21_BINS_LDS_BUDGET
#define XS21_BINS_LDS_BUDGET 131072
#endif

// Slot rows for bins [b0, b1) at size N with M = N / TS outputs per team
// member: member j outputs kz in [j M, j M + M), so none of its modes lies
// below the bin of min |nz|^2 over that range (|n|^2 >= nz^2; the DC mode is
// never binned, so at least 1).
template <int N, int TS>
BinSlots bin_slots(const int8_t* bintab_host, int b0, int b1) {
  constexpr int M = N / TS;
  BinSlots bs{};
  int rows = 0;
  for (int j = 0; j < TS; ++j) {
    int nzmin = N;
    for (int kz = j * M; kz < j * M + M; ++kz) {
      const int nz = kz < N / 2 ? kz : N - kz;
      nzmin = nz < nzmin ? nz : nzmin;
    }
    const int n2 = nzmin * nzmin > 0 ? nzmin * nzmin : 1;
    int lo = bintab_host[n2];
    lo = lo > b0 ? lo : b0;
    bs.lo[j] = static_cast<int16_t>(lo);
    bs.base[j] = static_cast<int16_t>(rows);
    rows += b1 > lo ? b1 - lo : 0;
  }
  bs.rows = rows;
  return bs;
}

long bins_tiles(int n) {
  long count = 0;
  (void)with_n(n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    count = BinTiles<N, BinShape<N>::TI>::COUNT;
    return hipSuccess;
  });
  return count;
}

// Blocks of the ionisation pass: many short blocks (4 row pairs each at
// N = 256) finish in near-even rounds; a grid of only the resident blocks
// measured slower (row locality of the blocks running together), a finer one
// no faster and with more x_HI partial sums to reduce.
// Default grid of the ionisation pass (the CPU emulation used by the tests
// builds with a tiny value so that every block walks many row pairs).
#ifndef XS21_ION_BLOCKS
#define XS21_ION_BLOCKS 8192
#endif
int ion_grid(int n, int blocks) {
  return static_cast<int>(grid_for(static_cast<long>(n) * n / 2, blocks > 0 ? blocks : XS21_ION_BLOCKS));
}
int ion_grid_max(int n) { return static_cast<int>(grid_for(static_cast<long>(n) * n / 2, kIonBlocksMax)); }

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

hipError_t launch_rows_r2c(int dtype, int n, const void* in, void* out, void* nyq, long nrows, const void* tw,
                           int ntab, hipStream_t s) {
  if (nyq && nrows != static_cast<long>(n) * n) return hipErrorInvalidValue;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_n(n, [&](auto nc) {
      constexpr int N = decltype(nc)::value;
      const long npairs = nrows / 2;
      const long groups = (npairs + RowShape<N>::WB - 1) / RowShape<N>::WB;
      hipLaunchKernelGGL((k_rows_r2c<T, N>), dim3(grid_for(groups, 8192)), dim3(RowShape<N>::NT), 0, s,
                         static_cast<const T*>(in), static_cast<cplx<T>*>(out), static_cast<cplx<T>*>(nyq),
                         npairs, static_cast<const cplx<T>*>(tw), ntab / N);
      return hipGetLastError();
    });
  });
}

hipError_t launch_rows_c2r(int dtype, int storage, int n, const void* in, void* out, long nrows, double scale,
                           const long* cut, int batch, long istride, long ostride, const void* tw, int ntab,
                           hipStream_t s, int blocks) {
  if (batch < 1 || batch > 65535) return hipErrorInvalidValue;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_storage<T>(storage, [&](auto sv) {
      using ST = decltype(sv);
      return with_n(n, [&](auto nc) {
        constexpr int N = decltype(nc)::value;
        const long npairs = nrows / 2;
        const long items = (npairs + RowShape<N>::WB - 1) / RowShape<N>::WB * batch;
        hipLaunchKernelGGL((k_rows_c2r<T, ST, N>), dim3(grid_for(items, blocks > 0 ? blocks : kPipeBlocks)),
                           dim3(RowShape<N>::NT), 0, s,
                           static_cast<const cplx<T>*>(in), static_cast<ST*>(out), npairs, items,
                           static_cast<T>(scale), cut, istride, ostride, static_cast<const cplx<T>*>(tw), ntab / N);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_axis(int dtype, int n, int dir, int mode, const void* src, void* dst, long outer, long inner,
                       long ilim, const long* cut, int batch, long sstride, long dstride, const void* tw, int ntab,
                       hipStream_t s) {
  if (ilim < 1 || ilim > inner || mode < 0 || mode > 4 || mode == 3 || ((mode == 1 || mode == 2) && !cut) ||
      batch < 1 || batch > 65535 || outer > 65535 || (mode == 4 && dir < 0))
    return hipErrorInvalidValue;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_n(n, [&](auto nc) {
      constexpr int N = decltype(nc)::value;
      using A = AxisShape<N>;
      const dim3 grid(static_cast<unsigned>((ilim + A::TI - 1) / A::TI), static_cast<unsigned>(outer),
                      static_cast<unsigned>(batch));
      const auto* sp = static_cast<const cplx<T>*>(src);
      auto* dp = static_cast<cplx<T>*>(dst);
      const auto* tp = static_cast<const cplx<T>*>(tw);
      const int ts = ntab / N;
      if (dir < 0) {
        // forward: when the last column sits alone in its tile (the Nyquist
        // column of a half spectrum), full tiles go first and that column of
        // every slice is gathered TI slices per block
        const long full = ilim / A::TI * A::TI;
        if (mode == 0 && batch == 1 && ilim - full <= 1 && full > 0) {
          const long ntiles = full / A::TI * outer;
          hipLaunchKernelGGL((k_axis_pipe<T, N, -1>), dim3(grid_for(ntiles, kPipeBlocks)), dim3(A::NT), 0, s, sp, dp,
                             inner, full / A::TI, ntiles, tp, ts);
          if (ilim > full) {
            const dim3 g2(static_cast<unsigned>((outer + A::TI - 1) / A::TI), 1, 1);
            hipLaunchKernelGGL((k_axis<T, N, -1, 3>), g2, dim3(A::NT), 0, s, sp, dp, inner, ilim, cut, sstride,
                               dstride, outer, tp, ts, nullptr, 0);
          }
        } else {
          hipLaunchKernelGGL((k_axis<T, N, -1, 0>), grid, dim3(A::NT), 0, s, sp, dp, inner, ilim, cut, sstride,
                             dstride, outer, tp, ts, nullptr, 0);
        }
      } else if (mode == 1) {
        hipLaunchKernelGGL((k_axis<T, N, +1, 1>), grid, dim3(A::NT), 0, s, sp, dp, inner, ilim, cut, sstride, dstride,
                           outer, tp, ts, nullptr, 0);
      } else if (mode == 2) {
        hipLaunchKernelGGL((k_axis<T, N, +1, 2>), grid, dim3(A::NT), 0, s, sp, dp, inner, ilim, cut, sstride, dstride,
                           outer, tp, ts, nullptr, 0);
      } else if (mode == 4) {
        hipLaunchKernelGGL((k_axis<T, N, +1, 4>), grid, dim3(A::NT), 0, s, sp, dp, inner, ilim, cut, sstride, dstride,
                           outer, tp, ts, nullptr, 0);
      } else {
        hipLaunchKernelGGL((k_axis<T, N, +1, 0>), grid, dim3(A::NT), 0, s, sp, dp, inner, ilim, cut, sstride, dstride,
                           outer, tp, ts, nullptr, 0);
      }
      return hipGetLastError();
    });
  });
}

hipError_t launch_axis_fwd_disk(int dtype, int n, void* data, long outer, long inner, long ilim, bool nyquist,
                                const void* tw, int ntab, hipStream_t s, int blocks) {
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_n(n, [&](auto nc) {
      constexpr int N = decltype(nc)::value;
      using A = AxisShape<N>;
      if (ilim < 1 || ilim > inner || ilim % A::TI != 0 || outer < 1)   // not whole tiles: the plain pass
        return launch_axis(dtype, n, -1, 0, data, data, outer, inner, ilim, nullptr, 1, 0, 0, tw, ntab, s);
      const long ntiles = ilim / A::TI * outer;
      const unsigned grid = grid_for(ntiles, blocks > 0 ? blocks : kPipeBlocks);
      auto* dp = static_cast<cplx<T>*>(data);
      if (nyquist)
        hipLaunchKernelGGL((k_axis_pipe<T, N, -1, 2>), dim3(grid), dim3(A::NT), 0, s, dp, dp, inner, ilim / A::TI,
                           ntiles, static_cast<const cplx<T>*>(tw), ntab / N);
      else
        hipLaunchKernelGGL((k_axis_pipe<T, N, -1, 1>), dim3(grid), dim3(A::NT), 0, s, dp, dp, inner, ilim / A::TI,
                           ntiles, static_cast<const cplx<T>*>(tw), ntab / N);
      return hipGetLastError();
    });
  });
}

int bins_tile_cols(int n) {
  int ti = 0;
  (void)with_n(n, [&](auto nc) {
    ti = BinShape<decltype(nc)::value>::TI;
    return hipSuccess;
  });
  return ti;
}

int axis_tile_cols(int n) {
  int ti = 0;
  (void)with_n(n, [&](auto nc) {
    ti = AxisShape<decltype(nc)::value>::TI;
    return hipSuccess;
  });
  return ti;
}

hipError_t launch_axis_live(int dtype, int n, const void* src, void* dst, long inner, const int32_t* tiles,
                            long ntiles, int r0, const long* cut, long dstride, const void* tw, int ntab,
                            hipStream_t s) {
  if (ntiles < 1 || ntiles > 0x7fffffffL || !tiles || !cut || r0 < 0) return hipErrorInvalidValue;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_n(n, [&](auto nc) {
      constexpr int N = decltype(nc)::value;
      using A = AxisShape<N>;
      hipLaunchKernelGGL((k_axis<T, N, +1, 5>), dim3(static_cast<unsigned>(ntiles)), dim3(A::NT), 0, s,
                         static_cast<const cplx<T>*>(src), static_cast<cplx<T>*>(dst), inner, inner, cut, 0L, dstride,
                         1L, static_cast<const cplx<T>*>(tw), ntab / N, tiles, r0);
      return hipGetLastError();
    });
  });
}

hipError_t launch_axis_live_y(int dtype, int n, void* data, long inner, long ilim, const int32_t* tiles, long ntiles,
                              int r0, const long* cut, long stride, const void* tw, int ntab, hipStream_t s) {
  if (ntiles < 1 || ntiles > 0x7fffffffL || !tiles || !cut || r0 < 0 || ilim < 1 || ilim > inner)
    return hipErrorInvalidValue;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_n(n, [&](auto nc) {
      constexpr int N = decltype(nc)::value;
      using A = AxisShape<N>;
      auto* dp = static_cast<cplx<T>*>(data);
      hipLaunchKernelGGL((k_axis<T, N, +1, 6>), dim3(static_cast<unsigned>(ntiles), static_cast<unsigned>(N)),
                         dim3(A::NT), 0, s, dp, dp, inner, ilim, cut, stride, stride, 1L,
                         static_cast<const cplx<T>*>(tw), ntab / N, tiles, r0);
      return hipGetLastError();
    });
  });
}

hipError_t launch_axis_bins(int dtype, int n, const void* src, const void* nyq, long outer, long parts,
                            const int32_t* tiles, long ntiles, const int8_t* bintab, const int8_t* bintab_host,
                            int nbins, double* part, const void* tw, int ntab, hipStream_t s) {
  if (nbins < 1 || nbins > kMaxBins || outer < 1 || outer > 65535 || ntiles < 1 || ntiles > bins_tiles(n) ||
      parts < 1 || parts > ntiles || !bintab_host || !tiles)
    return hipErrorInvalidValue;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_n(n, [&](auto nc) {
      constexpr int N = decltype(nc)::value;
      using A = BinShape<N>;
      constexpr long stat = (static_cast<long>(N) * A::TI + N) * static_cast<long>(sizeof(cplx<T>));
      const auto slot_bytes = [](const BinSlots& bs) { return static_cast<long>(bs.rows) * A::TI * 8; };
      hipError_t e = hipSuccess;
      for (int b0 = 0; b0 < nbins && e == hipSuccess;) {
        // the widest bin range [b0, b1) whose slots fit the budget (at least one bin)
        int b1 = b0 + 1;
        BinSlots bs = bin_slots<N, A::TS>(bintab_host, b0, b1);
        while (b1 < nbins) {
          const BinSlots wider = bin_slots<N, A::TS>(bintab_host, b0, b1 + 1);
          if (stat + slot_bytes(wider) > XS21_BINS_LDS_BUDGET) break;
          bs = wider;
          ++b1;
        }
        hipLaunchKernelGGL((k_axis_bins<T, N>), dim3(static_cast<unsigned>(outer * parts)), dim3(A::NT),
                           static_cast<size_t>(slot_bytes(bs)), s, static_cast<const cplx<T>*>(src),
                           static_cast<const cplx<T>*>(nyq), parts, tiles, ntiles, bintab, nbins, b0, b1 - b0, bs,
                           part, static_cast<const cplx<T>*>(tw), ntab / N);
        e = hipGetLastError();
        b0 = b1;
      }
      return e;
    });
  });
}

// Flag test of the constant-efficiency FP32 ionisation pass: the sorted
// tables (default) or one compare per walker and radius (XS21_ION_FLAGS =
// "ballot"), read once.
bool ion_sorted_default() {
  static const bool v = [] {
    const char* e = std::getenv("XS21_ION_FLAGS");
    return !(e && std::strcmp(e, "ballot") == 0);
  }();
  return v;
}

size_t slot_table_bytes() {
  // E: two FP32 sets in the space of one FP64 set; P: two sets
  return static_cast<size_t>(kNrMax) * kSortWidth * sizeof(double) +
         2 * static_cast<size_t>(kNrMax) * kMaskPitch * sizeof(uint64_t);
}

hipError_t launch_ion(int dtype, int storage, int n, const void* dR, const void* odens, int nr, const void* wc,
                      const void* thr, const void* zt, int nw, double tb, double dc, void* spec, void* nyq,
                      double* xpart, const void* tw, int ntab, hipStream_t s, int field_walker, void* x_hi,
                      void* dtb, void* slot_tab, int blocks, int flag_test) {
  if (nr < 1 || nr > kNrMax || nw < 1 || nw > kMaxGroup || blocks > kIonBlocksMax) return hipErrorInvalidValue;
  const bool fields = field_walker >= 0;
  if (fields && (field_walker >= nw || !x_hi || !dtb)) return hipErrorInvalidValue;
  const bool want_sorted = flag_test < 0 ? ion_sorted_default() : flag_test == 1;
  const bool sorted = slot_tab && dtype == kF32 && want_sorted;
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    return with_storage<T>(storage, [&](auto sv) {
      using ST = decltype(sv);
      return with_n(n, [&](auto nc) {
        constexpr int N = decltype(nc)::value;
        T* E = static_cast<T*>(slot_tab);
        uint64_t* P = reinterpret_cast<uint64_t*>(static_cast<unsigned char*>(slot_tab) +
                                                  static_cast<size_t>(kNrMax) * kSortWidth * sizeof(double));
        auto go = [&](auto two, auto withf) {
          hipLaunchKernelGGL((k_ion_rows<T, ST, N, decltype(two)::value, decltype(withf)::value>),
                             dim3(ion_grid(N, blocks)), dim3(IonShape<N>::NT), 0, s, static_cast<const ST*>(dR),
                             static_cast<const T*>(odens), nr, static_cast<const WalkerConst<T>*>(wc),
                             static_cast<const T*>(thr), static_cast<const T*>(zt), nw, static_cast<T>(tb),
                             static_cast<T>(dc), static_cast<cplx<T>*>(spec), static_cast<cplx<T>*>(nyq), xpart,
                             static_cast<const cplx<T>*>(tw), ntab / N, field_walker, static_cast<T*>(x_hi),
                             static_cast<T*>(dtb));
          return hipGetLastError();
        };
        if (sorted) {   // FP32 only (see `sorted` above)
          const int sets = zt ? 2 : 1;   // two-population walkers: intervals
          hipLaunchKernelGGL((k_slot_tables<T>), dim3(static_cast<unsigned>(sets * kNrMax)), dim3(kSortWidth), 0, s,
                             static_cast<const T*>(thr), sets * kNrMax, nw, E, P);
          hipError_t e = hipGetLastError();
          if (e != hipSuccess) return e;
          if constexpr (std::is_same<T, float>::value) {
            const auto teams = [&](auto withf, auto two) {
              hipLaunchKernelGGL((k_ion_teams<ST, N, decltype(withf)::value, decltype(two)::value>),
                                 dim3(ion_grid(N, blocks)),
                                 dim3(IonShape<N>::NT), 0, s, static_cast<const ST*>(dR),
                                 static_cast<const T*>(odens), nr, static_cast<const WalkerConst<T>*>(wc), nw,
                                 static_cast<T>(tb), static_cast<T>(dc), static_cast<cplx<T>*>(spec),
                                 static_cast<cplx<T>*>(nyq), xpart, static_cast<const cplx<T>*>(tw), ntab / N,
                                 field_walker, static_cast<T*>(x_hi), static_cast<T*>(dtb),
                                 static_cast<const T*>(E), static_cast<const uint64_t*>(P),
                                 static_cast<const T*>(zt));
              return hipGetLastError();
            };
            if (zt) return fields ? teams(std::true_type{}, std::true_type{}) : teams(std::false_type{}, std::true_type{});
            return fields ? teams(std::true_type{}, std::false_type{}) : teams(std::false_type{}, std::false_type{});
          }
        }
        if (zt) return fields ? go(std::true_type{}, std::true_type{}) : go(std::true_type{}, std::false_type{});
        return fields ? go(std::false_type{}, std::true_type{}) : go(std::false_type{}, std::false_type{});
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

hipError_t launch_los_factor(int dtype, const void* delta, const void* g, void* odens, size_t count, double tmax,
                             hipStream_t s) {
  return with_real(dtype, [&](auto tv) {
    using T = decltype(tv);
    hipLaunchKernelGGL((k_los_factor<T>), dim3(grid_for(static_cast<long>((count + 255) / 256), 16384)), dim3(256), 0,
                       s, static_cast<const T*>(delta), static_cast<const T*>(g), static_cast<T*>(odens), count,
                       static_cast<T>(tmax));
    return hipGetLastError();
  });
}

hipError_t launch_erfc(const float* x, float* y, size_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_erfc, dim3(grid_for(static_cast<long>((count + 255) / 256), 4096)), dim3(256), 0, s, x, y,
                     count);
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
