// Radix-2^k FFT building blocks for gfx950: register DFTs of size 2..16 and
// in-place Stockham stages over LDS, executed by "teams" of threads.
//
// A team of TS = N / RMAX threads transforms one sequence of N complex points
// that sits in LDS with element stride `es`.  Each stage of radix R reads R
// points per butterfly (stride N/R), applies the inter-stage twiddles, runs the
// register DFT and writes the results back in autosorted (Stockham) order, so
// the output is in natural order with no bit reversal.  Twiddles come from a
// table tw[m] = exp(-2 pi i m / NTAB) built on the host in FP64 and rounded
// once to T; stage twiddle exponents are exact integers.
#pragma once

#include <utility>

#include "common.hpp"

namespace xs21 {

// Radix plan per transform length: up to three stages; RMAX = largest radix.
template <int N>
struct FftPlan;
template <> struct FftPlan<8>   { static constexpr int R0 = 8,  R1 = 1,  R2 = 1; };
template <> struct FftPlan<16>  { static constexpr int R0 = 16, R1 = 1,  R2 = 1; };
template <> struct FftPlan<32>  { static constexpr int R0 = 8,  R1 = 4,  R2 = 1; };
template <> struct FftPlan<64>  { static constexpr int R0 = 8,  R1 = 8,  R2 = 1; };
template <> struct FftPlan<128> { static constexpr int R0 = 16, R1 = 8,  R2 = 1; };
template <> struct FftPlan<256> { static constexpr int R0 = 16, R1 = 16, R2 = 1; };
template <> struct FftPlan<512> { static constexpr int R0 = 8,  R1 = 8,  R2 = 8; };

// A radix plan: three stages (radix 1 = unused).
template <int A, int B, int C>
struct Radices {
  static constexpr int R0 = A, R1 = B, R2 = C;
};

template <int N, typename P = FftPlan<N>>
struct FftShape {
  static constexpr int R0 = P::R0, R1 = P::R1, R2 = P::R2;
  static constexpr int RMAX = R0 > R1 ? (R0 > R2 ? R0 : R2) : (R1 > R2 ? R1 : R2);
  static constexpr int TS = N / RMAX;  // threads per transform (team size)
  static_assert(R0 * R1 * R2 == N, "radix plan does not multiply to N");
};

// cos and sin of 2 pi k / 16, k in [0, 16).
__host__ __device__ constexpr double cos16(int k) {
  constexpr double c1 = 0.92387953251128675613, c2 = 0.70710678118654752440, c3 = 0.38268343236508977173;
  switch (k & 15) {
    case 0: return 1.0;   case 1: return c1;   case 2: return c2;   case 3: return c3;
    case 4: return 0.0;   case 5: return -c3;  case 6: return -c2;  case 7: return -c1;
    case 8: return -1.0;  case 9: return -c1;  case 10: return -c2; case 11: return -c3;
    case 12: return 0.0;  case 13: return c3;  case 14: return c2;  default: return c1;
  }
}
__host__ __device__ constexpr double sin16(int k) { return cos16(k - 4); }

// x * exp(DIR * 2 pi i K / M), M in {2, 4, 8, 16}; DIR = -1 forward, +1 inverse.
template <int DIR, int K, int M, typename T>
__host__ __device__ __forceinline__ cplx<T> rot(cplx<T> x) {
  constexpr int k = ((K % M) + M) % M;
  constexpr int k16 = k * (16 / M);
  if constexpr (k == 0) {
    return x;
  } else if constexpr (2 * k == M) {
    return {-x.x, -x.y};
  } else if constexpr (4 * k == M) {  // multiply by DIR * i
    return DIR > 0 ? cplx<T>{-x.y, x.x} : cplx<T>{x.y, -x.x};
  } else if constexpr (4 * k == 3 * M) {  // multiply by -DIR * i
    return DIR > 0 ? cplx<T>{x.y, -x.x} : cplx<T>{-x.y, x.x};
  } else {
    constexpr double c = cos16(k16);
    constexpr double s = DIR * sin16(k16);
    if constexpr (k16 == 2 || k16 == 6 || k16 == 10 || k16 == 14) {
      // |c| = |s| = sqrt(1/2): (c x.x - s x.y, c x.y + s x.x) with one scale
      constexpr double sg = (c > 0) == (s > 0) ? 1.0 : -1.0;  // s = sg * c
      const T cc = static_cast<T>(c);
      return {cc * (x.x - static_cast<T>(sg) * x.y), cc * (x.y + static_cast<T>(sg) * x.x)};
    } else {
      const T cc = static_cast<T>(c), ss = static_cast<T>(s);
      return {cc * x.x - ss * x.y, cc * x.y + ss * x.x};
    }
  }
}

template <int R, int DIR, typename T>
struct Dft;

template <int DIR, typename T>
struct Dft<1, DIR, T> {
  __host__ __device__ __forceinline__ static void run(cplx<T>*) {}
};

// Radix-2 decimation in time on registers: v[k] = sum_n v[n] exp(DIR 2 pi i n k / R).
template <int R, int DIR, typename T>
struct Dft {
  template <int... K>
  __host__ __device__ __forceinline__ static void combine(cplx<T>* v, const cplx<T>* e, const cplx<T>* o,
                                                          std::integer_sequence<int, K...>) {
    ((v[K] = cadd(e[K], rot<DIR, K, R>(o[K])), v[K + R / 2] = csub(e[K], rot<DIR, K, R>(o[K]))), ...);
  }
  __host__ __device__ __forceinline__ static void run(cplx<T>* v) {
    cplx<T> e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    Dft<R / 2, DIR, T>::run(e);
    Dft<R / 2, DIR, T>::run(o);
    combine(v, e, o, std::make_integer_sequence<int, R / 2>{});
  }
};

// Twiddle exp(DIR 2 pi i m / N) from the forward table of length ntab.
template <int DIR, typename T>
__device__ __forceinline__ cplx<T> twiddle(const cplx<T>* __restrict__ tw, int m, int tstride) {
  cplx<T> w = tw[m * tstride];
  if constexpr (DIR > 0) w.y = -w.y;
  return w;
}

// Synchronisation between the reads and writes of a stage: the whole block,
// or (WAVE) only the compiler's ordering within the wave.  WAVE holds when
// every team lies within one wave and only its team touches a sequence: the
// lanes of a wave issue each LDS instruction together and LDS executes one
// wave's instructions in order, so a lane reads what another lane of its wave
// wrote before, and the wave's reads of a stage precede its writes.
template <bool WAVE>
__device__ __forceinline__ void stage_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One Stockham stage of radix R after spans of length NS are complete.
// Butterflies b = j, j + TS, ... (N/R of them); results overwrite buf in place,
// so the stage reads everything into registers, synchronises, then writes.
template <int N, int R, int NS, int DIR, typename T, int TS, bool WAVE = false>
__device__ __forceinline__ void stockham_stage(cplx<T>* buf, int es, int j, const cplx<T>* __restrict__ tw,
                                               int tstride) {
  static_assert(!WAVE || (TS <= 64 && 64 % TS == 0), "wave-level stages need teams within one wave");
  constexpr int NB = N / R;          // butterflies in this stage
  constexpr int BPT = NB / TS;       // butterflies per thread
  static_assert(NB % TS == 0, "team size must divide the butterfly count");
  cplx<T> v[BPT][R];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = j + q * TS;
#pragma unroll
    for (int r = 0; r < R; ++r) v[q][r] = buf[(b + r * NB) * es];
    if constexpr (NS > 1) {
      const int k = b % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], twiddle<DIR>(tw, r * k * (N / (NS * R)), tstride));
    }
    Dft<R, DIR, T>::run(v[q]);
  }
  stage_sync<WAVE>();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = j + q * TS;
    const int o = (b / NS) * NS * R + (b % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) buf[(o + r * NS) * es] = v[q][r];
  }
  stage_sync<WAVE>();
}

// The first stage from registers, in two calls.  fft_first_from_regs: the
// caller already holds its butterfly's inputs v[r] = x[j + r N/R0] (team
// member j; one butterfly per member, i.e. TS = N / R0); the stage transforms
// them and writes the outputs to buf (the caller has synchronised the block
// if buf may still be in use).  fft_rest: synchronises the block and runs
// the remaining stages.  Between the two the caller may reuse v's registers
// (say, for the next loads).
template <int N, int DIR, typename T, typename Plan = FftPlan<N>>
__device__ __forceinline__ void fft_first_from_regs(cplx<T> (&v)[Plan::R0], cplx<T>* buf, int es, int j) {
  using P = FftShape<N, Plan>;
  static_assert(N / P::R0 == P::TS, "one first-stage butterfly per team member");
  Dft<P::R0, DIR, T>::run(v);
  // autosorted output of butterfly b = j with spans of 1: positions j R0 + r
#pragma unroll
  for (int r = 0; r < P::R0; ++r) buf[(j * P::R0 + r) * es] = v[r];
}
template <int N, int DIR, typename T, typename Plan = FftPlan<N>, bool WAVE = false>
__device__ __forceinline__ void fft_rest(cplx<T>* buf, int es, int j, const cplx<T>* __restrict__ tw, int tstride) {
  using P = FftShape<N, Plan>;
  stage_sync<WAVE>();
  if constexpr (P::R1 > 1) stockham_stage<N, P::R1, P::R0, DIR, T, P::TS, WAVE>(buf, es, j, tw, tstride);
  if constexpr (P::R2 > 1) stockham_stage<N, P::R2, P::R0 * P::R1, DIR, T, P::TS, WAVE>(buf, es, j, tw, tstride);
}

// Full length-N transform of the sequence buf[0], buf[es], ..., buf[(N-1) es]
// by team member j in [0, TS).  Every thread of the block must call this
// (it synchronises the block); data must be in LDS and visible on entry.
// DIR = -1: X[k] = sum_n x[n] exp(-2 pi i n k / N); DIR = +1: unnormalised inverse.
// WAVE: the team lies within one wave and synchronises only there (the
// caller synchronises the block before and after, as its data needs).
template <int N, int DIR, typename T, typename Plan = FftPlan<N>, bool WAVE = false>
__device__ __forceinline__ void fft_team(cplx<T>* buf, int es, int j, const cplx<T>* __restrict__ tw,
                                         int tstride) {
  using P = FftShape<N, Plan>;
  stockham_stage<N, P::R0, 1, DIR, T, P::TS, WAVE>(buf, es, j, tw, tstride);
  if constexpr (P::R1 > 1) stockham_stage<N, P::R1, P::R0, DIR, T, P::TS, WAVE>(buf, es, j, tw, tstride);
  if constexpr (P::R2 > 1) stockham_stage<N, P::R2, P::R0 * P::R1, DIR, T, P::TS, WAVE>(buf, es, j, tw, tstride);
}

// Copies the twiddles of a length-N transform into LDS (twl[m] = exp(-2 pi i m / N)).
// All threads of the block must call it; it synchronises the block.
template <int N, typename T>
__device__ __forceinline__ void load_twiddles(cplx<T>* twl, const cplx<T>* __restrict__ tw, int tstride) {
  for (int m = threadIdx.x; m < N; m += blockDim.x) twl[m] = tw[m * tstride];
  __syncthreads();
}

}  // namespace xs21
