// Shared device/host types: complex numbers, bf16 storage, storage loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xs21 {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.x, -a.y}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }

// Streaming (non-temporal) global stores and loads of complex values, for
// data touched once per pass: the cache lines are not kept for reuse.
template <typename T>
struct Pair;
template <>
struct Pair<float> {
  typedef float type __attribute__((vector_size(8)));
};
template <>
struct Pair<double> {
  typedef double type __attribute__((vector_size(16)));
};
template <typename T>
__device__ __forceinline__ void store_stream(cplx<T>* p, cplx<T> v) {
  const typename Pair<T>::type w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<typename Pair<T>::type*>(p));
}
template <typename T>
__device__ __forceinline__ cplx<T> load_stream(const cplx<T>* p) {
  const typename Pair<T>::type w = __builtin_nontemporal_load(reinterpret_cast<const typename Pair<T>::type*>(p));
  return {w[0], w[1]};
}

// bf16 stored as raw 16-bit patterns (upper half of an IEEE binary32).
struct bf16 {
  uint16_t bits;
};

__host__ __device__ __forceinline__ float bf16_to_f32(bf16 v) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(v.bits) << 16);
}

// Round to nearest, ties to even; NaN stays NaN.
__host__ __device__ __forceinline__ bf16 f32_to_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return bf16{static_cast<uint16_t>((u >> 16) | 0x40u)};
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return bf16{static_cast<uint16_t>(u >> 16)};
}

// Load a stored smoothed-box value as the working type T.
template <typename T, typename S>
__host__ __device__ __forceinline__ T load_as(const S* p, size_t i) { return static_cast<T>(p[i]); }
template <>
__host__ __device__ __forceinline__ float load_as<float, bf16>(const bf16* p, size_t i) { return bf16_to_f32(p[i]); }

template <typename S, typename T>
__host__ __device__ __forceinline__ void store_as(S* p, size_t i, T v) { p[i] = static_cast<S>(v); }
template <>
__host__ __device__ __forceinline__ void store_as<bf16, float>(bf16* p, size_t i, float v) { p[i] = f32_to_bf16(v); }
// Same, as a streaming store (FP32 / FP64; BF16 pairs are stored plainly).
template <typename S, typename T>
__device__ __forceinline__ void store_as_stream(S* p, size_t i, T v) {
  __builtin_nontemporal_store(static_cast<S>(v), p + i);
}
template <>
__device__ __forceinline__ void store_as_stream<bf16, float>(bf16* p, size_t i, float v) { p[i] = f32_to_bf16(v); }

// Columns (complex values) per tile of the binning pass's strided reads, and
// of the HBM probe that mimics them.  (Overridable for timing variants.)
#ifndef XS21_BINS_TI
#define XS21_BINS_TI 8
#endif
constexpr int kBinsTileCols = XS21_BINS_TI;

// Per-(walker, box) constants consumed by the per-cell ionisation pass
// (32 bytes for FP32, 64 for FP64; 32-byte aligned).
template <typename T>
struct alignas(32) WalkerConst {
  T zeta;      // ionising efficiency
  T a_cell;    // 1 / sqrt(2 (sigma^2(M_min) - sigma^2(R_cell))), valid if partial != 0
  int32_t chunks;   // radius slots tested, in groups of 8 (slots run from the cell radius up)
  // 0: no halo above M_min fits in a cell, x_HI = 1 when unflagged;
  // 1: x_HI = 1 - zeta erfc(a_cell (delta_c - delta_cell)) when unflagged;
  // 2: the same, and zeta > 1, so that the cell-radius threshold lies below
  //    delta_c and every unflagged cell has delta_c - delta_cell > 0
  int32_t partial;
  float ha;    // a_cell / 2 and a_cell^2 log2(e) in FP32, for the FP32 erfc of a
  float a2l;   // positive argument (partial == 2)
  int32_t upper;    // two-population walkers: 1 if some slot's flag interval is bounded above
};
static_assert(sizeof(WalkerConst<float>) == 32 && sizeof(WalkerConst<double>) == 64, "32- and 64-byte records");

// One walker's constants; for FP32 the whole record in one 32-byte load.
template <typename T>
__host__ __device__ __forceinline__ WalkerConst<T> load_walker(const WalkerConst<T>* p) {
  WalkerConst<T> c;
  if constexpr (sizeof(T) == 4) {
    typedef int32_t V8 __attribute__((vector_size(32)));
    const V8 raw = *reinterpret_cast<const V8*>(p);
    __builtin_memcpy(&c, &raw, sizeof raw);
  } else {
    c = *p;
  }
  return c;
}

// The fields of the partial ionisation alone (zeta, a_cell, partial, ha, a2l;
// the others zero), in loads whose every register is used: a load left in
// flight across other work then holds no dead register that the compiler
// would hand to other values (and so wait for the load early).
__device__ __forceinline__ WalkerConst<float> load_walker_partial(const WalkerConst<float>* p) {
  typedef float F2 __attribute__((vector_size(8)));
  WalkerConst<float> c{};
  const F2 za = *reinterpret_cast<const F2*>(&p->zeta);
  const F2 h = *reinterpret_cast<const F2*>(&p->ha);
  c.zeta = za[0];
  c.a_cell = za[1];
  c.partial = p->partial;
  c.ha = h[0];
  c.a2l = h[1];
  return c;
}

// Two-population efficiency of eq. (9): radius-slot constants (walker
// independent) and walker inputs of the device planning pass, FP64.
struct SlotPlan2 {
  double s_r;       // sigma^2(R)
  double ds_cool;   // sigma^2(M_cool) - sigma^2(R), M_cool the 1e4 K halo mass; <= 0: F = 0
  double lny_r;     // ln y at R, y = (k_c / k0)^2 (halo mass ~ y^-3/2)
  double lam_a;     // quadrature range in ln(S - S_R): from lam_a ...
  double lam_b;     // ... to lam_b = ln(ds_cool)
  double cvar;      // c of sigma^2 = c (ln(1 + y) - y / (1 + y))
  double radius;    // R (Mpc)
};
struct WalkerPlan2 {
  double zeta0, alpha, beta;
  double lny_f;     // ln y of the feedback mass M(T_feed)
  double s_f;       // sigma^2(M(T_feed))
  int32_t used;     // radius slots the walker filters at (from the cell radius up)
  int32_t pad;
};
// Walker-independent scalars of one box for planning on the device from
// device-resident walker parameters (the ensemble sampler): M_min(T) = m1
// T^1.5, R(M) = (rfac M)^(1/3), k_c(R) = kcnum / R, sigma^2 = cvar (ln(1 + y) -
// y / (1 + y)) with y = (k_c / k0)^2.
struct BoxPlan {
  double m1, rfac, kcnum, k0, cvar, dc;
  int32_t nr;       // ladder radii (slots)
  int32_t pad;
};

// Uniform prior box and stretch scale of the ensemble sampler; d = 3 for
// (zeta, R_mfp, T_vir), 5 for (zeta0, R_mfp, T_feed, alpha, beta).
struct SamplerSpec {
  double lo[5], hi[5];
  double a;
  int32_t d;
  int32_t pad;
};

// Effective-efficiency table of the cell radius: entry k holds F / erfc(t) at
// t = (k h)^2, h = sqrt(t_max) / (kZetaTab - 1); rows are kZetaPitch long.
constexpr int kZetaTab = 1025;
constexpr int kZetaPitch = 1032;
constexpr double kZetaTmax = 8.0;

}  // namespace xs21
