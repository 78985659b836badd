// Wave64 reductions with DPP (data-parallel primitives) and a fast erfc.
#pragma once

#include <stdint.h>

#include "common.hpp"

namespace xs21 {

// DPP controls (GFX9): quad permutes, row mirrors, row broadcasts.
constexpr int kDppQuadSwap1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadSwap2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane j of each 8 reads 7 - j
constexpr int kDppRowMirror = 0x140;  // lane j of each 16 reads 15 - j
constexpr int kDppBcast15 = 0x142;    // lane 15 of row r feeds row r + 1
constexpr int kDppBcast31 = 0x143;    // lane 31 feeds rows 2 and 3

template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_move(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}

// One reduction step: every enabled lane combines its value with a partner
// lane's; lanes of disabled rows combine with the identity `idb`.
template <int CTRL, int ROWS, typename Op>
__device__ __forceinline__ float dpp_step(float v, float id, Op op) {
  return op(v, __int_as_float(dpp_move<CTRL, ROWS>(__float_as_int(id), __float_as_int(v))));
}
template <int CTRL, int ROWS, typename Op>
__device__ __forceinline__ int dpp_step(int v, int id, Op op) {
  return op(v, dpp_move<CTRL, ROWS>(id, v));
}
template <int CTRL, int ROWS, typename Op>
__device__ __forceinline__ double dpp_step(double v, double id, Op op) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v), ib = __builtin_bit_cast(uint64_t, id);
  const uint32_t lo = static_cast<uint32_t>(dpp_move<CTRL, ROWS>(static_cast<int>(ib), static_cast<int>(b)));
  const uint32_t hi =
      static_cast<uint32_t>(dpp_move<CTRL, ROWS>(static_cast<int>(ib >> 32), static_cast<int>(b >> 32)));
  return op(v, __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo));
}

template <typename T>
__device__ __forceinline__ T read_lane63(T v);
template <>
__device__ __forceinline__ float read_lane63<float>(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
template <>
__device__ __forceinline__ int read_lane63<int>(int v) {
  return __builtin_amdgcn_readlane(v, 63);
}
template <>
__device__ __forceinline__ double read_lane63<double>(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b), 63));
  const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), 63));
  return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// Reduction of v over the 64 lanes of a full wave; the result is returned in
// every lane (read back from lane 63, so it is wave-uniform).  The combining
// order is fixed, so results are deterministic.
template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v, T id, Op op) {
  v = dpp_step<kDppQuadSwap1, 0xf>(v, id, op);
  v = dpp_step<kDppQuadSwap2, 0xf>(v, id, op);
  v = dpp_step<kDppHalfMirror, 0xf>(v, id, op);
  v = dpp_step<kDppRowMirror, 0xf>(v, id, op);
  v = dpp_step<kDppBcast15, 0xa>(v, id, op);
  v = dpp_step<kDppBcast31, 0xc>(v, id, op);
  return read_lane63(v);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  return wave_reduce(v, T(0), [](T a, T b) { return a + b; });
}

// Sum of v over the 16 lanes of each row of the wave, returned in every lane
// of that row (four DPP steps, fixed order).
template <typename T>
__device__ __forceinline__ T row_sum(T v) {
  const auto add = [](T a, T b) { return a + b; };
  v = dpp_step<kDppQuadSwap1, 0xf>(v, T(0), add);
  v = dpp_step<kDppQuadSwap2, 0xf>(v, T(0), add);
  v = dpp_step<kDppHalfMirror, 0xf>(v, T(0), add);
  return dpp_step<kDppRowMirror, 0xf>(v, T(0), add);
}
__device__ __forceinline__ int wave_min(int v) {
  return wave_reduce(v, 0x7fffffff, [](int a, int b) { return a < b ? a : b; });
}
__device__ __forceinline__ int wave_max(int v) {
  return wave_reduce(v, -0x7fffffff - 1, [](int a, int b) { return a > b ? a : b; });
}

// erfc(x) = t exp(-z^2 + P(t)), t = 1 / (1 + z/2), z = |x|, P a degree-9
// Chebyshev fit (Press, Teukolsky, Vetterling & Flannery, Numerical Recipes,
// 2nd ed., section 6.2, "erfcc"): fractional error below 1.2e-7 for all x;
// erfc(-z) = 2 - erfc(z).  Evaluated as t 2^(P'(t) - z^2 log2 e) with P' =
// P log2 e (coefficients scaled in double, rounded once), so that for x = a u
// the walker part (a/2, a^2 log2 e) and the cell part (u, u^2) of the
// argument are formed once each: erfc_pos below.  The reciprocal and the
// base-2 exponential are the hardware's approximate ones (about 1 ulp each).
namespace erfc_detail {
constexpr double kLog2e = 1.4426950408889634074;
constexpr float c(double v) { return static_cast<float>(v * kLog2e); }
}  // namespace erfc_detail

// erfc(a u) for a u >= 0, from ha = a / 2, a2l = a^2 log2(e), u and u2 = u^2.
__device__ __forceinline__ float erfc_pos(float ha, float a2l, float u, float u2) {
  using erfc_detail::c;
  const float t = __builtin_amdgcn_rcpf(fmaf(ha, u, 1.0f));  // v_rcp_f32, 1 ulp
  float p = c(0.17087277);
  p = fmaf(p, t, c(-0.82215223));
  p = fmaf(p, t, c(1.48851587));
  p = fmaf(p, t, c(-1.13520398));
  p = fmaf(p, t, c(0.27886807));
  p = fmaf(p, t, c(-0.18628806));
  p = fmaf(p, t, c(0.09678418));
  p = fmaf(p, t, c(0.37409196));
  p = fmaf(p, t, c(1.00002368));
  p = fmaf(p, t, c(-1.26551223));
  return t * __builtin_amdgcn_exp2f(fmaf(-a2l, u2, p));   // v_exp_f32, 1 ulp
}

__device__ __forceinline__ float erfc_fast(float x) {
  constexpr float kL = static_cast<float>(erfc_detail::kLog2e);
  const float z = fabsf(x);
  const float r = erfc_pos(0.5f, kL, z, z * z);
  return x >= 0.0f ? r : 2.0f - r;
}

}  // namespace xs21
