// HBM bandwidth probes: the practical ceilings the path's memory-bound passes
// are measured against, with the access patterns those passes use.
//
//   read    every 16-byte vector of the buffer once (streaming loads), one
//           FP32 sum per block written so that the loads are live
//   write   every 16-byte vector once (streaming stores)
//   copy    first half -> second half, 16-byte vectors
//   tile    the strided pattern of the binning pass: 128-byte row segments
//           (16 complex FP32) of a [N][N][HP] half spectrum, N = 256, HP = 144,
//           read for all N z-planes of one segment column per block step
//
// Each kernel is a grid-stride loop over 8192 blocks of 256 threads.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "common.hpp"
#include "launch.hpp"

namespace xs21 {

namespace {

typedef float F4 __attribute__((vector_size(16)));

constexpr int kProbeThreads = 256;
constexpr unsigned kProbeBlocks = 8192;

__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const F4* __restrict__ in, size_t n4,
                                                              float* __restrict__ sink) {
  float acc = 0.0f;
  const size_t stride = static_cast<size_t>(gridDim.x) * kProbeThreads;
  size_t i = static_cast<size_t>(blockIdx.x) * kProbeThreads + threadIdx.x;
  // four independent loads in flight per thread and iteration
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const F4 a = __builtin_nontemporal_load(in + i);
    const F4 b = __builtin_nontemporal_load(in + i + stride);
    const F4 c = __builtin_nontemporal_load(in + i + 2 * stride);
    const F4 d = __builtin_nontemporal_load(in + i + 3 * stride);
    acc += (a[0] + b[1]) + (c[2] + d[3]);
  }
  for (; i < n4; i += stride) acc += __builtin_nontemporal_load(in + i)[0];
  __shared__ float red[kProbeThreads];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kProbeThreads / 2; h >= 1; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_write(F4* __restrict__ out, size_t n4, float v) {
  const size_t stride = static_cast<size_t>(gridDim.x) * kProbeThreads;
  const F4 x = {v, v, v, v};
  for (size_t i = static_cast<size_t>(blockIdx.x) * kProbeThreads + threadIdx.x; i < n4; i += stride)
    __builtin_nontemporal_store(x, out + i);
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const F4* __restrict__ in, F4* __restrict__ out,
                                                              size_t n4) {
  const size_t stride = static_cast<size_t>(gridDim.x) * kProbeThreads;
  size_t i = static_cast<size_t>(blockIdx.x) * kProbeThreads + threadIdx.x;
  for (; i + stride < n4; i += 2 * stride) {
    const F4 a = __builtin_nontemporal_load(in + i);
    const F4 b = __builtin_nontemporal_load(in + i + stride);
    __builtin_nontemporal_store(a, out + i);
    __builtin_nontemporal_store(b, out + i + stride);
  }
  if (i < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(in + i), out + i);
}

// Strided tiles of [nsp][N][N][HP] complex FP32 spectra (N = 256, HP = 144),
// the binning pass's z-strided reads in whole lines: a tile is the 128-byte
// segment kx in [16 c, 16 c + 16) of row (z, y) for all N values of z (every
// segment of the padded rows, so the whole buffer is read once; blocks
// running together read neighbouring segments); the block's 256 threads read
// 16 z-planes x 16 complex values per step, as the pass does at N = 256.
constexpr int kTileN = 256;
constexpr int kTileHP = 144;
constexpr int kTileSeg = 16;   // complex values per 128-byte segment
static_assert(kTileHP % kTileSeg == 0 && kProbeThreads % kTileSeg == 0, "segments tile the rows and the block");

__global__ __launch_bounds__(kProbeThreads) void k_probe_tile(const cplx<float>* __restrict__ in, long ntiles,
                                                              float* __restrict__ sink) {
  constexpr long PLANE = static_cast<long>(kTileN) * kTileHP;
  constexpr long SPEC = PLANE * kTileN;
  constexpr int SEGS = kTileHP / kTileSeg;        // segments per row
  constexpr int ZR = kProbeThreads / kTileSeg;    // z-planes per step
  const int c = threadIdx.x % kTileSeg, zr = threadIdx.x / kTileSeg;
  float acc = 0.0f;
  for (long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const long sp = t / (static_cast<long>(kTileN) * SEGS), r = t % (static_cast<long>(kTileN) * SEGS);
    const long y = r / SEGS, seg = r % SEGS;
    const cplx<float>* base = in + sp * SPEC + y * kTileHP + seg * kTileSeg + c;
    cplx<float> v[kTileN / ZR];
#pragma unroll
    for (int k = 0; k < kTileN / ZR; ++k) v[k] = base[(zr + ZR * k) * PLANE];
#pragma unroll
    for (int k = 0; k < kTileN / ZR; ++k) acc += v[k].x + v[k].y;
  }
  __shared__ float red[kProbeThreads];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kProbeThreads / 2; h >= 1; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

}  // namespace

size_t probe_sink_bytes() { return kProbeBlocks * sizeof(float); }

size_t probe_tile_spectrum_bytes() {
  return static_cast<size_t>(kTileN) * kTileN * kTileHP * sizeof(cplx<float>);
}

hipError_t launch_probe(int kind, void* buf, size_t bytes, float* sink, double* moved, hipStream_t s) {
  const size_t n4 = bytes / 16;
  if (!buf || !sink || n4 < 2) return hipErrorInvalidValue;
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(k_probe_read, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, static_cast<const F4*>(buf), n4,
                         sink);
      *moved = static_cast<double>(n4) * 16.0;
      break;
    case 1:
      hipLaunchKernelGGL(k_probe_write, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, static_cast<F4*>(buf), n4,
                         1.0f);
      *moved = static_cast<double>(n4) * 16.0;
      break;
    case 2: {
      const size_t h = n4 / 2;
      hipLaunchKernelGGL(k_probe_copy, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, static_cast<const F4*>(buf),
                         static_cast<F4*>(buf) + h, h);
      *moved = static_cast<double>(h) * 32.0;
      break;
    }
    case 3: {
      const long nsp = static_cast<long>(bytes / probe_tile_spectrum_bytes());
      if (nsp < 1) return hipErrorInvalidValue;
      const long ntiles = nsp * kTileN * (kTileHP / kTileSeg);
      hipLaunchKernelGGL(k_probe_tile, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s,
                         static_cast<const cplx<float>*>(buf), ntiles, sink);
      *moved = static_cast<double>(nsp) * probe_tile_spectrum_bytes();
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace xs21
