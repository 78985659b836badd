// Host-side entry points of the kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace xs21 {

// Element types; values match xs21_dtype.
constexpr int kF32 = 0;
constexpr int kF64 = 1;
constexpr int kBF16 = 2;

int axis_tile(int n);                   // inner columns per block of the strided passes
long axis_tiles(int n, long inner);     // blocks along the inner dimension
int ion_grid(int n);                    // blocks of the ionisation pass
int max_group();                        // walkers per ionisation launch
int max_radii();                        // radii per ladder
int max_bins();                         // bins per spectrum

// Real rows [nrows][n] of `dtype` -> half-spectrum rows [nrows][n/2+1].
hipError_t launch_rows_r2c(int dtype, int n, const void* in, void* out, long nrows, const void* tw, int ntab,
                           hipStream_t s);
// Half-spectrum rows -> real rows * scale, stored as `storage`.
hipError_t launch_rows_c2r(int dtype, int storage, int n, const void* in, void* out, long nrows, double scale,
                           const void* tw, int ntab, hipStream_t s);
// Transform along the middle axis of [outer][n][inner] (dir -1 forward, +1
// inverse); n2max >= 0 applies the sharp-k mask before an inverse z pass.
hipError_t launch_axis(int dtype, int n, int dir, const void* src, void* dst, long outer, long inner, long n2max,
                       const void* tw, int ntab, hipStream_t s);
// Forward z pass of [outer][n][n*(n/2+1)] fused with |X|^2 binning into
// part[outer][axis_tiles][nbins] (FP64).
hipError_t launch_axis_bins(int dtype, int n, const void* src, long outer, long inner, const int8_t* bintab,
                            int nbins, double* part, const void* tw, int ntab, hipStream_t s);
// Ionisation + dT_b + forward x pass for nw walkers on one box.
hipError_t launch_ion(int dtype, int storage, int n, const void* dR, const void* delta, int nr, const void* wc,
                      const void* thr, int nw, double tb, double dc, void* spec, double* xpart, const void* tw,
                      int ntab, hipStream_t s);
// x_HI and dT_b boxes of one walker (either output may be null).
hipError_t launch_materialize(int dtype, int storage, int n, const void* dR, const void* delta, int nr,
                              const void* wc, const void* thr, double tb, double dc, void* xhi, void* dtb,
                              hipStream_t s);
// Deterministic reduction of the bin and x_HI partial sums, one walker per block.
hipError_t launch_finalize(int nwalkers, const double* part, long ntiles, int nbins, const double* xpart, long nblk,
                           const double* counts, double pscale, double inv_cells, double* pk, long pk_stride,
                           int nbins_out, double* xhi, long xhi_stride, hipStream_t s);
// out[i] = (dtype) in[i] for `count` stored values.
hipError_t launch_cast(int dtype, int storage, const void* in, void* out, size_t count, hipStream_t s);

}  // namespace xs21
