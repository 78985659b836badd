// chi^2 likelihood epilogue on the device (Section 2.5; redshifts added
// linearly as in Section 3.4), read from the P(k) that the evaluation writes.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace xs21 {
namespace {

// One thread per walker.  tab holds three rows of nbins values for one box:
// f_b = k_b^3 / (2 pi^2) (P_b -> Delta^2_b), the mock Delta^2_b, and the bin's
// variance noise^2 + (model_err mock)^2, set to 0 for bins outside the fitted
// k range or without modes.  The walker's chi^2 of this box is added to
// chi2[w] (or replaces it when `first`), bins in order: deterministic.
__global__ __launch_bounds__(256) void k_chi2(const double* __restrict__ pk, long pk_stride, int nw,
                                              const double* __restrict__ tab, int nbins, double* __restrict__ chi2,
                                              int first) {
  const int w = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  if (w >= nw) return;
  const double* p = pk + static_cast<long>(w) * pk_stride;
  double s = 0.0;
  for (int b = 0; b < nbins; ++b) {
    const double var = tab[2 * nbins + b];
    if (var > 0.0) {
      const double r = tab[b] * p[b] - tab[nbins + b];
      s += r * r / var;
    }
  }
  chi2[w] = first ? s : chi2[w] + s;
}

}  // namespace

hipError_t launch_chi2(const double* pk, long pk_stride, int nw, const double* tab, int nbins, double* chi2,
                       int first, hipStream_t s) {
  if (nw < 1 || nbins < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chi2, dim3(static_cast<unsigned>((nw + 255) / 256)), dim3(256), 0, s, pk, pk_stride, nw, tab,
                     nbins, chi2, first);
  return hipGetLastError();
}

}  // namespace xs21
