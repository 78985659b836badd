// Device-resident ensemble sampler (Section 2.3: the affine invariant
// stretch move of Goodman & Weare 2010, in its two-halves parallel form), and
// the planning of walker tables from device-resident parameters it needs.
//
// A half-step moves the walkers of one half: walker X_k takes a partner X_j
// from the other half, j = floor(u0 n), a stretch z = ((a - 1) u1 + 1)^2 / a
// (the inverse CDF of g(z) ~ 1/sqrt(z) on [1/a, a]), the proposal
// Y = X_j + z (X_k - X_j), and accepts it when
// ln u2 < (d - 1) ln z + ln p(Y) - ln p(X_k), ln p = -chi^2 / 2 inside the
// prior box and -inf outside.  Uniforms are inputs, three per walker and
// half-step.  The proposals of a chunk of the half are evaluated by the same
// kernels as xs21_eval_batch, planned here on the device.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "launch.hpp"

namespace xs21 {
namespace {

// Ladder index of the first radius <= r_mfp (the cell radius if none), and
// the slots used from the cell radius up.
__device__ int used_slots(const SlotPlan2* __restrict__ slots, int nr, double r_mfp) {
  int first = nr - 1;
  for (int j = 0; j < nr - 1; ++j)
    if (slots[nr - 1 - j].radius <= r_mfp) {
      first = j;
      break;
    }
  return nr - first;
}

__device__ double sigma2_of_radius(const BoxPlan& b, double r) {
  const double k = b.kcnum / r / b.k0;
  const double y = k * k;
  return b.cvar * (log1p(y) - y / (1.0 + y));
}

// Sampler coordinates are the paper's parameters with the temperature as its
// decimal logarithm: (zeta, R_mfp, log10 T_vir) and (zeta0, R_mfp,
// log10 T_feed, alpha, beta).
//
// Constant-efficiency walkers (zeta, R_mfp, log10 T_vir), one thread each: the
// walker constants and the flag thresholds delta_c - sqrt(2 dsig2) erfc^-1(1/zeta)
// in radius slots (eq. 1 rewritten, +inf where unused or impossible).
template <typename T>
__global__ __launch_bounds__(64) void k_plan1(const double* __restrict__ par, int nw, BoxPlan b,
                                              const SlotPlan2* __restrict__ slots, WalkerConst<T>* __restrict__ wc,
                                              T* __restrict__ thr, int stride) {
  const int w = static_cast<int>(blockIdx.x) * 64 + static_cast<int>(threadIdx.x);
  if (w >= nw) return;
  const double zeta = par[3 * w], r_mfp = par[3 * w + 1], t_vir = pow(10.0, par[3 * w + 2]);
  const double s_min = sigma2_of_radius(b, cbrt(b.rfac * b.m1 * pow(t_vir, 1.5)));
  const double inv = 1.0 / zeta;
  const bool can = inv < 2.0;
  const double ustar = can ? erfcinv(inv) : 0.0;
  const int used = used_slots(slots, b.nr, r_mfp);
  T* t = thr + static_cast<size_t>(w) * stride;
  const T inf = static_cast<T>(__builtin_huge_val());
  for (int s = 0; s < stride; ++s) {
    T v = inf;
    if (s < used) {
      const double ds = s_min - slots[s].s_r;
      if (ds > 0.0 && can) v = static_cast<T>(b.dc - sqrt(2.0 * ds) * ustar);
    }
    t[s] = v;
  }
  const double dcell = s_min - slots[0].s_r;
  const double a = dcell > 0.0 ? 1.0 / sqrt(2.0 * dcell) : 0.0;
  WalkerConst<T> c{};
  c.zeta = static_cast<T>(zeta);
  c.a_cell = static_cast<T>(a);
  c.chunks = (used + 7) / 8;
  // mode 2 iff zeta > 1: the cell-radius threshold lies below delta_c
  c.partial = dcell > 0.0 ? (ustar > 0.0 ? 2 : 1) : 0;
  c.ha = static_cast<float>(0.5 * a);
  c.a2l = static_cast<float>(a * a * 1.4426950408889634074);
  c.upper = 0;
  wc[w] = c;
}

// Two-population walkers (zeta0, R_mfp, log10 T_feed, alpha, beta), one thread each:
// the walker constants and the inputs of the planning pass of eq. (9).
template <typename T>
__global__ __launch_bounds__(64) void k_walker2(const double* __restrict__ par, int nw, BoxPlan b,
                                                const SlotPlan2* __restrict__ slots, WalkerConst<T>* __restrict__ wc,
                                                WalkerPlan2* __restrict__ wp) {
  const int w = static_cast<int>(blockIdx.x) * 64 + static_cast<int>(threadIdx.x);
  if (w >= nw) return;
  const double* p = par + 5 * w;
  const double rf = cbrt(b.rfac * b.m1 * pow(pow(10.0, p[2]), 1.5));
  const double kf = b.kcnum / rf / b.k0;
  const int used = used_slots(slots, b.nr, p[1]);
  WalkerPlan2 o;
  o.zeta0 = p[0];
  o.alpha = p[3];
  o.beta = p[4];
  o.lny_f = 2.0 * log(kf);
  o.s_f = sigma2_of_radius(b, rf);
  o.used = used;
  o.pad = 0;
  wp[w] = o;
  const double ds = slots[0].ds_cool;
  WalkerConst<T> c{};
  c.zeta = T(1);
  c.a_cell = static_cast<T>(ds > 0.0 ? 1.0 / sqrt(2.0 * ds) : 0.0);
  c.chunks = (used + 7) / 8;
  c.partial = ds > 0.0 ? 1 : 0;
  c.upper = 0;   // set by the planning pass
  wc[w] = c;
}

__device__ bool in_prior(const SamplerSpec& s, const double* x) {
  bool ok = true;
  for (int i = 0; i < s.d; ++i) ok = ok && x[i] >= s.lo[i] && x[i] <= s.hi[i];
  return ok;
}

// Proposals of walkers k = k0 + i, i < count, of the moving half (partners
// from the other half, which starts at o0 and holds half walkers).  Writes
// the parameters to evaluate (the proposal, or X_k when it leaves the prior)
// and aux[i] = ((d - 1) ln z, 1 if inside the prior else 0).
__global__ __launch_bounds__(64) void k_propose(const double* __restrict__ x, int k0, int o0, int half, int count,
                                                const double* __restrict__ u, SamplerSpec s, double* __restrict__ prop,
                                                double* __restrict__ aux) {
  const int i = static_cast<int>(blockIdx.x) * 64 + static_cast<int>(threadIdx.x);
  if (i >= count) return;
  const int d = s.d;
  const double* ui = u + 3 * i;
  const double q = ui[0] * half;   // partner index, kept inside the other half for any input
  const int j = o0 + (q > 0.0 ? (q < half ? static_cast<int>(q) : half - 1) : 0);
  const double t = (s.a - 1.0) * ui[1] + 1.0;
  const double z = t * t / s.a;
  const double* xk = x + static_cast<size_t>(k0 + i) * d;
  const double* xj = x + static_cast<size_t>(j) * d;
  double y[5];
  for (int c = 0; c < d; ++c) y[c] = xj[c] + z * (xk[c] - xj[c]);
  const bool ok = in_prior(s, y);
  double* out = prop + static_cast<size_t>(i) * d;
  for (int c = 0; c < d; ++c) out[c] = ok ? y[c] : xk[c];
  aux[2 * i] = (d - 1) * log(z);
  aux[2 * i + 1] = ok ? 1.0 : 0.0;
}

// Acceptance of the proposals of k_propose given their chi^2 (summed over
// boxes): ln p(Y) = -chi^2 / 2 inside the prior, -inf outside.
__global__ __launch_bounds__(64) void k_accept(double* __restrict__ x, double* __restrict__ lp, int k0, int count,
                                               int d, const double* __restrict__ u, const double* __restrict__ prop,
                                               const double* __restrict__ aux, const double* __restrict__ chi2,
                                               int32_t* __restrict__ accepted) {
  const int i = static_cast<int>(blockIdx.x) * 64 + static_cast<int>(threadIdx.x);
  if (i >= count) return;
  const int k = k0 + i;
  const double lpy = aux[2 * i + 1] != 0.0 ? -0.5 * chi2[i] : -__builtin_huge_val();
  const double log_r = aux[2 * i] + lpy - lp[k];
  const double u2 = u[3 * i + 2];
  const double log_u = u2 > 0.0 ? log(u2) : -__builtin_huge_val();
  const bool take = log_u < log_r;
  if (take) {
    for (int c = 0; c < d; ++c) x[static_cast<size_t>(k) * d + c] = prop[static_cast<size_t>(i) * d + c];
    lp[k] = lpy;
  }
  if (accepted) accepted[k] = take ? 1 : 0;
}

// ln p of walkers from their chi^2: -chi^2 / 2 inside the prior, -inf outside.
__global__ __launch_bounds__(64) void k_lnprob(const double* __restrict__ x, int count, SamplerSpec s,
                                               const double* __restrict__ chi2, double* __restrict__ lp) {
  const int i = static_cast<int>(blockIdx.x) * 64 + static_cast<int>(threadIdx.x);
  if (i >= count) return;
  lp[i] = in_prior(s, x + static_cast<size_t>(i) * s.d) ? -0.5 * chi2[i] : -__builtin_huge_val();
}

unsigned blocks64(int n) { return static_cast<unsigned>((n + 63) / 64); }

}  // namespace

hipError_t launch_plan1(int dtype, const double* par, int nw, const BoxPlan& b, const SlotPlan2* slots, void* wc,
                        void* thr, int stride, hipStream_t s) {
  if (nw < 1 || b.nr < 1 || b.nr > stride) return hipErrorInvalidValue;
  if (dtype == kF64)
    hipLaunchKernelGGL(k_plan1<double>, dim3(blocks64(nw)), dim3(64), 0, s, par, nw, b, slots,
                       static_cast<WalkerConst<double>*>(wc), static_cast<double*>(thr), stride);
  else
    hipLaunchKernelGGL(k_plan1<float>, dim3(blocks64(nw)), dim3(64), 0, s, par, nw, b, slots,
                       static_cast<WalkerConst<float>*>(wc), static_cast<float*>(thr), stride);
  return hipGetLastError();
}

hipError_t launch_walker2(int dtype, const double* par, int nw, const BoxPlan& b, const SlotPlan2* slots, void* wc,
                          WalkerPlan2* wp, hipStream_t s) {
  if (nw < 1 || b.nr < 1) return hipErrorInvalidValue;
  if (dtype == kF64)
    hipLaunchKernelGGL(k_walker2<double>, dim3(blocks64(nw)), dim3(64), 0, s, par, nw, b, slots,
                       static_cast<WalkerConst<double>*>(wc), wp);
  else
    hipLaunchKernelGGL(k_walker2<float>, dim3(blocks64(nw)), dim3(64), 0, s, par, nw, b, slots,
                       static_cast<WalkerConst<float>*>(wc), wp);
  return hipGetLastError();
}

hipError_t launch_propose(const double* x, int k0, int o0, int half, int count, const double* u,
                          const SamplerSpec& spec, double* prop, double* aux, hipStream_t s) {
  if (count < 1 || half < 1 || spec.d < 1 || spec.d > 5) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_propose, dim3(blocks64(count)), dim3(64), 0, s, x, k0, o0, half, count, u, spec, prop, aux);
  return hipGetLastError();
}

hipError_t launch_accept(double* x, double* lp, int k0, int count, int d, const double* u, const double* prop,
                         const double* aux, const double* chi2, int32_t* accepted, hipStream_t s) {
  if (count < 1 || d < 1 || d > 5) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_accept, dim3(blocks64(count)), dim3(64), 0, s, x, lp, k0, count, d, u, prop, aux, chi2,
                     accepted);
  return hipGetLastError();
}

hipError_t launch_lnprob(const double* x, int count, const SamplerSpec& spec, const double* chi2, double* lp,
                         hipStream_t s) {
  if (count < 1 || spec.d < 1 || spec.d > 5) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lnprob, dim3(blocks64(count)), dim3(64), 0, s, x, count, spec, chi2, lp);
  return hipGetLastError();
}

}  // namespace xs21
