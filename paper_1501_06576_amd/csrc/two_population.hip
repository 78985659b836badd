// Device planning of the two-population efficiency (Section 4, eq. 9).
//
// With zeta a function of halo mass, the ionisation criterion of eq. (1)
// weighs each collapsed halo by its own efficiency:
//   F(delta_R, R) = int zeta(M) dF_coll(>M | delta_R, R),
// the extended Press-Schechter conditional mass function on the halo-mass
// variance S in (S_R, S(M_cool)], M_cool the 1e4 K halo.  Per (walker,
// radius) this pass turns F >= 1 into an interval [lo, hi] of delta_R (F
// rises with delta_R to one maximum, then falls to zeta(M_R) at delta_c), and
// per walker tabulates the effective efficiency F / erfc(t) at the cell
// radius, t = (delta_c - delta) / sqrt(2 (S(M_cool) - S_R)), for the partial
// ionisation of unflagged cells.
//
// Quadrature: lambda = ln(S - S_R) from ln S_R - 32 to ln(S(M_cool) - S_R),
// split at the feedback mass (zeta has a kink there), on 8-point
// Gauss-Legendre panels at most 0.4 wide; below the first panel zeta is
// zeta(M_R) and that head is added in closed form.  In lambda the
// first-crossing density is nu / sqrt(2 pi (S - S_R)) exp(-nu^2 / (2 (S - S_R)))
// per unit lambda, so each node keeps C = weight zeta / sqrt(2 pi (S - S_R)) and
// E = 1 / (2 (S - S_R)):  F(nu) = nu sum C exp(-nu^2 E) + zeta(M_R) erfc(nu head).
// zeta(M) = zeta0 (y_f / y)^gamma with y = (k_c / k0)^2 (M ~ y^-3/2, T ~ M^2/3),
// gamma = beta above the feedback mass and alpha below; y of a variance S is
// found by Newton's method on S = c (ln(1 + y) - y / (1 + y)).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "launch.hpp"
#include "wave.hpp"

namespace xs21 {
namespace {

constexpr int kGL = 8;
constexpr double kPanel = 0.4;
constexpr int kMaxPanels = 128;
constexpr int kNodesMax = kMaxPanels * kGL;
constexpr double kInvSqrt2Pi = 0.3989422804014327;
constexpr double kInvSqrtPi = 0.5641895835477563;

__constant__ double kGLx[kGL] = {-0.9602898564975362, -0.7966664774136267, -0.525532409916329,
                                 -0.18343464249564978, 0.18343464249564978, 0.525532409916329,
                                 0.7966664774136267,  0.9602898564975362};
__constant__ double kGLw[kGL] = {0.10122853629037669, 0.22238103445337434, 0.31370664587788705,
                                 0.36268378337836177, 0.36268378337836177, 0.31370664587788705,
                                 0.22238103445337434, 0.10122853629037669};

// ln y with c (ln(1 + y) - y / (1 + y)) = c s: Newton in ln y, whose residual is
// convex, from the large-y form ln y ~ s + 1 - 2 / y.
__device__ double lny_of(double s) {
  double l = s + 1.0 - 2.0 * exp(-(s + 1.0));
  for (int it = 0; it < 60; ++it) {
    const double y = exp(l);
    const double g = log1p(y) - y / (1.0 + y);
    const double r = (1.0 + y) / y;
    const double dl = (g - s) * r * r;
    l -= dl;
    if (fabs(dl) <= 1e-15 * fmax(1.0, fabs(l))) break;
  }
  return l;
}

__device__ __forceinline__ double efficiency(const WalkerPlan2& w, double lny) {
  const double g = lny <= w.lny_f ? w.beta : w.alpha;
  return w.zeta0 * exp(g * (w.lny_f - lny));
}

struct Quad2 {
  int count;     // nodes
  double ztop;   // zeta(M_R)
  double head;   // 1 / sqrt(2 exp(lam_a))
};

// Quadrature nodes of one (walker, radius) into C[] / E[], threads tid of nt.
__device__ Quad2 setup_nodes(const SlotPlan2& S, const WalkerPlan2& W, double* C, double* E, int tid, int nt) {
  const double a = S.lam_a, b = S.lam_b;
  double f = b;
  if (W.s_f > S.s_r && W.s_f - S.s_r < S.ds_cool) {
    const double lf = log(W.s_f - S.s_r);
    if (lf > a && lf < b) f = lf;
  }
  int p1 = max(1, static_cast<int>(ceil((f - a) / kPanel)));
  int p2 = f < b ? max(1, static_cast<int>(ceil((b - f) / kPanel))) : 0;
  if (p1 + p2 > kMaxPanels) {   // wider panels, at most kMaxPanels in all
    if (p2) {
      p1 = min(max(1, p1 * kMaxPanels / (p1 + p2)), kMaxPanels - 1);
      p2 = kMaxPanels - p1;
    } else {
      p1 = kMaxPanels;
    }
  }
  const double h1 = (f - a) / p1, h2 = p2 ? (b - f) / p2 : 0.0;
  const int count = (p1 + p2) * kGL;
  for (int j = tid; j < count; j += nt) {
    const int q = j / kGL, k = j % kGL;
    const double lo = q < p1 ? a + q * h1 : f + (q - p1) * h2;
    const double h = q < p1 ? h1 : h2;
    const double lam = lo + 0.5 * h * (kGLx[k] + 1.0);
    const double ds = exp(lam);
    const double z = efficiency(W, lny_of((S.s_r + ds) / S.cvar));
    C[j] = 0.5 * h * kGLw[k] * z * kInvSqrt2Pi / sqrt(ds);
    E[j] = 0.5 / ds;
  }
  Quad2 out;
  out.count = count;
  out.ztop = efficiency(W, S.lny_r);
  out.head = 1.0 / sqrt(2.0 * exp(a));
  return out;
}

// F(nu) by one thread over every node.
__device__ double f_thread(double nu, const double* C, const double* E, const Quad2& q) {
  if (!(nu > 0.0)) return q.ztop;
  const double nu2 = nu * nu;
  double s = 0.0;
  for (int j = 0; j < q.count; ++j) s += C[j] * exp(-nu2 * E[j]);
  return nu * s + q.ztop * erfc(nu * q.head);
}

// F(nu) and dF/dnu by a whole wave (nu wave-uniform); wave-uniform results.
__device__ void f_wave(double nu, const double* C, const double* E, const Quad2& q, int lane, double& F,
                       double& dF) {
  if (!(nu > 0.0)) {
    F = q.ztop;
    dF = 0.0;
    return;
  }
  const double nu2 = nu * nu;
  double s = 0.0, d = 0.0;
  for (int j = lane; j < q.count; j += 64) {
    const double e = C[j] * exp(-nu2 * E[j]);
    s += e;
    d += e * (1.0 - 2.0 * nu2 * E[j]);
  }
  s = wave_sum(s);
  d = wave_sum(d);
  const double xh = nu * q.head;
  F = nu * s + q.ztop * erfc(xh);
  dF = d - q.ztop * 2.0 * q.head * kInvSqrtPi * exp(-xh * xh);
}

// Root of F(nu) = 1 inside [a, b], where F - 1 changes sign (Fa, Fb given):
// Newton's method on ln F, kept inside the shrinking bracket (bisection when
// a step leaves it), stopped when ln F is within a few ulps of 0 or the step
// is below 1e-14 relative.
__device__ double root_f1(double a, double Fa, double b, double Fb, const double* C, const double* E,
                          const Quad2& q, int lane) {
  auto lnf = [](double F) { return F > 0.0 ? log(F) : -800.0; };
  double fa = lnf(Fa), fb = lnf(Fb);
  if ((fa >= 0.0) == (fb >= 0.0)) return fa >= fb ? a : b;   // round-off at a sample: keep the flagged one
  double x = a - fa * (b - a) / (fb - fa);
  if (!(x > fmin(a, b) && x < fmax(a, b))) x = 0.5 * (a + b);
  for (int it = 0; it < 60; ++it) {
    double F, dF;
    f_wave(x, C, E, q, lane, F, dF);
    const double f = lnf(F);
    if (fabs(f) <= 4e-15) break;
    if ((f >= 0.0) == (fa >= 0.0)) {
      a = x;
      fa = f;
    } else {
      b = x;
      fb = f;
    }
    const double d = F > 0.0 ? dF / F : 0.0;
    double xn = d != 0.0 ? x - f / d : 0.5 * (a + b);
    if (!(xn > fmin(a, b) && xn < fmax(a, b))) xn = 0.5 * (a + b);
    const bool done = fabs(xn - x) <= 1e-14 * fabs(x);
    x = xn;
    if (done) break;
  }
  return x;
}

// One wave per (radius slot, walker): thresholds thr[w][0][s] = lo and
// thr[w][1][s] = hi (stride slots each) with F >= 1 exactly for lo <= delta_R
// <= hi; both +inf where no cell can be flagged (unused slot, sphere lighter
// than M_cool, or F < 1 everywhere).  A finite hi sets the walker's `upper`
// (which starts at 0).
template <typename T>
__global__ __launch_bounds__(64) void k_plan2_thr(const SlotPlan2* __restrict__ slots, int nr,
                                                  const WalkerPlan2* __restrict__ wp, WalkerConst<T>* __restrict__ wc,
                                                  T* __restrict__ thr, int stride, double dc) {
  __shared__ double C[kNodesMax];
  __shared__ double E[kNodesMax];
  __shared__ double fs[64];
  const int s = blockIdx.x, w = blockIdx.y, lane = threadIdx.x;
  T* lo = thr + static_cast<size_t>(w) * 2 * stride;
  T* hi = lo + stride;
  const T inf = static_cast<T>(__builtin_huge_val());
  const WalkerPlan2 W = wp[w];
  if (s >= nr || s >= W.used || !(slots[s].ds_cool > 0.0)) {
    if (lane == 0) {
      lo[s] = inf;
      hi[s] = inf;
    }
    return;
  }
  const SlotPlan2 S = slots[s];
  const Quad2 q = setup_nodes(S, W, C, E, lane, 64);
  __syncthreads();
  // scan nu in [0, 8 sqrt(2 (S_cool - S_R))] (t <= 8: erfc(8) ~ 1e-29), then
  // zoom twice around the largest sample when none reaches 1
  double g0 = 0.0, gs = 8.0 * sqrt(2.0 * S.ds_cool) / 63.0;
  double f = f_thread(g0 + lane * gs, C, E, q);
  unsigned long long m = __ballot(f >= 1.0);
  bool top = true;
  for (int zoom = 0; zoom < 2 && m == 0ull; ++zoom) {
    fs[lane] = f;
    __syncthreads();
    int kb = 0;
    for (int k = 1; k < 64; ++k)
      if (fs[k] > fs[kb]) kb = k;
    __syncthreads();
    const double a = g0 + max(kb - 1, 0) * gs, b = g0 + min(kb + 1, 63) * gs;
    g0 = a;
    gs = (b - a) / 63.0;
    f = f_thread(g0 + lane * gs, C, E, q);
    m = __ballot(f >= 1.0);
    top = false;
  }
  fs[lane] = f;
  __syncthreads();
  double dlo = __builtin_huge_val(), dhi = __builtin_huge_val();
  if (m != 0ull) {
    const int i0 = __builtin_ctzll(m), i1 = 63 - __builtin_clzll(m);
    // largest nu with F >= 1 gives the lower delta threshold; F >= 1 at the
    // end of the first scan (t = 8) flags every cell below too.  The ends of a
    // zoomed grid are samples of the coarser one that stayed below 1 there, so
    // a zoomed grid flagged at an end is round-off at that sample.
    if (i1 == 63)
      dlo = top ? -__builtin_huge_val() : dc - (g0 + 63 * gs);
    else
      dlo = dc - root_f1(g0 + i1 * gs, fs[i1], g0 + (i1 + 1) * gs, fs[i1 + 1], C, E, q, lane);
    // smallest nu with F >= 1 gives the upper one (none when zeta(M_R) >= 1)
    if (i0 == 0)
      dhi = top ? __builtin_huge_val() : dc - g0;
    else
      dhi = dc - root_f1(g0 + (i0 - 1) * gs, fs[i0 - 1], g0 + i0 * gs, fs[i0], C, E, q, lane);
  }
  if (lane == 0) {
    lo[s] = static_cast<T>(dlo);
    hi[s] = static_cast<T>(dhi);
    if (static_cast<T>(dhi) < inf) atomicOr(&wc[w].upper, 1);   // the walker needs two-sided tests
  }
}

// Effective efficiency of the cell radius (slot 0) for walker blockIdx.y:
// zt[w][k] = F / erfc(t_k), t_k = (k h)^2, one entry per thread.
template <typename T>
__global__ __launch_bounds__(256) void k_plan2_tab(const SlotPlan2* __restrict__ slots,
                                                   const WalkerPlan2* __restrict__ wp, T* __restrict__ zt,
                                                   int pitch) {
  __shared__ double C[kNodesMax];
  __shared__ double E[kNodesMax];
  const int w = blockIdx.y, t = threadIdx.x;
  const int k = blockIdx.x * 256 + t;
  T* row = zt + static_cast<size_t>(w) * pitch;
  const SlotPlan2 S = slots[0];
  if (!(S.ds_cool > 0.0)) {   // no halo above M_cool fits in a cell: the table is not read
    if (k < pitch) row[k] = T(0);
    return;
  }
  const Quad2 q = setup_nodes(S, wp[w], C, E, t, 256);
  __syncthreads();
  if (k < kZetaTab) {
    const double h = sqrt(kZetaTmax) / (kZetaTab - 1);
    const double tk = (k * h) * (k * h);
    const double e = erfc(tk);
    const double F = f_thread(tk * sqrt(2.0 * S.ds_cool), C, E, q);
    row[k] = static_cast<T>(F / e);
  } else if (k < pitch) {
    row[k] = T(0);
  }
}

}  // namespace

hipError_t launch_plan2(int dtype, const SlotPlan2* slots, int nr, const WalkerPlan2* wp, int nw, void* wc,
                        void* thr, int stride, void* zt, int pitch, double dc, hipStream_t s) {
  if (nr < 1 || nr > stride || nw < 1 || pitch < kZetaTab) return hipErrorInvalidValue;
  const unsigned tab_blocks = static_cast<unsigned>((pitch + 255) / 256);
  if (dtype == kF64) {
    hipLaunchKernelGGL(k_plan2_thr<double>, dim3(static_cast<unsigned>(stride), static_cast<unsigned>(nw)), dim3(64),
                       0, s, slots, nr, wp, static_cast<WalkerConst<double>*>(wc), static_cast<double*>(thr), stride,
                       dc);
    hipLaunchKernelGGL(k_plan2_tab<double>, dim3(tab_blocks, static_cast<unsigned>(nw)), dim3(256), 0, s, slots, wp,
                       static_cast<double*>(zt), pitch);
  } else {
    hipLaunchKernelGGL(k_plan2_thr<float>, dim3(static_cast<unsigned>(stride), static_cast<unsigned>(nw)), dim3(64),
                       0, s, slots, nr, wp, static_cast<WalkerConst<float>*>(wc), static_cast<float*>(thr), stride,
                       dc);
    hipLaunchKernelGGL(k_plan2_tab<float>, dim3(tab_blocks, static_cast<unsigned>(nw)), dim3(256), 0, s, slots, wp,
                       static_cast<float*>(zt), pitch);
  }
  return hipGetLastError();
}

}  // namespace xs21
