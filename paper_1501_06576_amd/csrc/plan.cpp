#include "plan.hpp"

#include <cmath>
#include <cstdint>
#include <limits>

namespace xs21 {
namespace plan {

namespace {
constexpr double kPi = 3.14159265358979323846;
constexpr double kRhoCritH2 = 2.775e11;  // Msun Mpc^-3 h^-2

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Bit length of m^e (m >= 1), computed exactly with 32-bit limbs.
long pow_bitlen(uint64_t m, int e) {
  std::vector<uint32_t> a{1u};
  for (int i = 0; i < e; ++i) {
    uint64_t carry = 0;
    for (auto& limb : a) {
      const uint64_t v = static_cast<uint64_t>(limb) * m + carry;
      limb = static_cast<uint32_t>(v);
      carry = v >> 32;
    }
    while (carry) {
      a.push_back(static_cast<uint32_t>(carry));
      carry >>= 32;
    }
  }
  const uint32_t top = a.back();
  long bits = 32L * static_cast<long>(a.size() - 1);
  for (uint32_t t = top; t; t >>= 1) ++bits;
  return bits;
}

// m^e >= 2^E  <=>  bitlen(m^e) >= E + 1.
bool pow_ge_pow2(uint64_t m, int e, long E) { return pow_bitlen(m, e) >= E + 1; }
}  // namespace

bool valid_physics(const xs21_physics& p) {
  return std::isfinite(p.delta_c) && finite_pos(p.omega_m) && std::isfinite(p.omega_l) && finite_pos(p.h) &&
         std::isfinite(p.tb0_mK) && finite_pos(p.pk_amp) && finite_pos(p.pk_k0) && std::isfinite(p.z_ref) &&
         p.z_ref > -1.0 && std::isfinite(p.radius_step) && p.radius_step > 1.0 && finite_pos(p.ladder_top) &&
         finite_pos(p.mu) && (p.mmin_form == 0 || p.mmin_form == 1) && (p.velocity == 0 || p.velocity == 1) &&
         std::isfinite(p.dvdr_max) && p.dvdr_max >= 0.0 && p.dvdr_max < 1.0;
}

bool valid_walker(const xs21_walker& w) { return finite_pos(w.zeta) && finite_pos(w.r_mfp) && finite_pos(w.t_vir); }

bool valid_walker2(const xs21_walker2& w) {
  return finite_pos(w.zeta0) && w.zeta0 <= 1e6 && finite_pos(w.r_mfp) && std::isfinite(w.t_feed) &&
         w.t_feed >= 1e4 && w.t_feed <= 1e9 && std::isfinite(w.alpha) && std::fabs(w.alpha) <= 10.0 &&
         std::isfinite(w.beta) && std::fabs(w.beta) <= 10.0;
}

std::vector<double> ladder(double r_top, double r_cell, double step) {
  std::vector<double> out;
  for (int i = 0;; ++i) {
    const double r = r_top / std::pow(step, i);
    if (!(r > r_cell)) break;
    out.push_back(r);
  }
  out.push_back(r_cell);
  return out;
}

double cutoff(double radius) { return std::cbrt(4.5 * kPi) / radius; }

long n2max(double radius, double box) {
  const double x = cutoff(radius) * box / (2.0 * kPi);
  return static_cast<long>(std::floor(x * x));
}

double sigma2(const xs21_physics& p, double radius, double z) {
  const double u = std::pow(cutoff(radius) / p.pk_k0, 2);
  const double d = (1.0 + p.z_ref) / (1.0 + z);
  // ln(1+U) + 1/(1+U) - 1 = ln(1+U) - U/(1+U); log1p keeps small U accurate
  const double bracket = std::log1p(u) - u / (1.0 + u);
  return d * d * p.pk_amp * std::pow(p.pk_k0, 4) / (4.0 * kPi * kPi) * bracket;
}

double min_mass(const xs21_physics& p, double t_vir, double z) {
  if (p.mmin_form == 0) return 1e8 * std::pow(t_vir / 1e4, 1.5) * std::pow((1.0 + z) / 10.0, -1.5);
  const double a3 = p.omega_m * std::pow(1.0 + z, 3);
  const double om_z = a3 / (a3 + p.omega_l);
  const double d = om_z - 1.0;
  const double delta_vir = 18.0 * kPi * kPi + 82.0 * d - 39.0 * d * d;
  return 1e8 / p.h * std::pow(p.mu / 0.6, -1.5) *
         std::pow(p.omega_m / om_z * delta_vir / (18.0 * kPi * kPi), -0.5) * std::pow(t_vir / 1.98e4, 1.5) *
         std::pow((1.0 + z) / 10.0, -1.5);
}

double radius_of_mass(const xs21_physics& p, double mass) {
  const double rho = p.omega_m * kRhoCritH2 * p.h * p.h;
  return std::cbrt(3.0 * mass / (4.0 * kPi * rho));
}

double erfcinv(double y) {
  if (!(y > 0.0 && y < 2.0)) return std::numeric_limits<double>::quiet_NaN();
  // erfc is strictly decreasing: bracket by bisection, then polish with Newton.
  double lo = -6.0, hi = 27.0;
  for (int i = 0; i < 80; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (std::erfc(mid) > y) lo = mid; else hi = mid;
  }
  double x = 0.5 * (lo + hi);
  for (int i = 0; i < 3; ++i) {
    const double f = std::erfc(x) - y;
    const double df = -2.0 / std::sqrt(kPi) * std::exp(-x * x);
    if (df == 0.0) break;
    const double nx = x - f / df;
    if (!(nx >= lo && nx <= hi)) break;
    x = nx;
  }
  return x;
}

WalkerPlan walker(const xs21_physics& p, double z, const double* radii, int nr, const xs21_walker& w) {
  WalkerPlan out;
  out.thr.resize(nr);
  out.dsig2.resize(nr);
  out.m_min = min_mass(p, w.t_vir, z);
  const double s_min = sigma2(p, radius_of_mass(p, out.m_min), z);
  const double inv_zeta = 1.0 / w.zeta;
  const bool can_flag = inv_zeta < 2.0;  // zeta f_coll >= 1 needs f_coll >= 1/zeta, and f_coll < 2
  const double u_star = can_flag ? erfcinv(inv_zeta) : 0.0;
  out.u_star = u_star;
  const double inf = std::numeric_limits<double>::infinity();
  out.first = nr - 1;
  for (int j = 0; j < nr; ++j) {
    const double ds = s_min - sigma2(p, radii[j], z);
    out.dsig2[j] = ds;
    // zeta erfc((delta_c - delta_R) / sqrt(2 ds)) >= 1  <=>  delta_R >= delta_c - sqrt(2 ds) erfc^-1(1/zeta)
    out.thr[j] = (ds > 0.0 && can_flag) ? p.delta_c - std::sqrt(2.0 * ds) * u_star : inf;
    if (j < out.first && radii[j] <= w.r_mfp) out.first = j;
  }
  const double dc = out.dsig2[nr - 1];
  out.partial = dc > 0.0;
  out.a_cell = out.partial ? 1.0 / std::sqrt(2.0 * dc) : 0.0;
  return out;
}

namespace {
// ln y, y = (k_c(R) / k0)^2: halo mass ~ R^3 ~ y^-3/2
double lny_of_radius(const xs21_physics& p, double radius) { return 2.0 * std::log(cutoff(radius) / p.pk_k0); }
}  // namespace

std::vector<SlotPlan2> slots2(const xs21_physics& p, double z, const std::vector<double>& radii) {
  const int nr = static_cast<int>(radii.size());
  const double d = (1.0 + p.z_ref) / (1.0 + z);
  const double cvar = d * d * p.pk_amp * std::pow(p.pk_k0, 4) / (4.0 * kPi * kPi);
  const double s_cool = sigma2(p, radius_of_mass(p, min_mass(p, 1e4, z)), z);
  std::vector<SlotPlan2> out(nr);
  for (int s = 0; s < nr; ++s) {
    const double r = radii[nr - 1 - s];
    SlotPlan2& o = out[s];
    o.s_r = sigma2(p, r, z);
    o.ds_cool = s_cool - o.s_r;
    o.lny_r = lny_of_radius(p, r);
    o.lam_a = std::log(o.s_r) - 32.0;
    o.lam_b = o.ds_cool > 0.0 ? std::log(o.ds_cool) : o.lam_a;
    o.cvar = cvar;
    o.radius = r;
  }
  return out;
}

BoxPlan box_plan(const xs21_physics& p, double z, int nr) {
  BoxPlan b{};
  b.m1 = min_mass(p, 1.0, z);
  b.rfac = 3.0 / (4.0 * kPi * p.omega_m * kRhoCritH2 * p.h * p.h);
  b.kcnum = std::cbrt(4.5 * kPi);
  b.k0 = p.pk_k0;
  const double d = (1.0 + p.z_ref) / (1.0 + z);
  b.cvar = d * d * p.pk_amp * std::pow(p.pk_k0, 4) / (4.0 * kPi * kPi);
  b.dc = p.delta_c;
  b.nr = nr;
  return b;
}

WalkerPlan2 walker2(const xs21_physics& p, double z, const xs21_walker2& w, int used) {
  WalkerPlan2 o{};
  o.zeta0 = w.zeta0;
  o.alpha = w.alpha;
  o.beta = w.beta;
  const double rf = radius_of_mass(p, min_mass(p, w.t_feed, z));
  o.lny_f = lny_of_radius(p, rf);
  o.s_f = sigma2(p, rf, z);
  o.used = used;
  return o;
}

std::vector<int8_t> bins(int n, int nbins) {
  const long half = n / 2;
  int p = 0;
  while ((1L << p) < half) ++p;  // half = 2^p
  // t[b]: first integer n2 with n2^nbins >= (n/2)^(2b) = 2^(2 b p)
  std::vector<long> t(nbins + 1, 1);
  for (int b = 1; b <= nbins; ++b) {
    long lo = 1, hi = half * half;
    const long E = 2L * b * p;
    while (lo < hi) {
      const long mid = lo + (hi - lo) / 2;
      if (pow_ge_pow2(static_cast<uint64_t>(mid), nbins, E)) hi = mid; else lo = mid + 1;
    }
    t[b] = lo;
  }
  const long top = 3 * half * half;
  std::vector<int8_t> out(top + 1, -1);
  for (long v = 1; v <= half * half; ++v) {
    int b = 0;
    for (int c = 1; c <= nbins; ++c)
      if (v >= t[c]) b = c;
    out[v] = static_cast<int8_t>(b < nbins ? b : nbins - 1);
  }
  return out;
}

void bin_stats(int n, int nbins, double box, const std::vector<int8_t>& table, std::vector<double>& counts,
               std::vector<double>& kmean) {
  const long half = n / 2;
  std::vector<double> mult(3 * half * half + 1, 0.0);
  std::vector<long> sq(n);
  for (int i = 0; i < n; ++i) {
    const long f = i < half ? i : i - n;
    sq[i] = f * f;
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const long s = sq[a] + sq[b];
      for (long c = 0; c <= half; ++c) mult[s + c * c] += (c == 0 || c == half) ? 1.0 : 2.0;
    }
  counts.assign(nbins, 0.0);
  std::vector<double> ksum(nbins, 0.0);
  const double kf = 2.0 * kPi / box;
  for (size_t v = 0; v < mult.size(); ++v) {
    const int b = table[v];
    if (b < 0 || mult[v] == 0.0) continue;
    counts[b] += mult[v];
    ksum[b] += mult[v] * kf * std::sqrt(static_cast<double>(v));
  }
  kmean.assign(nbins, 0.0);
  for (int b = 0; b < nbins; ++b) kmean[b] = counts[b] > 0.0 ? ksum[b] / counts[b] : 0.0;
}

std::vector<double> twiddles(int ntab) {
  std::vector<double> out(2 * static_cast<size_t>(ntab));
  for (int m = 0; m < ntab; ++m) {
    // exact values on the axes and diagonals, libm elsewhere
    const double a = 2.0 * kPi * m / ntab;
    double c = std::cos(a), s = std::sin(a);
    if (4 * m % ntab == 0) {
      const int q = 4 * m / ntab;
      c = (q == 0) ? 1.0 : (q == 2 ? -1.0 : 0.0);
      s = (q == 1) ? 1.0 : (q == 3 ? -1.0 : 0.0);
    }
    out[2 * m] = c;
    out[2 * m + 1] = -s;
  }
  return out;
}

}  // namespace plan
}  // namespace xs21
