// FP64 host planning: radius ladders, mass variance, halo-mass threshold,
// per-walker flag thresholds, exact k-bin tables, FFT twiddles.
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/xs21.h"
#include "common.hpp"

namespace xs21 {
namespace plan {

// Section 2.1: radii from r_top down by `step` while above r_cell, then r_cell.
std::vector<double> ladder(double r_top, double r_cell, double step);

// Sharp-k cutoff of a sphere of radius R (volume matching): (9 pi / 2)^(1/3) / R.
double cutoff(double radius);

// Largest integer |n|^2 kept by the sharp-k filter of radius R on a box of side L.
long n2max(double radius, double box);

// sigma^2(R, z) = D(z)^2 / (2 pi^2) int_0^{k_c} k^2 P(k) dk for P = A k (1 + (k/k0)^2)^-2,
// in closed form: D^2 A k0^4 / (4 pi^2) [ln(1 + U) + 1 / (1 + U) - 1], U = (k_c / k0)^2.
double sigma2(const xs21_physics& p, double radius, double z);

// Section 2.1.3: minimum halo mass (Msun) from the virial temperature.
double min_mass(const xs21_physics& p, double t_vir, double z);

// Lagrangian radius of a mass M (Mpc): (3 M / (4 pi rho_m))^(1/3).
double radius_of_mass(const xs21_physics& p, double mass);

// Inverse of the complementary error function on (0, 2).
double erfcinv(double y);

struct WalkerPlan {
  std::vector<double> thr;    // flag threshold per radius (+inf: never)
  std::vector<double> dsig2;  // sigma^2(M_min) - sigma^2(R)
  int first = 0;              // first radius <= R_mfp
  double m_min = 0.0;
  double a_cell = 0.0;        // 1 / sqrt(2 dsig2 at the cell radius)
  bool partial = false;       // dsig2 at the cell radius > 0
  double u_star = 0.0;        // erfc^-1(1/zeta) (0 when zeta <= 1/2: nothing flags)
};

// Thresholds of one walker on a radius list (eq. 1 rewritten with erfc^-1).
WalkerPlan walker(const xs21_physics& p, double z, const double* radii, int nr, const xs21_walker& w);

// Bin of each integer |n|^2 in [0, 3 (n/2)^2]; -1 for DC and |n| > n/2.
std::vector<int8_t> bins(int n, int nbins);

// Mode counts and count-weighted mean |k| of each bin over the half spectrum.
void bin_stats(int n, int nbins, double box, const std::vector<int8_t>& table, std::vector<double>& counts,
               std::vector<double>& kmean);

// Forward twiddles exp(-2 pi i m / ntab), m in [0, ntab), interleaved (re, im).
std::vector<double> twiddles(int ntab);

// Two-population efficiency (Section 4, eq. 9): walker-independent constants
// of each radius slot of a ladder (slot s = radius nr - 1 - s, slot 0 the cell
// radius), and one walker's inputs of the device planning pass.
std::vector<SlotPlan2> slots2(const xs21_physics& p, double z, const std::vector<double>& radii);
WalkerPlan2 walker2(const xs21_physics& p, double z, const xs21_walker2& w, int used);
// Scalars of a box for planning on the device (BoxPlan).
BoxPlan box_plan(const xs21_physics& p, double z, int nr);

bool valid_physics(const xs21_physics& p);
bool valid_walker(const xs21_walker& w);
bool valid_walker2(const xs21_walker2& w);

}  // namespace plan
}  // namespace xs21
