// Host-side parameter choice (FP64): truncation ell and uniform quadrature per level.
#pragma once

#include <vector>

namespace ffmm {

// The transfer-function part of the rounding floor is a coherent worst case; measured errors sit
// several times under it, so a quarter of it enters the predicted error.
constexpr double kFloorScale = 0.25;
// Radius (box units) at which truncation is balanced against the floor in the breakdown regime.
constexpr double kBreakdownRadius = 1.0;
// Above this box size in wavelength units (ka) the design radius widens to the box diagonal.
constexpr double kWideKa = 100.0;
constexpr double kUnitRoundoffFP64 = 1.1102230246251565e-16;  // 2^-53
constexpr double kUnitRoundoffFP32 = 5.9604644775390625e-08;  // 2^-24

struct LevelParams {
    int ell = 0;
    int ntheta = 0;
    std::vector<int> nphi;  // N_phi(theta_n), n = 0..ntheta/2
    double predicted = 0.0;
};

void sph_bessel_j(int nmax, double x, double* out);
void sph_bessel_y(int nmax, double x, double* out);
void bessel_j_abs(int nmax, double x, double* out);

int ell_search_max(double ka, double r);
void predicted_error(double ka, double r, double r0, int emax, double u, double* out);
int select_ell(double ka, double r, double r0, double eps, double u, double* predicted);
int select_ntheta(double ka, double r, double r0, int ell, double eps);
void select_nphi(double ka, double r, double r0, int ell, int ntheta, double eps, int* nphi);

// The design alpha of one level: the given alpha, or 1 (the box diagonal) for ka > kWideKa when
// some ell reaches eps at |r| = sqrt(3).
double design_alpha(double ka, double alpha, double eps, double u);

// ka = kappa a_l (box units), |r| = design_alpha sqrt(3), |r0| = 2; ell_in > 0 forces ell.
void level_params(double ka, double alpha, double eps, double u, int ell_in, LevelParams* lp);

// Whether the smallest predicted error over ell at the leaf level is below eps.
bool leaf_feasible(double ka_leaf, double alpha, double eps, double u);

}  // namespace ffmm
