// Host-side (FP64) parameter choice of the Fourier-basis FMM: truncation ell (Section 2.1),
// N_theta (Section 3.3.1, Alg. Ntheta) and N_phi(theta_n) (Section 3.3.2, Alg. Nphi), together
// with the special functions they need. Everything is in units of the box size: ka = kappa a_l,
// |r| = alpha sqrt(3), |r0| = 2 (Section 3.3.3).
#include "params.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace ffmm {

using cd = std::complex<double>;
static const double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------------------------
// Special functions (Table 1 notation).
// ---------------------------------------------------------------------------------------------

// j_n(x), n = 0..nmax. For n > x the upward recurrence loses accuracy, so the values come from a
// downward (Miller) recurrence started well above max(nmax, x) and normalised by j_0 = sin x / x.
void sph_bessel_j(int nmax, double x, double* out)
{
    if (x == 0.0) {
        out[0] = 1.0;
        for (int n = 1; n <= nmax; ++n) out[n] = 0.0;
        return;
    }
    const int top = std::max(nmax, (int)x) + 30 + (int)std::sqrt(40.0 * (std::max(nmax, (int)x) + 1));
    std::vector<double> v(top + 2, 0.0);
    double jp1 = 0.0, j = 1e-300;
    for (int n = top; n >= 1; --n) {
        double jm1 = (2.0 * n + 1.0) / x * j - jp1;
        jp1 = j;
        j = jm1;
        if (n - 1 <= nmax + 1) v[n - 1] = j;
        if (std::fabs(j) > 1e250) {  // rescale to stay finite
            j *= 1e-250;
            jp1 *= 1e-250;
            for (int k = n - 1; k <= std::min(top, nmax + 1); ++k) v[k] *= 1e-250;
        }
    }
    // v[n] is proportional to j_n; normalise with j_0 or, near its zeros, with j_1.
    const double j0 = std::sin(x) / x;
    const double j1 = std::sin(x) / (x * x) - std::cos(x) / x;
    double scale = (std::fabs(j0) > std::fabs(j1)) ? j0 / v[0] : j1 / v[1];
    for (int n = 0; n <= nmax; ++n) out[n] = v[n] * scale;
}

// y_n(x), n = 0..nmax, by the upward recurrence (stable for the second kind).
void sph_bessel_y(int nmax, double x, double* out)
{
    out[0] = -std::cos(x) / x;
    if (nmax >= 1) out[1] = -std::cos(x) / (x * x) - std::sin(x) / x;
    for (int n = 1; n < nmax; ++n) {
        double v = (2.0 * n + 1.0) / x * out[n] - out[n - 1];
        out[n + 1] = std::isfinite(v) ? v : -HUGE_VAL;
    }
}

// |J_n(x)|, n = 0..nmax, integer order, x >= 0 (plane-wave spectrum, eqn. PlaneWaveSpec). Miller's
// downward recurrence normalised by J_0 + 2 sum_k J_2k = 1.
void bessel_j_abs(int nmax, double x, double* out)
{
    if (x == 0.0) {
        out[0] = 1.0;
        for (int n = 1; n <= nmax; ++n) out[n] = 0.0;
        return;
    }
    int top = std::max(nmax, (int)x) + 30 + (int)std::sqrt(40.0 * (std::max(nmax, (int)x) + 1));
    if (top % 2) ++top;
    std::vector<double> v(top + 2, 0.0);
    double jp1 = 0.0, j = 1e-300, norm = 0.0;
    v[top] = j;
    for (int n = top; n >= 1; --n) {
        double jm1 = (2.0 * n) / x * j - jp1;
        jp1 = j;
        j = jm1;
        v[n - 1] = j;
        if (std::fabs(j) > 1e250) {
            for (int k = n - 1; k <= top; ++k) v[k] *= 1e-250;
            j *= 1e-250;
            jp1 *= 1e-250;
        }
    }
    norm = v[0];
    for (int k = 2; k <= top; k += 2) norm += 2.0 * v[k];
    for (int n = 0; n <= nmax; ++n) out[n] = std::fabs(v[n] / norm);
}

// P_n(t), n = 0..nmax, three-term recurrence.
static void legendre(int nmax, double t, double* out)
{
    out[0] = 1.0;
    if (nmax >= 1) out[1] = t;
    for (int n = 1; n < nmax; ++n) out[n + 1] = ((2.0 * n + 1.0) * t * out[n] - n * out[n - 1]) / (n + 1.0);
}

// Fourier coefficient of |sin t| (Section 3.1.3): ((-1)^n + 1) / (pi (1 - n^2)).
static double sin_abs_coeff(long n)
{
    if (n % 2 != 0) return 0.0;
    double nn = (double)n;
    return 2.0 / (kPi * (1.0 - nn * nn));
}

// ---------------------------------------------------------------------------------------------
// Truncation ell (Section 2.1) with the low-frequency rounding floor.
// ---------------------------------------------------------------------------------------------

int ell_search_max(double ka, double r)
{
    double x = ka * r;
    return (int)std::ceil(x + 10.0 * std::cbrt(std::max(x, 1.0)) + 40.0);
}

// max over gamma in [0, pi] (129 points) of |eps_G(ell)|, ell = 0..emax (eqn. eps_G), plus the
// rounding floor of the low-frequency breakdown (Sections 2.1 and 3.5.1), in two parts:
//  * evaluating T (always FP64) sums terms up to |c_n|; integrated over the sphere the error is at
//    most u64 ka sum_{n<=ell} (2n+1) |h_n(ka r0)| (a coherent bound, scaled by kFloorScale);
//  * the signature arithmetic in precision u rounds each of the ~(4/pi)(ell+1)^2 quadrature terms
//    independently: a random walk of size u ka sqrt(sum (2n+1) |h_n|^2 / K).
void predicted_error(double ka, double r, double r0, int emax, double u, double* out)
{
    const int ng = 129;
    std::vector<double> jn(emax + 1), yn(emax + 1), hy(emax + 1), P(emax + 1);
    sph_bessel_j(emax, ka * r, jn.data());
    sph_bessel_y(emax, ka * r0, yn.data());
    sph_bessel_j(emax, ka * r0, hy.data());  // real part of h_n(ka r0)
    std::vector<cd> coef(emax + 1);
    for (int n = 0; n <= emax; ++n) {
        cd h(hy[n], yn[n]);
        coef[n] = cd(0.0, ka) * ((n % 2) ? -1.0 : 1.0) * (2.0 * n + 1.0) * h * jn[n];
    }
    std::vector<double> err(emax + 1, 0.0);
    for (int g = 0; g < ng; ++g) {
        double gam = kPi * g / (ng - 1);
        double c = std::cos(gam);
        double R = std::sqrt(r * r + r0 * r0 + 2.0 * r * r0 * c);
        cd exact = std::exp(cd(0.0, ka * R)) / R;
        legendre(emax, c, P.data());
        cd partial(0.0, 0.0);
        for (int n = 0; n <= emax; ++n) {
            partial += coef[n] * P[n];
            double e = std::abs(exact - partial);
            if (!(e <= err[n])) err[n] = std::isfinite(e) ? std::max(err[n], e) : HUGE_VAL;
        }
    }
    double lin = 0.0, sq = 0.0;
    for (int n = 0; n <= emax; ++n) {
        double hab = std::hypot(hy[n], yn[n]);
        if (!std::isfinite(hab)) hab = HUGE_VAL;
        lin += (2.0 * n + 1.0) * hab;
        sq += (2.0 * n + 1.0) * hab * hab;
        const double kq = (4.0 / kPi) * (n + 1.0) * (n + 1.0);
        out[n] = err[n] + kFloorScale * kUnitRoundoffFP64 * ka * lin + u * ka * std::sqrt(sq / kq);
    }
}

// Smallest ell whose predicted error (truncation at |r| plus rounding floor) is below eps. In the
// low-frequency breakdown no ell reaches eps; the achievable accuracy is then set by roundoff and
// ell minimises the truncation error at |r| = kBreakdownRadius (the box size) plus the floor.
int select_ell(double ka, double r, double r0, double eps, double u, double* predicted)
{
    const int emax = ell_search_max(ka, r);
    std::vector<double> tot(emax + 1);
    predicted_error(ka, r, r0, emax, u, tot.data());
    for (int l = 1; l <= emax; ++l)
        if (tot[l] < eps) {
            if (predicted) *predicted = tot[l];
            return l;
        }
    predicted_error(ka, std::min(r, kBreakdownRadius), r0, emax, u, tot.data());
    int best = 1;
    for (int l = 2; l <= emax; ++l)
        if (tot[l] < tot[best]) best = l;
    if (predicted) *predicted = tot[best];
    return best;
}

// ---------------------------------------------------------------------------------------------
// Band-limited modified transfer function on the host (Alg. BMTF), used by Alg. Ntheta/Nphi.
// ---------------------------------------------------------------------------------------------

// For one phi column: 1/2 T_{ell,r0} at theta'_j = 2 pi j / (2 ell + 1) (eqn. TransferFn), its
// Fourier coefficients p = -ell..ell, then convolved with the |sin| coefficients for
// |k| <= kmax. out[k + kmax], k = -kmax..kmax.
static void bmtf_column_spectrum(double ka, const double r0[3], int ell, double phi, int kmax,
                                 const std::vector<cd>& cn, cd* out)
{
    const int nt = 2 * ell + 1;
    const double r0n = std::sqrt(r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
    std::vector<cd> half(nt), spec(nt);
    std::vector<double> P(ell + 1);
    for (int j = 0; j < nt; ++j) {
        double th = 2.0 * kPi * j / nt;
        double s[3] = {std::cos(phi) * std::sin(th), std::sin(phi) * std::sin(th), std::cos(th)};
        double t = (s[0] * r0[0] + s[1] * r0[1] + s[2] * r0[2]) / r0n;
        t = std::max(-1.0, std::min(1.0, t));
        legendre(ell, t, P.data());
        cd acc(0.0, 0.0);
        for (int n = 0; n <= ell; ++n) acc += cn[n] * P[n];
        half[j] = 0.5 * acc;
    }
    for (int p = -ell; p <= ell; ++p) {
        cd acc(0.0, 0.0);
        for (int j = 0; j < nt; ++j) {
            double a = -2.0 * kPi * (double)((long)p * j % nt) / nt;
            acc += half[j] * cd(std::cos(a), std::sin(a));
        }
        spec[p + ell] = acc / (double)nt;
    }
    for (int k = -kmax; k <= kmax; ++k) {
        cd acc(0.0, 0.0);
        for (int p = -ell; p <= ell; ++p) acc += sin_abs_coeff(k - p) * spec[p + ell];
        out[k + kmax] = acc;
    }
}

// c_n = (i ka / 4 pi) i^n (2n+1) h_n(ka |r0|), n = 0..ell (eqn. TransferFn, box units).
static std::vector<cd> transfer_coeffs(double ka, double r0n, int ell)
{
    std::vector<double> jn(ell + 1), yn(ell + 1);
    sph_bessel_j(ell, ka * r0n, jn.data());
    sph_bessel_y(ell, ka * r0n, yn.data());
    std::vector<cd> c(ell + 1);
    cd ipow(1.0, 0.0);
    for (int n = 0; n <= ell; ++n) {
        c[n] = cd(0.0, ka / (4.0 * kPi)) * ipow * (2.0 * n + 1.0) * cd(jn[n], yn[n]);
        ipow *= cd(0.0, 1.0);
    }
    return c;
}

int select_ntheta(double ka, double r, double r0, int ell, double eps)
{
    const int nmax = 4 * ell + 64;
    const int kmax = nmax / 2 - 1;
    const double z[3] = {0.0, 0.0, r0};
    std::vector<cd> cn = transfer_coeffs(ka, r0, ell);
    std::vector<cd> spec(2 * kmax + 1);
    bmtf_column_spectrum(ka, z, ell, 0.0, kmax, cn, spec.data());
    std::vector<double> e(nmax + 1);
    bessel_j_abs(nmax, ka * r, e.data());
    const double tol = eps / (4.0 * kPi * kPi);
    for (int nth = 2 * ell; nth <= nmax; nth += 2) {
        double acc = 0.0;
        for (int k = -kmax; k <= kmax; ++k) {
            int ak = std::abs(k);
            int m = (ak < nth / 2) ? nth - ak : ak;
            acc += std::abs(spec[k + kmax]) * e[m];
        }
        if (acc < tol) return nth;
    }
    return nmax;
}

void select_nphi(double ka, double r, double r0, int ell, int ntheta, double eps, int* nphi)
{
    const int nc = 2 * ell + 1;
    const int kmax = ntheta / 2 - 1;
    const int rows = ntheta / 2 + 1;
    const double x[3] = {r0, 0.0, 0.0};
    std::vector<cd> cn = transfer_coeffs(ka, r0, ell);
    // T^{s,L}(theta_n, phi_m) for the 2 ell + 1 phi columns
    std::vector<cd> grid((size_t)rows * nc), spec(2 * kmax + 1);
    for (int m = 0; m < nc; ++m) {
        double phi = 2.0 * kPi * m / nc;
        bmtf_column_spectrum(ka, x, ell, phi, kmax, cn, spec.data());
        for (int n = 0; n < rows; ++n) {
            double th = 2.0 * kPi * n / ntheta;
            cd acc(0.0, 0.0);
            for (int k = -kmax; k <= kmax; ++k) acc += spec[k + kmax] * std::exp(cd(0.0, k * th));
            grid[(size_t)n * nc + m] = acc;
        }
    }
    const int nphi_max = 4 * ((2 * ell + 2 + 64 + 3) / 4);
    const double tol = eps / (4.0 * kPi * kPi);
    std::vector<double> coef(nc), e(nphi_max + 1);
    std::vector<int> out(rows);
    for (int n = 0; n < rows; ++n) {
        for (int p = -ell; p <= ell; ++p) {
            cd acc(0.0, 0.0);
            for (int m = 0; m < nc; ++m) {
                double a = -2.0 * kPi * (double)((long)p * m % nc) / nc;
                acc += grid[(size_t)n * nc + m] * cd(std::cos(a), std::sin(a));
            }
            coef[p + ell] = std::abs(acc / (double)nc);
        }
        double st = std::fabs(std::sin(2.0 * kPi * n / ntheta));
        bessel_j_abs(nphi_max, ka * r * st, e.data());
        out[n] = nphi_max;
        for (int np = 4; np <= nphi_max; np += 4) {
            double acc = 0.0;
            for (int p = -ell; p <= ell; ++p) {
                int ap = std::abs(p);
                int m = (ap < np / 2) ? np - ap : ap;
                acc += coef[p + ell] * e[m];
            }
            if (acc < tol) {
                out[n] = np;
                break;
            }
        }
    }
    for (int n = 0; n < rows; ++n) nphi[n] = std::max(out[n], out[rows - 1 - n]);
}

// The representative |r| = alpha sqrt(3) of Section 3.3.3 for one level. The paper's alpha (0.8)
// stands for the typical pair of interacting points; pairs near opposite corners reach |r| =
// sqrt(3). The truncation rule places ell just past ka|r| (Section 2.1), so for large ka an ell
// chosen at 0.8 sqrt(3) leaves those pairs short of it and their error exceeds eps: above kWideKa
// the full diagonal (alpha = 1) is used whenever some ell reaches eps there.
double design_alpha(double ka, double alpha, double eps, double u)
{
    if (!(ka > kWideKa) || alpha >= 1.0) return alpha;
    const double r = std::sqrt(3.0);
    const int emax = ell_search_max(ka, r);
    std::vector<double> tot(emax + 1);
    predicted_error(ka, r, 2.0, emax, u, tot.data());
    for (int l = 1; l <= emax; ++l)
        if (tot[l] < eps) return 1.0;
    return alpha;
}

void level_params(double ka, double alpha, double eps, double u, int ell_in, LevelParams* lp)
{
    const double r = design_alpha(ka, alpha, eps, u) * std::sqrt(3.0), r0 = 2.0;
    if (ell_in > 0) {
        lp->ell = ell_in;
        int emax = std::max(ell_in, 1);
        std::vector<double> tot(emax + 1);
        predicted_error(ka, r, r0, emax, u, tot.data());
        lp->predicted = tot[ell_in];
    } else {
        lp->ell = select_ell(ka, r, r0, eps, u, &lp->predicted);
    }
    lp->ntheta = select_ntheta(ka, r, r0, lp->ell, eps);
    lp->nphi.assign(lp->ntheta / 2 + 1, 4);
    select_nphi(ka, r, r0, lp->ell, lp->ntheta, eps, lp->nphi.data());
}

bool leaf_feasible(double ka_leaf, double alpha, double eps, double u)
{
    double pred = 0.0;
    select_ell(ka_leaf, alpha * std::sqrt(3.0), 2.0, 0.0, u, &pred);
    return pred < eps;
}

}  // namespace ffmm
