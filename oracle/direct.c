/* Direct O(N^2) Helmholtz sums in FP64 -- TEST INFRASTRUCTURE ONLY (the oracle).
 *
 * sigma_i = sum_{j != i} e^{i kappa R_ij} / R_ij q_j        (Section 2, eqn. HelmholtzMatrixVector)
 * F_i     = sum_{j != i} G'(R_ij) (x_i - x_j) / R_ij q_j,   G'(R) = e^{i kappa R} (i kappa R - 1) / R^2
 *           (the gradient of sigma_i with respect to x_i; used for position gradients)
 * Pairs at distance exactly 0 are skipped like j = i. Complex values are interleaved (re, im).
 * Each target's sum is accumulated in blocks of 256 sources, then the block sums are added, to
 * keep the FP64 rounding of the long sums small. */
#include <math.h>
#include <stdint.h>

#define BLK 256

void oracle_direct_matvec(int64_t n, const double* x, const double* q, double kappa,
                          int64_t ntarg, const int64_t* targ, double* out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ntarg; ++t) {
        int64_t i = targ ? targ[t] : t;
        double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
        double sr = 0.0, si = 0.0;
        for (int64_t j0 = 0; j0 < n; j0 += BLK) {
            int64_t j1 = j0 + BLK < n ? j0 + BLK : n;
            double br = 0.0, bi = 0.0;
            for (int64_t j = j0; j < j1; ++j) {
                double dx = xi - x[3 * j], dy = yi - x[3 * j + 1], dz = zi - x[3 * j + 2];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                if (j == i || r == 0.0) continue;
                double c = cos(kappa * r) / r, s = sin(kappa * r) / r;
                br += c * q[2 * j] - s * q[2 * j + 1];
                bi += c * q[2 * j + 1] + s * q[2 * j];
            }
            sr += br;
            si += bi;
        }
        out[2 * t] = sr;
        out[2 * t + 1] = si;
    }
}

void oracle_direct_gradient(int64_t n, const double* x, const double* q, double kappa,
                            int64_t ntarg, const int64_t* targ, double* out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ntarg; ++t) {
        int64_t i = targ ? targ[t] : t;
        double xi[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int64_t j0 = 0; j0 < n; j0 += BLK) {
            int64_t j1 = j0 + BLK < n ? j0 + BLK : n;
            double b[6] = {0, 0, 0, 0, 0, 0};
            for (int64_t j = j0; j < j1; ++j) {
                double d[3] = {xi[0] - x[3 * j], xi[1] - x[3 * j + 1], xi[2] - x[3 * j + 2]};
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (j == i || r == 0.0) continue;
                /* G'(R)/R = e^{i kappa R} (i kappa R - 1) / R^3 */
                double c = cos(kappa * r), s = sin(kappa * r), r3 = r * r * r;
                double gr = (-c - s * kappa * r) / r3;  /* Re[(c + i s)(-1 + i kappa r)] / r^3 */
                double gi = (c * kappa * r - s) / r3;   /* Im[...] / r^3 */
                double vr = gr * q[2 * j] - gi * q[2 * j + 1];
                double vi = gr * q[2 * j + 1] + gi * q[2 * j];
                for (int a = 0; a < 3; ++a) {
                    b[2 * a] += d[a] * vr;
                    b[2 * a + 1] += d[a] * vi;
                }
            }
            for (int a = 0; a < 6; ++a) acc[a] += b[a];
        }
        for (int a = 0; a < 6; ++a) out[6 * t + a] = acc[a];
    }
}
