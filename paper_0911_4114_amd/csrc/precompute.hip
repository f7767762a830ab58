// Plan-time tables of every level (FP64 arithmetic; stored in the plan precision):
//  * level quadrature (Section 3.4): rows theta_n = 2 pi n / N_theta, n = 0..N_theta/2, row n with
//    N_phi(theta_n) samples at phi_m = 2 pi m / N_phi(theta_n); s = [cos phi sin theta,
//    sin phi sin theta, cos theta]; leaf weights 4 pi^2 / (N_theta N_phi(theta_n)), doubled for
//    the interior rows because each also stands for row N_theta - n (eqn. eps_T folded onto the
//    stored half, eqn. NumSphereSym);
//  * band-limited modified transfer functions T^{s,LL} of the 316 transfer vectors (Alg. BMTF,
//    Section 3.2, then the per-row phi anterpolation of Section 3.3.2), computed on the GPU;
//  * translation tables e^{i kappa s.(c_child - c_parent)} for the 8 child octants;
//  * the real Fourier-resample operators of the five-step inter/anterpolation (Section 3.4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "internal.hpp"

namespace ffmm {

namespace {

using cd = std::complex<double>;
constexpr double kPi = 3.14159265358979323846;

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// A[ob][j][m] = 1/2 sum_n c_n P_n(s(theta'_j, phi_m) . r0hat), theta'_j = 2 pi j / (2 ell + 1),
// phi_m = 2 pi m / ncols (eqn. TransferFn; the 1/2 of T^s = 1/2 T |sin|).
__global__ void bmtf_sample(int nb, int ell, int ncols, const double2* __restrict__ cn,
                            const double* __restrict__ r0hat, double2* __restrict__ A)
{
    const int nt = 2 * ell + 1;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nb * nt * ncols;
    if (idx >= total) return;
    const int m = (int)(idx % ncols);
    const int j = (int)((idx / ncols) % nt);
    const int ob = (int)(idx / ((int64_t)ncols * nt));
    double st, ct, sp, cp;
    sincospi(2.0 * j / nt, &st, &ct);
    sincospi(2.0 * m / ncols, &sp, &cp);
    const double* rh = r0hat + 3 * ob;
    double t = cp * st * rh[0] + sp * st * rh[1] + ct * rh[2];
    t = fmin(1.0, fmax(-1.0, t));
    const double2* c = cn + (int64_t)ob * (ell + 1);
    double p0 = 1.0, p1 = t;
    double re = c[0].x, im = c[0].y;
    if (ell >= 1) {
        re += c[1].x * p1;
        im += c[1].y * p1;
    }
    for (int n = 1; n < ell; ++n) {
        double p2 = ((2.0 * n + 1.0) * t * p1 - n * p0) / (n + 1.0);
        re += c[n + 1].x * p2;
        im += c[n + 1].y * p2;
        p0 = p1;
        p1 = p2;
    }
    A[idx] = make_double2(0.5 * re, 0.5 * im);
}

// TL[ob][n][m] = sum_j B[n][j] A[ob][j][m]: theta Fourier coefficients of the samples, convolved
// with the |sin| coefficients, truncated to |k| <= N_theta/2 - 1 and evaluated at theta_n; the
// three linear steps of Alg. BMTF folded into the real matrix B (host).
__global__ void bmtf_theta(int nb, int nt, int rows, int ncols, const double* __restrict__ B,
                           const double2* __restrict__ A, double2* __restrict__ TL)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nb * rows * ncols;
    if (idx >= total) return;
    const int m = (int)(idx % ncols);
    const int n = (int)((idx / ncols) % rows);
    const int ob = (int)(idx / ((int64_t)ncols * rows));
    const double2* a = A + (int64_t)ob * nt * ncols + m;
    const double* b = B + (int64_t)n * nt;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < nt; ++j) {
        double2 v = a[(int64_t)j * ncols];
        re += b[j] * v.x;
        im += b[j] * v.y;
    }
    TL[idx] = make_double2(re, im);
}

// Per row: phi Fourier coefficients c_mu, |mu| <= ncols/2 - 1, of the ncols samples
// (tw[t] = e^{-2 pi i t / ncols}). Cf[ob][n][mu + ncols/2 - 1].
__global__ void bmtf_phi_coef(int nb, int rows, int ncols, const double2* __restrict__ tw,
                              const double2* __restrict__ TL, double2* __restrict__ Cf)
{
    const int nc = ncols - 1;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nb * rows * nc;
    if (idx >= total) return;
    const int mu = (int)(idx % nc) - (ncols / 2 - 1);
    const int64_t rowid = idx / nc;
    const double2* row = TL + rowid * ncols;
    double cr = 0.0, ci = 0.0;
    for (int m = 0; m < ncols; ++m) {
        long t = ((long)mu * m) % ncols;
        if (t < 0) t += ncols;
        double2 w = tw[t];
        double2 v = row[m];
        cr += v.x * w.x - v.y * w.y;
        ci += v.x * w.y + v.y * w.x;
    }
    Cf[idx] = make_double2(cr / ncols, ci / ncols);
}

// Each row evaluated at its own N_phi(theta_n) points keeping |mu| <= min(ncols, N_phi)/2 - 1
// (Section 3.3.2: the anterpolation from the full column count to N_phi(theta_n)).
__global__ void bmtf_phi_eval(int nb, int rows, int ncols, int K, const int32_t* __restrict__ row_off,
                              const int32_t* __restrict__ nphi, const int32_t* __restrict__ row_of_k,
                              const double2* __restrict__ Cf, double2* __restrict__ out)
{
    const int nc = ncols - 1;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nb * K;
    if (idx >= total) return;
    const int k = (int)(idx % K);
    const int ob = (int)(idx / K);
    const int n = row_of_k[k];
    const int len = nphi[n];
    const int jp = k - row_off[n];
    const int band = min(ncols, len) / 2 - 1;
    const double2* c = Cf + ((int64_t)ob * rows + n) * nc + (ncols / 2 - 1);
    double re = 0.0, im = 0.0;
    for (int mu = -band; mu <= band; ++mu) {
        long t = ((long)mu * jp) % len;
        if (t < 0) t += len;
        double sn, cs;
        sincospi(2.0 * (double)t / len, &sn, &cs);
        double2 v = c[mu];
        re += v.x * cs - v.y * sn;
        im += v.x * sn + v.y * cs;
    }
    out[idx] = make_double2(re, im);
}

template <class R>
__global__ void to_precision(const double2* __restrict__ in, int64_t n, void* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if constexpr (sizeof(R) == 8) {
        ((double2*)out)[i] = in[i];
    } else {
        ((float2*)out)[i] = make_float2((float)in[i].x, (float)in[i].y);
    }
}

// |sin t| Fourier coefficient (Section 3.1.3)
double sin_abs_coeff(long n)
{
    if (n % 2 != 0) return 0.0;
    double nn = (double)n;
    return 2.0 / (kPi * (1.0 - nn * nn));
}

// Real Fourier-resample (Dirichlet) matrix entry: samples j of N points -> sample jp of N' points,
// keeping |k| <= min(N, N')/2 - 1 (the Nyquist bin dropped):
//   (1/N) sum_{|k|<=B} e^{i k (2 pi jp / N' - 2 pi j / N)} = sin((2B+1) pi t / NN') / (N sin(pi t / NN'))
// with t = jp N - j N' reduced modulo N N' (exact integers).
double dirichlet(int N, int Np, int j, int jp)
{
    const int B = std::min(N, Np) / 2 - 1;
    const long M = (long)N * Np;
    long t = ((long)jp * N - (long)j * Np) % M;
    if (t < 0) t += M;
    if (t == 0) return (2.0 * B + 1.0) / N;
    long u = ((2L * B + 1L) * t) % (2 * M);
    double num = std::sin(kPi * (double)u / (double)M);
    double den = std::sin(kPi * (double)t / (double)M);
    return num / (N * den);
}

template <class R>
void upload_real(DeviceArena& a, void** dst, const std::vector<double>& v, hipStream_t s)
{
    std::vector<R> h(v.begin(), v.end());
    *dst = a.alloc(sizeof(R) * std::max<size_t>(h.size(), 1));
    FFMM_HIP(hipMemcpyAsync(*dst, h.data(), sizeof(R) * h.size(), hipMemcpyHostToDevice, s));
    FFMM_HIP(hipStreamSynchronize(s));
}

template <class R>
void upload_complex(DeviceArena& a, void** dst, const std::vector<cd>& v, hipStream_t s)
{
    std::vector<R> h(2 * v.size());
    for (size_t i = 0; i < v.size(); ++i) {
        h[2 * i] = (R)v[i].real();
        h[2 * i + 1] = (R)v[i].imag();
    }
    *dst = a.alloc(sizeof(R) * std::max<size_t>(h.size(), 1));
    FFMM_HIP(hipMemcpyAsync(*dst, h.data(), sizeof(R) * h.size(), hipMemcpyHostToDevice, s));
    FFMM_HIP(hipStreamSynchronize(s));
}

int32_t* upload_int(DeviceArena& a, const std::vector<int>& v, hipStream_t s)
{
    int32_t* d = a.alloc_n<int32_t>(std::max<size_t>(v.size(), 1));
    FFMM_HIP(hipMemcpyAsync(d, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice, s));
    FFMM_HIP(hipStreamSynchronize(s));
    return d;
}

// The real matrix B of the BMTF theta step: T^{s,L}(theta_n) = sum_j B[n][j] T(theta'_j), with
//   B[n][j] = Re sum_{|k|<=kmax} e^{i k theta_n} sum_{|p|<=ell} s_{k-p} e^{-i p theta'_j} / nt,
// theta'_j = 2 pi j / nt (nt = 2 ell + 1 samples of T), theta_n = 2 pi n / N_theta, kmax =
// N_theta/2 - 1, s the |sin| coefficients (Section 3.2, Alg. BMTF). Two O(ell^3) contractions,
// on the device: C[k][j] = sum_p s_{k-p} e^{-i p theta'_j}, then B.
__global__ void bmtf_conv(int ell, int kmax, const double2* __restrict__ tw, double2* __restrict__ C)
{
    const int nt = 2 * ell + 1;
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)(2 * kmax + 1) * nt) return;
    const int j = (int)(idx % nt);
    const int k = (int)(idx / nt) - kmax;
    double re = 0.0, im = 0.0;
    for (int pp = -ell; pp <= ell; ++pp) {
        const long d = (long)k - pp;
        if (d % 2 != 0) continue;
        const double sk = 2.0 / (kPi * (1.0 - (double)d * (double)d));
        long t = ((long)pp * j) % nt;
        if (t < 0) t += nt;
        const double2 w = tw[t];
        re += sk * w.x;
        im += sk * w.y;
    }
    C[idx] = make_double2(re, im);
}

__global__ void bmtf_rows(int nt, int kmax, int rows, int ntheta, const double2* __restrict__ tw2,
                          const double2* __restrict__ C, double* __restrict__ B)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * nt) return;
    const int j = (int)(idx % nt);
    const int n = (int)(idx / nt);
    double acc = 0.0;
    for (int k = -kmax; k <= kmax; ++k) {
        long t = ((long)k * n) % ntheta;
        if (t < 0) t += ntheta;
        const double2 e = tw2[t], c = C[(int64_t)(k + kmax) * nt + j];
        acc += e.x * c.x - e.y * c.y;
    }
    B[idx] = acc / nt;
}

// B of (ell, ntheta) in device memory of arena a
double* bmtf_theta_matrix(DeviceArena& a, int ell, int ntheta, hipStream_t s)
{
    const int nt = 2 * ell + 1, kmax = ntheta / 2 - 1, rows = ntheta / 2 + 1;
    std::vector<cd> tw(nt), tw2(ntheta);
    for (int t = 0; t < nt; ++t) tw[t] = std::exp(cd(0.0, -2.0 * kPi * (double)t / nt));
    for (int t = 0; t < ntheta; ++t) tw2[t] = std::exp(cd(0.0, 2.0 * kPi * (double)t / ntheta));
    double2* dtw = a.alloc_n<double2>(nt);
    double2* dtw2 = a.alloc_n<double2>(ntheta);
    FFMM_HIP(hipMemcpyAsync(dtw, tw.data(), sizeof(double2) * nt, hipMemcpyHostToDevice, s));
    FFMM_HIP(hipMemcpyAsync(dtw2, tw2.data(), sizeof(double2) * ntheta, hipMemcpyHostToDevice, s));
    double2* C = a.alloc_n<double2>((size_t)(2 * kmax + 1) * nt);
    double* B = a.alloc_n<double>((size_t)rows * nt);
    hipLaunchKernelGGL(bmtf_conv, dim3(nblk((int64_t)(2 * kmax + 1) * nt, 256)), dim3(256), 0, s, ell, kmax,
                       dtw, C);
    FFMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(bmtf_rows, dim3(nblk((int64_t)rows * nt, 256)), dim3(256), 0, s, nt, kmax, rows,
                       ntheta, dtw2, C, B);
    FFMM_LAUNCH_CHECK();
    FFMM_HIP(hipStreamSynchronize(s));   // the host twiddle vectors go out of scope
    return B;
}

// Alg. Nphi error sums: out[n][c] = sum_{|p|<=ell} |Cf_n,p| |J_{M(N,p)}(ka r sin theta_n)| for
// N = 4 (c + 1), M(N, p) = N - |p| if |p| < N/2 else |p| (eqn. EpsIPhi's aliasing index).
__global__ void nphi_error(int rows, int ell, int ncols, int ncand, int emax,
                           const double2* __restrict__ Cf, const double* __restrict__ E,
                           double* __restrict__ out)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)rows * ncand) return;
    const int c = (int)(idx % ncand), n = (int)(idx / ncand);
    const int np = 4 * (c + 1);
    const double2* cf = Cf + (int64_t)n * (ncols - 1) + (ncols / 2 - 1);
    const double* e = E + (int64_t)n * (emax + 1);
    double acc = 0.0;
    for (int pp = -ell; pp <= ell; ++pp) {
        const int ap = pp < 0 ? -pp : pp;
        const int m = (ap < np / 2) ? np - ap : ap;
        acc += hypot(cf[pp].x, cf[pp].y) * e[m];
    }
    out[idx] = acc;
}

// Alg. Nphi with the band-limited transfer function of r0 = |r0| x (box units) computed on the
// device by the BMTF kernels (the same quantities the host search forms with O(ell^3) DFTs).
void select_nphi_device(const DeviceArena& hooks, double ka, double r, double r0, int ell, int ntheta,
                        double eps, const double* dB, int* nphi, hipStream_t s)
{
    const int rows = ntheta / 2 + 1, nt = 2 * ell + 1;
    const int ncols = 4 * ((2 * ell + 2 + 3) / 4);
    const int nphi_max = 4 * ((2 * ell + 2 + 64 + 3) / 4);
    const int ncand = nphi_max / 4;
    DeviceArena tmp;
    tmp.inherit(hooks);
    try {
        std::vector<double> jn(ell + 1), yn(ell + 1);
        sph_bessel_j(ell, ka * r0, jn.data());
        sph_bessel_y(ell, ka * r0, yn.data());
        std::vector<cd> cn(ell + 1);
        cd ipow(1.0, 0.0);
        for (int n = 0; n <= ell; ++n) {
            cn[n] = cd(0.0, ka / (4.0 * kPi)) * ipow * (2.0 * n + 1.0) * cd(jn[n], yn[n]);
            ipow *= cd(0.0, 1.0);
        }
        const double xhat[3] = {1.0, 0.0, 0.0};
        double2* dcn = tmp.alloc_n<double2>(ell + 1);
        double* dr0 = tmp.alloc_n<double>(3);
        FFMM_HIP(hipMemcpyAsync(dcn, cn.data(), sizeof(double2) * (ell + 1), hipMemcpyHostToDevice, s));
        FFMM_HIP(hipMemcpyAsync(dr0, xhat, sizeof(xhat), hipMemcpyHostToDevice, s));
        double2* A = tmp.alloc_n<double2>((size_t)nt * ncols);
        double2* TL = tmp.alloc_n<double2>((size_t)rows * ncols);
        double2* Cf = tmp.alloc_n<double2>((size_t)rows * (ncols - 1));
        std::vector<cd> tw(ncols);
        for (int t = 0; t < ncols; ++t) tw[t] = std::exp(cd(0.0, -2.0 * kPi * t / ncols));
        double2* dtw = tmp.alloc_n<double2>(ncols);
        FFMM_HIP(hipMemcpyAsync(dtw, tw.data(), sizeof(double2) * ncols, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(bmtf_sample, dim3(nblk((int64_t)nt * ncols, 256)), dim3(256), 0, s, 1, ell, ncols,
                           dcn, dr0, A);
        FFMM_LAUNCH_CHECK();
        hipLaunchKernelGGL(bmtf_theta, dim3(nblk((int64_t)rows * ncols, 256)), dim3(256), 0, s, 1, nt, rows,
                           ncols, dB, A, TL);
        FFMM_LAUNCH_CHECK();
        hipLaunchKernelGGL(bmtf_phi_coef, dim3(nblk((int64_t)rows * (ncols - 1), 256)), dim3(256), 0, s, 1,
                           rows, ncols, dtw, TL, Cf);
        FFMM_LAUNCH_CHECK();
        // |J_m(ka r sin theta_n)|, m = 0..nphi_max, per row
        std::vector<double> E((size_t)rows * (nphi_max + 1));
        for (int n = 0; n < rows; ++n)
            bessel_j_abs(nphi_max, ka * r * std::fabs(std::sin(2.0 * kPi * n / ntheta)),
                         &E[(size_t)n * (nphi_max + 1)]);
        double* dE = tmp.alloc_n<double>(E.size());
        FFMM_HIP(hipMemcpyAsync(dE, E.data(), sizeof(double) * E.size(), hipMemcpyHostToDevice, s));
        double* dout = tmp.alloc_n<double>((size_t)rows * ncand);
        hipLaunchKernelGGL(nphi_error, dim3(nblk((int64_t)rows * ncand, 256)), dim3(256), 0, s, rows, ell,
                           ncols, ncand, nphi_max, Cf, dE, dout);
        FFMM_LAUNCH_CHECK();
        std::vector<double> err((size_t)rows * ncand);
        FFMM_HIP(hipMemcpyAsync(err.data(), dout, sizeof(double) * err.size(), hipMemcpyDeviceToHost, s));
        FFMM_HIP(hipStreamSynchronize(s));
        const double tol = eps / (4.0 * kPi * kPi);
        std::vector<int> out(rows, nphi_max);
        for (int n = 0; n < rows; ++n)
            for (int c = 0; c < ncand; ++c)
                if (err[(size_t)n * ncand + c] < tol) {
                    out[n] = 4 * (c + 1);
                    break;
                }
        for (int n = 0; n < rows; ++n) nphi[n] = std::max(out[n], out[rows - 1 - n]);
    } catch (...) {
        tmp.release();
        throw;
    }
    tmp.release();
}

// Transfer tables of one level, FP64 on the device, stored in precision R.
template <class R>
void transfer_tables(ffmm_plan* p, LevelData& L, hipStream_t s)
{
    const int ell = L.par.ell, ntheta = L.par.ntheta, rows = L.nrows, K = L.K;
    const int nt = 2 * ell + 1;
    const int ncols = 4 * ((2 * ell + 2 + 3) / 4);
    DeviceArena tmp;
    tmp.inherit(p->arena);
    try {
        const double* dB = bmtf_theta_matrix(tmp, ell, ntheta, s);
        std::vector<int> row_of_k(K);
        for (int n = 0; n < rows; ++n)
            for (int k = L.row_off[n]; k < L.row_off[n + 1]; ++k) row_of_k[k] = n;
        int32_t* d_rok = upload_int(tmp, row_of_k, s);
        // the 34 representative transfer vectors (the other 282 are their images under the
        // quadrature's symmetries, read through tperm), coefficient sets per vector
        std::vector<double> r0hat(3 * kNumReps);
        std::vector<cd> cn((size_t)kNumReps * (ell + 1));
        std::vector<double> jn(ell + 1), yn(ell + 1);
        for (int o = 0; o < kNumReps; ++o) {
            int d[3];
            rep_offset(o, d);
            double len = std::sqrt((double)(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
            for (int a = 0; a < 3; ++a) r0hat[3 * o + a] = d[a] / len;
            const double r0 = len * L.a;   // physical |r0|
            sph_bessel_j(ell, p->kappa * r0, jn.data());
            sph_bessel_y(ell, p->kappa * r0, yn.data());
            cd ipow(1.0, 0.0);
            for (int n = 0; n <= ell; ++n) {
                // c_n = (i kappa / 4 pi) i^n (2n+1) h_n(kappa |r0|)  (eqn. TransferFn)
                cn[(size_t)o * (ell + 1) + n] =
                    cd(0.0, p->kappa / (4.0 * kPi)) * ipow * (2.0 * n + 1.0) * cd(jn[n], yn[n]);
                ipow *= cd(0.0, 1.0);
            }
        }
        double2* dcn = tmp.alloc_n<double2>(cn.size());
        FFMM_HIP(hipMemcpy(dcn, cn.data(), sizeof(double2) * cn.size(), hipMemcpyHostToDevice));
        double* dr0 = tmp.alloc_n<double>(r0hat.size());
        FFMM_HIP(hipMemcpy(dr0, r0hat.data(), sizeof(double) * r0hat.size(), hipMemcpyHostToDevice));
        // batch the offsets so that the samples stay below ~256 MB
        const size_t per_off = sizeof(double2) * ((size_t)nt * ncols + 2 * (size_t)rows * ncols);
        int batch = (int)std::max<size_t>(1, std::min<size_t>(kNumReps, (256u << 20) / per_off));
        double2* A = tmp.alloc_n<double2>((size_t)batch * nt * ncols);
        double2* TL = tmp.alloc_n<double2>((size_t)batch * rows * ncols);
        double2* Cf = tmp.alloc_n<double2>((size_t)batch * rows * (ncols - 1));
        double2* T64 = tmp.alloc_n<double2>((size_t)kNumReps * K);
        std::vector<cd> tw(ncols);
        for (int t = 0; t < ncols; ++t) tw[t] = std::exp(cd(0.0, -2.0 * kPi * t / ncols));
        double2* dtw = tmp.alloc_n<double2>(ncols);
        FFMM_HIP(hipMemcpy(dtw, tw.data(), sizeof(double2) * ncols, hipMemcpyHostToDevice));
        for (int o0 = 0; o0 < kNumReps; o0 += batch) {
            const int nb = std::min(batch, kNumReps - o0);
            int64_t tot = (int64_t)nb * nt * ncols;
            hipLaunchKernelGGL(bmtf_sample, dim3(nblk(tot, 256)), dim3(256), 0, s, nb, ell, ncols,
                               dcn + (size_t)o0 * (ell + 1), dr0 + 3 * o0, A);
            FFMM_LAUNCH_CHECK();
            tot = (int64_t)nb * rows * ncols;
            hipLaunchKernelGGL(bmtf_theta, dim3(nblk(tot, 256)), dim3(256), 0, s, nb, nt, rows, ncols,
                               dB, A, TL);
            FFMM_LAUNCH_CHECK();
            tot = (int64_t)nb * rows * (ncols - 1);
            hipLaunchKernelGGL(bmtf_phi_coef, dim3(nblk(tot, 256)), dim3(256), 0, s, nb, rows, ncols,
                               dtw, TL, Cf);
            FFMM_LAUNCH_CHECK();
            tot = (int64_t)nb * K;
            hipLaunchKernelGGL(bmtf_phi_eval, dim3(nblk(tot, 256)), dim3(256), 0, s, nb, rows, ncols, K,
                               L.d_row_off, L.d_nphi, d_rok, Cf, T64 + (size_t)o0 * K);
            FFMM_LAUNCH_CHECK();
        }
        const int64_t tot = (int64_t)kNumReps * K;
        L.transfer = p->arena.alloc(sizeof(R) * 2 * tot);
        hipLaunchKernelGGL(to_precision<R>, dim3(nblk(tot, 256)), dim3(256), 0, s, T64, tot, L.transfer);
        FFMM_LAUNCH_CHECK();
        // tperm[g][k]: direction g^{-1}(s_k), so that T_{g rep}(s_k) = T_rep(s_{tperm[g][k]})
        std::vector<int> perm((size_t)kNumSym * K);
        for (int g = 0; g < kNumSym; ++g)
            for (int n = 0; n < rows; ++n)
                for (int m = 0; m < L.par.nphi[n]; ++m)
                    perm[(size_t)g * K + L.row_off[n] + m] =
                        sym_direction(g, n, m, ntheta, L.par.nphi[n], L.row_off);
        L.tperm = upload_int(p->arena, perm, s);
        FFMM_HIP(hipStreamSynchronize(s));
    } catch (...) {
        tmp.release();
        throw;
    }
    tmp.release();
}

// Common phi length of steps 1-5: the smaller of the two largest row lengths. Upward the source
// rows fit on it without loss, downward the destination rows keep no mode it lacks, and the theta
// step acts on each phi mode separately; on data with the doubled-sphere symmetry (every
// signature) this gives the same operator as the largest row length of either grid.
int common_nphi(const LevelData& S, const LevelData& D)
{
    int na_s = 0, na_d = 0;
    for (int v : S.par.nphi) na_s = std::max(na_s, v);
    for (int v : D.par.nphi) na_d = std::max(na_d, v);
    return std::min(na_s, na_d);
}

// Quarter-range form of a row step y_j = sum_m D[m][j] x_m from N to M samples (both multiples of
// 4, grids starting at 0; D the Dirichlet kernel of dirichlet()). The half-range parts u (even
// modes) and v (odd modes) are split again by the reflection phi -> -phi, under which the kernel
// is even: for m = 0..N/4, with h = N/2 and x taken modulo N,
//   u_m = x_m + x_{m+h}, ub_m = x_{h-m} + x_{-m}, v_m = x_m - x_{m+h}, vb_m = x_{h-m} - x_{-m},
//   us = u + ub, ua = u - ub, vm = v - vb, vp = v + vb,
// and per output j = 0..M/4 the four sums S = Cs us, A = Ca ua, Mv = Cm vm, P = Cp vp give
//   y_j = S + A + Mv + P, y_{j+M/2} = S + A - Mv - P, and for 0 < j < M/4
//   y_{M/2-j} = S - A + P - Mv, y_{M-j} = S - A - P + Mv.
// With De, Do the half-range operators (D[m][j] +- D[m+h][j]) / 2 and r = h - m (Do at r = h is
// -Do at 0): Cs, Ca = (De[m] +- De[r]) / 2, Cm, Cp = (Do[m] -+ Do[r]) / 2, halved at the
// reflection's fixed points m = 0 and m = N/4. Stored [N/4 + 1][4][ld] (channels S, A, Mv, P; ld
// = M/4 + 1 rounded up to 4, zero padded): a quarter of the full operator's work.
void quarter_block(int N, int M, int ld, double* blk)
{
    const int h = N / 2, q = N / 4, Q = M / 4;
    for (int m = 0; m <= q; ++m) {
        const int r = (h - m) % h;
        const double wt = (m == 0 || m == q) ? 0.5 : 1.0;
        for (int j = 0; j <= Q; ++j) {
            const double a = dirichlet(N, M, m, j), b = dirichlet(N, M, m + h, j);
            const double c = m == 0 ? a : dirichlet(N, M, r, j), d = m == 0 ? b : dirichlet(N, M, r + h, j);
            const double e0 = 0.5 * (a + b), e1 = 0.5 * (c + d), o0 = 0.5 * (a - b);
            const double o1 = m == 0 ? -o0 : 0.5 * (c - d);
            blk[((size_t)m * 4 + 0) * ld + j] = wt * 0.5 * (e0 + e1);
            blk[((size_t)m * 4 + 1) * ld + j] = wt * 0.5 * (e0 - e1);
            blk[((size_t)m * 4 + 2) * ld + j] = wt * 0.5 * (o0 - o1);
            blk[((size_t)m * 4 + 3) * ld + j] = wt * 0.5 * (o0 + o1);
        }
    }
}

template <class R>
void make_resampler(ffmm_plan* p, const LevelData& S, const LevelData& D, Resampler& rs, hipStream_t s)
{
    const int na = common_nphi(S, D);
    rs.nphi_all = na;
    rs.nt_src = S.par.ntheta;
    rs.nt_dst = D.par.ntheta;
    rs.rows_src = S.nrows;
    rs.rows_dst = D.nrows;
    rs.K_src = S.K;
    rs.K_dst = D.K;
    const int ldt = rs.nt_dst;   // row stride of the full-range theta operator (host only)
    std::vector<double> dth((size_t)rs.nt_src * ldt, 0.0);
    // Half-range row steps. Every row length is even (a multiple of 4) and the phi grids start at
    // 0, so sample m + N/2 lies half a turn from sample m. With u_m = x_m + x_{m+N/2} (even modes
    // only) and v_m = x_m - x_{m+N/2} (odd modes only), a resample y_j = sum_m D[m][j] x_m onto an
    // even grid of N' points is y_j = a_j + b_j, y_{j+N'/2} = a_j - b_j for j < N'/2, with
    // a = sum_m De[m][j] u_m, b = sum_m Do[m][j] v_m over m < N/2 and
    // De, Do = (D[m][j] +- D[m + N/2][j]) / 2: the Dirichlet kernel's even frequencies are
    // unchanged by the half-turn shift, its odd ones change sign. Each operator is stored as
    // [N/2][2][ld] (De then Do per source sample, ld = N'/2 rounded up to a multiple of 4, zero
    // padded), so that one 16-byte load serves four destination samples.
    for (int v : S.par.nphi)
        if (v % 2 != 0) fail(FFMM_ERR_INTERNAL, "odd quadrature row length");
    for (int v : D.par.nphi)
        if (v % 2 != 0) fail(FFMM_ERR_INTERNAL, "odd quadrature row length");
    // quarter-range row steps where the common phi length makes the contractions long (then the
    // half-range operators of this transition are not built)
    bool mult4 = na % 4 == 0;
    for (int v : S.par.nphi) mult4 = mult4 && v % 4 == 0;
    for (int v : D.par.nphi) mult4 = mult4 && v % 4 == 0;
    rs.quarter = mult4 && na >= (p->opt.quarter_nphi > 0 ? p->opt.quarter_nphi : kQuarterMinNphi);
    const int H = na / 2;
    rs.ldj = (H + 3) / 4 * 4;
    std::vector<double> d1h(rs.quarter ? 0 : (size_t)S.K * rs.ldj, 0.0);
    for (int n = 0; n < S.nrows && !rs.quarter; ++n) {
        const int len = S.par.nphi[n], h = len / 2;
        double* blk = &d1h[(size_t)S.row_off[n] * rs.ldj];   // (row_off / 2) source pairs x 2 x ldj
        for (int m = 0; m < h; ++m)
            for (int j = 0; j < H; ++j) {
                const double a = dirichlet(len, na, m, j), b = dirichlet(len, na, m + h, j);
                blk[((size_t)m * 2 + 0) * rs.ldj + j] = 0.5 * (a + b);
                blk[((size_t)m * 2 + 1) * rs.ldj + j] = 0.5 * (a - b);
            }
    }
    std::vector<int> off5(D.nrows + 1, 0);
    if (!rs.quarter) {
        int64_t o = 0;
        for (int n = 0; n < D.nrows; ++n) {
            o += (int64_t)H * 2 * ((D.par.nphi[n] / 2 + 3) / 4 * 4);
            if (o > INT32_MAX) fail(FFMM_ERR_UNSUPPORTED, "step-5 operator exceeds 2^31 elements");
            off5[n + 1] = (int)o;
        }
    }
    std::vector<double> d5h((size_t)off5[D.nrows], 0.0);
    for (int n = 0; n < D.nrows && !rs.quarter; ++n) {
        const int len = D.par.nphi[n], h = len / 2, ld = (h + 3) / 4 * 4;
        double* blk = &d5h[(size_t)off5[n]];
        for (int j = 0; j < H; ++j)
            for (int jp = 0; jp < h; ++jp) {
                const double a = dirichlet(na, len, j, jp), b = dirichlet(na, len, j + H, jp);
                blk[((size_t)j * 2 + 0) * ld + jp] = 0.5 * (a + b);
                blk[((size_t)j * 2 + 1) * ld + jp] = 0.5 * (a - b);
            }
    }
    for (int t = 0; t < rs.nt_src; ++t)
        for (int tp = 0; tp < rs.nt_dst; ++tp)
            dth[(size_t)t * ldt + tp] = dirichlet(rs.nt_src, rs.nt_dst, t, tp);
    if (!rs.quarter) upload_real<R>(p->arena, &rs.d1h, d1h, s);
    if (rs.quarter) {
        const int Q = na / 4;
        rs.ldq = (Q + 1 + 3) / 4 * 4;
        std::vector<int> o1(S.nrows), o5(D.nrows);
        int64_t t1 = 0, t5 = 0;
        for (int n = 0; n < S.nrows; ++n) {
            o1[n] = (int)t1;
            t1 += (int64_t)(S.par.nphi[n] / 4 + 1) * 4 * rs.ldq;
        }
        for (int n = 0; n < D.nrows; ++n) {
            o5[n] = (int)t5;
            t5 += (int64_t)(Q + 1) * 4 * ((D.par.nphi[n] / 4 + 1 + 3) / 4 * 4);
        }
        if (t1 > INT32_MAX || t5 > INT32_MAX) fail(FFMM_ERR_UNSUPPORTED, "quarter-range operator exceeds 2^31 elements");
        std::vector<double> q1((size_t)t1, 0.0), q5((size_t)t5, 0.0);
        for (int n = 0; n < S.nrows; ++n) quarter_block(S.par.nphi[n], na, rs.ldq, &q1[o1[n]]);
        for (int n = 0; n < D.nrows; ++n)
            quarter_block(na, D.par.nphi[n], (D.par.nphi[n] / 4 + 1 + 3) / 4 * 4, &q5[o5[n]]);
        upload_real<R>(p->arena, &rs.d1q, q1, s);
        upload_real<R>(p->arena, &rs.d5q, q5, s);
        rs.d1q_off = upload_int(p->arena, o1, s);
        rs.d5q_off = upload_int(p->arena, o5, s);
    }
    {
        // half-range theta operators: an even (odd) circle sequence x, x(N - t) = +-x(t), is
        // resampled by sum over the half range of x(t) (D[t][t'] +- D[N - t][t']), the rows t = 0,
        // N/2 counted once (even) or vanishing (odd)
        const int ns = rs.nt_src, nsh = ns / 2 + 1, ndh = rs.nt_dst / 2 + 1;
        rs.ldh = (ndh + 3) / 4 * 4;
        std::vector<double> dh(2 * (size_t)nsh * rs.ldh, 0.0);
        double* de = dh.data();
        double* dodd = dh.data() + (size_t)nsh * rs.ldh;
        for (int t = 0; t < nsh; ++t)
            for (int tp = 0; tp < ndh; ++tp) {
                const double a = dth[(size_t)t * ldt + tp];
                const bool edge = (t == 0 || 2 * t == ns);
                const double b = edge ? 0.0 : dth[(size_t)(ns - t) * ldt + tp];
                de[(size_t)t * rs.ldh + tp] = 0.5 * (a + b);
                dodd[(size_t)t * rs.ldh + tp] = edge ? 0.0 : 0.5 * (a - b);
            }
        upload_real<R>(p->arena, &rs.dth_h, dh, s);
    }
    if (!rs.quarter) {
        upload_real<R>(p->arena, &rs.d5h, d5h, s);
        off5.pop_back();
        rs.d5h_off = upload_int(p->arena, off5, s);
    }
    rs.d_src_row_off = S.d_row_off;
    rs.d_src_nphi = S.d_nphi;
    rs.d_dst_row_off = D.d_row_off;
    rs.d_dst_nphi = D.d_nphi;
    std::vector<int> rok(D.K);
    for (int n = 0; n < D.nrows; ++n)
        for (int k = D.row_off[n]; k < D.row_off[n + 1]; ++k) rok[k] = n;
    rs.d_dst_row_of_k = upload_int(p->arena, rok, s);
}

template <class R>
void build_tables_t(ffmm_plan* p, hipStream_t s)
{
    const int depth = p->depth;
    const double u = p->prec == FFMM_FP32 ? kUnitRoundoffFP32 : kUnitRoundoffFP64;
    p->predicted.assign(depth + 1, 0.0);
    for (int l = 2; l <= depth; ++l) {
        LevelData& L = p->lev[l];
        const double ka = p->kappa * L.a;
        const int ell_in = (l < FFMM_MAX_LEVELS) ? p->opt.ell_override[l] : 0;
        {
            // ell and N_theta on the host (O(ell^2)); the O(ell^3) N_phi search on the device
            LevelParams& lp = L.par;
            const double eps_l = p->opt.eps_safety * p->eps;
            const double r = design_alpha(ka, p->opt.alpha, eps_l, u) * std::sqrt(3.0), r0 = 2.0;
            if (ell_in > 0) {
                lp.ell = ell_in;
                std::vector<double> tot(ell_in + 1);
                predicted_error(ka, r, r0, ell_in, u, tot.data());
                lp.predicted = tot[ell_in];
            } else {
                lp.ell = select_ell(ka, r, r0, eps_l, u, &lp.predicted);
            }
            // the truncation and rounding floor of this level alone already exceed the target
            // (low-frequency breakdown at every admissible depth, Section 3.5.1)
            if (lp.predicted > p->eps && !p->opt.best_effort)
                fail(FFMM_ERR_ACCURACY,
                     "level " + std::to_string(l) + " (kappa a = " + std::to_string(ka) +
                         ") cannot reach eps = " + std::to_string(p->eps) + ": predicted error " +
                         std::to_string(lp.predicted) +
                         " (low-frequency breakdown); set options.best_effort to build it anyway");
            lp.ntheta = select_ntheta(ka, r, r0, lp.ell, eps_l);
            lp.nphi.assign(lp.ntheta / 2 + 1, 4);
            DeviceArena bt;
            bt.inherit(p->arena);
            try {
                const double* dB = bmtf_theta_matrix(bt, lp.ell, lp.ntheta, s);
                select_nphi_device(p->arena, ka, r, r0, lp.ell, lp.ntheta, eps_l, dB, lp.nphi.data(), s);
            } catch (...) {
                bt.release();
                throw;
            }
            bt.release();
        }
        p->predicted[l] = L.par.predicted;
        L.nrows = L.par.ntheta / 2 + 1;
        {
            // quadrature sizes whose table rows and signatures stay below 2^31 bytes per box
            // (32-bit byte offsets inside one row in the M2L table reads)
            int64_t k64 = 0;
            for (int n = 0; n < L.nrows; ++n) k64 += L.par.nphi[n];
            if (k64 * (int64_t)(2 * sizeof(R)) > (int64_t)INT32_MAX)
                fail(FFMM_ERR_UNSUPPORTED, "level " + std::to_string(l) + " quadrature of " +
                                               std::to_string(k64) + " directions exceeds 2^31 bytes per box");
        }
        L.row_off.assign(L.nrows + 1, 0);
        for (int n = 0; n < L.nrows; ++n) L.row_off[n + 1] = L.row_off[n] + L.par.nphi[n];
        L.K = L.row_off[L.nrows];
        L.d_row_off = upload_int(p->arena, L.row_off, s);
        L.d_nphi = upload_int(p->arena, L.par.nphi, s);
        // directions (and leaf weights)
        std::vector<double> dirs(3 * (size_t)L.K), w(L.K);
        for (int n = 0; n < L.nrows; ++n) {
            const double th = 2.0 * kPi * n / L.par.ntheta;
            const int len = L.par.nphi[n];
            const double wn = 4.0 * kPi * kPi / ((double)L.par.ntheta * len) *
                              ((n == 0 || n == L.nrows - 1) ? 1.0 : 2.0);
            for (int m = 0; m < len; ++m) {
                const double ph = 2.0 * kPi * m / len;
                const int k = L.row_off[n] + m;
                dirs[3 * k] = std::cos(ph) * std::sin(th);
                dirs[3 * k + 1] = std::sin(ph) * std::sin(th);
                dirs[3 * k + 2] = std::cos(th);
                w[k] = wn;
            }
        }
        upload_real<R>(p->arena, &L.dirs, dirs, s);
        if (l == depth) upload_real<R>(p->arena, &L.weights, w, s);
        {
            // antipodal pairs: row theta_n at phi_m and row pi - theta_n (index N_theta/2 - n) at
            // phi_m + pi give s and -s; the rows have equal N_phi (Alg. Nphi takes the larger of
            // the two) and every N_phi is a multiple of 4, so all K directions pair up
            const int half = L.par.ntheta / 2;
            std::vector<int> pr;
            pr.reserve(L.K);
            for (int n = 0; n <= half - n; ++n) {
                const int n2 = half - n, len = L.par.nphi[n];
                if (L.par.nphi[n2] != len || len % 2 != 0) fail(FFMM_ERR_INTERNAL, "unpaired quadrature rows");
                for (int m = 0; m < (n == n2 ? len / 2 : len); ++m) {
                    pr.push_back(L.row_off[n] + m);
                    pr.push_back(L.row_off[n2] + (m + len / 2) % len);
                }
            }
            if ((int)pr.size() != L.K) fail(FFMM_ERR_INTERNAL, "unpaired quadrature directions");
            L.Kp = L.K / 2;
            L.pairs = upload_int(p->arena, pr, s);
        }
        transfer_tables<R>(p, L, s);
        if (l < depth) {
            // e^{i kappa s.(oct - 1/2) a_{l+1}}, oct = (x, y, z) bits of the child position
            const double ac = p->lev[l + 1].a;
            std::vector<cd> tr(8 * (size_t)L.K);
            for (int o = 0; o < 8; ++o) {
                const double d[3] = {((o & 1) - 0.5) * ac, (((o >> 1) & 1) - 0.5) * ac,
                                     (((o >> 2) & 1) - 0.5) * ac};
                for (int k = 0; k < L.K; ++k) {
                    const double ph = p->kappa * (dirs[3 * k] * d[0] + dirs[3 * k + 1] * d[1] +
                                                  dirs[3 * k + 2] * d[2]);
                    tr[(size_t)o * L.K + k] = cd(std::cos(ph), std::sin(ph));
                }
            }
            upload_complex<R>(p->arena, &L.trans, tr, s);
            // octants o + 4 and o differ by a_{l+1} in z only: their translations differ by a
            // factor that is constant on each theta row
            std::vector<cd> zr(L.nrows);
            for (int n = 0; n < L.nrows; ++n) {
                const double ph = p->kappa * dirs[3 * (size_t)L.row_off[n] + 2] * ac;
                zr[n] = cd(std::cos(ph), std::sin(ph));
            }
            upload_complex<R>(p->arena, &L.zrot, zr, s);
        }
    }
    p->up.assign(depth + 1, Resampler{});
    p->down.assign(depth + 1, Resampler{});
    for (int l = 3; l <= depth; ++l) {
        // z pairs of the children of level l - 1, and the upward tiles over them
        LevelData& Cl = p->lev[l];
        LevelData& Pl = p->lev[l - 1];
        std::vector<int32_t> oct(Cl.n), cs(Pl.n), cc(Pl.n);
        FFMM_HIP(hipMemcpy(oct.data(), Cl.octant, sizeof(int32_t) * Cl.n, hipMemcpyDeviceToHost));
        FFMM_HIP(hipMemcpy(cs.data(), Pl.child_start, sizeof(int32_t) * Pl.n, hipMemcpyDeviceToHost));
        FFMM_HIP(hipMemcpy(cc.data(), Pl.child_count, sizeof(int32_t) * Pl.n, hipMemcpyDeviceToHost));
        std::vector<int> zlo, zhi, zpar, zoct, zst(Pl.n), zct(Pl.n);
        for (int64_t pp = 0; pp < Pl.n; ++pp) {
            int at[8];
            std::fill(at, at + 8, -1);
            for (int c = cs[pp]; c < cs[pp] + cc[pp]; ++c) at[oct[c]] = c;
            zst[pp] = (int)zlo.size();
            for (int o = 0; o < 4; ++o) {
                if (at[o] < 0 && at[o + 4] < 0) continue;
                zlo.push_back(at[o] >= 0 ? at[o] : at[o + 4]);
                zhi.push_back(at[o] >= 0 ? at[o + 4] : -1);
                zpar.push_back((int)pp);
                zoct.push_back(at[o] >= 0 ? o : o + 4);
            }
            zct[pp] = (int)zlo.size() - zst[pp];
        }
        std::vector<int> zsrc(Cl.n, -1);
        for (size_t e = 0; e < zlo.size(); ++e)
            if (zhi[e] >= 0) zsrc[zhi[e]] = zlo[e];
        Cl.nz = (int64_t)zlo.size();
        Cl.zlo = upload_int(p->arena, zlo, s);
        Cl.zhi = upload_int(p->arena, zhi, s);
        Cl.zsrc = upload_int(p->arena, zsrc, s);
        Cl.zpar = upload_int(p->arena, zpar, s);
        Cl.zoct = upload_int(p->arena, zoct, s);
        Pl.zstart = upload_int(p->arena, zst, s);
        Pl.zcount = upload_int(p->arena, zct, s);
        std::vector<int32_t> tb, te;
        make_parent_tiles(std::vector<int32_t>(zct.begin(), zct.end()), tb, te);
        std::vector<int> pb(tb.size()), pe(tb.size());
        for (size_t t = 0; t < tb.size(); ++t) {
            pb[t] = zpar[tb[t]];
            pe[t] = zpar[te[t] - 1] + 1;
        }
        Resampler& ru = p->up[l];
        // the upward theta step's columns: per pair and phi_m the members present (lo, or lo and
        // hi side by side), so a pair takes NPhi/2 columns per member; each 32-column tile starts
        // in the pair recorded for it
        {
            const int64_t half = common_nphi(Cl, Pl) / 2;
            std::vector<int> zmp(zlo.size() + 1, 0);
            for (size_t e = 0; e < zlo.size(); ++e) zmp[e + 1] = zmp[e] + (zhi[e] >= 0 ? 2 : 1);
            const int64_t ncol = half * zmp.back();
            std::vector<int> tp0((ncol + 31) / 32);
            size_t e = 0;
            for (size_t t = 0; t < tp0.size(); ++t) {
                while (half * zmp[e + 1] <= 32 * (int64_t)t) ++e;
                tp0[t] = (int)e;
            }
            Cl.zmp = upload_int(p->arena, zmp, s);
            ru.zcol_tile = upload_int(p->arena, tp0, s);
        }
        ru.nztiles = (int)tb.size();
        ru.ztile_begin = upload_int(p->arena, std::vector<int>(tb.begin(), tb.end()), s);
        ru.ztile_end = upload_int(p->arena, std::vector<int>(te.begin(), te.end()), s);
        ru.ztile_pbeg = upload_int(p->arena, pb, s);
        ru.ztile_pend = upload_int(p->arena, pe, s);
    }
    for (int l = 3; l <= depth; ++l) make_resampler<R>(p, p->lev[l], p->lev[l - 1], p->up[l], s);
    for (int l = 2; l < depth; ++l) make_resampler<R>(p, p->lev[l], p->lev[l + 1], p->down[l], s);
}

}  // namespace

void build_tables(ffmm_plan* p, hipStream_t s)
{
    if (p->prec == FFMM_FP32)
        build_tables_t<float>(p, s);
    else
        build_tables_t<double>(p, s);
}

}  // namespace ffmm
