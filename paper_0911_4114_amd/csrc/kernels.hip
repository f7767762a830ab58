// Matvec-time kernels of the Fourier-basis FMM (Section 2 steps with the Section 3 quadrature):
//   gather (+conj)  ->  P2M  ->  M2M (five-step resample, translate, sum)  ->  M2L  ->
//   L2L (translate, five-step resample, add)  ->  L2P (+ gradient)  ->  P2P (+ gradient)  ->
//   scatter (+conj).
// R = double (FP64 path) or float (FP32 path). In the FP32 path the near-field distance and the
// phase kappa R are computed in FP64 and reduced modulo 2 pi before the FP32 sine/cosine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace ffmm {

namespace {

constexpr int kWave = 64;
constexpr double kTwoPi = 6.283185307179586476925287;

template <class R> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };

template <class C> __device__ inline C cz() { C c; c.x = 0; c.y = 0; return c; }

template <class C, class R> __device__ inline C cmk(R x, R y) { C c; c.x = x; c.y = y; return c; }

// acc += a * b
template <class C> __device__ inline void cmac(C& acc, C a, C b)
{
    acc.x += a.x * b.x - a.y * b.y;
    acc.y += a.x * b.y + a.y * b.x;
}

template <class C> __device__ inline C cmul(C a, C b)
{
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

template <class C> __device__ inline C cmulconj(C a, C b)  // a * conj(b)
{
    C r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.y * b.x - a.x * b.y;
    return r;
}

// e^{i phase}. FP32: phase given in revolutions (hardware sine/cosine take revolutions);
// FP64: phase in radians.
__device__ inline void cis(float rev, float& c, float& s)
{
    s = __builtin_amdgcn_sinf(rev);
    c = __builtin_amdgcn_cosf(rev);
}
__device__ inline void cis(double rad, double& c, double& s) { sincos(rad, &s, &c); }

// Phase scale: FP32 phases are carried in revolutions, FP64 phases in radians.
template <class R> inline R phase_scale(double kappa)
{
    return sizeof(R) == 4 ? (R)(kappa / kTwoPi) : (R)kappa;
}

// Knuth's TwoSum: s + e == a + b exactly.
template <class R> __device__ inline void two_sum(R a, R b, R& s, R& e)
{
    s = a + b;
    R bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

template <class R> __device__ inline R shfl_down(R v, int d) { return __shfl_down(v, d, kWave); }

// ------------------------------------------------------------------------------------------
// permutation with optional conjugation
// ------------------------------------------------------------------------------------------
template <class C>
__global__ void gather_q(const C* __restrict__ q, const int64_t* __restrict__ perm, int64_t n,
                         int conj, C* __restrict__ qs)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = blockIdx.y;
    C v = q[r * n + perm[i]];
    if (conj) v.y = -v.y;
    qs[r * n + i] = v;
}

template <class C>
__global__ void scatter_out(const C* __restrict__ phis, const int64_t* __restrict__ perm, int64_t n,
                            int width, int conj, C* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = blockIdx.y;
    for (int a = 0; a < width; ++a) {
        C v = phis[(r * n + i) * width + a];
        if (conj) v.y = -v.y;
        out[(r * n + perm[i]) * width + a] = v;
    }
}

// ------------------------------------------------------------------------------------------
// P2M (Initialization, Section 2): M_b(s_k) = sum_{i in b} q_i e^{i kappa s_k . (x_i - c_b)}.
// Block: one leaf box and 256 quadrature directions; the box's points are staged in LDS.
// ------------------------------------------------------------------------------------------
template <class R, class C>
__global__ __launch_bounds__(256) void p2m_kernel(int K, int kchunks, const R* __restrict__ dirs,
                                                  R kfac, const int32_t* __restrict__ start,
                                                  const int32_t* __restrict__ count,
                                                  const R* __restrict__ rel, const C* __restrict__ q,
                                                  C* __restrict__ M, int64_t n, int64_t nb)
{
    __shared__ R sx[256], sy[256], sz[256];
    __shared__ C sq[256];
    const int64_t b = blockIdx.x / kchunks;
    const int k = (blockIdx.x % kchunks) * 256 + threadIdx.x;
    const int64_t r = blockIdx.y;
    R dx = 0, dy = 0, dz = 0;
    if (k < K) {
        dx = dirs[3 * k] * kfac;
        dy = dirs[3 * k + 1] * kfac;
        dz = dirs[3 * k + 2] * kfac;
    }
    const int s0 = start[b], cnt = count[b];
    C acc = cz<C>();
    for (int p0 = 0; p0 < cnt; p0 += 256) {
        const int np = min(256, cnt - p0);
        __syncthreads();
        if ((int)threadIdx.x < np) {
            const int64_t i = s0 + p0 + threadIdx.x;
            sx[threadIdx.x] = rel[3 * i];
            sy[threadIdx.x] = rel[3 * i + 1];
            sz[threadIdx.x] = rel[3 * i + 2];
            sq[threadIdx.x] = q[r * n + i];
        }
        __syncthreads();
        for (int t = 0; t < np; ++t) {
            R ph = dx * sx[t] + dy * sy[t] + dz * sz[t];
            R c, s;
            cis(ph, c, s);
            cmac(acc, cmk<C>(c, s), sq[t]);
        }
    }
    if (k < K) M[(r * nb + b) * K + k] = acc;
}

// ------------------------------------------------------------------------------------------
// Five-step inter/anterpolation between level quadratures (Section 3.4), each 1D step a real
// Fourier-resample matrix (the Dirichlet kernel with the Nyquist bin dropped).
// step 1: G1[c][n][j] = sum_m D1_n[m][j] in_c(row n, m), j < NA.
//   UP:   in_c = M^l_c (child signature, level-l grid).
//   DOWN: in_c = L^l_{parent(c)} * conj(E_oct(c)) (translation applied on the parent grid).
// ------------------------------------------------------------------------------------------
template <class R, class C, bool DOWN>
__global__ __launch_bounds__(256) void rs_step1(int64_t nb, int rows, int NA,
                                                const int32_t* __restrict__ row_off,
                                                const int32_t* __restrict__ nphi,
                                                const R* __restrict__ d1, const C* __restrict__ sig,
                                                int Ksrc, int64_t nb_in,
                                                const int32_t* __restrict__ parent,
                                                const int32_t* __restrict__ octant,
                                                const C* __restrict__ trans, C* __restrict__ G1)
{
    const int64_t total = nb * rows * NA;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t r = blockIdx.y;
    const int j = (int)(idx % NA);
    const int nrow = (int)((idx / NA) % rows);
    const int64_t c = idx / ((int64_t)NA * rows);
    const int len = nphi[nrow], off = row_off[nrow];
    const R* D = d1 + (int64_t)off * NA + j;
    const int64_t cin = DOWN ? parent[c] : c;
    const C* in = sig + (r * nb_in + cin) * Ksrc + off;
    const C* tr = DOWN ? trans + (int64_t)octant[c] * Ksrc + off : nullptr;
    C acc = cz<C>();
    for (int m = 0; m < len; ++m) {
        C v = in[m];
        if (DOWN) v = cmulconj(v, tr[m]);
        const R d = D[(int64_t)m * NA];
        acc.x += d * v.x;
        acc.y += d * v.y;
    }
    G1[((r * nb + c) * rows + nrow) * NA + j] = acc;
}

// step 2 + 3: theta-periodic sequence of column m (< NA/2) built with the symmetry
// F(theta_t, phi_m) = F(theta_{ntS - t}, phi_{m + NA/2}) (eqn. NumSphereSym) and resampled from
// ntS to ntD points. G2[c][m][t'].
template <class R, class C>
__global__ __launch_bounds__(256) void rs_step3(int64_t nb, int NA, int rowsS, int ntS, int ntD,
                                                const R* __restrict__ dth,
                                                const C* __restrict__ G1, C* __restrict__ G2)
{
    const int half = NA / 2;
    const int64_t total = nb * half * ntD;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t r = blockIdx.y;
    const int tp = (int)(idx % ntD);
    const int m = (int)((idx / ntD) % half);
    const int64_t c = idx / ((int64_t)ntD * half);
    const C* g = G1 + (r * nb + c) * rowsS * NA;
    C acc = cz<C>();
    for (int t = 0; t < ntS; ++t) {
        C v = (t <= ntS / 2) ? g[t * NA + m] : g[(ntS - t) * NA + m + half];
        const R d = dth[(int64_t)t * ntD + tp];
        acc.x += d * v.x;
        acc.y += d * v.y;
    }
    G2[((r * nb + c) * half + m) * ntD + tp] = acc;
}

// steps 4 + 5 for one box: destination row n' rebuilt over NA columns by the same symmetry, then
// resampled to N'_phi(theta'_n'); returns the value at destination sample k.
template <class R, class C>
__device__ inline C rs_row_value(const C* __restrict__ g2, int NA, int ntD, int nrow, int jp,
                                 int len, const R* __restrict__ d5blk)
{
    const int half = NA / 2;
    const int tneg = (ntD - nrow) % ntD;
    C acc = cz<C>();
    for (int j = 0; j < NA; ++j) {
        C v = (j < half) ? g2[(int64_t)j * ntD + nrow] : g2[(int64_t)(j - half) * ntD + tneg];
        const R d = d5blk[(int64_t)j * len + jp];
        acc.x += d * v.x;
        acc.y += d * v.y;
    }
    return acc;
}

// UP (M2M, Section 2): M^{l-1}_p(s_k) = sum_{c child of p} E_oct(c)(s_k) R(M^l_c)(s_k).
template <class R, class C>
__global__ __launch_bounds__(256) void rs_step5_up(int64_t np, int Kd, int NA, int ntD,
                                                   const int32_t* __restrict__ row_of_k,
                                                   const int32_t* __restrict__ row_off,
                                                   const int32_t* __restrict__ nphi,
                                                   const R* __restrict__ d5, const C* __restrict__ G2,
                                                   int64_t nb_child,
                                                   const int32_t* __restrict__ child_start,
                                                   const int32_t* __restrict__ child_count,
                                                   const int32_t* __restrict__ octant,
                                                   const C* __restrict__ trans, C* __restrict__ out)
{
    const int64_t total = np * Kd;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t r = blockIdx.y;
    const int k = (int)(idx % Kd);
    const int64_t p = idx / Kd;
    const int nrow = row_of_k[k];
    const int off = row_off[nrow], len = nphi[nrow];
    const R* blk = d5 + (int64_t)off * NA;
    const int half = NA / 2;
    C acc = cz<C>();
    const int c0 = child_start[p], cn = child_count[p];
    for (int c = c0; c < c0 + cn; ++c) {
        const C* g2 = G2 + (r * nb_child + c) * half * ntD;
        C v = rs_row_value<R, C>(g2, NA, ntD, nrow, k - off, len, blk);
        cmac(acc, v, trans[(int64_t)octant[c] * Kd + k]);
    }
    out[(r * np + p) * Kd + k] = acc;
}

// DOWN (L2L, Section 2): L^{l+1}_c += R(L^l_p conj(E_oct(c))) (L^{l+1}_c already holds I^{l+1}_c).
template <class R, class C>
__global__ __launch_bounds__(256) void rs_step5_down(int64_t nc, int Kd, int NA, int ntD,
                                                     const int32_t* __restrict__ row_of_k,
                                                     const int32_t* __restrict__ row_off,
                                                     const int32_t* __restrict__ nphi,
                                                     const R* __restrict__ d5,
                                                     const C* __restrict__ G2, C* __restrict__ out)
{
    const int64_t total = nc * Kd;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int64_t r = blockIdx.y;
    const int k = (int)(idx % Kd);
    const int64_t c = idx / Kd;
    const int nrow = row_of_k[k];
    const int off = row_off[nrow], len = nphi[nrow];
    const C* g2 = G2 + (r * nc + c) * (NA / 2) * ntD;
    C v = rs_row_value<R, C>(g2, NA, ntD, nrow, k - off, len, d5 + (int64_t)off * NA);
    C& o = out[(r * nc + c) * Kd + k];
    o.x += v.x;
    o.y += v.y;
}

// ------------------------------------------------------------------------------------------
// M2L (Transfer pass, Section 2): I_b(s_k) = sum_{e in I(b)} M_src(e)(s_k) T_off(e)(s_k).
// Block: one target box, 256 directions; the interaction list is staged in LDS.
// ------------------------------------------------------------------------------------------
template <class C>
__global__ __launch_bounds__(256) void m2l_kernel(int K, int kchunks,
                                                  const int32_t* __restrict__ il_ptr,
                                                  const int32_t* __restrict__ il_src,
                                                  const int32_t* __restrict__ il_tix,
                                                  const C* __restrict__ T, const C* __restrict__ M,
                                                  C* __restrict__ out, int64_t nb)
{
    __shared__ int32_t s_src[192], s_tix[192];
    const int64_t b = blockIdx.x / kchunks;
    const int k = (blockIdx.x % kchunks) * 256 + threadIdx.x;
    const int64_t r = blockIdx.y;
    const int e0 = il_ptr[b], ne = il_ptr[b + 1] - e0;
    for (int t = threadIdx.x; t < ne; t += 256) {
        s_src[t] = il_src[e0 + t];
        s_tix[t] = il_tix[e0 + t];
    }
    __syncthreads();
    if (k >= K) return;
    const C* Mr = M + r * nb * K + k;
    const C* Tk = T + k;
    C acc = cz<C>();
    for (int e = 0; e < ne; ++e) cmac(acc, Mr[(int64_t)s_src[e] * K], Tk[(int64_t)s_tix[e] * K]);
    out[(r * nb + b) * K + k] = acc;
}

// ------------------------------------------------------------------------------------------
// L2P (far part of eqn. FMM_FinalStep): phi_i += sum_k w_k L_b(s_k) e^{i kappa s_k.(c_b - x_i)};
// with GRAD the gradient with respect to x_i, sum_k w_k L_b(s_k) (-i kappa s_k) e^{...}.
// One wave per target point, lanes split k; the partial sums are carried with TwoSum so that the
// FP32 sum of large cancelling terms keeps its accumulation error at the size of the result.
// ------------------------------------------------------------------------------------------
template <class R, class C, bool GRAD>
__global__ __launch_bounds__(256) void l2p_kernel(int K, const R* __restrict__ dirs,
                                                  const R* __restrict__ w, R kfac, R kappa,
                                                  const int32_t* __restrict__ start,
                                                  const int32_t* __restrict__ count,
                                                  const R* __restrict__ rel, const C* __restrict__ L,
                                                  C* __restrict__ out, int64_t n, int64_t nb)
{
    constexpr int NC = GRAD ? 3 : 1;
    const int64_t b = blockIdx.x;
    const int64_t r = blockIdx.y;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int s0 = start[b], cnt = count[b];
    const C* Lb = L + (r * nb + b) * K;
    for (int pt = wave; pt < cnt; pt += 4) {
        const int64_t i = s0 + pt;
        const R x = -rel[3 * i], y = -rel[3 * i + 1], z = -rel[3 * i + 2];  // c_b - x_i
        R sre[NC], sim[NC], ere[NC], eim[NC];
        for (int a = 0; a < NC; ++a) sre[a] = sim[a] = ere[a] = eim[a] = 0;
        for (int k = lane; k < K; k += kWave) {
            const R sx = dirs[3 * k], sy = dirs[3 * k + 1], sz = dirs[3 * k + 2];
            R c, s;
            cis(kfac * (sx * x + sy * y + sz * z), c, s);
            C lv = Lb[k];
            const R wk = w[k];
            C t = cmul(cmk<C>(c, s), cmk<C>(wk * lv.x, wk * lv.y));
            if (GRAD) {
                // (-i kappa s_a) t
                const R sa[3] = {sx, sy, sz};
                for (int a = 0; a < 3; ++a) {
                    R tr = kappa * sa[a] * t.y, ti = -kappa * sa[a] * t.x;
                    R e1, e2;
                    two_sum(sre[a], tr, sre[a], e1);
                    two_sum(sim[a], ti, sim[a], e2);
                    ere[a] += e1;
                    eim[a] += e2;
                }
            } else {
                R e1, e2;
                two_sum(sre[0], t.x, sre[0], e1);
                two_sum(sim[0], t.y, sim[0], e2);
                ere[0] += e1;
                eim[0] += e2;
            }
        }
        for (int a = 0; a < NC; ++a) {
            for (int d = kWave / 2; d > 0; d >>= 1) {
                R os = shfl_down(sre[a], d), oe = shfl_down(ere[a], d);
                R s1, e1;
                two_sum(sre[a], os, s1, e1);
                sre[a] = s1;
                ere[a] += oe + e1;
                os = shfl_down(sim[a], d);
                oe = shfl_down(eim[a], d);
                two_sum(sim[a], os, s1, e1);
                sim[a] = s1;
                eim[a] += oe + e1;
            }
        }
        if (lane == 0)
            for (int a = 0; a < NC; ++a) {
                C& o = out[(r * n + i) * NC + a];
                o.x += sre[a] + ere[a];
                o.y += sim[a] + eim[a];
            }
    }
}

// ------------------------------------------------------------------------------------------
// P2P (near part of eqn. FMM_FinalStep): phi_i += sum_{j in N(b), j != i, R > 0} e^{i kappa R}/R q_j;
// with GRAD: sum G'(R) (x_i - x_j)/R q_j, G'(R) = e^{i kappa R}(i kappa R - 1)/R^2.
// One wave per leaf box, lanes = targets, source points staged in LDS 64 at a time.
// R and kappa R in FP64; in the FP32 path kappa R is reduced modulo 2 pi in FP64 and the
// sine/cosine, 1/R and the sums are FP32.
// ------------------------------------------------------------------------------------------
template <class R, class C, bool GRAD>
__global__ __launch_bounds__(kWave) void p2p_kernel(const double* __restrict__ xs,
                                                    const C* __restrict__ q,
                                                    const int32_t* __restrict__ start,
                                                    const int32_t* __restrict__ count,
                                                    const int32_t* __restrict__ nb_ptr,
                                                    const int32_t* __restrict__ nb_src, double kappa,
                                                    C* __restrict__ out, int64_t n)
{
    constexpr int NC = GRAD ? 3 : 1;
    __shared__ double sx[kWave], sy[kWave], sz[kWave];
    __shared__ C sq[kWave];
    const int64_t b = blockIdx.x;
    const int64_t r = blockIdx.y;
    const int lane = threadIdx.x;
    const int tb = start[b], tc = count[b];
    const double inv2pi = 1.0 / kTwoPi;
    for (int t0 = 0; t0 < tc; t0 += kWave) {
        const bool valid = t0 + lane < tc;
        const int64_t i = tb + t0 + lane;
        double xi = 0, yi = 0, zi = 0;
        if (valid) {
            xi = xs[3 * i];
            yi = xs[3 * i + 1];
            zi = xs[3 * i + 2];
        }
        C acc[NC];
        for (int a = 0; a < NC; ++a) acc[a] = cz<C>();
        for (int e = nb_ptr[b]; e < nb_ptr[b + 1]; ++e) {
            const int c = nb_src[e];
            const int sb = start[c], sc = count[c];
            for (int s0 = 0; s0 < sc; s0 += kWave) {
                const int ns = min(kWave, sc - s0);
                __syncthreads();
                if (lane < ns) {
                    const int64_t j = sb + s0 + lane;
                    sx[lane] = xs[3 * j];
                    sy[lane] = xs[3 * j + 1];
                    sz[lane] = xs[3 * j + 2];
                    sq[lane] = q[r * n + j];
                }
                __syncthreads();
                if (!valid) continue;
                for (int t = 0; t < ns; ++t) {
                    const int64_t j = sb + s0 + t;
                    const double dx = xi - sx[t], dy = yi - sy[t], dz = zi - sz[t];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (j == i || r2 == 0.0) continue;
                    const double rr = sqrt(r2);
                    R c, s, inv;
                    if constexpr (sizeof(R) == 4) {
                        double rev = kappa * rr * inv2pi;
                        rev -= floor(rev);
                        cis((float)rev, c, s);
                        inv = 1.0f / (float)rr;
                    } else {
                        cis(kappa * rr, c, s);
                        inv = 1.0 / rr;
                    }
                    if (GRAD) {
                        // e^{i kR}(i kR - 1)/R^3 (x_i - x_j)
                        const R kr = (R)(kappa * rr);
                        const R inv3 = inv * inv * inv;
                        const R gr = (-c - s * kr) * inv3, gi = (c * kr - s) * inv3;
                        C g = cmul(cmk<C>(gr, gi), sq[t]);
                        const R d[3] = {(R)dx, (R)dy, (R)dz};
                        for (int a = 0; a < 3; ++a) {
                            acc[a].x += d[a] * g.x;
                            acc[a].y += d[a] * g.y;
                        }
                    } else {
                        cmac(acc[0], cmk<C>(c * inv, s * inv), sq[t]);
                    }
                }
            }
        }
        if (valid)
            for (int a = 0; a < NC; ++a) {
                C& o = out[(r * n + i) * NC + a];
                o.x += acc[a].x;
                o.y += acc[a].y;
            }
    }
}

// coordinates relative to the leaf centre, in the plan precision
template <class R>
__global__ void rel_coords(const double* __restrict__ xs, const int32_t* __restrict__ point_box,
                           const double* __restrict__ centers, int64_t n, R* __restrict__ rel)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = point_box[i];
    for (int a = 0; a < 3; ++a) rel[3 * i + a] = (R)(xs[3 * i + a] - centers[3 * b + a]);
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <class R>
void run_matvec_t(ffmm_plan* p, const void* qv, void* outv, int nrhs, int stages, bool conj_io,
                  bool gradient, hipStream_t s)
{
    using C = typename cplx_t<R>::type;
    const int64_t n = p->n;
    const int L = p->depth;
    const int width = gradient ? 3 : 1;
    C* qs = (C*)p->qs;
    C* phis = (C*)p->phis;
    const R kfac = phase_scale<R>(p->kappa);

    {
        StageScope sc(p, FFMM_PROF_GATHER, s);
        hipLaunchKernelGGL(gather_q<C>, dim3(nblk(n, 256), nrhs), dim3(256), 0, s, (const C*)qv,
                           p->perm, n, conj_io ? 1 : 0, qs);
        FFMM_LAUNCH_CHECK();
        FFMM_HIP(hipMemsetAsync(phis, 0, sizeof(C) * (size_t)nrhs * n * width, s));
    }

    if (stages & FFMM_STAGE_FAR) {
        LevelData& leaf = p->lev[L];
        // P2M
        {
            StageScope sc(p, FFMM_PROF_P2M, s);
            const int kch = (leaf.K + 255) / 256;
            hipLaunchKernelGGL((p2m_kernel<R, C>), dim3((unsigned)(leaf.n * kch), nrhs), dim3(256), 0, s,
                               leaf.K, kch, (const R*)leaf.dirs, kfac, p->leaf_start, p->leaf_count,
                               (const R*)p->rel, qs, (C*)leaf.sigM, n, leaf.n);
            FFMM_LAUNCH_CHECK();
        }
        // M2M, l = L..3
        for (int l = L; l >= 3; --l) {
            StageScope sc(p, FFMM_PROF_M2M, s);
            LevelData& Cl = p->lev[l];
            LevelData& P = p->lev[l - 1];
            Resampler& rs = p->up[l];
            C* G1 = (C*)p->scratch1;
            C* G2 = (C*)p->scratch2;
            int64_t tot = Cl.n * rs.rows_src * rs.nphi_all;
            hipLaunchKernelGGL((rs_step1<R, C, false>), dim3(nblk(tot, 256), nrhs), dim3(256), 0, s,
                               Cl.n, rs.rows_src, rs.nphi_all, rs.d_src_row_off, rs.d_src_nphi,
                               (const R*)rs.d1, (const C*)Cl.sigM, Cl.K, Cl.n, (const int32_t*)nullptr,
                               (const int32_t*)nullptr, (const C*)nullptr, G1);
            FFMM_LAUNCH_CHECK();
            tot = Cl.n * (rs.nphi_all / 2) * rs.nt_dst;
            hipLaunchKernelGGL((rs_step3<R, C>), dim3(nblk(tot, 256), nrhs), dim3(256), 0, s, Cl.n,
                               rs.nphi_all, rs.rows_src, rs.nt_src, rs.nt_dst, (const R*)rs.dth,
                               (const C*)G1, G2);
            FFMM_LAUNCH_CHECK();
            tot = P.n * P.K;
            hipLaunchKernelGGL((rs_step5_up<R, C>), dim3(nblk(tot, 256), nrhs), dim3(256), 0, s, P.n,
                               P.K, rs.nphi_all, rs.nt_dst, rs.d_dst_row_of_k, rs.d_dst_row_off,
                               rs.d_dst_nphi, (const R*)rs.d5, (const C*)G2, Cl.n, P.child_start,
                               P.child_count, Cl.octant, (const C*)P.trans, (C*)P.sigM);
            FFMM_LAUNCH_CHECK();
        }
        // M2L, l = 2..L (written into the L buffers, which then receive the downward pass)
        for (int l = 2; l <= L; ++l) {
            StageScope sc(p, l == L ? FFMM_PROF_LEAF_M2L : FFMM_PROF_M2L, s);
            LevelData& Lv = p->lev[l];
            const int kch = (Lv.K + 255) / 256;
            hipLaunchKernelGGL((m2l_kernel<C>), dim3((unsigned)(Lv.n * kch), nrhs), dim3(256), 0, s, Lv.K,
                               kch, Lv.il_ptr, Lv.il_src, Lv.il_tix, (const C*)Lv.transfer,
                               (const C*)Lv.sigM, (C*)Lv.sigL, Lv.n);
            FFMM_LAUNCH_CHECK();
        }
        // L2L, l = 2..L-1
        for (int l = 2; l < L; ++l) {
            StageScope sc(p, FFMM_PROF_L2L, s);
            LevelData& P = p->lev[l];
            LevelData& Cl = p->lev[l + 1];
            Resampler& rs = p->down[l];
            C* G1 = (C*)p->scratch1;
            C* G2 = (C*)p->scratch2;
            int64_t tot = Cl.n * rs.rows_src * rs.nphi_all;
            hipLaunchKernelGGL((rs_step1<R, C, true>), dim3(nblk(tot, 256), nrhs), dim3(256), 0, s,
                               Cl.n, rs.rows_src, rs.nphi_all, rs.d_src_row_off, rs.d_src_nphi,
                               (const R*)rs.d1, (const C*)P.sigL, P.K, P.n, Cl.parent, Cl.octant,
                               (const C*)P.trans, G1);
            FFMM_LAUNCH_CHECK();
            tot = Cl.n * (rs.nphi_all / 2) * rs.nt_dst;
            hipLaunchKernelGGL((rs_step3<R, C>), dim3(nblk(tot, 256), nrhs), dim3(256), 0, s, Cl.n,
                               rs.nphi_all, rs.rows_src, rs.nt_src, rs.nt_dst, (const R*)rs.dth,
                               (const C*)G1, G2);
            FFMM_LAUNCH_CHECK();
            tot = Cl.n * Cl.K;
            hipLaunchKernelGGL((rs_step5_down<R, C>), dim3(nblk(tot, 256), nrhs), dim3(256), 0, s, Cl.n,
                               Cl.K, rs.nphi_all, rs.nt_dst, rs.d_dst_row_of_k, rs.d_dst_row_off,
                               rs.d_dst_nphi, (const R*)rs.d5, (const C*)G2, (C*)Cl.sigL);
            FFMM_LAUNCH_CHECK();
        }
        // L2P
        StageScope sc(p, FFMM_PROF_L2P, s);
        if (gradient)
            hipLaunchKernelGGL((l2p_kernel<R, C, true>), dim3((unsigned)leaf.n, nrhs), dim3(256), 0, s,
                               leaf.K, (const R*)leaf.dirs, (const R*)leaf.weights, kfac, (R)p->kappa,
                               p->leaf_start, p->leaf_count, (const R*)p->rel, (const C*)leaf.sigL,
                               phis, n, leaf.n);
        else
            hipLaunchKernelGGL((l2p_kernel<R, C, false>), dim3((unsigned)leaf.n, nrhs), dim3(256), 0, s,
                               leaf.K, (const R*)leaf.dirs, (const R*)leaf.weights, kfac, (R)p->kappa,
                               p->leaf_start, p->leaf_count, (const R*)p->rel, (const C*)leaf.sigL,
                               phis, n, leaf.n);
        FFMM_LAUNCH_CHECK();
    }
    if (stages & FFMM_STAGE_NEAR) {
        StageScope sc(p, FFMM_PROF_P2P, s);
        const int64_t nl = p->lev[L].n;
        if (gradient)
            hipLaunchKernelGGL((p2p_kernel<R, C, true>), dim3((unsigned)nl, nrhs), dim3(kWave), 0, s,
                               p->xs, qs, p->leaf_start, p->leaf_count, p->nb_ptr, p->nb_src, p->kappa,
                               phis, n);
        else
            hipLaunchKernelGGL((p2p_kernel<R, C, false>), dim3((unsigned)nl, nrhs), dim3(kWave), 0, s,
                               p->xs, qs, p->leaf_start, p->leaf_count, p->nb_ptr, p->nb_src, p->kappa,
                               phis, n);
        FFMM_LAUNCH_CHECK();
    }
    {
        StageScope sc(p, FFMM_PROF_SCATTER, s);
        hipLaunchKernelGGL(scatter_out<C>, dim3(nblk(n, 256), nrhs), dim3(256), 0, s, (const C*)phis,
                           p->perm, n, width, conj_io ? 1 : 0, (C*)outv);
        FFMM_LAUNCH_CHECK();
    }
}

template <class R>
void prepare_rel_t(ffmm_plan* p, hipStream_t s)
{
    p->rel = p->arena.alloc(sizeof(R) * 3 * p->n);
    hipLaunchKernelGGL(rel_coords<R>, dim3(nblk(p->n, 256)), dim3(256), 0, s, p->xs, p->point_box,
                       p->lev[p->depth].centers, p->n, (R*)p->rel);
    FFMM_LAUNCH_CHECK();
}

}  // namespace

void prepare_rel(ffmm_plan* p, hipStream_t s)
{
    if (p->prec == FFMM_FP32)
        prepare_rel_t<float>(p, s);
    else
        prepare_rel_t<double>(p, s);
}

void run_matvec(ffmm_plan* p, const void* q, void* out, int nrhs, int stages, bool conj_io,
                bool gradient, hipStream_t s)
{
    if (p->prec == FFMM_FP32)
        run_matvec_t<float>(p, q, out, nrhs, stages, conj_io, gradient, s);
    else
        run_matvec_t<double>(p, q, out, nrhs, stages, conj_io, gradient, s);
}

}  // namespace ffmm
