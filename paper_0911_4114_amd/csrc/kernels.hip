// Matvec-time kernels of the Fourier-basis FMM (Section 2 steps with the Section 3 quadrature):
//   gather (+conj)  ->  P2M  ->  M2M (five-step resample, translate, sum)  ->  M2L  ->
//   L2L (translate, five-step resample, add)  ->  L2P (+ gradient)  ->  P2P (+ gradient)  ->
//   scatter (+conj).
// R = double (FP64 path) or float (FP32 path). In the FP32 path the near-field distance and the
// phase kappa R are computed in FP64 and reduced modulo 2 pi before the FP32 sine/cosine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

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

// acc += a b with explicit fused operations, so that the rounding does not depend on how the
// compiler schedules the surrounding loop (batched and single right-hand sides agree bit for bit)
template <class C> __device__ inline void cmac(C& acc, C a, C b)
{
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

template <class C> __device__ inline C cmulconj(C a, C b)  // a * conj(b)
{
    C r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.y * b.x - a.x * b.y;
    return r;
}

// e^{i phase}, the phase given in revolutions. FP32: the hardware sine/cosine take revolutions.
__device__ inline void cis(float rev, float& c, float& s)
{
    s = __builtin_amdgcn_sinf(rev);
    c = __builtin_amdgcn_cosf(rev);
}
// FP64: (cos, sin)(2 pi k / 256), k < 256, each correctly rounded (filled by init_cis_table for
// the device a plan is created on)
__device__ double2 g_cis256[256];

// FP64 e^{2 pi i rev}: the fraction of a revolution (exact), split as k / 256 + r with k the nearest
// integer to 256 fract(rev) and |r| <= 1/512 (both exact); (cos, sin) of 2 pi k / 256 from the
// table, of x = 2 pi r (|x| <= pi/256) from their Taylor series to x^6 (the first omitted terms are
// below 2e-20), joined by the angle-sum formulas with cos x - 1 kept apart, so that no digit of
// the table values is lost.
__device__ inline void cis(double rev, double& c, double& s)
{
    const double t = __builtin_amdgcn_fract(rev) * 256.0;
    const double k = __builtin_rint(t);
    const double x = (t - k) * (kTwoPi / 256.0);
    const double2 e = g_cis256[(int)k & 255];
    const double x2 = x * x;
    const double sx = x * fma(x2, fma(x2, fma(x2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), 1.0);
    const double cm1 = x2 * fma(x2, fma(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5);
    c = fma(-e.y, sx, fma(e.x, cm1, e.x));
    s = fma(e.x, sx, fma(e.y, cm1, e.y));
}

// Phase scale: phases are carried in revolutions, kappa / 2 pi per unit of length.
template <class R> inline R phase_scale(double kappa) { return (R)(kappa / kTwoPi); }

// Knuth's TwoSum: s + e == a + b exactly.
template <class R> __device__ inline void two_sum(R a, R b, R& s, R& e)
{
    s = a + b;
    R bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

template <class R> __device__ inline R shfl_down(R v, int d) { return __shfl_down(v, d, kWave); }

// Kernels that give each wave its own box run kWpb waves per block: blocks of one wave are few
// per CU and leave the SIMDs short of waves to hide latency with. The waves of a block then work
// on different boxes and hand LDS data between their own lanes only: a wave executes its LDS
// operations in order, so a fence at wavefront scope (which also stops the compiler moving memory
// operations across it) is the whole synchronisation.
constexpr int kWpb = 4;

// Largest near-field phase range, in revolutions, for which P2P takes its FP32 phase form.
constexpr double kFastRev = 8.0;
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

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
__global__ void scatter_out(const C* __restrict__ far, const C* __restrict__ near,
                            const int64_t* __restrict__ perm, int64_t n, int width, int conj,
                            C* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = blockIdx.y;
    for (int a = 0; a < width; ++a) {
        const int64_t k = (r * n + i) * width + a;
        C v = cz<C>();
        if (far) v = far[k];
        if (near) {
            v.x += near[k].x;
            v.y += near[k].y;
        }
        if (conj) v.y = -v.y;
        out[(r * n + perm[i]) * width + a] = v;
    }
}

// Position gradient (ffmm_position_gradient): per point, in caller order,
//   gx_i (+)= sum_{rr < cnt} Re[conj(G_rr,i) F_i(q_rr) + q_rr,i F_i(conj G_rr)]
// F_i(q_rr) at field-gradient rows fq_row + rr of the far and near results (Morton order, [..][n][3]),
// F_i(conj G_rr) at rows fg_row + rr; a row base of -1 leaves that term out. Sums in FP64.
template <class C>
__global__ void posgrad_combine(const C* __restrict__ far, const C* __restrict__ near,
                                const int64_t* __restrict__ perm, int64_t n, int cnt, int fq_row,
                                int fg_row, const C* __restrict__ q, const C* __restrict__ g,
                                int accumulate, double* __restrict__ gx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    double acc[3] = {0.0, 0.0, 0.0};
    if (accumulate)
        for (int a = 0; a < 3; ++a) acc[a] = gx[3 * u + a];
    auto field = [&](int row, int a) {
        const int64_t k = ((int64_t)row * n + i) * 3 + a;
        double fx = 0.0, fy = 0.0;
        if (far) {
            fx += (double)far[k].x;
            fy += (double)far[k].y;
        }
        fx += (double)near[k].x;
        fy += (double)near[k].y;
        return make_double2(fx, fy);
    };
    for (int rr = 0; rr < cnt; ++rr) {
        const C qv = q[(int64_t)rr * n + u], gv = g[(int64_t)rr * n + u];
        for (int a = 0; a < 3; ++a) {
            if (fq_row >= 0) {   // Re[conj(G) F(q)]
                const double2 f = field(fq_row + rr, a);
                acc[a] += (double)gv.x * f.x + (double)gv.y * f.y;
            }
            if (fg_row >= 0) {   // Re[q F(conj G)]
                const double2 f = field(fg_row + rr, a);
                acc[a] += (double)qv.x * f.x - (double)qv.y * f.y;
            }
        }
    }
    for (int a = 0; a < 3; ++a) gx[3 * u + a] = acc[a];
}

// ------------------------------------------------------------------------------------------
// P2M (Initialization, Section 2): M_b(s_k) = sum_{i in b} q_i e^{i kappa s_k . (x_i - c_b)}.
// The quadrature holds every direction with its antipode, so one phase and one sine/cosine per
// point serve both. Block: one leaf box and NTH antipodal pairs (64, 128 or 256: the width that
// leaves the fewest idle lanes at this K); the box's points staged in LDS NTH at a time.
// ------------------------------------------------------------------------------------------
template <class R, class C, int NTH>
__global__ __launch_bounds__(NTH) void p2m_kernel(int Kp, int kchunks, const R* __restrict__ dirs,
                                                  const int32_t* __restrict__ pairs, R kfac,
                                                  const int32_t* __restrict__ start,
                                                  const int32_t* __restrict__ count,
                                                  const R* __restrict__ rel, const C* __restrict__ q,
                                                  C* __restrict__ M, int64_t n, int64_t nb, int K)
{
    __shared__ R sx[NTH], sy[NTH], sz[NTH];
    __shared__ C sq[NTH];
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t b = lb / kchunks;
    const int pi = (lb % kchunks) * NTH + threadIdx.x;
    const bool pvalid = pi < Kp;
    const int64_t r = blockIdx.y;
    int k1 = 0, k2 = 0;
    R dx = 0, dy = 0, dz = 0;
    if (pvalid) {
        k1 = pairs[2 * pi];
        k2 = pairs[2 * pi + 1];
        dx = dirs[3 * k1] * kfac;
        dy = dirs[3 * k1 + 1] * kfac;
        dz = dirs[3 * k1 + 2] * kfac;
    }
    const int s0 = start[b], cnt = count[b];
    // s_k2 = -s_k1: M(s_k1) = A + iB, M(s_k2) = A - iB with A = sum cos(ph) q, B = sum sin(ph) q
    C A = cz<C>(), B = cz<C>();
    for (int p0 = 0; p0 < cnt; p0 += NTH) {
        const int np = min(NTH, cnt - p0);
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
            const C qt = sq[t];
            A.x = fma(c, qt.x, A.x);
            A.y = fma(c, qt.y, A.y);
            B.x = fma(s, qt.x, B.x);
            B.y = fma(s, qt.y, B.y);
        }
    }
    if (pvalid) {
        C* Mb = M + (r * nb + b) * K;
        Mb[k1] = cmk<C>(A.x - B.y, A.y + B.x);
        Mb[k2] = cmk<C>(A.x + B.y, A.y - B.x);
    }
}

// ------------------------------------------------------------------------------------------
// M2L (Transfer pass, Section 2): I_b(s_k) = sum_{e in I(b)} M_src(e)(s_k) T_off(e)(s_k).
// Block: one target box, 256 directions; the interaction list is staged in LDS; each T value read
// serves RB right-hand sides. T is stored for the 34 representative transfer vectors only: the
// entry's vector is g(rep) for a symmetry g of the quadrature, and T_{g rep}(s_k) =
// T_rep(s_{tperm[g][k]}); each thread keeps its 16 permuted directions in registers.
// ------------------------------------------------------------------------------------------
template <class C, int RB>
__global__ __launch_bounds__(256) void m2l_kernel(int K, int kchunks,
                                                  const int32_t* __restrict__ il_ptr,
                                                  const int32_t* __restrict__ il_src,
                                                  const int32_t* __restrict__ il_tix,
                                                  const int32_t* __restrict__ tperm,
                                                  const C* __restrict__ T, const C* __restrict__ M,
                                                  C* __restrict__ out, int64_t nb, int nrhs)
{
    __shared__ int32_t s_src[192], s_tix[192];
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t b = lb / kchunks;
    const int k = (lb % kchunks) * 256 + threadIdx.x;
    const int r0 = blockIdx.y * RB;
    const int e0 = il_ptr[b], ne = il_ptr[b + 1] - e0;
    for (int t = threadIdx.x; t < ne; t += 256) {
        s_src[t] = il_src[e0 + t];
        s_tix[t] = il_tix[e0 + t];
    }
    __syncthreads();
    if (k >= K) return;
    const int64_t plane = nb * (int64_t)K;
    const C* Mk = M + (int64_t)r0 * plane + k;
    int kp[kNumSym];
#pragma unroll
    for (int g = 0; g < kNumSym; ++g) kp[g] = tperm[(int64_t)g * K + k];
    // T value of entry e (its packed index is uniform across the block)
    auto tval = [&](int e) {
        const int tx = __builtin_amdgcn_readfirstlane(s_tix[e]);
        return T[(uint64_t)(uint32_t)(tx >> 4) * (uint32_t)K + kp[tx & (kNumSym - 1)]];
    };
    const int nr = min(RB, nrhs - r0);
    C acc[RB];
    for (int q = 0; q < RB; ++q) acc[q] = cz<C>();
    // entries in batches of U: all loads of a batch are issued before the first product, so a
    // wave keeps U (T, M) pairs in flight instead of one
    constexpr int U = RB == 4 ? 4 : 8;
    int e = 0;
    for (; e + U <= ne; e += U) {
        C t[U], m[U][RB];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            t[u] = tval(e + u);
            const C* mp = Mk + (uint64_t)(uint32_t)s_src[e + u] * (uint32_t)K;
#pragma unroll
            for (int q = 0; q < RB; ++q) m[u][q] = (q < nr) ? mp[(int64_t)q * plane] : cz<C>();
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < RB; ++q) cmac(acc[q], m[u][q], t[u]);
    }
    for (; e < ne; ++e) {
        const C t = tval(e);
        const C* mp = Mk + (uint64_t)(uint32_t)s_src[e] * (uint32_t)K;
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (q < nr) cmac(acc[q], mp[(int64_t)q * plane], t);
    }
    for (int q = 0; q < RB; ++q)
        if (q < nr) out[(int64_t)(r0 + q) * plane + b * K + k] = acc[q];
}

// ------------------------------------------------------------------------------------------
// M2L by parent pairs: the same I_b(s_k) = sum_{e in I(b)} M_src(e)(s_k) T_off(e)(s_k), organised
// by the definition of I(b) (Section 2): the children b of a parent P receive from the children
// b' of every neighbour P' of P that are not neighbours of b. For P' at offset D from P and
// octants o(b), o(b'), the transfer vector is 2D + (o(b') - o(b)), one of 27 per D; so a block
// (P, NTH = 128 or 256 directions, whichever leaves fewer idle lanes at this K) loads the <= 8 source signatures of each P' once and each of the 27
// transfer functions once, and applies them to every child pair they serve (up to 64 pairs),
// instead of reading one M and one T per pair. T is read through the quadrature symmetry as in
// m2l_kernel.
// ------------------------------------------------------------------------------------------
// T value through a raw buffer resource: the table row's byte offset in a scalar register, the
// permuted direction's byte offset per lane; reads past the table's size return zero.
__device__ inline __amdgpu_buffer_rsrc_t table_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
template <class C> __device__ inline C buf_load(__amdgpu_buffer_rsrc_t rs, int voff, int soff);
template <> __device__ inline float2 buf_load<float2>(__amdgpu_buffer_rsrc_t rs, int voff, int soff)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0);
    float2 c;
    __builtin_memcpy(&c, &v, sizeof(c));
    return c;
}
template <> __device__ inline double2 buf_load<double2>(__amdgpu_buffer_rsrc_t rs, int voff, int soff)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
    double2 c;
    __builtin_memcpy(&c, &v, sizeof(c));
    return c;
}

template <class C, int RB, int NTH>
__global__ __launch_bounds__(NTH) void m2lp_kernel(int K, int kchunks,
                                                   const int32_t* __restrict__ pslots,
                                                   const int32_t* __restrict__ child_start,
                                                   const int32_t* __restrict__ child_count,
                                                   const int32_t* __restrict__ octant,
                                                   const int32_t* __restrict__ code_map,
                                                   const int32_t* __restrict__ tperm,
                                                   const C* __restrict__ T, const C* __restrict__ M,
                                                   C* __restrict__ out, int64_t nb, int nrhs)
{
    // per occupied neighbour P' of P (compacted): D, first child, octant mask of its children;
    // per (P', child-offset difference e): the representative's T row (-1 where no pair of
    // present children is far apart at that offset: all of them neighbours, or none present)
    // and the symmetry index, with the target octants of the present pairs in bits 8..15
    __shared__ int32_t s_d[27], s_sb[27], s_sm[27];
    __shared__ int2 s_tx[27][27];
    __shared__ int32_t s_n, s_tmask;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t P = lb / kchunks;
    const int kraw = (lb % kchunks) * NTH + threadIdx.x;
    const bool kvalid = kraw < K;
    const int k = kvalid ? kraw : K - 1;   // tail lanes compute on a valid direction, store nothing
    const int r0 = blockIdx.y * RB;
    const int tb = child_start[P], tn = child_count[P];
    if (threadIdx.x < kWave) {
        // wave 0: lane D reads neighbour slot D (compacted by a ballot); lanes < tn read the
        // octants of P's own children
        const int D = threadIdx.x;
        const int Pn = D < 27 ? pslots[P * 27 + D] : -1;
        int sb = 0, sm = 0;
        if (Pn >= 0) {
            sb = child_start[Pn];
            const int sn = child_count[Pn];
            for (int i = 0; i < sn; ++i) sm |= 1 << octant[sb + i];
        }
        const uint64_t occ = __ballot(Pn >= 0);
        if (Pn >= 0) {
            const int pos = __popcll(occ & ((1ull << D) - 1));
            s_d[pos] = D;
            s_sb[pos] = sb;
            s_sm[pos] = sm;
        }
        const int ot = D < tn ? octant[tb + D] : -1;
        int tm = 0;
#pragma unroll
        for (int o = 0; o < 8; ++o) tm |= (__ballot(ot == o) != 0 ? 1 : 0) << o;
        if (D == 0) {
            s_n = __popcll(occ);
            s_tmask = tm;
        }
    }
    __syncthreads();
    const int nn = s_n, tmask = s_tmask;
    for (int t = threadIdx.x; t < nn * 27; t += NTH) {
        const int i = t / 27, e = t % 27, D = s_d[i];
        const int ex = e % 3 - 1, ey = (e / 3) % 3 - 1, ez = e / 9 - 1;
        const int code = (2 * (D % 3 - 1) + ex + 3) + 7 * (2 * ((D / 3) % 3 - 1) + ey + 3) +
                         49 * (2 * (D / 9 - 1) + ez + 3);
        int tx = code_map[code];
        int pairs = 0;
        for (int ot = 0; ot < 8; ++ot) {
            const int ax = (ot & 1) + ex, ay = ((ot >> 1) & 1) + ey, az = ((ot >> 2) & 1) + ez;
            if (ax < 0 || ax > 1 || ay < 0 || ay > 1 || az < 0 || az > 1) continue;
            pairs |= ((tmask >> ot) & (s_sm[i] >> (ax + 2 * ay + 4 * az)) & 1) << ot;
        }
        const bool use = pairs && tx >= 0;
        s_tx[i][e] = make_int2(use ? (tx >> 4) : -1, (tx & (kNumSym - 1)) | (pairs << 8));
    }
    __syncthreads();
    const int64_t plane = nb * (int64_t)K;
    const int nr = min(RB, nrhs - r0);
    // byte offsets of the permuted directions inside one table row (K sizeof(C) < 2^31: the plan
    // rejects larger quadratures)
    int kp8[kNumSym];
#pragma unroll
    for (int g = 0; g < kNumSym; ++g) kp8[g] = tperm[(int64_t)g * K + k] * (int)sizeof(C);
    const uint32_t row_bytes = (uint32_t)K * (uint32_t)sizeof(C);
    C acc[8][RB];
#pragma unroll
    for (int o = 0; o < 8; ++o)
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[o][q] = cz<C>();
    for (int i = 0; i < nn; ++i) {
        const int sb = s_sb[i], smask = s_sm[i];
        // source signatures of the present octants (absent ones read the first child's address
        // and are never used)
        C ms[8][RB];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            const bool present = (smask >> o) & 1;
            const int ci = sb + (present ? __builtin_popcount(smask & ((1 << o) - 1)) : 0);
            const C* mp = M + (int64_t)r0 * plane + (uint64_t)(uint32_t)ci * (uint32_t)K + k;
#pragma unroll
            for (int q = 0; q < RB; ++q) ms[o][q] = mp[(int64_t)(q < nr ? q : 0) * plane];
        }
#pragma unroll
        for (int e = 0; e < 27; ++e) {
            const int2 v = s_tx[i][e];
            const int rep = __builtin_amdgcn_readfirstlane(v.x);
            if (rep < 0) continue;
            const int gp = __builtin_amdgcn_readfirstlane(v.y);
            const int pairs = gp >> 8;
            // a buffer resource per table row: its 64-bit base is scalar arithmetic, the row
            // offset never enters a 32-bit byte offset
            const __amdgpu_buffer_rsrc_t trs = table_rsrc(T + (int64_t)rep * K, row_bytes);
            const C tv = buf_load<C>(trs, kp8[gp & (kNumSym - 1)], 0);
            const int ex = e % 3 - 1, ey = (e / 3) % 3 - 1, ez = e / 9 - 1;
#pragma unroll
            for (int ot = 0; ot < 8; ++ot) {
                const int ax = (ot & 1) + ex, ay = ((ot >> 1) & 1) + ey, az = ((ot >> 2) & 1) + ez;
                if (ax < 0 || ax > 1 || ay < 0 || ay > 1 || az < 0 || az > 1) continue;
                if (!((pairs >> ot) & 1)) continue;
                // an absent pair costs a scalar test; the empty volatile asm keeps the compiler
                // from turning this branch into multiply-adds and selects
                __asm__ __volatile__("");
                const int os = ax + 2 * ay + 4 * az;
#pragma unroll
                for (int q = 0; q < RB; ++q) cmac(acc[ot][q], ms[os][q], tv);
            }
        }
    }
    if (!kvalid) return;
    for (int i = 0; i < tn; ++i) {
        const int c = tb + i;
        const int o = __builtin_amdgcn_readfirstlane(octant[c]);
#pragma unroll
        for (int oo = 0; oo < 8; ++oo)
            if (oo == o)
#pragma unroll
                for (int q = 0; q < RB; ++q)
                    if (q < nr) out[(int64_t)(r0 + q) * plane + (int64_t)c * K + k] = acc[oo][q];
    }
}

// ------------------------------------------------------------------------------------------
// M2L by parent pairs with the transfer functions of a chunk of directions in LDS (FP32): the sums
// of m2lp_kernel, I_b(s) = sum M_b'(s) T_{2D + o' - o}(s) over the far child pairs (o, o') of each
// parent pair (P, P' = P + D), with every T value read from LDS. A block takes CW antipodal
// direction pairs (s, -s) and a Morton range of parents. It first gathers into LDS the values at
// its CW directions s of all 316 transfer functions (from the 34 representatives through the
// quadrature symmetry; Fig. SemiOctant); the values at -s need no second table, since
// T_r0(-s) = T_{-r0}(s) and, in code order, the row of -r0 is 315 minus the row of r0. Then each
// wave takes parents of the range in turn, one lane per direction pair, and serves both
// directions of its pair from each scalar decision (target octant present, source octant
// present and far), so that the per-pair bookkeeping is shared by twice the multiply-adds. The
// table is read from memory once per block and reused by every parent and right-hand side.
// Per parent: lane D < 27 holds neighbour slot D (first child, octant mask of its children);
// per occupied neighbour, a [27][27] table gives the LDS row of 2D + e (-1 where the boxes are
// neighbours) and a [27][8] table the source octants far from each target octant.
// ------------------------------------------------------------------------------------------
constexpr int kTW = 16;   // waves per block of m2lt_kernel

// SM (FP64, whose 16-byte values would need 64 registers for the source signatures alone): the
// loop runs source-octant-major, each source octant's two values loaded when it is reached and
// applied to every present target octant far from it. Its chunks hold 32 pairs (the table of 64
// would not fit the LDS), so the two halves of a wave take the same pairs and split the target
// octants by their x bit: half h serves the octants 2 j + h, whose offset row from a source octant
// is that of 2 j minus one (one select per lane), and keeps their sums only.
template <class C, int CW, bool SM>
__global__ __launch_bounds__(kWave * kTW) void m2lt_kernel(
    int K, int Kp, int nranges, int64_t np, const int32_t* __restrict__ pslots,
    const int32_t* __restrict__ child_start, const int32_t* __restrict__ child_count,
    const int32_t* __restrict__ octant, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ pairs, const int32_t* __restrict__ tperm,
    const C* __restrict__ T, const C* __restrict__ M, C* __restrict__ out,
    int64_t nb, int nrhs)
{
    static_assert(CW <= kWave && CW % 16 == 0, "chunk width");
    static_assert(!SM || 2 * CW == kWave, "the source-octant-major loop splits a wave in two halves");
    __shared__ C Ts[kNumOffsets][CW];
    __shared__ int s_next;
    const unsigned lb = xcd_block(blockIdx.x, gridDim.x);
    const int chunk = (int)(lb / (unsigned)nranges), range = (int)(lb % (unsigned)nranges);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    // the lane's direction pair in the chunk, and with SM the half of the wave (x bit of its
    // target octants)
    const int cl = SM ? lane % CW : (lane < CW ? lane : CW - 1);
    const int hb = SM ? lane / CW : 0;
    const int pi = chunk * CW + cl;
    const bool pvalid = (SM || lane < CW) && pi < Kp;
    // idle lanes work on the first pair and store nothing
    const int k1 = pairs[2 * (pvalid ? pi : 0)], k2 = pairs[2 * (pvalid ? pi : 0) + 1];
    // T_{g rep}(s_k1) = T_rep(s_{tperm[g][k1]}) of every transfer vector, row t of the table
    const int32_t* row_tix = rows + 27 * 27;
    const int32_t* farm = rows + 27 * 27 + kNumOffsets;
    const int32_t* farmt = farm + 27 * 8;
    constexpr int kRowsPerWave = (kNumOffsets + kTW - 1) / kTW;
#pragma unroll 5
    for (int j = 0; j < kRowsPerWave; ++j) {
        const int t = j * kTW + w;
        if (t < kNumOffsets) {
            const int tx = row_tix[t];
            const C v = T[(int64_t)(tx >> 4) * K + tperm[(int64_t)(tx & (kNumSym - 1)) * K + k1]];
            if (lane < CW) Ts[t][lane] = v;
        }
    }
    if (threadIdx.x == 0) s_next = 0;
    __syncthreads();
    const int64_t pb = np * range / nranges, pe = np * (range + 1) / nranges;
    const int64_t plane = nb * (int64_t)K;
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(&s_next, 1);
        item = __builtin_amdgcn_readfirstlane(item);   // every lane is active here: lane 0's value
        const int64_t P = pb + item;
        if (P >= pe) break;
        const int tb = child_start[P], tn = child_count[P];
        // lane D: neighbour slot D (the centre slot, P itself, has no far pairs)
        int sb = 0, sm = 0;
        bool occ_l = false;
        if (lane < 27 && lane != 13) {
            const int Pn = pslots[P * 27 + lane];
            if (Pn >= 0) {
                occ_l = true;
                sb = child_start[Pn];
                const int sn = child_count[Pn];
                for (int i = 0; i < sn; ++i) sm |= 1 << octant[sb + i];
            }
        }
        const uint64_t occ0 = __ballot(occ_l);
        const int ot_l = lane < tn ? octant[tb + lane] : -1;
        int tm = 0;
#pragma unroll
        for (int o = 0; o < 8; ++o) tm |= (__ballot(ot_l == o) != 0 ? 1 : 0) << o;
        for (int r = 0; r < nrhs; ++r) {
            const C* Mr = M + (int64_t)r * plane;
            // per target octant (with SM: per octant 2 j + hb of this half, at j)
            constexpr int NO = SM ? 4 : 8;
            C acc[NO][2];
#pragma unroll
            for (int o = 0; o < NO; ++o) acc[o][0] = acc[o][1] = cz<C>();
            uint64_t occ = occ0;
            while (occ) {
                const int D = __builtin_ctzll(occ);
                occ &= occ - 1;
                const int sbD = __builtin_amdgcn_readlane(sb, D);
                const int smD = __builtin_amdgcn_readlane(sm, D);
                const int32_t* pr = rows + 27 * D;
                const int32_t* fm = farm + 8 * D;
                int rr[27];
#pragma unroll
                for (int e = 0; e < 27; ++e) rr[e] = pr[e];
                if constexpr (SM) {
                    const int32_t* ft = farmt + 8 * D;
#pragma unroll
                    for (int os = 0; os < 8; ++os) {
                        if (!((smD >> os) & 1)) continue;
                        const int m = ft[os] & tm;
                        if (!m) continue;
                        const int ci = sbD + __builtin_popcount(smD & ((1 << os) - 1));
                        const C* mp = Mr + (int64_t)ci * K;
                        const C m1 = mp[k1], m2 = mp[k2];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            // the target octants 2 j (half 0) and 2 j + 1 (half 1)
                            const int mj = (m >> (2 * j)) & 3;
                            if (!mj) continue;
                            __asm__ __volatile__("");
                            const int e = ((os & 1) + 1) + 3 * (((os >> 1) & 1) - (j & 1) + 1) +
                                          9 * (((os >> 2) & 1) - ((j >> 1) & 1) + 1);
                            const int row = hb ? rr[e - 1] : rr[e];
                            if ((mj >> hb) & 1) {
                                cmac(acc[j][0], m1, Ts[row][cl]);
                                cmac(acc[j][1], m2, Ts[kNumOffsets - 1 - row][cl]);
                            }
                        }
                    }
                } else {
                // source signatures of the present octants at s and -s
                C ms[8][2];
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    ms[o][0] = ms[o][1] = cz<C>();
                    if ((smD >> o) & 1) {
                        const int ci = sbD + __builtin_popcount(smD & ((1 << o) - 1));
                        const C* mp = Mr + (int64_t)ci * K;
                        ms[o][0] = mp[k1];
                        ms[o][1] = mp[k2];
                    }
                }
                // per present target octant, the present source octants far from it
#pragma unroll
                for (int ot = 0; ot < 8; ++ot) {
                    if (!((tm >> ot) & 1)) continue;
                    const int m = fm[ot] & smD;
                    if (!m) continue;
#pragma unroll
                    for (int os = 0; os < 8; ++os) {
                        if (!((m >> os) & 1)) continue;
                        __asm__ __volatile__("");
                        const int e = ((os & 1) - (ot & 1) + 1) + 3 * (((os >> 1) & 1) - ((ot >> 1) & 1) + 1) +
                                      9 * (((os >> 2) & 1) - ((ot >> 2) & 1) + 1);
                        const int row = rr[e];
                        cmac(acc[ot][0], ms[os][0], Ts[row][cl]);
                        cmac(acc[ot][1], ms[os][1], Ts[kNumOffsets - 1 - row][cl]);
                    }
                }
                }
            }
            if (pvalid)
                for (int i = 0; i < tn; ++i) {
                    const int c = tb + i;
                    const int o = __builtin_amdgcn_readfirstlane(octant[c]);
                    if (SM && (o & 1) != hb) continue;   // the other half holds this child
                    const int oa = SM ? o >> 1 : o;
                    C* op = out + (int64_t)r * plane + (int64_t)c * K;
#pragma unroll
                    for (int oo = 0; oo < NO; ++oo)
                        if (oo == oa) {
                            op[k1] = acc[oo][0];
                            op[k2] = acc[oo][1];
                        }
                }
        }
    }
}

// ------------------------------------------------------------------------------------------
// L2P (far part of eqn. FMM_FinalStep): phi_i += sum_k w_k L_b(s_k) e^{i kappa s_k.(c_b - x_i)};
// with GRAD the gradient with respect to x_i, sum_k w_k L_b(s_k) (-i kappa s_k) e^{...}.
// One wave per leaf box (four per block), one lane per target point; the directions are taken in
// antipodal pairs (one phase and one sine/cosine per pair), staged in the wave's own LDS in
// chunks. The sum over k is blocked: plain sums of up to 16 directions, combined with TwoSum, which
// keeps the FP32 accumulation error of the large cancelling terms near the size of the result.
// ------------------------------------------------------------------------------------------
constexpr int kL2PChunk = 256;

// NR right-hand sides per block (blockIdx.y: the group r0 .. r0 + NR - 1) share each pair's phase and
// sine/cosine; without GRAD only.
template <class R, class C, bool GRAD, int NR>
__global__ __launch_bounds__(kWave * kWpb) void l2p_kernel(int Kp, const R* __restrict__ dirs,
                                                    const int32_t* __restrict__ pairs,
                                                    const R* __restrict__ w, R kfac, R kappa,
                                                    const int32_t* __restrict__ start,
                                                    const int32_t* __restrict__ count,
                                                    const R* __restrict__ rel, const C* __restrict__ L,
                                                    C* __restrict__ out, int64_t n, int64_t nb, int K, int nrhs)
{
    constexpr int NC = GRAD ? 3 : 1;
    static_assert(NR == 1 || !GRAD, "the gradient serves one right-hand side per block");
    // per antipodal pair (s, -s) with weighted values u1 = w L(s) = a1 + i b1, u2 = w L(-s):
    // s and P = a1 + a2, Q = b1 - b2, V = b1 + b2, S = a1 - a2, so that the pair contributes
    // (c P - sn Q) + i (c V + sn S) for e^{i ph} = c + i sn, ph = kappa s.(c_b - x_i)
    // pairs staged per chunk: 256, or 128 for the FP64 potential (28 KB of LDS per block, so that
    // several blocks share a CU; the FP64 gradient keeps 256 for its combine area); with NR
    // right-hand sides 256 / NR (FP32) or 128 / NR (FP64)
    constexpr int CH = NR > 1 ? (sizeof(R) == 4 ? kL2PChunk : kL2PChunk / 2) / NR
                              : ((sizeof(R) == 4 || GRAD) ? kL2PChunk : kL2PChunk / 2);
    static_assert(CH % 64 == 0, "chunks hold whole runs of 64 pairs");
    __shared__ R sxa[kWpb][CH], sya[kWpb][CH], sza[kWpb][CH];
    __shared__ R spa[kWpb][NR][CH], sqa[kWpb][NR][CH], sva[kWpb][NR][CH], ssa[kWpb][NR][CH];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t b = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kWpb + wv;
    if (b >= nb) return;
    R* sx = sxa[wv];
    R* sy = sya[wv];
    R* sz = sza[wv];
    R (*sP)[CH] = spa[wv];
    R (*sQ)[CH] = sqa[wv];
    R (*sV)[CH] = sva[wv];
    R (*sS)[CH] = ssa[wv];
    const int64_t r0 = (int64_t)blockIdx.y * NR;
    const int nr = min(NR, nrhs - (int)r0);
    const int s0 = start[b], cnt = count[b];
    const int64_t plane = nb * K;
    const C* Lb = L + r0 * plane + b * K;
    for (int t0 = 0; t0 < cnt; t0 += kWave) {
        // g lanes per target split its pairs when the chunk has few targets (a power of two, so
        // that a lane takes exactly 8 pairs of every block of 8 g)
        const int tcnt = min(kWave, cnt - t0);
        const int g = 1 << (31 - __builtin_clz(kWave / tcnt));
        const int my = lane / g, sub = lane % g;
        const bool valid = my < tcnt;
        const int64_t i = s0 + t0 + (valid ? my : 0);
        R x = 0, y = 0, z = 0;
        if (valid) {
            x = -rel[3 * i] * kfac;      // kappa (c_b - x_i), in the phase units of R
            y = -rel[3 * i + 1] * kfac;
            z = -rel[3 * i + 2] * kfac;
        }
        R sre[NR][NC], sim[NR][NC], ere[NR][NC], eim[NR][NC];
        for (int u = 0; u < NR; ++u)
            for (int a = 0; a < NC; ++a) sre[u][a] = sim[u][a] = ere[u][a] = eim[u][a] = 0;
        for (int k0 = 0; k0 < Kp; k0 += CH) {
            const int nk = min(CH, Kp - k0);
            wave_lds_sync();
            // pairs past the chunk's end up to a multiple of 64 are zero: they add exactly nothing,
            // so that every block of 8 g pairs runs whole
            for (int k = nk + lane; k < ((nk + 63) & ~63); k += kWave) {
                sx[k] = sy[k] = sz[k] = 0;
#pragma unroll
                for (int u = 0; u < NR; ++u) sP[u][k] = sQ[u][k] = sV[u][k] = sS[u][k] = 0;
            }
            for (int k = lane; k < nk; k += kWave) {
                const int k1 = pairs[2 * (k0 + k)], k2 = pairs[2 * (k0 + k) + 1];
                sx[k] = dirs[3 * k1];
                sy[k] = dirs[3 * k1 + 1];
                sz[k] = dirs[3 * k1 + 2];
                const R w1 = w[k1], w2 = w[k2];
#pragma unroll
                for (int u = 0; u < NR; ++u) {
                    R a1 = 0, b1 = 0, a2 = 0, b2 = 0;
                    if (u < nr) {
                        const C l1 = Lb[u * plane + k1], l2 = Lb[u * plane + k2];
                        a1 = w1 * l1.x;
                        b1 = w1 * l1.y;
                        a2 = w2 * l2.x;
                        b2 = w2 * l2.y;
                    }
                    sP[u][k] = a1 + a2;
                    sQ[u][k] = b1 - b2;
                    sV[u][k] = b1 + b2;
                    sS[u][k] = a1 - a2;
                }
            }
            wave_lds_sync();
            // each lane: plain sums over 8 of its pairs (16 directions), combined with TwoSum;
            // blocks of 8 g pairs, at most 64, so that they tile every chunk size alike and a
            // right-hand side gets the same sums alone or in a group
            const int B = min(64, 8 * g);
            auto term = [&](R (&pre)[NR][NC], R (&pim)[NR][NC], int k) {
                R c, sn;
                cis(sx[k] * x + sy[k] * y + sz[k] * z, c, sn);
                if (GRAD) {
                    // (-i kappa s)[c (u1 - u2) + i sn (u1 + u2)] = kappa s (Y - i X)
                    const R X = c * sS[0][k] - sn * sV[0][k], Y = c * sQ[0][k] + sn * sP[0][k];
                    const R sa[3] = {sx[k], sy[k], sz[k]};
                    for (int a = 0; a < NC; ++a) {
                        pre[0][a] += kappa * sa[a] * Y;
                        pim[0][a] -= kappa * sa[a] * X;
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < NR; ++u) {
                        // explicit fused multiply-adds, two per component: the same rounding in
                        // every instantiation
                        pre[u][0] = fma(-sn, sQ[u][k], fma(c, sP[u][k], pre[u][0]));
                        pim[u][0] = fma(sn, sS[u][k], fma(c, sV[u][k], pim[u][0]));
                    }
                }
            };
            // one block: the lane's plain sums, then TwoSum into its running sums
            auto block = [&](auto&& body) {
                R pre[NR][NC], pim[NR][NC];
                for (int u = 0; u < NR; ++u)
                    for (int a = 0; a < NC; ++a) pre[u][a] = pim[u][a] = 0;
                body(pre, pim);
                for (int u = 0; u < NR; ++u)
                    for (int a = 0; a < NC; ++a) {
                        R e1, e2;
                        two_sum(sre[u][a], pre[u][a], sre[u][a], e1);
                        two_sum(sim[u][a], pim[u][a], sim[u][a], e2);
                        ere[u][a] += e1;
                        eim[u][a] += e2;
                    }
            };
            // separate loops for one lane per target (stride 1: the LDS reads of consecutive
            // pairs pair up) and for g lanes per target
            // (unrolled for one right-hand side's potential only: with several right-hand sides or
            // the gradient, the unrolled block holds every staged value in registers and occupancy
            // drops)
            constexpr int kUnroll = NR == 1 && !GRAD ? 8 : 1;
            if (g == 1) {
                for (int kb = 0; kb < nk; kb += 8)
                    block([&](R (&pre)[NR][NC], R (&pim)[NR][NC]) {
#pragma unroll kUnroll
                        for (int kk = 0; kk < 8; ++kk) term(pre, pim, kb + kk);
                    });
            } else {
                for (int kb = 0; kb < nk; kb += B)
                    block([&](R (&pre)[NR][NC], R (&pim)[NR][NC]) {
                        if (B == 8 * g) {
#pragma unroll kUnroll
                            for (int kk = 0; kk < 8; ++kk) term(pre, pim, kb + sub + g * kk);
                        } else {
                            for (int k = kb + sub; k < kb + B; k += g) term(pre, pim, k);
                        }
                    });
            }
        }
        if (g > 1) {
            // the g lanes of a target combine their compensated sums in lane order, through this
            // wave's staging arrays, read flat (free now; entry (u NC + a) kWave + lane of each)
            static_assert(NC * kWave <= CH, "combine area");
            R* cP = &sP[0][0];
            R* cQ = &sQ[0][0];
            R* cV = &sV[0][0];
            R* cS = &sS[0][0];
            wave_lds_sync();
            for (int u = 0; u < NR; ++u)
                for (int a = 0; a < NC; ++a) {
                    const int e = (u * NC + a) * kWave + lane;
                    cP[e] = sre[u][a];
                    cQ[e] = sim[u][a];
                    cV[e] = ere[u][a];
                    cS[e] = eim[u][a];
                }
            wave_lds_sync();
            if (valid && sub == 0)
                for (int u = 0; u < NR; ++u)
                    for (int a = 0; a < NC; ++a)
                        for (int v = 1; v < g; ++v) {
                            const int e = (u * NC + a) * kWave + lane + v;
                            R e1, e2;
                            two_sum(sre[u][a], cP[e], sre[u][a], e1);
                            two_sum(sim[u][a], cQ[e], sim[u][a], e2);
                            ere[u][a] += cV[e] + e1;
                            eim[u][a] += cS[e] + e2;
                        }
            wave_lds_sync();
        }
        if (valid && sub == 0)   // every point lies in one leaf: a plain store
            for (int u = 0; u < nr; ++u)
                for (int a = 0; a < NC; ++a)
                    out[((r0 + u) * n + i) * NC + a] = cmk<C>(sre[u][a] + ere[u][a], sim[u][a] + eim[u][a]);
    }
}

// ------------------------------------------------------------------------------------------
// P2P (near part of eqn. FMM_FinalStep): phi_i += sum_{j in N(b), j != i, R > 0} e^{i kappa R}/R q_j;
// with GRAD: sum G'(R) (x_i - x_j)/R q_j, G'(R) = e^{i kappa R}(i kappa R - 1)/R^2.
// One wave per leaf box (four per block), lanes = targets (g lanes per target when the box has few
// points), source points staged in the wave's own LDS 64 at a time.
// R and kappa R in FP64; in the FP32 path kappa R is reduced modulo 2 pi in FP64 and the
// sine/cosine, 1/R and the sums are FP32.
// ------------------------------------------------------------------------------------------
// The charge-independent part of one near-field term: g = e^{i kR}/R, or with GRAD the factor
// e^{i kR}(i kR - 1)/R^3 and x_i - x_j; pair_apply then adds g q_j (with GRAD (x_i - x_j) g q_j).
template <class R, class C, bool GRAD> struct NearTerm {
    C g;
    R d[GRAD ? 3 : 1];
};

template <class R, class C, bool GRAD, bool FAST = false>
__device__ __forceinline__ NearTerm<R, C, GRAD> pair_geom(double xi, double yi, double zi, double4 pj,
                                                          double kappa, double kappa_rev)
{
    const double dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    R c, s, inv, kr;
    if constexpr (FAST) {
        static_assert(sizeof(R) == 4, "FAST is an FP32 form");
        const float r2f = (float)r2;
        const bool ok = r2f > 0.0f;
        const float y = __builtin_amdgcn_rsqf(ok ? r2f : 1.0f);
        const float rf = r2f * y;
        cis(rf * (float)kappa_rev, c, s);
        inv = ok ? y : 0.0f;
        if constexpr (GRAD) kr = (float)kappa * rf;
    } else if constexpr (sizeof(R) == 4) {
        // y0 = hardware reciprocal square root of the FP32-rounded R^2 (about 1 ulp of FP32); one
        // Newton step in FP64 written as R = u (1 + e), u = R^2 y0, e = (1 - u y0) / 2, so R and
        // the phase kappa R / 2 pi stay FP64-accurate (relative ~1e-14); the phase is reduced
        // modulo 1 in FP64 before the FP32 sine/cosine, and the FP32 1/R is y0 itself.
        // the pair of a point with itself (R = 0) is computed on a clamped R^2 and dropped by the
        // select of 1/R below
        const bool ok = r2 > 0.0;
        const double r2s = fmax(r2, 1e-30);
        const float y0f = __builtin_amdgcn_rsqf((float)r2s);
        const double y0 = (double)y0f;
        const double u = r2s * y0;
        const double eh = fma(-0.5, u * y0, 0.5);
        const double rr = fma(u, eh, u);
        // the phase in revolutions, reduced to [0, 1) by the hardware fraction (rev >= 0)
        const double rev = __builtin_amdgcn_fract(rr * kappa_rev);
        cis((float)rev, c, s);
        inv = ok ? y0f : 0.0f;
        if constexpr (GRAD) kr = (R)(kappa * rr);
    } else {
        // 1/R from the hardware reciprocal square root refined by two Newton steps
        // y <- y (3 - R^2 y^2) / 2 (each squares the relative error), R = R^2 y
        const bool ok = r2 > 0.0;
        const double r2s = ok ? r2 : 1.0;
        double y = __builtin_amdgcn_rsq(r2s);
        y = y * fma(-0.5 * r2s, y * y, 1.5);
        y = y * fma(-0.5 * r2s, y * y, 1.5);
        const double rr = r2s * y;
        cis(kappa_rev * rr, c, s);
        inv = ok ? y : 0.0;
        if constexpr (GRAD) kr = kappa * rr;
    }
    NearTerm<R, C, GRAD> t;
    if constexpr (GRAD) {
        // explicit fused multiply-adds here and in pair_apply: the rounding is the same in every
        // instantiation, so a right-hand side gets the same bits alone or in a group
        const R inv3 = inv * inv * inv;
        t.g = cmk<C>(fma(-s, kr, -c) * inv3, fma(c, kr, -s) * inv3);
        t.d[0] = (R)dx;
        t.d[1] = (R)dy;
        t.d[2] = (R)dz;
    } else {
        t.g = cmk<C>(c * inv, s * inv);
    }
    return t;
}

template <class R, class C, bool GRAD>
__device__ __forceinline__ void pair_apply(const NearTerm<R, C, GRAD>& t, C qj, C (&acc)[GRAD ? 3 : 1])
{
    if constexpr (GRAD) {
        const R gx = fma(t.g.x, qj.x, -(t.g.y * qj.y)), gy = fma(t.g.x, qj.y, t.g.y * qj.x);
        for (int a = 0; a < 3; ++a) {
            acc[a].x = fma(t.d[a], gx, acc[a].x);
            acc[a].y = fma(t.d[a], gy, acc[a].y);
        }
    } else {
        cmac(acc[0], t.g, qj);
    }
}

// One near-field term of target (xi, yi, zi) and source pj (x, y, z) with charge qj: with GRAD the
// gradient e^{i kR}(i kR - 1)/R^3 (x_i - x_j) q_j, else e^{i kR}/R q_j, added to acc. R = 0 exactly
// (the target itself, or a coincident point) contributes nothing. The coordinate differences and
// R^2 are FP64 always: close pairs lose their digits to cancellation otherwise.
// FAST (FP32 only, for near-field ranges of at most kFastRev revolutions of the phase): R^2 is
// rounded to FP32 and 1/R, R and the phase kR/2pi follow in FP32, relative error ~1e-7, so the
// phase is good to ~1e-6 of a revolution.
template <class R, class C, bool GRAD, bool FAST = false>
__device__ __forceinline__ void pair_term(double xi, double yi, double zi, double4 pj, C qj, double kappa,
                                          double kappa_rev, C (&acc)[GRAD ? 3 : 1])
{
    pair_apply<R, C, GRAD>(pair_geom<R, C, GRAD, FAST>(xi, yi, zi, pj, kappa, kappa_rev), qj, acc);
}

// NR right-hand sides per block share each pair's geometry, phase and 1/R (blockIdx.y: the group
// of right-hand sides r0 .. r0 + NR - 1).
template <class R, class C, bool GRAD, bool FAST, int NR>
__global__ __launch_bounds__(kWave * kWpb) void p2p_kernel(const double* __restrict__ xs,
                                                    const C* __restrict__ q,
                                                    const int32_t* __restrict__ start,
                                                    const int32_t* __restrict__ count,
                                                    const int32_t* __restrict__ nb_ptr,
                                                    const int32_t* __restrict__ nb_src, double kappa,
                                                    C* __restrict__ out, int64_t n, int64_t nleaf, int nrhs)
{
    constexpr int NC = GRAD ? 3 : 1;
    __shared__ double4 spa[kWpb][kWave];   // staged sources: x, y, z (w unused)
    __shared__ C sqa[kWpb][NR][kWave];
    __shared__ C parta[kWpb][NC][kWave];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
    double4* sp = spa[wv];
    C (*sq)[kWave] = sqa[wv];
    C (*part)[kWave] = parta[wv];
    const int64_t r0 = (int64_t)blockIdx.y * NR;
    const int nr = min(NR, nrhs - (int)r0);
    const double kappa_rev = kappa / kTwoPi;
    // A block serves logical blocks of kWpb leaves in a loop (the grid may hold fewer blocks than
    // there are leaves, so that P2P leaves room for the far-field kernels running beside it). With
    // one block per logical block, or a grid of whole XCD rounds, each XCD walks a contiguous
    // Morton range, so that the neighbour boxes a leaf reads are mostly in its XCD's L2 already.
    const unsigned nlog = (unsigned)((nleaf + kWpb - 1) / kWpb);
    constexpr unsigned kXcd = 8;
    unsigned j0, jstep, jend, base;
    if (gridDim.x == nlog) {
        base = xcd_block(blockIdx.x, nlog);
        j0 = 0;
        jend = 1;
        jstep = 1;
    } else if (gridDim.x % kXcd == 0) {
        const unsigned x = blockIdx.x % kXcd, per = nlog / kXcd, rem = nlog % kXcd;
        base = x * per + min(x, rem);
        jend = per + (x < rem ? 1 : 0);
        j0 = blockIdx.x / kXcd;
        jstep = gridDim.x / kXcd;
    } else {
        base = 0;
        jend = nlog;
        j0 = blockIdx.x;
        jstep = gridDim.x;
    }
    for (unsigned j = j0; j < jend; j += jstep) {
    const int64_t b = (int64_t)(base + j) * kWpb + wv;
    if (b >= nleaf) continue;
    const int tb = start[b], tc = count[b];
    for (int t0 = 0; t0 < tc; t0 += kWave) {
        // g lanes per target split its sources: chunks of few targets keep the wave busy
        const int tcnt = min(kWave, tc - t0);
        const int g = kWave / tcnt;
        const int my = lane / g, sub = lane % g;
        const bool valid = my < tcnt;
        const int64_t i = tb + t0 + (valid ? my : 0);
        const double xi = xs[3 * i], yi = xs[3 * i + 1], zi = xs[3 * i + 2];
        C acc[NR][NC];
        for (int u = 0; u < NR; ++u)
            for (int a = 0; a < NC; ++a) acc[u][a] = cz<C>();
        // the pair's geometry once, then its product with each right-hand side's charge
        auto term = [&](int t) {
            const NearTerm<R, C, GRAD> tt = pair_geom<R, C, GRAD, FAST>(xi, yi, zi, sp[t], kappa, kappa_rev);
#pragma unroll
            for (int u = 0; u < NR; ++u) pair_apply<R, C, GRAD>(tt, sq[u][t], acc[u]);
        };
        for (int e = nb_ptr[b]; e < nb_ptr[b + 1]; ++e) {
            const int c = nb_src[e];
            const int sb = start[c], sc = count[c];
            for (int s0 = 0; s0 < sc; s0 += kWave) {
                const int ns = min(kWave, sc - s0);
                wave_lds_sync();
                if (lane < ns) {
                    const int64_t j = sb + s0 + lane;
                    sp[lane] = make_double4(xs[3 * j], xs[3 * j + 1], xs[3 * j + 2], 0.0);
#pragma unroll
                    for (int u = 0; u < NR; ++u) sq[u][lane] = u < nr ? q[(r0 + u) * n + j] : cz<C>();
                }
                wave_lds_sync();
                if (g == 1) {
                    // one target per lane: a loop the whole wave runs in step (lanes past the
                    // chunk repeat its first target and store nothing)
#pragma unroll 4
                    for (int t = 0; t < ns; ++t) term(t);
                } else if (valid) {
                    for (int t = sub; t < ns; t += g) term(t);
                }
            }
        }
        // combine the g partial sums of every target, one right-hand side at a time
        for (int u = 0; u < nr; ++u) {
            for (int a = 0; a < NC; ++a) part[a][lane] = acc[u][a];
            wave_lds_sync();
            if (valid && sub == 0)
                for (int a = 0; a < NC; ++a) {
                    C sum = part[a][lane];
                    for (int v = 1; v < g; ++v) {
                        sum.x += part[a][lane + v].x;
                        sum.y += part[a][lane + v].y;
                    }
                    out[((r0 + u) * n + i) * NC + a] = sum;   // every point lies in one leaf: a plain store
                }
            wave_lds_sync();
        }
    }
    }
}

// ------------------------------------------------------------------------------------------
// Direct sum over all pairs (the O(N^2) evaluation of eqn. HelmholtzMatrixVector the FMM is
// measured against), with the near-field arithmetic. A block: 64 targets (one per lane of each
// wave); the four waves take interleaved quarters of every 256-source tile staged in LDS, and
// their partial sums are added at the end.
// ------------------------------------------------------------------------------------------
template <class R, class C, bool GRAD>
__global__ __launch_bounds__(256) void direct_kernel(const double* __restrict__ xs, const C* __restrict__ q,
                                                     int64_t n, double kappa, C* __restrict__ out)
{
    constexpr int NC = GRAD ? 3 : 1;
    __shared__ double4 sp[256];
    __shared__ C sq[256];
    __shared__ C part[4][NC][kWave];
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int64_t r = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * kWave + lane;
    const bool valid = i < n;
    const int64_t ii = valid ? i : 0;
    const double xi = xs[3 * ii], yi = xs[3 * ii + 1], zi = xs[3 * ii + 2];
    const double kappa_rev = kappa / kTwoPi;
    C acc[NC];
    for (int a = 0; a < NC; ++a) acc[a] = cz<C>();
    for (int64_t s0 = 0; s0 < n; s0 += 256) {
        const int ns = (int)min<int64_t>(256, n - s0);
        __syncthreads();
        if (tid < ns) {
            const int64_t j = s0 + tid;
            sp[tid] = make_double4(xs[3 * j], xs[3 * j + 1], xs[3 * j + 2], 0.0);
            sq[tid] = q[r * n + j];
        }
        __syncthreads();
        for (int t = wv; t < ns; t += 4) pair_term<R, C, GRAD>(xi, yi, zi, sp[t], sq[t], kappa, kappa_rev, acc);
    }
    for (int a = 0; a < NC; ++a) part[wv][a][lane] = acc[a];
    __syncthreads();
    if (wv == 0 && valid)
        for (int a = 0; a < NC; ++a) {
            C v = part[0][a][lane];
            for (int u = 1; u < 4; ++u) {
                v.x += part[u][a][lane].x;
                v.y += part[u][a][lane].y;
            }
            out[(r * n + i) * NC + a] = v;
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

// caller order -> Morton order into the plan's charges at right-hand side r_off.. (+ conjugation)
template <class R>
void gather_t(ffmm_plan* p, const void* qv, int nrhs, bool conj, int r_off, hipStream_t s)
{
    using C = typename cplx_t<R>::type;
    StageScope sc(p, FFMM_PROF_GATHER, s);
    hipLaunchKernelGGL(gather_q<C>, dim3(nblk(p->n, 256), nrhs), dim3(256), 0, s, (const C*)qv, p->perm,
                       p->n, conj ? 1 : 0, (C*)p->qs + (int64_t)r_off * p->n);
    FFMM_LAUNCH_CHECK();
}

// Everything between the gather and the scatter: from the Morton-ordered charges of nrhs
// right-hand sides to the far field (p->phis, L2P) and the near field (p->phin, P2P, or the whole
// sum with the direct method), [nrhs][n] ([nrhs][n][3] with gradient), in Morton order.
template <class R>
void core_t(ffmm_plan* p, int nrhs, int stages, bool gradient, hipStream_t s)
{
    using C = typename cplx_t<R>::type;
    const int64_t n = p->n;
    const int L = p->depth;
    C* qs = (C*)p->qs;
    C* phis = (C*)p->phis;
    C* phin = (C*)p->phin;
    const R kfac = phase_scale<R>(p->kappa);
    if (p->direct) {
        // all pairs are near: one direct-sum launch
        if (stages & FFMM_STAGE_NEAR) {
            StageScope sc(p, FFMM_PROF_P2P, s);
            if (gradient)
                hipLaunchKernelGGL((direct_kernel<R, C, true>), dim3(nblk(n, kWave), nrhs), dim3(256), 0, s,
                                   p->xs, qs, n, p->kappa, phin);
            else
                hipLaunchKernelGGL((direct_kernel<R, C, false>), dim3(nblk(n, kWave), nrhs), dim3(256), 0, s,
                                   p->xs, qs, n, p->kappa, phin);
            FFMM_LAUNCH_CHECK();
        }
        return;
    }
    // P2P needs only the gathered charges: it runs on the plan's near-field stream (not while
    // stages are timed: each stage's event interval then holds its own kernels alone)
    const bool fork = (stages & FFMM_STAGE_NEAR) && p->tune.near_stream && !p->profile;
    auto launch_p2p = [&](hipStream_t sn) {
        StageScope sc(p, FFMM_PROF_P2P, sn);
        const int64_t nl = p->lev[L].n;
        const int64_t nlog = (nl + kWpb - 1) / kWpb;
        const int bpc = p->tune.p2p_blocks_per_cu;
        const unsigned grid = (unsigned)(bpc > 0 ? std::min<int64_t>(nlog, (int64_t)p->n_cu * bpc) : nlog);
        // FP32 phase when the near-field range spans few revolutions (sources within two leaf
        // sides per axis: R <= 2 sqrt(3) a)
        const bool fast = sizeof(R) == 4 && p->opt.fast_near_phase &&
                          p->kappa * 2.0 * std::sqrt(3.0) * p->lev[L].a / kTwoPi <= kFastRev;
        // right-hand sides sharing each pair's geometry (fewer with gradients and in FP64, whose
        // per-RHS accumulators take more registers)
        const int nr_max = gradient ? 2 : (sizeof(R) == 4 ? 8 : 4);
        const int NRv = nrhs >= 8 && nr_max >= 8 ? 8 : (nrhs >= 4 && nr_max >= 4 ? 4 : (nrhs >= 2 ? 2 : 1));
        const unsigned gy = (unsigned)((nrhs + NRv - 1) / NRv);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(grid, gy), dim3(kWave * kWpb), 0, sn, p->xs, qs, p->leaf_start,
                               p->leaf_count, p->nb_ptr, p->nb_src, p->kappa, phin, n, (int64_t)nl, nrhs);
        };
        auto pick = [&](auto grad_tag, auto fast_tag) {
            constexpr bool G = decltype(grad_tag)::value, F = decltype(fast_tag)::value;
            if constexpr (!G && sizeof(R) == 4) {
                if (NRv == 8) return go(p2p_kernel<R, C, G, F, 8>);
            }
            if constexpr (!G) {
                if (NRv == 4) return go(p2p_kernel<R, C, G, F, 4>);
            }
            if (NRv == 2) return go(p2p_kernel<R, C, G, F, 2>);
            go(p2p_kernel<R, C, G, F, 1>);
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        constexpr bool fp32 = sizeof(R) == 4;
        if (gradient) {
            if (fast) pick(T_{}, std::integral_constant<bool, fp32>{});
            else pick(T_{}, F_{});
        } else {
            if (fast) pick(F_{}, std::integral_constant<bool, fp32>{});
            else pick(F_{}, F_{});
        }
        FFMM_LAUNCH_CHECK();
    };
    // fork point: before the far field (near_stream 2, or P2P alone), else after the upward pass
    const bool fork_early = fork && (!(stages & FFMM_STAGE_FAR) || p->tune.near_stream == 2);
    if (fork_early) {
        FFMM_HIP(hipEventRecord(p->ev_fork, s));
        FFMM_HIP(hipStreamWaitEvent(p->near_stream, p->ev_fork, 0));
        launch_p2p(p->near_stream);
    }
    if (stages & FFMM_STAGE_FAR) {
        LevelData& leaf = p->lev[L];
        // P2M
        {
            StageScope sc(p, FFMM_PROF_P2M, s);
            int nth = 256;
            for (int w : {128, 64})
                if ((leaf.Kp + w - 1) / w * w < (leaf.Kp + nth - 1) / nth * nth) nth = w;
            const int kch = (leaf.Kp + nth - 1) / nth;
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3((unsigned)(leaf.n * kch), nrhs), dim3(nth), 0, s, leaf.Kp, kch,
                                   (const R*)leaf.dirs, leaf.pairs, kfac, p->leaf_start, p->leaf_count,
                                   (const R*)p->rel, qs, (C*)leaf.sigM, n, leaf.n, leaf.K);
            };
            if (nth == 64)
                go(p2m_kernel<R, C, 64>);
            else if (nth == 128)
                go(p2m_kernel<R, C, 128>);
            else
                go(p2m_kernel<R, C, 256>);
            FFMM_LAUNCH_CHECK();
        }
        // M2M, l = L..3 (five-step resample to the parent grid, translate, sum children)
        for (int l = L; l >= 3; --l) {
            StageScope sc(p, FFMM_PROF_M2M, s);
            run_resample(p, l, l - 1, nrhs, s);
        }
        // P2P forks after the upward pass: beside M2L and the downward pass it costs the far field
        // less than beside M2M (measured: 3.59 against 3.68 ms per matvec at 2^20 points)
        if (fork && !fork_early) {
            FFMM_HIP(hipEventRecord(p->ev_fork, s));
            FFMM_HIP(hipStreamWaitEvent(p->near_stream, p->ev_fork, 0));
            launch_p2p(p->near_stream);
        }
        // M2L, l = 2..L (written into the L buffers, which then receive the downward pass)
        int rb = p->tune.m2l_rhs_block;
        if (rb == 0) rb = nrhs >= 4 ? 4 : (nrhs >= 2 ? 2 : 1);
        for (int l = 2; l <= L; ++l) {
            StageScope sc(p, l == L ? FFMM_PROF_LEAF_M2L : FFMM_PROF_M2L, s);
            LevelData& Lv = p->lev[l];
            LevelData& Pv = p->lev[l - 1];
            if (!((p->m2l_levels >> l) & 1u)) {
                // error studies: this level's interaction lists contribute nothing
                FFMM_HIP(hipMemsetAsync(Lv.sigL, 0, sizeof(C) * (size_t)nrhs * Lv.n * Lv.K, s));
                continue;
            }
            const int kch = (Lv.K + 255) / 256;
            {
                if (p->tune.m2l_by_parent == 2) {
                    // chunks of CW antipodal direction pairs; ranges of parents so that the grid
                    // is about one block per compute unit (a block holds most of a CU's LDS)
                    // FP64: 32-pair chunks (the 16-byte values of 32 pairs fill the LDS as 64 do
                    // in FP32), lanes 32..63 idle
                    const int cw = sizeof(R) == 8 ? 32 : p->tune.m2l_chunk;
                    const int64_t nch = (Lv.Kp + cw - 1) / cw;
                    const int64_t nr = std::max<int64_t>(1, std::min<int64_t>(Pv.n, p->n_cu / std::max<int64_t>(nch, 1)));
                    const dim3 grid((unsigned)(nch * nr));
                    auto go = [&](auto kern) {
                        hipLaunchKernelGGL(kern, grid, dim3(kWave * kTW), 0, s, Lv.K, Lv.Kp, (int)nr, Pv.n,
                                           Pv.nb_slots, Pv.child_start, Pv.child_count, Lv.octant, p->m2l_rows,
                                           Lv.pairs, Lv.tperm, (const C*)Lv.transfer, (const C*)Lv.sigM,
                                           (C*)Lv.sigL, Lv.n, nrhs);
                    };
                    if constexpr (sizeof(R) == 8) {
                        go(m2lt_kernel<C, 32, true>);
                    } else {
                        if (cw == 64) go(m2lt_kernel<C, 64, false>);
                        else if (cw == 48) go(m2lt_kernel<C, 48, false>);
                        else go(m2lt_kernel<C, 32, false>);
                    }
                    FFMM_LAUNCH_CHECK();
                    continue;
                }
            }
            if (p->tune.m2l_by_parent) {
                const int rbp = rb >= 2 ? 2 : 1;
                // 128-direction blocks where they leave fewer idle lanes than 256-direction ones
                const bool narrow = (Lv.K + 127) / 128 * 128 < (Lv.K + 255) / 256 * 256;
                const int nth = narrow ? 128 : 256, kc = (Lv.K + nth - 1) / nth;
                const dim3 grid((unsigned)(Pv.n * kc), (nrhs + rbp - 1) / rbp);
                auto go = [&](auto kern) {
                    hipLaunchKernelGGL(kern, grid, dim3(nth), 0, s, Lv.K, kc, Pv.nb_slots, Pv.child_start,
                                       Pv.child_count, Lv.octant, p->code_map, Lv.tperm, (const C*)Lv.transfer,
                                       (const C*)Lv.sigM, (C*)Lv.sigL, Lv.n, nrhs);
                };
                if (rbp == 2)
                    narrow ? go(m2lp_kernel<C, 2, 128>) : go(m2lp_kernel<C, 2, 256>);
                else
                    narrow ? go(m2lp_kernel<C, 1, 128>) : go(m2lp_kernel<C, 1, 256>);
                FFMM_LAUNCH_CHECK();
                continue;
            }
            const unsigned gx = (unsigned)(Lv.n * kch);
            const dim3 grid(gx, (nrhs + rb - 1) / rb);
            if (rb == 4)
                hipLaunchKernelGGL((m2l_kernel<C, 4>), grid, dim3(256), 0, s, Lv.K, kch, Lv.il_ptr,
                                   Lv.il_src, Lv.il_tix, Lv.tperm, (const C*)Lv.transfer,
                                   (const C*)Lv.sigM, (C*)Lv.sigL, Lv.n, nrhs);
            else if (rb == 2)
                hipLaunchKernelGGL((m2l_kernel<C, 2>), grid, dim3(256), 0, s, Lv.K, kch, Lv.il_ptr,
                                   Lv.il_src, Lv.il_tix, Lv.tperm, (const C*)Lv.transfer,
                                   (const C*)Lv.sigM, (C*)Lv.sigL, Lv.n, nrhs);
            else
                hipLaunchKernelGGL((m2l_kernel<C, 1>), grid, dim3(256), 0, s, Lv.K, kch, Lv.il_ptr,
                                   Lv.il_src, Lv.il_tix, Lv.tperm, (const C*)Lv.transfer,
                                   (const C*)Lv.sigM, (C*)Lv.sigL, Lv.n, nrhs);
            FFMM_LAUNCH_CHECK();
        }
        // L2L, l = 2..L-1 (translate on the parent grid, five-step resample, add to I)
        for (int l = 2; l < L; ++l) {
            StageScope sc(p, FFMM_PROF_L2L, s);
            run_resample(p, l, l + 1, nrhs, s);
        }
        // L2P
        StageScope sc(p, FFMM_PROF_L2P, s);
        // right-hand sides sharing each pair's sine/cosine: up to 4 (FP32) or 2 (FP64), one with
        // gradients
        const int nr_l2p = gradient ? 1 : (sizeof(R) == 4 && nrhs >= 4 ? 4 : (nrhs >= 2 ? 2 : 1));
        auto go_l2p = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(nblk(leaf.n, kWpb), (nrhs + nr_l2p - 1) / nr_l2p), dim3(kWave * kWpb),
                               0, s, leaf.Kp, (const R*)leaf.dirs, leaf.pairs, (const R*)leaf.weights, kfac,
                               (R)p->kappa, p->leaf_start, p->leaf_count, (const R*)p->rel,
                               (const C*)leaf.sigL, phis, n, leaf.n, leaf.K, nrhs);
        };
        if (gradient)
            go_l2p(l2p_kernel<R, C, true, 1>);
        else if (nr_l2p == 4) {
            if constexpr (sizeof(R) == 4) go_l2p(l2p_kernel<R, C, false, 4>);
        } else if (nr_l2p == 2)
            go_l2p(l2p_kernel<R, C, false, 2>);
        else
            go_l2p(l2p_kernel<R, C, false, 1>);
        FFMM_LAUNCH_CHECK();
    }
    if (fork) {
        // join: the scatter waits for P2P (and the next call's gather for this P2P's reads of qs)
        FFMM_HIP(hipEventRecord(p->ev_join, p->near_stream));
        FFMM_HIP(hipStreamWaitEvent(s, p->ev_join, 0));
    } else if (stages & FFMM_STAGE_NEAR) {
        launch_p2p(s);
    }
}

template <class R>
void run_matvec_t(ffmm_plan* p, const void* qv, void* outv, int nrhs, int stages, bool conj_io,
                  bool gradient, hipStream_t s)
{
    using C = typename cplx_t<R>::type;
    const int64_t n = p->n;
    gather_t<R>(p, qv, nrhs, conj_io, 0, s);
    core_t<R>(p, nrhs, stages, gradient, s);
    StageScope sc(p, FFMM_PROF_SCATTER, s);
    const bool far = (stages & FFMM_STAGE_FAR) && !p->direct;
    hipLaunchKernelGGL(scatter_out<C>, dim3(nblk(n, 256), nrhs), dim3(256), 0, s,
                       far ? (const C*)p->phis : (const C*)nullptr,
                       (stages & FFMM_STAGE_NEAR) ? (const C*)p->phin : (const C*)nullptr, p->perm, n,
                       gradient ? 3 : 1, conj_io ? 1 : 0, (C*)outv);
    FFMM_LAUNCH_CHECK();
}

// Position gradient: field gradients of q_r and conj(G_r) through the FMM, combined per point.
template <class R>
void run_position_gradient_t(ffmm_plan* p, const void* qv, const void* gv, double* gx, int nrhs,
                             hipStream_t s)
{
    using C = typename cplx_t<R>::type;
    const int64_t n = p->n;
    const C* q = (const C*)qv;
    const C* g = (const C*)gv;
    const C* far = p->direct ? nullptr : (const C*)p->phis;
    const C* near = (const C*)p->phin;
    auto combine = [&](int cnt, int fq_row, int fg_row, int r0, bool accumulate) {
        hipLaunchKernelGGL(posgrad_combine<C>, dim3(nblk(n, 256)), dim3(256), 0, s, far, near, p->perm, n,
                           cnt, fq_row, fg_row, q + (int64_t)r0 * n, g + (int64_t)r0 * n,
                           accumulate ? 1 : 0, gx);
        FFMM_LAUNCH_CHECK();
    };
    const int mr = p->opt.max_rhs;
    if (mr >= 2) {
        // groups of c right-hand sides: rows 0..c-1 hold q_r, rows c..2c-1 conj(G_r)
        const int c = mr / 2;
        for (int r0 = 0; r0 < nrhs; r0 += c) {
            const int cc = std::min(c, nrhs - r0);
            gather_t<R>(p, q + (int64_t)r0 * n, cc, false, 0, s);
            gather_t<R>(p, g + (int64_t)r0 * n, cc, true, cc, s);
            core_t<R>(p, 2 * cc, FFMM_STAGE_ALL, true, s);
            combine(cc, 0, cc, r0, r0 > 0);
        }
        return;
    }
    // one right-hand side of workspace: F(q_r), then F(conj G_r)
    for (int r = 0; r < nrhs; ++r) {
        gather_t<R>(p, q + (int64_t)r * n, 1, false, 0, s);
        core_t<R>(p, 1, FFMM_STAGE_ALL, true, s);
        combine(1, 0, -1, r, r > 0);
        gather_t<R>(p, g + (int64_t)r * n, 1, true, 0, s);
        core_t<R>(p, 1, FFMM_STAGE_ALL, true, s);
        combine(1, -1, 0, r, true);
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

// The FP64 phase table, on the current device (from long-double values rounded once).
void init_cis_table(hipStream_t s)
{
    static const std::vector<double2> tab = [] {
        std::vector<double2> t(256);
        const long double two_pi = 2.0L * std::acos(-1.0L);
        for (int k = 0; k < 256; ++k) {
            const long double a = two_pi * (long double)k / 256.0L;
            t[k] = make_double2((double)std::cos(a), (double)std::sin(a));
        }
        return t;
    }();
    FFMM_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(g_cis256), tab.data(), sizeof(double2) * tab.size(), 0,
                                    hipMemcpyHostToDevice, s));
}

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

void run_position_gradient(ffmm_plan* p, const void* q, const void* g, double* gx, int nrhs, hipStream_t s)
{
    if (p->prec == FFMM_FP32)
        run_position_gradient_t<float>(p, q, g, gx, nrhs, s);
    else
        run_position_gradient_t<double>(p, q, g, gx, nrhs, s);
}

}  // namespace ffmm
