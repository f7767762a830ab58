// Five-step inter/anterpolation between level quadratures (Section 3.4) for the upward (M2M) and
// downward (L2L) passes. Each 1D step applies one real Fourier-resample matrix (the Dirichlet
// kernel with the Nyquist bin dropped) to a batch of boxes, i.e. a dense contraction
//     Y[i][col] = sum_k D[i][k] X[k][col],
// computed with 64 x 64 register/LDS tiles (4 x 4 outputs per thread, 16-deep k slabs). Complex
// data enter as interleaved (re, im) real columns.
//   step 1      per source row n:  G1[c][n][j]  = sum_m D1_n[j][m] in_c(n, m),          j < NA
//   steps 2+3   per column m<NA/2: G2[c][t'][m] = sum_t Dth[t'][t] circ_{c,m}(t)
//               circ_{c,m}(t) = G1[c][t][m] (t <= N_theta/2), G1[c][N_theta - t][m + NA/2] (else),
//               the symmetry F(theta_t, phi_m) = F(theta_{N_theta - t}, phi_{m + NA/2})
//               (eqn. NumSphereSym)
//   steps 4+5   per destination row n': out_c(n', j') = sum_j D5_n'[j'][j] row_{c,n'}(j)
//               row_{c,n'}(j) = G2[c][n'][j] (j < NA/2), G2[c][N'_theta - n'][j - NA/2] (else)
// UP (M2M, Section 2):   in_c = M^l_c; the parent signature is the sum over its children of
//                         E_oct(c) * out_c, summed in LDS over whole parents per tile.
// DOWN (L2L, Section 2): in_c = L^l_parent(c) * conj(E_oct(c)); out_c is added to L^{l+1}_c,
//                         which already holds I^{l+1}_c.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"

namespace ffmm {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;
constexpr int BC = BN / 2;  // complex columns per tile

template <class R> struct cpx;
template <> struct cpx<float> { using type = float2; };
template <> struct cpx<double> { using type = double2; };

// acc[4][4] += A[BM x BK slab] * B[BK x BN slab] from LDS; thread (tr, tc) owns rows 4tr..4tr+3
// and columns 4tc..4tc+3 (two complex columns).
template <class R>
__device__ inline void mma_slab(const R* __restrict__ As, const R* __restrict__ Bs, R (&acc)[4][4],
                                int tr, int tc)
{
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
        R a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = As[kk * BM + tr * 4 + i];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Bs[kk * BN + tc * 4 + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
}

template <class C, class R> __device__ inline void put_complex(R* Bs, int kk, int cc, C v)
{
    Bs[kk * BN + 2 * cc] = v.x;
    Bs[kk * BN + 2 * cc + 1] = v.y;
}

// step 1 -------------------------------------------------------------------------------------
template <class R, bool DOWN>
__global__ __launch_bounds__(NT) void rs1_gemm(int64_t nb, int rows, int NA, int mtiles,
                                               const int32_t* __restrict__ row_off,
                                               const int32_t* __restrict__ nphi,
                                               const R* __restrict__ d1,
                                               const typename cpx<R>::type* __restrict__ sig, int Ksrc,
                                               int64_t nb_in, const int32_t* __restrict__ parent,
                                               const int32_t* __restrict__ octant,
                                               const typename cpx<R>::type* __restrict__ trans,
                                               typename cpx<R>::type* __restrict__ G1)
{
    using C = typename cpx<R>::type;
    __shared__ R As[BK * BM], Bs[BK * BN];
    const int row = blockIdx.y / mtiles, i0 = (blockIdx.y % mtiles) * BM;
    const int64_t r = blockIdx.z;
    if (i0 >= NA) return;
    const int len = nphi[row], off = row_off[row];
    const int64_t c0 = (int64_t)blockIdx.x * BC;
    const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
    R acc[4][4] = {};
    for (int k0 = 0; k0 < len; k0 += BK) {
        for (int e = tid; e < BM * BK; e += NT) {
            const int i = e % BM, kk = e / BM;
            const int k = k0 + kk, ii = i0 + i;
            As[kk * BM + i] = (k < len && ii < NA) ? d1[(int64_t)(off + k) * NA + ii] : R(0);
        }
        for (int e = tid; e < BK * BC; e += NT) {
            const int kk = e % BK, cc = e / BK;
            const int k = k0 + kk;
            const int64_t c = c0 + cc;
            C v;
            v.x = 0;
            v.y = 0;
            if (k < len && c < nb) {
                const int64_t cin = DOWN ? (int64_t)parent[c] : c;
                v = sig[(r * nb_in + cin) * Ksrc + off + k];
                if (DOWN) {
                    const C t = trans[(int64_t)octant[c] * Ksrc + off + k];
                    const R x = v.x * t.x + v.y * t.y, y = v.y * t.x - v.x * t.y;  // v conj(t)
                    v.x = x;
                    v.y = y;
                }
            }
            put_complex(Bs, kk, cc, v);
        }
        __syncthreads();
        mma_slab(As, Bs, acc, tr, tc);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = i0 + tr * 4 + i;
        if (j >= NA) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t c = c0 + tc * 2 + h;
            if (c >= nb) continue;
            C v;
            v.x = acc[i][2 * h];
            v.y = acc[i][2 * h + 1];
            G1[((r * nb + c) * rows + row) * NA + j] = v;
        }
    }
}

// steps 2 + 3 --------------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(NT) void rs3_gemm(int64_t nb, int NA, int rowsS, int ntS, int ntD,
                                               const R* __restrict__ dth,
                                               const typename cpx<R>::type* __restrict__ G1,
                                               typename cpx<R>::type* __restrict__ G2)
{
    using C = typename cpx<R>::type;
    __shared__ R As[BK * BM], Bs[BK * BN];
    const int half = NA / 2;
    const int i0 = blockIdx.y * BM;
    const int64_t r = blockIdx.z;
    const int64_t ncols = nb * half;
    const int64_t g0 = (int64_t)blockIdx.x * BC;
    const int64_t cbase = g0 / half;                 // first (box, column) of the tile
    const int m0 = (int)(g0 - cbase * half);
    const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
    R acc[4][4] = {};
    for (int k0 = 0; k0 < ntS; k0 += BK) {
        for (int e = tid; e < BM * BK; e += NT) {
            const int i = e % BM, kk = e / BM;
            const int t = k0 + kk, tp = i0 + i;
            As[kk * BM + i] = (t < ntS && tp < ntD) ? dth[(int64_t)t * ntD + tp] : R(0);
        }
        for (int e = tid; e < BK * BC; e += NT) {
            const int cc = e % BC, kk = e / BC;
            const int t = k0 + kk;
            C v;
            v.x = 0;
            v.y = 0;
            if (t < ntS && g0 + cc < ncols) {
                int m = m0 + cc;
                int64_t c = cbase;
                while (m >= half) {   // at most BC / half + 1 steps
                    m -= half;
                    ++c;
                }
                const C* base = G1 + (r * nb + c) * rowsS * NA;
                v = (t <= ntS / 2) ? base[(int64_t)t * NA + m] : base[(int64_t)(ntS - t) * NA + m + half];
            }
            put_complex(Bs, kk, cc, v);
        }
        __syncthreads();
        mma_slab(As, Bs, acc, tr, tc);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int tp = i0 + tr * 4 + i;
        if (tp >= ntD) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t g = g0 + tc * 2 + h;
            if (g >= ncols) continue;
            int m = m0 + tc * 2 + h;
            int64_t c = cbase;
            while (m >= half) {
                m -= half;
                ++c;
            }
            C v;
            v.x = acc[i][2 * h];
            v.y = acc[i][2 * h + 1];
            G2[((r * nb + c) * ntD + tp) * half + m] = v;
        }
    }
}

// steps 4 + 5 --------------------------------------------------------------------------------
template <class R, bool UP>
__global__ __launch_bounds__(NT) void rs5_gemm(
    int64_t nb, int NA, int ntD, int mtiles, const int32_t* __restrict__ row_off,
    const int32_t* __restrict__ nphi, const R* __restrict__ d5,
    const typename cpx<R>::type* __restrict__ G2, int Kd, const int32_t* __restrict__ tile_begin,
    const int32_t* __restrict__ tile_end, const int32_t* __restrict__ parent,
    const int32_t* __restrict__ octant, const int32_t* __restrict__ child_start,
    const int32_t* __restrict__ child_count, const typename cpx<R>::type* __restrict__ trans,
    int64_t nb_out, typename cpx<R>::type* __restrict__ out)
{
    using C = typename cpx<R>::type;
    __shared__ R As[BK * BM], Bs[BK * BN];
    __shared__ C S[UP ? BM * BC : 1];
    const int row = blockIdx.y / mtiles, i0 = (blockIdx.y % mtiles) * BM;
    const int64_t r = blockIdx.z;
    const int len = nphi[row], off = row_off[row];
    if (i0 >= len) return;
    int64_t cb, ce;
    if (UP) {
        cb = tile_begin[blockIdx.x];
        ce = tile_end[blockIdx.x];
    } else {
        cb = (int64_t)blockIdx.x * BC;
        ce = min(cb + BC, nb);
    }
    const int half = NA / 2;
    const int tneg = (ntD - row) % ntD;
    const int tid = threadIdx.x, tr = tid / 16, tc = tid % 16;
    const R* D = d5 + (int64_t)off * NA;
    R acc[4][4] = {};
    for (int k0 = 0; k0 < NA; k0 += BK) {
        for (int e = tid; e < BM * BK; e += NT) {
            const int i = e % BM, kk = e / BM;
            const int j = k0 + kk, jp = i0 + i;
            As[kk * BM + i] = (j < NA && jp < len) ? D[(int64_t)j * len + jp] : R(0);
        }
        for (int e = tid; e < BK * BC; e += NT) {
            const int kk = e % BK, cc = e / BK;
            const int j = k0 + kk;
            const int64_t c = cb + cc;
            C v;
            v.x = 0;
            v.y = 0;
            if (j < NA && c < ce) {
                const C* g = G2 + (r * nb + c) * ntD * half;
                v = (j < half) ? g[(int64_t)row * half + j] : g[(int64_t)tneg * half + (j - half)];
            }
            put_complex(Bs, kk, cc, v);
        }
        __syncthreads();
        mma_slab(As, Bs, acc, tr, tc);
        __syncthreads();
    }
    if (!UP) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int jp = i0 + tr * 4 + i;
            if (jp >= len) continue;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t c = cb + tc * 2 + h;
                if (c >= ce) continue;
                C& o = out[(r * nb_out + c) * Kd + off + jp];
                o.x += acc[i][2 * h];
                o.y += acc[i][2 * h + 1];
            }
        }
        return;
    }
    // UP: translate each child on the parent grid, then sum the children of every parent
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int jp = i0 + tr * 4 + i;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int cc = tc * 2 + h;
            const int64_t c = cb + cc;
            C v;
            v.x = 0;
            v.y = 0;
            if (jp < len && c < ce) {
                const C t = trans[(int64_t)octant[c] * Kd + off + jp];
                const R x = acc[i][2 * h], y = acc[i][2 * h + 1];
                v.x = x * t.x - y * t.y;
                v.y = x * t.y + y * t.x;
            }
            S[(tr * 4 + i) * BC + cc] = v;
        }
    }
    __syncthreads();
    const int64_t p0 = parent[cb], p1 = parent[ce - 1];
    const int npar = (int)(p1 - p0 + 1);
    for (int e = tid; e < BM * npar; e += NT) {
        const int i = e % BM, pi = e / BM;
        const int jp = i0 + i;
        if (jp >= len) continue;
        const int64_t pp = p0 + pi;
        const int64_t a = child_start[pp], bcount = child_count[pp];
        C sum;
        sum.x = 0;
        sum.y = 0;
        for (int64_t c = a; c < a + bcount; ++c) {
            const C v = S[i * BC + (int)(c - cb)];
            sum.x += v.x;
            sum.y += v.y;
        }
        out[(r * nb_out + pp) * Kd + off + jp] = sum;
    }
}

// ---- FP32 on the matrix cores ------------------------------------------------------------------
// The same three contractions with v_mfma_f32_32x32x2f32 (FP32 products and sums, so the results
// carry the same rounding model as the vector path). Operand lanes: A[i][k] and B[k][j] with
// i, j = lane % 32 and k = lane / 32; result register q of a lane holds row
// (q / 4) * 8 + (lane / 32) * 4 + q % 4 and column lane % 32 of the 32 x 32 tile.
// A block is four waves on a 64 x 64 tile (each wave a 32 x 32 quadrant), with 16-deep k slabs
// double-buffered in LDS (one barrier per slab).
//   steps 1 and 5: rows are (box, re/im) pairs, columns the output samples of one row, so the
//                  two registers q = 2p, 2p + 1 of a lane hold the (re, im) of one output and a
//                  wave stores 32 consecutive complex samples;
//   steps 2 + 3:   rows are the output theta_t', columns (box, phi_m, re/im).
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MM = 64, MN = 64, MK = 16;
constexpr int MAP = MM + 2;   // LDS row stride of the A slab (conflict-free 8-byte stores)
constexpr int MBP = MN;       // LDS row stride of the B slab

__device__ inline void mfma_slab(const float* __restrict__ As, const float* __restrict__ Bs, f32x16& acc,
                                 int wr, int wc, int lane)
{
    const int i = lane & 31, kh = lane >> 5;
#pragma unroll
    for (int kk = 0; kk < MK; kk += 2) {
        const float a = As[(kk + kh) * MAP + wr + i];
        const float b = Bs[(kk + kh) * MBP + wc + i];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
}

// box (0..31 within the block tile) of result pair p (registers 2p, 2p + 1) of this lane
__device__ inline int pair_box(int wr, int lane, int p) { return wr / 2 + (p >> 1) * 4 + (lane >> 5) * 2 + (p & 1); }

template <bool DOWN>
__global__ __launch_bounds__(NT) void rs1_mfma(int64_t nb, int rows, int NA, int ntj,
                                               const int32_t* __restrict__ row_off,
                                               const int32_t* __restrict__ nphi,
                                               const float* __restrict__ d1,
                                               const float2* __restrict__ sig, int Ksrc, int64_t nb_in,
                                               const int32_t* __restrict__ parent,
                                               const int32_t* __restrict__ octant,
                                               const float2* __restrict__ trans, float2* __restrict__ G1)
{
    __shared__ __align__(16) float As[2][MK * MAP];
    __shared__ __align__(16) float Bs[2][MK * MBP];
    const int row = blockIdx.y / ntj, j0 = (blockIdx.y % ntj) * MN;
    const int64_t r = blockIdx.z;
    const int len = nphi[row], off = row_off[row];
    const int64_t c0 = (int64_t)blockIdx.x * (MM / 2);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    float2 ra[2];
    float4 rb;
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + NT * q, kk = e & (MK - 1), bc = e >> 4;
            const int k = k0 + kk;
            const int64_t c = c0 + bc;
            float2 v = make_float2(0.f, 0.f);
            if (k < len && c < nb) {
                const int64_t cin = DOWN ? (int64_t)parent[c] : c;
                v = sig[(r * nb_in + cin) * Ksrc + off + k];
                if (DOWN) {
                    const float2 t = trans[(int64_t)octant[c] * Ksrc + off + k];
                    v = make_float2(v.x * t.x + v.y * t.y, v.y * t.x - v.x * t.y);  // v conj(t)
                }
            }
            ra[q] = v;
        }
        const int k = k0 + (tid >> 4), j = j0 + 4 * (tid & 15);
        rb = (k < len && j < NA) ? *(const float4*)(d1 + (int64_t)(off + k) * NA + j)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + NT * q;
            *(float2*)&As[buf][(e & (MK - 1)) * MAP + 2 * (e >> 4)] = ra[q];
        }
        *(float4*)&Bs[buf][(tid >> 4) * MBP + 4 * (tid & 15)] = rb;
    };
    f32x16 acc = {};
    const int nslab = (len + MK - 1) / MK;
    load(0);
    store(0);
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        if (sl + 1 < nslab) load((sl + 1) * MK);
        mfma_slab(As[sl & 1], Bs[sl & 1], acc, wr, wc, lane);
        if (sl + 1 < nslab) store((sl + 1) & 1);
        __syncthreads();
    }
    const int j = j0 + wc + (lane & 31);
    if (j >= NA) return;
#pragma unroll
    for (int pq = 0; pq < 8; ++pq) {
        const int64_t c = c0 + pair_box(wr, lane, pq);
        if (c < nb) G1[((r * nb + c) * rows + row) * NA + j] = make_float2(acc[2 * pq], acc[2 * pq + 1]);
    }
}

__global__ __launch_bounds__(NT) void rs3_mfma(int64_t nb, int NA, int rowsS, int ntS, int ntD,
                                               const float* __restrict__ dth,
                                               const float2* __restrict__ G1, float2* __restrict__ G2)
{
    __shared__ __align__(16) float As[2][MK * MAP];
    __shared__ __align__(16) float Bs[2][MK * MBP];
    const int half = NA / 2;
    const int i0 = blockIdx.y * MM;
    const int64_t r = blockIdx.z;
    const int64_t ncols = nb * half;
    const int64_t g0 = (int64_t)blockIdx.x * (MN / 2);
    const int64_t cbase = g0 / half;   // first (box, column) of the tile
    const int m0 = (int)(g0 - cbase * half);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    // this thread's two staged columns never change: resolve (box, phi index) once
    int64_t scol[2];
    int sm[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int cc = (tid + NT * q) & 31;
        int m = m0 + cc;
        int64_t c = cbase;
        while (m >= half) {
            m -= half;
            ++c;
        }
        scol[q] = c;
        sm[q] = m;
    }
    float ra[4];
    float2 rbv[2];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + NT * q, i = e & 63, kk = e >> 6;
            const int t = k0 + kk, tp = i0 + i;
            ra[q] = (t < ntS && tp < ntD) ? dth[(int64_t)t * ntD + tp] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + NT * q, cc = e & 31, kk = e >> 5;
            const int t = k0 + kk;
            float2 v = make_float2(0.f, 0.f);
            if (t < ntS && g0 + cc < ncols) {
                const float2* base = G1 + (r * nb + scol[q]) * rowsS * NA;
                v = (t <= ntS / 2) ? base[(int64_t)t * NA + sm[q]]
                                   : base[(int64_t)(ntS - t) * NA + sm[q] + half];
            }
            rbv[q] = v;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + NT * q;
            As[buf][(e >> 6) * MAP + (e & 63)] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + NT * q;
            *(float2*)&Bs[buf][(e >> 5) * MBP + 2 * (e & 31)] = rbv[q];
        }
    };
    f32x16 acc = {};
    const int nslab = (ntS + MK - 1) / MK;
    load(0);
    store(0);
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        if (sl + 1 < nslab) load((sl + 1) * MK);
        mfma_slab(As[sl & 1], Bs[sl & 1], acc, wr, wc, lane);
        if (sl + 1 < nslab) store((sl + 1) & 1);
        __syncthreads();
    }
    const int col = wc + (lane & 31), cc = col >> 1, part = col & 1;
    if (g0 + cc >= ncols) return;
    int m = m0 + cc;
    int64_t c = cbase;
    while (m >= half) {
        m -= half;
        ++c;
    }
    float* base = (float*)(G2 + (r * nb + c) * ntD * half + m) + part;
    const int h = lane >> 5;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int tp = i0 + wr + (q >> 2) * 8 + h * 4 + (q & 3);
        if (tp < ntD) base[(int64_t)tp * half * 2] = acc[q];
    }
}

template <bool UP>
__global__ __launch_bounds__(NT) void rs5_mfma(
    int64_t nb, int NA, int ntD, int ntj, const int32_t* __restrict__ row_off,
    const int32_t* __restrict__ nphi, const float* __restrict__ d5, const float2* __restrict__ G2, int Kd,
    const int32_t* __restrict__ tile_begin, const int32_t* __restrict__ tile_end,
    const int32_t* __restrict__ parent, const int32_t* __restrict__ octant,
    const int32_t* __restrict__ child_start, const int32_t* __restrict__ child_count,
    const float2* __restrict__ trans, int64_t nb_out, float2* __restrict__ out)
{
    __shared__ __align__(16) float As[2][MK * MAP];
    __shared__ __align__(16) float Bs[2][MK * MBP];
    __shared__ float2 S[UP ? (MM / 2) * MN : 1];
    const int row = blockIdx.y / ntj, j0 = (blockIdx.y % ntj) * MN;
    const int64_t r = blockIdx.z;
    const int len = nphi[row], off = row_off[row];
    if (j0 >= len) return;
    int64_t cb, ce;
    if (UP) {
        cb = tile_begin[blockIdx.x];
        ce = tile_end[blockIdx.x];
    } else {
        cb = (int64_t)blockIdx.x * (MM / 2);
        ce = min(cb + MM / 2, nb);
    }
    const int half = NA / 2;
    const int tneg = (ntD - row) % ntD;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const float* D = d5 + (int64_t)off * NA;
    float2 ra[2];
    float4 rb;
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + NT * q, kk = e & (MK - 1), bc = e >> 4;
            const int j = k0 + kk;
            const int64_t c = cb + bc;
            float2 v = make_float2(0.f, 0.f);
            if (j < NA && c < ce) {
                const float2* g = G2 + (r * nb + c) * ntD * half;
                v = (j < half) ? g[(int64_t)row * half + j] : g[(int64_t)tneg * half + (j - half)];
            }
            ra[q] = v;
        }
        const int j = k0 + (tid >> 4), jp = j0 + 4 * (tid & 15);
        rb = (j < NA && jp < len) ? *(const float4*)(D + (int64_t)j * len + jp)
                                  : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + NT * q;
            *(float2*)&As[buf][(e & (MK - 1)) * MAP + 2 * (e >> 4)] = ra[q];
        }
        *(float4*)&Bs[buf][(tid >> 4) * MBP + 4 * (tid & 15)] = rb;
    };
    f32x16 acc = {};
    const int nslab = (NA + MK - 1) / MK;
    load(0);
    store(0);
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        if (sl + 1 < nslab) load((sl + 1) * MK);
        mfma_slab(As[sl & 1], Bs[sl & 1], acc, wr, wc, lane);
        if (sl + 1 < nslab) store((sl + 1) & 1);
        __syncthreads();
    }
    const int colw = wc + (lane & 31);
    const int jp = j0 + colw;
    if (!UP) {
        if (jp >= len) return;
#pragma unroll
        for (int pq = 0; pq < 8; ++pq) {
            const int64_t c = cb + pair_box(wr, lane, pq);
            if (c >= ce) continue;
            float2& o = out[(r * nb_out + c) * Kd + off + jp];
            o.x += acc[2 * pq];
            o.y += acc[2 * pq + 1];
        }
        return;
    }
    // UP: translate each child on the parent grid, then sum the children of every parent
#pragma unroll
    for (int pq = 0; pq < 8; ++pq) {
        const int bx = pair_box(wr, lane, pq);
        const int64_t c = cb + bx;
        float2 v = make_float2(0.f, 0.f);
        if (jp < len && c < ce) {
            const float2 t = trans[(int64_t)octant[c] * Kd + off + jp];
            const float x = acc[2 * pq], y = acc[2 * pq + 1];
            v = make_float2(x * t.x - y * t.y, x * t.y + y * t.x);
        }
        S[bx * MN + colw] = v;
    }
    __syncthreads();
    const int64_t p0 = parent[cb], p1 = parent[ce - 1];
    const int npar = (int)(p1 - p0 + 1);
    for (int e = tid; e < MN * npar; e += NT) {
        const int i = e % MN, pi = e / MN;
        const int jj = j0 + i;
        if (jj >= len) continue;
        const int64_t pp = p0 + pi;
        const int64_t a = child_start[pp], cnt = child_count[pp];
        float2 sum = make_float2(0.f, 0.f);
        for (int64_t c = a; c < a + cnt; ++c) {
            const float2 v = S[(int)(c - cb) * MN + i];
            sum.x += v.x;
            sum.y += v.y;
        }
        out[(r * nb_out + pp) * Kd + off + jj] = sum;
    }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <class R>
void run_resample_t(ffmm_plan* p, int l_src, int l_dst, int nrhs, hipStream_t s)
{
    const bool up = l_dst == l_src - 1;
    Resampler& rs = up ? p->up[l_src] : p->down[l_src];
    LevelData& S = p->lev[l_src];
    LevelData& D = p->lev[l_dst];
    LevelData& Cl = up ? S : D;   // the child level: one resample per child box
    using C = typename cpx<R>::type;
    C* G1 = (C*)p->scratch1;
    C* G2 = (C*)p->scratch2;
    const int NA = rs.nphi_all;
    const int64_t nb = Cl.n;
    // step 1 (per source row)
    {
        const int mt = cdiv(NA, BM);
        dim3 grid(cdiv(nb, BC), mt * rs.rows_src, nrhs);
        if (up)
            hipLaunchKernelGGL((rs1_gemm<R, false>), grid, dim3(NT), 0, s, nb, rs.rows_src, NA, mt,
                               rs.d_src_row_off, rs.d_src_nphi, (const R*)rs.d1, (const C*)S.sigM, S.K,
                               S.n, (const int32_t*)nullptr, (const int32_t*)nullptr,
                               (const C*)nullptr, G1);
        else
            hipLaunchKernelGGL((rs1_gemm<R, true>), grid, dim3(NT), 0, s, nb, rs.rows_src, NA, mt,
                               rs.d_src_row_off, rs.d_src_nphi, (const R*)rs.d1, (const C*)S.sigL, S.K,
                               S.n, Cl.parent, Cl.octant, (const C*)S.trans, G1);
        FFMM_LAUNCH_CHECK();
    }
    // steps 2 + 3
    {
        dim3 grid(cdiv(nb * (NA / 2), BC), cdiv(rs.nt_dst, BM), nrhs);
        hipLaunchKernelGGL((rs3_gemm<R>), grid, dim3(NT), 0, s, nb, NA, rs.rows_src, rs.nt_src,
                           rs.nt_dst, (const R*)rs.dth, (const C*)G1, G2);
        FFMM_LAUNCH_CHECK();
    }
    // steps 4 + 5
    {
        int mx = 0;
        for (int v : D.par.nphi) mx = std::max(mx, v);
        const int mt = cdiv(mx, BM);
        if (up) {
            dim3 grid((unsigned)rs.ntiles, mt * rs.rows_dst, nrhs);
            hipLaunchKernelGGL((rs5_gemm<R, true>), grid, dim3(NT), 0, s, nb, NA, rs.nt_dst, mt,
                               rs.d_dst_row_off, rs.d_dst_nphi, (const R*)rs.d5, (const C*)G2, D.K,
                               rs.tile_begin, rs.tile_end, Cl.parent, Cl.octant, D.child_start,
                               D.child_count, (const C*)D.trans, D.n, (C*)D.sigM);
        } else {
            dim3 grid(cdiv(nb, BC), mt * rs.rows_dst, nrhs);
            hipLaunchKernelGGL((rs5_gemm<R, false>), grid, dim3(NT), 0, s, nb, NA, rs.nt_dst, mt,
                               rs.d_dst_row_off, rs.d_dst_nphi, (const R*)rs.d5, (const C*)G2, D.K,
                               (const int32_t*)nullptr, (const int32_t*)nullptr,
                               (const int32_t*)nullptr, (const int32_t*)nullptr,
                               (const int32_t*)nullptr, (const int32_t*)nullptr, (const C*)nullptr,
                               D.n, (C*)D.sigL);
        }
        FFMM_LAUNCH_CHECK();
    }
}

}  // namespace

// Child tiles of the upward pass: consecutive whole parents, at most 32 children per tile (the
// box rows of one tile of either resample path).
void make_parent_tiles(const std::vector<int32_t>& child_count, std::vector<int32_t>& begin,
                       std::vector<int32_t>& end)
{
    begin.clear();
    end.clear();
    int32_t c = 0, tb = 0, in_tile = 0;
    for (size_t pidx = 0; pidx < child_count.size(); ++pidx) {
        const int32_t k = child_count[pidx];
        if (in_tile + k > BC) {
            begin.push_back(tb);
            end.push_back(c);
            tb = c;
            in_tile = 0;
        }
        c += k;
        in_tile += k;
    }
    if (in_tile > 0) {
        begin.push_back(tb);
        end.push_back(c);
    }
}

namespace {

void run_resample_mfma(ffmm_plan* p, int l_src, int l_dst, int nrhs, hipStream_t s)
{
    const bool up = l_dst == l_src - 1;
    Resampler& rs = up ? p->up[l_src] : p->down[l_src];
    LevelData& S = p->lev[l_src];
    LevelData& D = p->lev[l_dst];
    LevelData& Cl = up ? S : D;
    float2* G1 = (float2*)p->scratch1;
    float2* G2 = (float2*)p->scratch2;
    const int NA = rs.nphi_all;
    const int64_t nb = Cl.n;
    {
        const int ntj = cdiv(NA, MN);
        dim3 grid(cdiv(nb, MM / 2), ntj * rs.rows_src, nrhs);
        if (up)
            hipLaunchKernelGGL((rs1_mfma<false>), grid, dim3(NT), 0, s, nb, rs.rows_src, NA, ntj,
                               rs.d_src_row_off, rs.d_src_nphi, (const float*)rs.d1,
                               (const float2*)S.sigM, S.K, S.n, (const int32_t*)nullptr,
                               (const int32_t*)nullptr, (const float2*)nullptr, G1);
        else
            hipLaunchKernelGGL((rs1_mfma<true>), grid, dim3(NT), 0, s, nb, rs.rows_src, NA, ntj,
                               rs.d_src_row_off, rs.d_src_nphi, (const float*)rs.d1,
                               (const float2*)S.sigL, S.K, S.n, Cl.parent, Cl.octant,
                               (const float2*)S.trans, G1);
        FFMM_LAUNCH_CHECK();
    }
    {
        dim3 grid(cdiv(nb * (NA / 2), MN / 2), cdiv(rs.nt_dst, MM), nrhs);
        hipLaunchKernelGGL(rs3_mfma, grid, dim3(NT), 0, s, nb, NA, rs.rows_src, rs.nt_src, rs.nt_dst,
                           (const float*)rs.dth, (const float2*)G1, G2);
        FFMM_LAUNCH_CHECK();
    }
    {
        int mx = 0;
        for (int v : D.par.nphi) mx = std::max(mx, v);
        const int ntj = cdiv(mx, MN);
        if (up) {
            dim3 grid((unsigned)rs.ntiles, ntj * rs.rows_dst, nrhs);
            hipLaunchKernelGGL((rs5_mfma<true>), grid, dim3(NT), 0, s, nb, NA, rs.nt_dst, ntj,
                               rs.d_dst_row_off, rs.d_dst_nphi, (const float*)rs.d5, (const float2*)G2,
                               D.K, rs.tile_begin, rs.tile_end, Cl.parent, Cl.octant, D.child_start,
                               D.child_count, (const float2*)D.trans, D.n, (float2*)D.sigM);
        } else {
            dim3 grid(cdiv(nb, MM / 2), ntj * rs.rows_dst, nrhs);
            hipLaunchKernelGGL((rs5_mfma<false>), grid, dim3(NT), 0, s, nb, NA, rs.nt_dst, ntj,
                               rs.d_dst_row_off, rs.d_dst_nphi, (const float*)rs.d5, (const float2*)G2,
                               D.K, (const int32_t*)nullptr, (const int32_t*)nullptr,
                               (const int32_t*)nullptr, (const int32_t*)nullptr,
                               (const int32_t*)nullptr, (const int32_t*)nullptr,
                               (const float2*)nullptr, D.n, (float2*)D.sigL);
        }
        FFMM_LAUNCH_CHECK();
    }
}

}  // namespace

void run_resample(ffmm_plan* p, int l_src, int l_dst, int nrhs, hipStream_t s)
{
    if (p->prec == FFMM_FP32)
        run_resample_mfma(p, l_src, l_dst, nrhs, s);
    else
        run_resample_t<double>(p, l_src, l_dst, nrhs, s);
}

}  // namespace ffmm
