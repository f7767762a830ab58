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
                                               int ldth, const R* __restrict__ dth,
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
            As[kk * BM + i] = (t < ntS && tp < ntD) ? dth[(int64_t)t * ldth + tp] : R(0);
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
// A block is four waves on a 64 x 64 tile (each wave a 32 x 32 quadrant). The contraction runs in
// KS-deep k slabs staged in LDS (KS = 16, 32 or 64 per kernel: deeper slabs keep more of a
// block's data in flight, shallower ones waste less on short rows and allow more blocks per CU).
//   steps 1 and 5: rows are (box, re/im) pairs, columns the output samples of one row, so the
//                  two registers q = 2p, 2p + 1 of a lane hold the (re, im) of one output and a
//                  wave stores 32 consecutive complex samples;
//   steps 2 + 3:   rows are the output theta_t', columns (box, phi_m, re/im).
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MM = 64, MN = 64;
constexpr int MAP = MM + 4;   // LDS row stride of the A slab (rows stay 16-byte aligned)
constexpr int MBP = MN;       // LDS row stride of the B slab

// acc += A[:, 0:kc] B[0:kc, :] for this wave's quadrant; kc is block-uniform, slab rows >= kc
// hold zeros up to the next multiple of 8 (kc <= KS)
__device__ inline void mfma_slab(const float* __restrict__ As, const float* __restrict__ Bs, f32x16& acc,
                                 int wr, int wc, int lane, int kc)
{
    const int i = lane & 31, kh = lane >> 5;
    for (int k8 = 0; k8 < kc; k8 += 8) {
        float a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = As[(k8 + 2 * u + kh) * MAP + wr + i];
            b[u] = Bs[(k8 + 2 * u + kh) * MBP + wc + i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u], b[u], acc, 0, 0, 0);
    }
}

// box (0..31 within the block tile) of result pair p (registers 2p, 2p + 1) of this lane
__device__ inline int pair_box(int wr, int lane, int p) { return wr / 2 + (p >> 1) * 4 + (lane >> 5) * 2 + (p & 1); }

// Shared main loop over one LDS slab buffer. Stage::load(k0) issues the global loads of the slab
// starting at k0 into registers; Stage::store(As, Bs) writes them (zeroing invalid entries) once
// they have landed. The next slab's loads are in flight during the current slab's MFMAs.
template <int KS, class Stage>
__device__ inline void mfma_mainloop(Stage& st, float* As, float* Bs, int K, f32x16& acc, int wr, int wc,
                                     int lane)
{
    const int nslab = (K + KS - 1) / KS;
    st.load(0);
    st.store(As, Bs);
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        const bool more = sl + 1 < nslab;
        if (more) st.load((sl + 1) * KS);
        const int kc = min(KS, K - sl * KS);
        mfma_slab(As, Bs, acc, wr, wc, lane, (kc + 7) & ~7);
        if (more) {
            __syncthreads();   // every wave is done with this slab
            st.store(As, Bs);
        }
        __syncthreads();
    }
}

// step 1 staging: A = source row data of 32 boxes, or in the downward pass of 32 z pairs (lo, hi)
// of children: the parent's data times conj(E_oct(lo)); hi's input differs from lo's by the factor
// conj(rho(n)), constant on the source row n, so step 1 runs once per pair. B = the Dirichlet
// block of the row.
template <bool DOWN, int KS> struct Rs1Stage {
    int tid, len, NA, j0;
    int64_t c0, nb;
    const float* d1;
    int off;
    static constexpr int QA = KS / 8, QB = KS / 16, QT = DOWN ? QA : 1;
    // source row n of this thread's tile rows (fixed over the slabs), and downward the row of
    // the translation of lo's octant
    const float2* gs[QA];
    const float2* gt[QT];
    // load() only issues the loads; store() applies conj(E) once they have landed, so that the
    // next slab's loads stay in flight during the current slab's MFMAs
    float2 ra[QA], rt[QT];
    float4 rb[QB];
    bool oka[QA], okb[QB];
    __device__ void init(const float2* sig, int Ksrc, int64_t nb_in, int64_t r, const int32_t* zpar,
                         const int32_t* zoct, const float2* trans)
    {
        const uint32_t rb0 = (uint32_t)(r * nb_in);
        int bi[QA], oi[QA];
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int64_t c = min(c0 + (tid + NT * q) / KS, nb - 1);
            bi[q] = DOWN ? zpar[c] : (int)c;
            if (DOWN) oi[q] = zoct[c];
        }
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            gs[q] = sig + off + (uint64_t)(rb0 + (uint32_t)bi[q]) * (uint32_t)Ksrc;
            if (DOWN) gt[q] = trans + off + (uint32_t)oi[q] * (uint32_t)Ksrc;
        }
    }
    __device__ void load(int k0)
    {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q, kk = e % KS, bc = e / KS;
            const int k = min(k0 + kk, len - 1);
            ra[q] = gs[q][k];
            if (DOWN) rt[q] = gt[q][k];
            oka[q] = k0 + kk < len && c0 + bc < nb;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q, kr = k0 + (e >> 4), j = j0 + 4 * (e & 15);
            rb[q] = *(const float4*)(d1 + (int64_t)(off + min(kr, len - 1)) * NA + (j < NA ? j : 0));
            okb[q] = kr < len && j < NA;
        }
    }
    __device__ void store(float* As, float* Bs)
    {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            float2 v = ra[q];
            if (DOWN) {
                const float2 t = rt[q];
                v = make_float2(v.x * t.x + v.y * t.y, v.y * t.x - v.x * t.y);  // v conj(t)
            }
            const bool ok = oka[q];
            *(float2*)&As[(e % KS) * MAP + 2 * (e / KS)] = make_float2(ok ? v.x : 0.f, ok ? v.y : 0.f);
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q;
            const float4 v = rb[q];
            const bool ok = okb[q];
            *(float4*)&Bs[(e >> 4) * MBP + 4 * (e & 15)] =
                make_float4(ok ? v.x : 0.f, ok ? v.y : 0.f, ok ? v.z : 0.f, ok ? v.w : 0.f);
        }
    }
};

// nt: the tile rows (boxes, or z pairs in the downward pass); nb: the boxes of the G1 layout
template <bool DOWN, int KS>
__global__ __launch_bounds__(NT) void rs1_mfma(int64_t nt, int64_t nb, int rows, int NA, int ntj,
                                               const int32_t* __restrict__ row_off,
                                               const int32_t* __restrict__ nphi,
                                               const float* __restrict__ d1,
                                               const float2* __restrict__ sig, int Ksrc, int64_t nb_in,
                                               const int32_t* __restrict__ zpar,
                                               const int32_t* __restrict__ zoct,
                                               const int32_t* __restrict__ zlo,
                                               const int32_t* __restrict__ zhi,
                                               const float2* __restrict__ zrot,
                                               const float2* __restrict__ trans, float2* __restrict__ G1)
{
    const int row = blockIdx.y / ntj, j0 = (blockIdx.y % ntj) * MN;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    __shared__ __align__(16) float As[KS * MAP];
    __shared__ __align__(16) float Bs[KS * MBP];
    Rs1Stage<DOWN, KS> st;
    st.tid = tid;
    st.len = nphi[row];
    st.off = row_off[row];
    st.NA = NA;
    st.j0 = j0;
    st.c0 = (int64_t)blockIdx.x * (MM / 2);
    st.nb = nt;
    st.d1 = d1;
    st.init(sig, Ksrc, nb_in, blockIdx.z, zpar, zoct, trans);
    f32x16 acc = {};
    mfma_mainloop<KS>(st, As, Bs, st.len, acc, wr, wc, lane);
    const int j = j0 + wc + (lane & 31);
    if (j >= NA) return;
    const uint32_t rb0 = (uint32_t)(blockIdx.z * nb), bs = (uint32_t)rows * NA;   // box stride
    float2* g = G1 + (int64_t)row * NA + j;
    if (!DOWN) {
#pragma unroll
        for (int pq = 0; pq < 8; ++pq) {
            const int64_t c = st.c0 + pair_box(wr, lane, pq);
            if (c < nt) g[(uint64_t)(rb0 + (uint32_t)c) * bs] = make_float2(acc[2 * pq], acc[2 * pq + 1]);
        }
        return;
    }
    // lo's result as computed, hi's times conj(rho(n)); the pair indices are loaded first
    const float2 z = zrot[row];
    int lo[8], hi[8];
#pragma unroll
    for (int pq = 0; pq < 8; ++pq) {
        const int64_t c = min(st.c0 + pair_box(wr, lane, pq), nt - 1);
        lo[pq] = zlo[c];
        hi[pq] = zhi[c];
    }
#pragma unroll
    for (int pq = 0; pq < 8; ++pq) {
        if (st.c0 + pair_box(wr, lane, pq) >= nt) continue;
        const float x = acc[2 * pq], y = acc[2 * pq + 1];
        g[(uint64_t)(rb0 + (uint32_t)lo[pq]) * bs] = make_float2(x, y);
        if (hi[pq] >= 0)
            g[(uint64_t)(rb0 + (uint32_t)hi[pq]) * bs] = make_float2(x * z.x + y * z.y, y * z.x - x * z.y);
    }
}

// steps 2 + 3 on half ranges (eqn. FourierSphereSym): per phi column m < NPhi/2 the source rows
// 0..N_theta/2 split into u = F_m + F_{m + NPhi/2} (even phi modes, even in theta) and
// v = F_m - F_{m + NPhi/2} (odd modes, odd in theta); the theta step is then two half-range
// contractions u' = De^T u, v' = Do^T v (De, Do carry the factor 1/2) onto the destination rows
// 0..N'_theta/2, where F'_m = u' + v', F'_{m + NPhi/2} = u' - v' (formed by steps 4 + 5). Half the
// work of resampling the full theta circle. A block tile stacks 32 rows t' of De (the waves on
// tile rows 0..31, which read u) over the same 32 rows of Do (tile rows 32..63, which read v).
// G2 of the FP32 path: [rhs][box][N'_theta/2 + 1][2][NPhi/2] complex: u' then v' of each row.
// dh holds De then Do, each [N_theta/2 + 1][ldh].
template <int KS>
__global__ __launch_bounds__(NT) void rs3h_mfma(int64_t nb, int NA, int rowsS, int ntSh, int ntDh,
                                                int ldh, const float* __restrict__ dh,
                                                const float2* __restrict__ G1, float2* __restrict__ G2)
{
    constexpr int QA = KS / 16, QB = KS / 8;
    __shared__ __align__(16) float As[KS * MAP];
    __shared__ __align__(16) float Bs[2 * KS * MBP];
    const int half = NA / 2;
    const int i0 = blockIdx.y * (MM / 2);
    const int64_t r = blockIdx.z;
    const int64_t ncols = nb * half;
    const int64_t g0 = (int64_t)blockIdx.x * (MN / 2);
    const int64_t cbase = g0 / half;   // first (box, column) of the tile
    const int m0 = (int)(g0 - cbase * half);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const bool odd = wr != 0;
    const int64_t mat_off = (int64_t)ntSh * ldh;   // Do after De
    // this thread's staged column (phi_m of its box), row 0
    const float2* sbase;
    bool scol_ok;
    {
        const int cc = tid & 31;
        int m = m0 + cc;
        int64_t c = cbase;
        while (m >= half) {
            m -= half;
            ++c;
        }
        scol_ok = g0 + cc < ncols;
        sbase = scol_ok ? G1 + (r * nb + c) * rowsS * NA + m : G1;
    }
    float4 ra[QA];
    float4 rab[QB];   // (F_m, F_{m + NPhi/2}) of each staged row
    bool oka[QA], okb[QB];
    auto load = [&](int k0) {
        // A tile column c4: 0..31 are De rows i0.., 32..63 the same rows of Do
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q, t = k0 + (e >> 4), c4 = 4 * (e & 15);
            const int tp = i0 + (c4 & 31);
            const bool ok = t < ntSh && tp < ldh;
            const int64_t idx = ok ? (c4 >= 32 ? mat_off : 0) + (int64_t)t * ldh + tp : 0;
            ra[q] = *(const float4*)(dh + idx);
            oka[q] = ok;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int tt = k0 + (tid >> 5) + 8 * q;
            const int64_t row = (int64_t)min(tt, ntSh - 1) * NA;
            const float2 a = sbase[row], b = sbase[row + half];
            rab[q] = make_float4(a.x, a.y, b.x, b.y);
            okb[q] = tt < ntSh && scol_ok;
        }
    };
    // invalid entries become zeros component by component (a select of whole vectors makes the
    // compiler stage them through private memory)
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            const float4 v = ra[q];
            const bool ok = oka[q];
            *(float4*)&As[(e >> 4) * MAP + 4 * (e & 15)] =
                make_float4(ok ? v.x : 0.f, ok ? v.y : 0.f, ok ? v.z : 0.f, ok ? v.w : 0.f);
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int o = ((tid >> 5) + 8 * q) * MBP + 2 * (tid & 31);
            const float4 ab = rab[q];
            const bool ok = okb[q];
            *(float2*)&Bs[o] = make_float2(ok ? ab.x + ab.z : 0.f, ok ? ab.y + ab.w : 0.f);
            *(float2*)&Bs[KS * MBP + o] = make_float2(ok ? ab.x - ab.z : 0.f, ok ? ab.y - ab.w : 0.f);
        }
    };
    f32x16 acc = {};
    const int nslab = (ntSh + KS - 1) / KS;
    load(0);
    store();
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        const bool more = sl + 1 < nslab;
        if (more) load((sl + 1) * KS);
        const int kc = (min(KS, ntSh - sl * KS) + 7) & ~7;
        mfma_slab(As, Bs + (odd ? KS * MBP : 0), acc, wr, wc, lane, kc);
        if (more) {
            __syncthreads();
            store();
        }
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
    float* base = (float*)(G2 + ((r * nb + c) * ntDh * 2 + (odd ? 1 : 0)) * half + m) + part;
    const int h = lane >> 5;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int tp = i0 + (q >> 2) * 8 + h * 4 + (q & 3);
        if (tp < ntDh) base[(int64_t)tp * 2 * half * 2] = acc[q];
    }
}

// steps 4 + 5 staging: A = the destination row's samples on the common phi grid (row n' of the
// half-range theta output), B = the Dirichlet block of the destination row. In the upward pass a
// tile row is a z pair (lo, hi) of children: row(lo) + rho * row(hi), rho = e^{i kappa cos(theta_n')
// a_child} (the translations of the two differ by this factor on row n', which step 5 does not
// mix), so that step 5 runs once per pair and the pair's sum is translated with lo's octant.
template <bool UP, int KS> struct Rs5Stage {
    static constexpr int QA = KS / 8, QB = KS / 16, QH = UP ? QA : 1;
    int tid, NA, len, j0;
    int64_t cb, ce;
    const float* D;
    float2 rho;
    // row n' of this thread's tile rows (fixed over the slabs): lo and, upward, hi (lo's row when
    // the pair has no hi)
    const float2* glo[QA];
    const float2* ghi[QH];
    bool has_hi[QH];
    // load() only issues the loads; store() forms the samples once they have landed, so that
    // the next slab's loads stay in flight during the current slab's MFMAs
    float4 rlo[QA], rhi[QH];   // (u', v') at the sample's column
    bool lowh[QA];             // sample in the first half of the phi grid: u' + v', else u' - v'
    float4 rb[QB];
    bool oka[QA], okb[QB];
    __device__ void init(const float2* G2, int64_t nb, int64_t r, int ntDh, int row, const int32_t* zlo,
                         const int32_t* zhi)
    {
        const uint32_t rs = 2 * (NA / 2), bs = (uint32_t)ntDh * rs;   // row and box strides
        const float2* g = G2 + (int64_t)row * rs;
        const uint32_t rb0 = (uint32_t)(r * nb);
        int lo[QA], hi[QA];
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int64_t c = min(cb + (tid + NT * q) / KS, ce - 1);
            lo[q] = UP ? zlo[c] : (int)c;
            if (UP) hi[q] = zhi[c];
        }
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            glo[q] = g + (uint64_t)(rb0 + (uint32_t)lo[q]) * bs;
            if (UP) {
                has_hi[q] = hi[q] >= 0;
                ghi[q] = hi[q] >= 0 ? g + (uint64_t)(rb0 + (uint32_t)hi[q]) * bs : glo[q];
            }
        }
    }
    __device__ void load(int k0)
    {
        const int half = NA / 2;
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q, kk = e % KS, bc = e / KS;
            const int j = min(k0 + kk, NA - 1), jj = j < half ? j : j - half;
            float2 u = glo[q][jj], v = glo[q][jj + half];
            rlo[q] = make_float4(u.x, u.y, v.x, v.y);
            if (UP) {
                u = ghi[q][jj];
                v = ghi[q][jj + half];
                rhi[q] = make_float4(u.x, u.y, v.x, v.y);
            }
            lowh[q] = j < half;
            oka[q] = k0 + kk < NA && cb + bc < ce;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q, j = k0 + (e >> 4), jp = j0 + 4 * (e & 15);
            rb[q] = *(const float4*)(D + (int64_t)min(j, NA - 1) * len + (jp < len ? jp : 0));
            okb[q] = j < NA && jp < len;
        }
    }
    __device__ void store(float* As, float* Bs)
    {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            const float sg = lowh[q] ? 1.f : -1.f;
            const float4 a = rlo[q];
            float x = a.x + sg * a.z, y = a.y + sg * a.w;
            if (UP && has_hi[q]) {
                const float4 h = rhi[q];
                const float hx = h.x + sg * h.z, hy = h.y + sg * h.w;
                x += rho.x * hx - rho.y * hy;
                y += rho.x * hy + rho.y * hx;
            }
            const bool ok = oka[q];
            *(float2*)&As[(e % KS) * MAP + 2 * (e / KS)] = make_float2(ok ? x : 0.f, ok ? y : 0.f);
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q;
            const float4 v = rb[q];
            const bool ok = okb[q];
            *(float4*)&Bs[(e >> 4) * MBP + 4 * (e & 15)] =
                make_float4(ok ? v.x : 0.f, ok ? v.y : 0.f, ok ? v.z : 0.f, ok ? v.w : 0.f);
        }
    }
};

// UP: tiles of whole parents' z pairs (tile_begin/tile_end over the pairs, zstart/zcount each
// parent's pairs); DOWN: tiles of 32 consecutive child boxes.
template <bool UP, int KS>
__global__ __launch_bounds__(NT) void rs5_mfma(
    int64_t nb, int NA, int ntD, int ntj, const int32_t* __restrict__ row_off,
    const int32_t* __restrict__ nphi, const float* __restrict__ d5, const float2* __restrict__ G2, int Kd,
    const int32_t* __restrict__ tile_begin, const int32_t* __restrict__ tile_end,
    const int32_t* __restrict__ tile_pbeg, const int32_t* __restrict__ tile_pend,
    const int32_t* __restrict__ zlo, const int32_t* __restrict__ zhi, const int32_t* __restrict__ zoct,
    const float2* __restrict__ zrot, const int32_t* __restrict__ zstart, const int32_t* __restrict__ zcount,
    const float2* __restrict__ trans, int64_t nb_out, float2* __restrict__ out)
{
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
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    // one LDS array: the A and B slabs during the contraction, then (upward) the translated
    // pairs (32 x 64 complex) for the sums over each parent's pairs
    constexpr int kL = (UP && KS * (MAP + MBP) < 2 * (MM / 2) * MN) ? 2 * (MM / 2) * MN : KS * (MAP + MBP);
    __shared__ __align__(16) float Ls[kL];
    __shared__ int pz[2][MM / 2];   // upward: zstart - cb and zcount of the tile's parents
    float* As = Ls;
    float* Bs = Ls + KS * MAP;
    Rs5Stage<UP, KS> st;
    st.tid = tid;
    st.NA = NA;
    st.len = len;
    st.j0 = j0;
    st.cb = cb;
    st.ce = ce;
    st.D = d5 + (int64_t)off * NA;
    st.rho = UP ? zrot[row] : make_float2(1.f, 0.f);
    st.init(G2, nb, r, ntD / 2 + 1, row, zlo, zhi);
    const int colw = wc + (lane & 31);
    const int jp = j0 + colw;
    const int jpc = min(jp, len - 1);
    // upward: the pair ranges of the tile's parents, staged in LDS before the contraction
    int p0 = 0, npar = 0;
    const uint32_t rbo = (uint32_t)(r * nb_out);
    if (UP) {
        p0 = tile_pbeg[blockIdx.x];
        npar = tile_pend[blockIdx.x] - p0;
        if (tid < npar) {
            pz[0][tid] = zstart[p0 + tid] - (int)cb;
            pz[1][tid] = zcount[p0 + tid];
        }
    }
    f32x16 acc = {};
    mfma_mainloop<KS>(st, As, Bs, NA, acc, wr, wc, lane);
    float2 ev[8];
    if (!UP) {
        // add to I: the eight reads are issued before any write
        if (jp >= len) return;
        float2* o = out + off + jp;
#pragma unroll
        for (int pq = 0; pq < 8; ++pq)
            ev[pq] = o[(uint64_t)(rbo + (uint32_t)min(cb + pair_box(wr, lane, pq), ce - 1)) * (uint32_t)Kd];
#pragma unroll
        for (int pq = 0; pq < 8; ++pq) {
            const int64_t c = cb + pair_box(wr, lane, pq);
            if (c < ce)
                o[(uint64_t)(rbo + (uint32_t)c) * (uint32_t)Kd] =
                    make_float2(ev[pq].x + acc[2 * pq], ev[pq].y + acc[2 * pq + 1]);
        }
        return;
    }
    {
        // the octant of each result's pair, then its translation: all loads issued before use
        int oc[8];
#pragma unroll
        for (int pq = 0; pq < 8; ++pq) oc[pq] = zoct[min(cb + pair_box(wr, lane, pq), ce - 1)];
        const float2* tr = trans + off + jpc;
#pragma unroll
        for (int pq = 0; pq < 8; ++pq) ev[pq] = tr[(uint32_t)oc[pq] * (uint32_t)Kd];
    }
    // UP: translate each pair on the parent grid, then sum the pairs of every parent (the slabs
    // are free after the main loop's last barrier)
    float2* S = (float2*)Ls;   // 32 x 64 complex
#pragma unroll
    for (int pq = 0; pq < 8; ++pq) {
        const int bx = pair_box(wr, lane, pq);
        const bool ok = jp < len && cb + bx < ce;
        const float2 t = ev[pq];
        const float x = acc[2 * pq], y = acc[2 * pq + 1];
        S[bx * MN + colw] = make_float2(ok ? x * t.x - y * t.y : 0.f, ok ? x * t.y + y * t.x : 0.f);
    }
    __syncthreads();
    for (int e = tid; e < MN * npar; e += NT) {
        const int i = e % MN, pi = e / MN;
        const int jj = j0 + i;
        if (jj >= len) continue;
        const int a = pz[0][pi], cnt = pz[1][pi];
        float2 sum = make_float2(0.f, 0.f);
        for (int c = a; c < a + cnt; ++c) {
            const float2 v = S[c * MN + i];
            sum.x += v.x;
            sum.y += v.y;
        }
        out[(uint64_t)(rbo + (uint32_t)(p0 + pi)) * (uint32_t)Kd + off + jj] = sum;
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
                           rs.nt_dst, rs.nt_dth, (const R*)rs.dth, (const C*)G1, G2);
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

template <int V> struct KsTag { static constexpr int value = V; };

// runs f(KsTag<KS>{}) for the slab depth ks (16, 32 or 64)
template <class F> void with_ks(int ks, F&& f)
{
    if (ks == 16)
        f(KsTag<16>{});
    else if (ks == 32)
        f(KsTag<32>{});
    else
        f(KsTag<64>{});
}

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
        if (up) {
            dim3 grid(cdiv(nb, MM / 2), ntj * rs.rows_src, nrhs);
            with_ks(p->tune.rs_slab[0], [&](auto t) {
                hipLaunchKernelGGL((rs1_mfma<false, decltype(t)::value>), grid, dim3(NT), 0, s, nb, nb,
                                   rs.rows_src, NA, ntj, rs.d_src_row_off, rs.d_src_nphi,
                                   (const float*)rs.d1, (const float2*)S.sigM, S.K, S.n,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr,
                                   (const float2*)nullptr, (const float2*)nullptr, G1);
            });
        } else {
            // one contraction per z pair of children
            dim3 grid(cdiv(Cl.nz, MM / 2), ntj * rs.rows_src, nrhs);
            with_ks(p->tune.rs_slab[0], [&](auto t) {
                hipLaunchKernelGGL((rs1_mfma<true, decltype(t)::value>), grid, dim3(NT), 0, s, Cl.nz, nb,
                                   rs.rows_src, NA, ntj, rs.d_src_row_off, rs.d_src_nphi,
                                   (const float*)rs.d1, (const float2*)S.sigL, S.K, S.n, Cl.zpar,
                                   Cl.zoct, Cl.zlo, Cl.zhi, (const float2*)S.zrot,
                                   (const float2*)S.trans, G1);
            });
        }
        FFMM_LAUNCH_CHECK();
    }
    {
        const int ntSh = rs.nt_src / 2 + 1, ntDh = rs.nt_dst / 2 + 1;
        dim3 grid(cdiv(nb * (NA / 2), MN / 2), cdiv(ntDh, MM / 2), nrhs);
        with_ks(p->tune.rs_slab[1], [&](auto t) {
            hipLaunchKernelGGL((rs3h_mfma<decltype(t)::value>), grid, dim3(NT), 0, s, nb, NA, rs.rows_src,
                               ntSh, ntDh, rs.ldh, (const float*)rs.dth_h, (const float2*)G1, G2);
        });
        FFMM_LAUNCH_CHECK();
    }
    {
        int mx = 0;
        for (int v : D.par.nphi) mx = std::max(mx, v);
        const int ntj = cdiv(mx, MN);
        if (up) {
            // tiles of whole parents' z pairs
            dim3 grid((unsigned)rs.nztiles, ntj * rs.rows_dst, nrhs);
            with_ks(p->tune.rs_slab[2], [&](auto t) {
                hipLaunchKernelGGL((rs5_mfma<true, decltype(t)::value>), grid, dim3(NT), 0, s, nb, NA,
                                   rs.nt_dst, ntj, rs.d_dst_row_off, rs.d_dst_nphi, (const float*)rs.d5,
                                   (const float2*)G2, D.K, rs.ztile_begin, rs.ztile_end, rs.ztile_pbeg,
                                   rs.ztile_pend, Cl.zlo, Cl.zhi, Cl.zoct, (const float2*)D.zrot,
                                   D.zstart, D.zcount, (const float2*)D.trans, D.n, (float2*)D.sigM);
            });
        } else {
            dim3 grid(cdiv(nb, MM / 2), ntj * rs.rows_dst, nrhs);
            with_ks(p->tune.rs_slab[3], [&](auto t) {
                hipLaunchKernelGGL((rs5_mfma<false, decltype(t)::value>), grid, dim3(NT), 0, s, nb, NA,
                                   rs.nt_dst, ntj, rs.d_dst_row_off, rs.d_dst_nphi, (const float*)rs.d5,
                                   (const float2*)G2, D.K, (const int32_t*)nullptr,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, (const float2*)nullptr,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, (const float2*)nullptr,
                                   D.n, (float2*)D.sigL);
            });
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
