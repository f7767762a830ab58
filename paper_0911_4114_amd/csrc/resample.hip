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

// Child tiles of the upward pass: consecutive whole parents, at most 32 children per tile.
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

void run_resample(ffmm_plan* p, int l_src, int l_dst, int nrhs, hipStream_t s)
{
    if (p->prec == FFMM_FP32)
        run_resample_t<float>(p, l_src, l_dst, nrhs, s);
    else
        run_resample_t<double>(p, l_src, l_dst, nrhs, s);
}

}  // namespace ffmm
