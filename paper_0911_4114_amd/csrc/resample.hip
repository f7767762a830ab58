// Five-step inter/anterpolation between level quadratures (Section 3.4) for the upward (M2M) and
// downward (L2L) passes. Each 1D step applies one real Fourier-resample matrix (the Dirichlet
// kernel with the Nyquist bin dropped) to a batch of boxes, i.e. a dense contraction
//     Y[i][col] = sum_k D[i][k] X[k][col],
// computed on the matrix cores in the plan precision. Complex data enter as interleaved (re, im)
// real rows or columns.
//   step 1      per source row n:  G1[c][n][j]  = sum_m D1_n[j][m] in_c(n, m),          j < NA
//   steps 2+3   per column m < NA/2, on half ranges of theta (eqn. FourierSphereSym, below)
//   steps 4+5   per destination row n': out_c(n', j') = sum_j D5_n'[j'][j] row_{c,n'}(j)
// Steps 1 and 5 run on half ranges of phi (every row length is even and sample m + N/2 lies half a
// turn from sample m): u = x_m + x_{m+N/2} carries the even modes, v = x_m - x_{m+N/2} the odd
// ones, a = De u and b = Do v are contracted over m < N/2 in one MFMA tile (32 samples of each),
// and the outputs are y_j = a_j + b_j, y_{j+N'/2} = a_j - b_j: half the work of the full rows.
// Where the common phi length is long (rs1q_mfma, rs5q_mfma), u and v are split again by the
// reflection phi -> -phi, under which the kernel is even: four channels contracted over
// m <= N/4 give the four samples j, j + N'/2, N'/2 - j and N' - j of each j <= N'/4.
// UP (M2M, Section 2):   in_c = M^l_c; the parent signature is the sum over its children of
//                         E_oct(c) * out_c, summed in LDS over whole parents per tile.
// DOWN (L2L, Section 2): in_c = L^l_parent(c) * conj(E_oct(c)); out_c is added to L^{l+1}_c,
//                         which already holds I^{l+1}_c.
// The children of one parent at octants o and o + 4 (same x and y, z apart by the child side)
// have translations that differ by a factor rho(n) = e^{i kappa cos(theta_n) a_child}, constant
// on each theta row; the row steps 1 and 5 do not mix rows, so such a z pair shares one
// contraction: upward the theta step writes row(lo) + rho row(hi) on each destination row, which
// step 5 resamples once and translates with lo's octant; downward step 1 resamples the parent data
// times conj(E_oct(lo)) and hi's result is lo's times conj(rho(n)).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"

namespace ffmm {

namespace {

constexpr int NT = 256;          // threads per block: four waves
constexpr int MM = 64, MN = 64;  // block tile
constexpr int BC = MM / 2;       // boxes (complex rows) per block tile
constexpr int MAP = MM + 4;      // LDS row stride of the A slab (rows stay 16-byte aligned)
constexpr int MBP = MN;          // LDS row stride of the B slab

template <class R> struct cpx;
template <> struct cpx<float> { using type = float2; };
template <> struct cpx<double> { using type = double2; };

template <class R> __device__ inline typename cpx<R>::type cx(R x, R y)
{
    typename cpx<R>::type v;
    v.x = x;
    v.y = y;
    return v;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// One wave's 32 x 32 quadrant (rows wr.., columns wc..) of the 64 x 64 block tile: the slab
// contraction acc += A[wr.., 0:kc] B[0:kc, wc..] (kc a multiple of 8; slab rows at and beyond the
// valid depth hold zeros) and where each accumulator value lands in the quadrant:
//   result p < 8 of this lane in the row steps, whose quadrant rows 2 box and 2 box + 1 are
//   (re, im) of one box: rbox(lane, p), rcol(lane, p), re(acc, p), im(acc, p);
//   value q < 16 of this lane: vrow(lane, q), vcol(lane, q), val(acc, q).
template <class R> struct MT;

// FP32: one v_mfma_f32_32x32x2f32 tile; operand lanes A[i][k], B[k][j] with i, j = lane % 32,
// k = lane / 32; register q holds row (q / 4) * 8 + (lane / 32) * 4 + q % 4, column lane % 32.
template <> struct MT<float> {
    using acc_t = f32x16;
    template <int LDB = MBP>
    __device__ static void slab(const float* __restrict__ As, const float* __restrict__ Bs, acc_t& acc, int wr,
                                int wc, int lane, int kc)
    {
        const int i = lane & 31, kh = lane >> 5;
        for (int k8 = 0; k8 < kc; k8 += 8) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[(k8 + 2 * u + kh) * MAP + wr + i];
                b[u] = Bs[(k8 + 2 * u + kh) * LDB + wc + i];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u], b[u], acc, 0, 0, 0);
        }
    }
    __device__ static int rbox(int lane, int p) { return (p >> 1) * 4 + (lane >> 5) * 2 + (p & 1); }
    __device__ static int rcol(int lane, int) { return lane & 31; }
    __device__ static float re(const acc_t& a, int p) { return a[2 * p]; }
    __device__ static float im(const acc_t& a, int p) { return a[2 * p + 1]; }
    __device__ static int vrow(int lane, int q) { return (q >> 2) * 8 + (lane >> 5) * 4 + (q & 3); }
    __device__ static int vcol(int lane, int) { return lane & 31; }
    __device__ static float val(const acc_t& a, int q) { return a[q]; }
};

// FP64: 2 x 2 tiles (ti, tj) of v_mfma_f64_16x16x4f64; operand lanes A[i][k], B[k][j] with
// i, j = lane % 16, k = lane / 16; register r holds D[lane / 16 + 4 r][lane % 16]. Lane i of the
// A operand reads tile row pi(i) = 4 (i % 4) + i / 4 of the slab, so that register r of a tile
// holds tile row 16 ti + 4 (lane / 16) + r, column 16 tj + lane % 16: a box's (re, im) rows sit in
// registers 2b, 2b + 1 of one lane. Result p = (ti, tj, b) = (p / 4, (p / 2) % 2, p % 2); value
// q = (ti, tj, r) = (q / 8, (q / 4) % 2, q % 4).
template <> struct MT<double> {
    struct acc_t {
        f64x4 t[4];   // tile (ti, tj) at 2 ti + tj
    };
    template <int LDB = MBP>
    __device__ static void slab(const double* __restrict__ As, const double* __restrict__ Bs, acc_t& acc,
                                int wr, int wc, int lane, int kc)
    {
        const int i = lane & 15, kq = lane >> 4, pi = 4 * (i & 3) + (i >> 2);
        for (int k4 = 0; k4 < kc; k4 += 4) {
            const int k = k4 + kq;
            const double a0 = As[k * MAP + wr + pi], a1 = As[k * MAP + wr + 16 + pi];
            const double b0 = Bs[k * LDB + wc + i], b1 = Bs[k * LDB + wc + 16 + i];
            acc.t[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.t[0], 0, 0, 0);
            acc.t[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.t[1], 0, 0, 0);
            acc.t[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.t[2], 0, 0, 0);
            acc.t[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.t[3], 0, 0, 0);
        }
    }
    __device__ static int rbox(int lane, int p) { return 8 * (p >> 2) + 2 * (lane >> 4) + (p & 1); }
    __device__ static int rcol(int lane, int p) { return 16 * ((p >> 1) & 1) + (lane & 15); }
    __device__ static double re(const acc_t& a, int p) { return a.t[2 * (p >> 2) + ((p >> 1) & 1)][2 * (p & 1)]; }
    __device__ static double im(const acc_t& a, int p)
    {
        return a.t[2 * (p >> 2) + ((p >> 1) & 1)][2 * (p & 1) + 1];
    }
    __device__ static int vrow(int lane, int q) { return 16 * (q >> 3) + 4 * (lane >> 4) + (q & 3); }
    __device__ static int vcol(int lane, int q) { return 16 * ((q >> 2) & 1) + (lane & 15); }
    __device__ static double val(const acc_t& a, int q) { return a.t[2 * (q >> 3) + ((q >> 2) & 1)][q & 3]; }
};

// four consecutive reals (16-byte aligned), and their LDS store with invalid entries zeroed
// component by component (a select of whole vectors makes the compiler stage them through
// private memory)
template <class R> struct V4;
template <> struct V4<float> {
    float4 v;
    __device__ static V4 ld(const float* p) { return {*(const float4*)p}; }
    __device__ void st(float* p, bool ok) const
    {
        *(float4*)p = make_float4(ok ? v.x : 0.f, ok ? v.y : 0.f, ok ? v.z : 0.f, ok ? v.w : 0.f);
    }
};
template <> struct V4<double> {
    double2 a, b;
    __device__ static V4 ld(const double* p) { return {*(const double2*)p, *(const double2*)(p + 2)}; }
    __device__ void st(double* p, bool ok) const
    {
        *(double2*)p = make_double2(ok ? a.x : 0.0, ok ? a.y : 0.0);
        *(double2*)(p + 2) = make_double2(ok ? b.x : 0.0, ok ? b.y : 0.0);
    }
};

// Shared main loop of the row steps over one LDS slab buffer. Stage::load(k0) issues the global
// loads of the slab starting at k0 into registers; Stage::store(As, Bs) writes them (zeroing
// invalid entries) once they have landed. The next slab's loads are in flight during the current
// slab's MFMAs. The A slab is two [KS][MAP] halves, u then v: the waves of tile columns 0..31
// (the even operator's block) read u, those of columns 32..63 (the odd operator's) read v.
template <class R, int KS, class Stage>
__device__ inline void mfma_mainloop(Stage& st, R* As, R* Bs, int K, typename MT<R>::acc_t& acc, int wr, int wc,
                                     int lane)
{
    const int nslab = (K + KS - 1) / KS;
    const R* Aw = As + (wc ? KS * MAP : 0);
    st.load(0);
    st.store(As, Bs);
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        const bool more = sl + 1 < nslab;
        if (more) st.load((sl + 1) * KS);
        const int kc = min(KS, K - sl * KS);
        MT<R>::slab(Aw, Bs, acc, wr, wc, lane, (kc + 7) & ~7);
        if (more) {
            __syncthreads();   // every wave is done with this slab
            st.store(As, Bs);
        }
        __syncthreads();
    }
}

// The row steps' epilogue exchange: each wave's 32 x 32 quadrant of the 64 x 64 block tile into
// LDS (row = (box, re/im), column: 0..31 even part a, 32..63 odd part b of the same 32 samples)
template <class R>
__device__ inline void tile_to_lds(R* Ls, const typename MT<R>::acc_t& acc, int wr, int wc, int lane)
{
    using T = MT<R>;
#pragma unroll
    for (int q = 0; q < 16; ++q) Ls[(wr + T::vrow(lane, q)) * MN + wc + T::vcol(lane, q)] = T::val(acc, q);
}

// a + sg b of box b, sample i of the tile held in LDS by tile_to_lds
template <class R>
__device__ inline typename cpx<R>::type tile_out(const R* Ls, int b, int i, R sg)
{
    const R* r = Ls + 2 * b * MN + i;
    return cx<R>(r[0] + sg * r[32], r[MN] + sg * r[MN + 32]);
}

// ---- quarter ranges of phi (long rows): the half-range parts split again by phi -> -phi --------
// A block tile: 32 boxes (64 rows) x 128 columns, the S, A, Mv and P sums of 32 output indices j;
// the A operand is four [KS][MAP] slabs (us, ua, vm, vp), the B operand [KS][128] (the four
// operator blocks side by side). The waves of column half wc compute channels 2 wc and 2 wc + 1.
constexpr int MQ = 128;   // LDS row stride of the quarter-range B slab and exchange tile

template <class R, int KS, class Stage>
__device__ inline void mfma_mainloop_q(Stage& st, R* As, R* Bs, int K, typename MT<R>::acc_t (&acc)[2], int wr,
                                       int wc, int lane)
{
    const int nslab = (K + KS - 1) / KS;
    st.load(0);
    st.store(As, Bs);
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        const bool more = sl + 1 < nslab;
        if (more) st.load((sl + 1) * KS);
        const int kc = (min(KS, K - sl * KS) + 7) & ~7;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int ch = 2 * (wc != 0) + c;
            MT<R>::template slab<MQ>(As + ch * KS * MAP, Bs + ch * 32, acc[c], wr, 0, lane, kc);
        }
        if (more) {
            __syncthreads();
            st.store(As, Bs);
        }
        __syncthreads();
    }
}

// the two channel tiles of each wave into LDS: row (box, re/im), column channel * 32 + j
template <class R>
__device__ inline void tile_to_lds_q(R* Ls, const typename MT<R>::acc_t (&acc)[2], int wr, int wc, int lane)
{
    using T = MT<R>;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int col0 = (2 * (wc != 0) + c) * 32;
#pragma unroll
        for (int q = 0; q < 16; ++q)
            Ls[(wr + T::vrow(lane, q)) * MQ + col0 + T::vcol(lane, q)] = T::val(acc[c], q);
    }
}

// the four outputs of box b, index jj of the tile: y_j, y_{j+M/2}, y_{M/2-j}, y_{M-j}
template <class R>
__device__ inline void tile_out_q(const R* Ls, int b, int jj, typename cpx<R>::type (&y)[4])
{
    const R* r = Ls + 2 * b * MQ + jj;   // re row; the im row follows
    const R sx = r[0], ax = r[32], mx = r[64], px = r[96];
    const R sy = r[MQ], ay = r[MQ + 32], my = r[MQ + 64], py = r[MQ + 96];
    y[0] = cx<R>(sx + ax + mx + px, sy + ay + my + py);
    y[1] = cx<R>(sx + ax - mx - px, sy + ay - my - py);
    y[2] = cx<R>(sx - ax + px - mx, sy - ay + py - my);
    y[3] = cx<R>(sx - ax - px + mx, sy - ay - py + my);
}

// staging of the quarter-range channels from the samples m, m + h, h - m, -m (mod N) of a row of N
// samples (h = N/2, 0 <= m <= N/4): us, ua, vm, vp as above
template <class R>
__device__ inline void quarter_channels(typename cpx<R>::type x0, typename cpx<R>::type x1,
                                        typename cpx<R>::type x2, typename cpx<R>::type x3, bool ok, R* As,
                                        int KSMAP, int o)
{
    using C = typename cpx<R>::type;
    const R ux = x0.x + x1.x, uy = x0.y + x1.y, bx = x2.x + x3.x, by = x2.y + x3.y;
    const R vx = x0.x - x1.x, vy = x0.y - x1.y, wx = x2.x - x3.x, wy = x2.y - x3.y;
    *(C*)&As[o] = cx<R>(ok ? ux + bx : R(0), ok ? uy + by : R(0));
    *(C*)&As[KSMAP + o] = cx<R>(ok ? ux - bx : R(0), ok ? uy - by : R(0));
    *(C*)&As[2 * KSMAP + o] = cx<R>(ok ? vx - wx : R(0), ok ? vy - wy : R(0));
    *(C*)&As[3 * KSMAP + o] = cx<R>(ok ? vx + wx : R(0), ok ? vy + wy : R(0));
}

// step 1 on quarter ranges: A = the source row data of 32 boxes (downward, z pairs: the parent's
// data times conj(E_oct(lo))), B = the row's quarter-range operator block.
template <class R, bool DOWN, int KS> struct Rs1QStage {
    using C = typename cpx<R>::type;
    static constexpr int QA = KS / 8, QB = KS / 8, QT = DOWN ? QA : 1;
    int tid, N, h, q, ldq, j0, Qp1;   // source row: N samples, h = N/2, q = N/4; Qp1 = NPhi/4 + 1
    int64_t c0, nb;
    const R* d1;
    int off;
    const C* gs[QA];
    const C* gt[QT];
    C ra[QA][4], rt[QT][4];
    V4<R> rb[QB];
    bool oka[QA], okb[QB];
    __device__ void init(const C* sig, int Ksrc, int64_t nb_in, int64_t r, const int32_t* zpar,
                         const int32_t* zoct, const C* trans)
    {
        const uint32_t rb0 = (uint32_t)(r * nb_in);
        int bi[QA], oi[QA];
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            const int64_t c = min(c0 + (tid + NT * u) / KS, nb - 1);
            bi[u] = DOWN ? zpar[c] : (int)c;
            if (DOWN) oi[u] = zoct[c];
        }
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            gs[u] = sig + off + (uint64_t)(rb0 + (uint32_t)bi[u]) * (uint32_t)Ksrc;
            if (DOWN) gt[u] = trans + off + (uint32_t)oi[u] * (uint32_t)Ksrc;
        }
    }
    __device__ void load(int k0)
    {
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            const int e = tid + NT * u, kk = e % KS, bc = e / KS;
            const int m = min(k0 + kk, q);
            const int i[4] = {m, m + h, h - m, m == 0 ? 0 : N - m};
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                ra[u][a] = gs[u][i[a]];
                if (DOWN) rt[u][a] = gt[u][i[a]];
            }
            oka[u] = k0 + kk <= q && c0 + bc < nb;
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            const int e = tid + NT * u, kr = k0 + (e >> 5), c4 = 4 * (e & 31), j = j0 + (c4 & 31);
            rb[u] = V4<R>::ld(d1 + ((int64_t)min(kr, q) * 4 + (c4 >> 5)) * ldq + (j < ldq ? j : 0));
            okb[u] = kr <= q && j < Qp1;
        }
    }
    __device__ void store(R* As, R* Bs)
    {
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            const int e = tid + NT * u;
            C x[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                x[a] = ra[u][a];
                if (DOWN) {
                    const C t = rt[u][a];   // times conj(E)
                    x[a] = cx<R>(x[a].x * t.x + x[a].y * t.y, x[a].y * t.x - x[a].x * t.y);
                }
            }
            quarter_channels<R>(x[0], x[1], x[2], x[3], oka[u], As, KS * MAP, (e % KS) * MAP + 2 * (e / KS));
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            const int e = tid + NT * u;
            rb[u].st(&Bs[(e >> 5) * MQ + 4 * (e & 31)], okb[u]);
        }
    }
};

// Block (tile of 32 boxes, source row n, output indices j0.. j0 + 31 of 0..NPhi/4): G1 samples j,
// j + NPhi/2, NPhi/2 - j and NPhi - j.
template <class R, bool DOWN, int KS>
__global__ __launch_bounds__(NT) void rs1q_mfma(int64_t nt, int64_t nb, int rows, int NA, int ldq, int ntj,
                                                const int32_t* __restrict__ row_off,
                                                const int32_t* __restrict__ nphi, const R* __restrict__ d1q,
                                                const int32_t* __restrict__ d1q_off,
                                                const typename cpx<R>::type* __restrict__ sig, int Ksrc,
                                                int64_t nb_in, const int32_t* __restrict__ zpar,
                                                const int32_t* __restrict__ zoct,
                                                const int32_t* __restrict__ zlo,
                                                const typename cpx<R>::type* __restrict__ trans,
                                                typename cpx<R>::type* __restrict__ G1)
{
    using C = typename cpx<R>::type;
    using T = MT<R>;
    const int row = blockIdx.y / ntj, j0 = (blockIdx.y % ntj) * 32;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    constexpr int kL = 4 * KS * MAP + KS * MQ > MM * MQ ? 4 * KS * MAP + KS * MQ : MM * MQ;
    __shared__ __align__(16) R Ls[kL];
    R* As = Ls;
    R* Bs = Ls + 4 * KS * MAP;
    const int Q = NA / 4, H = NA / 2;
    Rs1QStage<R, DOWN, KS> st;
    st.tid = tid;
    st.N = nphi[row];
    st.h = st.N / 2;
    st.q = st.N / 4;
    st.ldq = ldq;
    st.j0 = j0;
    st.Qp1 = Q + 1;
    st.off = row_off[row];
    st.c0 = (int64_t)blockIdx.x * BC;
    st.nb = nt;
    st.d1 = d1q + d1q_off[row];
    st.init(sig, Ksrc, nb_in, blockIdx.z, zpar, zoct, trans);
    typename T::acc_t acc[2] = {};
    mfma_mainloop_q<R, KS>(st, As, Bs, st.q + 1, acc, wr, wc, lane);
    // downward: lo's result only (hi's is lo's times conj(rho(n)), applied by the theta step)
    const int jj = tid & 31, j = j0 + jj;
    int dst[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        const int64_t c = min(st.c0 + (tid >> 5) + 8 * it, nt - 1);
        dst[it] = DOWN ? zlo[c] : (int)c;
    }
    tile_to_lds_q<R>(Ls, acc, wr, wc, lane);
    __syncthreads();
    if (j > Q) return;
    const uint32_t rb0 = (uint32_t)(blockIdx.z * nb), bs = (uint32_t)rows * NA;   // box stride
    const bool inner = j > 0 && j < Q;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        const int b = (tid >> 5) + 8 * it;
        if (st.c0 + b >= nt) break;
        C y[4];
        tile_out_q<R>(Ls, b, jj, y);
        C* g = G1 + (uint64_t)(rb0 + (uint32_t)dst[it]) * bs + (int64_t)row * NA;
        g[j] = y[0];
        g[j + H] = y[1];
        if (inner) {
            g[H - j] = y[2];
            g[NA - j] = y[3];
        }
    }
}

// step 1 staging, on half ranges of phi: A = u, v of the source row data of 32 boxes (samples m
// and m + N_phi,n/2), or in the downward pass of 32 z pairs (lo, hi) of children: the parent's data
// times conj(E_oct(lo)). B = the row's even and odd operator blocks (32 samples each).
template <class R, bool DOWN, int KS> struct Rs1Stage {
    using C = typename cpx<R>::type;
    int tid, h, H, ldj, j0;   // h, H: half the source row length and half NPhi
    int64_t c0, nb;
    const R* d1;              // the row's operator block
    int off;
    static constexpr int QA = KS / 8, QB = KS / 16, QT = DOWN ? QA : 1;
    // source row n of this thread's tile rows (fixed over the slabs), and downward the row of
    // the translation of lo's octant
    const C* gs[QA];
    const C* gt[QT];
    // load() only issues the loads; store() applies conj(E) and forms u, v once they have
    // landed, so that the next slab's loads stay in flight during the current slab's MFMAs
    C ra[QA], rc[QA], rt[QT], rtc[QT];
    V4<R> rb[QB];
    bool oka[QA], okb[QB];
    __device__ void init(const C* sig, int Ksrc, int64_t nb_in, int64_t r, const int32_t* zpar,
                         const int32_t* zoct, const C* trans)
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
            const int k = min(k0 + kk, h - 1);
            ra[q] = gs[q][k];
            rc[q] = gs[q][k + h];
            if (DOWN) {
                rt[q] = gt[q][k];
                rtc[q] = gt[q][k + h];
            }
            oka[q] = k0 + kk < h && c0 + bc < nb;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q, kr = k0 + (e >> 4), c4 = 4 * (e & 15), j = j0 + (c4 & 31);
            rb[q] = V4<R>::ld(d1 + ((int64_t)min(kr, h - 1) * 2 + (c4 >> 5)) * ldj + (j < ldj ? j : 0));
            okb[q] = kr < h && j < H;
        }
    }
    __device__ void store(R* As, R* Bs)
    {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            C x = ra[q], y = rc[q];
            if (DOWN) {
                const C t = rt[q], tc = rtc[q];   // times conj(E)
                x = cx<R>(x.x * t.x + x.y * t.y, x.y * t.x - x.x * t.y);
                y = cx<R>(y.x * tc.x + y.y * tc.y, y.y * tc.x - y.x * tc.y);
            }
            const bool ok = oka[q];
            const int o = (e % KS) * MAP + 2 * (e / KS);
            *(C*)&As[o] = cx<R>(ok ? x.x + y.x : R(0), ok ? x.y + y.y : R(0));
            *(C*)&As[KS * MAP + o] = cx<R>(ok ? x.x - y.x : R(0), ok ? x.y - y.y : R(0));
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q;
            rb[q].st(&Bs[(e >> 4) * MBP + 4 * (e & 15)], okb[q]);
        }
    }
};

// nt: the tile rows (boxes, or z pairs in the downward pass); nb: the boxes of the G1 layout.
// Block (tile of 32 boxes, source row n, 32 samples j0.. of the first half of the common phi
// grid): G1 samples j and j + NPhi/2.
template <class R, bool DOWN, int KS>
__global__ __launch_bounds__(NT) void rs1_mfma(int64_t nt, int64_t nb, int rows, int NA, int ldj, int ntj,
                                               const int32_t* __restrict__ row_off,
                                               const int32_t* __restrict__ nphi, const R* __restrict__ d1h,
                                               const typename cpx<R>::type* __restrict__ sig, int Ksrc,
                                               int64_t nb_in, const int32_t* __restrict__ zpar,
                                               const int32_t* __restrict__ zoct,
                                               const int32_t* __restrict__ zlo,
                                               const typename cpx<R>::type* __restrict__ trans,
                                               typename cpx<R>::type* __restrict__ G1)
{
    using C = typename cpx<R>::type;
    using T = MT<R>;
    const int row = blockIdx.y / ntj, j0 = (blockIdx.y % ntj) * (MN / 2);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    constexpr int kL = 2 * KS * MAP + KS * MBP > MM * MN ? 2 * KS * MAP + KS * MBP : MM * MN;
    __shared__ __align__(16) R Ls[kL];
    R* As = Ls;
    R* Bs = Ls + 2 * KS * MAP;
    const int H = NA / 2;
    Rs1Stage<R, DOWN, KS> st;
    st.tid = tid;
    st.h = nphi[row] / 2;
    st.off = row_off[row];
    st.H = H;
    st.ldj = ldj;
    st.j0 = j0;
    st.c0 = (int64_t)blockIdx.x * BC;
    st.nb = nt;
    st.d1 = d1h + (int64_t)st.off * ldj;
    st.init(sig, Ksrc, nb_in, blockIdx.z, zpar, zoct, trans);
    typename T::acc_t acc = {};
    mfma_mainloop<R, KS>(st, As, Bs, st.h, acc, wr, wc, lane);
    // downward: lo's result only (hi's is lo's times conj(rho(n)), which the theta step applies as
    // it reads lo's rows for hi); the pair indices are loaded before the exchange
    const int i = tid & 31, hh = (tid >> 5) & 1;
    int dst[8];
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int64_t c = min(st.c0 + (tid >> 6) + 4 * it, nt - 1);
        dst[it] = DOWN ? zlo[c] : (int)c;
    }
    tile_to_lds<R>(Ls, acc, wr, wc, lane);
    __syncthreads();
    if (j0 + i >= H) return;
    const uint32_t rb0 = (uint32_t)(blockIdx.z * nb), bs = (uint32_t)rows * NA;   // box stride
    C* g = G1 + (int64_t)row * NA + j0 + i + (hh ? H : 0);
    const R sg = hh ? R(-1) : R(1);
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int b = (tid >> 6) + 4 * it;
        if (st.c0 + b >= nt) break;
        g[(uint64_t)(rb0 + (uint32_t)dst[it]) * bs] = tile_out<R>(Ls, b, i, sg);
    }
}

// steps 2 + 3 on half ranges (eqn. FourierSphereSym): per phi column m < NPhi/2 the source rows
// 0..N_theta/2 split into u = F_m + F_{m + NPhi/2} (even phi modes, even in theta) and
// v = F_m - F_{m + NPhi/2} (odd modes, odd in theta); the theta step is then two half-range
// contractions u' = De^T u, v' = Do^T v (De, Do carry the factor 1/2) onto the destination rows
// 0..N'_theta/2, where F'_m = u' + v', F'_{m + NPhi/2} = u' - v'. Half the work of resampling the
// full theta circle. A block tile stacks 32 rows t' of De (the waves on tile rows 0..31, which
// read u) over the same 32 rows of Do (tile rows 32..63, which read v); the two halves meet in
// LDS after the contraction, and the u' waves write F'_m, the v' waves F'_{m + NPhi/2}.
// G2: [rhs][box][N'_theta/2 + 1][NPhi] complex, each row on the common phi grid.
// dh holds De then Do, each [N_theta/2 + 1][ldh].
// Grid: one dimension of column tiles x row tiles (ny of them). With several row tiles the row
// tiles of a column tile are consecutive logical blocks of one XCD, so that the tile's G1 columns,
// read by every row tile, come from that XCD's L2 after the first (with one row tile the plain
// order measured faster).
// ZP (downward pass): the column of a child that is the upper member of a z pair reads its pair's
// lower member's G1 rows (step 1 wrote only those), times conj(rho(n)) on source row n.
// PAIR (upward pass): the columns run over the z pairs, per pair and phi_m its members present (lo,
// or lo and hi side by side), so that pair e starts at column zmp[e] NPhi/2 (zmp counts the
// children before it; zcol_tile[tile] is the pair of a tile's first column); each G2 row is written
// per pair: row(lo) + rho(n') row(hi) on destination row n' (zrot of the destination level), the
// sum that step 5 resamples and translates with lo's octant. nb then counts the pairs (G2 layout)
// and nbox the children (G1 layout).
template <class R, int KS, bool ZP, bool PAIR>
__global__ __launch_bounds__(NT) void rs3h_mfma(int64_t nb, int64_t nbox, int NA, int rowsS, int ntSh, int ntDh,
                                                int ldh, int ny, const R* __restrict__ dh,
                                                const int32_t* __restrict__ zsrc,
                                                const int32_t* __restrict__ zlo,
                                                const int32_t* __restrict__ zhi,
                                                const int32_t* __restrict__ zmp,
                                                const int32_t* __restrict__ zcol_tile,
                                                const typename cpx<R>::type* __restrict__ zrot,
                                                const typename cpx<R>::type* __restrict__ G1,
                                                typename cpx<R>::type* __restrict__ G2)
{
    using C = typename cpx<R>::type;
    using T = MT<R>;
    constexpr int QA = KS / 16, QB = KS / 8;
    // the A slab and the u, v halves of the B slab; after the contraction, the 64 x 64 tile of
    // results (u' rows over v' rows)
    constexpr int kL = KS * MAP + 2 * KS * MBP > MM * MN ? KS * MAP + 2 * KS * MBP : MM * MN;
    __shared__ __align__(16) R Ls[kL];
    R* As = Ls;
    R* Bs = Ls + KS * MAP;
    const int half = NA / 2;
    const unsigned lb = ny > 1 ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int i0 = (int)(lb % (unsigned)ny) * (MM / 2);
    const int64_t r = blockIdx.z;
    const int64_t ncols = nbox * half;
    const unsigned tile = lb / (unsigned)ny;
    const int64_t g0 = (int64_t)tile * (MN / 2);
    // first (box, column) of the tile
    const int64_t cbase = g0 / half;
    const int m0 = (int)(g0 - cbase * half);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const bool odd = wr != 0;
    const int64_t mat_off = (int64_t)ntSh * ldh;   // Do after De
    // this thread's staged column (phi_m of its box), row 0; with PAIR also the column's pair, its
    // phi_m, whether it holds hi, and whether the pair has two members
    const C* sbase;
    bool scol_ok, zconj = false;
    int64_t zp = 0;
    int zm = 0;
    bool zhi_col = false, ztwo = false;
    {
        const int cc = tid & 31;
        int m = m0 + cc;
        int64_t c = cbase;
        scol_ok = g0 + cc < ncols;
        if (PAIR) {
            if (scol_ok) {
                const int64_t g = g0 + cc;
                zp = zcol_tile[tile];
                while ((int64_t)zmp[zp + 1] * half <= g) ++zp;
                const int a = zmp[zp], local = (int)(g - (int64_t)a * half);
                ztwo = zmp[zp + 1] - a == 2;
                zm = ztwo ? local >> 1 : local;
                zhi_col = ztwo && (local & 1);
                m = zm;
                c = zhi_col ? zhi[zp] : zlo[zp];
            }
        } else {
            while (m >= half) {
                m -= half;
                ++c;
            }
        }
        if (ZP && scol_ok) {
            const int zs = zsrc[c];
            if (zs >= 0) {
                c = zs;
                zconj = true;
            }
        }
        sbase = scol_ok ? G1 + (r * nbox + c) * rowsS * NA + m : G1;
    }
    V4<R> ra[QA];
    C rfa[QB], rfb[QB];   // F_m, F_{m + NPhi/2} of each staged row
    C rz[ZP ? QB : 1];    // rho(n) of each staged row
    bool oka[QA], okb[QB];
    auto load = [&](int k0) {
        // A tile column c4: 0..31 are De rows i0.., 32..63 the same rows of Do
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q, t = k0 + (e >> 4), c4 = 4 * (e & 15);
            const int tp = i0 + (c4 & 31);
            const bool ok = t < ntSh && tp < ldh;
            const int64_t idx = ok ? (c4 >= 32 ? mat_off : 0) + (int64_t)t * ldh + tp : 0;
            ra[q] = V4<R>::ld(dh + idx);
            oka[q] = ok;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int tt = k0 + (tid >> 5) + 8 * q;
            const int64_t row = (int64_t)min(tt, ntSh - 1) * NA;
            rfa[q] = sbase[row];
            rfb[q] = sbase[row + half];
            if (ZP) rz[q] = zrot[min(tt, ntSh - 1)];
            okb[q] = tt < ntSh && scol_ok;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            ra[q].st(&As[(e >> 4) * MAP + 4 * (e & 15)], oka[q]);
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int o = ((tid >> 5) + 8 * q) * MBP + 2 * (tid & 31);
            C a = rfa[q], b = rfb[q];
            if (ZP && zconj) {
                const C z = rz[q];   // times conj(rho(n))
                a = cx<R>(a.x * z.x + a.y * z.y, a.y * z.x - a.x * z.y);
                b = cx<R>(b.x * z.x + b.y * z.y, b.y * z.x - b.x * z.y);
            }
            const bool ok = okb[q];
            *(C*)&Bs[o] = cx<R>(ok ? a.x + b.x : R(0), ok ? a.y + b.y : R(0));
            *(C*)&Bs[KS * MBP + o] = cx<R>(ok ? a.x - b.x : R(0), ok ? a.y - b.y : R(0));
        }
    };
    typename T::acc_t acc = {};
    const int nslab = (ntSh + KS - 1) / KS;
    load(0);
    store();
    __syncthreads();
    for (int sl = 0; sl < nslab; ++sl) {
        const bool more = sl + 1 < nslab;
        if (more) load((sl + 1) * KS);
        const int kc = (min(KS, ntSh - sl * KS) + 7) & ~7;
        T::slab(As, Bs + (odd ? KS * MBP : 0), acc, wr, wc, lane, kc);
        if (more) {
            __syncthreads();
            store();
        }
        __syncthreads();
    }
    // value q: destination row i0 + vrow, tile column wc + vcol = (box, phi_m, re/im); the u'
    // waves (even) and v' waves (odd) exchange their values through LDS (the slabs are free after
    // the main loop's last barrier), then form F'_m = u' + v' and F'_{m + NPhi/2} = u' - v'
#pragma unroll
    for (int q = 0; q < 16; ++q) Ls[(wr + T::vrow(lane, q)) * MN + wc + T::vcol(lane, q)] = T::val(acc, q);
    __syncthreads();
    if (PAIR) {
        // per (destination row, lo column, half of the phi grid): the pair's sample
        // row(lo) + rho row(hi), or row(lo) alone; the thread's column is the one it staged, its
        // rows (tid >> 6) + 4 i and its half (tid >> 5) & 1
        if (!scol_ok || zhi_col) return;
        const int cc = tid & 31, hh = (tid >> 5) & 1;
        const R sg = hh ? R(-1) : R(1);
        C* g2 = G2 + (r * nb + zp) * ntDh * NA + zm + (hh ? half : 0);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int tr = (tid >> 6) + 4 * i, tp = i0 + tr;
            if (tp >= ntDh) break;
            const R* ur = Ls + tr * MN + 2 * cc;          // u' row: lo (re, im), then hi (re, im)
            const R* vr = Ls + (32 + tr) * MN + 2 * cc;   // v' row
            R x = ur[0] + sg * vr[0], y = ur[1] + sg * vr[1];
            if (ztwo) {
                const R hx = ur[2] + sg * vr[2], hy = ur[3] + sg * vr[3];
                const C z = zrot[tp];
                x += z.x * hx - z.y * hy;
                y += z.x * hy + z.y * hx;
            }
            g2[(int64_t)tp * NA] = cx<R>(x, y);
        }
        return;
    }
    const R sg = odd ? R(-1) : R(1);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int col = wc + T::vcol(lane, q), cc = col >> 1, part = col & 1;
        const int tr = T::vrow(lane, q), tp = i0 + tr;
        if (g0 + cc >= ncols || tp >= ntDh) continue;
        int m = m0 + cc;
        int64_t c = cbase;
        while (m >= half) {
            m -= half;
            ++c;
        }
        const R u = Ls[tr * MN + col], v = Ls[(32 + tr) * MN + col];
        R* base = (R*)(G2 + ((r * nb + c) * ntDh + tp) * NA + m + (odd ? half : 0)) + part;
        *base = u + sg * v;
    }
}

// steps 4 + 5 staging, on half ranges of phi: A = u, v of the destination row n' of G2 (samples j
// and j + NPhi/2 of the common phi grid; upward, a G2 box is a z pair of children, already
// combined by the theta step), B = the row's even and odd operator blocks (32 samples each).
template <class R, int KS> struct Rs5Stage {
    using C = typename cpx<R>::type;
    static constexpr int QA = KS / 8, QB = KS / 16;
    int tid, H, hp, ld, j0;   // H = NPhi/2; hp, ld: half the destination row length, its stride
    int64_t cb, ce;
    const R* D;               // the row's operator block
    // row n' of this thread's tile rows (fixed over the slabs)
    const C* g[QA];
    C rl[QA], rh[QA];
    V4<R> rb[QB];
    bool oka[QA], okb[QB];
    __device__ void init(const C* G2, int64_t nb, int64_t r, int ntDh, int row)
    {
        const uint32_t bs = (uint32_t)ntDh * (2 * H);   // box stride
        const C* g0 = G2 + (int64_t)row * (2 * H);
        const uint32_t rb0 = (uint32_t)(r * nb);
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int64_t c = min(cb + (tid + NT * q) / KS, ce - 1);
            g[q] = g0 + (uint64_t)(rb0 + (uint32_t)c) * bs;
        }
    }
    __device__ void load(int k0)
    {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q, kk = e % KS, bc = e / KS;
            const int k = min(k0 + kk, H - 1);
            rl[q] = g[q][k];
            rh[q] = g[q][k + H];
            oka[q] = k0 + kk < H && cb + bc < ce;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q, kr = k0 + (e >> 4), c4 = 4 * (e & 15), jp = j0 + (c4 & 31);
            rb[q] = V4<R>::ld(D + ((int64_t)min(kr, H - 1) * 2 + (c4 >> 5)) * ld + (jp < ld ? jp : 0));
            okb[q] = kr < H && jp < hp;
        }
    }
    __device__ void store(R* As, R* Bs)
    {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            const C x = rl[q], y = rh[q];
            const bool ok = oka[q];
            const int o = (e % KS) * MAP + 2 * (e / KS);
            *(C*)&As[o] = cx<R>(ok ? x.x + y.x : R(0), ok ? x.y + y.y : R(0));
            *(C*)&As[KS * MAP + o] = cx<R>(ok ? x.x - y.x : R(0), ok ? x.y - y.y : R(0));
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q;
            rb[q].st(&Bs[(e >> 4) * MBP + 4 * (e & 15)], okb[q]);
        }
    }
};

// Block (tile, destination row n', 32 samples j0.. of the first half of the row): samples j' and
// j' + N'_phi,n'/2. UP: tiles of whole parents' z pairs (tile_begin/tile_end over the pairs,
// zstart/zcount each parent's pairs); DOWN: tiles of 32 consecutive child boxes.
template <class R, bool UP, int KS>
__global__ __launch_bounds__(NT) void rs5_mfma(
    int64_t nb, int NA, int ntD, int ntj, const int32_t* __restrict__ row_off, const int32_t* __restrict__ nphi,
    const R* __restrict__ d5h, const int32_t* __restrict__ d5h_off, const typename cpx<R>::type* __restrict__ G2,
    int Kd, const int32_t* __restrict__ tile_begin, const int32_t* __restrict__ tile_end,
    const int32_t* __restrict__ tile_pbeg, const int32_t* __restrict__ tile_pend,
    const int32_t* __restrict__ zoct, const int32_t* __restrict__ zstart,
    const int32_t* __restrict__ zcount, const typename cpx<R>::type* __restrict__ trans, int64_t nb_out,
    typename cpx<R>::type* __restrict__ out)
{
    using C = typename cpx<R>::type;
    using T = MT<R>;
    const int row = blockIdx.y / ntj, j0 = (blockIdx.y % ntj) * (MN / 2);
    const int64_t r = blockIdx.z;
    const int len = nphi[row], hp = len / 2, off = row_off[row];
    if (j0 >= hp) return;
    int64_t cb, ce;
    if (UP) {
        cb = tile_begin[blockIdx.x];
        ce = tile_end[blockIdx.x];
    } else {
        cb = (int64_t)blockIdx.x * BC;
        ce = min(cb + BC, nb);
    }
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    // one LDS array: the A and B slabs during the contraction, then the tile for the exchange of
    // the even and odd parts, then (upward) the translated pairs (32 x 64 complex) for the sums
    // over each parent's pairs
    constexpr int kL = 2 * KS * MAP + KS * MBP > MM * MN ? 2 * KS * MAP + KS * MBP : MM * MN;
    __shared__ __align__(16) R Ls[kL];
    __shared__ int pz[2][BC];   // upward: zstart - cb and zcount of the tile's parents
    R* As = Ls;
    R* Bs = Ls + 2 * KS * MAP;
    Rs5Stage<R, KS> st;
    st.tid = tid;
    st.H = NA / 2;
    st.hp = hp;
    st.ld = (hp + 3) & ~3;
    st.j0 = j0;
    st.cb = cb;
    st.ce = ce;
    st.D = d5h + d5h_off[row];
    st.init(G2, nb, r, ntD / 2 + 1, row);
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
    typename T::acc_t acc = {};
    mfma_mainloop<R, KS>(st, As, Bs, NA / 2, acc, wr, wc, lane);
    // this thread's outputs: sample i of the half hh (j' = j0 + i + hh hp) of boxes
    // (tid >> 6) + 4 it, it < 8
    const int i = tid & 31, hh = (tid >> 5) & 1;
    const bool col_ok = j0 + i < hp;
    const int jp = min(j0 + i, hp - 1) + (hh ? hp : 0);
    const R sg = hh ? R(-1) : R(1);
    C ev[8];
    if (!UP) {
        // add to I: the eight reads are issued before the exchange (boxes clamped into the tile)
        C* o = out + off + jp;
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int64_t c = min(cb + (tid >> 6) + 4 * it, ce - 1);
            ev[it] = o[(uint64_t)(rbo + (uint32_t)c) * (uint32_t)Kd];
        }
        tile_to_lds<R>(Ls, acc, wr, wc, lane);
        __syncthreads();
        if (!col_ok) return;
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int b = (tid >> 6) + 4 * it;
            if (cb + b >= ce) break;
            const C v = tile_out<R>(Ls, b, i, sg);
            o[(uint64_t)(rbo + (uint32_t)(cb + b)) * (uint32_t)Kd] = cx<R>(ev[it].x + v.x, ev[it].y + v.y);
        }
        return;
    }
    {
        // the octant of each output's pair, then its translation: all loads issued before use
        int oc[8];
#pragma unroll
        for (int it = 0; it < 8; ++it) oc[it] = zoct[min(cb + (tid >> 6) + 4 * it, ce - 1)];
        const C* tr = trans + off + jp;
#pragma unroll
        for (int it = 0; it < 8; ++it) ev[it] = tr[(uint32_t)oc[it] * (uint32_t)Kd];
    }
    tile_to_lds<R>(Ls, acc, wr, wc, lane);
    __syncthreads();
    // UP: translate each pair on the parent grid, then sum the pairs of every parent
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        const int b = (tid >> 6) + 4 * it;
        const C v = tile_out<R>(Ls, b, i, sg), t = ev[it];
        const bool ok = col_ok && cb + b < ce;
        ev[it] = cx<R>(ok ? v.x * t.x - v.y * t.y : R(0), ok ? v.x * t.y + v.y * t.x : R(0));
    }
    __syncthreads();   // every exchange value is read
    C* S = (C*)Ls;     // 32 x 64 complex: [pair in tile][hh * 32 + i]
#pragma unroll
    for (int it = 0; it < 8; ++it) S[((tid >> 6) + 4 * it) * MN + hh * 32 + i] = ev[it];
    __syncthreads();
    for (int e = tid; e < MN * npar; e += NT) {
        const int c64 = e % MN, pi = e / MN, ii = c64 & 31;
        if (j0 + ii >= hp) continue;
        const int a = pz[0][pi], cnt = pz[1][pi];
        C sum = cx<R>(R(0), R(0));
        for (int c = a; c < a + cnt; ++c) {
            const C v = S[c * MN + c64];
            sum.x += v.x;
            sum.y += v.y;
        }
        out[(uint64_t)(rbo + (uint32_t)(p0 + pi)) * (uint32_t)Kd + off + j0 + ii + (c64 >> 5) * hp] = sum;
    }
}

// steps 4 + 5 on quarter ranges: A = the destination row n' of G2 (samples m, m + NPhi/2,
// NPhi/2 - m, -m of the common phi grid; upward a G2 box is a z pair), B = the row's quarter-range
// operator block.
template <class R, int KS> struct Rs5QStage {
    using C = typename cpx<R>::type;
    static constexpr int QA = KS / 8, QB = KS / 8;
    int tid, NA, H, q, ld, j0, Qp1;   // q = NPhi/4; Qp1 = N'_phi,n'/4 + 1, ld its stride
    int64_t cb, ce;
    const R* D;
    const C* g[QA];
    C ra[QA][4];
    V4<R> rb[QB];
    bool oka[QA], okb[QB];
    __device__ void init(const C* G2, int64_t nb, int64_t r, int ntDh, int row)
    {
        const uint32_t bs = (uint32_t)ntDh * NA;   // box stride
        const C* g0 = G2 + (int64_t)row * NA;
        const uint32_t rb0 = (uint32_t)(r * nb);
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            const int64_t c = min(cb + (tid + NT * u) / KS, ce - 1);
            g[u] = g0 + (uint64_t)(rb0 + (uint32_t)c) * bs;
        }
    }
    __device__ void load(int k0)
    {
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            const int e = tid + NT * u, kk = e % KS, bc = e / KS;
            const int m = min(k0 + kk, q);
            const int i[4] = {m, m + H, H - m, m == 0 ? 0 : NA - m};
#pragma unroll
            for (int a = 0; a < 4; ++a) ra[u][a] = g[u][i[a]];
            oka[u] = k0 + kk <= q && cb + bc < ce;
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            const int e = tid + NT * u, kr = k0 + (e >> 5), c4 = 4 * (e & 31), j = j0 + (c4 & 31);
            rb[u] = V4<R>::ld(D + ((int64_t)min(kr, q) * 4 + (c4 >> 5)) * ld + (j < ld ? j : 0));
            okb[u] = kr <= q && j < Qp1;
        }
    }
    __device__ void store(R* As, R* Bs)
    {
#pragma unroll
        for (int u = 0; u < QA; ++u) {
            const int e = tid + NT * u;
            quarter_channels<R>(ra[u][0], ra[u][1], ra[u][2], ra[u][3], oka[u], As, KS * MAP,
                                (e % KS) * MAP + 2 * (e / KS));
        }
#pragma unroll
        for (int u = 0; u < QB; ++u) {
            const int e = tid + NT * u;
            rb[u].st(&Bs[(e >> 5) * MQ + 4 * (e & 31)], okb[u]);
        }
    }
};

// Block (tile, destination row n', output indices j0.. j0 + 31 of 0..N'_phi,n'/4): samples j',
// j' + N'/2, N'/2 - j' and N' - j' of the row. UP: tiles of whole parents' z pairs, the translated
// pairs summed per parent in LDS; DOWN: tiles of 32 children, added to I.
template <class R, bool UP, int KS>
__global__ __launch_bounds__(NT) void rs5q_mfma(
    int64_t nb, int NA, int ntD, int ntj, const int32_t* __restrict__ row_off, const int32_t* __restrict__ nphi,
    const R* __restrict__ d5q, const int32_t* __restrict__ d5q_off, const typename cpx<R>::type* __restrict__ G2,
    int Kd, const int32_t* __restrict__ tile_begin, const int32_t* __restrict__ tile_end,
    const int32_t* __restrict__ tile_pbeg, const int32_t* __restrict__ tile_pend,
    const int32_t* __restrict__ zoct, const int32_t* __restrict__ zstart,
    const int32_t* __restrict__ zcount, const typename cpx<R>::type* __restrict__ trans, int64_t nb_out,
    typename cpx<R>::type* __restrict__ out)
{
    using C = typename cpx<R>::type;
    using T = MT<R>;
    const int row = blockIdx.y / ntj, j0 = (blockIdx.y % ntj) * 32;
    const int64_t r = blockIdx.z;
    const int len = nphi[row], Qd = len / 4, Hd = len / 2, off = row_off[row];
    if (j0 > Qd) return;
    int64_t cb, ce;
    if (UP) {
        cb = tile_begin[blockIdx.x];
        ce = tile_end[blockIdx.x];
    } else {
        cb = (int64_t)blockIdx.x * BC;
        ce = min(cb + BC, nb);
    }
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    // one LDS array: the slabs, then the exchange tile, then (upward) the translated pairs
    // (32 x 128 complex: the four outputs of 32 indices) for the sums over each parent's pairs
    constexpr int kL = 4 * KS * MAP + KS * MQ > MM * MQ ? 4 * KS * MAP + KS * MQ : MM * MQ;
    __shared__ __align__(16) R Ls[kL];
    __shared__ int pz[2][BC];
    R* As = Ls;
    R* Bs = Ls + 4 * KS * MAP;
    Rs5QStage<R, KS> st;
    st.tid = tid;
    st.NA = NA;
    st.H = NA / 2;
    st.q = NA / 4;
    st.Qp1 = Qd + 1;
    st.ld = (Qd + 1 + 3) & ~3;
    st.j0 = j0;
    st.cb = cb;
    st.ce = ce;
    st.D = d5q + d5q_off[row];
    st.init(G2, nb, r, ntD / 2 + 1, row);
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
    typename T::acc_t acc[2] = {};
    mfma_mainloop_q<R, KS>(st, As, Bs, NA / 4 + 1, acc, wr, wc, lane);
    // this thread's index jj (j' = j0 + jj) for boxes (tid >> 5) + 8 it, it < 4: outputs at
    // j', j' + N'/2 and, for 0 < j' < N'/4, N'/2 - j' and N' - j'
    const int jj = tid & 31, j = min(j0 + jj, Qd);
    const bool col_ok = j0 + jj <= Qd, inner = j > 0 && j < Qd;
    const int pos[4] = {j, j + Hd, inner ? Hd - j : j, inner ? len - j : j + Hd};
    C ev[4][4];
    if (!UP) {
        // add to I: the reads issued before the exchange (boxes clamped into the tile)
        C* o = out + off;
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int64_t c = min(cb + (tid >> 5) + 8 * it, ce - 1);
#pragma unroll
            for (int a = 0; a < 4; ++a) ev[it][a] = o[(uint64_t)(rbo + (uint32_t)c) * (uint32_t)Kd + pos[a]];
        }
        tile_to_lds_q<R>(Ls, acc, wr, wc, lane);
        __syncthreads();
        if (!col_ok) return;
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int b = (tid >> 5) + 8 * it;
            if (cb + b >= ce) break;
            C y[4];
            tile_out_q<R>(Ls, b, jj, y);
            C* ob = o + (uint64_t)(rbo + (uint32_t)(cb + b)) * (uint32_t)Kd;
#pragma unroll
            for (int a = 0; a < 4; ++a)
                if (a < 2 || inner) ob[pos[a]] = cx<R>(ev[it][a].x + y[a].x, ev[it][a].y + y[a].y);
        }
        return;
    }
    {
        // the octant of each output's pair, then its translations: all loads issued before use
        int oc[4];
#pragma unroll
        for (int it = 0; it < 4; ++it) oc[it] = zoct[min(cb + (tid >> 5) + 8 * it, ce - 1)];
        const C* tr = trans + off;
#pragma unroll
        for (int it = 0; it < 4; ++it)
#pragma unroll
            for (int a = 0; a < 4; ++a) ev[it][a] = tr[(uint32_t)oc[it] * (uint32_t)Kd + pos[a]];
    }
    tile_to_lds_q<R>(Ls, acc, wr, wc, lane);
    __syncthreads();
    // UP: translate each pair on the parent grid, then sum the pairs of every parent
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        const int b = (tid >> 5) + 8 * it;
        C y[4];
        tile_out_q<R>(Ls, b, jj, y);
        const bool ok = col_ok && cb + b < ce;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const C t = ev[it][a];
            ev[it][a] = cx<R>(ok ? y[a].x * t.x - y[a].y * t.y : R(0), ok ? y[a].x * t.y + y[a].y * t.x : R(0));
        }
    }
    __syncthreads();   // every exchange value is read
    C* S = (C*)Ls;     // 32 x 128 complex: [pair in tile][a * 32 + jj]
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
        for (int a = 0; a < 4; ++a) S[((tid >> 5) + 8 * it) * MQ + a * 32 + jj] = ev[it][a];
    __syncthreads();
    for (int e = tid; e < MQ * npar; e += NT) {
        const int c128 = e % MQ, pi = e / MQ, a = c128 >> 5, jx = j0 + (c128 & 31);
        if (jx > Qd || (a >= 2 && (jx == 0 || jx == Qd))) continue;
        const int p = a == 0 ? jx : a == 1 ? jx + Hd : a == 2 ? Hd - jx : len - jx;
        const int a0 = pz[0][pi], cnt = pz[1][pi];
        C sum = cx<R>(R(0), R(0));
        for (int c = a0; c < a0 + cnt; ++c) {
            const C v = S[c * MQ + c128];
            sum.x += v.x;
            sum.y += v.y;
        }
        out[(uint64_t)(rbo + (uint32_t)(p0 + pi)) * (uint32_t)Kd + off + p] = sum;
    }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

// Tiles of the upward pass: consecutive whole parents, at most 32 entries per tile (the box rows
// of one block tile), from each parent's entry count.
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

// runs f(KsTag<KS>{}) for the slab depth ks (16, 32 or 64; FP64 at most 32, whose 64-deep slabs
// would exceed a block's LDS)
template <class R, class F> void with_ks(int ks, F&& f)
{
    if (ks == 16)
        f(KsTag<16>{});
    else if (ks == 32 || sizeof(R) == 8)
        f(KsTag<32>{});
    else
        f(KsTag<64>{});
}

// the quarter-range kernels: FP32 slabs of 16 or 32, FP64 of 16 (their exchange tile and four A
// slabs would exceed a block's LDS budget beyond)
template <class R, class F> void with_ks_q(int ks, F&& f)
{
    if constexpr (sizeof(R) == 8)
        f(KsTag<16>{});
    else if (ks == 16)
        f(KsTag<16>{});
    else
        f(KsTag<32>{});
}

template <class R>
void run_resample_quarter(ffmm_plan* p, int l_src, int l_dst, int nrhs, hipStream_t s, bool step1)
{
    using C = typename cpx<R>::type;
    const bool up = l_dst == l_src - 1;
    Resampler& rs = up ? p->up[l_src] : p->down[l_src];
    LevelData& S = p->lev[l_src];
    LevelData& D = p->lev[l_dst];
    LevelData& Cl = up ? S : D;
    C* G1 = (C*)p->scratch1;
    C* G2 = (C*)p->scratch2;
    const int NA = rs.nphi_all;
    const int64_t nb = Cl.n;
    if (step1) {
        const int ntj = cdiv(NA / 4 + 1, 32);
        if (up) {
            dim3 grid(cdiv(nb, BC), ntj * rs.rows_src, nrhs);
            with_ks_q<R>(p->tune.rs_slab[0], [&](auto t) {
                hipLaunchKernelGGL((rs1q_mfma<R, false, decltype(t)::value>), grid, dim3(NT), 0, s, nb, nb,
                                   rs.rows_src, NA, rs.ldq, ntj, rs.d_src_row_off, rs.d_src_nphi,
                                   (const R*)rs.d1q, rs.d1q_off, (const C*)S.sigM, S.K, S.n,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, (const int32_t*)nullptr,
                                   (const C*)nullptr, G1);
            });
        } else {
            dim3 grid(cdiv(Cl.nz, BC), ntj * rs.rows_src, nrhs);
            with_ks_q<R>(p->tune.rs_slab[0], [&](auto t) {
                hipLaunchKernelGGL((rs1q_mfma<R, true, decltype(t)::value>), grid, dim3(NT), 0, s, Cl.nz, nb,
                                   rs.rows_src, NA, rs.ldq, ntj, rs.d_src_row_off, rs.d_src_nphi,
                                   (const R*)rs.d1q, rs.d1q_off, (const C*)S.sigL, S.K, S.n, Cl.zpar, Cl.zoct,
                                   Cl.zlo, (const C*)S.trans, G1);
            });
        }
        FFMM_LAUNCH_CHECK();
        return;
    }
    int mx = 0;
    for (int v : D.par.nphi) mx = std::max(mx, v);
    const int ntj = cdiv(mx / 4 + 1, 32);
    if (up) {
        dim3 grid((unsigned)rs.nztiles, ntj * rs.rows_dst, nrhs);
        with_ks_q<R>(p->tune.rs_slab[2], [&](auto t) {
            hipLaunchKernelGGL((rs5q_mfma<R, true, decltype(t)::value>), grid, dim3(NT), 0, s, Cl.nz, NA,
                               rs.nt_dst, ntj, rs.d_dst_row_off, rs.d_dst_nphi, (const R*)rs.d5q, rs.d5q_off,
                               (const C*)G2, D.K, rs.ztile_begin, rs.ztile_end, rs.ztile_pbeg, rs.ztile_pend,
                               Cl.zoct, D.zstart, D.zcount, (const C*)D.trans, D.n, (C*)D.sigM);
        });
    } else {
        dim3 grid(cdiv(nb, BC), ntj * rs.rows_dst, nrhs);
        with_ks_q<R>(p->tune.rs_slab[3], [&](auto t) {
            hipLaunchKernelGGL((rs5q_mfma<R, false, decltype(t)::value>), grid, dim3(NT), 0, s, nb, NA,
                               rs.nt_dst, ntj, rs.d_dst_row_off, rs.d_dst_nphi, (const R*)rs.d5q, rs.d5q_off,
                               (const C*)G2, D.K, (const int32_t*)nullptr, (const int32_t*)nullptr,
                               (const int32_t*)nullptr, (const int32_t*)nullptr, (const int32_t*)nullptr,
                               (const int32_t*)nullptr, (const int32_t*)nullptr, (const C*)nullptr, D.n,
                               (C*)D.sigL);
        });
    }
    FFMM_LAUNCH_CHECK();
}

template <class R>
void run_resample_mfma(ffmm_plan* p, int l_src, int l_dst, int nrhs, hipStream_t s)
{
    using C = typename cpx<R>::type;
    const bool up = l_dst == l_src - 1;
    Resampler& rs = up ? p->up[l_src] : p->down[l_src];
    LevelData& S = p->lev[l_src];
    LevelData& D = p->lev[l_dst];
    LevelData& Cl = up ? S : D;
    C* G1 = (C*)p->scratch1;
    C* G2 = (C*)p->scratch2;
    const int NA = rs.nphi_all;
    const int64_t nb = Cl.n;
    if (rs.quarter) {
        run_resample_quarter<R>(p, l_src, l_dst, nrhs, s, true);
    } else {
        const int ntj = cdiv(NA / 2, MN / 2);   // 32-sample tiles of the first half of the phi grid
        if (up) {
            dim3 grid(cdiv(nb, BC), ntj * rs.rows_src, nrhs);
            with_ks<R>(p->tune.rs_slab[0], [&](auto t) {
                hipLaunchKernelGGL((rs1_mfma<R, false, decltype(t)::value>), grid, dim3(NT), 0, s, nb, nb,
                                   rs.rows_src, NA, rs.ldj, ntj, rs.d_src_row_off, rs.d_src_nphi, (const R*)rs.d1h,
                                   (const C*)S.sigM, S.K, S.n, (const int32_t*)nullptr,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, (const C*)nullptr, G1);
            });
        } else {
            // one contraction per z pair of children
            dim3 grid(cdiv(Cl.nz, BC), ntj * rs.rows_src, nrhs);
            with_ks<R>(p->tune.rs_slab[0], [&](auto t) {
                hipLaunchKernelGGL((rs1_mfma<R, true, decltype(t)::value>), grid, dim3(NT), 0, s, Cl.nz, nb,
                                   rs.rows_src, NA, rs.ldj, ntj, rs.d_src_row_off, rs.d_src_nphi, (const R*)rs.d1h,
                                   (const C*)S.sigL, S.K, S.n, Cl.zpar, Cl.zoct, Cl.zlo, (const C*)S.trans,
                                   G1);
            });
        }
        FFMM_LAUNCH_CHECK();
    }
    {
        const int ntSh = rs.nt_src / 2 + 1, ntDh = rs.nt_dst / 2 + 1;
        const int ny = cdiv(ntDh, MM / 2);
        // one column per child and phi_m < NPhi/2 (upward ordered by z pair)
        dim3 grid(cdiv(nb * (NA / 2), MN / 2) * ny, 1, nrhs);
        with_ks<R>(p->tune.rs_slab[1], [&](auto t) {
            if (up)
                hipLaunchKernelGGL((rs3h_mfma<R, decltype(t)::value, false, true>), grid, dim3(NT), 0, s,
                                   Cl.nz, nb, NA, rs.rows_src, ntSh, ntDh, rs.ldh, ny, (const R*)rs.dth_h,
                                   (const int32_t*)nullptr, Cl.zlo, Cl.zhi, Cl.zmp, rs.zcol_tile,
                                   (const C*)D.zrot, (const C*)G1, G2);
            else
                hipLaunchKernelGGL((rs3h_mfma<R, decltype(t)::value, true, false>), grid, dim3(NT), 0, s, nb,
                                   nb, NA, rs.rows_src, ntSh, ntDh, rs.ldh, ny, (const R*)rs.dth_h, Cl.zsrc,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, (const int32_t*)nullptr,
                                   (const int32_t*)nullptr, (const C*)S.zrot, (const C*)G1, G2);
        });
        FFMM_LAUNCH_CHECK();
    }
    if (rs.quarter) {
        run_resample_quarter<R>(p, l_src, l_dst, nrhs, s, false);
    } else {
        int mx = 0;
        for (int v : D.par.nphi) mx = std::max(mx, v);
        const int ntj = cdiv(mx / 2, MN / 2);   // 32-sample tiles of the first half of the longest row
        if (up) {
            // tiles of whole parents' z pairs
            dim3 grid((unsigned)rs.nztiles, ntj * rs.rows_dst, nrhs);
            with_ks<R>(p->tune.rs_slab[2], [&](auto t) {
                hipLaunchKernelGGL((rs5_mfma<R, true, decltype(t)::value>), grid, dim3(NT), 0, s, Cl.nz,
                                   NA, rs.nt_dst, ntj, rs.d_dst_row_off, rs.d_dst_nphi, (const R*)rs.d5h,
                                   rs.d5h_off, (const C*)G2, D.K, rs.ztile_begin, rs.ztile_end, rs.ztile_pbeg,
                                   rs.ztile_pend, Cl.zoct, D.zstart, D.zcount, (const C*)D.trans, D.n,
                                   (C*)D.sigM);
            });
        } else {
            dim3 grid(cdiv(nb, BC), ntj * rs.rows_dst, nrhs);
            with_ks<R>(p->tune.rs_slab[3], [&](auto t) {
                hipLaunchKernelGGL((rs5_mfma<R, false, decltype(t)::value>), grid, dim3(NT), 0, s, nb, NA,
                                   rs.nt_dst, ntj, rs.d_dst_row_off, rs.d_dst_nphi, (const R*)rs.d5h,
                                   rs.d5h_off, (const C*)G2, D.K, (const int32_t*)nullptr, (const int32_t*)nullptr,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, (const int32_t*)nullptr,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, (const C*)nullptr, D.n,
                                   (C*)D.sigL);
            });
        }
        FFMM_LAUNCH_CHECK();
    }
}

}  // namespace

void run_resample(ffmm_plan* p, int l_src, int l_dst, int nrhs, hipStream_t s)
{
    if (p->prec == FFMM_FP32)
        run_resample_mfma<float>(p, l_src, l_dst, nrhs, s);
    else
        run_resample_mfma<double>(p, l_src, l_dst, nrhs, s);
}

}  // namespace ffmm
