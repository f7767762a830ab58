// Five-step inter/anterpolation between level quadratures (Section 3.4) for the upward (M2M) and
// downward (L2L) passes. Each 1D step applies one real Fourier-resample matrix (the Dirichlet
// kernel with the Nyquist bin dropped) to a batch of boxes, i.e. a dense contraction
//     Y[i][col] = sum_k D[i][k] X[k][col],
// computed on the matrix cores in the plan precision. Complex data enter as interleaved (re, im)
// real rows or columns.
//   step 1      per source row n:  G1[c][n][j]  = sum_m D1_n[j][m] in_c(n, m),          j < NA
//   steps 2+3   per column m < NA/2, on half ranges of theta (eqn. FourierSphereSym, below)
//   steps 4+5   per destination row n': out_c(n', j') = sum_j D5_n'[j'][j] row_{c,n'}(j)
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
    __device__ static void slab(const float* __restrict__ As, const float* __restrict__ Bs, acc_t& acc, int wr,
                                int wc, int lane, int kc)
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
    __device__ static void slab(const double* __restrict__ As, const double* __restrict__ Bs, acc_t& acc,
                                int wr, int wc, int lane, int kc)
    {
        const int i = lane & 15, kq = lane >> 4, pi = 4 * (i & 3) + (i >> 2);
        for (int k4 = 0; k4 < kc; k4 += 4) {
            const int k = k4 + kq;
            const double a0 = As[k * MAP + wr + pi], a1 = As[k * MAP + wr + 16 + pi];
            const double b0 = Bs[k * MBP + wc + i], b1 = Bs[k * MBP + wc + 16 + i];
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

// Shared main loop over one LDS slab buffer. Stage::load(k0) issues the global loads of the slab
// starting at k0 into registers; Stage::store(As, Bs) writes them (zeroing invalid entries) once
// they have landed. The next slab's loads are in flight during the current slab's MFMAs.
template <class R, int KS, class Stage>
__device__ inline void mfma_mainloop(Stage& st, R* As, R* Bs, int K, typename MT<R>::acc_t& acc, int wr, int wc,
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
        MT<R>::slab(As, Bs, acc, wr, wc, lane, (kc + 7) & ~7);
        if (more) {
            __syncthreads();   // every wave is done with this slab
            st.store(As, Bs);
        }
        __syncthreads();
    }
}

// step 1 staging: A = source row data of 32 boxes, or in the downward pass of 32 z pairs (lo, hi)
// of children: the parent's data times conj(E_oct(lo)). B = the Dirichlet block of the row.
template <class R, bool DOWN, int KS> struct Rs1Stage {
    using C = typename cpx<R>::type;
    int tid, len, NA, j0;
    int64_t c0, nb;
    const R* d1;
    int off;
    static constexpr int QA = KS / 8, QB = KS / 16, QT = DOWN ? QA : 1;
    // source row n of this thread's tile rows (fixed over the slabs), and downward the row of
    // the translation of lo's octant
    const C* gs[QA];
    const C* gt[QT];
    // load() only issues the loads; store() applies conj(E) once they have landed, so that the
    // next slab's loads stay in flight during the current slab's MFMAs
    C ra[QA], rt[QT];
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
            const int k = min(k0 + kk, len - 1);
            ra[q] = gs[q][k];
            if (DOWN) rt[q] = gt[q][k];
            oka[q] = k0 + kk < len && c0 + bc < nb;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q, kr = k0 + (e >> 4), j = j0 + 4 * (e & 15);
            rb[q] = V4<R>::ld(d1 + (int64_t)(off + min(kr, len - 1)) * NA + (j < NA ? j : 0));
            okb[q] = kr < len && j < NA;
        }
    }
    __device__ void store(R* As, R* Bs)
    {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            C v = ra[q];
            if (DOWN) {
                const C t = rt[q];
                v = cx<R>(v.x * t.x + v.y * t.y, v.y * t.x - v.x * t.y);  // v conj(t)
            }
            const bool ok = oka[q];
            *(C*)&As[(e % KS) * MAP + 2 * (e / KS)] = cx<R>(ok ? v.x : R(0), ok ? v.y : R(0));
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q;
            rb[q].st(&Bs[(e >> 4) * MBP + 4 * (e & 15)], okb[q]);
        }
    }
};

// nt: the tile rows (boxes, or z pairs in the downward pass); nb: the boxes of the G1 layout
template <class R, bool DOWN, int KS>
__global__ __launch_bounds__(NT) void rs1_mfma(int64_t nt, int64_t nb, int rows, int NA, int ntj,
                                               const int32_t* __restrict__ row_off,
                                               const int32_t* __restrict__ nphi, const R* __restrict__ d1,
                                               const typename cpx<R>::type* __restrict__ sig, int Ksrc,
                                               int64_t nb_in, const int32_t* __restrict__ zpar,
                                               const int32_t* __restrict__ zoct,
                                               const int32_t* __restrict__ zlo,
                                               const typename cpx<R>::type* __restrict__ trans,
                                               typename cpx<R>::type* __restrict__ G1)
{
    using C = typename cpx<R>::type;
    using T = MT<R>;
    const int row = blockIdx.y / ntj, j0 = (blockIdx.y % ntj) * MN;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    __shared__ __align__(16) R As[KS * MAP];
    __shared__ __align__(16) R Bs[KS * MBP];
    Rs1Stage<R, DOWN, KS> st;
    st.tid = tid;
    st.len = nphi[row];
    st.off = row_off[row];
    st.NA = NA;
    st.j0 = j0;
    st.c0 = (int64_t)blockIdx.x * BC;
    st.nb = nt;
    st.d1 = d1;
    st.init(sig, Ksrc, nb_in, blockIdx.z, zpar, zoct, trans);
    typename T::acc_t acc = {};
    mfma_mainloop<R, KS>(st, As, Bs, st.len, acc, wr, wc, lane);
    const uint32_t rb0 = (uint32_t)(blockIdx.z * nb), bs = (uint32_t)rows * NA;   // box stride
    C* g = G1 + (int64_t)row * NA + j0 + wc;
    if (!DOWN) {
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int64_t c = st.c0 + wr / 2 + T::rbox(lane, p);
            const int col = T::rcol(lane, p);
            if (c < nt && j0 + wc + col < NA)
                g[(uint64_t)(rb0 + (uint32_t)c) * bs + col] = cx<R>(T::re(acc, p), T::im(acc, p));
        }
        return;
    }
    // lo's result only: hi's is lo's times conj(rho(n)), which the theta step applies as it reads
    // lo's rows for hi; the pair indices are loaded first
    int lo[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) lo[p] = zlo[min(st.c0 + wr / 2 + T::rbox(lane, p), nt - 1)];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int col = T::rcol(lane, p);
        if (st.c0 + wr / 2 + T::rbox(lane, p) >= nt || j0 + wc + col >= NA) continue;
        g[(uint64_t)(rb0 + (uint32_t)lo[p]) * bs + col] = cx<R>(T::re(acc, p), T::im(acc, p));
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
// PAIR (upward pass): the columns are (z pair, phi_m, member), the two members of a pair adjacent
// (a pair without an upper member has a zero column there), and each G2 row is written per pair:
// row(lo) + rho(n') row(hi) on destination row n' (zrot of the destination level), the sum that
// step 5 resamples and translates with lo's octant. nb then counts the pairs (G2 layout) and
// nbox the children (G1 layout).
template <class R, int KS, bool ZP, bool PAIR>
__global__ __launch_bounds__(NT) void rs3h_mfma(int64_t nb, int64_t nbox, int NA, int rowsS, int ntSh, int ntDh,
                                                int ldh, int ny, const R* __restrict__ dh,
                                                const int32_t* __restrict__ zsrc,
                                                const int32_t* __restrict__ zlo,
                                                const int32_t* __restrict__ zhi,
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
    const int64_t ncols = (PAIR ? 2 : 1) * nb * half;
    const int64_t g0 = (int64_t)(lb / (unsigned)ny) * (MN / 2);
    // first (box, column) of the tile; with PAIR, first (pair, column) of the tile's column pairs
    const int64_t cbase = (PAIR ? g0 / 2 : g0) / half;
    const int m0 = (int)((PAIR ? g0 / 2 : g0) - cbase * half);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const bool odd = wr != 0;
    const int64_t mat_off = (int64_t)ntSh * ldh;   // Do after De
    // this thread's staged column (phi_m of its box), row 0
    const C* sbase;
    bool scol_ok, zconj = false;
    {
        const int cc = tid & 31;
        int m = m0 + (PAIR ? cc / 2 : cc);
        int64_t c = cbase;
        while (m >= half) {
            m -= half;
            ++c;
        }
        scol_ok = g0 + cc < ncols;
        if (PAIR && scol_ok) {
            // the pair's member of this column (lo on even columns, hi on odd ones)
            c = (cc & 1) ? zhi[c] : zlo[c];
            scol_ok = c >= 0;
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
        // per (destination row, column pair, half of the phi grid): the pair's sample
        // row(lo) + rho row(hi); thread t takes outputs t, t + 256, .. of 32 x 16 x 2
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = tid + NT * i, pc = o & 15, hh = (o >> 4) & 1, tr = o >> 5;
            const int tp = i0 + tr;
            if (g0 + 2 * pc >= ncols || tp >= ntDh) continue;
            int m = m0 + pc;
            int64_t c = cbase;
            while (m >= half) {
                m -= half;
                ++c;
            }
            const R sg = hh ? R(-1) : R(1);
            const R* ur = Ls + tr * MN + 4 * pc;          // u' row: lo (re, im), hi (re, im)
            const R* vr = Ls + (32 + tr) * MN + 4 * pc;   // v' row
            const R lx = ur[0] + sg * vr[0], ly = ur[1] + sg * vr[1];
            const R hx = ur[2] + sg * vr[2], hy = ur[3] + sg * vr[3];
            const C z = zrot[tp];
            G2[((r * nb + c) * ntDh + tp) * NA + m + (hh ? half : 0)] =
                cx<R>(lx + z.x * hx - z.y * hy, ly + z.x * hy + z.y * hx);
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

// steps 4 + 5 staging: A = the destination row n' of G2 (on the common phi grid; upward, a G2
// box is a z pair of children, already combined by the theta step), B = the Dirichlet block of
// the destination row.
template <class R, int KS> struct Rs5Stage {
    using C = typename cpx<R>::type;
    static constexpr int QA = KS / 8, QB = KS / 16;
    int tid, NA, len, j0;
    int64_t cb, ce;
    const R* D;
    // row n' of this thread's tile rows (fixed over the slabs)
    const C* g[QA];
    C rl[QA];
    V4<R> rb[QB];
    bool oka[QA], okb[QB];
    __device__ void init(const C* G2, int64_t nb, int64_t r, int ntDh, int row)
    {
        const uint32_t bs = (uint32_t)ntDh * NA;   // box stride
        const C* g0 = G2 + (int64_t)row * NA;
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
            rl[q] = g[q][min(k0 + kk, NA - 1)];
            oka[q] = k0 + kk < NA && cb + bc < ce;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q, j = k0 + (e >> 4), jp = j0 + 4 * (e & 15);
            rb[q] = V4<R>::ld(D + (int64_t)min(j, NA - 1) * len + (jp < len ? jp : 0));
            okb[q] = j < NA && jp < len;
        }
    }
    __device__ void store(R* As, R* Bs)
    {
#pragma unroll
        for (int q = 0; q < QA; ++q) {
            const int e = tid + NT * q;
            const bool ok = oka[q];
            *(C*)&As[(e % KS) * MAP + 2 * (e / KS)] = cx<R>(ok ? rl[q].x : R(0), ok ? rl[q].y : R(0));
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int e = tid + NT * q;
            rb[q].st(&Bs[(e >> 4) * MBP + 4 * (e & 15)], okb[q]);
        }
    }
};

// UP: tiles of whole parents' z pairs (tile_begin/tile_end over the pairs, zstart/zcount each
// parent's pairs); DOWN: tiles of 32 consecutive child boxes.
template <class R, bool UP, int KS>
__global__ __launch_bounds__(NT) void rs5_mfma(
    int64_t nb, int NA, int ntD, int ntj, const int32_t* __restrict__ row_off, const int32_t* __restrict__ nphi,
    const R* __restrict__ d5, const typename cpx<R>::type* __restrict__ G2, int Kd,
    const int32_t* __restrict__ tile_begin, const int32_t* __restrict__ tile_end,
    const int32_t* __restrict__ tile_pbeg, const int32_t* __restrict__ tile_pend,
    const int32_t* __restrict__ zoct, const int32_t* __restrict__ zstart,
    const int32_t* __restrict__ zcount, const typename cpx<R>::type* __restrict__ trans, int64_t nb_out,
    typename cpx<R>::type* __restrict__ out)
{
    using C = typename cpx<R>::type;
    using T = MT<R>;
    const int row = blockIdx.y / ntj, j0 = (blockIdx.y % ntj) * MN;
    const int64_t r = blockIdx.z;
    const int len = nphi[row], off = row_off[row];
    if (j0 >= len) return;
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
    // one LDS array: the A and B slabs during the contraction, then (upward) the translated
    // pairs (32 x 64 complex) for the sums over each parent's pairs
    constexpr int kL = (UP && KS * (MAP + MBP) < 2 * BC * MN) ? 2 * BC * MN : KS * (MAP + MBP);
    __shared__ __align__(16) R Ls[kL];
    __shared__ int pz[2][BC];   // upward: zstart - cb and zcount of the tile's parents
    R* As = Ls;
    R* Bs = Ls + KS * MAP;
    Rs5Stage<R, KS> st;
    st.tid = tid;
    st.NA = NA;
    st.len = len;
    st.j0 = j0;
    st.cb = cb;
    st.ce = ce;
    st.D = d5 + (int64_t)off * NA;
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
    mfma_mainloop<R, KS>(st, As, Bs, NA, acc, wr, wc, lane);
    C ev[8];
    if (!UP) {
        // add to I: the eight reads are issued before any write (columns clamped into the row)
        C* o = out + off;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int64_t c = min(cb + wr / 2 + T::rbox(lane, p), ce - 1);
            ev[p] = o[(uint64_t)(rbo + (uint32_t)c) * (uint32_t)Kd + min(j0 + wc + T::rcol(lane, p), len - 1)];
        }
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int64_t c = cb + wr / 2 + T::rbox(lane, p);
            const int jp = j0 + wc + T::rcol(lane, p);
            if (c < ce && jp < len)
                o[(uint64_t)(rbo + (uint32_t)c) * (uint32_t)Kd + jp] =
                    cx<R>(ev[p].x + T::re(acc, p), ev[p].y + T::im(acc, p));
        }
        return;
    }
    {
        // the octant of each result's pair, then its translation: all loads issued before use
        int oc[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) oc[p] = zoct[min(cb + wr / 2 + T::rbox(lane, p), ce - 1)];
        const C* tr = trans + off;
#pragma unroll
        for (int p = 0; p < 8; ++p)
            ev[p] = tr[(uint32_t)oc[p] * (uint32_t)Kd + min(j0 + wc + T::rcol(lane, p), len - 1)];
    }
    // UP: translate each pair on the parent grid, then sum the pairs of every parent (the slabs
    // are free after the main loop's last barrier)
    C* S = (C*)Ls;   // 32 x 64 complex
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int bx = wr / 2 + T::rbox(lane, p), col = wc + T::rcol(lane, p);
        const bool ok = j0 + col < len && cb + bx < ce;
        const C t = ev[p];
        const R x = T::re(acc, p), y = T::im(acc, p);
        S[bx * MN + col] = cx<R>(ok ? x * t.x - y * t.y : R(0), ok ? x * t.y + y * t.x : R(0));
    }
    __syncthreads();
    for (int e = tid; e < MN * npar; e += NT) {
        const int i = e % MN, pi = e / MN;
        const int jj = j0 + i;
        if (jj >= len) continue;
        const int a = pz[0][pi], cnt = pz[1][pi];
        C sum = cx<R>(R(0), R(0));
        for (int c = a; c < a + cnt; ++c) {
            const C v = S[c * MN + i];
            sum.x += v.x;
            sum.y += v.y;
        }
        out[(uint64_t)(rbo + (uint32_t)(p0 + pi)) * (uint32_t)Kd + off + jj] = sum;
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
    {
        const int ntj = cdiv(NA, MN);
        if (up) {
            dim3 grid(cdiv(nb, BC), ntj * rs.rows_src, nrhs);
            with_ks<R>(p->tune.rs_slab[0], [&](auto t) {
                hipLaunchKernelGGL((rs1_mfma<R, false, decltype(t)::value>), grid, dim3(NT), 0, s, nb, nb,
                                   rs.rows_src, NA, ntj, rs.d_src_row_off, rs.d_src_nphi, (const R*)rs.d1,
                                   (const C*)S.sigM, S.K, S.n, (const int32_t*)nullptr,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, (const C*)nullptr, G1);
            });
        } else {
            // one contraction per z pair of children
            dim3 grid(cdiv(Cl.nz, BC), ntj * rs.rows_src, nrhs);
            with_ks<R>(p->tune.rs_slab[0], [&](auto t) {
                hipLaunchKernelGGL((rs1_mfma<R, true, decltype(t)::value>), grid, dim3(NT), 0, s, Cl.nz, nb,
                                   rs.rows_src, NA, ntj, rs.d_src_row_off, rs.d_src_nphi, (const R*)rs.d1,
                                   (const C*)S.sigL, S.K, S.n, Cl.zpar, Cl.zoct, Cl.zlo, (const C*)S.trans,
                                   G1);
            });
        }
        FFMM_LAUNCH_CHECK();
    }
    {
        const int ntSh = rs.nt_src / 2 + 1, ntDh = rs.nt_dst / 2 + 1;
        const int ny = cdiv(ntDh, MM / 2);
        dim3 grid(cdiv(nb * (NA / 2), MN / 2) * ny, 1, nrhs);
        // upward: two columns (the z pair's members) per pair and phi_m
        dim3 gridz(cdiv(2 * Cl.nz * (NA / 2), MN / 2) * ny, 1, nrhs);
        with_ks<R>(p->tune.rs_slab[1], [&](auto t) {
            if (up)
                hipLaunchKernelGGL((rs3h_mfma<R, decltype(t)::value, false, true>), gridz, dim3(NT), 0, s,
                                   Cl.nz, nb, NA, rs.rows_src, ntSh, ntDh, rs.ldh, ny, (const R*)rs.dth_h,
                                   (const int32_t*)nullptr, Cl.zlo, Cl.zhi, (const C*)D.zrot, (const C*)G1, G2);
            else
                hipLaunchKernelGGL((rs3h_mfma<R, decltype(t)::value, true, false>), grid, dim3(NT), 0, s, nb,
                                   nb, NA, rs.rows_src, ntSh, ntDh, rs.ldh, ny, (const R*)rs.dth_h, Cl.zsrc,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, (const C*)S.zrot,
                                   (const C*)G1, G2);
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
            with_ks<R>(p->tune.rs_slab[2], [&](auto t) {
                hipLaunchKernelGGL((rs5_mfma<R, true, decltype(t)::value>), grid, dim3(NT), 0, s, Cl.nz,
                                   NA, rs.nt_dst, ntj, rs.d_dst_row_off, rs.d_dst_nphi, (const R*)rs.d5,
                                   (const C*)G2, D.K, rs.ztile_begin, rs.ztile_end, rs.ztile_pbeg,
                                   rs.ztile_pend, Cl.zoct, D.zstart, D.zcount, (const C*)D.trans, D.n,
                                   (C*)D.sigM);
            });
        } else {
            dim3 grid(cdiv(nb, BC), ntj * rs.rows_dst, nrhs);
            with_ks<R>(p->tune.rs_slab[3], [&](auto t) {
                hipLaunchKernelGGL((rs5_mfma<R, false, decltype(t)::value>), grid, dim3(NT), 0, s, nb, NA,
                                   rs.nt_dst, ntj, rs.d_dst_row_off, rs.d_dst_nphi, (const R*)rs.d5,
                                   (const C*)G2, D.K, (const int32_t*)nullptr, (const int32_t*)nullptr,
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
