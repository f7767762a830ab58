// Plan-time octree on the GPU (Section 2): root cube, Morton keys, stable radix sort, occupied
// boxes of every level, parent/child links, the leaf neighbour list N(B) and the interaction
// lists I(B). Integer work, bit-exact by construction:
//  * root cube: corner lo = per-axis minimum, side S = largest per-axis extent (1 if all points
//    coincide);
//  * per-axis index at 21 bits: min(floor((x - lo) * (2^21 / S)), 2^21 - 1), FP64; a depth-L
//    index is that index shifted right by 21 - L bits (2^21 / S is 2^(21-L) times 2^L / S
//    exactly, so this equals quantising with 2^L / S);
//  * key bit 3b <- x bit b, 3b+1 <- y bit b, 3b+2 <- z bit b; points sorted stably by key;
//  * neighbours: Chebyshev distance <= 1 (the 316 = 7^3 - 3^3 transfer vectors of Section 3.2);
//    I(B): children of the parent's neighbours that are not neighbours of B;
//  * every list sorted by source box index.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace ffmm {

namespace {

constexpr int kWave = 64;

// ------------------------------------------------------------------------------------------
// exclusive scan (int32)
// ------------------------------------------------------------------------------------------
constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

__global__ void scan_tiles(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                           int32_t* __restrict__ tile_sums, int64_t n)
{
    __shared__ int32_t sm[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t sum = 0;
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0;
        sum += v[i];
    }
    sm[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int32_t t = threadIdx.x >= off ? sm[threadIdx.x - off] : 0;
        __syncthreads();
        sm[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t run = sm[threadIdx.x] - sum;  // exclusive prefix of this thread
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < n) out[idx] = run;
        run += v[i];
    }
    if (threadIdx.x == kScanBlock - 1) tile_sums[blockIdx.x] = sm[kScanBlock - 1];
}

__global__ void scan_add(int32_t* __restrict__ out, const int32_t* __restrict__ tile_off, int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int32_t add = tile_off[blockIdx.x];
    for (int i = threadIdx.x; i < kScanTile; i += kScanBlock) {
        int64_t idx = base + i;
        if (idx < n) out[idx] += add;
    }
}

}  // namespace

int64_t exclusive_scan(DeviceArena& tmp, const int32_t* in, int32_t* out, int64_t n, hipStream_t s)
{
    if (n == 0) return 0;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    int32_t* sums = tmp.alloc_n<int32_t>(tiles);
    int32_t* offs = tmp.alloc_n<int32_t>(tiles);
    hipLaunchKernelGGL(scan_tiles, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, in, out, sums, n);
    FFMM_LAUNCH_CHECK();
    int64_t total;
    if (tiles == 1) {
        int32_t t;
        FFMM_HIP(hipMemcpyAsync(&t, sums, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FFMM_HIP(hipStreamSynchronize(s));
        FFMM_HIP(hipMemsetAsync(offs, 0, sizeof(int32_t), s));
        total = t;
    } else {
        total = exclusive_scan(tmp, sums, offs, tiles, s);
    }
    hipLaunchKernelGGL(scan_add, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, out, offs, n);
    FFMM_LAUNCH_CHECK();
    return total;
}

namespace {

// ------------------------------------------------------------------------------------------
// bounding box and validity
// ------------------------------------------------------------------------------------------
constexpr int kBoxBlock = 256;

__global__ void bbox_partial(const double* __restrict__ x, int64_t n, double* __restrict__ part,
                             int32_t* __restrict__ bad)
{
    __shared__ double smin[3][kBoxBlock], smax[3][kBoxBlock];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * kBoxBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBoxBlock) {
        for (int a = 0; a < 3; ++a) {
            double v = x[3 * i + a];
            if (!isfinite(v)) atomicOr(bad, 1);
            mn[a] = fmin(mn[a], v);
            mx[a] = fmax(mx[a], v);
        }
    }
    for (int a = 0; a < 3; ++a) {
        smin[a][threadIdx.x] = mn[a];
        smax[a][threadIdx.x] = mx[a];
    }
    __syncthreads();
    for (int off = kBoxBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int a = 0; a < 3; ++a) {
                smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + off]);
                smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) {
            part[6 * blockIdx.x + a] = smin[a][0];
            part[6 * blockIdx.x + 3 + a] = smax[a][0];
        }
}

// ------------------------------------------------------------------------------------------
// Morton keys
// ------------------------------------------------------------------------------------------
__device__ inline uint64_t spread3(uint64_t v)
{
    // bit b of v -> bit 3b
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ inline uint32_t compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (uint32_t)v;
}

__global__ void morton_keys(const double* __restrict__ x, int64_t n, double lox, double loy,
                            double loz, double scale, uint64_t* __restrict__ keys,
                            int64_t* __restrict__ idx)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {lox, loy, loz};
    uint64_t key = 0;
    for (int a = 0; a < 3; ++a) {
        double t = (x[3 * i + a] - lo[a]) * scale;   // two roundings, no fusion possible
        int64_t q = (int64_t)floor(t);
        q = q < 0 ? 0 : q;
        q = q > ((1 << kMaxDepth) - 1) ? ((1 << kMaxDepth) - 1) : q;
        key |= spread3((uint64_t)q) << a;
    }
    keys[i] = key;
    idx[i] = i;
}

// ------------------------------------------------------------------------------------------
// stable LSD radix sort of (key, index), 8-bit digits, one wave per tile
// ------------------------------------------------------------------------------------------
constexpr int kRadix = 256;
constexpr int kChunks = 16;
constexpr int kSortTile = kWave * kChunks;

__global__ __launch_bounds__(kWave) void radix_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                    int shift, int64_t ntiles,
                                                    int32_t* __restrict__ hist)
{
    __shared__ int32_t h[kRadix];
    for (int d = threadIdx.x; d < kRadix; d += kWave) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int c = 0; c < kChunks; ++c) {
        int64_t i = base + c * kWave + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kWave) hist[(int64_t)d * ntiles + blockIdx.x] = h[d];
}

__global__ __launch_bounds__(kWave) void radix_scatter(
    const uint64_t* __restrict__ keys, const int64_t* __restrict__ vals, int64_t n, int shift,
    int64_t ntiles, const int32_t* __restrict__ offs, uint64_t* __restrict__ okeys,
    int64_t* __restrict__ ovals)
{
    __shared__ int32_t cnt[kRadix];
    for (int d = threadIdx.x; d < kRadix; d += kWave) cnt[d] = offs[(int64_t)d * ntiles + blockIdx.x];
    __syncthreads();
    const int lane = threadIdx.x;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int c = 0; c < kChunks; ++c) {
        int64_t i = base + c * kWave + lane;
        bool valid = i < n;
        uint64_t key = valid ? keys[i] : 0;
        int64_t val = valid ? vals[i] : 0;
        uint32_t d = (uint32_t)((key >> shift) & (kRadix - 1));
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bb : ~bb;
        }
        int rank = __popcll(peers & lt);
        int total = __popcll(peers);
        int pos = 0;
        if (valid) pos = cnt[d] + rank;
        __syncthreads();
        if (valid && rank == 0) cnt[d] += total;
        __syncthreads();
        if (valid) {
            okeys[pos] = key;
            ovals[pos] = val;
        }
    }
}

// flag[L] = 1 if some depth-L leaf holds more than m points (sorted keys: a run longer than m
// exists iff key_L[i] == key_L[i + m] for some i).
__global__ void occupancy_flags(const uint64_t* __restrict__ keys, int64_t n, int m,
                                int32_t* __restrict__ flags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i + m >= n) return;
    uint64_t a = keys[i], b = keys[i + m];
    for (int L = 2; L <= kMaxDepth; ++L) {
        int sh = 3 * (kMaxDepth - L);
        if ((a >> sh) == (b >> sh)) flags[L] = 1;
    }
}

__global__ void gather_points(const double* __restrict__ x, const int64_t* __restrict__ perm,
                              int64_t n, double* __restrict__ xs)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    xs[3 * i] = x[3 * j];
    xs[3 * i + 1] = x[3 * j + 1];
    xs[3 * i + 2] = x[3 * j + 2];
}

// segment starts of (key >> shift) over a sorted array
__global__ void seg_flags(const uint64_t* __restrict__ keys, int64_t n, int shift,
                          int32_t* __restrict__ flags)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flags[i] = (i == 0 || (keys[i] >> shift) != (keys[i - 1] >> shift)) ? 1 : 0;
}

// For every element: its segment id; at segment starts also write the segment's key and start.
__global__ void seg_fill(const uint64_t* __restrict__ keys, int64_t n, int shift,
                         const int32_t* __restrict__ flags, const int32_t* __restrict__ ex,
                         int32_t* __restrict__ seg_of, uint64_t* __restrict__ seg_key,
                         int32_t* __restrict__ seg_start)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t sid = ex[i] + flags[i] - 1;
    if (seg_of) seg_of[i] = sid;
    if (flags[i]) {
        seg_key[sid] = keys[i] >> shift;
        seg_start[sid] = (int32_t)i;
    }
}

__global__ void seg_count(const int32_t* __restrict__ start, int64_t nseg, int64_t n,
                          int32_t* __restrict__ count)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    int64_t e = (s + 1 < nseg) ? start[s + 1] : n;
    count[s] = (int32_t)(e - start[s]);
}

__global__ void box_geometry(const uint64_t* __restrict__ keys, int64_t n, double a, double lox,
                             double loy, double loz, double* __restrict__ centers,
                             int32_t* __restrict__ octant)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    uint64_t k = keys[b];
    const double lo[3] = {lox, loy, loz};
    for (int ax = 0; ax < 3; ++ax) {
        uint32_t q = compact3(k >> ax);
        centers[3 * b + ax] = lo[ax] + ((double)q + 0.5) * a;
    }
    if (octant) octant[b] = (int32_t)(k & 7);
}

__global__ void parent_from_seg(const int32_t* __restrict__ seg_of, int64_t n,
                                int32_t* __restrict__ parent)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    parent[b] = seg_of[b];
}

__global__ void point_box_fill(const int32_t* __restrict__ start, const int32_t* __restrict__ count,
                               int64_t nb, int32_t* __restrict__ point_box)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    for (int32_t i = 0; i < count[b]; ++i) point_box[start[b] + i] = (int32_t)b;
}

__device__ inline int64_t find_key(const uint64_t* __restrict__ keys, int64_t n, uint64_t k)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < k) lo = mid + 1; else hi = mid;
    }
    return (lo < n && keys[lo] == k) ? lo : -1;
}

__device__ inline uint64_t key_of(int32_t i, int32_t j, int32_t k)
{
    return spread3((uint64_t)i) | (spread3((uint64_t)j) << 1) | (spread3((uint64_t)k) << 2);
}

// Occupied same-level boxes at Chebyshev distance <= 1 (B included), ascending index.
__device__ inline int neighbours27(const uint64_t* __restrict__ keys, int64_t n, int l,
                                   uint64_t key, int32_t* out)
{
    const int32_t ci = (int32_t)compact3(key), cj = (int32_t)compact3(key >> 1),
                  ck = (int32_t)compact3(key >> 2);
    const int32_t lim = 1 << l;
    int cnt = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int32_t i = ci + dx, j = cj + dy, k = ck + dz;
                if (i < 0 || j < 0 || k < 0 || i >= lim || j >= lim || k >= lim) continue;
                int64_t f = find_key(keys, n, key_of(i, j, k));
                if (f >= 0) {
                    int p = cnt++;
                    while (p > 0 && out[p - 1] > f) {  // insertion sort
                        out[p] = out[p - 1];
                        --p;
                    }
                    out[p] = (int32_t)f;
                }
            }
    return cnt;
}

__global__ void neighbour_lists(const uint64_t* __restrict__ keys, int64_t n, int l,
                                const int32_t* __restrict__ ptr, int32_t* __restrict__ counts,
                                int32_t* __restrict__ src)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    int32_t nb[27];
    int c = neighbours27(keys, n, l, keys[b], nb);
    if (counts) counts[b] = c;
    if (src)
        for (int i = 0; i < c; ++i) src[ptr[b] + i] = nb[i];
}

// The 27 neighbour slots of every box of level l: slot (dx+1) + 3(dy+1) + 9(dz+1) holds the index
// of the box at offset (dx, dy, dz), -1 where that box is empty or outside the root.
__global__ void neighbour_slots(const uint64_t* __restrict__ keys, int64_t n, int l,
                                int32_t* __restrict__ slots)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const uint64_t key = keys[b];
    const int32_t ci = (int32_t)compact3(key), cj = (int32_t)compact3(key >> 1),
                  ck = (int32_t)compact3(key >> 2);
    const int32_t lim = 1 << l;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int32_t i = ci + dx, j = cj + dy, k = ck + dz;
                int64_t f = -1;
                if (i >= 0 && j >= 0 && k >= 0 && i < lim && j < lim && k < lim)
                    f = find_key(keys, n, key_of(i, j, k));
                slots[b * 27 + (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] = (int32_t)f;
            }
}

// I(B) of level l: children (level l) of the neighbours (level l-1) of B's parent that are not
// neighbours of B. Parents are visited in ascending index and children of a parent are
// contiguous and ascending, so entries come out sorted by source index.
__global__ void interaction_lists(const uint64_t* __restrict__ keys, int64_t n, int l,
                                  const uint64_t* __restrict__ pkeys, int64_t np,
                                  const int32_t* __restrict__ parent,
                                  const int32_t* __restrict__ child_start,
                                  const int32_t* __restrict__ child_count,
                                  const int32_t* __restrict__ ptr, int32_t* __restrict__ counts,
                                  int32_t* __restrict__ src, int32_t* __restrict__ code)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const uint64_t kb = keys[b];
    const int32_t bi = (int32_t)compact3(kb), bj = (int32_t)compact3(kb >> 1),
                  bk = (int32_t)compact3(kb >> 2);
    int32_t pn[27];
    int npn = neighbours27(pkeys, np, l - 1, pkeys[parent[b]], pn);
    int cnt = 0;
    int64_t w = src ? ptr[b] : 0;
    for (int t = 0; t < npn; ++t) {
        int32_t p = pn[t];
        for (int32_t c = child_start[p]; c < child_start[p] + child_count[p]; ++c) {
            uint64_t kc = keys[c];
            int32_t dx = (int32_t)compact3(kc) - bi, dy = (int32_t)compact3(kc >> 1) - bj,
                    dz = (int32_t)compact3(kc >> 2) - bk;
            int32_t m = max(abs(dx), max(abs(dy), abs(dz)));
            if (m <= 1) continue;
            if (src) {
                src[w] = c;
                code[w] = (dx + 3) + 7 * (dy + 3) + 49 * (dz + 3);
                ++w;
            }
            ++cnt;
        }
    }
    if (counts) counts[b] = cnt;
}

__global__ void code_to_table_index(const int32_t* __restrict__ code, int64_t n,
                                    const int32_t* __restrict__ map, int32_t* __restrict__ tix)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    tix[i] = map[code[i]];
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void rep_offset(int rep, int d[3])
{
    int r = 0;
    for (int dz = 0; dz <= 3; ++dz)
        for (int dx = 0; dx <= 3; ++dx)
            for (int dy = 0; dy <= dx; ++dy) {
                if (std::max(dx, dz) <= 1) continue;
                if (r++ == rep) {
                    d[0] = dx;
                    d[1] = dy;
                    d[2] = dz;
                    return;
                }
            }
    d[0] = d[1] = d[2] = 0;
}

bool offset_symmetry(int code, int* rep, int* g)
{
    const int d[3] = {code % 7 - 3, (code / 7) % 7 - 3, code / 49 - 3};
    const int ax = std::abs(d[0]), ay = std::abs(d[1]), az = std::abs(d[2]);
    if (std::max(ax, std::max(ay, az)) <= 1) return false;
    const int rx = std::max(ax, ay), ry = std::min(ax, ay);
    int r = 0, found = -1;
    for (int dz = 0; dz <= 3 && found < 0; ++dz)
        for (int dx = 0; dx <= 3 && found < 0; ++dx)
            for (int dy = 0; dy <= dx; ++dy) {
                if (std::max(dx, dz) <= 1) continue;
                if (dx == rx && dy == ry && dz == az) {
                    found = r;
                    break;
                }
                ++r;
            }
    *rep = found;
    *g = (ax < ay ? 1 : 0) | (d[0] < 0 ? 2 : 0) | (d[1] < 0 ? 4 : 0) | (d[2] < 0 ? 8 : 0);
    return true;
}

int sym_direction(int g, int n, int m, int ntheta, int nphi_n, const std::vector<int>& row_off)
{
    // g^{-1} = (reflections, then the swap): z -> -z maps theta to pi - theta (row N_theta/2 - n),
    // x -> -x maps phi to pi - phi, y -> -y phi to -phi, x <-> y phi to pi/2 - phi
    const int np = nphi_n;
    if (g & 8) n = ntheta / 2 - n;
    if (g & 2) m = np / 2 - m;
    if (g & 4) m = -m;
    if (g & 1) m = np / 4 - m;
    m %= np;
    if (m < 0) m += np;
    return row_off[n] + m;
}

// Host map offset code (0..342) -> packed table index 16 rep + g (see offset_symmetry), -1 for
// the inner 27 codes.
void offset_code_map(int32_t* map)
{
    for (int c = 0; c < kNumCodes; ++c) {
        int rep, g;
        map[c] = offset_symmetry(c, &rep, &g) ? kNumSym * rep + g : -1;
    }
}

void build_tree(ffmm_plan* p, const double* d_points, hipStream_t s)
{
    const int64_t n = p->n;
    DeviceArena tmp;
    tmp.inherit(p->arena);
    try {
        // --- root cube ---------------------------------------------------------------------
        const int nbb = (int)std::min<int64_t>(1024, (n + kBoxBlock - 1) / kBoxBlock);
        double* part = tmp.alloc_n<double>(6 * nbb);
        int32_t* bad = tmp.alloc_n<int32_t>(1);
        FFMM_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(bbox_partial, dim3(nbb), dim3(kBoxBlock), 0, s, d_points, n, part, bad);
        FFMM_LAUNCH_CHECK();
        std::vector<double> hpart(6 * nbb);
        int32_t hbad = 0;
        FFMM_HIP(hipMemcpyAsync(hpart.data(), part, sizeof(double) * 6 * nbb, hipMemcpyDeviceToHost, s));
        FFMM_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FFMM_HIP(hipStreamSynchronize(s));
        if (hbad) fail(FFMM_ERR_INVALID_ARG, "points contain non-finite coordinates");
        double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int b = 0; b < nbb; ++b)
            for (int a = 0; a < 3; ++a) {
                mn[a] = std::min(mn[a], hpart[6 * b + a]);
                mx[a] = std::max(mx[a], hpart[6 * b + 3 + a]);
            }
        double side = 0.0;
        for (int a = 0; a < 3; ++a) {
            p->lo[a] = mn[a];
            side = std::max(side, mx[a] - mn[a]);
        }
        if (side == 0.0) side = 1.0;
        p->side = side;
        const double scale21 = (double)(1 << kMaxDepth) / side;

        // --- keys and stable sort ----------------------------------------------------------
        uint64_t* keys = tmp.alloc_n<uint64_t>(n);
        uint64_t* keys2 = tmp.alloc_n<uint64_t>(n);
        int64_t* idx = tmp.alloc_n<int64_t>(n);
        int64_t* idx2 = tmp.alloc_n<int64_t>(n);
        hipLaunchKernelGGL(morton_keys, dim3(blocks_for(n, 256)), dim3(256), 0, s, d_points, n,
                           p->lo[0], p->lo[1], p->lo[2], scale21, keys, idx);
        FFMM_LAUNCH_CHECK();
        const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
        int32_t* hist = tmp.alloc_n<int32_t>(kRadix * ntiles);
        int32_t* offs = tmp.alloc_n<int32_t>(kRadix * ntiles);
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 8 * pass;
            hipLaunchKernelGGL(radix_hist, dim3((unsigned)ntiles), dim3(kWave), 0, s, keys, n,
                               shift, ntiles, hist);
            FFMM_LAUNCH_CHECK();
            exclusive_scan(tmp, hist, offs, kRadix * ntiles, s);
            hipLaunchKernelGGL(radix_scatter, dim3((unsigned)ntiles), dim3(kWave), 0, s, keys, idx,
                               n, shift, ntiles, offs, keys2, idx2);
            FFMM_LAUNCH_CHECK();
            std::swap(keys, keys2);
            std::swap(idx, idx2);
        }

        // --- depth -------------------------------------------------------------------------
        int depth = p->opt.depth;
        if (depth <= 0) {
            int32_t* flags = tmp.alloc_n<int32_t>(kMaxDepth + 1);
            FFMM_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t) * (kMaxDepth + 1), s));
            const int m = p->opt.max_leaf_points;
            if (n > m)
                hipLaunchKernelGGL(occupancy_flags, dim3(blocks_for(n - m, 256)), dim3(256), 0, s,
                                   keys, n, m, flags);
            FFMM_LAUNCH_CHECK();
            int32_t hf[kMaxDepth + 1];
            FFMM_HIP(hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, s));
            FFMM_HIP(hipStreamSynchronize(s));
            depth = kMaxDepth;
            for (int L = 2; L <= kMaxDepth; ++L)
                if (!hf[L]) {
                    depth = L;
                    break;
                }
            if (p->opt.reduce_depth) {
                const double u = p->prec == FFMM_FP32 ? kUnitRoundoffFP32 : kUnitRoundoffFP64;
                while (depth > 2 &&
                       !leaf_feasible(p->kappa * side / (double)(1 << depth), p->opt.alpha, p->eps, u))
                    --depth;
            }
        }
        p->depth = depth;
        p->lev.assign(depth + 1, LevelData{});

        // --- sorted points -----------------------------------------------------------------
        p->perm = p->arena.alloc_n<int64_t>(n);
        FFMM_HIP(hipMemcpyAsync(p->perm, idx, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s));
        p->xs = p->arena.alloc_n<double>(3 * n);
        hipLaunchKernelGGL(gather_points, dim3(blocks_for(n, 256)), dim3(256), 0, s, d_points, p->perm,
                           n, p->xs);
        FFMM_LAUNCH_CHECK();

        // --- leaf level ---------------------------------------------------------------------
        int32_t* flags = tmp.alloc_n<int32_t>(n);
        int32_t* ex = tmp.alloc_n<int32_t>(n);
        {
            LevelData& L = p->lev[depth];
            L.l = depth;
            L.a = side / (double)(1 << depth);
            const int shift = 3 * (kMaxDepth - depth);
            hipLaunchKernelGGL(seg_flags, dim3(blocks_for(n, 256)), dim3(256), 0, s, keys, n, shift, flags);
            FFMM_LAUNCH_CHECK();
            L.n = exclusive_scan(tmp, flags, ex, n, s);   // total = number of segment starts
            if (L.n < 1 || L.n > n) fail(FFMM_ERR_INTERNAL, "leaf box count out of range");
            L.keys = p->arena.alloc_n<uint64_t>(L.n);
            p->leaf_start = p->arena.alloc_n<int32_t>(L.n);
            p->leaf_count = p->arena.alloc_n<int32_t>(L.n);
            p->point_box = p->arena.alloc_n<int32_t>(n);
            hipLaunchKernelGGL(seg_fill, dim3(blocks_for(n, 256)), dim3(256), 0, s, keys, n, shift, flags,
                               ex, p->point_box, L.keys, p->leaf_start);
            FFMM_LAUNCH_CHECK();
            hipLaunchKernelGGL(seg_count, dim3(blocks_for(L.n, 256)), dim3(256), 0, s, p->leaf_start,
                               L.n, n, p->leaf_count);
            FFMM_LAUNCH_CHECK();
        }
        // --- upper levels -------------------------------------------------------------------
        for (int l = depth - 1; l >= 0; --l) {
            LevelData& C = p->lev[l + 1];
            LevelData& P = p->lev[l];
            P.l = l;
            P.a = side / (double)(1 << l);
            hipLaunchKernelGGL(seg_flags, dim3(blocks_for(C.n, 256)), dim3(256), 0, s, C.keys, C.n, 3, flags);
            FFMM_LAUNCH_CHECK();
            P.n = exclusive_scan(tmp, flags, ex, C.n, s);   // total = number of segment starts
            if (P.n < 1 || P.n > C.n || P.n > ((int64_t)1 << (3 * l)))
                fail(FFMM_ERR_INTERNAL, "box count out of range at level " + std::to_string(l));
            P.keys = p->arena.alloc_n<uint64_t>(P.n);
            P.child_start = p->arena.alloc_n<int32_t>(P.n);
            P.child_count = p->arena.alloc_n<int32_t>(P.n);
            C.parent = p->arena.alloc_n<int32_t>(C.n);
            hipLaunchKernelGGL(seg_fill, dim3(blocks_for(C.n, 256)), dim3(256), 0, s, C.keys, C.n, 3,
                               flags, ex, C.parent, P.keys, P.child_start);
            FFMM_LAUNCH_CHECK();
            hipLaunchKernelGGL(seg_count, dim3(blocks_for(P.n, 256)), dim3(256), 0, s, P.child_start,
                               P.n, C.n, P.child_count);
            FFMM_LAUNCH_CHECK();
        }
        for (int l = 0; l <= depth; ++l) {
            LevelData& L = p->lev[l];
            L.centers = p->arena.alloc_n<double>(3 * L.n);
            if (l >= 1) L.octant = p->arena.alloc_n<int32_t>(L.n);
            hipLaunchKernelGGL(box_geometry, dim3(blocks_for(L.n, 256)), dim3(256), 0, s, L.keys, L.n,
                               L.a, p->lo[0], p->lo[1], p->lo[2], L.centers, L.octant);
            FFMM_LAUNCH_CHECK();
        }
        {
            LevelData& L = p->lev[depth];
            hipLaunchKernelGGL(point_box_fill, dim3(blocks_for(L.n, 256)), dim3(256), 0, s,
                               p->leaf_start, p->leaf_count, L.n, p->point_box);
            FFMM_LAUNCH_CHECK();
            // neighbour list of the leaves
            int32_t* cnt = tmp.alloc_n<int32_t>(L.n);
            p->nb_ptr = p->arena.alloc_n<int32_t>(L.n + 1);
            hipLaunchKernelGGL(neighbour_lists, dim3(blocks_for(L.n, 128)), dim3(128), 0, s, L.keys,
                               L.n, depth, (const int32_t*)nullptr, cnt, (int32_t*)nullptr);
            FFMM_LAUNCH_CHECK();
            p->n_nb = exclusive_scan(tmp, cnt, p->nb_ptr, L.n, s);
            const int32_t tot32 = (int32_t)p->n_nb;   // CSR end
            FFMM_HIP(hipMemcpyAsync(p->nb_ptr + L.n, &tot32, sizeof(int32_t), hipMemcpyHostToDevice, s));
            FFMM_HIP(hipStreamSynchronize(s));
            p->nb_src = p->arena.alloc_n<int32_t>(std::max<int64_t>(p->n_nb, 1));
            hipLaunchKernelGGL(neighbour_lists, dim3(blocks_for(L.n, 128)), dim3(128), 0, s, L.keys,
                               L.n, depth, p->nb_ptr, (int32_t*)nullptr, p->nb_src);
            FFMM_LAUNCH_CHECK();
            FFMM_HIP(hipStreamSynchronize(s));
            // near-field pair count and largest leaf (host copies of small arrays)
            std::vector<int32_t> hs(L.n), hc(L.n), hp(L.n + 1), hn(p->n_nb);
            FFMM_HIP(hipMemcpy(hc.data(), p->leaf_count, sizeof(int32_t) * L.n, hipMemcpyDeviceToHost));
            FFMM_HIP(hipMemcpy(hp.data(), p->nb_ptr, sizeof(int32_t) * (L.n + 1), hipMemcpyDeviceToHost));
            FFMM_HIP(hipMemcpy(hn.data(), p->nb_src, sizeof(int32_t) * p->n_nb, hipMemcpyDeviceToHost));
            int64_t pairs = 0;
            int mx_leaf = 0;
            for (int64_t b = 0; b < L.n; ++b) {
                int64_t srcs = 0;
                for (int32_t e = hp[b]; e < hp[b + 1]; ++e) srcs += hc[hn[e]];
                pairs += (int64_t)hc[b] * srcs - hc[b];
                mx_leaf = std::max(mx_leaf, hc[b]);
            }
            p->near_pairs = pairs;
            p->max_leaf_count = mx_leaf;
        }
        // --- interaction lists ------------------------------------------------------------
        int32_t map[kNumCodes];
        offset_code_map(map);
        int32_t* dmap = tmp.alloc_n<int32_t>(kNumCodes);
        FFMM_HIP(hipMemcpyAsync(dmap, map, sizeof(map), hipMemcpyHostToDevice, s));
        for (int l = 2; l <= depth; ++l) {
            LevelData& L = p->lev[l];
            LevelData& P = p->lev[l - 1];
            int32_t* cnt = tmp.alloc_n<int32_t>(L.n);
            L.il_ptr = p->arena.alloc_n<int32_t>(L.n + 1);
            hipLaunchKernelGGL(interaction_lists, dim3(blocks_for(L.n, 128)), dim3(128), 0, s, L.keys,
                               L.n, l, P.keys, P.n, L.parent, P.child_start, P.child_count,
                               (const int32_t*)nullptr, cnt, (int32_t*)nullptr, (int32_t*)nullptr);
            FFMM_LAUNCH_CHECK();
            L.n_il = exclusive_scan(tmp, cnt, L.il_ptr, L.n, s);
            if (L.n_il > INT32_MAX) fail(FFMM_ERR_UNSUPPORTED, "interaction list too long");
            {
                // every list holds at most 6^3 - 3^3 = 189 boxes (the M2L kernel relies on it)
                std::vector<int32_t> hc(L.n);
                FFMM_HIP(hipMemcpy(hc.data(), cnt, sizeof(int32_t) * L.n, hipMemcpyDeviceToHost));
                for (int32_t c : hc)
                    if (c < 0 || c > 189) fail(FFMM_ERR_INTERNAL, "interaction list longer than 189");
            }
            const int32_t tot32 = (int32_t)L.n_il;
            FFMM_HIP(hipMemcpyAsync(L.il_ptr + L.n, &tot32, sizeof(int32_t), hipMemcpyHostToDevice, s));
            FFMM_HIP(hipStreamSynchronize(s));
            const int64_t cap = std::max<int64_t>(L.n_il, 1);
            L.il_src = p->arena.alloc_n<int32_t>(cap);
            L.il_code = p->arena.alloc_n<int32_t>(cap);
            L.il_tix = p->arena.alloc_n<int32_t>(cap);
            hipLaunchKernelGGL(interaction_lists, dim3(blocks_for(L.n, 128)), dim3(128), 0, s, L.keys,
                               L.n, l, P.keys, P.n, L.parent, P.child_start, P.child_count,
                               (const int32_t*)L.il_ptr, (int32_t*)nullptr, L.il_src, L.il_code);
            FFMM_LAUNCH_CHECK();
            if (L.n_il > 0)
                hipLaunchKernelGGL(code_to_table_index, dim3(blocks_for(L.n_il, 256)), dim3(256), 0, s,
                                   L.il_code, L.n_il, dmap, L.il_tix);
            FFMM_LAUNCH_CHECK();
        }
        // neighbour slots of the parent levels (M2L by parent pairs) and the offset-code map
        for (int l = 1; l < depth; ++l) {
            LevelData& L = p->lev[l];
            L.nb_slots = p->arena.alloc_n<int32_t>(27 * (size_t)std::max<int64_t>(L.n, 1));
            hipLaunchKernelGGL(neighbour_slots, dim3(blocks_for(L.n, 128)), dim3(128), 0, s, L.keys, L.n,
                               l, L.nb_slots);
            FFMM_LAUNCH_CHECK();
        }
        p->code_map = p->arena.alloc_n<int32_t>(kNumCodes);
        FFMM_HIP(hipMemcpyAsync(p->code_map, map, sizeof(map), hipMemcpyHostToDevice, s));
        // M2L with the transfer functions in LDS: the 316 transfer vectors as LDS rows in code
        // order; per parent offset D and child offset e (both x + 3y + 9z of components + 1) the
        // row of 2D + e (-1 where that vector joins neighbours), then per row its packed
        // representative and symmetry (16 rep + g), then per D and target octant the mask of the
        // source octants that are far from it
        std::vector<int32_t> rows(27 * 27 + kNumOffsets + 2 * 27 * 8);
        {
            int32_t code_row[kNumCodes];
            int r = 0;
            for (int c = 0; c < kNumCodes; ++c) {
                code_row[c] = map[c] >= 0 ? r : -1;
                if (map[c] >= 0) rows[27 * 27 + r++] = map[c];
            }
            if (r != kNumOffsets) fail(FFMM_ERR_INTERNAL, "transfer vector count");
            for (int D = 0; D < 27; ++D)
                for (int e = 0; e < 27; ++e) {
                    const int cx = 2 * (D % 3 - 1) + (e % 3 - 1) + 3;
                    const int cy = 2 * ((D / 3) % 3 - 1) + ((e / 3) % 3 - 1) + 3;
                    const int cz = 2 * (D / 9 - 1) + (e / 9 - 1) + 3;
                    rows[27 * D + e] = code_row[cx + 7 * cy + 49 * cz];
                }
            // per D and target octant ot: bit os set where source octant os is far from ot
            // (the vector 2D + os - ot is one of the 316)
            for (int D = 0; D < 27; ++D)
                for (int ot = 0; ot < 8; ++ot) {
                    int m = 0;
                    for (int os = 0; os < 8; ++os) {
                        const int e = ((os & 1) - (ot & 1) + 1) + 3 * (((os >> 1) & 1) - ((ot >> 1) & 1) + 1) +
                                      9 * (((os >> 2) & 1) - ((ot >> 2) & 1) + 1);
                        if (rows[27 * D + e] >= 0) m |= 1 << os;
                    }
                    rows[27 * 27 + kNumOffsets + 8 * D + ot] = m;
                }
            // the same relation per D and source octant os: bit ot set where ot is far from os
            for (int D = 0; D < 27; ++D)
                for (int os = 0; os < 8; ++os) {
                    int m = 0;
                    for (int ot = 0; ot < 8; ++ot)
                        if ((rows[27 * 27 + kNumOffsets + 8 * D + ot] >> os) & 1) m |= 1 << ot;
                    rows[27 * 27 + kNumOffsets + 27 * 8 + 8 * D + os] = m;
                }
        }
        p->m2l_rows = p->arena.alloc_n<int32_t>(rows.size());
        FFMM_HIP(hipMemcpyAsync(p->m2l_rows, rows.data(), sizeof(int32_t) * rows.size(),
                                hipMemcpyHostToDevice, s));
        FFMM_HIP(hipStreamSynchronize(s));
    } catch (...) {
        tmp.release();
        throw;
    }
    tmp.release();
}

}  // namespace ffmm
