// Internal declarations of the MI355X Fourier-basis FMM library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/ffmm.h"
#include "params.hpp"

namespace ffmm {

// Errors inside the library are C++ exceptions of this type; the C ABI turns them into a status.
struct Error {
    ffmm_status status;
    std::string message;
};
[[noreturn]] void fail(ffmm_status st, const std::string& msg);

#define FFMM_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            ::ffmm::fail(FFMM_ERR_HIP, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

#define FFMM_LAUNCH_CHECK() FFMM_HIP(hipGetLastError())

constexpr int kMaxDepth = 21;        // bits per axis of the Morton keys
constexpr int kNumOffsets = 316;     // transfer vectors per level (Section 3.2)
constexpr int kNumCodes = 343;       // 7^3 offset codes, inner 3^3 unused
constexpr int kNumReps = 34;         // transfer vectors up to the quadrature's symmetries (Fig. SemiOctant)
constexpr int kNumSym = 16;          // those symmetries: x <-> y swap, then reflections of x, y, z

// Device allocations owned by a plan. With a caller's allocator (ffmm_allocator) every block
// comes from its alloc hook and goes back through its free hook; otherwise hipMalloc/hipFree.
struct DeviceArena {
    std::vector<void*> ptrs;
    size_t bytes = 0;
    ffmm_allocator hooks{};      // alloc == nullptr: hipMalloc
    hipStream_t stream = nullptr;
    // temporaries of the set-up take their memory from the plan's hooks too
    void inherit(const DeviceArena& o)
    {
        hooks = o.hooks;
        stream = o.stream;
    }
    void* alloc(size_t nbytes);
    template <class T>
    T* alloc_n(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
    void release();
};

// One level of the octree with its quadrature and tables.
// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2. This bijection of
// [0, nblocks) gives every XCD a contiguous range of logical blocks, so blocks that read the same
// data (Morton-adjacent boxes, or the tiles of one column range) are served by one L2.
__device__ inline unsigned xcd_block(unsigned b, unsigned nblocks)
{
    constexpr unsigned kXcd = 8;
    const unsigned per = nblocks / kXcd, rem = nblocks % kXcd;
    const unsigned x = b % kXcd, i = b / kXcd;
    return x * per + min(x, rem) + i;
}

struct LevelData {
    int l = 0;
    int64_t n = 0;            // occupied boxes
    double a = 0.0;           // box side
    uint64_t* keys = nullptr; // Morton keys, ascending
    int32_t* parent = nullptr;      // index in level l-1
    int32_t* octant = nullptr;      // position inside the parent, 0..7 (x + 2y + 4z)
    int32_t* child_start = nullptr; // children in level l+1 are contiguous
    int32_t* child_count = nullptr;
    double* centers = nullptr;      // [n][3]
    // interaction list (levels >= 2)
    int64_t n_il = 0;
    int32_t* il_ptr = nullptr;      // [n+1]
    int32_t* il_src = nullptr;      // [n_il]
    int32_t* il_code = nullptr;     // [n_il] offset code 0..342
    int32_t* il_tix = nullptr;      // [n_il] 16 rep + g: representative table and symmetry (tsym)
    int32_t* nb_slots = nullptr;    // levels 1..L-1: [n][27] box at offset (dx,dy,dz), -1 if none
    // quadrature (levels >= 2)
    LevelParams par;
    int K = 0;
    int nrows = 0;
    std::vector<int> row_off;       // host [nrows+1]
    int32_t* d_row_off = nullptr;
    int32_t* d_nphi = nullptr;
    void* dirs = nullptr;           // [K][3] real
    void* weights = nullptr;        // [K] real (leaf level)
    int Kp = 0;                     // K / 2 antipodal direction pairs
    int32_t* pairs = nullptr;       // [Kp][2] (k, k') with s_k' = -s_k
    void* transfer = nullptr;       // [34][K] complex: T of the representative transfer vectors
    int32_t* tperm = nullptr;       // [16][K]: T_{g rep}(s_k) = T_rep(s_{tperm[g][k]})
    void* trans = nullptr;          // [8][K] complex: e^{i kappa s.(oct - 1/2) a_{l+1}} (l < L)
    // z pairs (levels >= 3): the children of one parent with the same (x, y) position, octants o
    // and o + 4, as one entry (zlo, zhi) with zlo the lower one present and zhi the upper one or
    // -1, ordered by parent then by o; zstart/zcount (levels l < L) give each parent's entries
    int64_t nz = 0;
    int32_t* zlo = nullptr;
    int32_t* zhi = nullptr;
    int32_t* zpar = nullptr;        // parent of each entry (index in level l - 1)
    int32_t* zoct = nullptr;        // octant of zlo
    int32_t* zmp = nullptr;         // [nz + 1] children in the entries before each (1 or 2 each)
    int32_t* zsrc = nullptr;        // [n] per child: its pair's zlo when it is a zhi (its downward
                                    // step-1 result is then zlo's times conj(rho)), else -1
    int32_t* zstart = nullptr;
    int32_t* zcount = nullptr;
    // (l < L) [nrows] complex: e^{i kappa cos(theta_n) a_{l+1}}, the ratio of the translations of
    // octants o + 4 and o on row n, which does not depend on phi
    void* zrot = nullptr;
    void* sigM = nullptr;           // [max_rhs][n][K] complex
    void* sigL = nullptr;           // [max_rhs][n][K] complex
};

// Dense real Fourier-resample operators between two level quadratures (Section 3.4).
// the common phi length from which the row steps run on quarter ranges unless the plan's options
// set another (below it the 32-sample output tiles of a quarter range would stay mostly empty)
constexpr int kQuarterMinNphi = 64;

struct Resampler {
    int nphi_all = 0;               // common phi length: min of the two quadratures' largest rows
    int nt_src = 0, nt_dst = 0;
    int rows_src = 0, rows_dst = 0;
    int K_src = 0, K_dst = 0;
    // the row steps on half ranges of phi (u = x_m + x_{m+N/2}, v = x_m - x_{m+N/2} in, a + b and
    // a - b out): step 1 per source row n [N_phi,n/2][2][ldj] (even then odd operator per source
    // sample, destination sample fastest, ldj = nphi_all/2 rounded up to 4, zero padded),
    // at element row_off[n] * ldj
    void* d1h = nullptr;
    int ldj = 0;
    // the theta step on half ranges (eqn. FourierSphereSym): operators for the even
    // and the odd parts of the phi columns, rows 0..N_theta/2 -> 0..N'_theta/2, each
    // [nt_src/2+1][ldh] (zero-padded), the even one first, the factor 1/2 of the split folded in
    void* dth_h = nullptr;
    int ldh = 0;
    // step 5 per destination row n': [nphi_all/2][2][ld'] with ld' = N'_phi,n'/2 rounded up to 4,
    // at element d5h_off[n']
    void* d5h = nullptr;
    int32_t* d5h_off = nullptr;
    // quarter ranges of phi (the half-range parts split again by phi -> -phi) where nphi_all >=
    // kQuarterMinNphi: step 1 per source row [N_phi,n/4 + 1][4][ldq] at element d1q_off[n], step 5
    // per destination row [nphi_all/4 + 1][4][ld'] (ld' = N'_phi,n'/4 + 1 rounded up to 4) at
    // element d5q_off[n']; channels S, A, Mv, P
    bool quarter = false;
    int ldq = 0;
    void* d1q = nullptr;
    void* d5q = nullptr;
    int32_t* d1q_off = nullptr;
    int32_t* d5q_off = nullptr;
    int32_t* d_src_row_off = nullptr;
    int32_t* d_src_nphi = nullptr;
    int32_t* d_dst_row_off = nullptr;
    int32_t* d_dst_nphi = nullptr;
    int32_t* d_dst_row_of_k = nullptr; // [K_dst] row of each destination sample
    // upward pass: tiles of z pairs made of whole parents (at most 32 pairs each)
    int nztiles = 0;
    int32_t* ztile_begin = nullptr;
    int32_t* ztile_end = nullptr;
    int32_t* ztile_pbeg = nullptr;  // first parent of each tile
    int32_t* ztile_pend = nullptr;  // one past its last parent
    int32_t* zcol_tile = nullptr;   // upward theta step: the z pair of each 32-column tile's first column
};

}  // namespace ffmm

struct ffmm_plan {
    int64_t n = 0;
    bool direct = false;            // FFMM_METHOD_DIRECT: no tree, all pairs evaluated
    double kappa = 0.0, eps = 0.0;
    ffmm_options opt{};
    int prec = FFMM_FP64;
    int depth = 0;
    double lo[3] = {0, 0, 0};
    double side = 1.0;
    ffmm::DeviceArena arena;
    int64_t* perm = nullptr;        // [n] caller index of each Morton-ordered point
    double* xs = nullptr;           // [n][3] sorted coordinates (FP64)
    void* rel = nullptr;            // [n][3] coordinates minus leaf centre (plan precision)
    int32_t* point_box = nullptr;   // [n] leaf box of each sorted point
    int32_t* leaf_start = nullptr;  // [nL]
    int32_t* leaf_count = nullptr;  // [nL]
    int32_t* nb_ptr = nullptr;      // leaf neighbour list CSR
    int32_t* nb_src = nullptr;
    int64_t n_nb = 0;
    int64_t near_pairs = 0;
    int max_leaf_count = 0;
    std::vector<ffmm::LevelData> lev;       // 0..depth
    std::vector<ffmm::Resampler> up;        // up[l]: level l -> l-1 (l = 3..L)
    std::vector<ffmm::Resampler> down;      // down[l]: level l -> l+1 (l = 2..L-1)
    void* qs = nullptr;             // [max_rhs][n] complex, sorted charges
    void* phis = nullptr;           // far field (L2P): [max_rhs][n] complex ([..][3] for gradients)
    void* phin = nullptr;           // near field (P2P), same shape
    // P2P runs on its own stream, forked after the upward pass and joined before the scatter,
    // so that it overlaps the far-field stages (default priority, non-blocking)
    hipStream_t near_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    ffmm_tuning tune{};             // launch configuration (ffmm_plan_set_tuning)
    int32_t* code_map = nullptr;    // [343] offset code -> 16 rep + g, -1 for the inner codes
    int32_t* m2l_rows = nullptr;    // [27][27] LDS row of 2D + e (-1: neighbours), [316] 16 rep + g,
                                    // [27][8] mask of the source octants far from target octant ot,
                                    // [27][8] mask of the target octants far from source octant os
    int device = 0;                 // HIP device the plan was created on
    int n_cu = 0;                   // compute units of the plan's device
    void* scratch1 = nullptr;       // resample workspaces
    void* scratch2 = nullptr;
    size_t scratch1_bytes = 0, scratch2_bytes = 0;
    std::vector<double> predicted;  // per level
    bool has_run = false;
    uint32_t m2l_levels = 0xffffffffu;   // ffmm_plan_set_m2l_levels
    // stage timing (ffmm_profile_enable)
    bool profile = false;
    struct EventPair {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<EventPair> events;
    double prof_ms[16] = {0};
    int64_t prof_calls[16] = {0};
};

namespace ffmm {

// Runs f, turning a library Error (or any exception) into a status and the thread's last error
// message; nothing throws across the C ABI.
ffmm_status guarded_call(const std::function<void()>& f);
// Argument checks shared by the matvec-type entry points (plan, pointers, nrhs <= max_rhs).
void check_call(ffmm_plan* plan, const void* in, void* out, int32_t nrhs);

void build_tree(ffmm_plan* p, const double* d_points, hipStream_t s);
void build_tables(ffmm_plan* p, hipStream_t s);
void run_matvec(ffmm_plan* p, const void* q, void* out, int nrhs, int stages, bool conj_io,
                bool gradient, hipStream_t s);
// gx = sum_r Re[conj(G_r) F(q_r) + q_r F(conj G_r)] (ffmm_position_gradient)
void run_position_gradient(ffmm_plan* p, const void* q, const void* g, double* gx, int nrhs,
                           hipStream_t s);

// Records a HIP event pair around a stage when the plan profiles (no-op otherwise).
struct StageScope {
    ffmm_plan* p;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    StageScope(ffmm_plan* plan, int st, hipStream_t stream);
    ~StageScope() noexcept(false);
};

// five-step resample between adjacent levels: M2M when l_dst = l_src - 1, L2L when l_src + 1
void run_resample(ffmm_plan* p, int l_src, int l_dst, int nrhs, hipStream_t s);
void make_parent_tiles(const std::vector<int32_t>& child_count, std::vector<int32_t>& begin,
                       std::vector<int32_t>& end);

// map offset code (0..342) -> transfer table row (0..315), -1 for the inner 27 codes
void offset_code_map(int32_t* map);
// Symmetry decomposition of a transfer vector d (|d_a| <= 3, max >= 2): d = g(rep) with rep =
// (dx >= dy >= 0, dz >= 0) one of 34 representatives and g = swap x <-> y (bit 0) followed by the
// reflections of x (bit 1), y (bit 2), z (bit 3). Returns false for the 27 inner codes.
bool offset_symmetry(int code, int* rep, int* g);
void rep_offset(int rep, int d[3]);
// Index of the direction g^{-1}(s_k) on a level quadrature (rows 0..N_theta/2, row lengths
// N_phi(theta_n), row n and N_theta/2 - n of equal length).
int sym_direction(int g, int n, int m, int ntheta, int nphi_n, const std::vector<int>& row_off);

// exclusive prefix sum of n int32 values; returns the total (synchronises the stream)
int64_t exclusive_scan(DeviceArena& tmp, const int32_t* in, int32_t* out, int64_t n, hipStream_t s);

}  // namespace ffmm
