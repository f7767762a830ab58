/*
 * ffmm.h -- C ABI of the MI355X Fourier-basis Helmholtz FMM (Cecka & Darve, arXiv 0911.4114).
 *
 * The library computes the matrix-vector product of Section 2, eqn. HelmholtzMatrixVector,
 *
 *      phi_i = sum_{j != i} e^{i kappa |x_i - x_j|} / |x_i - x_j| q_j ,   i, j = 1..N,
 *
 * to a requested tolerance eps, by the multilevel FMM of Section 2 with the Fourier-basis
 * quadrature, the band-limited modified transfer function (Section 3.2) and the FFT
 * inter/anterpolation between levels (Section 3.4). Pairs at distance exactly 0 are skipped like
 * j = i. All compute runs on one AMD GPU (gfx950).
 *
 * Conventions for every entry point:
 *  - Every call returns an ffmm_status; nothing throws across this boundary. On failure the
 *    text of ffmm_last_error_message() (thread-local) says what went wrong.
 *  - "device pointer" means memory on the current HIP device (e.g. a torch CUDA tensor's
 *    data_ptr). The caller owns every input and output buffer; the plan owns its tree, tables
 *    and workspaces and frees them in ffmm_plan_destroy.
 *  - Complex arrays are interleaved (re, im). Their element type follows the plan precision:
 *    complex128 (double re, im) for FFMM_FP64 and complex64 (float re, im) for FFMM_FP32.
 *  - hip_stream is a hipStream_t (NULL = the default stream). Matvec-type calls enqueue work on
 *    it and return without waiting; ffmm_plan_create synchronises the stream once.
 *  - One plan must not be used by two streams or threads at the same time.
 *  - On error, outputs are unspecified; the plan stays usable unless the error is FFMM_ERR_HIP.
 */
#ifndef FFMM_H
#define FFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FFMM_OK = 0,
    FFMM_ERR_INVALID_ARG = -1,   /* bad argument: null pointer, n < 1, non-finite input, ... */
    FFMM_ERR_OUT_OF_MEMORY = -2, /* a device or host allocation failed */
    FFMM_ERR_HIP = -3,           /* a HIP runtime call failed (message holds hipGetErrorString) */
    FFMM_ERR_UNSUPPORTED = -4,   /* a valid request this build does not handle */
    FFMM_ERR_ACCURACY = -5,      /* eps cannot be met: some level's predicted error (Gegenbauer
                                    truncation plus the rounding floor of the low-frequency
                                    breakdown, Sections 2.1 and 3.5.1) exceeds eps at every
                                    admissible depth; see ffmm_options.best_effort */
    FFMM_ERR_INTERNAL = -6       /* a consistency check inside the library failed */
} ffmm_status;

typedef enum {
    FFMM_FP64 = 0, /* signatures, tables and sums in FP64; complex128 input/output */
    FFMM_FP32 = 1  /* signatures, FFT resampling, M2L, P2M/L2P in FP32 (complex64 I/O); the
                      transfer-function precompute and the near-field distance and phase stay
                      in FP64 (see ffmm_options.fast_near_phase), the sine/cosine, 1/R and the
                      near-field sums are FP32 */
} ffmm_precision;

#define FFMM_MAX_LEVELS 22 /* levels 0..21; the Morton keys hold 21 bits per axis */

/* Stage selection for ffmm_matvec_stages. */
#define FFMM_STAGE_NEAR 1 /* P2P: sources in the leaf's neighbour list (eqn. FMM_FinalStep) */
#define FFMM_STAGE_FAR 2  /* P2M, M2M, M2L, L2L, L2P */
#define FFMM_STAGE_ALL 3

typedef struct {
    int32_t struct_size;     /* sizeof(ffmm_options); set by ffmm_options_default */
    int32_t precision;       /* ffmm_precision; default FFMM_FP64 */
    int32_t max_leaf_points; /* automatic depth: smallest depth whose leaves hold at most this
                                many points (default 64); ignored when depth > 0 */
    int32_t depth;           /* 0 = automatic; otherwise the leaf level L, 2 <= L <= 21 */
    double alpha;            /* representative |r| = alpha sqrt(3) a_l, Section 3.3.3
                                (default 0.8); levels with kappa a_l > 100 use alpha = 1 (the
                                box diagonal) wherever some ell reaches eps there */
    double eps_safety;       /* per-level tolerance = eps_safety * eps (default 0.1) */
    int32_t max_rhs;         /* largest nrhs of a later call; sizes the workspaces (default 1) */
    int32_t reduce_depth;    /* with depth = 0: 1 (default) lowers the depth while the leaf level
                                cannot reach eps (low-frequency breakdown, Section 3.5.1) */
    int32_t ell_override[FFMM_MAX_LEVELS]; /* > 0 forces ell at that level (tests); 0 = auto */
    int32_t method;          /* ffmm_method: FFMM_METHOD_FMM (default), FFMM_METHOD_DIRECT or
                                FFMM_METHOD_AUTO */
    int32_t best_effort;     /* 0 (default): plan creation fails with FFMM_ERR_ACCURACY when a
                                level's predicted error exceeds eps; 1: build the plan anyway with
                                the most accurate parameters the precision allows (the predicted
                                error is reported in ffmm_plan_info.predicted_err) */
    int32_t fast_near_phase; /* FFMM_FP32 only. 0 (default): the near-field distance R and the
                                phase kappa R are FP64, the phase reduced modulo one revolution
                                before the FP32 sine/cosine; 1: where the leaves span at most 8
                                revolutions of the phase (kappa 2 sqrt(3) a_L <= 16 pi), R^2 is
                                rounded to FP32 and 1/R, R and the phase follow in FP32 (relative
                                phase error ~1e-7; faster) */
    int32_t quarter_nphi;    /* the common phi length of a level transition from which the resample's
                                row steps run on quarter ranges of phi (Section 3.4's interpolation
                                split by the two half-turn and reflection symmetries of the
                                Dirichlet kernel: a quarter of the full contraction); 0 (default):
                                64; a value >= 4 sets it (4: every transition). Same results to
                                rounding either way. */
} ffmm_options;

/*
 * Device-memory hooks for the plan (for example a framework's caching allocator). alloc returns
 * device memory of at least `bytes` bytes usable on `stream` (NULL on failure, which becomes
 * FFMM_ERR_OUT_OF_MEMORY), free releases a pointer alloc returned. The library calls them only
 * inside ffmm_plan_create (the plan's tables and workspaces, and temporaries of the set-up) and
 * ffmm_plan_destroy (which synchronises the device first); ctx is passed through unchanged. The
 * hooks must stay valid until the plan is destroyed.
 */
typedef struct {
    void* ctx;
    void* (*alloc)(void* ctx, size_t bytes, void* stream);
    void (*free)(void* ctx, void* ptr, void* stream);
} ffmm_allocator;

/*
 * FFMM_METHOD_DIRECT evaluates the sum over all pairs (the O(N^2) method the FMM is compared
 * with; FP64 distance and phase in both precisions). FFMM_METHOD_AUTO times, at plan creation,
 * the direct sum (for n <= 2^18) and the FMM at the automatic depth and its feasible neighbours
 * (one level shallower, one deeper; a level whose leaves cannot reach eps is skipped), with
 * max_rhs unit charges, and keeps the fastest plan: the time-optimal level count and the
 * FMM/direct crossover of Section 4 on the caller's point set. depth must be 0 with AUTO.
 */
typedef enum { FFMM_METHOD_FMM = 0, FFMM_METHOD_DIRECT = 1, FFMM_METHOD_AUTO = 2 } ffmm_method;

typedef struct ffmm_plan ffmm_plan; /* opaque */

typedef struct {
    int32_t depth;                       /* leaf level L */
    int32_t precision;                   /* ffmm_precision */
    int64_t n_points;
    double kappa, eps;
    double root_lo[3], root_side;        /* root cube: corner and side */
    int32_t ell[FFMM_MAX_LEVELS];        /* per level l = 2..L (0 elsewhere) */
    int32_t ntheta[FFMM_MAX_LEVELS];
    int32_t nphi_max[FFMM_MAX_LEVELS];
    int64_t K[FFMM_MAX_LEVELS];          /* quadrature size */
    int64_t n_boxes[FFMM_MAX_LEVELS];    /* occupied boxes, levels 0..L */
    int64_t n_ilist[FFMM_MAX_LEVELS];    /* interaction-list entries, levels 2..L */
    double predicted_err[FFMM_MAX_LEVELS]; /* predicted truncation + rounding error */
    int64_t n_near_pairs;                /* ordered source/target pairs of the near field */
    int64_t device_bytes;                /* device memory held by the plan */
    int32_t max_rhs;
    int32_t method;                      /* FFMM_METHOD_FMM or FFMM_METHOD_DIRECT (depth 0) */
    int32_t max_leaf_count;              /* points in the fullest leaf (FMM plans) */
    int32_t reserved;
} ffmm_plan_info;

/* Fill *o with the defaults listed above. o must not be NULL. */
ffmm_status ffmm_options_default(ffmm_options* o);

/*
 * Build a plan: octree and Morton sort (Section 2), per-level truncation ell (Section 2.1) and
 * quadrature (Section 3.3, Alg. Ntheta, Alg. Nphi), band-limited transfer functions for the 316
 * transfer vectors of every level (Alg. BMTF, Section 3.2), translation and resample tables.
 *   d_points : device pointer, n x 3 row-major FP64 coordinates; copied, may be freed after.
 *   n        : number of points, n >= 1.
 *   kappa    : wavenumber, finite and > 0.
 *   eps      : target relative error, 1e-12 <= eps <= 0.5 (1e-7 <= eps for FFMM_FP32).
 *   o        : options or NULL for the defaults.
 *   alloc    : device-memory hooks (see ffmm_allocator) or NULL for hipMalloc/hipFree; both
 *              function pointers must be set when alloc is not NULL.
 *   out      : receives the plan.
 * Errors: INVALID_ARG (nulls, ranges, non-finite coordinates), UNSUPPORTED (FP32 with
 * eps < 1e-7; a quadrature of more than 2^27 directions), ACCURACY (eps unreachable, see
 * FFMM_ERR_ACCURACY and options.best_effort), OUT_OF_MEMORY, HIP. Synchronises hip_stream.
 */
ffmm_status ffmm_plan_create(const double* d_points, int64_t n, double kappa, double eps,
                             const ffmm_options* o, const ffmm_allocator* alloc, void* hip_stream,
                             ffmm_plan** out);

/*
 * phi = A q (eqn. HelmholtzMatrixVector) for nrhs right-hand sides.
 *   d_q   : device, [nrhs][n] complex in the caller's point order.
 *   d_phi : device, [nrhs][n] complex output (may not alias d_q).
 *   nrhs  : 1 <= nrhs <= max_rhs of the plan.
 */
ffmm_status ffmm_matvec(ffmm_plan* plan, const void* d_q, void* d_phi, int32_t nrhs,
                        void* hip_stream);

/* As ffmm_matvec, running only the stages in the mask (FFMM_STAGE_NEAR / _FAR / _ALL);
 * phi receives the sum of the selected parts. */
ffmm_status ffmm_matvec_stages(ffmm_plan* plan, const void* d_q, void* d_phi, int32_t nrhs,
                               int32_t stages, void* hip_stream);

/*
 * Adjoint product out = A^H g. The kernel matrix is complex-symmetric (A_ij = A_ji), so
 * A^H g = conj(A conj(g)); the conjugations are fused into the gather and scatter.
 * Same layout and limits as ffmm_matvec.
 */
ffmm_status ffmm_adjoint(ffmm_plan* plan, const void* d_g, void* d_out, int32_t nrhs,
                         void* hip_stream);

/*
 * Field gradient F_i(q) = sum_{j != i} G'(R_ij) (x_i - x_j)/R_ij q_j with
 * G'(R) = e^{i kappa R} (i kappa R - 1) / R^2, the gradient of phi_i with respect to x_i.
 * The far part differentiates the local expansion (L2P with the factor -i kappa s_k), the near
 * part differentiates the kernel (P2P).
 *   d_q    : device, [nrhs][n] complex.
 *   d_grad : device, [nrhs][n][3] complex output.
 */
ffmm_status ffmm_field_gradient(ffmm_plan* plan, const void* d_q, void* d_grad, int32_t nrhs,
                                void* hip_stream);

/*
 * Gradient of a real loss L(phi), phi = A(x) q, with respect to the point positions, for a fixed
 * tree (the quantity torch.autograd needs for the points). With G = dL/dRe(phi) + i dL/dIm(phi)
 * per right-hand side and F the field gradient above,
 *      gx_i = sum_r Re[ conj(G_{r,i}) F_i(q_r) + q_{r,i} F_i(conj G_r) ]
 * (A_ij depends on x_i and x_j only through |x_i - x_j|, so both ends of each pair contribute;
 * the kernel's derivative G'(R) is that of eqn. HelmholtzMatrixVector). Runs the field-gradient
 * FMM on q_r and conj(G_r) together (in groups of max_rhs / 2 right-hand sides, or one after
 * the other when max_rhs = 1) and combines the two on the GPU.
 *   d_q   : device, [nrhs][n] complex charges (caller order).
 *   d_g   : device, [nrhs][n] complex G (caller order).
 *   d_gx  : device, [n][3] FP64 output (caller order), overwritten.
 *   nrhs  : >= 1 (any number; processed in groups).
 */
ffmm_status ffmm_position_gradient(ffmm_plan* plan, const void* d_q, const void* d_g, double* d_gx,
                                   int32_t nrhs, void* hip_stream);

/*
 * Allocation-free variant of ffmm_matvec, for callers that cannot allocate device memory during
 * the call (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same product, arguments, layout and limits as ffmm_matvec, and the same kernels; the per-call
 * workspaces (the charges in Morton order, the far- and near-field partial results and the
 * resample intermediates, about 3 N nrhs complex values plus the two resample buffers of the
 * plan scaled to nrhs) come from one static device array of FFMM_STATIC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends, instead of the plan's own
 * buffers. The call allocates nothing (no hipMalloc, hipFree or event creation; stage profiling
 * is off for it). Every region of the array that a call reads is written earlier in that call,
 * so nothing carries over from the previous call.
 *   Errors: as ffmm_matvec; UNSUPPORTED when the workspace of nrhs right-hand sides exceeds
 *   FFMM_STATIC_SCRATCH_BYTES (the message states both sizes); INVALID_ARG when the current
 *   device is not the plan's.
 *   Calls that overlap in time on one GPU (other streams, other threads, other plans) share the
 *   array and race: the caller orders them, e.g. on one stream.
 */
#define FFMM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
ffmm_status ffmm_matvec_static(ffmm_plan* plan, const void* d_q, void* d_phi, int32_t nrhs,
                               void* hip_stream);

/* Stages timed by the profiling calls below. */
enum {
    FFMM_PROF_GATHER = 0, /* caller order -> Morton order (+ conjugation) */
    FFMM_PROF_P2M = 1,
    FFMM_PROF_M2M = 2,    /* all levels */
    FFMM_PROF_M2L = 3,    /* all levels */
    FFMM_PROF_L2L = 4,    /* all levels */
    FFMM_PROF_L2P = 5,
    FFMM_PROF_P2P = 6,
    FFMM_PROF_SCATTER = 7,
    FFMM_PROF_LEAF_M2L = 8, /* the leaf level's share of FFMM_PROF_M2L */
    FFMM_PROF_NUM = 9
};

/*
 * Stage timing. With on = 1 every later matvec-type call records a pair of HIP events around
 * each stage on its stream (a small overhead) and runs P2P on the calling stream, after the far
 * field, so that no two stages overlap; ffmm_profile_read waits for them, returns the
 * accumulated milliseconds ms[FFMM_PROF_NUM] and launch counts calls[FFMM_PROF_NUM] since the
 * last read (either may be NULL), and resets the accumulators.
 */
ffmm_status ffmm_profile_enable(ffmm_plan* plan, int32_t on);
ffmm_status ffmm_profile_read(ffmm_plan* plan, double* ms, int64_t* calls);

/*
 * Launch configuration of a plan's kernels. None of it changes what is computed; only the
 * rounding order of the resample contractions depends on rs_slab. Callers with many right-hand
 * sides or unusual point sets can let ffmm_plan_autotune choose it.
 */
typedef struct {
    int32_t struct_size;        /* sizeof(ffmm_tuning); set by ffmm_tuning_default */
    int32_t near_stream;        /* 2 (default): P2P runs on a second stream of the plan, forked before
                                   P2M and overlapping the far-field stages; 1: the same, forked after
                                   the upward pass; 0: every stage in order on the caller's stream */
    int32_t p2p_blocks_per_cu;  /* P2P blocks per compute unit, each looping over leaves (1..16);
                                   0 (default) = one block per four leaves */
    int32_t m2l_rhs_block;      /* right-hand sides sharing each transfer-function read in M2L:
                                   1, 2 or 4 (at most 2 with m2l_by_parent); 0 (default) = the
                                   largest that does not exceed nrhs */
    int32_t rs_slab[4];         /* resample k-slab depth (16, 32 or 64; FP64 plans take 32 for 64)
                                   of step 1, steps 2+3, upward steps 4+5 and downward steps 4+5;
                                   the quarter-range forms of steps 1 and 5 take 16 or 32 (32 for
                                   64; FP64: 16); default 16, 32, 32, 16 */
    int32_t m2l_by_parent;      /* M2L form. 2 (default): by parent pairs, with the transfer
                                   functions of a chunk of m2l_chunk directions gathered into LDS
                                   once per block and reused for a range of parents (FP64 plans:
                                   chunks of 32 pairs, whatever m2l_chunk); 1: by parent pairs, each source
                                   signature and transfer function read once per parent pair (2.5x
                                   faster than 0 at the leaves of a volume distribution); 0: one
                                   target box per block over its interaction list. Forms 1 and 2
                                   give the same bits. */
    int32_t m2l_chunk;          /* antipodal direction pairs per block of M2L form 2: 64 (default;
                                   158 KB of LDS, one block per compute unit, so that no P2P block of
                                   a persistent P2P grid fits beside it), 48 (121 KB, leaving room
                                   for one) or 32 (81 KB) */
} ffmm_tuning;

/* Fill *t with the defaults listed above. t must not be NULL. */
ffmm_status ffmm_tuning_default(ffmm_tuning* t);

/* Replace the plan's launch configuration (validated; FFMM_ERR_INVALID_ARG for values outside
 * the ranges above). Takes effect at the next call on the plan. */
ffmm_status ffmm_plan_set_tuning(ffmm_plan* plan, const ffmm_tuning* t);
ffmm_status ffmm_plan_get_tuning(const ffmm_plan* plan, ffmm_tuning* out);

/*
 * Autotuner: time matvecs of the nrhs right-hand sides at d_q (device, layout of ffmm_matvec)
 * under candidate launch configurations: the P2P placement (near_stream, p2p_blocks_per_cu) and
 * the M2L chunk width over a joint grid (they compete for the same LDS), then coordinate descent
 * over the other fields and the P2P grid once more, then a confirmation in which the starting
 * configuration, the search's choice and that choice with the other P2P fork point are timed in
 * turn over three rounds; the fastest is kept on the plan (also copied to *best when best is not
 * NULL). Each configuration is timed as the best of three groups of three back-to-back
 * products after one warm-up. d_out receives the products (its contents are those of the last
 * candidate). Runs about 60 configurations x 10 matvecs, ordered on hip_stream; synchronises it.
 */
ffmm_status ffmm_plan_autotune(ffmm_plan* plan, const void* d_q, void* d_out, int32_t nrhs,
                               void* hip_stream, ffmm_tuning* best);

/* Copy the plan's parameters into *out. */
ffmm_status ffmm_plan_info_get(const ffmm_plan* plan, ffmm_plan_info* out);

/* Release every resource of the plan (NULL is accepted). Synchronises the device. */
ffmm_status ffmm_plan_destroy(ffmm_plan* plan);

/* Static text for a status code. */
const char* ffmm_status_string(ffmm_status s);

/* Thread-local detail of the last failure on this thread ("" if none). */
const char* ffmm_last_error_message(void);

/* ----------------------------------------------------------------------------------------
 * Inspection calls. They copy plan data to HOST buffers that the caller allocates, for stage-by-
 * stage checks against an independent implementation. They synchronise the device.
 * ---------------------------------------------------------------------------------------- */

/*
 * Host-only parameter choice for one level in box units (no GPU needed): ka = kappa a_l,
 * |r| = alpha' sqrt(3), |r0| = 2 (Section 3.3.3), alpha' = alpha, or 1 when ka > 100 and some
 * ell reaches eps at |r| = sqrt(3). ell from the Gegenbauer truncation error of
 * eqn. eps_G plus the low-frequency rounding floor of the given precision (Section 2.1), N_theta
 * by Alg. Ntheta, N_phi(theta_n) by Alg. Nphi (Section 3.3).
 *   ell_in      : > 0 to force ell, 0 to choose it.
 *   nphi        : host, capacity nphi_cap ints; receives N_phi(theta_n) for n = 0..N_theta/2.
 *   ell, ntheta : outputs; predicted: predicted error at the chosen ell (may be NULL).
 * Returns INVALID_ARG if nphi_cap < N_theta/2 + 1.
 */
ffmm_status ffmm_select_level_params(double ka, double alpha, double eps, int32_t precision,
                                     int32_t ell_in, int32_t* ell, int32_t* ntheta,
                                     int32_t* nphi, int32_t nphi_cap, double* predicted);

/*
 * Point permutation: perm[i] = caller index of the i-th point in Morton order (host int64[n]).
 */
ffmm_status ffmm_plan_get_perm(const ffmm_plan* plan, int64_t* perm);

/*
 * Level l (0..L) of the tree. Each output may be NULL. Sizes: n = info.n_boxes[l].
 *   keys   : uint64[n]  Morton keys of the occupied boxes, ascending.
 *   parent : int32[n]   index of the parent box in level l-1 (l >= 1).
 *   start, count : int32[n] leaf point ranges in Morton order (leaf level only).
 *   il_ptr : int32[n+1], il_src : int32[info.n_ilist[l]], il_code : int32[...] interaction list
 *            (levels >= 2) in CSR form, rows sorted by source index; code = (dx+3) + 7 (dy+3) +
 *            49 (dz+3) of the source-minus-target offset in box units.
 *   nb_ptr, nb_src : neighbour list of the leaf level in CSR form (capacity n*27 for nb_src).
 */
ffmm_status ffmm_plan_get_level(const ffmm_plan* plan, int32_t l, uint64_t* keys, int32_t* parent,
                                int32_t* start, int32_t* count, int32_t* il_ptr, int32_t* il_src,
                                int32_t* il_code, int32_t* nb_ptr, int32_t* nb_src);

/*
 * Error studies: restrict the transfer pass (M2L, Section 2) of later calls to the levels whose
 * bit is set in level_mask (bit l = level l; all levels by default, mask 0xffffffff). The far
 * field then holds only the contributions of the interaction lists of those levels, passed down
 * the tree as usual; the local expansions of the other levels start from zero. Not for products.
 */
ffmm_status ffmm_plan_set_m2l_levels(ffmm_plan* plan, uint32_t level_mask);

/* N_phi(theta_n) of level l's quadrature: host int32[ntheta/2 + 1]. */
ffmm_status ffmm_plan_get_nphi(const ffmm_plan* plan, int32_t l, int32_t* nphi);

/*
 * Band-limited modified transfer function T^{s,LL} of level l for offset code `code`
 * (0..342, not an inner code) sampled on the level quadrature: host complex128[K_l]
 * (converted to FP64 for an FP32 plan). The plan stores T for the 34 transfer vectors that are
 * distinct up to the quadrature's symmetries (Section 3.2, Fig. SemiOctant); this call rebuilds
 * the requested one by the direction permutation of its symmetry.
 */
ffmm_status ffmm_plan_get_transfer(const ffmm_plan* plan, int32_t l, int32_t code, double* out);

/*
 * Signatures of the last matvec for right-hand side rhs: kind 0 = outgoing M^l, kind 1 =
 * local L^l (incoming I^l plus the downward pass). host complex128[n_boxes[l] * K_l].
 */
ffmm_status ffmm_plan_get_signature(const ffmm_plan* plan, int32_t kind, int32_t l, int32_t rhs,
                                    double* out);

#ifdef __cplusplus
}
#endif

#endif /* FFMM_H */
