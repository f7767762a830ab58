// C ABI of the library (include/ffmm.h): argument checks, plan assembly and inspection calls.
// No exception crosses this boundary; failures become an ffmm_status plus a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <new>
#include <string>

#include "internal.hpp"

namespace ffmm {

static thread_local std::string g_last_error;

void fail(ffmm_status st, const std::string& msg) { throw Error{st, msg}; }

void* DeviceArena::alloc(size_t nbytes)
{
    void* p = nullptr;
    if (nbytes == 0) nbytes = 16;
    if (hooks.alloc) {
        p = hooks.alloc(hooks.ctx, nbytes, (void*)stream);
        if (!p)
            fail(FFMM_ERR_OUT_OF_MEMORY, "the caller's allocator returned NULL for " +
                                             std::to_string(nbytes) + " bytes");
        ptrs.push_back(p);
        bytes += nbytes;
        return p;
    }
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? FFMM_ERR_OUT_OF_MEMORY : FFMM_ERR_HIP,
             std::string("hipMalloc of ") + std::to_string(nbytes) + " bytes failed: " +
                 hipGetErrorString(e));
    }
    ptrs.push_back(p);
    bytes += nbytes;
    return p;
}

void DeviceArena::release()
{
    for (void* p : ptrs) {
        if (hooks.free)
            hooks.free(hooks.ctx, p, (void*)stream);
        else
            (void)hipFree(p);
    }
    ptrs.clear();
    bytes = 0;
}

void prepare_rel(ffmm_plan* p, hipStream_t s);
void init_cis_table(hipStream_t s);

StageScope::StageScope(ffmm_plan* plan, int st, hipStream_t stream) : p(plan), stage(st), s(stream)
{
    if (!p->profile) return;
    FFMM_HIP(hipEventCreate(&a));
    FFMM_HIP(hipEventCreate(&b));
    FFMM_HIP(hipEventRecord(a, s));
}

StageScope::~StageScope() noexcept(false)
{
    if (!a) return;
    if (std::uncaught_exceptions()) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return;
    }
    FFMM_HIP(hipEventRecord(b, s));
    p->events.push_back({stage, a, b});
}

static void drain_events(ffmm_plan* p, bool accumulate)
{
    for (auto& e : p->events) {
        if (accumulate) {
            FFMM_HIP(hipEventSynchronize(e.b));
            float ms = 0.0f;
            FFMM_HIP(hipEventElapsedTime(&ms, e.a, e.b));
            p->prof_ms[e.stage] += ms;
            p->prof_calls[e.stage] += 1;
        }
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    p->events.clear();
}

template <class F>
static ffmm_status guarded(F&& f)
{
    try {
        f();
        g_last_error.clear();
        return FFMM_OK;
    } catch (const Error& e) {
        g_last_error = e.message;
        return e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return FFMM_ERR_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return FFMM_ERR_INTERNAL;
    } catch (...) {
        g_last_error = "unknown failure";
        return FFMM_ERR_INTERNAL;
    }
}

ffmm_status guarded_call(const std::function<void()>& f) { return guarded(f); }

void check_call(ffmm_plan* plan, const void* in, void* out, int32_t nrhs)
{
    if (!plan) fail(FFMM_ERR_INVALID_ARG, "plan is NULL");
    if (!in || !out) fail(FFMM_ERR_INVALID_ARG, "input or output pointer is NULL");
    if (in == out) fail(FFMM_ERR_INVALID_ARG, "input and output must not alias");
    if (nrhs < 1 || nrhs > plan->opt.max_rhs)
        fail(FFMM_ERR_INVALID_ARG, "nrhs must lie in [1, max_rhs] (max_rhs = " +
                                       std::to_string(plan->opt.max_rhs) + ")");
}

static size_t csize(const ffmm_plan* p) { return p->prec == FFMM_FP32 ? 8 : 16; }

static void allocate_workspaces(ffmm_plan* p)
{
    const int mr = p->opt.max_rhs;
    const size_t cs = csize(p);
    for (int l = 2; l <= p->depth; ++l) {
        LevelData& L = p->lev[l];
        L.sigM = p->arena.alloc(cs * (size_t)mr * L.n * L.K);
        L.sigL = p->arena.alloc(cs * (size_t)mr * L.n * L.K);
    }
    size_t s1 = 1, s2 = 1;
    for (int l = 3; l <= p->depth; ++l) {
        const Resampler& rs = p->up[l];
        const int64_t nb = p->lev[l].n;
        s1 = std::max(s1, (size_t)nb * rs.rows_src * rs.nphi_all);
        s2 = std::max(s2, (size_t)nb * rs.nphi_all * (rs.nt_dst / 2 + 1));   // theta rows 0..N'/2
    }
    for (int l = 2; l < p->depth; ++l) {
        const Resampler& rs = p->down[l];
        const int64_t nb = p->lev[l + 1].n;
        s1 = std::max(s1, (size_t)nb * rs.rows_src * rs.nphi_all);
        s2 = std::max(s2, (size_t)nb * rs.nphi_all * (rs.nt_dst / 2 + 1));
    }
    p->scratch1_bytes = cs * s1 * mr;
    p->scratch2_bytes = cs * s2 * mr;
    p->scratch1 = p->arena.alloc(p->scratch1_bytes);
    p->scratch2 = p->arena.alloc(p->scratch2_bytes);
    p->qs = p->arena.alloc(cs * (size_t)mr * p->n);
    p->phis = p->arena.alloc(cs * (size_t)mr * p->n * 3);
    p->phin = p->arena.alloc(cs * (size_t)mr * p->n * 3);
    FFMM_HIP(hipStreamCreateWithFlags(&p->near_stream, hipStreamNonBlocking));
    FFMM_HIP(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    FFMM_HIP(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
}

static void release_streams(ffmm_plan* p)
{
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->near_stream) (void)hipStreamDestroy(p->near_stream);
    p->ev_fork = p->ev_join = nullptr;
    p->near_stream = nullptr;
}

// FFMM_METHOD_DIRECT: the points in the caller's order and the identity permutation.
static void build_direct(ffmm_plan* p, const double* d_points, hipStream_t s)
{
    p->direct = true;
    p->depth = 0;
    p->lev.assign(1, LevelData{});
    p->lev[0].n = 1;
    std::vector<int64_t> id(p->n);
    for (int64_t i = 0; i < p->n; ++i) id[i] = i;
    p->perm = p->arena.alloc_n<int64_t>(p->n);
    FFMM_HIP(hipMemcpyAsync(p->perm, id.data(), sizeof(int64_t) * p->n, hipMemcpyHostToDevice, s));
    p->xs = p->arena.alloc_n<double>(3 * p->n);
    FFMM_HIP(hipMemcpyAsync(p->xs, d_points, sizeof(double) * 3 * p->n, hipMemcpyDeviceToDevice, s));
    FFMM_HIP(hipStreamSynchronize(s));
    p->near_pairs = p->n * (p->n - 1);
}

}  // namespace ffmm

using namespace ffmm;

// FFMM_METHOD_AUTO: build the candidate plans, time each on unit charges, keep the fastest.
static ffmm_plan* create_fastest(const double* d_points, int64_t n, double kappa, double eps,
                                 const ffmm_options& opt, const ffmm_allocator* hooks, hipStream_t s)
{
    std::vector<ffmm_plan*> plans;
    DeviceArena tmp;
    if (hooks) tmp.hooks = *hooks;
    tmp.stream = s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&](ffmm_plan* keep) {
        for (ffmm_plan* q : plans)
            if (q != keep) ffmm_plan_destroy(q);
        tmp.release();
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    try {
        auto make = [&](int method, int depth) {
            ffmm_options o = opt;
            o.method = method;
            o.depth = depth;
            ffmm_plan* q = nullptr;
            const ffmm_status st = ffmm_plan_create(d_points, n, kappa, eps, &o, hooks, s, &q);
            if (st == FFMM_OK) plans.push_back(q);
            // a candidate that does not fit or cannot reach eps is left out
            else if (st != FFMM_ERR_OUT_OF_MEMORY && st != FFMM_ERR_ACCURACY) fail(st, g_last_error);
            return q;
        };
        ffmm_plan* first = make(FFMM_METHOD_FMM, 0);
        if (first) {
            const int d0 = first->depth;
            const double u = opt.precision == FFMM_FP32 ? kUnitRoundoffFP32 : kUnitRoundoffFP64;
            for (int d : {d0 - 1, d0 + 1})
                if (d >= 2 && d <= kMaxDepth &&
                    leaf_feasible(kappa * first->side / (double)(1 << d), opt.alpha, eps, u))
                    make(FFMM_METHOD_FMM, d);
        }
        if (n <= (int64_t(1) << 18)) make(FFMM_METHOD_DIRECT, 0);
        if (plans.empty())
            fail(FFMM_ERR_ACCURACY, "no FMM depth reaches eps and the point set is too large for "
                                    "the direct method (n > 2^18), or no candidate fits in memory");
        // unit charges for every right-hand side
        const size_t cs = opt.precision == FFMM_FP32 ? 8 : 16;
        const size_t cnt = (size_t)opt.max_rhs * n;
        std::vector<char> ones(cs * cnt, 0);
        for (size_t i = 0; i < cnt; ++i) {
            if (cs == 8) ((float*)ones.data())[2 * i] = 1.0f;
            else ((double*)ones.data())[2 * i] = 1.0;
        }
        void* dq = tmp.alloc(cs * cnt);
        void* dout = tmp.alloc(cs * cnt);
        FFMM_HIP(hipMemcpyAsync(dq, ones.data(), cs * cnt, hipMemcpyHostToDevice, s));
        FFMM_HIP(hipEventCreate(&e0));
        FFMM_HIP(hipEventCreate(&e1));
        ffmm_plan* best = nullptr;
        float best_ms = 1e30f;
        for (ffmm_plan* q : plans) {
            run_matvec(q, dq, dout, opt.max_rhs, FFMM_STAGE_ALL, false, false, s);
            float ms_min = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                FFMM_HIP(hipEventRecord(e0, s));
                run_matvec(q, dq, dout, opt.max_rhs, FFMM_STAGE_ALL, false, false, s);
                FFMM_HIP(hipEventRecord(e1, s));
                FFMM_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                FFMM_HIP(hipEventElapsedTime(&ms, e0, e1));
                ms_min = std::min(ms_min, ms);
            }
            if (ms_min < best_ms) {
                best_ms = ms_min;
                best = q;
            }
        }
        cleanup(best);
        best->opt.method = FFMM_METHOD_AUTO;
        return best;
    } catch (...) {
        cleanup(nullptr);
        throw;
    }
}

extern "C" {

ffmm_status ffmm_options_default(ffmm_options* o)
{
    if (!o) {
        g_last_error = "options pointer is NULL";
        return FFMM_ERR_INVALID_ARG;
    }
    std::memset(o, 0, sizeof(*o));
    o->struct_size = (int32_t)sizeof(ffmm_options);
    o->precision = FFMM_FP64;
    o->max_leaf_points = 64;
    o->depth = 0;
    o->alpha = 0.8;
    o->eps_safety = 0.1;
    o->max_rhs = 1;
    o->reduce_depth = 1;
    o->best_effort = 0;
    o->fast_near_phase = 0;
    o->quarter_nphi = 0;
    g_last_error.clear();
    return FFMM_OK;
}

ffmm_status ffmm_tuning_default(ffmm_tuning* t)
{
    if (!t) {
        g_last_error = "tuning pointer is NULL";
        return FFMM_ERR_INVALID_ARG;
    }
    std::memset(t, 0, sizeof(*t));
    t->struct_size = (int32_t)sizeof(ffmm_tuning);
    t->near_stream = 2;
    t->p2p_blocks_per_cu = 0;
    t->m2l_rhs_block = 0;
    t->rs_slab[0] = 16;
    t->rs_slab[1] = 32;
    t->rs_slab[2] = 32;
    t->rs_slab[3] = 16;
    t->m2l_by_parent = 2;
    t->m2l_chunk = 64;
    g_last_error.clear();
    return FFMM_OK;
}

ffmm_status ffmm_plan_create(const double* d_points, int64_t n, double kappa, double eps,
                             const ffmm_options* o, const ffmm_allocator* alloc, void* hip_stream,
                             ffmm_plan** out)
{
    ffmm_plan* p = nullptr;
    ffmm_status st = guarded([&] {
        if (!out) fail(FFMM_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!d_points) fail(FFMM_ERR_INVALID_ARG, "points pointer is NULL");
        if (n < 1) fail(FFMM_ERR_INVALID_ARG, "n must be >= 1");
        if (n > (int64_t)INT32_MAX - 1) fail(FFMM_ERR_UNSUPPORTED, "n exceeds 2^31 - 2");
        if (!std::isfinite(kappa) || kappa <= 0.0) fail(FFMM_ERR_INVALID_ARG, "kappa must be finite and > 0");
        if (!std::isfinite(eps) || eps < 1e-12 || eps > 0.5)
            fail(FFMM_ERR_INVALID_ARG, "eps must lie in [1e-12, 0.5]");
        ffmm_options opt;
        ffmm_options_default(&opt);
        if (o) {
            if (o->struct_size != (int32_t)sizeof(ffmm_options))
                fail(FFMM_ERR_INVALID_ARG, "options.struct_size does not match this library");
            opt = *o;
        }
        if (opt.precision != FFMM_FP64 && opt.precision != FFMM_FP32)
            fail(FFMM_ERR_INVALID_ARG, "unknown precision");
        if (opt.precision == FFMM_FP32 && eps < 1e-7)
            fail(FFMM_ERR_UNSUPPORTED, "FP32 plans need eps >= 1e-7");
        if (opt.depth != 0 && (opt.depth < 2 || opt.depth > kMaxDepth))
            fail(FFMM_ERR_INVALID_ARG, "depth must be 0 or in [2, 21]");
        if (opt.depth == 0 && opt.max_leaf_points < 1) fail(FFMM_ERR_INVALID_ARG, "max_leaf_points must be >= 1");
        if (!(opt.alpha > 0.0 && opt.alpha <= 1.0)) fail(FFMM_ERR_INVALID_ARG, "alpha must lie in (0, 1]");
        if (!(opt.eps_safety > 0.0 && opt.eps_safety <= 1.0))
            fail(FFMM_ERR_INVALID_ARG, "eps_safety must lie in (0, 1]");
        if (opt.max_rhs < 1 || opt.max_rhs > 65535) fail(FFMM_ERR_INVALID_ARG, "max_rhs must lie in [1, 65535]");
        for (int l = 0; l < FFMM_MAX_LEVELS; ++l)
            if (opt.ell_override[l] < 0 || opt.ell_override[l] > 2000)
                fail(FFMM_ERR_INVALID_ARG, "ell_override out of range");
        if (opt.method != FFMM_METHOD_FMM && opt.method != FFMM_METHOD_DIRECT && opt.method != FFMM_METHOD_AUTO)
            fail(FFMM_ERR_INVALID_ARG, "unknown method");
        if (opt.method == FFMM_METHOD_AUTO && opt.depth != 0)
            fail(FFMM_ERR_INVALID_ARG, "depth must be 0 with FFMM_METHOD_AUTO");
        if (opt.best_effort != 0 && opt.best_effort != 1) fail(FFMM_ERR_INVALID_ARG, "best_effort must be 0 or 1");
        if (opt.fast_near_phase != 0 && opt.fast_near_phase != 1)
            fail(FFMM_ERR_INVALID_ARG, "fast_near_phase must be 0 or 1");
        if (opt.quarter_nphi < 0) fail(FFMM_ERR_INVALID_ARG, "quarter_nphi must be >= 0");
        if (alloc && (!alloc->alloc || !alloc->free))
            fail(FFMM_ERR_INVALID_ARG, "allocator needs both its alloc and free hooks");
        int ndev = 0;
        FFMM_HIP(hipGetDeviceCount(&ndev));
        if (ndev < 1) fail(FFMM_ERR_HIP, "no HIP device");
        hipStream_t s = (hipStream_t)hip_stream;
        if (opt.method == FFMM_METHOD_AUTO) {
            *out = create_fastest(d_points, n, kappa, eps, opt, alloc, s);
            return;
        }
        p = new ffmm_plan();
        if (alloc) p->arena.hooks = *alloc;
        p->arena.stream = s;
        p->n = n;
        p->kappa = kappa;
        p->eps = eps;
        p->opt = opt;
        p->prec = opt.precision;
        ffmm_tuning_default(&p->tune);
        {
            int dev = 0;
            FFMM_HIP(hipGetDevice(&dev));
            p->device = dev;
            FFMM_HIP(hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        }
        init_cis_table(s);
        if (opt.method == FFMM_METHOD_DIRECT) {
            build_direct(p, d_points, s);
        } else {
            build_tree(p, d_points, s);
            build_tables(p, s);
            prepare_rel(p, s);
        }
        allocate_workspaces(p);
        FFMM_HIP(hipStreamSynchronize(s));
        *out = p;
    });
    if (st != FFMM_OK && p) {
        (void)hipDeviceSynchronize();
        release_streams(p);
        p->arena.release();
        delete p;
    }
    return st;
}


ffmm_status ffmm_matvec_stages(ffmm_plan* plan, const void* d_q, void* d_phi, int32_t nrhs,
                               int32_t stages, void* hip_stream)
{
    return guarded([&] {
        check_call(plan, d_q, d_phi, nrhs);
        if (stages < 1 || stages > FFMM_STAGE_ALL) fail(FFMM_ERR_INVALID_ARG, "bad stage mask");
        run_matvec(plan, d_q, d_phi, nrhs, stages, false, false, (hipStream_t)hip_stream);
        plan->has_run = true;
    });
}

ffmm_status ffmm_matvec(ffmm_plan* plan, const void* d_q, void* d_phi, int32_t nrhs, void* hip_stream)
{
    return ffmm_matvec_stages(plan, d_q, d_phi, nrhs, FFMM_STAGE_ALL, hip_stream);
}

ffmm_status ffmm_adjoint(ffmm_plan* plan, const void* d_g, void* d_out, int32_t nrhs, void* hip_stream)
{
    return guarded([&] {
        check_call(plan, d_g, d_out, nrhs);
        run_matvec(plan, d_g, d_out, nrhs, FFMM_STAGE_ALL, true, false, (hipStream_t)hip_stream);
        plan->has_run = true;
    });
}

ffmm_status ffmm_field_gradient(ffmm_plan* plan, const void* d_q, void* d_grad, int32_t nrhs,
                                void* hip_stream)
{
    return guarded([&] {
        check_call(plan, d_q, d_grad, nrhs);
        run_matvec(plan, d_q, d_grad, nrhs, FFMM_STAGE_ALL, false, true, (hipStream_t)hip_stream);
        plan->has_run = true;
    });
}

ffmm_status ffmm_position_gradient(ffmm_plan* plan, const void* d_q, const void* d_g, double* d_gx,
                                   int32_t nrhs, void* hip_stream)
{
    return guarded([&] {
        if (!plan) fail(FFMM_ERR_INVALID_ARG, "plan is NULL");
        if (!d_q || !d_g || !d_gx) fail(FFMM_ERR_INVALID_ARG, "input or output pointer is NULL");
        if ((const void*)d_gx == d_q || (const void*)d_gx == d_g)
            fail(FFMM_ERR_INVALID_ARG, "output must not alias an input");
        if (nrhs < 1) fail(FFMM_ERR_INVALID_ARG, "nrhs must be >= 1");
        run_position_gradient(plan, d_q, d_g, d_gx, nrhs, (hipStream_t)hip_stream);
        plan->has_run = true;
    });
}

static void check_tuning(const ffmm_tuning* t)
{
    if (!t) fail(FFMM_ERR_INVALID_ARG, "tuning is NULL");
    if (t->struct_size != (int32_t)sizeof(ffmm_tuning))
        fail(FFMM_ERR_INVALID_ARG, "tuning.struct_size does not match this library");
    if (t->near_stream < 0 || t->near_stream > 2) fail(FFMM_ERR_INVALID_ARG, "near_stream must be 0, 1 or 2");
    if (t->p2p_blocks_per_cu < 0 || t->p2p_blocks_per_cu > 16)
        fail(FFMM_ERR_INVALID_ARG, "p2p_blocks_per_cu must lie in [0, 16]");
    if (t->m2l_rhs_block != 0 && t->m2l_rhs_block != 1 && t->m2l_rhs_block != 2 && t->m2l_rhs_block != 4)
        fail(FFMM_ERR_INVALID_ARG, "m2l_rhs_block must be 0, 1, 2 or 4");
    for (int i = 0; i < 4; ++i)
        if (t->rs_slab[i] != 16 && t->rs_slab[i] != 32 && t->rs_slab[i] != 64)
            fail(FFMM_ERR_INVALID_ARG, "rs_slab entries must be 16, 32 or 64");
    if (t->m2l_by_parent < 0 || t->m2l_by_parent > 2) fail(FFMM_ERR_INVALID_ARG, "m2l_by_parent must be 0, 1 or 2");
    if (t->m2l_chunk != 32 && t->m2l_chunk != 48 && t->m2l_chunk != 64)
        fail(FFMM_ERR_INVALID_ARG, "m2l_chunk must be 32, 48 or 64");
}

ffmm_status ffmm_plan_set_tuning(ffmm_plan* p, const ffmm_tuning* t)
{
    return guarded([&] {
        if (!p) fail(FFMM_ERR_INVALID_ARG, "plan is NULL");
        check_tuning(t);
        p->tune = *t;
    });
}

ffmm_status ffmm_plan_get_tuning(const ffmm_plan* p, ffmm_tuning* out)
{
    return guarded([&] {
        if (!p || !out) fail(FFMM_ERR_INVALID_ARG, "NULL argument");
        *out = p->tune;
    });
}

ffmm_status ffmm_plan_autotune(ffmm_plan* p, const void* d_q, void* d_out, int32_t nrhs,
                               void* hip_stream, ffmm_tuning* best)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = p ? p->profile : false;
    ffmm_status st = guarded([&] {
        check_call(p, d_q, d_out, nrhs);
        hipStream_t s = (hipStream_t)hip_stream;
        p->profile = false;
        FFMM_HIP(hipEventCreate(&e0));
        FFMM_HIP(hipEventCreate(&e1));
        // time of one matvec under t: after one warm-up call, three groups of three calls back to
        // back (the steady state of repeated products, where one call's P2P and the next call's
        // far field meet), the best group's time per call
        auto measure = [&](const ffmm_tuning& t) {
            p->tune = t;
            run_matvec(p, d_q, d_out, nrhs, FFMM_STAGE_ALL, false, false, s);
            float best_ms = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                FFMM_HIP(hipEventRecord(e0, s));
                for (int c = 0; c < 3; ++c) run_matvec(p, d_q, d_out, nrhs, FFMM_STAGE_ALL, false, false, s);
                FFMM_HIP(hipEventRecord(e1, s));
                FFMM_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                FFMM_HIP(hipEventElapsedTime(&ms, e0, e1));
                best_ms = std::min(best_ms, ms / 3.0f);
            }
            return best_ms;
        };
        ffmm_tuning cur = p->tune;
        if (cur.m2l_rhs_block == 0) cur.m2l_rhs_block = nrhs >= 4 ? 4 : (nrhs >= 2 ? 2 : 1);
        const ffmm_tuning start = cur;
        // a few untimed calls first, so that the first configuration is not timed cold
        for (int w = 0; w < 3; ++w) run_matvec(p, d_q, d_out, nrhs, FFMM_STAGE_ALL, false, false, s);
        float cur_ms = measure(cur);
        // coordinate descent: each field in turn over its candidate values
        auto try_field = [&](int32_t* field, std::initializer_list<int32_t> values) {
            const int32_t keep = *field;
            for (int32_t v : values) {
                if (v == keep) continue;
                ffmm_tuning t = cur;
                *(int32_t*)((char*)&t + ((char*)field - (char*)&cur)) = v;
                const float ms = measure(t);
                if (ms < cur_ms) {
                    cur_ms = ms;
                    cur = t;
                }
            }
        };
        // the P2P placement and the M2L chunk width together (a 64-pair chunk takes the LDS a P2P
        // block beside it would need, so the best of one depends on the other)
        {
            const ffmm_tuning base = cur;
            for (int32_t ns : {1, 2, 0})
                for (int32_t bpc : {0, 1, 2, 4})
                    for (int32_t cw : {48, 64, 32}) {
                        if (ns == 0 && bpc != base.p2p_blocks_per_cu) continue;
                        if (p->prec != FFMM_FP32 && cw != base.m2l_chunk) continue;
                        ffmm_tuning t = base;
                        t.near_stream = ns;
                        t.p2p_blocks_per_cu = bpc;
                        t.m2l_chunk = cw;
                        if (t.near_stream == cur.near_stream && t.p2p_blocks_per_cu == cur.p2p_blocks_per_cu &&
                            t.m2l_chunk == cur.m2l_chunk)
                            continue;
                        const float ms = measure(t);
                        if (ms < cur_ms) {
                            cur_ms = ms;
                            cur = t;
                        }
                    }
        }
        try_field(&cur.m2l_by_parent, {2, 1, 0});
        if (nrhs >= 2) try_field(&cur.m2l_rhs_block, nrhs >= 4 ? std::initializer_list<int32_t>{1, 2, 4}
                                                              : std::initializer_list<int32_t>{1, 2});
        if (p->prec == FFMM_FP32)
            for (int i = 0; i < 4; ++i) try_field(&cur.rs_slab[i], {16, 32, 64});
        // the P2P grid once more, beside the far field as it now is
        try_field(&cur.p2p_blocks_per_cu, {0, 1, 2, 3, 4, 6, 8});
        // confirmation: the starting configuration, the descent's choice and that choice with the
        // other P2P placement, timed in turn over three rounds; the fastest is kept (one noisy
        // time early in the descent cannot then leave a slower configuration on the plan)
        ffmm_tuning cand[3] = {start, cur, cur};
        cand[2].near_stream = cur.near_stream == 1 ? 2 : 1;
        float cand_ms[3] = {1e30f, 1e30f, 1e30f};
        for (int round = 0; round < 3; ++round)
            for (int c = 0; c < 3; ++c) cand_ms[c] = std::min(cand_ms[c], measure(cand[c]));
        int win = 0;
        for (int c = 1; c < 3; ++c)
            if (cand_ms[c] < cand_ms[win]) win = c;
        cur = cand[win];
        p->tune = cur;
        if (best) *best = cur;
        p->has_run = true;
    });
    if (p) p->profile = prof;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return st;
}

ffmm_status ffmm_plan_info_get(const ffmm_plan* p, ffmm_plan_info* out)
{
    return guarded([&] {
        if (!p || !out) fail(FFMM_ERR_INVALID_ARG, "NULL argument");
        std::memset(out, 0, sizeof(*out));
        out->depth = p->depth;
        out->precision = p->prec;
        out->n_points = p->n;
        out->kappa = p->kappa;
        out->eps = p->eps;
        for (int a = 0; a < 3; ++a) out->root_lo[a] = p->lo[a];
        out->root_side = p->side;
        for (int l = 0; l <= p->depth; ++l) {
            const LevelData& L = p->lev[l];
            out->n_boxes[l] = L.n;
            if (l >= 2) {
                out->ell[l] = L.par.ell;
                out->ntheta[l] = L.par.ntheta;
                out->nphi_max[l] = *std::max_element(L.par.nphi.begin(), L.par.nphi.end());
                out->K[l] = L.K;
                out->n_ilist[l] = L.n_il;
                out->predicted_err[l] = p->predicted[l];
            }
        }
        out->n_near_pairs = p->near_pairs;
        out->device_bytes = (int64_t)p->arena.bytes;
        out->max_rhs = p->opt.max_rhs;
        out->method = p->direct ? FFMM_METHOD_DIRECT : FFMM_METHOD_FMM;
        out->max_leaf_count = p->max_leaf_count;
    });
}

ffmm_status ffmm_profile_enable(ffmm_plan* p, int32_t on)
{
    return guarded([&] {
        if (!p) fail(FFMM_ERR_INVALID_ARG, "plan is NULL");
        p->profile = on != 0;
    });
}

ffmm_status ffmm_profile_read(ffmm_plan* p, double* ms, int64_t* calls)
{
    return guarded([&] {
        if (!p) fail(FFMM_ERR_INVALID_ARG, "plan is NULL");
        drain_events(p, true);
        for (int i = 0; i < FFMM_PROF_NUM; ++i) {
            if (ms) ms[i] = p->prof_ms[i];
            if (calls) calls[i] = p->prof_calls[i];
            p->prof_ms[i] = 0.0;
            p->prof_calls[i] = 0;
        }
    });
}

ffmm_status ffmm_plan_destroy(ffmm_plan* p)
{
    return guarded([&] {
        if (!p) return;
        (void)hipDeviceSynchronize();
        drain_events(p, false);
        release_streams(p);
        p->arena.release();
        delete p;
    });
}

const char* ffmm_status_string(ffmm_status s)
{
    switch (s) {
    case FFMM_OK: return "ok";
    case FFMM_ERR_INVALID_ARG: return "invalid argument";
    case FFMM_ERR_OUT_OF_MEMORY: return "out of memory";
    case FFMM_ERR_HIP: return "HIP runtime error";
    case FFMM_ERR_UNSUPPORTED: return "unsupported";
    case FFMM_ERR_ACCURACY: return "accuracy target unreachable";
    case FFMM_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char* ffmm_last_error_message(void) { return g_last_error.c_str(); }

ffmm_status ffmm_select_level_params(double ka, double alpha, double eps, int32_t precision,
                                     int32_t ell_in, int32_t* ell, int32_t* ntheta, int32_t* nphi,
                                     int32_t nphi_cap, double* predicted)
{
    return guarded([&] {
        if (!ell || !ntheta || !nphi) fail(FFMM_ERR_INVALID_ARG, "NULL output");
        if (!(ka > 0.0) || !std::isfinite(ka)) fail(FFMM_ERR_INVALID_ARG, "ka must be finite and > 0");
        if (!(alpha > 0.0 && alpha <= 1.0)) fail(FFMM_ERR_INVALID_ARG, "alpha must lie in (0, 1]");
        if (!(eps > 0.0) || !std::isfinite(eps)) fail(FFMM_ERR_INVALID_ARG, "eps must be > 0");
        if (precision != FFMM_FP64 && precision != FFMM_FP32) fail(FFMM_ERR_INVALID_ARG, "precision");
        if (ell_in < 0 || ell_in > 2000) fail(FFMM_ERR_INVALID_ARG, "ell_in out of range");
        LevelParams lp;
        level_params(ka, alpha, eps, precision == FFMM_FP32 ? kUnitRoundoffFP32 : kUnitRoundoffFP64,
                     ell_in, &lp);
        if ((int)lp.nphi.size() > nphi_cap) fail(FFMM_ERR_INVALID_ARG, "nphi_cap too small");
        *ell = lp.ell;
        *ntheta = lp.ntheta;
        for (size_t i = 0; i < lp.nphi.size(); ++i) nphi[i] = lp.nphi[i];
        if (predicted) *predicted = lp.predicted;
    });
}

ffmm_status ffmm_plan_get_perm(const ffmm_plan* p, int64_t* perm)
{
    return guarded([&] {
        if (!p || !perm) fail(FFMM_ERR_INVALID_ARG, "NULL argument");
        FFMM_HIP(hipDeviceSynchronize());
        FFMM_HIP(hipMemcpy(perm, p->perm, sizeof(int64_t) * p->n, hipMemcpyDeviceToHost));
    });
}

ffmm_status ffmm_plan_get_level(const ffmm_plan* p, int32_t l, uint64_t* keys, int32_t* parent,
                                int32_t* start, int32_t* count, int32_t* il_ptr, int32_t* il_src,
                                int32_t* il_code, int32_t* nb_ptr, int32_t* nb_src)
{
    return guarded([&] {
        if (!p) fail(FFMM_ERR_INVALID_ARG, "plan is NULL");
        if (l < 0 || l > p->depth) fail(FFMM_ERR_INVALID_ARG, "level out of range");
        const LevelData& L = p->lev[l];
        FFMM_HIP(hipDeviceSynchronize());
        auto cp = [](void* dst, const void* src, size_t bytes) {
            if (dst && src && bytes) FFMM_HIP(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
        };
        cp(keys, L.keys, sizeof(uint64_t) * L.n);
        if (l >= 1) cp(parent, L.parent, sizeof(int32_t) * L.n);
        if (l == p->depth) {
            cp(start, p->leaf_start, sizeof(int32_t) * L.n);
            cp(count, p->leaf_count, sizeof(int32_t) * L.n);
            cp(nb_ptr, p->nb_ptr, sizeof(int32_t) * (L.n + 1));
            cp(nb_src, p->nb_src, sizeof(int32_t) * p->n_nb);
        }
        if (l >= 2) {
            cp(il_ptr, L.il_ptr, sizeof(int32_t) * (L.n + 1));
            cp(il_src, L.il_src, sizeof(int32_t) * L.n_il);
            cp(il_code, L.il_code, sizeof(int32_t) * L.n_il);
        }
    });
}

ffmm_status ffmm_plan_set_m2l_levels(ffmm_plan* p, uint32_t level_mask)
{
    return guarded([&] {
        if (!p) fail(FFMM_ERR_INVALID_ARG, "plan is NULL");
        p->m2l_levels = level_mask;
    });
}

ffmm_status ffmm_plan_get_nphi(const ffmm_plan* p, int32_t l, int32_t* nphi)
{
    return guarded([&] {
        if (!p || !nphi) fail(FFMM_ERR_INVALID_ARG, "NULL argument");
        if (l < 2 || l > p->depth) fail(FFMM_ERR_INVALID_ARG, "level out of range");
        const LevelData& L = p->lev[l];
        for (int i = 0; i < L.nrows; ++i) nphi[i] = L.par.nphi[i];
    });
}

static void copy_complex_to_f64(const ffmm_plan* p, const void* src, size_t count, double* out)
{
    FFMM_HIP(hipDeviceSynchronize());
    if (p->prec == FFMM_FP64) {
        FFMM_HIP(hipMemcpy(out, src, 16 * count, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(2 * count);
        FFMM_HIP(hipMemcpy(tmp.data(), src, 8 * count, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < 2 * count; ++i) out[i] = tmp[i];
    }
}

ffmm_status ffmm_plan_get_transfer(const ffmm_plan* p, int32_t l, int32_t code, double* out)
{
    return guarded([&] {
        if (!p || !out) fail(FFMM_ERR_INVALID_ARG, "NULL argument");
        if (l < 2 || l > p->depth) fail(FFMM_ERR_INVALID_ARG, "level out of range");
        if (code < 0 || code >= kNumCodes) fail(FFMM_ERR_INVALID_ARG, "code out of range");
        int rep, g;
        if (!offset_symmetry(code, &rep, &g))
            fail(FFMM_ERR_INVALID_ARG, "inner offset code has no transfer function");
        // T_{g rep}(s_k) = T_rep(s_{tperm[g][k]}): gather the representative's table
        const LevelData& L = p->lev[l];
        const char* base = (const char*)L.transfer + csize(p) * (size_t)rep * L.K;
        std::vector<double> t(2 * (size_t)L.K);
        copy_complex_to_f64(p, base, L.K, t.data());
        std::vector<int32_t> perm(L.K);
        FFMM_HIP(hipMemcpy(perm.data(), L.tperm + (size_t)g * L.K, sizeof(int32_t) * L.K,
                           hipMemcpyDeviceToHost));
        for (int k = 0; k < L.K; ++k) {
            out[2 * k] = t[2 * (size_t)perm[k]];
            out[2 * k + 1] = t[2 * (size_t)perm[k] + 1];
        }
    });
}

ffmm_status ffmm_plan_get_signature(const ffmm_plan* p, int32_t kind, int32_t l, int32_t rhs,
                                    double* out)
{
    return guarded([&] {
        if (!p || !out) fail(FFMM_ERR_INVALID_ARG, "NULL argument");
        if (l < 2 || l > p->depth) fail(FFMM_ERR_INVALID_ARG, "level out of range");
        if (kind != 0 && kind != 1) fail(FFMM_ERR_INVALID_ARG, "kind must be 0 (M) or 1 (L)");
        if (rhs < 0 || rhs >= p->opt.max_rhs) fail(FFMM_ERR_INVALID_ARG, "rhs out of range");
        if (!p->has_run) fail(FFMM_ERR_INVALID_ARG, "no matvec has run on this plan");
        const LevelData& L = p->lev[l];
        const void* sig = kind == 0 ? L.sigM : L.sigL;
        const char* base = (const char*)sig + csize(p) * (size_t)rhs * L.n * L.K;
        copy_complex_to_f64(p, base, (size_t)L.n * L.K, out);
    });
}

}  // extern "C"
