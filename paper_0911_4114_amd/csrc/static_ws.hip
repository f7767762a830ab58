// Allocation-free matvec (ffmm_matvec_static): the product of ffmm_matvec with the per-call
// workspaces (the charges in Morton order, the far- and near-field partial results and the
// resample intermediates) taken from one file-scope device array instead of the plan's own
// buffers. The kernels are those of ffmm_matvec; only the workspace addresses differ.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // FFMM_STATIC_SCRATCH_BYTES
constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;

static_assert(kScratchBytes == FFMM_STATIC_SCRATCH_BYTES, "header and library disagree");

// One copy per GPU, held until the process ends. Host code never uses this name as an address:
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array, looked up on the first call on the device
// (with that device current).
void* scratch_ptr(int dev)
{
    if (dev < 0 || dev >= kMaxDevices)
        ffmm::fail(FFMM_ERR_UNSUPPORTED, "device index " + std::to_string(dev) + " beyond " +
                                             std::to_string(kMaxDevices));
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            ffmm::fail(FFMM_ERR_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_ptr[dev] = ptr;
    }
    return g_ptr[dev];
}

inline size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Swaps the plan's workspace pointers for regions of the static array for the length of one call
// and puts them back afterwards (also when the call fails).
struct WorkspaceSwap {
    ffmm_plan* p;
    void *qs, *phis, *phin, *s1, *s2;
    bool profile;
    WorkspaceSwap(ffmm_plan* plan, unsigned char* base, const size_t (&off)[5])
        : p(plan), qs(plan->qs), phis(plan->phis), phin(plan->phin), s1(plan->scratch1),
          s2(plan->scratch2), profile(plan->profile)
    {
        p->qs = base + off[0];
        p->phis = base + off[1];
        p->phin = base + off[2];
        p->scratch1 = base + off[3];
        p->scratch2 = base + off[4];
        p->profile = false;   // stage events would be created inside the call
    }
    ~WorkspaceSwap()
    {
        p->qs = qs;
        p->phis = phis;
        p->phin = phin;
        p->scratch1 = s1;
        p->scratch2 = s2;
        p->profile = profile;
    }
};

}  // namespace

extern "C" ffmm_status ffmm_matvec_static(ffmm_plan* plan, const void* d_q, void* d_phi, int32_t nrhs,
                                          void* hip_stream)
{
    return ffmm::guarded_call([&] {
        ffmm::check_call(plan, d_q, d_phi, nrhs);
        int dev = 0;
        FFMM_HIP(hipGetDevice(&dev));
        if (dev != plan->device)
            ffmm::fail(FFMM_ERR_INVALID_ARG, "the current device (" + std::to_string(dev) +
                                                 ") is not the plan's (" + std::to_string(plan->device) + ")");
        // regions: charges, far field, near field (one complex per point and right-hand side
        // each), the two resample intermediates (the plan's sizes per right-hand side)
        const size_t cs = plan->prec == FFMM_FP32 ? 8 : 16;
        const size_t r = (size_t)nrhs, mr = (size_t)plan->opt.max_rhs;
        const size_t vec = cs * r * (size_t)plan->n;
        const size_t need[5] = {vec, plan->direct ? 0 : vec, vec, plan->scratch1_bytes / mr * r,
                                plan->scratch2_bytes / mr * r};
        size_t off[5], total = 0;
        for (int i = 0; i < 5; ++i) {
            off[i] = total;
            total += align_up(need[i]);
        }
        if (total > kScratchBytes)
            ffmm::fail(FFMM_ERR_UNSUPPORTED,
                       "ffmm_matvec_static needs " + std::to_string(total) + " bytes of workspace for " +
                           std::to_string(nrhs) + " right-hand side(s) of this plan; the static array holds " +
                           std::to_string(kScratchBytes) + " (use ffmm_matvec)");
        unsigned char* base = (unsigned char*)scratch_ptr(dev);
        WorkspaceSwap sw(plan, base, off);
        ffmm::run_matvec(plan, d_q, d_phi, nrhs, FFMM_STAGE_ALL, false, false, (hipStream_t)hip_stream);
        plan->has_run = true;
    });
}
