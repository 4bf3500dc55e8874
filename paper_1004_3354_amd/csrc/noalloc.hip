// Allocation-free Rayleigh quotient.  ed_rayleigh keeps its per-workgroup
// partial sums in a reduction buffer the handle grows on demand; callers that
// must not allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid allocation) use ed_rayleigh_noalloc, whose
// partials live in a file-scope device array of fixed size instead.  Each GPU
// holds its own copy of the array for the life of the process; its device
// address is looked up once per device and kept.
#include <mutex>

#include "ed_internal.h"

namespace ed {

static constexpr int64_t kScratchPairs = 262144;  // (a, b) partial pairs: 4 MiB
static __device__ __align__(256) double scratch[2 * kScratchPairs + 8];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[64];  // device address of `scratch`, per device

// Address of this device's copy of `scratch` (the device must be current).
static double *scratch_ptr(int dev) {
    if (dev < 0 || dev >= 64) fail(ED_EDEVICE, "device %d outside [0, 64)", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(ED_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    return g_scratch_ptr[dev];
}

}  // namespace ed

using namespace ed;

extern "C" ed_status ed_rayleigh_noalloc(ed_ham_t h, const void *x, double *rq, double *resid, void *stream) {
    return guard([&] {
        if (!h || !x || !rq || !resid) fail(ED_EINVAL, "ed_rayleigh_noalloc: NULL argument");
        DeviceGuard g(h->device);
        const int64_t nb = rayleigh_pairs_cached(h);
        if (nb < 0) fail(ED_EINVAL, "ed_rayleigh_noalloc: the handle has no Rayleigh-quotient plan");
        if (nb > kScratchPairs)
            fail(ED_EINVAL, "ed_rayleigh_noalloc: the sector needs %lld partial sums, the static scratch holds %lld "
                 "(D_up x windows of the down basis); use ed_rayleigh",
                 (long long)nb, (long long)kScratchPairs);
        double *part = scratch_ptr(h->device);
        rayleigh_on(h, x, part, nb, rq, resid, (hipStream_t)stream);
    });
}
