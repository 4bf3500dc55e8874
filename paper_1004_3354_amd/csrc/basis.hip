// Error model, binomial tables and the sector basis (combinatorial ranking).
//
// A one-spin basis state is an Ns-bit string with N bits set; its rank is the
// combinatorial-number-system value sum_j C(p_j, j+1) over the ascending set-bit
// positions p_0 < p_1 < ..., which equals its position in ascending numeric
// order.  The sector (N_up, N_dn) of the paper's block structure (dimensions in
// the Introduction and Table 1) is the product of the two one-spin bases.
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "ed_internal.h"

namespace ed {

static thread_local std::string g_err;

void clear_error() { g_err.clear(); }

void fail(ed_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    throw Failure{st};
}

void throw_hip(hipError_t e, const char *what, const char *file, int line) {
    fail(ED_EDEVICE, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
}

// ---------------------------------------------------------------- binomials --
__constant__ uint32_t c_binom[33][33];

uint64_t binom_host(int n, int k) {
    if (k < 0 || n < 0 || k > n) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
    return r;
}

void ensure_device_binomials() {
    static std::mutex mu;
    static bool done[64] = {false};
    int dev = 0;
    ED_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if (dev < 64 && done[dev]) return;
    uint32_t t[33][33];
    for (int n = 0; n <= 32; ++n)
        for (int k = 0; k <= 32; ++k) t[n][k] = (uint32_t)binom_host(n, k);
    ED_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_binom), t, sizeof(t)));
    if (dev < 64) done[dev] = true;
}

int64_t basis_rank_host(uint32_t s, int ns, int n) {
    if ((ns < 32 && (s >> ns) != 0) || __builtin_popcount(s) != n) return -1;
    int64_t r = 0;
    int j = 0;
    while (s) {
        int p = __builtin_ctz(s);
        r += (int64_t)binom_host(p, j + 1);
        ++j;
        s &= s - 1;
    }
    return r;
}

// ------------------------------------------------------------ device code --
__device__ __forceinline__ uint32_t unrank_state(uint32_t r, int ns, int n) {
    uint32_t s = 0;
    for (int p = ns - 1; p >= 0 && n > 0; --p) {
        const uint32_t c = c_binom[p][n];
        if (r >= c) {
            s |= 1u << p;
            r -= c;
            --n;
        }
    }
    return s;
}

__device__ __forceinline__ int64_t rank_state(uint32_t s, int ns, int n) {
    if ((ns < 32 && (s >> ns) != 0u) || __popc(s) != n) return -1;
    uint32_t r = 0;
    int j = 0;
    while (s) {
        const int p = __ffs(s) - 1;
        r += c_binom[p][j + 1];
        ++j;
        s &= s - 1u;
    }
    return (int64_t)r;
}

__global__ void k_unrank(uint32_t *out, int64_t dim, int ns, int n) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x)
        out[r] = unrank_state((uint32_t)r, ns, n);
}

__global__ void k_rank(const uint32_t *st, int64_t cnt, int ns, int n, int64_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = rank_state(st[i], ns, n);
}

void basis_generate(BasisData &b, int ns, int nup, int ndn) {
    ensure_device_binomials();
    b.ns = ns;
    b.n[0] = nup;
    b.n[1] = ndn;
    for (int s = 0; s < 2; ++s) {
        const uint64_t d = binom_host(ns, b.n[s]);
        if (d > 0x7fffffffull) fail(ED_ENOMEM, "one-spin dimension C(%d,%d) exceeds 2^31-1", ns, b.n[s]);
        b.dim[s] = (int64_t)d;
        b.states[s].alloc((size_t)d * sizeof(uint32_t));
        k_unrank<<<grid_for((int64_t)d, 256), 256>>>(b.states[s].as<uint32_t>(), (int64_t)d, ns, b.n[s]);
        ED_LAUNCH_CHECK();
    }
    ED_HIP(hipDeviceSynchronize());
}

// Used by the table builder: ranks of arbitrary states.
void basis_rank_launch(const uint32_t *st, int64_t cnt, int ns, int n, int64_t *out, hipStream_t s) {
    ensure_device_binomials();
    if (cnt <= 0) return;
    k_rank<<<grid_for(cnt, 256), 256, 0, s>>>(st, cnt, ns, n, out);
    ED_LAUNCH_CHECK();
}

}  // namespace ed

using namespace ed;

extern "C" const char *ed_last_error(void) { return g_err.c_str(); }

extern "C" const char *ed_version(void) { return "edhip 0.1 (gfx950)"; }

extern "C" ed_status ed_basis(int Ns, int Nup, int Ndn, ed_basis_t *out) {
    return guard([&] {
        if (!out) fail(ED_EINVAL, "ed_basis: out is NULL");
        *out = nullptr;
        if (Ns < 1 || Ns > 32) fail(ED_EINVAL, "ed_basis: Ns=%d outside [1, 32]", Ns);
        if (Nup < 0 || Nup > Ns || Ndn < 0 || Ndn > Ns)
            fail(ED_EINVAL, "ed_basis: (Nup, Ndn)=(%d, %d) outside [0, Ns=%d]", Nup, Ndn, Ns);
        ed_basis_s *b = new ed_basis_s();
        try {
            ED_HIP(hipGetDevice(&b->device));
            basis_generate(b->b, Ns, Nup, Ndn);
        } catch (...) {
            delete b;
            throw;
        }
        *out = b;
    });
}

extern "C" ed_status ed_basis_dims(ed_basis_t b, int64_t *Dup, int64_t *Ddn, int64_t *D) {
    return guard([&] {
        if (!b) fail(ED_EINVAL, "ed_basis_dims: NULL handle");
        if (Dup) *Dup = b->b.dim[0];
        if (Ddn) *Ddn = b->b.dim[1];
        if (D) *D = b->b.dim[0] * b->b.dim[1];
    });
}

extern "C" ed_status ed_basis_states(ed_basis_t b, int spin, uint32_t *host_out) {
    return guard([&] {
        if (!b) fail(ED_EINVAL, "ed_basis_states: NULL handle");
        if (spin != 0 && spin != 1) fail(ED_EINVAL, "ed_basis_states: spin must be 0 or 1");
        if (!host_out) fail(ED_EINVAL, "ed_basis_states: host_out is NULL");
        DeviceGuard g(b->device);
        ED_HIP(hipMemcpy(host_out, b->b.states[spin].p, (size_t)b->b.dim[spin] * sizeof(uint32_t),
                         hipMemcpyDeviceToHost));
    });
}

extern "C" ed_status ed_basis_rank(ed_basis_t b, int spin, const uint32_t *states, int64_t n,
                                   int64_t *ranks, void *stream) {
    return guard([&] {
        if (!b) fail(ED_EINVAL, "ed_basis_rank: NULL handle");
        if (spin != 0 && spin != 1) fail(ED_EINVAL, "ed_basis_rank: spin must be 0 or 1");
        if (n < 0) fail(ED_EINVAL, "ed_basis_rank: n < 0");
        if (n > 0 && (!states || !ranks)) fail(ED_EINVAL, "ed_basis_rank: NULL array");
        DeviceGuard g(b->device);
        basis_rank_launch(states, n, b->b.ns, b->b.n[spin], ranks, (hipStream_t)stream);
    });
}

extern "C" void ed_basis_free(ed_basis_t b) {
    if (!b) return;
    try {
        DeviceGuard g(b->device);
        delete b;
    } catch (...) {
    }
}
