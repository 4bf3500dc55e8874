// Matrix-free, spin-factorised H.v -- the product the paper's Listing 1 forms
// from a stored CSR matrix, here with every element evaluated when needed (the
// improvement proposed at the end of Section 3.2).
//
// View x and y as D_up x D_dn row-major matrices (row = up rank, contiguous
// down rank).  For output element (u, d):
//   y[u,d] = (e_up[u] + e_dn[d] + W(s_up[u], s_dn[d])) x[u,d]         diagonal
//          + sum_{(d', a) in hop_dn(d)} a x[u, d']                    1 (x) H_dn
//          + sum_{(u', a) in hop_up(u)} a x[u', d]                    H_up (x) 1
//          + sum_q amp_q s_up s_dn x[mv_up_q(u), mv_dn_q(d)]          four-fermion terms
// Every term is "pulled" with the forward action on (u, d); that is exact
// because H is symmetric (the tables are symmetric and the four-fermion list is
// Hermitian, both checked at setup).
//
// Schedule: one workgroup owns R consecutive rows.  When R rows of x fit in
// LDS they are staged there and the down-spin gathers (random within a row)
// read LDS; the up-spin partner rows are read straight from memory, fully
// coalesced along d, with the hop entries wave-uniform.  The down-spin hop
// entries are in a 64-state sliced ELL layout, one coalesced load per hop per
// wave, reused across the R rows.  Workgroup -> row-group mapping is XCD-aware
// (consecutive row groups stay on one XCD so shared partner rows hit its L2).
#include <cmath>
#include <cstdlib>

#include "ed_internal.h"

namespace ed {

static constexpr int kLdsBudget = 163840 - 1024;

// Bijection of the launch order onto row groups that gives each XCD (work is
// dispatched round-robin over the 8 XCDs) a contiguous range of groups.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
    const int64_t q = G >> 3, rem = G & 7;
    const int64_t xcd = b & 7, i = b >> 3;
    return xcd * q + (xcd < rem ? xcd : rem) + i;
}

template <typename TX, typename TA>
__device__ __forceinline__ TA cross_term(const ApplyArgs<TX, TA> &a, uint32_t su, uint32_t sd, uint32_t cu,
                                         uint32_t cd) {
    TA c = (TA)0;
    if (a.umode == 1) {
        c = a.U0 * (TA)__popc(su & sd & a.umask);
    } else if (a.umode == 2) {
        uint32_t m = su & sd & a.umask;
        while (m) {
            const int b = __ffs(m) - 1;
            c += a.usite[b];
            m &= m - 1u;
        }
    }
    if (a.koff) c += a.xtab[(cu << a.koff) | cd];
    return c;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over the workgroup in a fixed order; result valid in thread 0.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < BS / 64; ++k) s += red[k];
    __syncthreads();
    return s;
}

// MODE 0: y = H x.  MODE 1: partials of <x,Hx> and <x,x>.  MODE 2: partials of
// ||Hx - theta x||^2.  TX = storage type of x and y, TA = arithmetic type.
template <typename TX, typename TA, int R, int BS, bool LDS, int MODE>
__global__ __launch_bounds__(BS) void k_apply(ApplyArgs<TX, TA> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[2][BS / 64];
    TX *xs = reinterpret_cast<TX *>(smem_raw);

    const int64_t ddn = a.ddn;
    const int64_t G = (a.dup + R - 1) / R;
    const int64_t g = xcd_remap(blockIdx.x, G);
    const int64_t u0 = g * R;
    const int nr = (int)((a.dup - u0) < R ? (a.dup - u0) : R);

    const TX *xrow[R];
#pragma unroll
    for (int r = 0; r < R; ++r) xrow[r] = a.x + (u0 + (r < nr ? r : 0)) * ddn;

    if constexpr (LDS) {
        for (int r = 0; r < nr; ++r)
            for (int64_t d = threadIdx.x; d < ddn; d += BS) xs[r * ddn + d] = xrow[r][d];
        __syncthreads();
    }

    TA eu[R];
    uint32_t su[R], cu[R];
    int32_t hb[R], he[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r < nr) {
            eu[r] = a.up_e[u0 + r];
            su[r] = a.up_st[u0 + r];
            cu[r] = a.up_c[u0 + r];
            hb[r] = a.up_off[u0 + r];
            he[r] = a.up_off[u0 + r + 1];
        } else {
            eu[r] = (TA)0;
            su[r] = 0u;
            cu[r] = 0u;
            hb[r] = 0;
            he[r] = 0;
        }
    }

    double p0 = 0.0, p1 = 0.0;
    const int lane = threadIdx.x & 63;
    for (int64_t d = threadIdx.x; d < ddn; d += BS) {
        const int64_t sl = d >> 6;
        const int32_t eb = a.dn_ell_off[sl], ee = a.dn_ell_off[sl + 1];
        const TA edn = a.dn_e[d];
        const uint32_t sd = a.dn_st[d];
        const uint32_t cd = a.dn_c[d];
        TA acc[R];
        TA xv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            xv[r] = LDS ? (TA)xs[r * ddn + d] : (TA)xrow[r][d];
            acc[r] = (eu[r] + edn + cross_term(a, su[r], sd, cu[r], cd)) * xv[r];
        }
        // 1 (x) H_dn: gathers within the row
        for (int32_t e = eb + lane; e < ee; e += 64) {
            const int32_t t = a.dn_ell_tgt[e];
            const TA s = a.dn_ell_sa[e];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += s * (LDS ? (TA)xs[r * ddn + t] : (TA)xrow[r][t]);
        }
        // H_up (x) 1: whole partner rows, coalesced along d
#pragma unroll
        for (int r = 0; r < R; ++r) {
            for (int32_t e = hb[r]; e < he[r]; ++e) {
                const int64_t src = a.up_tgt[e];
                acc[r] += a.up_sa[e] * (TA)a.x[src * ddn + d];
            }
        }
        // four-fermion terms: products of an up move and a down move
        for (int q = 0; q < a.nx; ++q) {
            const XTermDev<TA> xt = a.xt[q];
            const int32_t md = a.dn_mv[(int64_t)xt.dn_mv * ddn + d];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r >= nr) break;
                const int32_t mu = a.up_mv[(int64_t)xt.up_mv * a.dup + u0 + r];
                if (mu >= 0 && md >= 0) {
                    TA v = xt.amp * (TA)a.x[(int64_t)(mu >> 1) * ddn + (md >> 1)];
                    acc[r] += ((mu ^ md) & 1) ? -v : v;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r >= nr) break;
            if constexpr (MODE == 0) {
                a.y[(u0 + r) * ddn + d] = (TX)acc[r];
            } else if constexpr (MODE == 1) {
                p0 += (double)xv[r] * (double)acc[r];
                p1 += (double)xv[r] * (double)xv[r];
            } else {
                const double df = (double)acc[r] - a.theta * (double)xv[r];
                p0 += df * df;
            }
        }
    }
    if constexpr (MODE != 0) {
        const double s0 = block_sum<BS>(p0, red[0]);
        const double s1 = block_sum<BS>(p1, red[1]);
        if (threadIdx.x == 0) {
            a.partials[2 * (int64_t)blockIdx.x] = s0;
            a.partials[2 * (int64_t)blockIdx.x + 1] = s1;
        }
    }
}

// ---------------------------------------------------------- variant table --
struct Variant {
    int R, BS;
    bool lds;
    const char *name;
};
static const Variant kVariants[] = {
    {1, 256, true, "lds_r1_b256"},  {2, 256, true, "lds_r2_b256"},  {2, 512, true, "lds_r2_b512"},
    {4, 512, true, "lds_r4_b512"},  {1, 256, false, "gl_r1_b256"},  {2, 256, false, "gl_r2_b256"},
    {4, 256, false, "gl_r4_b256"},
};
static constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <typename TX, typename TA>
static ApplyArgs<TX, TA> make_args(const ed_ham_s *h, const void *x, void *y, double *partials, double theta);

template <>
ApplyArgs<double, double> make_args<double, double>(const ed_ham_s *h, const void *x, void *y, double *partials,
                                                    double theta) {
    ApplyArgs<double, double> a;
    const SpinTab &U = h->sp[0], &Dn = h->sp[1];
    a.x = (const double *)x;
    a.y = (double *)y;
    a.dup = h->dup;
    a.ddn = h->ddn;
    a.up_off = U.off.as<int32_t>();
    a.up_tgt = U.tgt.as<int32_t>();
    a.up_sa = U.sa64.as<double>();
    a.up_e = U.ediag64.as<double>();
    a.up_st = U.states.as<uint32_t>();
    a.up_c = U.cidx.as<uint8_t>();
    a.up_mv = U.mv.as<int32_t>();
    a.dn_ell_off = Dn.ell_off.as<int32_t>();
    a.dn_ell_tgt = Dn.ell_tgt.as<int32_t>();
    a.dn_ell_sa = Dn.ell_sa64.as<double>();
    a.dn_e = Dn.ediag64.as<double>();
    a.dn_st = Dn.states.as<uint32_t>();
    a.dn_c = Dn.cidx.as<uint8_t>();
    a.dn_mv = Dn.mv.as<int32_t>();
    a.umode = h->umode;
    a.umask = h->umask;
    a.U0 = h->U0;
    a.usite = h->usite64.as<double>();
    a.koff = h->koff;
    a.xtab = h->xtab64.as<double>();
    a.nx = h->nx;
    a.xt = h->xt64.as<XTermDev<double>>();
    a.partials = partials;
    a.theta = theta;
    return a;
}

template <>
ApplyArgs<float, float> make_args<float, float>(const ed_ham_s *h, const void *x, void *y, double *partials,
                                                double theta) {
    ApplyArgs<float, float> a;
    const SpinTab &U = h->sp[0], &Dn = h->sp[1];
    a.x = (const float *)x;
    a.y = (float *)y;
    a.dup = h->dup;
    a.ddn = h->ddn;
    a.up_off = U.off.as<int32_t>();
    a.up_tgt = U.tgt.as<int32_t>();
    a.up_sa = U.sa32.as<float>();
    a.up_e = U.ediag32.as<float>();
    a.up_st = U.states.as<uint32_t>();
    a.up_c = U.cidx.as<uint8_t>();
    a.up_mv = U.mv.as<int32_t>();
    a.dn_ell_off = Dn.ell_off.as<int32_t>();
    a.dn_ell_tgt = Dn.ell_tgt.as<int32_t>();
    a.dn_ell_sa = Dn.ell_sa32.as<float>();
    a.dn_e = Dn.ediag32.as<float>();
    a.dn_st = Dn.states.as<uint32_t>();
    a.dn_c = Dn.cidx.as<uint8_t>();
    a.dn_mv = Dn.mv.as<int32_t>();
    a.umode = h->umode;
    a.umask = h->umask;
    a.U0 = (float)h->U0;
    a.usite = h->usite32.as<float>();
    a.koff = h->koff;
    a.xtab = h->xtab32.as<float>();
    a.nx = h->nx;
    a.xt = h->xt32.as<XTermDev<float>>();
    a.partials = partials;
    a.theta = theta;
    return a;
}

// FP32-stored vectors with FP64 arithmetic and FP64 tables (refinement).
template <>
ApplyArgs<float, double> make_args<float, double>(const ed_ham_s *h, const void *x, void *y, double *partials,
                                                  double theta) {
    ApplyArgs<double, double> d = make_args<double, double>(h, nullptr, nullptr, partials, theta);
    ApplyArgs<float, double> a;
    std::memcpy(&a, &d, sizeof(a));  // identical layout apart from the x/y element type
    a.x = (const float *)x;
    a.y = (float *)y;
    return a;
}

template <typename TX, typename TA, int R, int BS, bool LDS, int MODE>
static void launch_one(const ApplyArgs<TX, TA> &a, int64_t G, hipStream_t s) {
    const size_t shm = LDS ? (size_t)R * (size_t)a.ddn * sizeof(TX) : 0;
    auto kern = k_apply<TX, TA, R, BS, LDS, MODE>;
    if (LDS) {
        static bool attr_set = false;
        if (!attr_set) {
            (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
            (void)hipGetLastError();
            attr_set = true;
        }
    }
    kern<<<(unsigned)G, BS, shm, s>>>(a);
    ED_LAUNCH_CHECK();
}

template <typename TX, typename TA, int MODE>
static void launch_variant(const ApplyArgs<TX, TA> &a, int v, hipStream_t s) {
    const Variant &V = kVariants[v];
    const int64_t G = (a.dup + V.R - 1) / V.R;
    switch (v) {
        case 0: launch_one<TX, TA, 1, 256, true, MODE>(a, G, s); break;
        case 1: launch_one<TX, TA, 2, 256, true, MODE>(a, G, s); break;
        case 2: launch_one<TX, TA, 2, 512, true, MODE>(a, G, s); break;
        case 3: launch_one<TX, TA, 4, 512, true, MODE>(a, G, s); break;
        case 4: launch_one<TX, TA, 1, 256, false, MODE>(a, G, s); break;
        case 5: launch_one<TX, TA, 2, 256, false, MODE>(a, G, s); break;
        case 6: launch_one<TX, TA, 4, 256, false, MODE>(a, G, s); break;
        default: fail(ED_EINVAL, "bad apply variant %d", v);
    }
}

static bool variant_fits(const ed_ham_s *h, int v, size_t elem) {
    const Variant &V = kVariants[v];
    if (!V.lds) return true;
    return (size_t)V.R * (size_t)h->ddn * elem <= (size_t)kLdsBudget;
}

int apply_variant_count(const ed_ham_s *) { return kNumVariants; }

const char *apply_variant_name(const ed_ham_s *, int v) {
    return (v >= 0 && v < kNumVariants) ? kVariants[v].name : "?";
}

static void launch_store(ed_ham_s *h, int v, const void *x, void *y, hipStream_t s) {
    if (h->prec == ED_FP64)
        launch_variant<double, double, 0>(make_args<double, double>(h, x, y, nullptr, 0.0), v, s);
    else
        launch_variant<float, float, 0>(make_args<float, float>(h, x, y, nullptr, 0.0), v, s);
}

void apply_launch_variant(ed_ham_s *h, int v, const void *x, void *y, hipStream_t s) {
    if (v < 0 || v >= kNumVariants) fail(ED_EINVAL, "apply variant %d out of range", v);
    const size_t elem = h->prec == ED_FP64 ? 8 : 4;
    if (!variant_fits(h, v, elem)) fail(ED_EINVAL, "apply variant %s needs more LDS than a workgroup has", kVariants[v].name);
    launch_store(h, v, x, y, s);
}

// First use on a handle: time every variant that fits on the caller's vectors
// (y is overwritten anyway) and keep the fastest.  ED_APPLY_VARIANT=<n> forces one.
static void tune(ed_ham_s *h, const void *x, void *y, hipStream_t s) {
    const size_t elem = h->prec == ED_FP64 ? 8 : 4;
    if (const char *env = std::getenv("ED_APPLY_VARIANT")) {
        const int v = std::atoi(env);
        if (v >= 0 && v < kNumVariants && variant_fits(h, v, elem)) {
            h->plan.variant = v;
            return;
        }
    }
    hipEvent_t e0, e1;
    ED_HIP(hipEventCreate(&e0));
    ED_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int bestv = -1;
    for (int v = 0; v < kNumVariants; ++v) {
        if (!variant_fits(h, v, elem)) continue;
        launch_store(h, v, x, y, s);  // warm-up
        ED_HIP(hipEventRecord(e0, s));
        for (int k = 0; k < 3; ++k) launch_store(h, v, x, y, s);
        ED_HIP(hipEventRecord(e1, s));
        ED_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        ED_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            bestv = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->plan.variant = bestv;
}

void apply_launch(ed_ham_s *h, const void *x, void *y, hipStream_t s) {
    if (h->plan.variant < 0) tune(h, x, y, s);
    launch_store(h, h->plan.variant, x, y, s);
}

// ------------------------------------------------------- FP64 refinement --
__global__ void k_sum_pairs(const double *part, int64_t n, double *out) {
    // fixed-order reduction of n (a, b) pairs by one workgroup of 256
    __shared__ double s0[256], s1[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s0[0];
        out[1] = s1[0];
    }
}

void ensure_redbuf(ed_ham_s *h, size_t doubles) {
    if (h->redbuf_doubles >= doubles) return;
    h->redbuf.alloc(doubles * sizeof(double));
    h->redbuf_doubles = doubles;
}

template <typename TX>
static void rayleigh_impl(ed_ham_s *h, const void *x, double *rq, double *resid, hipStream_t s) {
    // R = 1 global-gather schedule: valid for every sector size
    const int64_t G = h->dup;
    ensure_redbuf(h, (size_t)2 * G + 8);
    double *part = h->redbuf.as<double>();
    double *out = part + 2 * G;
    double hv[2];
    ApplyArgs<TX, double> a = make_args<TX, double>(h, x, nullptr, part, 0.0);
    launch_one<TX, double, 1, 256, false, 1>(a, G, s);
    k_sum_pairs<<<1, 256, 0, s>>>(part, G, out);
    ED_LAUNCH_CHECK();
    ED_HIP(hipMemcpyAsync(hv, out, sizeof(hv), hipMemcpyDeviceToHost, s));
    ED_HIP(hipStreamSynchronize(s));
    if (!(hv[1] > 0.0)) fail(ED_EINVAL, "ed_rayleigh: zero vector");
    const double theta = hv[0] / hv[1];
    a.theta = theta;
    launch_one<TX, double, 1, 256, false, 2>(a, G, s);
    k_sum_pairs<<<1, 256, 0, s>>>(part, G, out);
    ED_LAUNCH_CHECK();
    double r2[2];
    ED_HIP(hipMemcpyAsync(r2, out, sizeof(r2), hipMemcpyDeviceToHost, s));
    ED_HIP(hipStreamSynchronize(s));
    *rq = theta;
    *resid = std::sqrt(r2[0] / hv[1]);
}

void rayleigh_fp64(ed_ham_s *h, const void *x, double *rq, double *resid, hipStream_t s) {
    if (h->prec == ED_FP64)
        rayleigh_impl<double>(h, x, rq, resid, s);
    else
        rayleigh_impl<float>(h, x, rq, resid, s);
}

}  // namespace ed

using namespace ed;

extern "C" ed_status ed_apply_H(ed_ham_t h, const void *x, void *y, void *stream) {
    return guard([&] {
        if (!h) fail(ED_EINVAL, "ed_apply_H: NULL handle");
        if (!x || !y) fail(ED_EINVAL, "ed_apply_H: NULL vector");
        if (x == y) fail(ED_EINVAL, "ed_apply_H: x and y must not alias");
        DeviceGuard g(h->device);
        apply_launch(h, x, y, (hipStream_t)stream);
    });
}

extern "C" ed_status ed_apply_H_variant(ed_ham_t h, int variant, const void *x, void *y, void *stream) {
    return guard([&] {
        if (!h) fail(ED_EINVAL, "ed_apply_H_variant: NULL handle");
        if (!x || !y) fail(ED_EINVAL, "ed_apply_H_variant: NULL vector");
        if (x == y) fail(ED_EINVAL, "ed_apply_H_variant: x and y must not alias");
        DeviceGuard g(h->device);
        apply_launch_variant(h, variant, x, y, (hipStream_t)stream);
    });
}

extern "C" int ed_apply_variant_count(void) { return kNumVariants; }

extern "C" const char *ed_apply_variant_name(int v) { return apply_variant_name(nullptr, v); }

extern "C" int ed_apply_variant_fits(ed_ham_t h, int v) {
    if (!h || v < 0 || v >= kNumVariants) return 0;
    return variant_fits(h, v, h->prec == ED_FP64 ? 8 : 4) ? 1 : 0;
}

extern "C" int ed_apply_current_variant(ed_ham_t h) { return h ? h->plan.variant : -1; }

extern "C" ed_status ed_rayleigh(ed_ham_t h, const void *x, double *rq, double *resid, void *stream) {
    return guard([&] {
        if (!h || !x || !rq || !resid) fail(ED_EINVAL, "ed_rayleigh: NULL argument");
        DeviceGuard g(h->device);
        rayleigh_fp64(h, x, rq, resid, (hipStream_t)stream);
    });
}
