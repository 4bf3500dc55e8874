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
#include <algorithm>
#include <climits>
#include <map>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>

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

// value of m[q] for a runtime q < NMV (unrolled select; m stays in registers)
template <int NMV>
__device__ __forceinline__ int32_t pick(const int32_t (&m)[NMV > 0 ? NMV : 1], int q) {
    int32_t v = -1;
#pragma unroll
    for (int k = 0; k < NMV; ++k) v = (k == q) ? m[k] : v;
    return v;
}

// Row-window kernel.  A workgroup owns R consecutive rows and one window
// [w0, w0 + wl) of down ranks (a run of states sharing their top bits, so most
// down-spin hops stay inside it); the R x wl block of x is staged in LDS.  Each
// thread owns one column at a time and keeps R accumulators, so every hop
// table entry is loaded once per R output elements.
// UPX = true: full product (diagonal, 1 (x) H_dn, H_up (x) 1, four-fermion terms).
// UPX = false: row-local part only (diagonal and 1 (x) H_dn), the first pass of
// the two-pass schedule.  MODE 0 stores y; MODE 1 / 2 write per-workgroup
// partials of <x,Hx>, <x,x> / ||Hx - theta x||^2 instead.
template <typename TX, typename TA, int R, int BS, int MODE, bool UPX, bool PK = false>
__global__ __launch_bounds__(BS) void k_apply(ApplyArgs<TX, TA> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[2][BS / 64];
    TX *xs = reinterpret_cast<TX *>(smem_raw);
    // packed hops: distinct amplitudes after the staged block
    TA *amps = reinterpret_cast<TA *>(smem_raw + (((size_t)R * a.wmax * sizeof(TX) + 15) & ~(size_t)15));
    // per-row partner lists (up hops, allowed four-fermion terms) staged once per
    // workgroup, so the inner loops issue independent vector loads whose row
    // addresses are LDS broadcasts
    constexpr int UL = PK ? 32 : 1, XL = PK ? 16 : 1;
    __shared__ int32_t u_src[R][UL];
    __shared__ TA u_amp[R][UL];
    __shared__ int32_t x_src[R][XL], x_tab[R][XL];
    __shared__ uint32_t x_bits[R][XL];
    __shared__ TA x_amp[R][XL];
    if constexpr (PK) {
        for (int k = threadIdx.x; k < a.namp; k += BS) amps[k] = a.amp_tab[k];
    }

    const int64_t ddn = a.ddn;
    const int nwin = a.nwin;
    const int64_t G = (a.dup + R - 1) / R;
    const int64_t t = xcd_remap(blockIdx.x, G * nwin);
    const int64_t g = t / nwin;
    const int wi = (int)(t - g * nwin);
    const int64_t u0 = g * R;
    const int nr = (int)((a.dup - u0) < R ? (a.dup - u0) : R);
    const int32_t w0 = a.win[wi].x, wl = a.win[wi].y;

    for (int r = 0; r < nr; ++r) {
        const TX *src = a.x + (u0 + r) * ddn + w0;
        for (int k = threadIdx.x; k < wl; k += BS) xs[r * wl + k] = src[k];
    }
    __syncthreads();

    TA eu[R];
    uint32_t su[R], cu[R];
    int32_t hb[R], he[R], xb[R], xe[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool ok = r < nr;
        const int64_t u = u0 + (ok ? r : 0);
        eu[r] = ok ? a.up_e[u] : (TA)0;
        su[r] = ok ? a.up_st[u] : 0u;
        cu[r] = ok ? a.up_c[u] : 0u;
        hb[r] = ok ? a.up_off[u] : 0;
        he[r] = ok ? a.up_off[u + 1] : 0;
        xb[r] = ok ? a.xl_off[u] : 0;
        xe[r] = ok ? a.xl_off[u + 1] : 0;
    }
    if constexpr (PK && UPX) {
        for (int k = threadIdx.x; k < R * UL; k += BS) {
            const int r = k / UL, q = k - r * UL;
            if (r < nr && hb[r] + q < he[r]) {
                u_src[r][q] = a.up_tgt[hb[r] + q];
                u_amp[r][q] = a.up_sa[hb[r] + q];
            }
        }
        for (int k = threadIdx.x; k < R * XL; k += BS) {
            const int r = k / XL, q = k - r * XL;
            if (r < nr && xb[r] + q < xe[r]) {
                x_src[r][q] = a.xl_src[xb[r] + q];
                x_tab[r][q] = a.xl_tab[xb[r] + q];
                x_amp[r][q] = a.xl_amp[xb[r] + q];
            }
        }
        __syncthreads();
    }
    double p0 = 0.0, p1 = 0.0;
    const int lane = threadIdx.x & 63;
    const int64_t dend = (int64_t)w0 + wl;
    for (int64_t d0 = (int64_t)(w0 & ~63); d0 < dend; d0 += BS) {
        const int64_t d = d0 + threadIdx.x;
        if (d < w0 || d >= dend) continue;
        const int32_t ld = (int32_t)(d - w0);
        const int64_t sl = d >> 6;
        const int32_t eb = a.dn_ell_off[sl], ee = a.dn_ell_off[sl + 1];
        const TA edn = a.dn_e[d];
        const uint32_t sd = a.dn_st[d];
        const uint32_t cd = a.dn_c[d];
        int32_t mvd[PK ? 8 : 1];
        if constexpr (PK && UPX) {
#pragma unroll
            for (int q = 0; q < 8; ++q) mvd[q] = q < a.nmv_dn ? a.dn_mv[(int64_t)q * ddn + d] : -1;
        }
        TA acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            acc[r] = (eu[r] + edn + cross_term(a, su[r], sd, cu[r], cd)) * (TA)xs[r * wl + ld];
        // 1 (x) H_dn: four table entries in flight; targets inside the window
        // come from LDS, the rest from memory
        for (int32_t e = eb + lane; e < ee; e += 256) {
            int32_t tt[4];
            TA ss[4];
            if constexpr (PK) {
                uint32_t pk[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) pk[k] = e + 64 * k < ee ? a.dn_ell_pk[e + 64 * k] : (uint32_t)d;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    tt[k] = (int32_t)(pk[k] & 0xFFFFFu);
                    ss[k] = amps[pk[k] >> 20];
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const bool ok = e + 64 * k < ee;
                    tt[k] = ok ? a.dn_ell_tgt[e + 64 * k] : (int32_t)d;
                    ss[k] = ok ? a.dn_ell_sa[e + 64 * k] : (TA)0;
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int32_t l = tt[k] - w0;
                if ((uint32_t)l < (uint32_t)wl) {
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] += ss[k] * (TA)xs[r * wl + l];
                } else {
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        acc[r] += ss[k] * (TA)a.x[(u0 + (r < nr ? r : 0)) * ddn + tt[k]];
                }
            }
        }
        if constexpr (UPX && PK) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int nu = he[r] - hb[r];
#pragma unroll 4
                for (int k = 0; k < nu; ++k) acc[r] += u_amp[r][k] * (TA)a.x[(int64_t)u_src[r][k] * ddn + d];
                const int nxr = xe[r] - xb[r];
#pragma unroll 2
                for (int k = 0; k < nxr; ++k) {
                    // partner rows are nearby rows (L2-resident); read from memory
                    // (a select between an LDS and a memory address would become
                    // one generic-address load)
                    const int32_t m = pick<8>(mvd, x_tab[r][k]);
                    const int64_t c = m >= 0 ? (int64_t)(m >> 1) : d;
                    TA v = (TA)a.x[(int64_t)x_src[r][k] * ddn + c];
                    v = m >= 0 ? ((m & 1) ? -v : v) : (TA)0;
                    acc[r] += x_amp[r][k] * v;
                }
            }
        } else if constexpr (UPX) {
            // H_up (x) 1: partner rows, coalesced along d
#pragma unroll
            for (int r = 0; r < R; ++r) {
                int32_t e = hb[r];
                for (; e + 4 <= he[r]; e += 4) {
                    const TA v0 = (TA)a.x[(int64_t)a.up_tgt[e] * ddn + d];
                    const TA v1 = (TA)a.x[(int64_t)a.up_tgt[e + 1] * ddn + d];
                    const TA v2 = (TA)a.x[(int64_t)a.up_tgt[e + 2] * ddn + d];
                    const TA v3 = (TA)a.x[(int64_t)a.up_tgt[e + 3] * ddn + d];
                    acc[r] += a.up_sa[e] * v0 + a.up_sa[e + 1] * v1 + a.up_sa[e + 2] * v2 + a.up_sa[e + 3] * v3;
                }
                for (; e < he[r]; ++e) acc[r] += a.up_sa[e] * (TA)a.x[(int64_t)a.up_tgt[e] * ddn + d];
            }
            // four-fermion terms allowed on each row: per-row list, branch-free gathers
#pragma unroll
            for (int r = 0; r < R; ++r) {
                for (int32_t e = xb[r]; e < xe[r]; ++e) {
                    const int32_t m = a.dn_mv[(int64_t)a.xl_tab[e] * ddn + d];
                    const int64_t c = m >= 0 ? (int64_t)(m >> 1) : d;
                    TA v = (TA)a.x[(int64_t)a.xl_src[e] * ddn + c];
                    v = m >= 0 ? ((m & 1) ? -v : v) : (TA)0;
                    acc[r] += a.xl_amp[e] * v;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r >= nr) break;
            if constexpr (MODE == 0) {
                a.y[(u0 + r) * ddn + d] = (TX)acc[r];
            } else if constexpr (MODE == 1) {
                const double xv = (double)xs[r * wl + ld];
                p0 += xv * (double)acc[r];
                p1 += xv * xv;
            } else {
                const double df = (double)acc[r] - a.theta * (double)xs[r * wl + ld];
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

// 4-vectors at element alignment, R-vectors, and their element access
template <typename TX>
struct V4 {
    typedef TX t __attribute__((ext_vector_type(4), aligned(sizeof(TX))));
};
template <typename TX, int R>
struct RV {
    typedef TX t __attribute__((ext_vector_type(R)));
};
template <typename TX>
struct RV<TX, 1> {
    typedef TX t;
};
template <typename TX, int R>
__device__ __forceinline__ TX rv_get(const typename RV<TX, R>::t &v, int r) {
    if constexpr (R == 1) return v;
    else return v[r];
}
// component q of an R-vector by selects (a partner read from the LDS tile is a
// whole-column vector load, so it is never merged with a scalar memory load of
// the same value into one generic-address load)
template <typename TX, int R>
__device__ __forceinline__ TX rv_pick(const typename RV<TX, R>::t &v, int q) {
    if constexpr (R == 1) return v;
    else {
        TX o = v[0];
#pragma unroll
        for (int k = 1; k < R; ++k) o = q == k ? v[k] : o;
        return o;
    }
}
template <typename TX, bool NT>
__device__ __forceinline__ void st4(TX *p, typename V4<TX>::t v) {
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<typename V4<TX>::t *>(p));
    else *reinterpret_cast<typename V4<TX>::t *>(p) = v;
}
template <typename TX>
__device__ __forceinline__ typename V4<TX>::t ld4(const TX *p) {
    return *reinterpret_cast<const typename V4<TX>::t *>(p);
}

// Column-stationary kernel.  A workgroup owns one window of down ranks (at
// most BS*CPT of them, a run of states sharing their top bits) and streams over
// `rw` consecutive rows.  Each thread owns CPT columns and keeps everything
// that depends only on the column in registers for the whole row stream: its
// down-spin hop entries (target as a window-local LDS index, or the global
// rank when the hop leaves the window, and signed amplitude), its one-spin
// diagonal piece and bit string, and its entries of the down move tables of
// the four-fermion terms.  Per row only independent gathers remain: the row
// window (double-buffered in LDS), the up-spin partner rows and the
// four-fermion partners, so many loads are in flight per wave.

template <typename TX, typename TA, int BS, int RR, int KMAX, int NMV, int XMAX, int MODE, bool UPX>
__global__ __launch_bounds__(BS) void k_cs(ApplyArgs<TX, TA> a, int rw) {
    // RR rows are processed per step (all their gathers in flight together);
    // LDS holds two buffers of RR row windows, transposed (column l of the step
    // at l * RR), so one LDS read serves the RR rows and is never merged with
    // the scalar memory read of an out-of-window partner into one
    // generic-address load.
    using RVt = typename RV<TX, RR>::t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[2][BS / 64];
    const int wm = a.wmax;
    TX *bufs = reinterpret_cast<TX *>(smem_raw);
    const int64_t ddn = a.ddn;
    const int nwin = a.nwin;
    const int64_t G = (a.dup + rw - 1) / rw;
    const int64_t t = xcd_remap(blockIdx.x, G * nwin);
    const int64_t g = t / nwin;
    const int wi = (int)(t - g * nwin);
    const int64_t u0 = g * rw;
    const int nr = (int)((a.dup - u0) < rw ? (a.dup - u0) : rw);
    const int32_t w0 = a.win[wi].x, wl = a.win[wi].y;

    const int32_t li = (int32_t)threadIdx.x;
    const bool act = li < wl;
    const int64_t d = (int64_t)w0 + (act ? li : 0);
    const int32_t ld = (int32_t)(d - w0);
    int32_t lt[KMAX];
    TA sa[KMAX];
    {
        const int32_t o = a.dn_off[d], n = a.dn_off[d + 1] - o;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const bool ok = k < n;
            const int32_t tg = ok ? a.dn_tgt[o + k] : (int32_t)d;
            const int32_t l = tg - w0;
            lt[k] = ((uint32_t)l < (uint32_t)wl) ? l : (-1 - tg);
            sa[k] = ok ? a.dn_sa[o + k] : (TA)0;
        }
    }
    const TA edn = a.dn_e[d];
    const uint32_t sdn = a.dn_st[d], cdn = a.dn_c[d];
    int32_t mvd[NMV > 0 ? NMV : 1];
#pragma unroll
    for (int q = 0; q < NMV; ++q) mvd[q] = q < a.nmv_dn ? a.dn_mv[(int64_t)q * ddn + d] : -1;

    // stage the first RR rows
    if (act) {
        RVt o;
#pragma unroll
        for (int rr = 0; rr < RR; ++rr) o[rr] = rr < nr ? a.x[(u0 + rr) * ddn + w0 + li] : (TX)0;
        *reinterpret_cast<RVt *>(bufs + (int64_t)li * RR) = o;
    }
    __syncthreads();

    double p0 = 0.0, p1 = 0.0;
    int step = 0;
    for (int r0 = 0; r0 < nr; r0 += RR, ++step) {
        TX *cur = bufs + ((step & 1) ? RR * wm : 0);
        TX *nxt = bufs + ((step & 1) ? 0 : RR * wm);
        TX pf[RR];
#pragma unroll
        for (int rr = 0; rr < RR; ++rr) {
            const int rn = r0 + RR + rr;
            pf[rr] = (rn < nr && act) ? a.x[(u0 + rn) * ddn + w0 + li] : (TX)0;
        }
        TA acc[RR], xv[RR];
        const RVt self = *reinterpret_cast<const RVt *>(cur + (int64_t)ld * RR);
#pragma unroll
        for (int rr = 0; rr < RR; ++rr) {
            const int r = r0 + rr;
            const int64_t u = u0 + (r < nr ? r : 0);
            xv[rr] = (TA)self[rr];
            acc[rr] = (a.up_e[u] + edn + cross_term(a, a.up_st[u], sdn, a.up_c[u], cdn)) * xv[rr];
        }
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int32_t l = lt[k];
            const bool in = l >= 0;
            const RVt w = *reinterpret_cast<const RVt *>(cur + (int64_t)(in ? l : 0) * RR);
#pragma unroll
            for (int rr = 0; rr < RR; ++rr) {
                TA v = (TA)w[rr];
                if (!in) v = (TA)a.x[(u0 + (r0 + rr < nr ? r0 + rr : 0)) * ddn + (-1 - l)];
                acc[rr] += sa[k] * v;
            }
        }
        if (act) {
#pragma unroll
            for (int rr = 0; rr < RR; ++rr) {
                const int r = r0 + rr;
                if (r >= nr) break;
                if constexpr (MODE == 0) {
                    a.y[(u0 + r) * ddn + d] = (TX)acc[rr];
                } else if constexpr (MODE == 1) {
                    p0 += (double)xv[rr] * (double)acc[rr];
                    p1 += (double)xv[rr] * (double)xv[rr];
                } else {
                    const double df = (double)acc[rr] - a.theta * (double)xv[rr];
                    p0 += df * df;
                }
            }
            RVt o;
#pragma unroll
            for (int rr = 0; rr < RR; ++rr) o[rr] = pf[rr];
            *reinterpret_cast<RVt *>(nxt + (int64_t)li * RR) = o;
        }
        __syncthreads();
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

// ------------------------------------------------------ transposed tiles --
// Row-tile kernel with the tile transposed in LDS.  A workgroup owns R rows and
// one window of down ranks; LDS holds the tile column-major (xs[l*R + r]), so
// one LDS read returns a column's values for all R rows and every down-spin
// hop entry serves R output elements.  Each thread owns four consecutive
// columns: x rows, partner rows and y move as 16-byte accesses (rows need only
// element alignment), and the down-spin entries of its four states come from
// the four-state packed ELL in one 16-byte load.  Thread chunks start at a
// multiple of 256 columns so that a wave covers exactly one ELL slice.
// UPX = true: full product.  UPX = false: everything but H_up (x) 1 (the row
// pass of the two-pass schedule).  NTY: y is stored non-temporally (kept out of
// the caches so that x stays resident).

// cross term with the per-site U values and the 4^koff table taken from LDS
// copies (the kernels that use it require koff <= 4)
template <typename TX, typename TA>
__device__ __forceinline__ TA cross_term_l(const ApplyArgs<TX, TA> &a, const TA *usl, const TA *xtl, uint32_t su,
                                           uint32_t sd, uint32_t cu, uint32_t cd) {
    TA c = (TA)0;
    if (a.umode == 1) {
        c = a.U0 * (TA)__popc(su & sd & a.umask);
    } else if (a.umode == 2) {
        uint32_t m = su & sd & a.umask;
        while (m) {
            c += usl[__ffs(m) - 1];
            m &= m - 1u;
        }
    }
    if (a.koff) c += xtl[(cu << a.koff) | cd];
    return c;
}

// GRP = true: the grouped-order tile schedule (work list; windows are whole
// down components, so every down hop reads the staged tile; four-fermion
// partners lie in other tiles and are read from memory; element offsets are
// 32-bit, D < 2^32).
template <typename TX, typename TA, int R, int BS, bool UPX, bool NTY, bool GRP = false>
__global__ __launch_bounds__(BS) void k_rt(ApplyArgs<TX, TA> a) {
    using RVt = typename RV<TX, R>::t;
    using V = typename V4<TX>::t;
    constexpr int UL = 32, XL = 16;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TX *xs = reinterpret_cast<TX *>(smem_raw);
    TA *amps = reinterpret_cast<TA *>(smem_raw + (((size_t)R * a.wmax * sizeof(TX) + 15) & ~(size_t)15));
    __shared__ int32_t u_src[R][UL];
    __shared__ TA u_amp[R][UL];
    __shared__ int32_t x_src[R][XL], x_tab[R][XL];
    __shared__ uint32_t x_bits[R][XL];
    __shared__ TA x_amp[R][XL];
    __shared__ TA usl[32], xtl[256];
    for (int k = threadIdx.x; k < a.namp; k += BS) amps[k] = a.amp_tab[k];
    if (a.umode == 2)
        for (int k = threadIdx.x; k < 32; k += BS) usl[k] = a.usite[k];
    if (a.koff && a.koff <= 4)
        for (int k = threadIdx.x; k < (1 << (2 * a.koff)); k += BS) xtl[k] = a.xtab[k];

    const int64_t ddn = a.ddn;
    int64_t u0;
    int nr, wi;
    if (a.items) {  // grouped schedules: tile-major work list
        const int4 it = a.items[blockIdx.x];
        if (it.y <= 0) return;  // padding item (the whole workgroup leaves before any barrier)
        u0 = it.x;
        nr = it.y;
        wi = it.z;
    } else {
        const int nwin = a.nwin;
        const int64_t G = (a.dup + R - 1) / R;
        const int64_t t = xcd_remap(blockIdx.x, G * nwin);
        const int64_t g = t / nwin;
        wi = (int)(t - g * nwin);
        u0 = g * R;
        nr = (int)((a.dup - u0) < R ? (a.dup - u0) : R);
    }
    // rank of the row in each slot of the tile (unused slots repeat slot 0)
    int32_t ur[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ur[r] = (int32_t)(u0 + (r < nr ? r : 0));
    const int32_t w0 = a.win[wi].x, wl = a.win[wi].y;
    const int64_t cb = (int64_t)(w0 & ~255), cend = (int64_t)w0 + wl;

    TA eu[R];
    uint32_t su[R], cu[R];
    int nu[R], nxl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool ok = r < nr;
        const int64_t u = ur[r];
        eu[r] = ok ? a.up_e[u] : (TA)0;
        su[r] = ok ? a.up_st[u] : 0u;
        cu[r] = ok ? a.up_c[u] : 0u;
        const int32_t hb = a.up_off[u], he = a.up_off[u + 1];
        const int n = ok && UPX ? he - hb : 0;
        nu[r] = (n + 3) & ~3;
        nxl[r] = ok ? a.xl_off[u + 1] - a.xl_off[u] : 0;
        for (int k = threadIdx.x; k < nu[r]; k += BS) {
            u_src[r][k] = k < n ? a.up_tgt[hb + k] : (int32_t)u;
            u_amp[r][k] = k < n ? a.up_sa[hb + k] : (TA)0;
        }
        const int32_t xb = a.xl_off[u];
        for (int k = threadIdx.x; k < nxl[r]; k += BS) {
            x_src[r][k] = a.xl_src[xb + k];
            x_tab[r][k] = a.xl_tab[xb + k];
            x_bits[r][k] = a.dn_mvb[a.xl_tab[xb + k]];
            x_amp[r][k] = a.xl_amp[xb + k];
        }
    }
    // stage the tile, transposed
    for (int64_t c = cb + 4 * (int64_t)threadIdx.x; c < cend; c += 4 * BS) {
        if (c + 4 <= w0) continue;
        TX v[R][4];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j) v[r][j] = (TX)0;
        if (c >= w0 && c + 4 <= cend) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < nr) {
                    const typename V4<TX>::t q = ld4(a.x + (int64_t)ur[r] * ddn + c);
                    v[r][0] = q.x; v[r][1] = q.y; v[r][2] = q.z; v[r][3] = q.w;
                }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (r < nr && c + j >= w0 && c + j < cend) v[r][j] = a.x[(int64_t)ur[r] * ddn + c + j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t l = c + j - w0;
            if (l >= 0 && l < wl) {
                RVt o;
                if constexpr (R == 1) o = v[0][j];
                else {
#pragma unroll
                    for (int r = 0; r < R; ++r) o[r] = v[r][j];
                }
                *reinterpret_cast<RVt *>(xs + l * R) = o;
            }
        }
    }
    __syncthreads();
    auto chunk = [&](auto full_tag, int64_t c) {
        constexpr bool FULL = decltype(full_tag)::value;
        TA edn[4];
        uint32_t sd[4], cd[4];
        if constexpr (FULL) {
            const V e = *reinterpret_cast<const V *>(a.dn_e + c);  // c is a multiple of 4
            const uint4 st = *reinterpret_cast<const uint4 *>(a.dn_st + c);
            const uint32_t cc = *reinterpret_cast<const uint32_t *>(a.dn_c + c);
            edn[0] = (TA)e.x; edn[1] = (TA)e.y; edn[2] = (TA)e.z; edn[3] = (TA)e.w;
            sd[0] = st.x; sd[1] = st.y; sd[2] = st.z; sd[3] = st.w;
#pragma unroll
            for (int j = 0; j < 4; ++j) cd[j] = (cc >> (8 * j)) & 0xFFu;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool ok = c + j < ddn;
                edn[j] = ok ? (TA)a.dn_e[c + j] : (TA)0;
                sd[j] = ok ? a.dn_st[c + j] : 0u;
                cd[j] = ok ? (uint32_t)a.dn_c[c + j] : 0u;
            }
        }
        TA acc[R][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t l = c + j - w0;
            const bool inw = FULL || (l >= 0 && l < wl);
            RVt v = *reinterpret_cast<const RVt *>(xs + (inw ? l : 0) * R);
            if (!inw) v = (RVt)0;
#pragma unroll
            for (int r = 0; r < R; ++r)
                acc[r][j] = (eu[r] + edn[j] + cross_term_l(a, usl, xtl, su[r], sd[j], cu[r], cd[j])) *
                            (TA)rv_get<TX, R>(v, r);
        }
        // 1 (x) H_dn
        {
            const int lane = threadIdx.x & 63;
            const int64_t sl = c >> 8;
            const int32_t eb = a.dn_ell4_off[sl];
            const int32_t kk = (a.dn_ell4_off[sl + 1] - eb) >> 6;
            const uint4 *ep = a.dn_ell4 + eb + lane;
#pragma unroll 2
            for (int32_t k = 0; k < kk; ++k) {
                const uint4 e = ep[(int64_t)k * 64];
                const uint32_t ev[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int32_t t = (int32_t)(ev[j] & 0xFFFFFu);
                    const TA am = amps[ev[j] >> 20];
                    const int32_t l = t - w0;
                    if constexpr (GRP) {  // the window holds the whole component
                        // (a ragged chunk also computes columns outside the window,
                        // whose results are discarded: keep their reads in the tile)
                        const uint32_t lc = FULL ? (uint32_t)l : min((uint32_t)l, (uint32_t)(wl - 1));
                        const RVt v = *reinterpret_cast<const RVt *>(xs + lc * R);
#pragma unroll
                        for (int r = 0; r < R; ++r) acc[r][j] += am * (TA)rv_get<TX, R>(v, r);
                    } else if ((uint32_t)l < (uint32_t)wl) {
                        const RVt v = *reinterpret_cast<const RVt *>(xs + (int64_t)l * R);
#pragma unroll
                        for (int r = 0; r < R; ++r) acc[r][j] += am * (TA)rv_get<TX, R>(v, r);
                    } else {
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            acc[r][j] += am * (TA)a.x[(int64_t)ur[r] * ddn + t];
                    }
                }
            }
        }
        // four-fermion terms
        if constexpr (GRP) {
            // both moves leave the tile's components: partners from memory
            if (a.nx) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r >= nr) break;
                    for (int k = 0; k < nxl[r]; ++k) {
                        const TX *src = a.x + (uint32_t)x_src[r][k] * (uint32_t)ddn;
                        const TA am = x_amp[r][k];
                        const int32_t *mp = a.dn_mv + (uint32_t)x_tab[r][k] * (uint32_t)ddn;
                        int32_t m[4];
                        if constexpr (FULL) {
                            const int4 t4 = *reinterpret_cast<const int4 *>(mp + c);
                            m[0] = t4.x; m[1] = t4.y; m[2] = t4.z; m[3] = t4.w;
                        } else {
#pragma unroll
                            for (int j = 0; j < 4; ++j) m[j] = c + j < ddn ? mp[c + j] : -1;
                        }
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            if (m[j] < 0) continue;
                            const TA v = (TA)src[(uint32_t)m[j] >> 1];
                            acc[r][j] += (m[j] & 1) ? -am * v : am * v;
                        }
                    }
                }
            }
        } else if (a.nx) {
        // the rows' lists are ordered by down move, so each move table entry is
        // loaded once for all rows of the tile
            int p[R];
#pragma unroll
            for (int r = 0; r < R; ++r) p[r] = 0;
            // packed move words of the four columns (one 16-byte load for all moves)
            uint32_t mvw[4] = {0u, 0u, 0u, 0u};
            if (a.dn_mvp) {
                if constexpr (FULL) {
                    const uint4 t4 = *reinterpret_cast<const uint4 *>(a.dn_mvp + c);
                    mvw[0] = t4.x; mvw[1] = t4.y; mvw[2] = t4.z; mvw[3] = t4.w;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) mvw[j] = c + j < ddn ? a.dn_mvp[c + j] : 0u;
                }
            }
            for (int q = 0; q < a.nmv_dn; ++q) {
                bool any = false;
#pragma unroll
                for (int r = 0; r < R; ++r) any |= (p[r] < nxl[r] && x_tab[r][p[r]] == q);
                if (!any) continue;
                int32_t m[4];
                if (a.dn_mvp) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint32_t f = (mvw[j] >> (5 * q)) & 31u;
                        m[j] = (f & 16u) ? (int32_t)(((c + j + (int64_t)(f & 7u) - 4) << 1) | ((f >> 3) & 1u)) : -1;
                    }
                } else {
                    const int32_t *mp = a.dn_mv + (int64_t)q * ddn + c;
                    if constexpr (FULL) {
                        int32_t tmp[4];
                        __builtin_memcpy(tmp, mp, 16);
#pragma unroll
                        for (int j = 0; j < 4; ++j) m[j] = tmp[j];
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) m[j] = c + j < ddn ? mp[j] : -1;
                    }
                }
                int32_t col[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) col[j] = m[j] >= 0 ? (m[j] >> 1) : (int32_t)(c + j < ddn ? c + j : ddn - 1);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    while (p[r] < nxl[r] && x_tab[r][p[r]] == q) {
                        const int k = p[r]++;
                        const int32_t srow = x_src[r][k];
                        const TA am = x_amp[r][k];
                        int32_t rs = -1;
#pragma unroll
                        for (int s2 = 0; s2 < R; ++s2)
                            if (s2 < nr && ur[s2] == srow) rs = s2;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int32_t lc = col[j] - w0;
                            // the LDS read is unconditional (clamped index) so that
                            // it is not merged with the memory read into one
                            // generic-address load
                            const bool in = (uint32_t)rs < (uint32_t)nr && (uint32_t)lc < (uint32_t)wl;
                            TA v;
                            if constexpr (R == 1) {
                                v = (TA)a.x[(int64_t)srow * ddn + col[j]];  // a partner row is never the row itself
                            } else {
                                const RVt w = *reinterpret_cast<const RVt *>(xs + (in ? (int64_t)lc : 0) * R);
                                v = (TA)rv_pick<TX, R>(w, rs);
                                if (!in) v = (TA)a.x[(int64_t)srow * ddn + col[j]];
                            }
                            v = m[j] >= 0 ? ((m[j] & 1) ? -v : v) : (TA)0;
                            acc[r][j] += am * v;
                        }
                    }
                }
            }
        }
        // H_up (x) 1: partner rows, four independent 16-byte loads at a time
        if constexpr (UPX) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r >= nr) break;
                for (int k = 0; k < nu[r]; k += 4) {
                    if constexpr (FULL) {
                        V v[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            v[i] = GRP ? ld4(a.x + (uint32_t)((uint32_t)u_src[r][k + i] * (uint32_t)ddn + (uint32_t)c))
                                       : ld4(a.x + (int64_t)u_src[r][k + i] * ddn + c);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const TA am = u_amp[r][k + i];
                            acc[r][0] += am * (TA)v[i].x;
                            acc[r][1] += am * (TA)v[i].y;
                            acc[r][2] += am * (TA)v[i].z;
                            acc[r][3] += am * (TA)v[i].w;
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const TA am = u_amp[r][k + i];
                            const TX *row = a.x + (int64_t)u_src[r][k + i] * ddn;
#pragma unroll
                            for (int j = 0; j < 4; ++j)
                                if (c + j < ddn) acc[r][j] += am * (TA)row[c + j];
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r >= nr) break;
            TX *yr = a.y + (int64_t)ur[r] * ddn;
            if constexpr (FULL) {
                V o;
                o.x = (TX)acc[r][0]; o.y = (TX)acc[r][1]; o.z = (TX)acc[r][2]; o.w = (TX)acc[r][3];
                st4<TX, NTY>(yr + c, o);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (c + j >= w0 && c + j < cend) yr[c + j] = (TX)acc[r][j];
            }
        }
    };
    for (int64_t c = cb + 4 * (int64_t)threadIdx.x; c < cend; c += 4 * BS) {
        if (c + 4 <= w0) continue;
        if (c >= w0 && c + 4 <= cend) chunk(std::true_type{}, c);
        else chunk(std::false_type{}, c);
    }
}

// Band pass of the two-pass transposed schedule: y += (H_up (x) 1) x over
// column bands, band-major, four columns per thread.  The partner row segments
// of the band in flight stay in the last-level cache; y is read and written
// non-temporally so it does not evict them.
template <typename TX, typename TA, int RB, int BS, bool XT = false>
__global__ __launch_bounds__(BS) void k_upb(ApplyArgs<TX, TA> a, int64_t band, int rw) {
    using V = typename V4<TX>::t;
    const int64_t ddn = a.ddn;
    const int64_t G = (a.dup + rw - 1) / rw;
    const int64_t bi = blockIdx.x / G;  // band-major
    const int64_t g = blockIdx.x - bi * G;
    const int64_t u0 = g * rw;
    const int nr = (int)((a.dup - u0) < rw ? (a.dup - u0) : rw);
    const int64_t c = bi * band + 4 * (int64_t)threadIdx.x;
    if (4 * (int64_t)threadIdx.x >= band || c >= ddn) return;
    const bool full = c + 4 <= ddn;
    for (int r0 = 0; r0 < nr; r0 += RB) {
        TA acc[RB][4];
        int64_t u[RB];
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
            u[rr] = u0 + (r0 + rr < nr ? r0 + rr : 0);
            const bool ok = r0 + rr < nr;
            if (ok && full) {
                const V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(a.y + u[rr] * ddn + c));
                acc[rr][0] = (TA)v.x; acc[rr][1] = (TA)v.y; acc[rr][2] = (TA)v.z; acc[rr][3] = (TA)v.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[rr][j] = (ok && c + j < ddn) ? (TA)a.y[u[rr] * ddn + c + j] : (TA)0;
            }
        }
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
            if (r0 + rr >= nr) break;
            const int32_t hb = a.up_off[u[rr]], he = a.up_off[u[rr] + 1];
            int32_t e = hb;
            if (full) {
                for (; e + 4 <= he; e += 4) {
                    V v[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[i] = ld4(a.x + (int64_t)a.up_tgt[e + i] * ddn + c);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const TA am = a.up_sa[e + i];
                        acc[rr][0] += am * (TA)v[i].x;
                        acc[rr][1] += am * (TA)v[i].y;
                        acc[rr][2] += am * (TA)v[i].z;
                        acc[rr][3] += am * (TA)v[i].w;
                    }
                }
                for (; e < he; ++e) {
                    const V v = ld4(a.x + (int64_t)a.up_tgt[e] * ddn + c);
                    const TA am = a.up_sa[e];
                    acc[rr][0] += am * (TA)v.x;
                    acc[rr][1] += am * (TA)v.y;
                    acc[rr][2] += am * (TA)v.z;
                    acc[rr][3] += am * (TA)v.w;
                }
            } else {
                for (; e < he; ++e) {
                    const TX *row = a.x + (int64_t)a.up_tgt[e] * ddn;
                    const TA am = a.up_sa[e];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (c + j < ddn) acc[rr][j] += am * (TA)row[c + j];
                }
            }
        }
        if constexpr (XT) {
            // four-fermion terms; each row's list is ordered by down move, so
            // a move table entry is loaded once for the RB rows
            uint32_t mvw[4] = {0u, 0u, 0u, 0u};
            if (a.dn_mvp) {
                if (full) {
                    const uint4 t4 = *reinterpret_cast<const uint4 *>(a.dn_mvp + c);
                    mvw[0] = t4.x; mvw[1] = t4.y; mvw[2] = t4.z; mvw[3] = t4.w;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) mvw[j] = c + j < ddn ? a.dn_mvp[c + j] : 0u;
                }
            }
            int p[RB], pe[RB];
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
                const bool ok = r0 + rr < nr;
                p[rr] = ok ? a.xl_off[u[rr]] : 0;
                pe[rr] = ok ? a.xl_off[u[rr] + 1] : 0;
            }
            for (int q = 0; q < a.nmv_dn; ++q) {
                bool hit = false;
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) hit |= (p[rr] < pe[rr] && a.xl_tab[p[rr]] == q);
                if (!hit) continue;
                int32_t m[4];
                if (a.dn_mvp) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint32_t f = (mvw[j] >> (5 * q)) & 31u;
                        m[j] = (f & 16u) ? (int32_t)(((c + j + (int64_t)(f & 7u) - 4) << 1) | ((f >> 3) & 1u)) : -1;
                    }
                } else {
                    const int32_t *mp = a.dn_mv + (int64_t)q * ddn + c;
                    if (full) {
                        int32_t tmp[4];
                        __builtin_memcpy(tmp, mp, 16);
#pragma unroll
                        for (int j = 0; j < 4; ++j) m[j] = tmp[j];
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) m[j] = c + j < ddn ? mp[j] : -1;
                    }
                }
                int64_t col[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) col[j] = m[j] >= 0 ? (int64_t)(m[j] >> 1) : (c + j < ddn ? c + j : ddn - 1);
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) {
                    while (p[rr] < pe[rr] && a.xl_tab[p[rr]] == q) {
                        const TX *src = a.x + (int64_t)a.xl_src[p[rr]] * ddn;
                        const TA am = a.xl_amp[p[rr]];
                        ++p[rr];
                        TA v[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) v[j] = (TA)src[col[j]];
#pragma unroll
                        for (int j = 0; j < 4; ++j) acc[rr][j] += m[j] >= 0 ? ((m[j] & 1) ? -am * v[j] : am * v[j]) : (TA)0;
                    }
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) {
            if (r0 + rr >= nr) break;
            TX *yr = a.y + u[rr] * ddn;
            if (full) {
                V o;
                o.x = (TX)acc[rr][0]; o.y = (TX)acc[rr][1]; o.z = (TX)acc[rr][2]; o.w = (TX)acc[rr][3];
                st4<TX, true>(yr + c, o);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (c + j < ddn) yr[c + j] = (TX)acc[rr][j];
            }
        }
    }
}

// Band pass over a work list (grouped schedules): y[u, band] += (H_up (x) 1) x
// for the rows [u0, u0 + rows) of one item and one band of BAND columns.
// In the grouped order an up component's rows are contiguous and every up hop
// stays inside the component, so the items of one (component, band) tile run
// on one XCD one after another and the tile's slice of x (rows x BAND) stays
// in that XCD's L2 while its rows read it.  BS threads: BAND/4 column lanes x
// BS/(BAND/4) row lanes, four consecutive columns per thread (16-byte
// accesses at element alignment); y is read and written non-temporally.
template <typename TX, typename TA, int BS, int BAND>
__global__ __launch_bounds__(BS) void k_upt(ApplyArgs<TX, TA> a) {
    using V = typename V4<TX>::t;
    constexpr int CL = BAND / 4, RL = BS / CL;
    static_assert(BS % CL == 0, "band must divide the workgroup");
    const int4 it = a.items[blockIdx.x];
    const int64_t ddn = a.ddn;
    const int cl = (int)threadIdx.x % CL, rl = (int)threadIdx.x / CL;
    const int64_t c = (int64_t)it.z * BAND + 4 * cl;
    if (it.y <= 0 || c >= ddn) return;  // no barriers in this kernel
    const bool full = c + 4 <= ddn;
    for (int r = rl; r < it.y; r += RL) {
        const int64_t u = (int64_t)it.x + r;
        TX *yr = a.y + u * ddn;
        TA acc[4];
        if (full) {
            const V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(yr + c));
            acc[0] = (TA)v.x; acc[1] = (TA)v.y; acc[2] = (TA)v.z; acc[3] = (TA)v.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = c + j < ddn ? (TA)yr[c + j] : (TA)0;
        }
        const int32_t hb = a.up_off[u], he = a.up_off[u + 1];
        int32_t e = hb;
        if (full) {
            for (; e + 4 <= he; e += 4) {
                V v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = ld4(a.x + (int64_t)a.up_tgt[e + i] * ddn + c);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const TA am = a.up_sa[e + i];
                    acc[0] += am * (TA)v[i].x;
                    acc[1] += am * (TA)v[i].y;
                    acc[2] += am * (TA)v[i].z;
                    acc[3] += am * (TA)v[i].w;
                }
            }
            for (; e < he; ++e) {
                const V v = ld4(a.x + (int64_t)a.up_tgt[e] * ddn + c);
                const TA am = a.up_sa[e];
                acc[0] += am * (TA)v.x;
                acc[1] += am * (TA)v.y;
                acc[2] += am * (TA)v.z;
                acc[3] += am * (TA)v.w;
            }
            V o;
            o.x = (TX)acc[0]; o.y = (TX)acc[1]; o.z = (TX)acc[2]; o.w = (TX)acc[3];
            st4<TX, true>(yr + c, o);
        } else {
            for (; e < he; ++e) {
                const TX *row = a.x + (int64_t)a.up_tgt[e] * ddn;
                const TA am = a.up_sa[e];
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (c + j < ddn) acc[j] += am * (TA)row[c + j];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (c + j < ddn) yr[c + j] = (TX)acc[j];
        }
    }
}

// ------------------------------------------------- grouped tile kernel --
// k_gtile: grouped basis order.  A workgroup takes one work item: R rows of
// one up component and one window of whole down components (every down hop
// stays in it), staged in LDS transposed (xs[l*R + r]: one LDS read returns a
// column's values for all R rows, so each down-hop table entry serves R
// outputs; small windows leave room for many rows).  Threads own four
// consecutive columns of the window, whose own copy of the down hop table
// holds window-local targets (no range test per hop).  H_up (x) 1 reads the
// partner rows of the component from memory: with the XCD-partitioned work
// list the items of a tile run on one XCD one after another, so those rows'
// window segments are L2 hits; with the shared list (tiles too large for an
// L2) the whole chip runs one tile at a time and they are Infinity Cache hits.
// The four-fermion terms move both spins to other components and read memory.
// UPX = false leaves H_up (x) 1 to a band pass.  Element offsets are 32-bit
// (D < 2^32).
// FOLD: the cross term is one table over the fk sites of every w_ud entry
// (diagonal = e_up + e_dn + T[(c_up << fk) | c_dn]); otherwise it is a uniform
// on-site U, U0 popc(s_up & s_dn & umask), and nothing else.
template <typename TX, typename TA, int R, int BS, bool UPX, bool FOLD, bool H16>
__device__ __forceinline__ void gtile_body(const ApplyArgs<TX, TA> &a) {
    using RVt = typename RV<TX, R>::t;
    using V = typename V4<TX>::t;
    constexpr int UL = 32, XL = 16;
    static_assert(BS % 64 == 0, "workgroups of whole waves");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TX *xs = reinterpret_cast<TX *>(smem_raw);
    TA *amps = reinterpret_cast<TA *>(smem_raw + (((size_t)R * a.wmax * sizeof(TX) + 15) & ~(size_t)15));
    __shared__ int32_t u_src[R][UL];
    __shared__ TA u_amp[R][UL];
    __shared__ int32_t x_src[R][XL], x_tab[R][XL];
    __shared__ uint32_t x_bits[R][XL];
    __shared__ TA x_amp[R][XL];
    __shared__ TA usl[32], xtl[256];
    const int4 it = a.items[blockIdx.x];
    if (it.y <= 0) return;  // padding item: the whole workgroup leaves before any barrier
    const uint32_t ddn = (uint32_t)a.ddn;
    const int nr = it.y, wi = it.z;
    const uint32_t w0 = (uint32_t)a.win[wi].x;
    const int wl = a.win[wi].y;
    for (int k = threadIdx.x; k < a.namp; k += BS) amps[k] = a.amp_tab[k];
    if constexpr (FOLD)
        for (int k = threadIdx.x; k < (1 << (2 * a.fk)); k += BS) xtl[k] = a.ftab[k];
    uint32_t ur[R], su[R], cu[R];
    TA eu[R];
    int nu[R], nxl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool ok = r < nr;
        const uint32_t u = (uint32_t)it.x + (ok ? r : 0);
        ur[r] = u;
        eu[r] = ok ? a.up_e[u] : (TA)0;
        if constexpr (FOLD) {
            su[r] = 0u;
            cu[r] = ok ? ((uint32_t)a.up_fc[u] << a.fk) : 0u;
        } else {
            su[r] = ok ? (a.up_st[u] & a.umask) : 0u;
            cu[r] = 0u;
        }
        const int32_t hb = a.up_off[u];
        const int n = ok && UPX ? a.up_off[u + 1] - hb : 0;
        nu[r] = n;
        for (int k = threadIdx.x; k < n; k += BS) {
            u_src[r][k] = a.up_tgt[hb + k];
            u_amp[r][k] = a.up_sa[hb + k];
        }
        const int32_t xb = a.xl_off[u];
        nxl[r] = ok ? a.xl_off[u + 1] - xb : 0;
        for (int k = threadIdx.x; k < nxl[r]; k += BS) {
            x_src[r][k] = a.xl_src[xb + k];
            x_tab[r][k] = a.xl_tab[xb + k];
            x_bits[r][k] = a.dn_mvb[a.xl_tab[xb + k]];
            x_amp[r][k] = a.xl_amp[xb + k];
        }
    }
    // stage the tile, transposed
    for (int cl = 4 * (int)threadIdx.x; cl < wl; cl += 4 * BS) {
        TX v[R][4];
        if (cl + 4 <= wl) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const V q = ld4(a.x + (ur[r] * ddn + w0 + (uint32_t)cl));
                v[r][0] = q.x; v[r][1] = q.y; v[r][2] = q.z; v[r][3] = q.w;
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = 0; j < 4; ++j) v[r][j] = cl + j < wl ? a.x[ur[r] * ddn + w0 + (uint32_t)(cl + j)] : (TX)0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (cl + j >= wl) break;
            RVt o;
            if constexpr (R == 1) o = v[0][j];
            else {
#pragma unroll
                for (int r = 0; r < R; ++r) o[r] = v[r][j];
            }
            *reinterpret_cast<RVt *>(xs + (uint32_t)(cl + j) * R) = o;
        }
    }
    __syncthreads();
    const int lane = (int)threadIdx.x & 63;
    const int32_t gs0 = a.wsl_first[wi];
    for (int cl = 4 * (int)threadIdx.x; cl < wl; cl += 4 * BS) {
        const bool full = cl + 4 <= wl;
        const uint32_t c = w0 + (uint32_t)cl;
        // the column data first (the diagonal depends on it), one 16-byte load
        // per array for the four columns
        TA edn[4];
        uint32_t cd[4];
        if (full) {
            const typename V4<TA>::t e4 = ld4(a.dn_e + c);
            const typename V4<uint32_t>::t c4 = ld4(FOLD ? a.dn_fc32 + c : a.dn_st + c);
            edn[0] = e4.x; edn[1] = e4.y; edn[2] = e4.z; edn[3] = e4.w;
            cd[0] = c4.x; cd[1] = c4.y; cd[2] = c4.z; cd[3] = c4.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t q = c + (uint32_t)min(j, wl - 1 - cl);  // ragged end: repeat the last column
                edn[j] = (TA)a.dn_e[q];
                if constexpr (FOLD) cd[j] = a.dn_fc32[q];
                else cd[j] = a.dn_st[q];
            }
        }
        TA acc[R][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t l = (uint32_t)min(cl + j, wl - 1);
            const RVt v = *reinterpret_cast<const RVt *>(xs + l * R);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                TA dg;
                if constexpr (FOLD) dg = eu[r] + edn[j] + xtl[cu[r] | cd[j]];
                else dg = eu[r] + edn[j] + a.U0 * (TA)__popc(su[r] & cd[j]);
                acc[r][j] = dg * (TA)rv_get<TX, R>(v, r);
            }
        }
        // 1 (x) H_dn: the window's table (padding entries have amplitude 0
        // and a target inside the window)
        {
            const int32_t gs = gs0 + (cl >> 8);
            const int32_t eb = a.wsl_off[gs];
            const int32_t kk = (a.wsl_off[gs + 1] - eb) >> 6;
            const uint4 *ep = a.wel4 + eb + lane;
            if constexpr (H16) {
                // 16-bit entries: one 16-byte load gives two hops of the four columns
                for (int32_t k = 0; k < kk; ++k) {
                    const uint4 e = ep[k * 64];
                    const uint32_t ew[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
                    for (int hk = 0; hk < 2; ++hk)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const uint32_t h = (ew[2 * hk + (j >> 1)] >> (16 * (j & 1))) & 0xFFFFu;
                            const TA am = amps[h >> 10];
                            const RVt v = *reinterpret_cast<const RVt *>(xs + (h & 0x3FFu) * R);
#pragma unroll
                            for (int r = 0; r < R; ++r) acc[r][j] += am * (TA)rv_get<TX, R>(v, r);
                        }
                }
            } else {
#pragma unroll 2
                for (int32_t k = 0; k < kk; ++k) {
                    const uint4 e = ep[k * 64];
                    const uint32_t ev[4] = {e.x, e.y, e.z, e.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const TA am = amps[ev[j] >> 20];
                        const RVt v = *reinterpret_cast<const RVt *>(xs + (ev[j] & 0xFFFFFu) * R);
#pragma unroll
                        for (int r = 0; r < R; ++r) acc[r][j] += am * (TA)rv_get<TX, R>(v, r);
                    }
                }
            }
        }
        // H_up (x) 1: partner rows of the component, four 16-byte loads in
        // flight, then the row's last one to three partners
        if constexpr (UPX) {
            // several rows: their first partners in common groups of four, so
            // that 4 R loads are in flight together
            int kc = 0;
            if constexpr (R > 1) {
                if (full) {
                    kc = nu[0];
#pragma unroll
                    for (int r = 1; r < R; ++r) kc = r < nr ? min(kc, nu[r]) : kc;
                    kc &= ~3;
                    for (int k = 0; k < kc; k += 4) {
                        V v[R][4];
#pragma unroll
                        for (int r = 0; r < R; ++r)
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                v[r][i] = ld4(a.x + ((uint32_t)u_src[r < nr ? r : 0][k + i] * ddn + c));
#pragma unroll
                        for (int r = 0; r < R; ++r)
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const TA am = r < nr ? u_amp[r][k + i] : (TA)0;
                                acc[r][0] += am * (TA)v[r][i].x;
                                acc[r][1] += am * (TA)v[r][i].y;
                                acc[r][2] += am * (TA)v[r][i].z;
                                acc[r][3] += am * (TA)v[r][i].w;
                            }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r >= nr) break;
                if (full) {
                    int k = kc;
                    for (; k + 4 <= nu[r]; k += 4) {
                        V v[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) v[i] = ld4(a.x + ((uint32_t)u_src[r][k + i] * ddn + c));
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const TA am = u_amp[r][k + i];
                            acc[r][0] += am * (TA)v[i].x;
                            acc[r][1] += am * (TA)v[i].y;
                            acc[r][2] += am * (TA)v[i].z;
                            acc[r][3] += am * (TA)v[i].w;
                        }
                    }
                    for (; k < nu[r]; ++k) {
                        const V v = ld4(a.x + ((uint32_t)u_src[r][k] * ddn + c));
                        const TA am = u_amp[r][k];
                        acc[r][0] += am * (TA)v.x;
                        acc[r][1] += am * (TA)v.y;
                        acc[r][2] += am * (TA)v.z;
                        acc[r][3] += am * (TA)v.w;
                    }
                } else {
                    for (int k = 0; k < nu[r]; ++k) {
                        const TA am = u_amp[r][k];
                        const TX *row = a.x + (uint32_t)u_src[r][k] * ddn;
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (cl + j < wl) acc[r][j] += am * (TA)row[c + j];
                    }
                }
            }
        }
        // four-fermion terms: partners in other components, from memory.  A
        // thread none of whose columns has the term's down move (a test on the
        // column words it already holds) skips the term, table read included;
        // the others load only their valid columns' partners.  The rows' k-th
        // terms go together, so their table reads and then their partner
        // loads are in flight at once.
        if (a.nx) {
            int kx = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) kx = r < nr ? max(kx, nxl[r]) : kx;
#pragma unroll 2
            for (int k = 0; k < kx; ++k) {
                bool go[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    go[r] = r < nr && k < nxl[r];
                    if (go[r]) {
                        const uint32_t mb = x_bits[r][k];
                        if (mb >> 31) {
                            const uint32_t sb = mb & 0xFFu, db = (mb >> 8) & 0xFFu;
                            uint32_t any = 0u;
#pragma unroll
                            for (int j = 0; j < 4; ++j) any |= (cd[j] >> sb) & ~(cd[j] >> db);
                            go[r] = (any & 1u) != 0u;
                        }
                    }
                }
                int32_t m[R][4];
#pragma unroll
                for (int r = 0; r < R; ++r) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) m[r][j] = -1;
                    if (go[r]) {
                        const int32_t *mp = a.dn_mv + (uint32_t)x_tab[r][k] * ddn + c;
                        if (full) {
                            const int4 t4 = *reinterpret_cast<const int4 *>(mp);
                            m[r][0] = t4.x; m[r][1] = t4.y; m[r][2] = t4.z; m[r][3] = t4.w;
                        } else {
#pragma unroll
                            for (int j = 0; j < 4; ++j) m[r][j] = cl + j < wl ? mp[j] : -1;
                        }
                    }
                }
                TA v[R][4];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const TX *src = a.x + (uint32_t)x_src[r][go[r] ? k : 0] * ddn;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        v[r][j] = (TA)0;
                        if (m[r][j] >= 0) v[r][j] = (TA)src[(uint32_t)m[r][j] >> 1];
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const TA am = go[r] ? x_amp[r][k] : (TA)0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[r][j] += (m[r][j] & 1) ? -am * v[r][j] : am * v[r][j];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r >= nr) break;
            TX *yr = a.y + ur[r] * ddn;
            if (full) {
                V o;
                o.x = (TX)acc[r][0]; o.y = (TX)acc[r][1]; o.z = (TX)acc[r][2]; o.w = (TX)acc[r][3];
                st4<TX, true>(yr + c, o);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (cl + j < wl) yr[c + j] = (TX)acc[r][j];
            }
        }
    }
}

template <typename TX, typename TA, int R, int BS, bool UPX, bool FOLD, bool H16>
__global__ __launch_bounds__(BS) void k_gtile(ApplyArgs<TX, TA> a) {
    gtile_body<TX, TA, R, BS, UPX, FOLD, H16>(a);
}

// ---------------------------------------------------------- variant table --
// kind 0: single pass.  kind 1: two passes (row-local, then banded up spin).
struct Variant {
    int kind, R, BS;
    int64_t band;
    const char *name;
    int64_t wcap;  // kinds 6, 7, 9, 10: cap on the staged window (0 = LDS limit)
    int rw;        // kind 7: rows per workgroup of the band pass
};
static const Variant kVariants[] = {
    // row tiles, row-major LDS (generic: no packed-table requirement)
    {0, 1, 256, 0, "rw_r1_b256"},          {0, 2, 256, 0, "rw_r2_b256"},
    // row tiles over the packed 64-state ELL
    {4, 1, 256, 0, "rwpk_r1_b256"},        {4, 2, 512, 0, "rwpk_r2_b512"},
    {4, 4, 512, 0, "rwpk_r4_b512"},        {4, 2, 256, 0, "rwpk_r2_b256"},
    {4, 4, 1024, 0, "rwpk_r4_b1024"},
    // transposed row tiles, four columns per thread, single pass
    {6, 1, 256, 0, "rt_r1_b256"},           {6, 2, 256, 0, "rt_r2_b256"},
    {6, 2, 512, 0, "rt_r2_b512"},           {6, 4, 512, 0, "rt_r4_b512"},
    {6, 1, 512, 0, "rt_r1_b512"},
    // column-stationary row pass + band pass with H_up (x) 1 and the four-fermion terms
    {8, 2, 512, 256, "csx_rr2_rw32_band256", 0, 8},
    {8, 2, 512, 512, "csx_rr2_rw32_band512", 0, 8},
    {8, 4, 512, 256, "csx_rr4_rw32_band256", 0, 8},
    {8, 2, 1024, 512, "csx_rr2_b1024_rw32_band512", 0, 8},
    {8, 2, 1024, 256, "csx_rr2_b1024_rw64_band256", 0, 8},
    // grouped basis order only: tile-major work lists over (up component,
    // down window) tiles, windows = whole down components
    {10, 2, 512, 0, "grp_rt_r2_b512"},      {10, 4, 512, 0, "grp_rt_r4_b512"},
    {10, 1, 512, 0, "grp_rt_r1_b512"},
    // grouped two passes: row pass (diagonal, 1 (x) H_dn, four-fermion terms)
    // + band pass of H_up (x) 1 over (up component, band) tiles
    {11, 2, 512, 128, "grp2_rt_r2_band128", 0, 32}, {11, 2, 512, 64, "grp2_rt_r2_band64", 0, 32},
    {11, 1, 512, 128, "grp2_rt_r1_band128", 0, 32},
    // grouped order, lean tile kernel: R rows x a window of whole down
    // components of about `band` states, per-window hop table
    {12, 8, 256, 1024, "gt_r8_w1024"},      {12, 4, 256, 1024, "gt_r4_w1024"},
    {12, 8, 256, 512, "gt_r8_w512"},        {12, 8, 256, 2048, "gt_r8_w2048"},
    {12, 2, 512, 8192, "gt_r2_w8192"},      {12, 4, 512, 8192, "gt_r4_w8192"},
    // the same as the row pass of two passes, with the band pass of H_up (x) 1
    {13, 2, 512, 8192, "gt2_r2_w8192_band128", 0, 32}, {13, 8, 256, 1024, "gt2_r8_w1024_band128", 0, 32},
    // lean tile kernel, two rows or one row per item, smaller workgroups
    {12, 2, 256, 1024, "gt_r2_w1024"},      {12, 2, 128, 1024, "gt_r2_w1024_b128"},
    {12, 1, 512, 8192, "gt_r1_w8192"},
    // the whole chip on one tile at a time (shared work list, runs of 20 or
    // 128 rows per XCD): for tiles larger than an XCD's L2 (N_s = 18: up to
    // 8000 rows x 32 KB)
    {12, 1, 512, 8192, "gt_r1_w8192_shared_c20"}, {12, 1, 512, 8192, "gt_r1_w8192_shared_c128"},
};
static constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
static constexpr int64_t kDynBudget = 163840 - 8192;  // LDS left for the staged x block

// Windows of down ranks staged per workgroup: the whole row if it fits, else
// runs of states that share their top t bits (contiguous in rank order; a hop
// that does not touch those bits stays inside), merged greedily up to `cap`.
static std::vector<int2> plan_windows(const std::vector<uint32_t> &st, int ns, int64_t cap) {
    const int64_t n = (int64_t)st.size();
    std::vector<int2> w;
    if (n <= cap) {
        w.push_back(make_int2(0, (int)n));
        return w;
    }
    for (int t = 1; t <= ns; ++t) {
        const int sh = ns - t;
        std::vector<std::pair<int64_t, int64_t>> runs;
        int64_t a = 0;
        for (int64_t i = 1; i <= n; ++i)
            if (i == n || (st[i] >> sh) != (st[i - 1] >> sh)) {
                runs.push_back({a, i - a});
                a = i;
            }
        bool ok = true;
        for (auto &r : runs)
            if (r.second > cap) ok = false;
        if (!ok) continue;
        int64_t cs = runs[0].first, cl = 0;
        for (auto &r : runs) {
            if (cl + r.second > cap) {
                w.push_back(make_int2((int)cs, (int)cl));
                cs = r.first;
                cl = 0;
            }
            cl += r.second;
        }
        w.push_back(make_int2((int)cs, (int)cl));
        return w;
    }
    for (int64_t a = 0; a < n; a += cap) w.push_back(make_int2((int)a, (int)std::min(cap, n - a)));
    return w;
}

// Windows of a grouped handle: consecutive down components merged greedily up
// to `cap` states (every down hop stays inside its component); a component
// larger than `cap` is cut into equal parts.
static std::vector<int2> plan_windows_grouped(const std::vector<int32_t> &coff, int64_t cap) {
    std::vector<int2> w;
    int64_t cs = 0, cl = 0;
    for (size_t k = 0; k + 1 < coff.size(); ++k) {
        const int64_t a = coff[k], n = coff[k + 1] - coff[k];
        if (n > cap) {
            if (cl > 0) w.push_back(make_int2((int)cs, (int)cl));
            const int64_t parts = (n + cap - 1) / cap, step = (n + parts - 1) / parts;
            for (int64_t q = a; q < a + n; q += step) w.push_back(make_int2((int)q, (int)std::min(step, a + n - q)));
            cs = a + n;
            cl = 0;
            continue;
        }
        if (cl + n > cap) {
            w.push_back(make_int2((int)cs, (int)cl));
            cs = a;
            cl = 0;
        }
        cl += n;
    }
    if (cl > 0) w.push_back(make_int2((int)cs, (int)cl));
    return w;
}

static const int2 *windows_for(ed_ham_s *h, int64_t cap, int *nwin, int *wmax) {
    for (size_t i = 0; i < h->windows.size(); ++i)
        if (h->windows[i].first == cap) {
            *nwin = h->window_counts[2 * i];
            *wmax = h->window_counts[2 * i + 1];
            return h->windows[i].second->as<int2>();
        }
    std::vector<int2> w = h->grouped ? plan_windows_grouped(h->comp_off[1], cap)
                                     : plan_windows(h->dn_states_host, h->ns, cap);
    int mx = 0;
    for (auto &v : w) mx = std::max(mx, v.y);
    DevMem *m = new DevMem();
    m->alloc(w.size() * sizeof(int2));
    ED_HIP(hipMemcpy(m->p, w.data(), w.size() * sizeof(int2), hipMemcpyHostToDevice));
    h->windows.push_back({cap, m});
    h->window_counts.push_back((int)w.size());
    h->window_counts.push_back(mx);
    *nwin = (int)w.size();
    *wmax = mx;
    return m->as<int2>();
}

// Work list of a grouped schedule over column ranges `cols` (windows or
// bands): tiles (up component A, column range) in order, each cut into items
// of at most `rows` consecutive rows of A.  The list is split into 8 runs of
// about equal work (rows x columns) and run x is laid out at workgroup indices
// x, x + 8, x + 16, ..., so that the round-robin dispatch of workgroups over
// the 8 XCDs gives each XCD one run: the items of a tile then share one L2.
// Shorter runs are padded with empty items.
static const int4 *items_cached(const ed_ham_s *h, int64_t key, int64_t *count) {
    for (size_t i = 0; i < h->items.size(); ++i)
        if (h->items[i].first == key) {
            *count = h->item_counts[i];
            return h->items[i].second->as<int4>();
        }
    return nullptr;
}

static const int4 *items_for(ed_ham_s *h, int64_t key, const std::vector<int64_t> &cols, int rows,
                             int64_t *count) {
    if (const int4 *c = items_cached(h, key, count)) return c;
    const std::vector<int32_t> &co = h->comp_off[0];
    std::vector<int4> L;
    std::vector<double> cost;
    for (size_t A = 0; A + 1 < co.size(); ++A)
        for (size_t w = 0; w < cols.size(); ++w)
            for (int64_t u = co[A]; u < co[A + 1]; u += rows) {
                const int nr = (int)std::min<int64_t>(rows, co[A + 1] - u);
                L.push_back(make_int4((int)u, nr, (int)w, 0));
                cost.push_back((double)nr * (double)cols[w]);
            }
    double total = 0.0;
    for (double c : cost) total += c;
    constexpr int kX = 8;
    std::vector<std::vector<int4>> run(kX);
    double acc = 0.0;
    for (size_t i = 0; i < L.size(); ++i) {
        const int x = std::min(kX - 1, (int)(acc / total * kX));
        run[x].push_back(L[i]);
        acc += cost[i];
    }
    size_t len = 1;
    for (auto &r : run) len = std::max(len, r.size());
    std::vector<int4> out(len * kX, make_int4(0, 0, 0, 0));
    for (int x = 0; x < kX; ++x)
        for (size_t i = 0; i < run[x].size(); ++i) out[x + kX * i] = run[x][i];
    DevMem *m = new DevMem();
    m->alloc(out.size() * sizeof(int4));
    ED_HIP(hipMemcpy(m->p, out.data(), out.size() * sizeof(int4), hipMemcpyHostToDevice));
    h->items.push_back({key, m});
    h->item_counts.push_back((int64_t)out.size());
    *count = (int64_t)out.size();
    return m->as<int4>();
}

// Largest down component of a grouped handle.
static int64_t max_down_component(const ed_ham_s *h) {
    int64_t m = 0;
    const std::vector<int32_t> &co = h->comp_off[1];
    for (size_t k = 0; k + 1 < co.size(); ++k) m = std::max<int64_t>(m, co[k + 1] - co[k]);
    return m;
}

// Work list over (up component, window) tiles.  chunk = 0: XCD-partitioned
// (as items_for).  chunk > 0: shared, the tiles in order with runs of `chunk`
// consecutive items dealt to the eight XCDs in turn, so that the round-robin
// dispatch spreads each tile over the whole chip, which works on one tile at a
// time (its slice of x then stays in the Infinity Cache while its rows read
// their partner rows, when the tile is too large for one XCD's L2), while each
// run of consecutive rows (whose partners are partly each other) stays on one
// XCD.
static std::vector<int4> tile_items(const std::vector<int32_t> &co, const std::vector<int64_t> &cols, int rows,
                                    int chunk) {
    constexpr int kX = 8;
    std::vector<int4> L;
    std::vector<double> cost;
    for (size_t A = 0; A + 1 < co.size(); ++A)
        for (size_t w = 0; w < cols.size(); ++w)
            for (int64_t u = co[A]; u < co[A + 1]; u += rows) {
                const int nr = (int)std::min<int64_t>(rows, co[A + 1] - u);
                L.push_back(make_int4((int)u, nr, (int)w, 0));
                cost.push_back((double)nr * (double)cols[w]);
            }
    if (chunk > 0) {
        std::vector<std::vector<int4>> q(kX);
        for (size_t i = 0; i < L.size(); ++i) q[(i / (size_t)chunk) % kX].push_back(L[i]);
        size_t len = 1;
        for (auto &r : q) len = std::max(len, r.size());
        std::vector<int4> out(len * kX, make_int4(0, 0, 0, 0));
        for (int x = 0; x < kX; ++x)
            for (size_t i = 0; i < q[x].size(); ++i) out[x + kX * i] = q[x][i];
        return out;
    }
    double total = 0.0;
    for (double c : cost) total += c;
    std::vector<std::vector<int4>> run(kX);
    double acc = 0.0;
    for (size_t i = 0; i < L.size(); ++i) {
        const int x = std::min(kX - 1, (int)(acc / std::max(total, 1.0) * kX));
        run[x].push_back(L[i]);
        acc += cost[i];
    }
    size_t len = 1;
    for (auto &r : run) len = std::max(len, r.size());
    std::vector<int4> out(len * kX, make_int4(0, 0, 0, 0));
    for (int x = 0; x < kX; ++x)
        for (size_t i = 0; i < run[x].size(); ++i) out[x + kX * i] = run[x][i];
    return out;
}

// Plan of k_gtile with R rows per tile and windows of about `wtarget` states
// (consecutive down components merged while they fit; a larger component is a
// window of its own).  Cached on the handle.
static const TilePlan *tile_plan(ed_ham_s *h, int R, int64_t wtarget, int chunk) {
    const int64_t key = (int64_t)chunk << 48 | (int64_t)R << 32 | wtarget;
    for (auto *t : h->tplans)
        if (t->key == key) return t;
    const SpinTab &dn = h->sp[1];
    const int64_t dim = dn.dim;
    std::vector<int32_t> off((size_t)dim + 1), tgt((size_t)std::max<int64_t>(dn.nnz, 1));
    std::vector<double> sa((size_t)std::max<int64_t>(dn.nnz, 1));
    ED_HIP(hipMemcpy(off.data(), dn.off.p, off.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (dn.nnz > 0) {
        ED_HIP(hipMemcpy(tgt.data(), dn.tgt.p, (size_t)dn.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
        ED_HIP(hipMemcpy(sa.data(), dn.sa64.p, (size_t)dn.nnz * sizeof(double), hipMemcpyDeviceToHost));
    }
    // windows: whole components
    std::vector<int2> win;
    const std::vector<int32_t> &co = h->comp_off[1];
    int64_t cs = 0, cl = 0;
    for (size_t k = 0; k + 1 < co.size(); ++k) {
        const int64_t n = co[k + 1] - co[k];
        if (cl > 0 && cl + n > wtarget) {
            win.push_back(make_int2((int)cs, (int)cl));
            cs = co[k];
            cl = 0;
        }
        cl += n;
    }
    if (cl > 0) win.push_back(make_int2((int)cs, (int)cl));
    // distinct signed amplitudes (index 0 is the zero of the padding)
    std::vector<double> vals{0.0};
    std::map<double, int> idx;
    idx[0.0] = 0;
    for (int64_t e = 0; e < dn.nnz; ++e)
        if (!idx.count(sa[e])) {
            if (vals.size() >= 4095) fail(ED_EUNSUPPORTED, "down hop table has more than 4094 distinct amplitudes");
            idx.emplace(sa[e], (int)vals.size());
            vals.push_back(sa[e]);
        }
    // per-window slices of 256 states, lane l holding states 4l..4l+3; entry
    // (hop k, state q) = window-local target | amplitude index (padding: the
    // state itself with amplitude index 0)
    int wmax = 0;
    for (const int2 &w : win) wmax = std::max(wmax, w.y);
    // ED_TILE_ENTRY_BITS=32 keeps 32-bit entries for small windows too
    const char *bits = std::getenv("ED_TILE_ENTRY_BITS");
    const bool half = wmax <= 1024 && vals.size() <= 64 && !(bits && std::strcmp(bits, "32") == 0);
    auto entry = [&](const int2 &w, int64_t q, int k) -> uint32_t {
        uint32_t v = q < w.x + w.y ? (uint32_t)(q - w.x) : 0u;
        if (q < w.x + w.y && k < off[q + 1] - off[q]) {
            const int64_t e = off[q] + k, t = (int64_t)tgt[e] - w.x;
            if (t < 0 || t >= w.y) fail(ED_EDEVICE, "tile plan: a down hop leaves its component");
            v = (uint32_t)t | ((uint32_t)idx.at(sa[e]) << (half ? 10 : 20));
        }
        return v;
    };
    std::vector<int32_t> first, soff;
    std::vector<uint32_t> ent;
    for (const int2 &w : win) {
        first.push_back((int32_t)soff.size());
        for (int64_t s0 = 0; s0 < w.y; s0 += 256) {
            int kk = 0;
            for (int64_t q = w.x + s0; q < std::min<int64_t>(w.x + w.y, w.x + s0 + 256); ++q)
                kk = std::max(kk, off[q + 1] - off[q]);
            soff.push_back((int32_t)(ent.size() / 4));
            if (half) {
                for (int k = 0; k < kk; k += 2)
                    for (int l = 0; l < 64; ++l)
                        for (int hk = 0; hk < 2; ++hk)
                            for (int j = 0; j < 4; j += 2) {
                                const int64_t q = w.x + s0 + 4 * l + j;
                                ent.push_back(entry(w, q, k + hk) | entry(w, q + 1, k + hk) << 16);
                            }
            } else {
                for (int k = 0; k < kk; ++k)
                    for (int l = 0; l < 256; ++l) ent.push_back(entry(w, w.x + s0 + l, k));
            }
        }
    }
    first.push_back((int32_t)soff.size());
    soff.push_back((int32_t)(ent.size() / 4));
    if (ent.empty()) ent.assign(4, 0u);
    std::vector<int64_t> cols;
    for (const int2 &w : win) cols.push_back(w.y);
    const std::vector<int4> items = tile_items(h->comp_off[0], cols, R, chunk);
    TilePlan *t = new TilePlan();
    try {
        t->key = key;
        t->nwin = (int)win.size();
        t->wmax = wmax;
        t->namp = (int)vals.size();
        t->half = half ? 1 : 0;
        t->nitems = (int64_t)items.size();
        upload(t->win, win);
        upload(t->wsl_first, first);
        upload(t->wsl_off, soff);
        upload(t->wel4, ent);
        upload(t->amp64, vals);
        upload(t->amp32, std::vector<float>(vals.begin(), vals.end()));
        upload(t->items, items);
    } catch (...) {
        delete t;
        throw;
    }
    h->tplans.push_back(t);
    return t;
}

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
    a.dn_off = Dn.off.as<int32_t>();
    a.dn_tgt = Dn.tgt.as<int32_t>();
    a.dn_sa = Dn.sa64.as<double>();
    a.nmv_dn = Dn.nmv;
    a.dn_ell_pk = Dn.ell_pk.as<uint32_t>();
    a.dn_ell4_off = Dn.ell4_off.as<int32_t>();
    a.dn_ell4 = Dn.ell4.as<uint4>();
    a.amp_tab = Dn.amp64.as<double>();
    a.namp = Dn.namp;
    a.dn_e = Dn.ediag64.as<double>();
    a.dn_st = Dn.states.as<uint32_t>();
    a.dn_c = Dn.cidx.as<uint8_t>();
    a.dn_mv = Dn.mv.as<int32_t>();
    a.dn_mvb = Dn.mvb.as<uint32_t>();
    a.dn_mvp = Dn.mvp_ok ? Dn.mvp.as<uint32_t>() : nullptr;
    a.umode = h->umode;
    a.umask = h->umask;
    a.U0 = h->U0;
    a.usite = h->usite64.as<double>();
    a.koff = h->koff;
    a.xtab = h->xtab64.as<double>();
    a.nx = h->nx;
    a.xt = h->xt64.as<XTermDev<double>>();
    a.xl_off = h->xl_off.as<int32_t>();
    a.xl_src = h->xl_src.as<int32_t>();
    a.xl_tab = h->xl_tab.as<int32_t>();
    a.xl_amp = h->xl_amp64.as<double>();
    a.partials = partials;
    a.theta = theta;
    a.items = nullptr;
    a.fk = h->fk;
    a.ftab = h->ftab64.as<double>();
    a.up_fc = h->fcidx[0].as<uint8_t>();
    a.dn_fc = h->fcidx[1].as<uint8_t>();
    a.dn_fc32 = h->dn_fc32.as<uint32_t>();
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
    a.dn_off = Dn.off.as<int32_t>();
    a.dn_tgt = Dn.tgt.as<int32_t>();
    a.dn_sa = Dn.sa32.as<float>();
    a.nmv_dn = Dn.nmv;
    a.dn_ell_pk = Dn.ell_pk.as<uint32_t>();
    a.dn_ell4_off = Dn.ell4_off.as<int32_t>();
    a.dn_ell4 = Dn.ell4.as<uint4>();
    a.amp_tab = Dn.amp32.as<float>();
    a.namp = Dn.namp;
    a.dn_e = Dn.ediag32.as<float>();
    a.dn_st = Dn.states.as<uint32_t>();
    a.dn_c = Dn.cidx.as<uint8_t>();
    a.dn_mv = Dn.mv.as<int32_t>();
    a.dn_mvb = Dn.mvb.as<uint32_t>();
    a.dn_mvp = Dn.mvp_ok ? Dn.mvp.as<uint32_t>() : nullptr;
    a.umode = h->umode;
    a.umask = h->umask;
    a.U0 = (float)h->U0;
    a.usite = h->usite32.as<float>();
    a.koff = h->koff;
    a.xtab = h->xtab32.as<float>();
    a.nx = h->nx;
    a.xt = h->xt32.as<XTermDev<float>>();
    a.xl_off = h->xl_off.as<int32_t>();
    a.xl_src = h->xl_src.as<int32_t>();
    a.xl_tab = h->xl_tab.as<int32_t>();
    a.xl_amp = h->xl_amp32.as<float>();
    a.partials = partials;
    a.theta = theta;
    a.items = nullptr;
    a.fk = h->fk;
    a.ftab = h->ftab32.as<float>();
    a.up_fc = h->fcidx[0].as<uint8_t>();
    a.dn_fc = h->fcidx[1].as<uint8_t>();
    a.dn_fc32 = h->dn_fc32.as<uint32_t>();
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

template <class K>
static void allow_lds(K kern) {
    static std::vector<const void *> done;
    const void *f = (const void *)kern;
    for (const void *d : done)
        if (d == f) return;
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 163840 - 8192);
    (void)hipGetLastError();
    done.push_back(f);
}

template <typename TX, typename TA, int R, int BS, int MODE, bool UPX, bool PK = false>
static int64_t launch_rw(ed_ham_s *h, ApplyArgs<TX, TA> a, hipStream_t s, int64_t wcap = 0) {
    int nwin = 0, wmax = 0;
    const int64_t amp_bytes = PK ? (int64_t)h->sp[1].namp * (int64_t)sizeof(TA) + 16 : 0;
    int64_t cap = (kDynBudget - amp_bytes) / (int64_t)(R * sizeof(TX));
    if (wcap > 0 && wcap < cap) cap = wcap;
    a.win = windows_for(h, cap, &nwin, &wmax);
    a.nwin = nwin;
    a.wmax = wmax;
    const int64_t G = (a.dup + R - 1) / R;
    const size_t shm = (((size_t)R * (size_t)wmax * sizeof(TX) + 15) & ~(size_t)15) + (size_t)amp_bytes;
    auto kern = k_apply<TX, TA, R, BS, MODE, UPX, PK>;
    allow_lds(kern);
    kern<<<(unsigned)(G * nwin), BS, shm, s>>>(a);
    ED_LAUNCH_CHECK();
    return G * nwin;
}

// tiled = true: tile-major work list (grouped handles); UPX = false: row pass
// of a two-pass schedule (everything but H_up (x) 1)
template <typename TX, typename TA, int R, int BS, bool UPX = true>
static void launch_rt(ed_ham_s *h, ApplyArgs<TX, TA> a, hipStream_t s, int64_t wcap, bool tiled = false) {
    int nwin = 0, wmax = 0;
    const int64_t amp_bytes = (int64_t)h->sp[1].namp * (int64_t)sizeof(TA) + 16;
    int64_t cap = (kDynBudget - amp_bytes) / (int64_t)(R * sizeof(TX));
    if (wcap > 0 && wcap < cap) cap = wcap;
    a.win = windows_for(h, cap, &nwin, &wmax);
    a.nwin = nwin;
    a.wmax = wmax;
    int64_t nblk = ((a.dup + R - 1) / R) * nwin;
    if (tiled) {
        const int64_t key = (int64_t)1 << 40 | (int64_t)R << 32 | cap;
        a.items = items_cached(h, key, &nblk);
        if (!a.items) {
            std::vector<int2> w((size_t)nwin);
            ED_HIP(hipMemcpy(w.data(), a.win, w.size() * sizeof(int2), hipMemcpyDeviceToHost));
            std::vector<int64_t> cols;
            for (auto &v : w) cols.push_back(v.y);
            a.items = items_for(h, key, cols, R, &nblk);
        }
    }
    const size_t shm = (((size_t)R * (size_t)wmax * sizeof(TX) + 15) & ~(size_t)15) + (size_t)amp_bytes;
    if (tiled) {
        auto kern = k_rt<TX, TA, R, BS, UPX, true, true>;
        allow_lds(kern);
        kern<<<(unsigned)nblk, BS, shm, s>>>(a);
    } else {
        auto kern = k_rt<TX, TA, R, BS, UPX, true>;
        allow_lds(kern);
        kern<<<(unsigned)nblk, BS, shm, s>>>(a);
    }
    ED_LAUNCH_CHECK();
}

// band pass of the grouped two-pass schedules (work list over (component, band) tiles)
template <typename TX, typename TA>
static void launch_upt(ed_ham_s *h, ApplyArgs<TX, TA> a, int64_t band, int rows, hipStream_t s) {
    const int64_t key = (int64_t)2 << 40 | (int64_t)rows << 32 | band;
    int64_t n = 0;
    a.items = items_cached(h, key, &n);
    if (!a.items) {
        const int64_t nb = (a.ddn + band - 1) / band;
        std::vector<int64_t> cols((size_t)nb);
        for (int64_t b = 0; b < nb; ++b) cols[b] = std::min(band, a.ddn - b * band);
        a.items = items_for(h, key, cols, rows, &n);
    }
    if (band == 128) k_upt<TX, TA, 256, 128><<<(unsigned)n, 256, 0, s>>>(a);
    else if (band == 64) k_upt<TX, TA, 256, 64><<<(unsigned)n, 256, 0, s>>>(a);
    else fail(ED_EINVAL, "band pass: unsupported band %lld", (long long)band);
    ED_LAUNCH_CHECK();
}

template <typename TX, typename TA, bool XT = false>
static void launch_upb(const ApplyArgs<TX, TA> &a, int64_t band, int rw, hipStream_t s) {
    constexpr int RB = 2;
    const int bs = (int)(band / 4);
    const int64_t G = (a.dup + rw - 1) / rw;
    const int64_t nb = (a.ddn + band - 1) / band;
    if (bs == 64) k_upb<TX, TA, RB, 64, XT><<<(unsigned)(G * nb), 64, 0, s>>>(a, band, rw);
    else if (bs == 128) k_upb<TX, TA, RB, 128, XT><<<(unsigned)(G * nb), 128, 0, s>>>(a, band, rw);
    else if (bs == 256) k_upb<TX, TA, RB, 256, XT><<<(unsigned)(G * nb), 256, 0, s>>>(a, band, rw);
    else fail(ED_EINVAL, "band pass: unsupported band %lld", (long long)band);
    ED_LAUNCH_CHECK();
}

template <typename TX, typename TA, int R, int BS, bool UPX = true>
static void launch_gtile(ed_ham_s *h, ApplyArgs<TX, TA> a, int64_t wtarget, hipStream_t s, int chunk = 0) {
    if (h->fk < 0 && !(h->koff == 0 && h->umode <= 1))
        fail(ED_EINVAL, "tile schedule: the cross term is neither a small table nor a uniform on-site U");
    const TilePlan *t = tile_plan(h, R, wtarget, chunk);
    a.win = t->win.as<int2>();
    a.nwin = t->nwin;
    a.wmax = t->wmax;
    a.items = t->items.as<int4>();
    a.wsl_first = t->wsl_first.as<int32_t>();
    a.wsl_off = t->wsl_off.as<int32_t>();
    a.wel4 = t->wel4.as<uint4>();
    a.namp = t->namp;
    a.amp_tab = sizeof(TA) == 8 ? (const TA *)t->amp64.p : (const TA *)t->amp32.p;
    const size_t shm = (((size_t)R * (size_t)t->wmax * sizeof(TX) + 15) & ~(size_t)15) + (size_t)t->namp * sizeof(TA);
    auto kern = h->fk >= 0 ? (t->half ? k_gtile<TX, TA, R, BS, UPX, true, true> : k_gtile<TX, TA, R, BS, UPX, true, false>)
                           : (t->half ? k_gtile<TX, TA, R, BS, UPX, false, true> : k_gtile<TX, TA, R, BS, UPX, false, false>);
    allow_lds(kern);
    kern<<<(unsigned)t->nitems, BS, shm, s>>>(a);
    ED_LAUNCH_CHECK();
}

// register-tile sizes of the column-stationary kernels
static int cs_kmax(const ed_ham_s *h) {
    const int m = std::max(h->sp[0].max_hops, h->sp[1].max_hops);
    return m <= 8 ? 8 : (m <= 16 ? 16 : (m <= 32 ? 32 : 0));
}
static int cs_nmv(const ed_ham_s *h) {
    const int n = h->sp[1].nmv;
    return (h->nx == 0) ? 0 : (n <= 8 ? 8 : -1);
}
static int cs_xmax(const ed_ham_s *h) {
    return h->xl_max <= 4 ? 4 : (h->xl_max <= 8 ? 8 : 0);
}

template <typename TX, typename TA, int RR, int KMAX, int NMV, int XMAX, int MODE, bool UPX, int BS>
static int64_t launch_cs_k(ed_ham_s *h, ApplyArgs<TX, TA> a, int rw, hipStream_t s) {
    int nwin = 0, wmax = 0;
    a.win = windows_for(h, (int64_t)BS, &nwin, &wmax);
    a.nwin = nwin;
    a.wmax = wmax;
    const int64_t G = (a.dup + rw - 1) / rw;
    const size_t shm = 2 * (size_t)RR * (size_t)wmax * sizeof(TX);
    k_cs<TX, TA, BS, RR, KMAX, NMV, XMAX, MODE, UPX><<<(unsigned)(G * nwin), BS, shm, s>>>(a, rw);
    ED_LAUNCH_CHECK();
    return G * nwin;
}

template <typename TX, typename TA, int RR, int MODE, bool UPX, int KMAX, int BS>
static int64_t launch_cs_km(ed_ham_s *h, const ApplyArgs<TX, TA> &a, int rw, hipStream_t s) {
    const int nm = cs_nmv(h), xm = cs_xmax(h);
    if (nm == 0) return launch_cs_k<TX, TA, RR, KMAX, 0, 0, MODE, UPX, BS>(h, a, rw, s);
    if (nm == 8 && xm == 4) return launch_cs_k<TX, TA, RR, KMAX, 8, 4, MODE, UPX, BS>(h, a, rw, s);
    if (nm == 8 && xm == 8) return launch_cs_k<TX, TA, RR, KMAX, 8, 8, MODE, UPX, BS>(h, a, rw, s);
    fail(ED_EINVAL, "column-stationary schedule does not fit this Hamiltonian");
}

// BS threads own a window of BS down ranks
template <typename TX, typename TA, int RR, int MODE, bool UPX, int BS = 512>
static int64_t launch_cs(ed_ham_s *h, const ApplyArgs<TX, TA> &a, int rw, hipStream_t s) {
    const int km = cs_kmax(h);
    if (km == 8) return launch_cs_km<TX, TA, RR, MODE, UPX, 8, BS>(h, a, rw, s);
    if (km == 16) return launch_cs_km<TX, TA, RR, MODE, UPX, 16, BS>(h, a, rw, s);
    if constexpr (BS <= 512) {
        if (km == 32) return launch_cs_km<TX, TA, RR, MODE, UPX, 32, BS>(h, a, rw, s);
    }
    fail(ED_EINVAL, "column-stationary schedule does not fit this Hamiltonian");
}

template <typename TX, typename TA>
static void launch_variant(ed_ham_s *h, const ApplyArgs<TX, TA> &a, int v, hipStream_t s) {
    const Variant &V = kVariants[v];
    switch (v) {
        case 0: launch_rw<TX, TA, 1, 256, 0, true>(h, a, s); break;
        case 1: launch_rw<TX, TA, 2, 256, 0, true>(h, a, s); break;
        case 2: launch_rw<TX, TA, 1, 256, 0, true, true>(h, a, s); break;
        case 3: launch_rw<TX, TA, 2, 512, 0, true, true>(h, a, s); break;
        case 4: launch_rw<TX, TA, 4, 512, 0, true, true>(h, a, s); break;
        case 5: launch_rw<TX, TA, 2, 256, 0, true, true>(h, a, s); break;
        case 6: launch_rw<TX, TA, 4, 1024, 0, true, true>(h, a, s); break;
        case 7: launch_rt<TX, TA, 1, 256>(h, a, s, V.wcap); break;
        case 8: launch_rt<TX, TA, 2, 256>(h, a, s, V.wcap); break;
        case 9: launch_rt<TX, TA, 2, 512>(h, a, s, V.wcap); break;
        case 10: launch_rt<TX, TA, 4, 512>(h, a, s, V.wcap); break;
        case 11: launch_rt<TX, TA, 1, 512>(h, a, s, V.wcap); break;
        case 12:
        case 13: launch_cs<TX, TA, 2, 0, false>(h, a, 32, s); launch_upb<TX, TA, true>(a, V.band, V.rw, s); break;
        case 14: launch_cs<TX, TA, 4, 0, false>(h, a, 32, s); launch_upb<TX, TA, true>(a, V.band, V.rw, s); break;
        case 15:
            launch_cs<TX, TA, 2, 0, false, 1024>(h, a, 32, s);
            launch_upb<TX, TA, true>(a, V.band, V.rw, s);
            break;
        case 16:
            launch_cs<TX, TA, 2, 0, false, 1024>(h, a, 64, s);
            launch_upb<TX, TA, true>(a, V.band, V.rw, s);
            break;
        case 17: launch_rt<TX, TA, 2, 512>(h, a, s, 0, true); break;
        case 18: launch_rt<TX, TA, 4, 512>(h, a, s, 0, true); break;
        case 19: launch_rt<TX, TA, 1, 512>(h, a, s, 0, true); break;
        case 20:
        case 21:
            launch_rt<TX, TA, 2, 512, false>(h, a, s, 0, true);
            launch_upt<TX, TA>(h, a, V.band, V.rw, s);
            break;
        case 22:
            launch_rt<TX, TA, 1, 512, false>(h, a, s, 0, true);
            launch_upt<TX, TA>(h, a, V.band, V.rw, s);
            break;
        case 23: launch_gtile<TX, TA, 8, 256>(h, a, 1024, s); break;
        case 24: launch_gtile<TX, TA, 4, 256>(h, a, 1024, s); break;
        case 25: launch_gtile<TX, TA, 8, 256>(h, a, 512, s); break;
        case 26: launch_gtile<TX, TA, 8, 256>(h, a, 2048, s); break;
        case 27: launch_gtile<TX, TA, 2, 512>(h, a, 8192, s); break;
        case 28: launch_gtile<TX, TA, 4, 512>(h, a, 8192, s); break;
        case 29:
            launch_gtile<TX, TA, 2, 512, false>(h, a, 8192, s);
            launch_upt<TX, TA>(h, a, 128, V.rw, s);
            break;
        case 30:
            launch_gtile<TX, TA, 8, 256, false>(h, a, 1024, s);
            launch_upt<TX, TA>(h, a, 128, V.rw, s);
            break;
        case 31: launch_gtile<TX, TA, 2, 256>(h, a, 1024, s); break;
        case 32: launch_gtile<TX, TA, 2, 128>(h, a, 1024, s); break;
        case 33: launch_gtile<TX, TA, 1, 512>(h, a, 8192, s); break;
        case 34: launch_gtile<TX, TA, 1, 512>(h, a, 8192, s, 20); break;
        case 35: launch_gtile<TX, TA, 1, 512>(h, a, 8192, s, 128); break;
        default: fail(ED_EINVAL, "bad apply variant %d", v);
    }
}

static bool variant_fits(const ed_ham_s *h, int v, size_t elem) {
    (void)elem;
    if (v < 0 || v >= kNumVariants) return false;
    const Variant &V = kVariants[v];
    if (V.kind == 4 && (!h->sp[1].pk_ok || h->sp[0].max_hops > 32 || h->xl_max > 16 || h->sp[1].nmv > 8))
        return false;
    if (V.kind == 6 && (!h->sp[1].pk_ok || h->sp[0].max_hops > 32 || h->xl_max > 16 || h->koff > 4)) return false;
    if (V.kind == 8 && (h->sp[0].nnz == 0 || cs_kmax(h) == 0 || cs_nmv(h) < 0 || (h->nx > 0 && cs_xmax(h) == 0)))
        return false;
    if (V.kind == 8 && V.BS > 512 && cs_kmax(h) > 16) return false;
    if (V.kind == 12 || V.kind == 13) {
        // grouped tile kernel: every down component whole in a window that fits LDS
        if (!h->grouped || h->sp[0].max_hops > 32 || h->xl_max > 16 || h->D >= ((int64_t)1 << 32) ||
            h->ddn >= (1 << 20))
            return false;
        if (h->fk < 0 && !(h->koff == 0 && h->umode <= 1)) return false;
        const int64_t wmax = std::max<int64_t>(max_down_component(h), std::min<int64_t>(V.band, h->ddn));
        if ((int64_t)V.R * wmax * (int64_t)elem + 4096 * (int64_t)elem + 16 > kDynBudget) return false;
        if (max_down_component(h) > 2 * V.band) return false;
    }
    if (V.kind == 10 || V.kind == 11) {
        if (!h->grouped || !h->sp[1].pk_ok || h->sp[0].max_hops > 32 || h->xl_max > 16 || h->koff > 4 ||
            h->D >= ((int64_t)1 << 32))
            return false;
        // the tile kernel needs every down component whole in its window
        const int64_t amp_bytes = (int64_t)h->sp[1].namp * (int64_t)(h->prec == ED_FP64 ? 8 : 4) + 16;
        const int64_t cap = (kDynBudget - amp_bytes) / (int64_t)(V.R * elem);
        const std::vector<int32_t> &co = h->comp_off[1];
        for (size_t k = 0; k + 1 < co.size(); ++k)
            if (co[k + 1] - co[k] > cap) return false;
    }
    return true;
}

int apply_variant_count(const ed_ham_s *) { return kNumVariants; }

const char *apply_variant_name(const ed_ham_s *, int v) {
    return (v >= 0 && v < kNumVariants) ? kVariants[v].name : "?";
}

static void launch_store(ed_ham_s *h, int v, const void *x, void *y, hipStream_t s) {
    if (h->prec == ED_FP64)
        launch_variant<double, double>(h, make_args<double, double>(h, x, y, nullptr, 0.0), v, s);
    else
        launch_variant<float, float>(h, make_args<float, float>(h, x, y, nullptr, 0.0), v, s);
}

void apply_launch_variant(ed_ham_s *h, int v, const void *x, void *y, hipStream_t s) {
    if (v < 0 || v >= kNumVariants) fail(ED_EINVAL, "apply variant %d out of range", v);
    const size_t elem = h->prec == ED_FP64 ? 8 : 4;
    if (!variant_fits(h, v, elem)) fail(ED_EINVAL, "apply variant %s does not apply to this Hamiltonian", kVariants[v].name);
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

// Windows of the FP64-arithmetic apply of the Rayleigh quotient (the row
// tiles of k_apply with one row and no packed table).
static int64_t rayleigh_cap(const ed_ham_s *h) { return kDynBudget / (int64_t)(h->prec == ED_FP64 ? 8 : 4); }

// Number of (a, b) partial pairs the Rayleigh quotient writes, from the cached
// window plan only (-1 when it is not there yet).
int64_t rayleigh_pairs_cached(const ed_ham_s *h) {
    const int64_t cap = rayleigh_cap(h);
    for (size_t i = 0; i < h->windows.size(); ++i)
        if (h->windows[i].first == cap) return h->dup * (int64_t)h->window_counts[2 * i];
    return -1;
}

// At handle creation: the window plan of the Rayleigh quotient and the LDS
// attribute of its kernels, so that later calls allocate nothing for them.
void prepare_rayleigh(ed_ham_s *h) {
    int nwin = 0, wmax = 0;
    (void)windows_for(h, rayleigh_cap(h), &nwin, &wmax);
    if (h->prec == ED_FP64) {
        allow_lds(k_apply<double, double, 1, 512, 1, true, false>);
        allow_lds(k_apply<double, double, 1, 512, 2, true, false>);
    } else {
        allow_lds(k_apply<float, double, 1, 512, 1, true, false>);
        allow_lds(k_apply<float, double, 1, 512, 2, true, false>);
    }
}

// rq = <x,Hx>/<x,x>, resid = ||Hx - rq x|| / ||x|| with H x in FP64 arithmetic;
// part: 2 nb + 2 doubles of device memory for the per-workgroup partials and
// the two sums (nb = rayleigh_pairs_cached).
template <typename TX>
static void rayleigh_with(ed_ham_s *h, const void *x, double *part, int64_t nb, double *rq, double *resid,
                          hipStream_t s) {
    double *out = part + 2 * nb;
    double hv[2];
    ApplyArgs<TX, double> a = make_args<TX, double>(h, x, nullptr, part, 0.0);
    launch_rw<TX, double, 1, 512, 1, true>(h, a, s);
    k_sum_pairs<<<1, 256, 0, s>>>(part, nb, out);
    ED_LAUNCH_CHECK();
    ED_HIP(hipMemcpyAsync(hv, out, sizeof(hv), hipMemcpyDeviceToHost, s));
    ED_HIP(hipStreamSynchronize(s));
    if (!(hv[1] > 0.0)) fail(ED_EINVAL, "ed_rayleigh: zero vector");
    const double theta = hv[0] / hv[1];
    a.theta = theta;
    launch_rw<TX, double, 1, 512, 2, true>(h, a, s);
    k_sum_pairs<<<1, 256, 0, s>>>(part, nb, out);
    ED_LAUNCH_CHECK();
    double r2[2];
    ED_HIP(hipMemcpyAsync(r2, out, sizeof(r2), hipMemcpyDeviceToHost, s));
    ED_HIP(hipStreamSynchronize(s));
    *rq = theta;
    *resid = std::sqrt(r2[0] / hv[1]);
}

void rayleigh_on(ed_ham_s *h, const void *x, double *part, int64_t nb, double *rq, double *resid, hipStream_t s) {
    if (h->prec == ED_FP64)
        rayleigh_with<double>(h, x, part, nb, rq, resid, s);
    else
        rayleigh_with<float>(h, x, part, nb, rq, resid, s);
}

// The handle's own reduction buffer (grown on demand).
void rayleigh_fp64(ed_ham_s *h, const void *x, double *rq, double *resid, hipStream_t s) {
    int64_t nb = rayleigh_pairs_cached(h);
    if (nb < 0) {
        prepare_rayleigh(h);
        nb = rayleigh_pairs_cached(h);
    }
    ensure_redbuf(h, (size_t)2 * nb + 8);
    rayleigh_on(h, x, h->redbuf.as<double>(), nb, rq, resid, s);
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
