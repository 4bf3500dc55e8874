// Sector-batched Lanczos: every (N_up, N_dn) sector of one impurity problem is
// advanced together (the paper's solver visits the sectors of the block
// structure behind Table 1 one by one).  One Lanczos step of all running
// sectors is a fixed sequence of batched kernels -- apply, the Gram-Schmidt
// projections of the chosen reorthogonalisation with FP64 reductions, norm,
// per-sector tridiagonal eigensolve and convergence test -- captured once in a
// hipGraph and replayed.  Each sector keeps its own step index, state and
// basis in device memory, so sectors converge, fill their basis and restart
// independently: a converged sector drops out through its device flag, a
// sector whose basis is full waits (masked) until the host restarts it --
// implicitly (exact shifts, keeping `keep` vectors) or from its Ritz vector --
// with one batched combination kernel over all waiting sectors.
//
// Work decomposition (the paper's observation that equal splits of the matrix
// give unequal work, end of Section 3.2, is the reason the tiles are sized per
// sector): the apply runs over tiles of consecutive rows of one sector with
// about `tile` output elements each (picked by timing a few candidates on the
// actual sectors); the vector kernels run over element chunks of at most 8192
// of one sector, so a small sector is one workgroup and a large one many,
// each with four consecutive elements per thread; the per-sector reductions
// sum the chunk partials in a fixed order (one wave per sum).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <thread>
#include <vector>

#include "ed_internal.h"

namespace ed {

template <typename TX, typename TA>
struct BSec {
    int64_t D, dup, ddn;
    TX *base;  // slots: slot k = base + k * D
    const int32_t *up_off, *up_tgt, *dn_off, *dn_tgt;
    const TA *up_sa, *dn_sa, *up_e, *dn_e;
    const uint32_t *up_st, *dn_st;
    const uint8_t *up_c, *dn_c;
    const int32_t *up_mv, *dn_mv;
    int umode;
    uint32_t umask;
    TA U0;
    const TA *usite;
    int koff;
    const TA *xtab;
    int nx;
    const XTermDev<TA> *xt;
    // per up state: the four-fermion terms whose up move is allowed (source up
    // rank, down move table, amplitude with the up sign), CSR over up ranks
    const int32_t *xl_off, *xl_src, *xl_tab;
    const TA *xl_amp;
    int nch;       // reduction chunks of this sector
    int64_t pbase; // offset of this sector's partials
};

struct ATile {
    int32_t sec, u0, nr, lds;
};

struct RChunk {
    int32_t sec, c;
    int64_t a, b;
};

// Per-sector state.  Strides: ms = m + 2 (sig2, gamma, alpha, beta), mt = m + 8
// (tri: theta, residual, beta_last, eigenvector), rs = 2 m + 4 (raw sums), mg =
// (m + 1)^2 (Gram matrix), mc = (m + 1) * max(1, keep + 1) (restart coefficients).
struct BState {
    double *sig2, *gamma, *alpha, *beta, *tri, *raw, *gram, *coef, *a2b2;
    double *theta, *resid;
    int *active;  // 0 done, 1 running, 2 basis full (waiting for a restart)
    int *jcur;    // step index of the running cycle
    int *nsteps;  // size of the tridiagonal matrix behind theta / tri
    int *iters;   // steps taken, all cycles
    int *rnin, *rnout, *rmode;  // restart request: inputs, outputs, 1 explicit 2 implicit 3 final
    double *nvsum;              // stored vectors projected against, summed over all steps
};

struct BDims {
    int m, ms, mt, rs, mc, reorth, check;
    int64_t mg;
};

static constexpr int kBBS = 256;
static constexpr int kBatchBasisDefault = 60;  // basis per sector when max_basis = 0
static constexpr int kBChunk = 8192;           // elements per vector-kernel workgroup
static constexpr int kBRMaxC = 4400;           // restart coefficients held in LDS (nin * NO)

// Window of stored vectors the step projects against: all of S_0..S_j, or
// S_{j-1}, S_j for the plain three-term recurrence (reorth = 0).
__device__ __forceinline__ int win_begin(int reorth, int j) { return (reorth == 0 && j >= 2) ? j - 1 : 0; }

// ------------------------------------------------------------------ apply --
static constexpr int kBRows = 64;  // rows per apply tile at most

// Four consecutive rows r0..r0+3 (those < nr) of a row tile at column d:
// (diagonal + 1 (x) H_dn + H_up (x) 1 + four-fermion terms) x.  The column's
// data (state, diagonal piece, down hops, down moves) is read once for the
// four rows; the rows' data comes from LDS.  XT: the tile's rows are staged in
// LDS (else read from memory); XW: the tile is the whole sector, so every
// operand is in LDS.
template <typename TX, typename TA, bool XT, bool XW>
__device__ __forceinline__ void kb_four_rows(const BSec<TX, TA> &S, const TX *xs, const TX *x, const TX *xt0,
                                             uint32_t nr, uint32_t r0, uint32_t d, uint32_t ddn, uint32_t u0,
                                             const TA *s_eu, const uint32_t *s_su, const uint32_t *s_cu,
                                             const int32_t *s_ub, const int32_t *s_ue, const int32_t *s_xb,
                                             const int32_t *s_xe, TA acc[4]) {
    const TX *xt = XT ? xs : xt0;    // the tile's rows
    const TX *xa = XW ? xs : x;      // the sector's rows
    const uint32_t sd = S.dn_st[d];
    const TA edn = S.dn_e[d];
    const uint32_t cd = S.koff ? (uint32_t)S.dn_c[d] : 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t r = r0 + i < nr ? r0 + i : r0;
        TA c = (TA)0;
        if (S.umode == 1) c = S.U0 * (TA)__popc(s_su[r] & sd);
        else if (S.umode == 2) {
            uint32_t mm = s_su[r] & sd;
            while (mm) {
                c += S.usite[__ffs(mm) - 1];
                mm &= mm - 1u;
            }
        }
        if (S.koff) c += S.xtab[(s_cu[r] << S.koff) | cd];
        acc[i] = (s_eu[r] + edn + c) * (TA)xt[r * ddn + d];
    }
    const int32_t db = S.dn_off[d], de = S.dn_off[d + 1];
    for (int32_t e = db; e < de; ++e) {
        const uint32_t t = (uint32_t)S.dn_tgt[e];
        const TA am = S.dn_sa[e];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t r = r0 + i < nr ? r0 + i : r0;
            acc[i] += am * (TA)xt[r * ddn + t];
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (r0 + i >= nr) break;
        const int32_t ub = s_ub[r0 + i], ue = s_ue[r0 + i];
        for (int32_t e = ub; e < ue; ++e) acc[i] += S.up_sa[e] * (TA)xa[(uint32_t)S.up_tgt[e] * ddn + d];
    }
    // four-fermion terms allowed on each row (per-row lists: no test of the up move)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (r0 + i >= nr) break;
        const int32_t xb = s_xb[r0 + i], xe = s_xe[r0 + i];
        for (int32_t e = xb; e < xe; ++e) {
            const int32_t md = S.dn_mv[(int64_t)S.xl_tab[e] * ddn + d];
            if (md < 0) continue;
            const TA v = S.xl_amp[e] * (TA)xa[(uint32_t)S.xl_src[e] * ddn + (uint32_t)(md >> 1)];
            acc[i] += (md & 1) ? -v : v;
        }
    }
}

// MODE 0: slot (j+1) = H slot j with j the sector's own step index (running
// sectors only).  MODE 1: partials of <x,Hx>, <x,x> with x = slot `xslot`
// (FP64 arithmetic when TA = double).  A tile is nr <= kBRows consecutive rows
// of one sector (nr * ddn < 2^31, 32-bit index arithmetic); a work item is a
// column of four of its rows.  The tile's x rows are staged in LDS when they
// fit, and a tile that holds a whole sector reads every operand from LDS.
template <typename TX, typename TA, int MODE>
__global__ __launch_bounds__(kBBS) void kb_apply(const BSec<TX, TA> *secs, const ATile *tiles, const int *jcur,
                                                 const int *active, int xslot, double *tpart) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[2][kBBS / 64];
    __shared__ TA s_eu[kBRows];
    __shared__ uint32_t s_su[kBRows], s_cu[kBRows];
    __shared__ int32_t s_ub[kBRows], s_ue[kBRows], s_xb[kBRows], s_xe[kBRows];
    TX *xs = reinterpret_cast<TX *>(smem_raw);
    const ATile tl = tiles[blockIdx.x];
    const BSec<TX, TA> &S = secs[tl.sec];
    double p0 = 0.0, p1 = 0.0;
    const bool on = MODE == 1 || active[tl.sec] == 1;
    if (on) {
        const int j = MODE == 0 ? jcur[tl.sec] : xslot;
        const TX *x = S.base + (int64_t)j * S.D;
        TX *y = S.base + (int64_t)(j + 1) * S.D;
        const uint32_t ddn = (uint32_t)S.ddn, nr = (uint32_t)tl.nr, u0 = (uint32_t)tl.u0;
        const uint32_t ne = nr * ddn;
        const TX *xt0 = x + (int64_t)u0 * ddn;
        TX *yt0 = y + (int64_t)u0 * ddn;
        if (tl.lds) {
            for (uint32_t k = threadIdx.x; k < ne; k += kBBS) xs[k] = xt0[k];
        }
        for (uint32_t r = threadIdx.x; r < nr; r += kBBS) {
            const uint32_t u = u0 + r;
            s_eu[r] = S.up_e[u];
            s_su[r] = S.up_st[u] & S.umask;
            s_cu[r] = S.koff ? (uint32_t)S.up_c[u] : 0u;
            s_ub[r] = S.up_off[u];
            s_ue[r] = S.up_off[u + 1];
            s_xb[r] = S.nx ? S.xl_off[u] : 0;
            s_xe[r] = S.nx ? S.xl_off[u + 1] : 0;
        }
        __syncthreads();
        const bool whole = tl.lds && u0 == 0 && nr == (uint32_t)S.dup;
        const uint32_t nrg = (nr + 3) / 4;
        for (uint32_t k = threadIdx.x; k < nrg * ddn; k += kBBS) {
            const uint32_t g = k / ddn, d = k - g * ddn, r0 = 4 * g;
            TA acc[4];
            if (whole)
                kb_four_rows<TX, TA, true, true>(S, xs, x, xt0, nr, r0, d, ddn, u0, s_eu, s_su, s_cu, s_ub, s_ue, s_xb, s_xe, acc);
            else if (tl.lds)
                kb_four_rows<TX, TA, true, false>(S, xs, x, xt0, nr, r0, d, ddn, u0, s_eu, s_su, s_cu, s_ub, s_ue, s_xb, s_xe, acc);
            else
                kb_four_rows<TX, TA, false, false>(S, xs, x, xt0, nr, r0, d, ddn, u0, s_eu, s_su, s_cu, s_ub, s_ue,
                                                   s_xb, s_xe, acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (r0 + i >= nr) break;
                const uint32_t o = (r0 + i) * ddn + d;
                if constexpr (MODE == 0) {
                    yt0[o] = (TX)acc[i];
                } else {
                    const double xv = (double)xt0[o];
                    p0 += xv * (double)acc[i];
                    p1 += xv * xv;
                }
            }
        }
    }
    if constexpr (MODE == 1) {
        const double s0 = block_sum<kBBS>(p0, red[0]);
        const double s1 = block_sum<kBBS>(p1, red[1]);
        if (threadIdx.x == 0) {
            tpart[2 * (int64_t)blockIdx.x] = s0;
            tpart[2 * (int64_t)blockIdx.x + 1] = s1;
        }
    }
}

// ------------------------------------------------------------- reductions --
// partials[pbase + r * nch + c] = <S_{vb+r}, Y> over chunk c (Y = slot j + 1);
// with TWO also partials[pbase + (nv + r) * nch + c] = <S_{vb+r}, S_j>.
template <typename TX, int G, bool TWO>
__global__ __launch_bounds__(kBBS) void kb_dots_v4(const BSec<TX, TX> *secs, const RChunk *ch, BState st,
                                                   int reorth, double *part) {
    __shared__ double red[kBBS / 64];
    const RChunk c = ch[blockIdx.x];
    if (st.active[c.sec] != 1) return;
    const BSec<TX, TX> &S = secs[c.sec];
    const int j = st.jcur[c.sec];
    const int vb = win_begin(reorth, j), nv = j + 1 - vb;
    const TX *y = S.base + (int64_t)(j + 1) * S.D;
    const TX *z = S.base + (int64_t)j * S.D;
    for (int g0 = 0; g0 < nv; g0 += G) {
        double ay[G], az[G];
#pragma unroll
        for (int i = 0; i < G; ++i) ay[i] = az[i] = 0.0;
        const TX *vp[G];
#pragma unroll
        for (int i = 0; i < G; ++i) vp[i] = S.base + (int64_t)(vb + ((g0 + i < nv) ? g0 + i : g0)) * S.D;
        int64_t k = c.a + 4 * (int64_t)threadIdx.x;
        for (; k + 4 <= c.b; k += 4 * kBBS) {
            const Q4<TX> yv = load4(y + k);
            Q4<TX> zv;
            if constexpr (TWO) zv = load4(z + k);
            Q4<TX> sv[G];
#pragma unroll
            for (int i = 0; i < G; ++i)
                if (g0 + i < nv) sv[i] = load4(vp[i] + k);
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (g0 + i >= nv) break;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ay[i] += (double)sv[i].v[e] * (double)yv.v[e];
                    if constexpr (TWO) az[i] += (double)sv[i].v[e] * (double)zv.v[e];
                }
            }
        }
        for (int64_t e = k; e < c.b && e < k + 4; ++e) {  // ragged end of the chunk
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (g0 + i >= nv) break;
                ay[i] += (double)vp[i][e] * (double)y[e];
                if constexpr (TWO) az[i] += (double)vp[i][e] * (double)z[e];
            }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            if (g0 + i >= nv) break;
            const double sy = block_sum_any<kBBS>(ay[i], red);
            if (threadIdx.x == 0) part[S.pbase + (int64_t)(g0 + i) * S.nch + c.c] = sy;
            if constexpr (TWO) {
                const double sz = block_sum_any<kBBS>(az[i], red);
                if (threadIdx.x == 0) part[S.pbase + (int64_t)(nv + g0 + i) * S.nch + c.c] = sz;
            }
        }
    }
}

// Row sums of the chunk partials, one wave per (row, sector) in a fixed order:
// raw[s * rs + r] = sum_c part[pbase + r * nch + c].  Rows: what: 0 = the
// projection rows of the running sectors (nv, or 2 nv with the Gram read),
// 1 = row 0 of the running sectors (norm), 2 = row 0 of the sectors with a
// restart request.
template <typename TX>
__global__ __launch_bounds__(64) void kb_rowsum(const BSec<TX, TX> *secs, BState st, BDims dm, int what,
                                                const double *part) {
    const int r = blockIdx.x, s = blockIdx.y;
    int rows;
    if (what == 2) {
        if (st.rnout[s] <= 0) return;
        rows = 1;
    } else {
        if (st.active[s] != 1) return;
        if (what == 1) rows = 1;
        else {
            const int j = st.jcur[s];
            const int nv = j + 1 - win_begin(dm.reorth, j);
            rows = dm.reorth == 3 ? 2 * nv : nv;
        }
    }
    if (r >= rows) return;
    const BSec<TX, TX> &S = secs[s];
    const double *p = part + S.pbase + (int64_t)r * S.nch;
    double v = 0.0;
    for (int c = threadIdx.x; c < S.nch; c += 64) v += p[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (threadIdx.x == 0) st.raw[(int64_t)s * dm.rs + r] = v;
}

// Projection coefficients of the running sectors, gamma[vb + r] from the row
// sums; alpha_j += gamma_j.  reorth = 3: both CGS2 projections from the one
// read, the second through the Gram matrix of the stored vectors (whose row j
// is the second half of the sums).
__global__ __launch_bounds__(256) void kb_coef(BState st, BDims dm) {
    const int s = blockIdx.x;
    if (st.active[s] != 1) return;
    const int j = st.jcur[s];
    const int vb = win_begin(dm.reorth, j), nv = j + 1 - vb;
    const double *raw = st.raw + (int64_t)s * dm.rs;
    const double *sig2 = st.sig2 + (int64_t)s * dm.ms;
    double *gamma = st.gamma + (int64_t)s * dm.ms;
    if (dm.reorth == 3) {
        __shared__ double g1[1024];
        double *G = st.gram + (int64_t)s * dm.mg;
        const int ld = dm.m + 1;
        for (int i = threadIdx.x; i < nv; i += 256) {
            g1[i] = sig2[i] * raw[i];
            G[(int64_t)j * ld + i] = raw[nv + i];
            G[(int64_t)i * ld + j] = raw[nv + i];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nv; i += 256) {
            double t = 0.0;
            for (int k = 0; k < nv; ++k) t += G[(int64_t)i * ld + k] * g1[k];
            gamma[i] = g1[i] + sig2[i] * (raw[i] - t);
        }
        __syncthreads();
    } else {
        for (int r = threadIdx.x; r < nv; r += 256) gamma[vb + r] = sig2[vb + r] * raw[r];
        __syncthreads();
    }
    if (threadIdx.x == 0) st.alpha[(int64_t)s * dm.ms + j] += gamma[j];
}

// Y = post * (Y - sum_r gamma[vb + r] S_{vb+r}) over the chunk; the last pass
// scales by sigma_j (the stored vector is w'', of norm beta_j) and writes the
// chunk's norm partial at part[pbase + c].
template <typename TX>
__global__ __launch_bounds__(kBBS) void kb_update_v4(const BSec<TX, TX> *secs, const RChunk *ch, BState st,
                                                     BDims dm, double *part, int last) {
    __shared__ double g[1024];
    __shared__ const TX *p[1024];
    __shared__ double red[kBBS / 64];
    const RChunk c = ch[blockIdx.x];
    if (st.active[c.sec] != 1) return;
    const BSec<TX, TX> &S = secs[c.sec];
    const int j = st.jcur[c.sec];
    const int vb = win_begin(dm.reorth, j), nv = j + 1 - vb;
    for (int i = threadIdx.x; i < nv; i += kBBS) {
        g[i] = st.gamma[(int64_t)c.sec * dm.ms + vb + i];
        p[i] = S.base + (int64_t)(vb + i) * S.D;
    }
    __syncthreads();
    TX *y = S.base + (int64_t)(j + 1) * S.D;
    const double post = last ? sqrt(st.sig2[(int64_t)c.sec * dm.ms + j]) : 1.0;
    double nrm = 0.0;
    int64_t k = c.a + 4 * (int64_t)threadIdx.x;
    for (; k + 4 <= c.b; k += 4 * kBBS) {
        double v[4];
        {
            const Q4<TX> q = load4(y + k);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (double)q.v[e];
        }
        int i = 0;
        for (; i + 4 <= nv; i += 4) {
            Q4<TX> s4[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) s4[t] = load4(p[i + t] + k);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] -= g[i + t] * (double)s4[t].v[e];
        }
        for (; i < nv; ++i) {
            const Q4<TX> q = load4(p[i] + k);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] -= g[i] * (double)q.v[e];
        }
        Q4<TX> o;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            o.v[e] = (TX)(post * v[e]);
            nrm += (double)o.v[e] * (double)o.v[e];
        }
        store4(y + k, o);
    }
    for (int64_t e = k; e < c.b && e < k + 4; ++e) {
        double v = (double)y[e];
        for (int i = 0; i < nv; ++i) v -= g[i] * (double)p[i][e];
        const TX t = (TX)(post * v);
        y[e] = t;
        nrm += (double)t * (double)t;
    }
    if (last) {
        const double sm = block_sum_any<kBBS>(nrm, red);
        if (threadIdx.x == 0) part[S.pbase + c.c] = sm;
    }
}

// End of a step, per running sector: beta_j and sigma_{j+1}^2 from the norm sum,
// lowest eigenpair of T_{j+1}, convergence test; then the sector either stops
// (converged or broken down), waits for a restart (basis full) or moves on.
__global__ __launch_bounds__(256) void kb_tridiag(BState st, BDims dm, double tol) {
    const int s = blockIdx.x;
    if (st.active[s] != 1) return;
    const int j = st.jcur[s];
    const int m = j + 1;
    double *alpha = st.alpha + (int64_t)s * dm.ms, *beta = st.beta + (int64_t)s * dm.ms;
    const double n2 = st.raw[(int64_t)s * dm.rs];
    const double bj = sqrt(n2);
    if (threadIdx.x == 0) {
        beta[j] = bj;
        st.sig2[(int64_t)s * dm.ms + j + 1] = n2 > 0.0 ? 1.0 / n2 : 0.0;
    }
    // the eigensolve and test run every dm.check steps, at the first step, when
    // the basis is full and when beta_j is at the breakdown level; in between
    // the sector just moves on
    const bool tiny = !(bj > 64.0 * 2.220446049250313e-16 * fmax(fabs(st.theta[s]), 1.0));
    if (!(m == 1 || m == dm.m || m % dm.check == 0 || tiny)) {
        if (threadIdx.x == 0) {
            st.iters[s] += 1;
            st.nvsum[s] += (double)(j + 1 - win_begin(dm.reorth, j));
            st.jcur[s] = j + 1;
        }
        return;
    }
    __syncthreads();
    double *out = st.tri + (int64_t)s * dm.mt;
    k_tridiag_lowest_body(alpha, beta, m, out, nullptr);
    if (threadIdx.x == 0) {  // the body's result is complete in thread 0
        const double theta = out[0], res = out[1], bl = out[2];
        const double scale = fmax(fabs(theta), 1.0);
        st.theta[s] = theta;
        st.resid[s] = res;
        st.nsteps[s] = m;
        st.iters[s] += 1;
        st.nvsum[s] += (double)(j + 1 - win_begin(dm.reorth, j));
        const bool brk = fabs(bl) <= 64.0 * 2.220446049250313e-16 * scale;
        if (res <= tol * scale || brk || !isfinite(theta)) st.active[s] = 0;
        else if (m == dm.m) st.active[s] = 2;
        else st.jcur[s] = j + 1;
    }
}

// ---------------------------------------------------------------- restarts --
// For every sector with a request (rnout > 0), in place over its chunk:
// out_o = sum_i C[i * nout + o] S_i, i < nin, o < nout (out_o is the storage of
// S_o; every thread reads all inputs of its elements before writing).  Norm
// partial of the last output at part[pbase + c].  NO >= nout at compile time.
template <typename TX, int NO>
__global__ __launch_bounds__(kBBS) void kb_restart_v4(const BSec<TX, TX> *secs, const RChunk *ch, BState st,
                                                      BDims dm, double *part) {
    __shared__ double cf[kBRMaxC];
    __shared__ double red[kBBS / 64];
    const RChunk c = ch[blockIdx.x];
    const int nout = st.rnout[c.sec];
    if (nout <= 0) return;
    const int nin = st.rnin[c.sec];
    const BSec<TX, TX> &S = secs[c.sec];
    const double *C = st.coef + (int64_t)c.sec * dm.mc;
    for (int i = threadIdx.x; i < nin * NO; i += kBBS) {
        const int r = i / NO, o = i - r * NO;
        cf[i] = o < nout ? C[r * nout + o] : 0.0;
    }
    __syncthreads();
    double nrm = 0.0;
    int64_t k = c.a + 4 * (int64_t)threadIdx.x;
    for (; k + 4 <= c.b; k += 4 * kBBS) {
        double acc[NO][4];
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[o][e] = 0.0;
        int i = 0;
        for (; i + 2 <= nin; i += 2) {
            const Q4<TX> v0 = load4(S.base + (int64_t)i * S.D + k), v1 = load4(S.base + (int64_t)(i + 1) * S.D + k);
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                const double c0 = cf[i * NO + o], c1 = cf[(i + 1) * NO + o];
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[o][e] += c0 * (double)v0.v[e] + c1 * (double)v1.v[e];
            }
        }
        if (i < nin) {
            const Q4<TX> v0 = load4(S.base + (int64_t)i * S.D + k);
#pragma unroll
            for (int o = 0; o < NO; ++o)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[o][e] += cf[i * NO + o] * (double)v0.v[e];
        }
#pragma unroll
        for (int o = 0; o < NO; ++o)
            if (o < nout) {
                Q4<TX> q;
#pragma unroll
                for (int e = 0; e < 4; ++e) q.v[e] = (TX)acc[o][e];
                store4(S.base + (int64_t)o * S.D + k, q);
                if (o == nout - 1)
#pragma unroll
                    for (int e = 0; e < 4; ++e) nrm += (double)q.v[e] * (double)q.v[e];
            }
    }
    for (int64_t e = k; e < c.b && e < k + 4; ++e) {
        double acc[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[o] = 0.0;
        for (int i = 0; i < nin; ++i) {
            const double v = (double)S.base[(int64_t)i * S.D + e];
#pragma unroll
            for (int o = 0; o < NO; ++o) acc[o] += cf[i * NO + o] * v;
        }
#pragma unroll
        for (int o = 0; o < NO; ++o)
            if (o < nout) {
                const TX t = (TX)acc[o];
                S.base[(int64_t)o * S.D + e] = t;
                if (o == nout - 1) nrm += (double)t * (double)t;
            }
    }
    const double sm = block_sum_any<kBBS>(nrm, red);
    if (threadIdx.x == 0) part[S.pbase + c.c] = sm;
}

// After the combination, per sector with a request: reset the recurrence.
// Explicit (from the Ritz vector, now S_0): sigma_0^2 = 1 / ||S_0||^2, step 0.
// Implicit (k kept orthonormal vectors, residual in S_k): the new leading
// tridiagonal block from a2b2, beta_{k-1} = ||f||, the Gram block of the kept
// vectors = I, step k; when ||f|| vanishes the kept vectors span an invariant
// subspace and the sector finishes on T_k.  Every request is cleared.
__global__ __launch_bounds__(256) void kb_restart_fin(BState st, BDims dm) {
    const int s = blockIdx.x;
    const int mode = st.rmode[s];
    if (st.rnout[s] <= 0 || mode == 3) {
        if (threadIdx.x == 0) st.rnout[s] = 0;
        return;
    }
    __shared__ int brk_s;
    const int k = st.rnout[s] - 1;  // implicit: kept vectors
    const double n2 = st.raw[(int64_t)s * dm.rs];
    double *alpha = st.alpha + (int64_t)s * dm.ms, *beta = st.beta + (int64_t)s * dm.ms;
    double *sig2 = st.sig2 + (int64_t)s * dm.ms;
    const double *a2 = st.a2b2 + (int64_t)s * 2 * 17, *b2 = a2 + 17;
    for (int i = threadIdx.x; i < dm.ms; i += 256) {
        if (mode == 1) {
            alpha[i] = 0.0;
            beta[i] = 0.0;
            sig2[i] = 0.0;
        } else {
            alpha[i] = i < k ? a2[i] : 0.0;
            beta[i] = i + 1 < k ? b2[i] : 0.0;
            sig2[i] = i < k ? 1.0 : 0.0;
        }
    }
    if (mode == 2 && dm.reorth == 3) {
        double *G = st.gram + (int64_t)s * dm.mg;
        const int ld = dm.m + 1;
        for (int i = threadIdx.x; i < k * k; i += 256) {
            const int r = i / k, q = i - r * k;
            G[(int64_t)r * ld + q] = r == q ? 1.0 : 0.0;
        }
    }
    if (threadIdx.x == 0) {
        const double scale = fmax(fabs(st.theta[s]), 1.0);
        const double lim = 64.0 * 2.220446049250313e-16 * scale;
        brk_s = (mode == 2 && !(n2 > lim * lim)) || (mode == 1 && !(n2 > 0.0));
    }
    __syncthreads();
    if (mode == 1) {
        if (threadIdx.x == 0) {
            sig2[0] = n2 > 0.0 ? 1.0 / n2 : 0.0;
            st.jcur[s] = 0;
            st.active[s] = brk_s ? 0 : 1;
            st.rnout[s] = 0;
        }
        return;
    }
    if (brk_s) {  // finish on the kept block
        k_tridiag_lowest_body(alpha, beta, k, st.tri + (int64_t)s * dm.mt, nullptr);
        if (threadIdx.x == 0) {
            st.theta[s] = st.tri[(int64_t)s * dm.mt];
            st.resid[s] = 0.0;
            st.nsteps[s] = k;
            st.active[s] = 0;
            st.rnout[s] = 0;
        }
        return;
    }
    if (threadIdx.x == 0) {
        beta[k - 1] = sqrt(n2);
        sig2[k] = 1.0 / n2;
        st.jcur[s] = k;
        st.active[s] = 1;
        st.rnout[s] = 0;
    }
}

// per sector RQ from the apply partials of its tiles, which are contiguous
// (tiles [tfirst[s], tfirst[s] + tcount[s])): one wave per sector, fixed order
__global__ __launch_bounds__(64) void kb_fin_rq(const int *tfirst, const int *tcount, const double *tpart,
                                                double *out) {
    const int s = blockIdx.x;
    const int t0 = tfirst[s], n = tcount[s];
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < n; t += 64) {
        a += tpart[2 * (int64_t)(t0 + t)];
        b += tpart[2 * (int64_t)(t0 + t) + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if (threadIdx.x == 0) {
        out[2 * s] = a;
        out[2 * s + 1] = b;
    }
}

// ------------------------------------------------------------------ host --
struct Batch {
    int nsec = 0;
    BDims dm{};
    size_t elem = 4;
    std::vector<const ed_ham_s *> hs;
    std::vector<int64_t> D;
    std::vector<size_t> slot_off;  // byte offset of each sector's slots
    int64_t npart = 0;
    std::vector<int> nch;
    std::vector<int64_t> pbase;
};

struct BLast {
    int64_t tile = 0, steps = 0, restart_events = 0;
    double bytes = 0.0;
};
static BLast g_last;

// The batch's options: max_basis 0 -> kBatchBasisDefault vectors per sector
// (at most 1000); keep only with a basis of at most 256 vectors, below the basis.
static ed_lanczos_opts batch_opts(ed_lanczos_opts o) {
    o.max_basis = std::max(2, std::min(o.max_basis == 0 ? kBatchBasisDefault : o.max_basis, 1000));
    if (o.keep < 0 || o.max_basis > 256) o.keep = 0;
    o.keep = std::min(o.keep, std::min(16, o.max_basis - 1));
    return o;
}

static void batch_dims(Batch &B, const ed_lanczos_opts &o) {
    BDims &d = B.dm;
    d.m = o.max_basis;
    d.ms = d.m + 2;
    d.mt = d.m + 8;
    d.rs = 2 * d.m + 4;
    d.mg = o.reorth == 3 ? (int64_t)(d.m + 1) * (d.m + 1) : 0;
    d.mc = (d.m + 1) * std::max(1, o.keep + 1);
    d.reorth = o.reorth;
    d.check = std::max(1, o.check_every);
}

static int64_t nchunks_of(int64_t D) { return (std::max<int64_t>(D, 1) + kBChunk - 1) / kBChunk; }

static size_t batch_layout(Batch &B, char *base, void **secs32, void **secs64, void **chunks, void **part,
                           BState *st, double **rq, size_t *nchunks_out) {
    Carve c{base, 0, 0};
    const BDims &d = B.dm;
    B.slot_off.resize(B.nsec);
    for (int s = 0; s < B.nsec; ++s) {
        c.off = (c.off + 255) & ~(size_t)255;
        B.slot_off[s] = c.off;
        c.off += (size_t)(d.m + 1) * (size_t)B.D[s] * B.elem;
    }
    B.nch.resize(B.nsec);
    B.pbase.resize(B.nsec);
    int64_t np = 0;
    size_t nchunks = 0;
    for (int s = 0; s < B.nsec; ++s) {
        B.nch[s] = (int)nchunks_of(B.D[s]);
        B.pbase[s] = np;
        np += (int64_t)d.rs * B.nch[s];
        nchunks += B.nch[s];
    }
    B.npart = np;
    *nchunks_out = nchunks;
    void *p;
    p = c.take(sizeof(BSec<float, float>) * B.nsec + sizeof(BSec<double, double>) * B.nsec);
    if (secs32) *secs32 = p;
    p = c.take(sizeof(BSec<float, double>) * B.nsec + sizeof(BSec<double, double>) * B.nsec);
    if (secs64) *secs64 = p;
    p = c.take(sizeof(RChunk) * nchunks);
    if (chunks) *chunks = p;
    p = c.take(sizeof(double) * (size_t)std::max<int64_t>(np, 1));
    if (part) *part = p;
    const size_t S = (size_t)B.nsec;
    BState t;
    t.sig2 = (double *)c.take(S * d.ms * 8);
    t.gamma = (double *)c.take(S * d.ms * 8);
    t.alpha = (double *)c.take(S * d.ms * 8);
    t.beta = (double *)c.take(S * d.ms * 8);
    t.tri = (double *)c.take(S * d.mt * 8);
    t.raw = (double *)c.take(S * d.rs * 8);
    t.gram = (double *)c.take(std::max<size_t>(S * (size_t)d.mg * 8, 8));
    t.coef = (double *)c.take(S * d.mc * 8);
    t.a2b2 = (double *)c.take(S * 34 * 8);
    t.theta = (double *)c.take(S * 8);
    t.resid = (double *)c.take(S * 8);
    t.nvsum = (double *)c.take(S * 8);
    t.active = (int *)c.take(S * 4);
    t.jcur = (int *)c.take(S * 4);
    t.nsteps = (int *)c.take(S * 4);
    t.iters = (int *)c.take(S * 4);
    t.rnin = (int *)c.take(S * 4);
    t.rnout = (int *)c.take(S * 4);
    t.rmode = (int *)c.take(S * 4);
    if (st) *st = t;
    double *r = (double *)c.take(S * 16 + 64);
    if (rq) *rq = r;
    return c.off + 256;
}

template <typename TX, typename TA>
static BSec<TX, TA> make_bsec(const ed_ham_s *h, TX *base, int nch, int64_t pbase) {
    BSec<TX, TA> b;
    const bool dbl = sizeof(TA) == 8;
    const SpinTab &U = h->sp[0], &Dn = h->sp[1];
    b.D = h->D;
    b.dup = h->dup;
    b.ddn = h->ddn;
    b.base = base;
    b.up_off = U.off.as<int32_t>();
    b.up_tgt = U.tgt.as<int32_t>();
    b.dn_off = Dn.off.as<int32_t>();
    b.dn_tgt = Dn.tgt.as<int32_t>();
    b.up_sa = (const TA *)(dbl ? U.sa64.p : U.sa32.p);
    b.dn_sa = (const TA *)(dbl ? Dn.sa64.p : Dn.sa32.p);
    b.up_e = (const TA *)(dbl ? U.ediag64.p : U.ediag32.p);
    b.dn_e = (const TA *)(dbl ? Dn.ediag64.p : Dn.ediag32.p);
    b.up_st = U.states.as<uint32_t>();
    b.dn_st = Dn.states.as<uint32_t>();
    b.up_c = U.cidx.as<uint8_t>();
    b.dn_c = Dn.cidx.as<uint8_t>();
    b.up_mv = U.mv.as<int32_t>();
    b.dn_mv = Dn.mv.as<int32_t>();
    b.umode = h->umode;
    b.umask = h->umask;
    b.U0 = (TA)h->U0;
    b.usite = (const TA *)(dbl ? h->usite64.p : h->usite32.p);
    b.koff = h->koff;
    b.xtab = (const TA *)(dbl ? h->xtab64.p : h->xtab32.p);
    b.nx = h->nx;
    b.xt = (const XTermDev<TA> *)(dbl ? h->xt64.p : h->xt32.p);
    b.xl_off = h->nx ? h->xl_off.as<int32_t>() : nullptr;
    b.xl_src = h->nx ? h->xl_src.as<int32_t>() : nullptr;
    b.xl_tab = h->nx ? h->xl_tab.as<int32_t>() : nullptr;
    b.xl_amp = h->nx ? (const TA *)(dbl ? h->xl_amp64.p : h->xl_amp32.p) : nullptr;
    b.nch = nch;
    b.pbase = pbase;
    return b;
}

static std::vector<ATile> make_tiles(const Batch &B, int64_t tile, size_t elem, size_t *lds_max) {
    std::vector<ATile> t;
    size_t lmax = 0;
    const size_t budget = 64 * 1024;
    // largest sectors first so the long tiles start early
    std::vector<int> order(B.nsec);
    for (int s = 0; s < B.nsec; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return B.D[a] > B.D[b]; });
    for (int s : order) {
        const ed_ham_s *h = B.hs[s];
        int64_t R = std::max<int64_t>(1, tile / std::max<int64_t>(h->ddn, 1));
        R = std::min<int64_t>(std::min<int64_t>(R, h->dup), kBRows);
        for (int64_t u0 = 0; u0 < h->dup; u0 += R) {
            const int nr = (int)std::min<int64_t>(R, h->dup - u0);
            const size_t bytes = (size_t)nr * (size_t)h->ddn * elem;
            const int lds = bytes <= budget ? 1 : 0;
            if (lds) lmax = std::max(lmax, bytes);
            t.push_back(ATile{s, (int32_t)u0, nr, lds});
        }
    }
    *lds_max = lmax;
    return t;
}

template <typename TX>
static ed_status run_batched(int nsec, const ed_ham_t *hs, const ed_lanczos_opts &o, const void *const *v0s,
                             uint64_t seed, void *ws, size_t ws_bytes, double *E0, ed_info *info, hipStream_t s) {
    Batch B;
    B.nsec = nsec;
    B.elem = sizeof(TX);
    for (int i = 0; i < nsec; ++i) {
        B.hs.push_back(hs[i]);
        B.D.push_back(hs[i]->D);
    }
    batch_dims(B, o);
    const BDims dm = B.dm;
    const int m = dm.m;
    void *secs_a, *secs_b, *chunks_p, *part_p;
    BState st;
    double *rq;
    size_t nchunks;
    const size_t need = batch_layout(B, (char *)ws, &secs_a, &secs_b, &chunks_p, &part_p, &st, &rq, &nchunks);
    if (ws_bytes < need) fail(ED_EINVAL, "batched workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    double *part = (double *)part_p;
    const size_t S = (size_t)nsec;
    // descriptors
    std::vector<BSec<TX, TX>> dsc;
    std::vector<BSec<TX, double>> dsc64;
    for (int i = 0; i < nsec; ++i) {
        TX *base = (TX *)((char *)ws + B.slot_off[i]);
        dsc.push_back(make_bsec<TX, TX>(hs[i], base, B.nch[i], B.pbase[i]));
        dsc64.push_back(make_bsec<TX, double>(hs[i], base, B.nch[i], B.pbase[i]));
    }
    BSec<TX, TX> *d_sec = (BSec<TX, TX> *)secs_a;
    BSec<TX, double> *d_sec64 = (BSec<TX, double> *)secs_b;
    ED_HIP(hipMemcpyAsync(d_sec, dsc.data(), dsc.size() * sizeof(dsc[0]), hipMemcpyHostToDevice, s));
    ED_HIP(hipMemcpyAsync(d_sec64, dsc64.data(), dsc64.size() * sizeof(dsc64[0]), hipMemcpyHostToDevice, s));
    std::vector<RChunk> chv;
    for (int i = 0; i < nsec; ++i)
        for (int c = 0; c < B.nch[i]; ++c)
            chv.push_back(RChunk{i, c, (int64_t)c * kBChunk, std::min<int64_t>(B.D[i], (int64_t)(c + 1) * kBChunk)});
    RChunk *d_ch = (RChunk *)chunks_p;
    ED_HIP(hipMemcpyAsync(d_ch, chv.data(), chv.size() * sizeof(RChunk), hipMemcpyHostToDevice, s));
    const unsigned nch_u = (unsigned)chv.size();
    // zeroed state
    {
        std::vector<double> z0(S * std::max(dm.ms, dm.mt), 0.0);
        std::vector<int> i0(S, 0);
        for (double *p : {st.sig2, st.gamma, st.alpha, st.beta})
            ED_HIP(hipMemcpyAsync(p, z0.data(), S * dm.ms * 8, hipMemcpyHostToDevice, s));
        ED_HIP(hipMemcpyAsync(st.tri, z0.data(), S * dm.mt * 8, hipMemcpyHostToDevice, s));
        for (double *p : {st.theta, st.resid, st.nvsum}) ED_HIP(hipMemcpyAsync(p, z0.data(), S * 8, hipMemcpyHostToDevice, s));
        for (int *p : {st.active, st.jcur, st.nsteps, st.iters, st.rnin, st.rnout, st.rmode})
            ED_HIP(hipMemcpyAsync(p, i0.data(), S * 4, hipMemcpyHostToDevice, s));
    }
    // start vectors -> slot 0
    for (int i = 0; i < nsec; ++i) {
        TX *base = (TX *)((char *)ws + B.slot_off[i]);
        if (v0s && v0s[i])
            ED_HIP(hipMemcpyAsync(base, v0s[i], (size_t)B.D[i] * B.elem, hipMemcpyDeviceToDevice, s));
        else
            k_fill<<<grid_for(B.D[i], 256, 4096), 256, 0, s>>>(base, B.D[i], seed + (uint64_t)i, 1,
                                                              sizeof(TX) == 4 ? 1 : 0);
    }
    ED_LAUNCH_CHECK();

    // ---- restart requests: host-side coefficients, one batched combination
    std::vector<double> h_al(S * dm.ms), h_be(S * dm.ms), h_sg(S * dm.ms), h_tri(S * dm.mt);
    std::vector<double> h_coef(S * dm.mc, 0.0), h_a2b2(S * 34, 0.0);
    std::vector<int> h_nsteps(S), h_rnin(S), h_rnout(S), h_rmode(S);
    double restart_bytes = 0.0;
    auto launch_restart = [&](int maxout) {
        for (int q = 0; q < nsec; ++q)
            if (h_rnout[q] > 0) restart_bytes += (double)(h_rnin[q] + h_rnout[q]) * (double)B.D[q] * (double)B.elem;
        ED_HIP(hipMemcpyAsync(st.coef, h_coef.data(), h_coef.size() * 8, hipMemcpyHostToDevice, s));
        ED_HIP(hipMemcpyAsync(st.a2b2, h_a2b2.data(), h_a2b2.size() * 8, hipMemcpyHostToDevice, s));
        ED_HIP(hipMemcpyAsync(st.rnin, h_rnin.data(), S * 4, hipMemcpyHostToDevice, s));
        ED_HIP(hipMemcpyAsync(st.rnout, h_rnout.data(), S * 4, hipMemcpyHostToDevice, s));
        ED_HIP(hipMemcpyAsync(st.rmode, h_rmode.data(), S * 4, hipMemcpyHostToDevice, s));
        if (maxout <= 1) kb_restart_v4<TX, 1><<<nch_u, kBBS, 0, s>>>(d_sec, d_ch, st, dm, part);
        else if (maxout <= 3) kb_restart_v4<TX, 3><<<nch_u, kBBS, 0, s>>>(d_sec, d_ch, st, dm, part);
        else if (maxout <= 5) kb_restart_v4<TX, 5><<<nch_u, kBBS, 0, s>>>(d_sec, d_ch, st, dm, part);
        else if (maxout <= 9) kb_restart_v4<TX, 9><<<nch_u, kBBS, 0, s>>>(d_sec, d_ch, st, dm, part);
        else kb_restart_v4<TX, 17><<<nch_u, kBBS, 0, s>>>(d_sec, d_ch, st, dm, part);
        kb_rowsum<TX><<<dim3(1, (unsigned)nsec), 64, 0, s>>>(d_sec, st, dm, 2, part);
        kb_restart_fin<<<nsec, 256, 0, s>>>(st, dm);
        ED_LAUNCH_CHECK();
    };
    // explicit (or final) request for sector q: S_0 <- sum_l s_l sigma_l S_l
    auto ritz_request = [&](int q, int mode) {
        const int ns = h_nsteps[q];
        double *C = h_coef.data() + (size_t)q * dm.mc;
        for (int l = 0; l < ns; ++l)
            C[l] = h_tri[(size_t)q * dm.mt + 3 + l] * std::sqrt(h_sg[(size_t)q * dm.ms + l]);
        h_rnin[q] = ns;
        h_rnout[q] = ns > 0 ? 1 : 0;
        h_rmode[q] = mode;
    };
    auto fetch_state = [&]() {
        ED_HIP(hipMemcpyAsync(h_al.data(), st.alpha, S * dm.ms * 8, hipMemcpyDeviceToHost, s));
        ED_HIP(hipMemcpyAsync(h_be.data(), st.beta, S * dm.ms * 8, hipMemcpyDeviceToHost, s));
        ED_HIP(hipMemcpyAsync(h_sg.data(), st.sig2, S * dm.ms * 8, hipMemcpyDeviceToHost, s));
        ED_HIP(hipMemcpyAsync(h_tri.data(), st.tri, S * dm.mt * 8, hipMemcpyDeviceToHost, s));
        ED_HIP(hipMemcpyAsync(h_nsteps.data(), st.nsteps, S * 4, hipMemcpyDeviceToHost, s));
        ED_HIP(hipStreamSynchronize(s));
    };
    // initial request: S_0 as given (coefficient 1), explicit reset of every sector
    std::fill(h_rnin.begin(), h_rnin.end(), 1);
    std::fill(h_rnout.begin(), h_rnout.end(), 1);
    std::fill(h_rmode.begin(), h_rmode.end(), 1);
    for (int q = 0; q < nsec; ++q) h_coef[(size_t)q * dm.mc] = 1.0;
    launch_restart(1);
    ED_HIP(hipStreamSynchronize(s));

    // ---- tile schedule: time a few tile sizes on slot 0 -> slot 1 (every sector at step 0)
    std::vector<int64_t> cands = {2048, 8192, 32768, 131072};
    if (const char *env = std::getenv("ED_BATCH_TILE")) cands = {std::max<int64_t>(64, std::atoll(env))};
    std::vector<ATile> best_tiles;
    int64_t best_tile_size = 0;
    size_t best_lds = 0;
    float best_ms = 1e30f;
    DevMem tile_mem;
    hipEvent_t ev0, ev1;
    ED_HIP(hipEventCreate(&ev0));
    ED_HIP(hipEventCreate(&ev1));
    auto kern0 = kb_apply<TX, TX, 0>;
    (void)hipFuncSetAttribute((const void *)kern0, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipGetLastError();
    for (int64_t tsz : cands) {
        size_t lds = 0;
        std::vector<ATile> tl = make_tiles(B, tsz, B.elem, &lds);
        tile_mem.alloc(tl.size() * sizeof(ATile));
        ED_HIP(hipMemcpyAsync(tile_mem.p, tl.data(), tl.size() * sizeof(ATile), hipMemcpyHostToDevice, s));
        kern0<<<(unsigned)tl.size(), kBBS, lds, s>>>(d_sec, tile_mem.as<ATile>(), st.jcur, st.active, 0, nullptr);
        ED_HIP(hipEventRecord(ev0, s));
        for (int r = 0; r < 3; ++r)
            kern0<<<(unsigned)tl.size(), kBBS, lds, s>>>(d_sec, tile_mem.as<ATile>(), st.jcur, st.active, 0, nullptr);
        ED_HIP(hipEventRecord(ev1, s));
        ED_LAUNCH_CHECK();
        ED_HIP(hipEventSynchronize(ev1));
        float ms = 0.f;
        ED_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        if (ms < best_ms) {
            best_ms = ms;
            best_tiles = tl;
            best_lds = lds;
            best_tile_size = tsz;
        }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    DevMem tiles;
    tiles.alloc(best_tiles.size() * sizeof(ATile));
    ED_HIP(hipMemcpyAsync(tiles.p, best_tiles.data(), best_tiles.size() * sizeof(ATile), hipMemcpyHostToDevice, s));
    const unsigned nt = (unsigned)best_tiles.size();
    ED_HIP(hipStreamSynchronize(s));

    // ---- one step of every running sector, captured once
    const int passes = o.reorth == 2 ? 2 : 1;
    const unsigned prow = (unsigned)(o.reorth == 3 ? 2 * (m + 1) : m + 1);
    auto record_step = [&](hipStream_t cs) {
        kb_apply<TX, TX, 0><<<nt, kBBS, best_lds, cs>>>(d_sec, tiles.as<ATile>(), st.jcur, st.active, 0, nullptr);
        for (int ps = 0; ps < passes; ++ps) {
            if (o.reorth == 3) kb_dots_v4<TX, 8, true><<<nch_u, kBBS, 0, cs>>>(d_sec, d_ch, st, o.reorth, part);
            else kb_dots_v4<TX, 8, false><<<nch_u, kBBS, 0, cs>>>(d_sec, d_ch, st, o.reorth, part);
            kb_rowsum<TX><<<dim3(prow, (unsigned)nsec), 64, 0, cs>>>(d_sec, st, dm, 0, part);
            kb_coef<<<nsec, 256, 0, cs>>>(st, dm);
            kb_update_v4<TX><<<nch_u, kBBS, 0, cs>>>(d_sec, d_ch, st, dm, part, ps == passes - 1);
        }
        kb_rowsum<TX><<<dim3(1, (unsigned)nsec), 64, 0, cs>>>(d_sec, st, dm, 1, part);
        kb_tridiag<<<nsec, 256, 0, cs>>>(st, dm, o.tol);
    };
    hipStream_t cs;
    ED_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    ED_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    record_step(cs);
    ED_HIP(hipStreamEndCapture(cs, &graph));
    ED_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));

    std::vector<int> act(S), restarts(S, 0);
    int64_t launches = 0, events = 0;
    const int every = std::max(1, o.check_every);
    while (launches < o.max_iter) {
        const int n = (int)std::min<int64_t>(every, o.max_iter - launches);
        for (int r = 0; r < n; ++r) ED_HIP(hipGraphLaunch(gexec, s));
        launches += n;
        ED_HIP(hipMemcpyAsync(act.data(), st.active, S * 4, hipMemcpyDeviceToHost, s));
        ED_HIP(hipStreamSynchronize(s));
        int on = 0, pend = 0;
        for (int q = 0; q < nsec; ++q) {
            on += act[q] == 1;
            pend += act[q] == 2;
        }
        if (on == 0 && pend == 0) break;
        if (launches >= o.max_iter || pend == 0) continue;
        // restart every sector whose basis is full; the shift plans of the
        // waiting sectors are independent host computations, spread over threads
        fetch_state();
        std::fill(h_rnout.begin(), h_rnout.end(), 0);
        std::vector<int> pending;
        for (int q = 0; q < nsec; ++q)
            if (act[q] == 2) {
                ++restarts[q];
                pending.push_back(q);
            }
        std::vector<char> implicit(pending.size(), 0);
        auto plan_range = [&](size_t b, size_t e) {
            std::vector<double> Cq, a2q, b2q, evq;
            for (size_t t = b; t < e; ++t) {
                const int q = pending[t];
                if (!(o.keep > 0 && o.keep < m && h_nsteps[q] == m)) continue;
                std::vector<double> al(h_al.begin() + (size_t)q * dm.ms, h_al.begin() + (size_t)q * dm.ms + m);
                std::vector<double> be(h_be.begin() + (size_t)q * dm.ms, h_be.begin() + (size_t)q * dm.ms + m);
                std::vector<double> sg(h_sg.begin() + (size_t)q * dm.ms, h_sg.begin() + (size_t)q * dm.ms + m + 1);
                if (!ir_plan(al, be, sg, m, o.keep, Cq, a2q, b2q, evq)) continue;
                std::copy(Cq.begin(), Cq.end(), h_coef.begin() + (size_t)q * dm.mc);
                double *ab = h_a2b2.data() + (size_t)q * 34;
                for (int i = 0; i < o.keep; ++i) {
                    ab[i] = a2q[i];
                    ab[17 + i] = i + 1 < o.keep ? b2q[i] : 0.0;
                }
                implicit[t] = 1;
            }
        };
        const size_t nth = std::min<size_t>(std::min<size_t>(pending.size() / 4 + 1, 16),
                                            std::max(1u, std::thread::hardware_concurrency()));
        if (nth <= 1) {
            plan_range(0, pending.size());
        } else {
            std::vector<std::thread> pool;
            const size_t per = (pending.size() + nth - 1) / nth;
            for (size_t k = 0; k < nth; ++k) {
                const size_t b = k * per, e = std::min(pending.size(), b + per);
                if (b < e) pool.emplace_back(plan_range, b, e);
            }
            for (auto &t : pool) t.join();
        }
        int maxout = 1;
        for (size_t t = 0; t < pending.size(); ++t) {
            const int q = pending[t];
            if (implicit[t]) {
                h_rnin[q] = m + 1;
                h_rnout[q] = o.keep + 1;
                h_rmode[q] = 2;
                maxout = std::max(maxout, o.keep + 1);
            } else {
                ritz_request(q, 1);
            }
        }
        launch_restart(maxout);
        ++events;
    }
    (void)hipGraphExecDestroy(gexec);
    (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);

    // ---- final Ritz vectors (into S_0) for every sector, FP64 Rayleigh quotients
    ED_HIP(hipMemcpyAsync(act.data(), st.active, S * 4, hipMemcpyDeviceToHost, s));
    fetch_state();
    std::fill(h_rnout.begin(), h_rnout.end(), 0);
    for (int q = 0; q < nsec; ++q) ritz_request(q, 3);
    launch_restart(1);
    std::vector<double> theta(S), resid(S), rqv(2 * S, 0.0);
    std::vector<int> iters(S);
    std::vector<double> nvsum(S);
    ED_HIP(hipMemcpyAsync(nvsum.data(), st.nvsum, S * 8, hipMemcpyDeviceToHost, s));
    ED_HIP(hipMemcpyAsync(theta.data(), st.theta, S * 8, hipMemcpyDeviceToHost, s));
    ED_HIP(hipMemcpyAsync(resid.data(), st.resid, S * 8, hipMemcpyDeviceToHost, s));
    ED_HIP(hipMemcpyAsync(iters.data(), st.iters, S * 4, hipMemcpyDeviceToHost, s));
    if (o.refine) {
        DevMem tp;
        tp.alloc((size_t)nt * 2 * sizeof(double));
        auto kern = kb_apply<TX, double, 1>;
        (void)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
        (void)hipGetLastError();
        kern<<<nt, kBBS, best_lds, s>>>(d_sec64, tiles.as<ATile>(), st.jcur, st.active, 0, tp.as<double>());
        std::vector<int> tfc((size_t)2 * nsec, 0);  // first tile, tile count per sector
        for (size_t t = 0; t < best_tiles.size(); ++t) {
            const int q = best_tiles[t].sec;
            if (tfc[(size_t)nsec + q] == 0) tfc[q] = (int)t;
            ++tfc[(size_t)nsec + q];
        }
        DevMem tfd;
        tfd.alloc(tfc.size() * sizeof(int));
        ED_HIP(hipMemcpyAsync(tfd.p, tfc.data(), tfc.size() * sizeof(int), hipMemcpyHostToDevice, s));
        kb_fin_rq<<<nsec, 64, 0, s>>>(tfd.as<int>(), tfd.as<int>() + nsec, tp.as<double>(), rq);
        ED_LAUNCH_CHECK();
        ED_HIP(hipMemcpyAsync(rqv.data(), rq, 2 * S * sizeof(double), hipMemcpyDeviceToHost, s));
        ED_HIP(hipStreamSynchronize(s));  // before tp and tfd are released
    }
    ED_HIP(hipStreamSynchronize(s));
    // algorithmic bytes: per step x read + y write, and per projection pass the
    // window of nv stored vectors read twice (dot, update) plus Y read twice and
    // written once; each restart reads nin and writes nout vectors
    double bytes = restart_bytes;
    bool allconv = true;
    for (int q = 0; q < nsec; ++q) {
        const double bq = (double)B.D[q] * (double)B.elem *
                          (2.0 * iters[q] + passes * (2.0 * nvsum[q] + 3.0 * iters[q]));
        bytes += bq;
        const bool conv = act[q] == 0;
        allconv &= conv;
        const double rqi = (o.refine && rqv[2 * q + 1] > 0.0) ? rqv[2 * q] / rqv[2 * q + 1] : theta[q];
        E0[q] = rqi;
        if (info) {
            ed_info f{};
            f.iters = iters[q];
            f.restarts = restarts[q];
            f.converged = conv ? 1 : 0;
            f.basis_used = m;
            f.residual = resid[q];
            f.ritz = theta[q];
            f.rq_fp64 = rqi;
            f.gap_lower = std::nan("");
            f.e_lower = std::nan("");
            f.traffic = bq;
            info[q] = f;
        }
    }
    g_last.tile = best_tiles.empty() ? 0 : best_tile_size;
    g_last.steps = launches;
    g_last.restart_events = events;
    g_last.bytes = bytes;
    return allconv ? ED_OK : ED_ENOCONV;
}

}  // namespace ed

extern "C" int64_t ed_batched_last_tile(void) { return ed::g_last.tile; }

extern "C" void ed_batched_last_stats(int64_t *steps, int64_t *restart_events, double *bytes) {
    if (steps) *steps = ed::g_last.steps;
    if (restart_events) *restart_events = ed::g_last.restart_events;
    if (bytes) *bytes = ed::g_last.bytes;
}

using namespace ed;

extern "C" ed_status ed_batched_workspace_bytes(int nsec, const ed_ham_t *hs, const ed_lanczos_opts *opts,
                                                size_t *bytes) {
    return guard([&] {
        if (nsec < 1 || !hs || !bytes) fail(ED_EINVAL, "ed_batched_workspace_bytes: bad arguments");
        ed_lanczos_opts o = effective(opts, INT64_MAX);
        Batch B;
        B.nsec = nsec;
        for (int i = 0; i < nsec; ++i) {
            if (!hs[i]) fail(ED_EINVAL, "ed_batched_workspace_bytes: NULL handle %d", i);
            if (hs[i]->prec != hs[0]->prec) fail(ED_EINVAL, "batched sectors must share one precision");
            B.hs.push_back(hs[i]);
            B.D.push_back(hs[i]->D);
        }
        B.elem = hs[0]->prec == ED_FP64 ? 8 : 4;
        batch_dims(B, batch_opts(o));
        size_t nchunks;
        *bytes = batch_layout(B, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, &nchunks);
    });
}

extern "C" ed_status ed_lanczos_ground_batched(int nsec, const ed_ham_t *hs, const ed_lanczos_opts *opts,
                                               const void *const *v0s, uint64_t seed, void *ws, size_t ws_bytes,
                                               double *E0, ed_info *info, void *stream) {
    ed_status result = ED_OK;
    ed_status st = guard([&] {
        if (nsec < 1 || !hs || !ws || !E0) fail(ED_EINVAL, "ed_lanczos_ground_batched: bad arguments");
        for (int i = 0; i < nsec; ++i) {
            if (!hs[i]) fail(ED_EINVAL, "ed_lanczos_ground_batched: NULL handle %d", i);
            if (hs[i]->prec != hs[0]->prec) fail(ED_EINVAL, "batched sectors must share one precision");
            if (hs[i]->device != hs[0]->device) fail(ED_EINVAL, "batched sectors must live on one GPU");
            if (hs[i]->D >= ((int64_t)1 << 31))
                fail(ED_EINVAL, "batched sector %d has D = %lld >= 2^31 (solve it alone)", i, (long long)hs[i]->D);
        }
        const ed_lanczos_opts o = batch_opts(effective(opts, INT64_MAX));
        DeviceGuard g(hs[0]->device);
        if (hs[0]->prec == ED_FP64)
            result = run_batched<double>(nsec, hs, o, v0s, seed, ws, ws_bytes, E0, info, (hipStream_t)stream);
        else
            result = run_batched<float>(nsec, hs, o, v0s, seed, ws, ws_bytes, E0, info, (hipStream_t)stream);
    });
    if (st != ED_OK) return st;
    return result;
}
