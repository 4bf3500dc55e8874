// Setup phase in matrix-free form (the paper's "Hamiltonian construction",
// T_setup in Table 1): per-spin hop tables, one-spin diagonal pieces, the
// cross-spin density-density decomposition and the move tables of the
// four-fermion (spin-flip / pair-hopping) terms of Section 4.
//
// Hop table of spin s: for source rank r and each ordered pair (i, j), i != j,
// with h_ij != 0, j occupied and i empty, the entry (target rank of
// s ^ (1<<i) ^ (1<<j), sign, h_ij) of  h_ij c+_i c_j |r>.  The sign is the parity
// of occupied sites strictly between i and j (computed with a popcount).  Rows
// are sorted by target rank.  Because h is symmetric the same table serves the
// gather (pull) form of the product.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <map>
#include <tuple>

#include "ed_internal.h"

namespace ed {

__device__ __forceinline__ uint32_t between_mask(int i, int j) {
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    // bits lo+1 .. hi-1
    return ((1u << hi) - 1u) & ~((2u << lo) - 1u);
}

// ---------------------------------------------------------------- scan ----
// Exclusive prefix sum of n int64 values in one workgroup (setup only).
__global__ void k_scan_i64(const int64_t *in, int64_t *out, int64_t n) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + blockDim.x - 1) / blockDim.x;
    const int64_t a = t * chunk, b = (a + chunk < n) ? a + chunk : n;
    int64_t s = 0;
    for (int64_t i = a; i < b; ++i) s += in[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int k = 0; k < (int)blockDim.x; ++k) {
            const int64_t v = part[k];
            part[k] = run;
            run += v;
        }
        out[n] = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int64_t i = a; i < b; ++i) {
        const int64_t v = in[i];
        out[i] = run;
        run += v;
    }
}

// ------------------------------------------------------------ hop tables ----
// Same-spin two-body string c+_i c+_j c_l c_k (q = (i, j, k, l)) on a one-spin
// word: the operators act right to left, each contributing (-1)^(occupied
// modes below it); false when one of them annihilates the state.
__device__ __forceinline__ bool two_body_move(uint32_t s, int4 q, uint32_t *out, int *neg) {
    const int pos[4] = {q.z, q.w, q.y, q.x};
    const bool cre[4] = {false, false, true, true};
    int par = 0;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const uint32_t b = 1u << pos[o];
        if (((s & b) != 0u) == cre[o]) return false;
        par += __popc(s & (b - 1u));
        s ^= b;
    }
    *out = s;
    *neg = par & 1;
    return true;
}

__global__ void k_hop_count(const uint32_t *st, int64_t dim, const int2 *pairs, int np, const int4 *quads, int nq,
                            int64_t *cnt) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = st[r];
        int c = 0;
        for (int q = 0; q < np; ++q) {
            const int i = pairs[q].x, j = pairs[q].y;
            c += ((s >> j) & 1u) && !((s >> i) & 1u);
        }
        for (int q = 0; q < nq; ++q) {
            uint32_t s2;
            int ng;
            c += two_body_move(s, quads[q], &s2, &ng) ? 1 : 0;
        }
        cnt[r] = c;
    }
}

// ipos (nullptr = identity): position of each rank in the handle's basis order
__global__ void k_hop_fill(const uint32_t *st, int64_t dim, int ns, int n, const int2 *pairs,
                           const double *pamp, int np, const int4 *quads, const double *qamp, int nq,
                           const int64_t *off64, int32_t *off,
                           int32_t *tgt, int8_t *sgn, double *amp, double *sa64, float *sa32,
                           const int32_t *ipos) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = st[r];
        const int64_t a = off64[r];
        off[r] = (int32_t)a;
        if (r == dim - 1) off[dim] = (int32_t)off64[dim];
        int64_t k = a;
        for (int q = 0; q < np; ++q) {
            const int i = pairs[q].x, j = pairs[q].y;
            if (!(((s >> j) & 1u) && !((s >> i) & 1u))) continue;
            const uint32_t s2 = s ^ (1u << i) ^ (1u << j);
            int32_t t = (int32_t)rank_state(s2, ns, n);
            if (ipos) t = ipos[t];
            const int8_t sg = (__popc(s & between_mask(i, j)) & 1) ? (int8_t)-1 : (int8_t)1;
            // insertion into the sorted run [a, k)
            int64_t p = k;
            while (p > a && tgt[p - 1] > t) {
                tgt[p] = tgt[p - 1];
                sgn[p] = sgn[p - 1];
                amp[p] = amp[p - 1];
                --p;
            }
            tgt[p] = t;
            sgn[p] = sg;
            amp[p] = pamp[q];
            ++k;
        }
        for (int q = 0; q < nq; ++q) {
            uint32_t s2;
            int ng;
            if (!two_body_move(s, quads[q], &s2, &ng)) continue;
            int32_t t = (int32_t)rank_state(s2, ns, n);
            if (ipos) t = ipos[t];
            int64_t p = k;
            while (p > a && tgt[p - 1] > t) {
                tgt[p] = tgt[p - 1];
                sgn[p] = sgn[p - 1];
                amp[p] = amp[p - 1];
                --p;
            }
            tgt[p] = t;
            sgn[p] = ng ? (int8_t)-1 : (int8_t)1;
            amp[p] = qamp[q];
            ++k;
        }
        for (int64_t e = a; e < k; ++e) {
            const double v = (double)sgn[e] * amp[e];
            sa64[e] = v;
            sa32[e] = (float)v;
        }
    }
}

// sliced ELL: slice = 64 consecutive states, entries (slice, k, lane)
__global__ void k_ell_len(const int64_t *cnt, int64_t dim, int64_t nslices, int64_t *len) {
    for (int64_t sl = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; sl < nslices;
         sl += (int64_t)gridDim.x * blockDim.x) {
        int64_t m = 0;
        for (int l = 0; l < 64; ++l) {
            const int64_t r = sl * 64 + l;
            if (r < dim && cnt[r] > m) m = cnt[r];
        }
        len[sl] = m * 64;
    }
}

__global__ void k_ell_fill(const int64_t *off64, int64_t dim, int64_t nslices, const int64_t *ell64,
                           int32_t *ell_off, const int32_t *tgt, const double *sa64, int32_t *etgt,
                           double *esa64, float *esa32) {
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < nslices * 64;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t sl = idx >> 6;
        const int lane = (int)(idx & 63);
        const int64_t base = ell64[sl];
        const int64_t kk = (ell64[sl + 1] - base) >> 6;
        if (lane == 0) {
            ell_off[sl] = (int32_t)base;
            if (sl == nslices - 1) ell_off[nslices] = (int32_t)ell64[nslices];
        }
        const int64_t r = idx;
        const int64_t a = r < dim ? off64[r] : 0;
        const int64_t c = r < dim ? off64[r + 1] - a : 0;
        for (int64_t k = 0; k < kk; ++k) {
            const int64_t e = base + k * 64 + lane;
            if (k < c) {
                etgt[e] = tgt[a + k];
                esa64[e] = sa64[a + k];
                esa32[e] = (float)sa64[a + k];
            } else {
                etgt[e] = r < dim ? (int32_t)r : 0;
                esa64[e] = 0.0;
                esa32[e] = 0.0f;
            }
        }
    }
}

// packed ELL entries from the unpacked ones and the amplitude index map
__global__ void k_ell_pack(const int32_t *etgt, const int32_t *eamp_idx, int64_t n, uint32_t *out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (uint32_t)etgt[e] | ((uint32_t)eamp_idx[e] << 20);
}

// ------------------------------------------------------- diagonal pieces ----
// e_s(state) = sum_i eps_i n_i + sum_{i<j} w_ij n_i n_j  (FP64, cast for FP32)
__global__ void k_ediag(const uint32_t *st, int64_t dim, int ns, const double *eps, const double *wss,
                        double *e64, float *e32) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = st[r];
        double e = 0.0;
        for (int i = 0; i < ns; ++i) {
            if (!((s >> i) & 1u)) continue;
            e += eps[i];
            for (int j = i + 1; j < ns; ++j)
                if ((s >> j) & 1u) e += wss[i * ns + j];
        }
        e64[r] = e;
        e32[r] = (float)e;
    }
}

__global__ void k_cidx(const uint32_t *st, int64_t dim, const int *sites, int k, uint8_t *out) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = st[r];
        uint32_t c = 0;
        for (int q = 0; q < k; ++q) c |= ((s >> sites[q]) & 1u) << q;
        out[r] = (uint8_t)c;
    }
}

// move table: electron src -> dst on every state: (rank << 1 | sign bit) or -1
// (position instead of rank when ipos is given)
__global__ void k_move(const uint32_t *st, int64_t dim, int ns, int n, int src, int dst, int32_t *out,
                       const int32_t *ipos) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t s = st[r];
        int32_t v = -1;
        if (src == dst) {
            if ((s >> src) & 1u) v = (int32_t)(r << 1);  // c+_i c_i = n_i: same state, no sign
        } else if (((s >> src) & 1u) && !((s >> dst) & 1u)) {
            const uint32_t s2 = s ^ (1u << src) ^ (1u << dst);
            int64_t t = rank_state(s2, ns, n);
            if (ipos) t = ipos[t];
            const int neg = __popc(s & between_mask(src, dst)) & 1;
            v = (int32_t)((t << 1) | neg);
        }
        out[r] = v;
    }
}

// per up state u: the terms q whose up move applies to u, with the source rank
// and the signed amplitude folded together
__global__ void k_xlist_count(const int32_t *up_mv, int64_t dup, const XTermDev<double> *xt, int nx,
                              int64_t *cnt) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < dup; u += (int64_t)gridDim.x * blockDim.x) {
        int c = 0;
        for (int q = 0; q < nx; ++q) c += up_mv[(int64_t)xt[q].up_mv * dup + u] >= 0;
        cnt[u] = c;
    }
}

__global__ void k_xlist_fill(const int32_t *up_mv, int64_t dup, const XTermDev<double> *xt, int nx,
                             const int64_t *off64, int32_t *off, int32_t *src, int32_t *tab, double *a64,
                             float *a32) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < dup; u += (int64_t)gridDim.x * blockDim.x) {
        int64_t e = off64[u];
        off[u] = (int32_t)e;
        if (u == dup - 1) off[dup] = (int32_t)off64[dup];
        for (int q = 0; q < nx; ++q) {
            const int32_t mu = up_mv[(int64_t)xt[q].up_mv * dup + u];
            if (mu < 0) continue;
            const double a = (mu & 1) ? -xt[q].amp : xt[q].amp;
            src[e] = mu >> 1;
            tab[e] = xt[q].dn_mv;
            a64[e] = a;
            a32[e] = (float)a;
            ++e;
        }
    }
}

// ------------------------------------------------------------------ host ----
static bool finite_all(const double *a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

template <class T>
static void upload(DevMem &m, const std::vector<T> &v) {
    m.alloc(std::max<size_t>(v.size(), 1) * sizeof(T));
    if (!v.empty()) ED_HIP(hipMemcpy(m.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

static int move_index(SpinTab &t, int src, int dst) {
    for (int q = 0; q < (int)t.mv_src.size(); ++q)
        if (t.mv_src[q] == src && t.mv_dst[q] == dst) return q;
    t.mv_src.push_back(src);
    t.mv_dst.push_back(dst);
    return (int)t.mv_src.size() - 1;
}

static void build_spin(ed_ham_s *h, int s, const BasisData &b, const ed_params *p) {
    SpinTab &t = h->sp[s];
    const int ns = b.ns;
    t.ns = ns;
    t.n = b.n[s];
    t.dim = b.dim[s];
    const int64_t dim = t.dim;
    t.states.alloc((size_t)dim * sizeof(uint32_t));
    ED_HIP(hipMemcpy(t.states.p, b.states[s].p, (size_t)dim * sizeof(uint32_t), hipMemcpyDeviceToDevice));

    // ordered pairs (i, j) with h_ij != 0, in (i, j) lexicographic order
    std::vector<int2> pairs;
    std::vector<double> pamp;
    const double *hs = p->hop + (size_t)s * ns * ns;
    for (int i = 0; i < ns; ++i)
        for (int j = 0; j < ns; ++j)
            if (i != j && hs[i * ns + j] != 0.0) {
                pairs.push_back(make_int2(i, j));
                pamp.push_back(hs[i * ns + j]);
            }
    // same-spin two-body terms of this spin, (i, j, k, l) for c+_i c+_j c_l c_k
    std::vector<int4> quads;
    std::vector<double> qamp;
    for (int t2 = 0; t2 < p->n_x; ++t2) {
        const ed_xterm &x = p->x[t2];
        if (x.type == (s == 0 ? ED_UU_GENERAL : ED_DD_GENERAL)) {
            quads.push_back(make_int4(x.m, x.mp, x.k, x.l));
            qamp.push_back(x.coef);
        }
    }
    DevMem dpairs, dpamp, dquads, dqamp, cnt, off64;
    upload(dpairs, pairs);
    upload(dpamp, pamp);
    upload(dquads, quads);
    upload(dqamp, qamp);
    cnt.alloc((size_t)dim * sizeof(int64_t));
    off64.alloc((size_t)(dim + 1) * sizeof(int64_t));
    const unsigned g = grid_for(dim, 256, 1 << 16);
    k_hop_count<<<g, 256>>>(t.states.as<uint32_t>(), dim, dpairs.as<int2>(), (int)pairs.size(), dquads.as<int4>(),
                            (int)quads.size(), cnt.as<int64_t>());
    ED_LAUNCH_CHECK();
    k_scan_i64<<<1, 1024>>>(cnt.as<int64_t>(), off64.as<int64_t>(), dim);
    ED_LAUNCH_CHECK();
    int64_t nnz = 0;
    ED_HIP(hipMemcpy(&nnz, off64.as<int64_t>() + dim, sizeof(int64_t), hipMemcpyDeviceToHost));
    if (nnz > 0x7fffffffll) fail(ED_ENOMEM, "hop table of spin %d has %lld entries (> 2^31-1)", s, (long long)nnz);
    t.nnz = nnz;
    t.off.alloc((size_t)(dim + 1) * sizeof(int32_t));
    t.tgt.alloc((size_t)nnz * sizeof(int32_t));
    t.sgn.alloc((size_t)nnz);
    t.amp.alloc((size_t)nnz * sizeof(double));
    t.sa64.alloc((size_t)nnz * sizeof(double));
    t.sa32.alloc((size_t)nnz * sizeof(float));
    k_hop_fill<<<g, 256>>>(t.states.as<uint32_t>(), dim, ns, t.n, dpairs.as<int2>(), dpamp.as<double>(),
                           (int)pairs.size(), dquads.as<int4>(), dqamp.as<double>(), (int)quads.size(),
                           off64.as<int64_t>(), t.off.as<int32_t>(), t.tgt.as<int32_t>(),
                           t.sgn.as<int8_t>(), t.amp.as<double>(), t.sa64.as<double>(), t.sa32.as<float>(),
                           h->grouped ? h->gipos[s].as<int32_t>() : nullptr);
    ED_LAUNCH_CHECK();

    // sliced ELL
    t.nslices = (dim + 63) / 64;
    DevMem ellen, ell64;
    ellen.alloc((size_t)t.nslices * sizeof(int64_t));
    ell64.alloc((size_t)(t.nslices + 1) * sizeof(int64_t));
    k_ell_len<<<grid_for(t.nslices, 256, 1 << 16), 256>>>(cnt.as<int64_t>(), dim, t.nslices, ellen.as<int64_t>());
    ED_LAUNCH_CHECK();
    k_scan_i64<<<1, 1024>>>(ellen.as<int64_t>(), ell64.as<int64_t>(), t.nslices);
    ED_LAUNCH_CHECK();
    int64_t nell = 0;
    ED_HIP(hipMemcpy(&nell, ell64.as<int64_t>() + t.nslices, sizeof(int64_t), hipMemcpyDeviceToHost));
    if (nell > 0x7fffffffll) fail(ED_ENOMEM, "sliced hop table of spin %d too large", s);
    t.ell_off.alloc((size_t)(t.nslices + 1) * sizeof(int32_t));
    t.ell_tgt.alloc((size_t)nell * sizeof(int32_t));
    t.ell_sa64.alloc((size_t)nell * sizeof(double));
    t.ell_sa32.alloc((size_t)nell * sizeof(float));
    k_ell_fill<<<grid_for(t.nslices * 64, 256, 1 << 16), 256>>>(
        off64.as<int64_t>(), dim, t.nslices, ell64.as<int64_t>(), t.ell_off.as<int32_t>(), t.tgt.as<int32_t>(),
        t.sa64.as<double>(), t.ell_tgt.as<int32_t>(), t.ell_sa64.as<double>(), t.ell_sa32.as<float>());
    ED_LAUNCH_CHECK();
    {
        std::vector<int64_t> hc((size_t)dim);
        ED_HIP(hipMemcpy(hc.data(), cnt.p, (size_t)dim * sizeof(int64_t), hipMemcpyDeviceToHost));
        int64_t m = 0;
        for (int64_t v : hc) m = std::max(m, v);
        t.max_hops = (int)m;
    }
    // packed form: distinct signed amplitudes (index 0 is the zero of the padding)
    t.pk_ok = false;
    if (dim <= (1 << 20) && nell > 0) {
        std::vector<double> esa((size_t)nell);
        ED_HIP(hipMemcpy(esa.data(), t.ell_sa64.p, (size_t)nell * sizeof(double), hipMemcpyDeviceToHost));
        std::vector<double> vals{0.0};
        std::map<double, int> idx;
        idx[0.0] = 0;
        std::vector<int32_t> ai((size_t)nell);
        bool ok = true;
        for (int64_t e = 0; e < nell && ok; ++e) {
            auto it = idx.find(esa[e]);
            if (it == idx.end()) {
                if (vals.size() >= 4095) { ok = false; break; }
                it = idx.emplace(esa[e], (int)vals.size()).first;
                vals.push_back(esa[e]);
            }
            ai[e] = it->second;
        }
        if (ok) {
            DevMem dai;
            upload(dai, ai);
            t.ell_pk.alloc((size_t)nell * sizeof(uint32_t));
            k_ell_pack<<<grid_for(nell, 256, 1 << 16), 256>>>(t.ell_tgt.as<int32_t>(), dai.as<int32_t>(), nell,
                                                            t.ell_pk.as<uint32_t>());
            ED_LAUNCH_CHECK();
            upload(t.amp64, vals);
            std::vector<float> v32(vals.begin(), vals.end());
            upload(t.amp32, v32);
            t.namp = (int)vals.size();
            t.pk_ok = true;
            ED_HIP(hipDeviceSynchronize());
            // four-state packed ELL: a slice is 256 consecutive states, lane l of a
            // wave holds states 4l .. 4l+3 of it, one uint4 per (slice, hop k, lane);
            // padding entries point at the state itself (or the last state) with
            // amplitude index 0
            std::vector<int32_t> ho((size_t)dim + 1), ht((size_t)std::max<int64_t>(nnz, 1));
            std::vector<double> hs((size_t)std::max<int64_t>(nnz, 1));
            ED_HIP(hipMemcpy(ho.data(), t.off.p, (size_t)(dim + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
            if (nnz > 0) {
                ED_HIP(hipMemcpy(ht.data(), t.tgt.p, (size_t)nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
                ED_HIP(hipMemcpy(hs.data(), t.sa64.p, (size_t)nnz * sizeof(double), hipMemcpyDeviceToHost));
            }
            const int64_t n4 = (dim + 255) / 256;
            std::vector<int32_t> o4((size_t)n4 + 1);
            std::vector<uint32_t> e4;
            for (int64_t sl = 0; sl < n4; ++sl) {
                int kk = 0;
                for (int64_t q = sl * 256; q < std::min<int64_t>(dim, sl * 256 + 256); ++q)
                    kk = std::max(kk, ho[q + 1] - ho[q]);
                o4[sl] = (int32_t)(e4.size() / 4);
                for (int k = 0; k < kk; ++k)
                    for (int l = 0; l < 256; ++l) {
                        const int64_t q = sl * 256 + l;
                        uint32_t v = (uint32_t)std::min<int64_t>(q, dim - 1);
                        if (q < dim && k < ho[q + 1] - ho[q]) {
                            const int64_t e = ho[q] + k;
                            v = (uint32_t)ht[e] | ((uint32_t)idx.at(hs[e]) << 20);
                        }
                        e4.push_back(v);
                    }
            }
            o4[n4] = (int32_t)(e4.size() / 4);
            if (e4.empty()) e4.assign(4, 0u);
            t.nslices4 = n4;
            upload(t.ell4_off, o4);
            upload(t.ell4, e4);
        }
    }

    // one-spin diagonal piece
    std::vector<double> eps(p->eps + (size_t)s * ns, p->eps + (size_t)(s + 1) * ns);
    std::vector<double> wss(p->w_ss + (size_t)s * ns * ns, p->w_ss + (size_t)(s + 1) * ns * ns);
    DevMem deps, dwss;
    upload(deps, eps);
    upload(dwss, wss);
    t.ediag64.alloc((size_t)dim * sizeof(double));
    t.ediag32.alloc((size_t)dim * sizeof(float));
    k_ediag<<<g, 256>>>(t.states.as<uint32_t>(), dim, ns, deps.as<double>(), dwss.as<double>(),
                        t.ediag64.as<double>(), t.ediag32.as<float>());
    ED_LAUNCH_CHECK();
    ED_HIP(hipDeviceSynchronize());
}

static void build_cross(ed_ham_s *h, const ed_params *p) {
    const int ns = h->ns;
    const double *w = p->w_ud;
    // on-site part
    uint32_t umask = 0;
    double u0 = 0.0;
    bool uniform = true;
    std::vector<double> us(32, 0.0);
    for (int i = 0; i < ns; ++i) {
        const double v = w[i * ns + i];
        us[i] = v;
        if (v == 0.0) continue;
        if (umask == 0) u0 = v;
        else if (v != u0) uniform = false;
        umask |= 1u << i;
    }
    h->umask = umask;
    h->U0 = u0;
    h->umode = umask == 0 ? 0 : (uniform ? 1 : 2);
    upload(h->usite64, us);
    std::vector<float> us32(us.begin(), us.end());
    upload(h->usite32, us32);

    // off-diagonal part: sites touched by any w_ud[i][j], i != j
    std::vector<int> sites;
    for (int i = 0; i < ns; ++i) {
        bool any = false;
        for (int j = 0; j < ns; ++j)
            if (j != i && (w[i * ns + j] != 0.0 || w[j * ns + i] != 0.0)) any = true;
        if (any) sites.push_back(i);
    }
    if (sites.size() > 8)
        fail(ED_EUNSUPPORTED, "off-diagonal w_ud entries touch %zu sites (at most 8 supported)", sites.size());
    h->koff = (int)sites.size();
    const int k = h->koff;
    if (k > 0) {
        const int nt = 1 << k;
        std::vector<double> tab((size_t)nt * nt, 0.0);
        for (int cu = 0; cu < nt; ++cu)
            for (int cd = 0; cd < nt; ++cd) {
                double e = 0.0;
                for (int a = 0; a < k; ++a)
                    for (int c = 0; c < k; ++c)
                        if (a != c || sites[a] != sites[c])
                            if (((cu >> a) & 1) && ((cd >> c) & 1) && sites[a] != sites[c])
                                e += w[sites[a] * ns + sites[c]];
                tab[(size_t)cu * nt + cd] = e;
            }
        upload(h->xtab64, tab);
        std::vector<float> tab32(tab.begin(), tab.end());
        upload(h->xtab32, tab32);
        DevMem dsites;
        upload(dsites, sites);
        for (int s = 0; s < 2; ++s) {
            SpinTab &t = h->sp[s];
            t.cidx.alloc((size_t)t.dim);
            k_cidx<<<grid_for(t.dim, 256, 1 << 16), 256>>>(t.states.as<uint32_t>(), t.dim, dsites.as<int>(), k,
                                                          t.cidx.as<uint8_t>());
            ED_LAUNCH_CHECK();
        }
        ED_HIP(hipDeviceSynchronize());
    } else {
        upload(h->xtab64, std::vector<double>(1, 0.0));
        upload(h->xtab32, std::vector<float>(1, 0.0f));
        for (int s = 0; s < 2; ++s) {
            h->sp[s].cidx.alloc((size_t)h->sp[s].dim);
            ED_HIP(hipMemset(h->sp[s].cidx.p, 0, (size_t)h->sp[s].dim));
        }
    }
    // the whole cross term as one table when its sites are few
    {
        std::vector<int> fs;
        for (int i = 0; i < ns; ++i) {
            bool any = false;
            for (int j = 0; j < ns; ++j)
                if (w[i * ns + j] != 0.0 || w[j * ns + i] != 0.0) any = true;
            if (any) fs.push_back(i);
        }
        h->fk = -1;
        if (fs.size() <= 4) {
            const int k = (int)fs.size(), nt = 1 << k;
            std::vector<double> tab((size_t)nt * nt, 0.0);
            for (int cu = 0; cu < nt; ++cu)
                for (int cd = 0; cd < nt; ++cd) {
                    double e = 0.0;
                    for (int a = 0; a < k; ++a)
                        for (int c = 0; c < k; ++c)
                            if (((cu >> a) & 1) && ((cd >> c) & 1)) e += w[fs[a] * ns + fs[c]];
                    tab[(size_t)cu * nt + cd] = e;
                }
            upload(h->ftab64, tab);
            upload(h->ftab32, std::vector<float>(tab.begin(), tab.end()));
            DevMem dsites;
            upload(dsites, fs.empty() ? std::vector<int>{0} : fs);
            for (int s = 0; s < 2; ++s) {
                SpinTab &t = h->sp[s];
                h->fcidx[s].alloc((size_t)t.dim);
                k_cidx<<<grid_for(t.dim, 256, 1 << 16), 256>>>(t.states.as<uint32_t>(), t.dim, dsites.as<int>(), k,
                                                              h->fcidx[s].as<uint8_t>());
                ED_LAUNCH_CHECK();
            }
            ED_HIP(hipDeviceSynchronize());
            std::vector<uint8_t> f8((size_t)h->sp[1].dim);
            if (!f8.empty()) ED_HIP(hipMemcpy(f8.data(), h->fcidx[1].p, f8.size(), hipMemcpyDeviceToHost));
            upload(h->dn_fc32, f8.empty() ? std::vector<uint32_t>(1, 0u) : std::vector<uint32_t>(f8.begin(), f8.end()));
            h->fk = k;
            h->fk_sites = fs;
        }
    }
}

// Four-fermion terms as products of one-spin moves (Section 4):
//   d+_{m up} d_{m dn} d+_{m' dn} d_{m' up} = -(d+_{m up} d_{m' up})(d+_{m' dn} d_{m dn})
//   d+_{m up} d+_{m dn} d_{m' up} d_{m' dn} = -(d+_{m up} d_{m' up})(d+_{m dn} d_{m' dn})
//   c+_{i up} c+_{j dn} c_{l dn} c_{k up}   = +(c+_{i up} c_{k up})(c+_{j dn} c_{l dn})
// (anticommuting the operators past each other), and an even down-spin pair
// passes the up block without a sign.  So a term with coefficient c acting on
// (u, d) gives (up: m' -> m, down: m -> m' or m' -> m) with element -c s_up s_dn,
// or (up: k -> i, down: l -> j) with element +c s_up s_dn; a move onto its own
// site (k = i or l = j) is the number operator.
static void build_xterms(ed_ham_s *h, const ed_params *p) {
    std::map<std::pair<int, int>, double> acc;  // (up move, dn move) -> amplitude
    for (int t = 0; t < p->n_x; ++t) {
        const ed_xterm &x = p->x[t];
        if (x.type == ED_UU_GENERAL || x.type == ED_DD_GENERAL) continue;  // in the one-spin tables
        if (x.type == ED_UD_GENERAL) {
            acc[{move_index(h->sp[0], x.k, x.m), move_index(h->sp[1], x.l, x.mp)}] += x.coef;
            continue;
        }
        const int um = move_index(h->sp[0], x.mp, x.m);
        const int dm = (x.type == ED_SPIN_FLIP) ? move_index(h->sp[1], x.m, x.mp) : move_index(h->sp[1], x.mp, x.m);
        acc[{um, dm}] += -x.coef;
    }
    h->xterms.clear();
    for (auto &kv : acc)
        if (kv.second != 0.0) h->xterms.push_back(XTerm{kv.first.first, kv.first.second, kv.second});
    // ordered by down move, so that a row's list runs through the down move
    // tables in order and a kernel can load each table entry once for all rows
    std::stable_sort(h->xterms.begin(), h->xterms.end(),
                     [](const XTerm &l, const XTerm &r) { return l.dn_mv < r.dn_mv; });
    h->nx = (int)h->xterms.size();
    for (int s = 0; s < 2; ++s) {
        SpinTab &t = h->sp[s];
        t.nmv = (int)t.mv_src.size();
        t.mv.alloc((size_t)std::max(t.nmv, 1) * (size_t)t.dim * sizeof(int32_t));
        for (int q = 0; q < t.nmv; ++q) {
            k_move<<<grid_for(t.dim, 256, 1 << 16), 256>>>(t.states.as<uint32_t>(), t.dim, t.ns, t.n, t.mv_src[q],
                                                          t.mv_dst[q], t.mv.as<int32_t>() + (size_t)q * t.dim,
                                                          h->grouped ? h->gipos[s].as<int32_t>() : nullptr);
            ED_LAUNCH_CHECK();
        }
    }
    // down spin: each move's validity as a test on the column word of the tile
    // kernel (source occupied, destination empty), so a kernel can skip a term
    // for columns where the move does not apply before reading its table
    {
        SpinTab &t = h->sp[1];
        std::vector<uint32_t> mb((size_t)std::max(t.nmv, 1), 0u);
        for (int q = 0; q < t.nmv; ++q) {
            int sb = t.mv_src[q], db = t.mv_dst[q];
            if (h->fk >= 0) {
                sb = db = -1;
                for (size_t i = 0; i < h->fk_sites.size(); ++i) {
                    if (h->fk_sites[i] == t.mv_src[q]) sb = (int)i;
                    if (h->fk_sites[i] == t.mv_dst[q]) db = (int)i;
                }
            }
            if (sb >= 0 && db >= 0 && sb != db) mb[q] = 1u << 31 | (uint32_t)db << 8 | (uint32_t)sb;
        }
        upload(t.mvb, mb);
    }
    // down spin: all move tables packed into one word per state when every move
    // shifts the rank by -4..3 (moves on the lowest sites): 5 bits per move,
    // valid << 4 | sign << 3 | (shift + 4)
    {
        SpinTab &t = h->sp[1];
        t.mvp_ok = false;
        if (t.nmv > 0 && t.nmv <= 6 && t.dim > 0) {
            std::vector<int32_t> mv((size_t)t.nmv * t.dim);
            ED_HIP(hipMemcpy(mv.data(), t.mv.p, mv.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
            std::vector<uint32_t> w((size_t)t.dim, 0u);
            bool ok = true;
            for (int q = 0; q < t.nmv && ok; ++q)
                for (int64_t d = 0; d < t.dim; ++d) {
                    const int32_t m = mv[(size_t)q * t.dim + d];
                    if (m < 0) continue;
                    const int64_t sh = (int64_t)(m >> 1) - d;
                    if (sh < -4 || sh > 3) { ok = false; break; }
                    w[d] |= (16u | ((uint32_t)(m & 1) << 3) | (uint32_t)(sh + 4)) << (5 * q);
                }
            if (ok) {
                upload(t.mvp, w);
                t.mvp_ok = true;
            }
        }
    }
    std::vector<XTermDev<double>> x64;
    std::vector<XTermDev<float>> x32;
    for (auto &x : h->xterms) {
        x64.push_back(XTermDev<double>{x.up_mv, x.dn_mv, x.amp});
        x32.push_back(XTermDev<float>{x.up_mv, x.dn_mv, (float)x.amp});
    }
    upload(h->xt64, x64);
    upload(h->xt32, x32);
    // per-up-state lists
    const int64_t dup = h->sp[0].dim;
    DevMem cnt, off64;
    cnt.alloc((size_t)dup * sizeof(int64_t));
    off64.alloc((size_t)(dup + 1) * sizeof(int64_t));
    k_xlist_count<<<grid_for(dup, 256, 1 << 16), 256>>>(h->sp[0].mv.as<int32_t>(), dup, h->xt64.as<XTermDev<double>>(),
                                                       h->nx, cnt.as<int64_t>());
    ED_LAUNCH_CHECK();
    k_scan_i64<<<1, 1024>>>(cnt.as<int64_t>(), off64.as<int64_t>(), dup);
    ED_LAUNCH_CHECK();
    int64_t nl = 0;
    ED_HIP(hipMemcpy(&nl, off64.as<int64_t>() + dup, sizeof(int64_t), hipMemcpyDeviceToHost));
    {
        std::vector<int64_t> hc((size_t)dup);
        ED_HIP(hipMemcpy(hc.data(), cnt.p, (size_t)dup * sizeof(int64_t), hipMemcpyDeviceToHost));
        int64_t mx = 0;
        for (int64_t v : hc) mx = std::max(mx, v);
        h->xl_max = (int)mx;
    }
    h->xl_off.alloc((size_t)(dup + 1) * sizeof(int32_t));
    h->xl_src.alloc((size_t)std::max<int64_t>(nl, 1) * sizeof(int32_t));
    h->xl_tab.alloc((size_t)std::max<int64_t>(nl, 1) * sizeof(int32_t));
    h->xl_amp64.alloc((size_t)std::max<int64_t>(nl, 1) * sizeof(double));
    h->xl_amp32.alloc((size_t)std::max<int64_t>(nl, 1) * sizeof(float));
    k_xlist_fill<<<grid_for(dup, 256, 1 << 16), 256>>>(h->sp[0].mv.as<int32_t>(), dup, h->xt64.as<XTermDev<double>>(),
                                                      h->nx, off64.as<int64_t>(), h->xl_off.as<int32_t>(),
                                                      h->xl_src.as<int32_t>(), h->xl_tab.as<int32_t>(),
                                                      h->xl_amp64.as<double>(), h->xl_amp32.as<float>());
    ED_LAUNCH_CHECK();
    ED_HIP(hipDeviceSynchronize());
}

static void validate(const ed_params *p, int ns) {
    if (!p) fail(ED_EINVAL, "ed_ham_create: params is NULL");
    if (p->Ns != ns) fail(ED_EINVAL, "ed_ham_create: params Ns=%d but basis Ns=%d", p->Ns, ns);
    if (!p->eps || !p->hop || !p->w_ud || !p->w_ss) fail(ED_EINVAL, "ed_ham_create: NULL coefficient array");
    if (p->n_x < 0 || (p->n_x > 0 && !p->x)) fail(ED_EINVAL, "ed_ham_create: bad four-fermion term list");
    const size_t n = (size_t)ns;
    if (!finite_all(p->eps, 2 * n) || !finite_all(p->hop, 2 * n * n) || !finite_all(p->w_ud, n * n) ||
        !finite_all(p->w_ss, 2 * n * n))
        fail(ED_EINVAL, "ed_ham_create: non-finite coefficient");
    for (int s = 0; s < 2; ++s) {
        const double *hs = p->hop + (size_t)s * n * n;
        const double *ws = p->w_ss + (size_t)s * n * n;
        for (int i = 0; i < ns; ++i) {
            if (hs[i * ns + i] != 0.0) fail(ED_EINVAL, "ed_ham_create: hop[%d] has a nonzero diagonal (use eps)", s);
            for (int j = 0; j < ns; ++j) {
                if (hs[i * ns + j] != hs[j * ns + i])
                    fail(ED_EINVAL, "ed_ham_create: hop[%d] is not symmetric at (%d,%d)", s, i, j);
                if (j <= i && ws[i * ns + j] != 0.0)
                    fail(ED_EINVAL, "ed_ham_create: w_ss[%d] must be zero on and below the diagonal", s);
            }
        }
    }
    std::map<std::tuple<int, int, int>, double> sum;
    std::map<std::tuple<int, int, int, int>, double> gsum;
    std::map<std::tuple<int, int, int>, double> ssum;
    for (int t = 0; t < p->n_x; ++t) {
        const ed_xterm &x = p->x[t];
        if (x.type == ED_UD_GENERAL || x.type == ED_UU_GENERAL || x.type == ED_DD_GENERAL) {
            for (int q : {x.m, x.mp, x.k, x.l})
                if (q < 0 || q >= ns) fail(ED_EINVAL, "ed_ham_create: general term index %d outside [0, Ns)", q);
            if (!std::isfinite(x.coef)) fail(ED_EINVAL, "ed_ham_create: non-finite term coefficient");
            if (x.type == ED_UD_GENERAL) {
                gsum[std::make_tuple(x.m, x.mp, x.k, x.l)] += x.coef;
                continue;
            }
            // same spin: c+_i c+_j c_l c_k, i != j, k != l, not a density term;
            // the pair orders are normalised (i < j, k < l, each swap a sign)
            if (x.m == x.mp || x.k == x.l)
                fail(ED_EINVAL, "ed_ham_create: same-spin term (%d,%d,%d,%d) repeats a mode", x.m, x.mp, x.k, x.l);
            const int i = std::min(x.m, x.mp), j = std::max(x.m, x.mp);
            const int k = std::min(x.k, x.l), l = std::max(x.k, x.l);
            if (i == k && j == l)
                fail(ED_EINVAL, "ed_ham_create: same-spin density term (%d,%d): put it in w_ss", i, j);
            const double sg = ((x.m > x.mp) != (x.k > x.l)) ? -1.0 : 1.0;
            ssum[std::make_tuple(x.type, i * 32 + j, k * 32 + l)] += sg * x.coef;
            continue;
        }
        if (x.type != ED_SPIN_FLIP && x.type != ED_PAIR_HOP) fail(ED_EINVAL, "ed_ham_create: bad term type %d", x.type);
        if (x.m < 0 || x.mp < 0 || x.m >= ns || x.mp >= ns || x.m == x.mp)
            fail(ED_EINVAL, "ed_ham_create: bad orbital pair (%d,%d)", x.m, x.mp);
        if (!std::isfinite(x.coef)) fail(ED_EINVAL, "ed_ham_create: non-finite term coefficient");
        sum[std::make_tuple(x.type, x.m, x.mp)] += x.coef;
    }
    for (auto &kv : sum) {
        auto it = sum.find(std::make_tuple(std::get<0>(kv.first), std::get<2>(kv.first), std::get<1>(kv.first)));
        const double other = it == sum.end() ? 0.0 : it->second;
        if (other != kv.second)
            fail(ED_EINVAL, "ed_ham_create: four-fermion terms are not Hermitian (type %d, %d, %d)",
                 std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first));
    }
    for (auto &kv : gsum) {
        int i, j, k, l;
        std::tie(i, j, k, l) = kv.first;
        auto it = gsum.find(std::make_tuple(k, l, i, j));
        if ((it == gsum.end() ? 0.0 : it->second) != kv.second)
            fail(ED_EINVAL, "ed_ham_create: general terms are not Hermitian at (%d, %d, %d, %d)", i, j, k, l);
    }
    for (auto &kv : ssum) {
        auto it = ssum.find(std::make_tuple(std::get<0>(kv.first), std::get<2>(kv.first), std::get<1>(kv.first)));
        if ((it == ssum.end() ? 0.0 : it->second) != kv.second)
            fail(ED_EINVAL, "ed_ham_create: same-spin general terms are not Hermitian (type %d)", std::get<0>(kv.first));
    }
}

// Connected components of one spin's move graph (the hop table, which also
// holds the same-spin two-body moves) by union-find; the grouped order lists
// the components by their lowest rank and each component's states by number
// of hops (descending), then by their occupation of the sites in `fmask` (the
// sites the four-fermion terms move this spin between), then by rank.
// Returns the number of components; perm[p] = rank at position p.
static int component_order(const SpinTab &t, uint32_t fmask, const char *env, std::vector<int32_t> &perm,
                           std::vector<int32_t> &comp_off) {
    const int64_t dim = t.dim;
    std::vector<int32_t> off((size_t)dim + 1), tgt((size_t)std::max<int64_t>(t.nnz, 1));
    ED_HIP(hipMemcpy(off.data(), t.off.p, off.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (t.nnz > 0) ED_HIP(hipMemcpy(tgt.data(), t.tgt.p, (size_t)t.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> par((size_t)dim);
    for (int64_t r = 0; r < dim; ++r) par[r] = (int32_t)r;
    auto find = [&](int32_t x) {
        while (par[x] != x) {
            par[x] = par[par[x]];
            x = par[x];
        }
        return x;
    };
    for (int64_t r = 0; r < dim; ++r)
        for (int32_t e = off[r]; e < off[r + 1]; ++e) {
            int32_t a = find((int32_t)r), c = find(tgt[e]);
            if (a == c) continue;
            if (a < c) par[c] = a;  // the root is the lowest rank of the component
            else par[a] = c;
        }
    // components in order of their root (lowest rank), states by rank
    std::vector<int32_t> root((size_t)dim), cnt((size_t)dim, 0);
    for (int64_t r = 0; r < dim; ++r) {
        root[r] = find((int32_t)r);
        ++cnt[root[r]];
    }
    std::vector<int32_t> start((size_t)dim, -1);
    comp_off.assign(1, 0);
    for (int64_t r = 0; r < dim; ++r)
        if (root[r] == r) {
            start[r] = comp_off.back();
            comp_off.push_back(comp_off.back() + cnt[r]);
        }
    perm.assign((size_t)dim, 0);
    for (int64_t r = 0; r < dim; ++r) perm[start[root[r]]++] = (int32_t)r;
    // within a component: more hops first, so that runs of consecutive
    // positions (the slices of the tile kernels' hop tables) hold states with
    // similar hop counts and little padding; then by the occupation of the
    // four-fermion sites, so that a four-fermion move, which changes only those
    // sites, maps each run of equal occupation onto a run of the partner
    // component in the same order (its gathers read consecutive addresses);
    // then by rank.  `env` = "hops" drops the occupation key, "rank" keeps
    // plain rank order inside a component.
    const bool by_rank = env && std::strcmp(env, "rank") == 0;
    if (env && std::strcmp(env, "hops") == 0) fmask = 0u;
    if (!by_rank) {
        std::vector<uint32_t> st((size_t)dim);
        if (dim > 0) ED_HIP(hipMemcpy(st.data(), t.states.p, (size_t)dim * sizeof(uint32_t), hipMemcpyDeviceToHost));
        for (size_t c = 0; c + 1 < comp_off.size(); ++c)
            std::stable_sort(perm.begin() + comp_off[c], perm.begin() + comp_off[c + 1], [&](int32_t a, int32_t b) {
                const int32_t ha = off[a + 1] - off[a], hb = off[b + 1] - off[b];
                if (ha != hb) return ha > hb;
                return (st[a] & fmask) < (st[b] & fmask);
            });
    }
    return (int)comp_off.size() - 1;
}

// The same operator in the grouped basis order (see ed_ham_s), built when a
// one-spin move graph has more than one component.
static void build_twin(ed_ham_s *h, const ed_params *p, const BasisData &b) {
    std::vector<int32_t> perm[2], coff[2];
    int nc[2];
    for (int s = 0; s < 2; ++s) {
        uint32_t fmask = 0u;
        for (size_t q = 0; q < h->sp[s].mv_src.size(); ++q)
            fmask |= (1u << h->sp[s].mv_src[q]) | (1u << h->sp[s].mv_dst[q]);
        nc[s] = component_order(h->sp[s], fmask, std::getenv("ED_GROUP_ORDER"), perm[s], coff[s]);
    }
    if (nc[0] < 2 && nc[1] < 2) return;
    ed_ham_s *g = new ed_ham_s();
    try {
        g->device = h->device;
        g->prec = h->prec;
        g->grouped = true;
        BasisData bg;
        bg.ns = b.ns;
        for (int s = 0; s < 2; ++s) {
            bg.n[s] = b.n[s];
            bg.dim[s] = b.dim[s];
            std::vector<uint32_t> st((size_t)b.dim[s]), sg((size_t)b.dim[s]);
            ED_HIP(hipMemcpy(st.data(), b.states[s].p, st.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
            std::vector<int32_t> ip((size_t)b.dim[s]);
            for (int64_t q = 0; q < b.dim[s]; ++q) {
                sg[q] = st[perm[s][q]];
                ip[perm[s][q]] = (int32_t)q;
            }
            upload(bg.states[s], sg);
            upload(g->gperm[s], perm[s]);
            upload(g->gipos[s], ip);
            g->comp_off[s] = coff[s];
        }
        build_tables(g, p, bg);
    } catch (...) {
        delete g;
        throw;
    }
    h->twin = g;
}

void build_tables(ed_ham_s *h, const ed_params *p, const BasisData &b) {
    validate(p, b.ns);
    ensure_device_binomials();
    h->ns = b.ns;
    h->nup = b.n[0];
    h->ndn = b.n[1];
    h->dup = b.dim[0];
    h->ddn = b.dim[1];
    h->D = h->dup * h->ddn;
    if (h->dup > (1ll << 30) || h->ddn > (1ll << 30)) fail(ED_EUNSUPPORTED, "one-spin dimension above 2^30");
    for (int s = 0; s < 2; ++s) build_spin(h, s, b, p);
    build_cross(h, p);
    build_xterms(h, p);
    if (h->nx > 64) fail(ED_EUNSUPPORTED, "%d distinct four-fermion terms (at most 64 supported)", h->nx);
    h->dn_states_host.resize((size_t)h->ddn);
    ED_HIP(hipMemcpy(h->dn_states_host.data(), h->sp[1].states.p, (size_t)h->ddn * sizeof(uint32_t),
                     hipMemcpyDeviceToHost));
    if (!h->grouped) build_twin(h, p, b);
}

}  // namespace ed

using namespace ed;

extern "C" ed_status ed_ham_create(const ed_params *p, ed_basis_t b, int precision, ed_ham_t *out) {
    return guard([&] {
        if (!out) fail(ED_EINVAL, "ed_ham_create: out is NULL");
        *out = nullptr;
        if (!b) fail(ED_EINVAL, "ed_ham_create: NULL basis");
        if (precision != ED_FP64 && precision != ED_FP32) fail(ED_EINVAL, "ed_ham_create: bad precision");
        DeviceGuard g(b->device);
        ed_ham_s *h = new ed_ham_s();
        try {
            h->device = b->device;
            h->prec = precision;
            build_tables(h, p, b->b);
            prepare_rayleigh(h);
            if (h->twin) prepare_rayleigh(h->twin);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

extern "C" ed_status ed_ham_dims(ed_ham_t h, int64_t *Dup, int64_t *Ddn, int64_t *D) {
    return guard([&] {
        if (!h) fail(ED_EINVAL, "ed_ham_dims: NULL handle");
        if (Dup) *Dup = h->dup;
        if (Ddn) *Ddn = h->ddn;
        if (D) *D = h->D;
    });
}

extern "C" ed_status ed_hop_table_size(ed_ham_t h, int spin, int64_t *nnz) {
    return guard([&] {
        if (!h || !nnz) fail(ED_EINVAL, "ed_hop_table_size: NULL argument");
        if (spin != 0 && spin != 1) fail(ED_EINVAL, "ed_hop_table_size: spin must be 0 or 1");
        *nnz = h->sp[spin].nnz;
    });
}

extern "C" ed_status ed_hop_table(ed_ham_t h, int spin, int64_t *off, int32_t *tgt, int8_t *sign, double *amp) {
    return guard([&] {
        if (!h || !off) fail(ED_EINVAL, "ed_hop_table: NULL argument");
        if (spin != 0 && spin != 1) fail(ED_EINVAL, "ed_hop_table: spin must be 0 or 1");
        DeviceGuard g(h->device);
        const SpinTab &t = h->sp[spin];
        std::vector<int32_t> o((size_t)t.dim + 1);
        ED_HIP(hipMemcpy(o.data(), t.off.p, o.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < o.size(); ++i) off[i] = o[i];
        if (t.nnz > 0) {
            if (tgt) ED_HIP(hipMemcpy(tgt, t.tgt.p, (size_t)t.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
            if (sign) ED_HIP(hipMemcpy(sign, t.sgn.p, (size_t)t.nnz, hipMemcpyDeviceToHost));
            if (amp) ED_HIP(hipMemcpy(amp, t.amp.p, (size_t)t.nnz * sizeof(double), hipMemcpyDeviceToHost));
        }
    });
}

extern "C" void ed_ham_free(ed_ham_t h) {
    if (!h || h->grouped) return;  // a grouped twin belongs to its rank-order handle
    try {
        DeviceGuard g(h->device);
        (void)hipDeviceSynchronize();
        delete h;
    } catch (...) {
    }
}
