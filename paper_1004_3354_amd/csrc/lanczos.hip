// Lanczos iteration for the lowest eigenpairs (Section 3: an iterative solver
// built on repeated products of H with a trial vector; for real symmetric H the
// Arnoldi process of the paper's solver reduces to Lanczos with a tridiagonal
// projected matrix).
//
// Storage: basis vector i is v_i = sigma_i * S_i with S_i stored in the
// handle's precision and sigma_i an FP64 scale, so a new vector is never
// rescaled in memory.  One step j:
//   Y = H S_j                                  (matrix-free apply)
//   a_i = <S_i, Y> over locked vectors and S_0..S_j, gamma_i = sigma_i^2 a_i
//   Y <- Y - sum_i gamma_i S_i                 (classical Gram-Schmidt)
//   repeated once more ("twice is enough"), alpha_j = sum of the two gamma_j
// reorth = 3 gives the same two projections with one read of the basis per
// step: the second pass's dots are a_i - sum_k G_ik gamma_k with G_ik =
// <S_i, S_k> (exact for the update Y - sum gamma_k S_k), and the new row of G
// comes from the same multi-dot, which reads the basis once for two
// right-hand sides (Y and S_j); one update with the summed coefficients follows.
//   beta_j = sigma_j ||Y||, sigma_{j+1} = 1 / ||Y||, S_{j+1} = Y
// All dot products and updates accumulate in FP64 with a fixed reduction
// order, so runs are bit-reproducible.  The lowest eigenpair of the j x j
// tridiagonal matrix comes from a one-workgroup multisection (Sturm counts) and
// inverse iteration; convergence is |beta_j s_j| <= tol max(|theta|, 1).
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "ed_internal.h"

namespace ed {

static constexpr int kRedBS = 256;
static constexpr int kMaxVec = 1024;  // locked + stored basis vectors per kernel
static constexpr int kIRMaxIn = 257;  // implicit restart: at most 256 basis vectors + the residual
static constexpr int kIRMaxOut = 17;  // and at most 16 kept vectors + the new residual

int reduce_blocks(int64_t n) {
    int64_t b = (n + 4095) / 4096;
    if (b < 1) b = 1;
    if (b > 2048) b = 2048;
    return (int)b;
}

// contiguous element range of block `blk` out of `nblk`
__device__ __forceinline__ void block_range(int64_t n, int nblk, int blk, int64_t &a, int64_t &b) {
    int64_t chunk = (n + nblk - 1) / nblk;
    chunk = (chunk + 63) & ~(int64_t)63;
    a = (int64_t)blk * chunk;
    b = a + chunk;
    if (a > n) a = n;
    if (b > n) b = n;
}

template <int BS>
__device__ __forceinline__ double block_sum_any(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < BS / 64; ++k) s += red[k];
    __syncthreads();
    return s;
}

// partials[v * nblk + blk] = sum over the block's range of S_v[n] * Y[n]
template <typename TX, int G>
__global__ __launch_bounds__(kRedBS) void k_multidot(const TX *const *vecs, int nvec, const TX *y, int64_t n,
                                                     double *partials) {
    __shared__ double red[kRedBS / 64];
    const int nblk = gridDim.x, blk = blockIdx.x;
    int64_t a, b;
    block_range(n, nblk, blk, a, b);
    for (int g0 = 0; g0 < nvec; g0 += G) {
        double acc[G];
#pragma unroll
        for (int i = 0; i < G; ++i) acc[i] = 0.0;
        const TX *vp[G];
#pragma unroll
        for (int i = 0; i < G; ++i) vp[i] = vecs[(g0 + i < nvec) ? g0 + i : g0];
        for (int64_t k = a + threadIdx.x; k < b; k += kRedBS) {
            const double yv = (double)y[k];
#pragma unroll
            for (int i = 0; i < G; ++i)
                if (g0 + i < nvec) acc[i] += (double)vp[i][k] * yv;
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            if (g0 + i >= nvec) break;
            const double s = block_sum_any<kRedBS>(acc[i], red);
            if (threadIdx.x == 0) partials[(int64_t)(g0 + i) * nblk + blk] = s;
        }
    }
}

// Two right-hand sides in one read of the basis:
// partials[v * nblk + blk] = sum S_v Y, partials[(nvec + v) * nblk + blk] = sum S_v Z
template <typename TX, int G>
__global__ __launch_bounds__(kRedBS) void k_multidot2(const TX *const *vecs, int nvec, const TX *y, const TX *z,
                                                      int64_t n, double *partials) {
    __shared__ double red[kRedBS / 64];
    const int nblk = gridDim.x, blk = blockIdx.x;
    int64_t a, b;
    block_range(n, nblk, blk, a, b);
    for (int g0 = 0; g0 < nvec; g0 += G) {
        double ay[G], az[G];
#pragma unroll
        for (int i = 0; i < G; ++i) ay[i] = az[i] = 0.0;
        const TX *vp[G];
#pragma unroll
        for (int i = 0; i < G; ++i) vp[i] = vecs[(g0 + i < nvec) ? g0 + i : g0];
        for (int64_t k = a + threadIdx.x; k < b; k += kRedBS) {
            const double yv = (double)y[k], zv = (double)z[k];
#pragma unroll
            for (int i = 0; i < G; ++i)
                if (g0 + i < nvec) {
                    const double sv = (double)vp[i][k];
                    ay[i] += sv * yv;
                    az[i] += sv * zv;
                }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            if (g0 + i >= nvec) break;
            const double sy = block_sum_any<kRedBS>(ay[i], red);
            const double sz = block_sum_any<kRedBS>(az[i], red);
            if (threadIdx.x == 0) {
                partials[(int64_t)(g0 + i) * nblk + blk] = sy;
                partials[(int64_t)(nvec + g0 + i) * nblk + blk] = sz;
            }
        }
    }
}

// Y[n] = post * ((assign ? 0 : Y[n]) - sum_i coef[i] S_i[n]) with post =
// sqrt(*post_sig2) (1 if NULL); optional norm partials of the stored result.
template <typename TX>
__global__ __launch_bounds__(kRedBS) void k_lincomb(const TX *const *vecs, const double *coef, int nvec, TX *y,
                                                    int64_t n, int assign, double sign, double *norm_part,
                                                    const double *post_sig2) {
    __shared__ double c[kMaxVec];
    __shared__ const TX *p[kMaxVec];
    __shared__ double red[kRedBS / 64];
    for (int i = threadIdx.x; i < nvec; i += kRedBS) {
        c[i] = sign * coef[i];
        p[i] = vecs[i];
    }
    __syncthreads();
    int64_t a, b;
    block_range(n, gridDim.x, blockIdx.x, a, b);
    const double post = post_sig2 ? sqrt(*post_sig2) : 1.0;
    double nrm = 0.0;
    for (int64_t k = a + threadIdx.x; k < b; k += kRedBS) {
        double v = assign ? 0.0 : (double)y[k];
        for (int i = 0; i < nvec; ++i) v -= c[i] * (double)p[i][k];
        const TX st = (TX)(post * v);
        y[k] = st;
        nrm += (double)st * (double)st;
    }
    if (norm_part) {
        const double s = block_sum_any<kRedBS>(nrm, red);
        if (threadIdx.x == 0) norm_part[blockIdx.x] = s;
    }
}

// Vector forms of the three kernels above for the single-sector solver: each
// thread takes four consecutive elements per iteration (one 16-byte load per
// FP32 vector, two per FP64 vector) and keeps G vectors' loads in flight.
// Block ranges start at multiples of 64 elements and slots are 256-byte
// aligned, so every group of four inside a block is aligned; a block's ragged
// end is done element by element.  Same partial layout and fixed reduction
// order per block as the scalar forms.
// (vectors declared with element alignment only: a locked vector inside a
// caller's [k][D] array starts at a multiple of D elements, and gfx950 global
// memory accepts 16-byte accesses at element alignment)
typedef float f4e __attribute__((ext_vector_type(4), aligned(4)));
typedef double d2e __attribute__((ext_vector_type(2), aligned(8)));
template <typename TX>
struct Q4 {
    TX v[4];
};
template <typename TX>
__device__ __forceinline__ Q4<TX> load4(const TX *p) {
    Q4<TX> q;
    if constexpr (sizeof(TX) == 4) {
        const f4e t = *reinterpret_cast<const f4e *>(p);
        q.v[0] = t.x; q.v[1] = t.y; q.v[2] = t.z; q.v[3] = t.w;
    } else {
        const d2e a = *reinterpret_cast<const d2e *>(p), b = *reinterpret_cast<const d2e *>(p + 2);
        q.v[0] = a.x; q.v[1] = a.y; q.v[2] = b.x; q.v[3] = b.y;
    }
    return q;
}
template <typename TX>
__device__ __forceinline__ void store4(TX *p, const Q4<TX> &q) {
    if constexpr (sizeof(TX) == 4) {
        f4e t;
        t.x = q.v[0]; t.y = q.v[1]; t.z = q.v[2]; t.w = q.v[3];
        *reinterpret_cast<f4e *>(p) = t;
    } else {
        d2e a, b;
        a.x = q.v[0]; a.y = q.v[1]; b.x = q.v[2]; b.y = q.v[3];
        *reinterpret_cast<d2e *>(p) = a;
        *reinterpret_cast<d2e *>(p + 2) = b;
    }
}

// partials[v * nblk + blk] = sum S_v Y (and with Z, when z != NULL, at
// partials[(nvec + v) * nblk + blk])
template <typename TX, int G, bool TWO>
__global__ __launch_bounds__(kRedBS) void k_multidot_v4(const TX *const *vecs, int nvec, const TX *y, const TX *z,
                                                        int64_t n, double *partials) {
    __shared__ double red[kRedBS / 64];
    const int nblk = gridDim.x, blk = blockIdx.x;
    int64_t a, b;
    block_range(n, nblk, blk, a, b);
    for (int g0 = 0; g0 < nvec; g0 += G) {
        double ay[G], az[G];
#pragma unroll
        for (int i = 0; i < G; ++i) ay[i] = az[i] = 0.0;
        const TX *vp[G];
#pragma unroll
        for (int i = 0; i < G; ++i) vp[i] = vecs[(g0 + i < nvec) ? g0 + i : g0];
        int64_t k = a + 4 * (int64_t)threadIdx.x;
        for (; k + 4 <= b; k += 4 * kRedBS) {
            const Q4<TX> yv = load4(y + k);
            Q4<TX> zv;
            if constexpr (TWO) zv = load4(z + k);
            Q4<TX> sv[G];
#pragma unroll
            for (int i = 0; i < G; ++i)
                if (g0 + i < nvec) sv[i] = load4(vp[i] + k);
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (g0 + i >= nvec) break;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ay[i] += (double)sv[i].v[e] * (double)yv.v[e];
                    if constexpr (TWO) az[i] += (double)sv[i].v[e] * (double)zv.v[e];
                }
            }
        }
        for (int64_t e = k; e < b && e < k + 4; ++e) {  // ragged end of the block
#pragma unroll
            for (int i = 0; i < G; ++i) {
                if (g0 + i >= nvec) break;
                ay[i] += (double)vp[i][e] * (double)y[e];
                if constexpr (TWO) az[i] += (double)vp[i][e] * (double)z[e];
            }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            if (g0 + i >= nvec) break;
            const double sy = block_sum_any<kRedBS>(ay[i], red);
            if (threadIdx.x == 0) partials[(int64_t)(g0 + i) * nblk + blk] = sy;
            if constexpr (TWO) {
                const double sz = block_sum_any<kRedBS>(az[i], red);
                if (threadIdx.x == 0) partials[(int64_t)(nvec + g0 + i) * nblk + blk] = sz;
            }
        }
    }
}

// Y = post * ((assign ? 0 : Y) - sum_i coef[i] S_i) as k_lincomb, four
// elements per thread, four vectors' loads in flight.
template <typename TX>
__global__ __launch_bounds__(kRedBS) void k_lincomb_v4(const TX *const *vecs, const double *coef, int nvec, TX *y,
                                                       int64_t n, int assign, double sign, double *norm_part,
                                                       const double *post_sig2) {
    __shared__ double c[kMaxVec];
    __shared__ const TX *p[kMaxVec];
    __shared__ double red[kRedBS / 64];
    for (int i = threadIdx.x; i < nvec; i += kRedBS) {
        c[i] = sign * coef[i];
        p[i] = vecs[i];
    }
    __syncthreads();
    int64_t a, b;
    block_range(n, gridDim.x, blockIdx.x, a, b);
    const double post = post_sig2 ? sqrt(*post_sig2) : 1.0;
    double nrm = 0.0;
    int64_t k = a + 4 * (int64_t)threadIdx.x;
    for (; k + 4 <= b; k += 4 * kRedBS) {
        double v[4];
        if (assign) {
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = 0.0;
        } else {
            const Q4<TX> q = load4(y + k);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = (double)q.v[e];
        }
        int i = 0;
        for (; i + 4 <= nvec; i += 4) {
            Q4<TX> s4[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) s4[t] = load4(p[i + t] + k);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] -= c[i + t] * (double)s4[t].v[e];
        }
        for (; i < nvec; ++i) {
            const Q4<TX> q = load4(p[i] + k);
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] -= c[i] * (double)q.v[e];
        }
        Q4<TX> o;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            o.v[e] = (TX)(post * v[e]);
            nrm += (double)o.v[e] * (double)o.v[e];
        }
        store4(y + k, o);
    }
    for (int64_t e = k; e < b && e < k + 4; ++e) {
        double v = assign ? 0.0 : (double)y[e];
        for (int i = 0; i < nvec; ++i) v -= c[i] * (double)p[i][e];
        const TX st = (TX)(post * v);
        y[e] = st;
        nrm += (double)st * (double)st;
    }
    if (norm_part) {
        const double sm = block_sum_any<kRedBS>(nrm, red);
        if (threadIdx.x == 0) norm_part[blockIdx.x] = sm;
    }
}

// Implicit restart, in place: out_o[n] = sum_i C[i * nout + o] in_i[n] for
// o < nout, where out_o is the storage of in_o (each element's inputs are read
// by the thread that writes its outputs, before it writes them).  Four
// consecutive elements per thread, two inputs' loads in flight, FP64
// accumulation; NO >= nout is the compile-time output count (coefficients
// padded with zeros, so the inner loop has no branches).  Norm partials of the
// last output (the new residual).
template <typename TX, int NO>
__global__ __launch_bounds__(kRedBS) void k_restart_combine_v4(const TX *const *vin, const double *C, int nin,
                                                               int nout, int64_t n, double *norm_part) {
    __shared__ double c[kIRMaxIn * NO];
    __shared__ const TX *pin[kIRMaxIn];
    __shared__ double red[kRedBS / 64];
    for (int i = threadIdx.x; i < nin * NO; i += kRedBS) {
        const int r = i / NO, o = i - r * NO;
        c[i] = o < nout ? C[r * nout + o] : 0.0;
    }
    for (int i = threadIdx.x; i < nin; i += kRedBS) pin[i] = vin[i];
    __syncthreads();
    int64_t a, b;
    block_range(n, gridDim.x, blockIdx.x, a, b);
    double nrm = 0.0;
    int64_t k = a + 4 * (int64_t)threadIdx.x;
    for (; k + 4 <= b; k += 4 * kRedBS) {
        double acc[NO][4];
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[o][e] = 0.0;
        int i = 0;
        for (; i + 2 <= nin; i += 2) {
            const Q4<TX> v0 = load4(pin[i] + k), v1 = load4(pin[i + 1] + k);
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                const double c0 = c[i * NO + o], c1 = c[(i + 1) * NO + o];
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[o][e] += c0 * (double)v0.v[e] + c1 * (double)v1.v[e];
            }
        }
        if (i < nin) {
            const Q4<TX> v0 = load4(pin[i] + k);
#pragma unroll
            for (int o = 0; o < NO; ++o)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[o][e] += c[i * NO + o] * (double)v0.v[e];
        }
#pragma unroll
        for (int o = 0; o < NO; ++o)
            if (o < nout) {
                Q4<TX> q;
#pragma unroll
                for (int e = 0; e < 4; ++e) q.v[e] = (TX)acc[o][e];
                store4(const_cast<TX *>(pin[o]) + k, q);
                if (o == nout - 1)
#pragma unroll
                    for (int e = 0; e < 4; ++e) nrm += (double)q.v[e] * (double)q.v[e];
            }
    }
    for (int64_t e = k; e < b && e < k + 4; ++e) {  // ragged end of the block
        double acc[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) acc[o] = 0.0;
        for (int i = 0; i < nin; ++i) {
            const double v = (double)pin[i][e];
#pragma unroll
            for (int o = 0; o < NO; ++o) acc[o] += c[i * NO + o] * v;
        }
#pragma unroll
        for (int o = 0; o < NO; ++o)
            if (o < nout) {
                const TX st = (TX)acc[o];
                const_cast<TX *>(pin[o])[e] = st;
                if (o == nout - 1) nrm += (double)st * (double)st;
            }
    }
    const double sm = block_sum_any<kRedBS>(nrm, red);
    if (threadIdx.x == 0) norm_part[blockIdx.x] = sm;
}

template <typename TX>
static void launch_restart_combine(const TX *const *vin, const double *C, int nin, int nout, int64_t n,
                                   double *norm_part, int nblk, hipStream_t s) {
    if (nout <= 2) k_restart_combine_v4<TX, 2><<<nblk, kRedBS, 0, s>>>(vin, C, nin, nout, n, norm_part);
    else if (nout <= 3) k_restart_combine_v4<TX, 3><<<nblk, kRedBS, 0, s>>>(vin, C, nin, nout, n, norm_part);
    else if (nout <= 5) k_restart_combine_v4<TX, 5><<<nblk, kRedBS, 0, s>>>(vin, C, nin, nout, n, norm_part);
    else if (nout <= 9) k_restart_combine_v4<TX, 9><<<nblk, kRedBS, 0, s>>>(vin, C, nin, nout, n, norm_part);
    else k_restart_combine_v4<TX, kIRMaxOut><<<nblk, kRedBS, 0, s>>>(vin, C, nin, nout, n, norm_part);
}

__global__ void k_scale(void *y, int64_t n, double f, int is_f32) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        if (is_f32) {
            float *p = (float *)y;
            p[k] = (float)((double)p[k] * f);
        } else {
            double *p = (double *)y;
            p[k] = p[k] * f;
        }
    }
}

// Fixed-order sum of p[0..n), n <= 8 * 256, by one workgroup of 256: thread
// t adds p[t], p[t + 256], ... in that order (all its loads issued at once),
// then a shared-memory tree.  The result is valid in thread 0.
__device__ __forceinline__ double wg_sum_fixed(const double *p, int n, double *sh) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int i = (int)threadIdx.x + 256 * q;
        v[q] = i < n ? p[i] : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += v[q];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

// One workgroup per vector v (grid = nvec): raw[v] = sum of the v-th row of
// partials, gamma[v] = sig2[v] raw[v]; the workgroup of v = jidx adds
// gamma[jidx] to *alpha.
__global__ __launch_bounds__(256) void k_finalize_dots_par(const double *partials, int nblk, const double *sig2,
                                                          double *raw, double *gamma, double *alpha, int jidx) {
    __shared__ double sh[256];
    const int v = blockIdx.x;
    const double s = wg_sum_fixed(partials + (int64_t)v * nblk, nblk, sh);
    if (threadIdx.x == 0) {
        if (raw) raw[v] = s;
        const double g = (sig2 ? sig2[v] : 1.0) * s;
        if (gamma) gamma[v] = g;
        if (alpha && gamma && v == jidx) *alpha += g;
    }
}

// Row sums of the two-sided multi-dot (grid = 2 nvec): out[v] = sum of row v.
__global__ __launch_bounds__(256) void k_rowsums(const double *partials, int nblk, double *out) {
    __shared__ double sh[256];
    const double s = wg_sum_fixed(partials + (int64_t)blockIdx.x * nblk, nblk, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// The coefficients of both projections from the row sums (reorth = 3): as
// k_finalize_gram, with a[0..nvec) = <S_i, Y> and g = a[nvec..2 nvec) =
// <S_i, S_jr> already summed.  One workgroup.
__global__ __launch_bounds__(256) void k_gram_coef(const double *sums, int nvec, const double *sig2, double *gram,
                                                  int ld, double *gamma, double *alpha) {
    __shared__ double g1[kMaxVec];
    const int jr = nvec - 1;
    for (int i = threadIdx.x; i < nvec; i += 256) {
        g1[i] = sig2[i] * sums[i];
        gram[(int64_t)jr * ld + i] = sums[nvec + i];
        gram[(int64_t)i * ld + jr] = sums[nvec + i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nvec; i += 256) {
        double t = 0.0;
        for (int k = 0; k < nvec; ++k) t += gram[(int64_t)i * ld + k] * g1[k];
        gamma[i] = g1[i] + sig2[i] * (sums[i] - t);
    }
    __syncthreads();
    if (threadIdx.x == 0 && alpha) *alpha += gamma[jr];
}

// Fixed-order sum of partials[v*nblk + 0..nblk) for each v; gamma[v] =
// sig2[v] * sum.  If alpha != NULL, *alpha += gamma[jidx].
__global__ void k_finalize_dots(const double *partials, int nvec, int nblk, const double *sig2, double *raw,
                                double *gamma, double *alpha, int jidx) {
    __shared__ double sh[256];
    for (int v = 0; v < nvec; ++v) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nblk; i += 256) s += partials[(int64_t)v * nblk + i];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (raw) raw[v] = sh[0];
            if (gamma) gamma[v] = (sig2 ? sig2[v] : 1.0) * sh[0];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && alpha && gamma) *alpha += gamma[jidx];
}

// Coefficients of both projections from one two-sided multi-dot (reorth = 3).
// a_i = <S_i, Y>, g_i = <S_i, S_jr> (jr = nvec - 1, the newest vector): row jr
// of the Gram matrix G (ld x ld) is set from g, then gamma1_i = sig2_i a_i,
// a2_i = a_i - sum_k G_ik gamma1_k, gamma_i = gamma1_i + sig2_i a2_i, and
// *alpha += gamma_jr.  Fixed-order sums; one workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_finalize_gram(const double *partials, int nvec, int nblk,
                                                       const double *sig2, double *gram, int ld, double *gamma,
                                                       double *alpha) {
    __shared__ double sh[256];
    __shared__ double av[kMaxVec], g1[kMaxVec];
    const int jr = nvec - 1;
    for (int v = 0; v < 2 * nvec; ++v) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nblk; i += 256) s += partials[(int64_t)v * nblk + i];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (v < nvec) {
                av[v] = sh[0];
                g1[v] = sig2[v] * sh[0];
            } else {
                const int i = v - nvec;
                gram[(int64_t)jr * ld + i] = sh[0];
                gram[(int64_t)i * ld + jr] = sh[0];
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < nvec; i += 256) {
        double t = 0.0;
        for (int k = 0; k < nvec; ++k) t += gram[(int64_t)i * ld + k] * g1[k];
        gamma[i] = g1[i] + sig2[i] * (av[i] - t);
    }
    __syncthreads();
    if (threadIdx.x == 0 && alpha) *alpha += gamma[jr];
}

// After the last update of step j the stored Y is w'' = sigma_j (Y - ...):
// n2 = ||w''||^2 -> beta[j] = sqrt(n2), sig2[j+1] = 1/n2 (0 on exact breakdown).
__global__ void k_finalize_norm(const double *partials, int nblk, double *sig2, double *beta, int jidx, int j) {
    __shared__ double sh[256];
    const double n2s = wg_sum_fixed(partials, nblk, sh);
    if (threadIdx.x == 0) {
        const double n2 = n2s;
        beta[j] = sqrt(n2);
        sig2[jidx + 1] = n2 > 0.0 ? 1.0 / n2 : 0.0;
    }
}

__device__ int sturm_count(const double *al, const double *be, int m, double x, double pivmin) {
    int c = 0;
    double q = al[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
    for (int i = 1; i < m; ++i) {
        q = (al[i] - x) - be[i - 1] * be[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++c;
    }
    return c;
}

// Lowest eigenpair of the m x m symmetric tridiagonal (alpha, beta) matrix,
// m <= kTriMax.  out[0] = theta, out[1] = |beta_last s_{m-1}|, out[2] =
// beta_last, out[3 .. 3+m) = normalised eigenvector.  One workgroup of 256
// threads: 256-point multisection on the Sturm count (the first point whose
// count reaches 1 found by an LDS minimum), then thread 0 does inverse
// iteration on T - theta I with one LU factorisation (partial pivoting) and
// three solves; the running values of each recurrence stay in registers and
// the factors in LDS.  `work` is unused (kept for the callers' layout).
static constexpr int kTriMax = 1024;
__device__ void k_tridiag_lowest_body(const double *alpha, const double *beta, int m, double *out,
                                      double *work) {
    (void)work;
    __shared__ double al[kTriMax], be[kTriMax];
    __shared__ double fd[kTriMax], fl[kTriMax], fu[kTriMax], fu2[kTriMax], z[kTriMax];
    __shared__ unsigned char piv[kTriMax];
    __shared__ int first;
    __shared__ double lo, hi, pivs;
    const int t = threadIdx.x;
    for (int i = t; i < m; i += 256) {
        al[i] = alpha[i];
        be[i] = (i < m - 1) ? beta[i] : 0.0;
    }
    __syncthreads();
    if (t == 0) {
        double l = 1e300, h = -1e300, bmax = 0.0;
        for (int i = 0; i < m; ++i) {
            const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i < m - 1 ? fabs(be[i]) : 0.0);
            l = fmin(l, al[i] - r);
            h = fmax(h, al[i] + r);
            bmax = fmax(bmax, fabs(be[i]));
        }
        const double w = 1e-12 * fmax(fmax(fabs(l), fabs(h)), 1.0);
        lo = l - w;
        hi = h + w;
        pivs = fmax(1e-290, 1e-300 * bmax * bmax);
    }
    __syncthreads();
    const double pivmin = pivs;
    for (int it = 0; it < 60; ++it) {
        const double L = lo, H = hi;
        const double x = L + (H - L) * (double)(t + 1) / 257.0;
        const int c = sturm_count(al, be, m, x, pivmin);
        if (t == 0) first = 256;
        __syncthreads();
        if (c >= 1) atomicMin(&first, t);
        __syncthreads();
        if (t == 0) {
            const int f = first;
            double nl, nh;
            if (f == 256) {
                nl = L + (H - L) * 256.0 / 257.0;
                nh = H;
            } else {
                nh = L + (H - L) * (double)(f + 1) / 257.0;
                nl = (f > 0) ? L + (H - L) * (double)f / 257.0 : L;
            }
            lo = nl;
            hi = nh;
        }
        __syncthreads();
        if (hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + 1e-300) break;
    }
    if (t != 0) return;
    const double theta = 0.5 * (lo + hi);
    const double tiny = 1e-300 + 2.220446049250313e-16 * fmax(fabs(theta), 1.0) * 1e-3;
    // T - theta I = P L U: row i of U is (fd[i], fu[i], fu2[i]); fl[i] the multiplier
    {
        double cd = al[0] - theta, cdu = m > 1 ? be[0] : 0.0;
        for (int i = 0; i < m - 1; ++i) {
            const double sub = be[i];
            double nd = al[i + 1] - theta;
            double ndu = (i + 1 < m - 1) ? be[i + 1] : 0.0;
            double f;
            if (fabs(cd) >= fabs(sub)) {
                if (cd == 0.0) cd = tiny;
                f = sub / cd;
                fd[i] = cd;
                fu[i] = cdu;
                fu2[i] = 0.0;
                nd -= f * cdu;
                piv[i] = 0;
            } else {  // rows i and i + 1 swapped
                f = cd / sub;
                fd[i] = sub;
                fu[i] = nd;
                fu2[i] = (i < m - 2) ? ndu : 0.0;
                nd = cdu - f * nd;
                if (i < m - 2) ndu = -f * ndu;
                piv[i] = 1;
            }
            fl[i] = f;
            cd = nd;
            cdu = ndu;
        }
        if (cd == 0.0) cd = tiny;
        fd[m - 1] = cd;
    }
    for (int i = 0; i < m; ++i) z[i] = 1.0;
    for (int rep = 0; rep < 3; ++rep) {
        // z <- L^-1 P z
        double zc = z[0];
        for (int i = 0; i < m - 1; ++i) {
            double zn = z[i + 1];
            if (!piv[i]) {
                zn -= fl[i] * zc;
                z[i] = zc;
            } else {
                z[i] = zn;
                zn = zc - fl[i] * zn;
            }
            zc = zn;
        }
        z[m - 1] = zc;
        // z <- U^-1 z
        double z1 = z[m - 1] / fd[m - 1], z2 = 0.0;
        z[m - 1] = z1;
        for (int i = m - 2; i >= 0; --i) {
            const double v = (z[i] - fu[i] * z1 - fu2[i] * z2) / fd[i];
            z[i] = v;
            z2 = z1;
            z1 = v;
        }
        double mx = 0.0;
        for (int i = 0; i < m; ++i) mx = fmax(mx, fabs(z[i]));
        if (!(mx > 0.0) || !isfinite(mx)) {
            for (int i = 0; i < m; ++i) z[i] = 1.0;
            mx = 1.0;
        }
        double nn = 0.0;
        for (int i = 0; i < m; ++i) {
            const double v = z[i] / mx;
            z[i] = v;
            nn += v * v;
        }
        nn = sqrt(nn);
        for (int i = 0; i < m; ++i) z[i] /= nn;
    }
    const double sg = z[0] < 0.0 ? -1.0 : 1.0;
    const double bl = beta[m - 1];
    out[0] = theta;
    out[1] = fabs(bl * z[m - 1]);
    out[2] = bl;
    for (int i = 0; i < m; ++i) out[3 + i] = sg * z[i];
}

__global__ __launch_bounds__(256) void k_tridiag_lowest(const double *alpha, const double *beta, int m,
                                                        double unused, double *out, double *work) {
    k_tridiag_lowest_body(alpha, beta, m, out, work);
}

// coef[i] = s_i * sigma_i for the Ritz combination psi = sum_i s_i v_i
__global__ void k_ritz_coef(const double *s, const double *sig2, int m, double *coef) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) coef[i] = s[i] * sqrt(sig2[i]);
}

__global__ void k_set_sig2(double *sig2, int idx, const double *raw) {
    if (threadIdx.x == 0) sig2[idx] = raw[0] > 0.0 ? 1.0 / raw[0] : 0.0;
}

__global__ void k_zero(double *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

// ------------------------------------------------------------- workspace --
struct Carve {
    char *base;
    size_t off = 0, cap;
    void *take(size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        void *p = base ? base + off : nullptr;
        off += bytes;
        return p;
    }
};

struct Work {
    int m = 0, kmax = 0, nblk = 0;
    size_t elem = 0;
    std::vector<void *> slots;   // m + 1 basis slots
    std::vector<void *> locked;  // kmax locked-vector slots (may point into evecs)
    const void **vp = nullptr;   // device array of vector pointers [kmax + m + 1]
    double *sig2 = nullptr, *gamma = nullptr, *raw = nullptr, *alpha = nullptr, *beta = nullptr;
    double *partials = nullptr, *tri = nullptr, *triwork = nullptr, *coef = nullptr;
    double *gram = nullptr;      // (m+1) x (m+1) Gram matrix of the stored vectors (reorth = 3)
    double *rcoef = nullptr;     // implicit-restart combination coefficients
};

// ------------------------------------------------------- implicit restart --
// Host side of the implicitly restarted Lanczos method (Sorensen's exact-shift
// restart, as in ARPACK): T (m x m tridiagonal: alpha, beta[0..m-2]) gets the
// m - k largest of its eigenvalues applied as shifts, each by one QR step
// T - mu I = Q R, T <- R Q + mu I = Q^T T Q, with Q accumulated.  The leading
// k x k block of the result is again tridiagonal, and the new basis is
// V Q[:, 0..k), the new residual V Q[:, k] T+[k, k-1] + f Q[m-1, k-1].

// number of eigenvalues of the tridiagonal (a, b) below x (Sturm sequence)
static int sturm_count(const std::vector<double> &a, const std::vector<double> &b, int m, double x) {
    int cnt = 0;
    double d = a[0] - x;
    if (d < 0) ++cnt;
    for (int i = 1; i < m; ++i) {
        const double dd = (d == 0.0) ? 1e-300 : d;
        d = a[i] - x - b[i - 1] * b[i - 1] / dd;
        if (d < 0) ++cnt;
    }
    return cnt;
}

// eigenvalue number idx (ascending) of the tridiagonal, by bisection
static double tridiag_eig(const std::vector<double> &a, const std::vector<double> &b, int m, int idx) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b, m, mid) > idx) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Last component of the normalised eigenvector of the tridiagonal (a, b) for
// the eigenvalue theta, by inverse iteration with partial pivoting (three
// solves of (T - theta I) z = z from z = 1).
static double tridiag_evec_last(const std::vector<double> &a, const std::vector<double> &b, int m, double theta) {
    if (m == 1) return 1.0;
    std::vector<double> z((size_t)m, 1.0), d((size_t)m), dl((size_t)m), du((size_t)m), du2((size_t)m);
    std::vector<int> piv((size_t)m);
    const double tiny = 1e-300 + 2.220446049250313e-16 * std::max(std::fabs(theta), 1.0) * 1e-3;
    for (int rep = 0; rep < 3; ++rep) {
        for (int i = 0; i < m; ++i) {
            d[i] = a[i] - theta;
            dl[i] = du[i] = (i < m - 1) ? b[i] : 0.0;
            du2[i] = 0.0;
        }
        for (int i = 0; i < m - 1; ++i) {
            if (std::fabs(d[i]) >= std::fabs(dl[i])) {
                if (d[i] == 0.0) d[i] = tiny;
                const double f = dl[i] / d[i];
                dl[i] = f;
                d[i + 1] -= f * du[i];
                piv[i] = 0;
            } else {
                const double f = d[i] / dl[i];
                d[i] = dl[i];
                dl[i] = f;
                const double t = du[i];
                du[i] = d[i + 1];
                d[i + 1] = t - f * d[i + 1];
                if (i < m - 2) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -f * du[i + 1];
                }
                piv[i] = 1;
            }
        }
        if (d[m - 1] == 0.0) d[m - 1] = tiny;
        for (int i = 0; i < m - 1; ++i) {
            if (piv[i] == 0) {
                z[i + 1] -= dl[i] * z[i];
            } else {
                const double t = z[i];
                z[i] = z[i + 1];
                z[i + 1] = t - dl[i] * z[i];
            }
        }
        z[m - 1] /= d[m - 1];
        z[m - 2] = (z[m - 2] - du[m - 2] * z[m - 1]) / d[m - 2];
        for (int i = m - 3; i >= 0; --i) z[i] = (z[i] - du[i] * z[i + 1] - du2[i] * z[i + 2]) / d[i];
        double nn = 0.0;
        for (int i = 0; i < m; ++i) nn += z[i] * z[i];
        nn = std::sqrt(nn);
        if (!(nn > 0.0) || !std::isfinite(nn)) return std::nan("");
        for (int i = 0; i < m; ++i) z[i] /= nn;
    }
    return z[m - 1];
}

// Shifted QR steps on the dense copy of T; returns T+ (dense) and Q (m x m,
// row-major).  Rotation G_i acts on coordinates (i, i+1).
static void ir_shift(std::vector<double> &T, std::vector<double> &Q, int m, const std::vector<double> &shifts) {
    auto at = [m](std::vector<double> &M, int r, int c) -> double & { return M[(size_t)r * m + c]; };
    std::vector<double> M((size_t)m * m), cs((size_t)m), sn((size_t)m);
    for (double mu : shifts) {
        M = T;
        for (int i = 0; i < m; ++i) at(M, i, i) -= mu;
        for (int i = 0; i + 1 < m; ++i) {  // QR of T - mu I: zero M[i+1][i]
            const double x = at(M, i, i), z = at(M, i + 1, i);
            const double r = std::hypot(x, z);
            const double c = r > 0 ? x / r : 1.0, sv = r > 0 ? z / r : 0.0;
            cs[i] = c;
            sn[i] = sv;
            for (int k = 0; k < m; ++k) {
                const double p = at(M, i, k), q = at(M, i + 1, k);
                at(M, i, k) = c * p + sv * q;
                at(M, i + 1, k) = -sv * p + c * q;
            }
        }
        for (int i = 0; i + 1 < m; ++i) {  // T <- G_i^T T G_i, Q <- Q G_i
            const double c = cs[i], sv = sn[i];
            for (int k = 0; k < m; ++k) {
                const double p = at(T, i, k), q = at(T, i + 1, k);
                at(T, i, k) = c * p + sv * q;
                at(T, i + 1, k) = -sv * p + c * q;
            }
            for (int k = 0; k < m; ++k) {
                const double p = at(T, k, i), q = at(T, k, i + 1);
                at(T, k, i) = c * p + sv * q;
                at(T, k, i + 1) = -sv * p + c * q;
                const double pq = at(Q, k, i), qq = at(Q, k, i + 1);
                at(Q, k, i) = c * pq + sv * qq;
                at(Q, k, i + 1) = -sv * pq + c * qq;
            }
        }
    }
}

// Coefficients of the exact-shift implicit restart of a full cycle of m
// stored steps keeping k vectors.  al[0..m), be[0..m) (be[m-1] is the norm of
// the residual) and sg[0..m] (1 / ||S_i||^2 of the stored vectors S_0..S_m).
// C ((m+1) x (k+1), row-major): the kept vectors u_o = sum_l C[l][o] S_l
// (o < k, orthonormal) and the new residual f = sum_l C[l][k] S_l; a2[0..k),
// b2[0..k-1) the new leading tridiagonal block; ev the m Ritz values, ascending.
// false when the restart does not apply (non-finite data, or the kept block no
// longer holds the lowest Ritz value); the caller then restarts explicitly.
static bool ir_plan(const std::vector<double> &al, const std::vector<double> &be, const std::vector<double> &sg,
                    int m, int k, std::vector<double> &C, std::vector<double> &a2, std::vector<double> &b2,
                    std::vector<double> &ev) {
    for (int i = 0; i < m; ++i)
        if (!std::isfinite(al[i]) || !std::isfinite(be[i]) || !(sg[i] > 0.0)) return false;
    if (!(sg[m] > 0.0)) return false;
    ev.assign((size_t)m, 0.0);
    std::vector<double> shifts;
    for (int i = 0; i < m; ++i) ev[i] = tridiag_eig(al, be, m, i);
    for (int i = k; i < m; ++i) shifts.push_back(ev[i]);
    std::vector<double> T((size_t)m * m, 0.0), Q((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) {
        T[(size_t)i * m + i] = al[i];
        Q[(size_t)i * m + i] = 1.0;
        if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = be[i];
    }
    ir_shift(T, Q, m, shifts);
    a2.assign((size_t)k, 0.0);
    b2.assign((size_t)std::max(k, 1), 0.0);
    for (int i = 0; i < k; ++i) {
        a2[i] = T[(size_t)i * m + i];
        if (i + 1 < k) b2[i] = 0.5 * (T[(size_t)(i + 1) * m + i] + T[(size_t)i * m + i + 1]);
    }
    const double t0 = tridiag_eig(a2, b2, k, 0);
    if (!(std::fabs(t0 - ev[0]) <= 1e-8 * std::max(1.0, std::fabs(ev[0])))) return false;
    // inputs S_0..S_m, outputs u_0..u_{k-1} and the new residual f
    const int nin = m + 1, nout = k + 1;
    const double tk = T[(size_t)k * m + (k - 1)];
    C.assign((size_t)nin * nout, 0.0);
    for (int l = 0; l < m; ++l) {
        const double sl = std::sqrt(sg[l]);
        for (int o = 0; o < k; ++o) C[(size_t)l * nout + o] = Q[(size_t)l * m + o] * sl;
        C[(size_t)l * nout + k] = Q[(size_t)l * m + k] * sl * tk;
    }
    C[(size_t)m * nout + k] = be[m - 1] * std::sqrt(sg[m]) * Q[(size_t)(m - 1) * m + (k - 1)];
    return true;
}

static constexpr int kAutoBasisMax = 120;  // largest planned basis (max_basis = 0)

static void fill_defaults(ed_lanczos_opts &o) {
    o.max_iter = 600;
    o.max_basis = 0;
    o.tol = 1e-10;
    o.reorth = 2;
    o.check_every = 4;
    o.refine = 1;
    o.keep = 0;
    o.layout = 0;
}

static ed_lanczos_opts effective(const ed_lanczos_opts *opts, int64_t D) {
    ed_lanczos_opts o;
    fill_defaults(o);
    if (opts) o = *opts;
    if (o.max_iter <= 0) o.max_iter = 600;
    if (o.layout != 1) o.layout = 0;
    if (o.max_basis < 0) o.max_basis = 0;      // 0: planned from the memory available
    if (o.max_basis == 1) o.max_basis = 2;
    if (o.max_basis > 1000) o.max_basis = 1000;
    if ((int64_t)o.max_basis > D) o.max_basis = (int)std::max<int64_t>(D, 1);
    if (!(o.tol > 0.0)) o.tol = 1e-10;
    if (o.reorth < 0 || o.reorth > 3) o.reorth = 2;
    if (o.check_every <= 0) o.check_every = 4;
    if (o.keep < 0 || o.max_basis > kIRMaxIn - 1) o.keep = 0;
    if (o.keep > kIRMaxOut - 1) o.keep = kIRMaxOut - 1;
    if (o.max_basis > 0 && o.keep >= o.max_basis) o.keep = o.max_basis - 1;
    return o;
}

// Lay out the workspace; with base == nullptr only the size is computed.
// nslots: basis slots of D elements (m + 1, or 3 for the three-term
// recurrence of ed_lanczos_tridiag, which only ever holds S_{j-1}, S_j, S_{j+1}).
static size_t layout(Work &w, char *base, int64_t D, size_t elem, int m, int kmax, bool locked_in_ws,
                     int nslots = -1) {
    Carve c{base, 0, 0};
    w.m = m;
    w.kmax = kmax;
    w.elem = elem;
    w.nblk = reduce_blocks(D);
    if (nslots < 0) nslots = m + 1;
    w.slots.assign(nslots, nullptr);
    for (int i = 0; i < nslots; ++i) w.slots[i] = c.take((size_t)D * elem);
    w.locked.assign(kmax, nullptr);
    if (locked_in_ws)
        for (int i = 0; i < kmax; ++i) w.locked[i] = c.take((size_t)D * elem);
    const int nv = kmax + m + 2;
    w.vp = (const void **)c.take((size_t)nv * sizeof(void *));
    w.sig2 = (double *)c.take((size_t)nv * sizeof(double));
    w.gamma = (double *)c.take((size_t)nv * sizeof(double));
    w.raw = (double *)c.take((size_t)2 * nv * sizeof(double));
    w.coef = (double *)c.take((size_t)nv * sizeof(double));
    w.alpha = (double *)c.take((size_t)(m + 2) * sizeof(double));
    w.beta = (double *)c.take((size_t)(m + 2) * sizeof(double));
    w.partials = (double *)c.take((size_t)2 * nv * (size_t)w.nblk * sizeof(double));
    w.gram = (double *)c.take((size_t)(m + 1) * (size_t)(m + 1) * sizeof(double));
    w.rcoef = (double *)c.take((size_t)kIRMaxIn * kIRMaxOut * sizeof(double));
    w.tri = (double *)c.take((size_t)(m + 8) * sizeof(double));
    w.triwork = (double *)c.take((size_t)(8 + 6 * (m + 2)) * sizeof(double) + (size_t)(m + 2) * sizeof(int) + 64);
    return c.off + 256;
}

// ----------------------------------------------------------------- solver --
struct Solver {
    ed_ham_s *h;               // the operator the iteration runs on
    ed_ham_s *flat = nullptr;  // the rank-order handle when h is its grouped twin
    hipStream_t s;
    ed_lanczos_opts o;
    Work w;
    int nlock = 0;
    std::vector<double> lock_sig2;
    double moved = 0.0;  // algorithmic bytes of the vector kernels launched so far
    void count(double nvec) { moved += nvec * (double)h->D * (double)w.elem; }

    template <typename TX>
    void multidot(int vbeg, int nvec, const void *y) {
        const TX *const *vecs = (const TX *const *)(w.vp + vbeg);
        k_multidot_v4<TX, 8, false><<<w.nblk, kRedBS, 0, s>>>(vecs, nvec, (const TX *)y, nullptr, h->D, w.partials);
        ED_LAUNCH_CHECK();
    }
    template <typename TX>
    void lincomb(int vbeg, const double *coef, int nvec, void *y, int assign, double sign, double *normp,
                 const double *post) {
        const TX *const *vecs = (const TX *const *)(w.vp + vbeg);
        k_lincomb_v4<TX><<<w.nblk, kRedBS, 0, s>>>(vecs, coef, nvec, (TX *)y, h->D, assign, sign, normp, post);
        ED_LAUNCH_CHECK();
    }
    void dots(int vbeg, int nvec, const void *y, double *alpha, int jrel) {
        count(nvec + 1);
        if (h->prec == ED_FP64) multidot<double>(vbeg, nvec, y);
        else multidot<float>(vbeg, nvec, y);
        k_finalize_dots_par<<<nvec, 256, 0, s>>>(w.partials, w.nblk, w.sig2 + vbeg, w.raw, w.gamma + vbeg, alpha,
                                                 jrel);
        ED_LAUNCH_CHECK();
    }
    // both projections of one step from a single read of the basis (reorth = 3)
    void dots_gram(int nvec, const void *y, const void *z, double *alpha) {
        count(nvec + 2);
        if (h->prec == ED_FP64)
            k_multidot_v4<double, 8, true><<<w.nblk, kRedBS, 0, s>>>((const double *const *)w.vp, nvec,
                                                                    (const double *)y, (const double *)z, h->D,
                                                                    w.partials);
        else
            k_multidot_v4<float, 8, true><<<w.nblk, kRedBS, 0, s>>>((const float *const *)w.vp, nvec,
                                                                   (const float *)y, (const float *)z, h->D,
                                                                   w.partials);
        ED_LAUNCH_CHECK();
        k_rowsums<<<2 * nvec, 256, 0, s>>>(w.partials, w.nblk, w.raw);
        ED_LAUNCH_CHECK();
        k_gram_coef<<<1, 256, 0, s>>>(w.raw, nvec, w.sig2, w.gram, w.m + 1, w.gamma, alpha);
        ED_LAUNCH_CHECK();
    }
    void update(int vbeg, int nvec, void *y, double *normp, const double *post = nullptr) {
        count(nvec + 2);
        if (h->prec == ED_FP64) lincomb<double>(vbeg, w.gamma + vbeg, nvec, y, 0, 1.0, normp, post);
        else lincomb<float>(vbeg, w.gamma + vbeg, nvec, y, 0, 1.0, normp, post);
    }
    void combine(int vbeg, const double *coef, int nvec, void *out) {  // out = sum coef_i S_i
        count(nvec + 1);
        if (h->prec == ED_FP64) lincomb<double>(vbeg, coef, nvec, out, 1, -1.0, nullptr, nullptr);
        else lincomb<float>(vbeg, coef, nvec, out, 1, -1.0, nullptr, nullptr);
    }
    void upload_pointers(const std::vector<void *> &krylov) {
        std::vector<const void *> v;
        for (int i = 0; i < nlock; ++i) v.push_back(w.locked[i]);
        for (void *p : krylov) v.push_back(p);
        ED_HIP(hipMemcpyAsync(w.vp, v.data(), v.size() * sizeof(void *), hipMemcpyHostToDevice, s));
        if (nlock)
            ED_HIP(hipMemcpyAsync(w.sig2, lock_sig2.data(), (size_t)nlock * sizeof(double), hipMemcpyHostToDevice, s));
        ED_HIP(hipStreamSynchronize(s));
    }
    // caller vector (rank order) -> workspace slot (the operator's order)
    void load_vector(const void *src, void *dst) {
        count(2);
        if (flat) permute_vector(h, src, dst, 0, s);
        else ED_HIP(hipMemcpyAsync(dst, src, (size_t)h->D * w.elem, hipMemcpyDeviceToDevice, s));
    }
    // a caller-owned vector converted in place between the two orders, through
    // a free workspace slot (dir 0: to the grouped order, 1: back)
    void convert_in_place(void *v, int dir) {
        if (!flat) return;
        void *tmp = w.slots[0];
        ED_HIP(hipMemcpyAsync(tmp, v, (size_t)h->D * w.elem, hipMemcpyDeviceToDevice, s));
        permute_vector(h, tmp, v, dir, s);
    }
    // vector norm^2 of y via a one-vector multidot with pointer slot `idx`
    double norm2_sync(int idx, const void *y) {
        count(1);
        if (h->prec == ED_FP64) multidot<double>(idx, 1, y);
        else multidot<float>(idx, 1, y);
        k_finalize_dots_par<<<1, 256, 0, s>>>(w.partials, w.nblk, nullptr, w.raw, nullptr, nullptr, 0);
        ED_LAUNCH_CHECK();
        double r = 0.0;
        ED_HIP(hipMemcpyAsync(&r, w.raw, sizeof(double), hipMemcpyDeviceToHost, s));
        ED_HIP(hipStreamSynchronize(s));
        return r;
    }
    // orthogonalise the first Krylov slot against the locked vectors (twice),
    // scale it to unit norm and set sigma_0 from the stored values.
    double prepare_start(void *s0) {
        for (int rep = 0; rep < 2 && nlock > 0; ++rep) {
            dots(0, nlock, s0, nullptr, 0);
            update(0, nlock, s0, nullptr);
        }
        double n2 = norm2_sync(nlock, s0);
        if (!(n2 > 0.0) || !std::isfinite(n2)) fail(ED_EINVAL, "start vector is zero (or lies in the locked subspace)");
        count(2);
        k_scale<<<grid_for(h->D, 256, 1 << 16), 256, 0, s>>>(s0, h->D, 1.0 / std::sqrt(n2), h->prec == ED_FP32);
        ED_LAUNCH_CHECK();
        n2 = norm2_sync(nlock, s0);
        if (!(n2 > 0.0) || !std::isfinite(n2)) fail(ED_EINVAL, "start vector is zero (or lies in the locked subspace)");
        const double sg = 1.0 / n2;
        ED_HIP(hipMemcpyAsync(w.sig2 + nlock, &sg, sizeof(double), hipMemcpyHostToDevice, s));
        ED_HIP(hipStreamSynchronize(s));
        return n2;
    }

    // One eigenpair by restarted Lanczos.  `out` receives the Ritz vector
    // normalised to 1 (it must not be one of the slots).  Returns the status.
    // fresh >= 0: start from the SplitMix64 normal stream `fresh` instead of v0.
    // Implicit restart keeping k vectors after a full cycle of m steps (slots
    // kr[0..m] hold S_0..S_m).  All checks come before the in-place rebuild of
    // the basis; false = not applicable (the caller restarts explicitly).
    // Returns with alpha/beta/sig2 (and the Gram block) set for continuing at
    // step k; *breakdown when the kept vectors span an invariant subspace.
    bool implicit_restart(int m, int k, bool *breakdown) {
        *breakdown = false;
        std::vector<double> al((size_t)m), be((size_t)m), sg((size_t)m + 1);
        ED_HIP(hipMemcpyAsync(al.data(), w.alpha, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
        ED_HIP(hipMemcpyAsync(be.data(), w.beta, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
        // Krylov entries of the pointer and sigma tables follow the nlock locked ones
        ED_HIP(hipMemcpyAsync(sg.data(), w.sig2 + nlock, (size_t)(m + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
        ED_HIP(hipStreamSynchronize(s));
        std::vector<double> C, a2, b2, ev;
        if (!ir_plan(al, be, sg, m, k, C, a2, b2, ev)) return false;
        const int nin = m + 1, nout = k + 1;
        ED_HIP(hipMemcpyAsync(w.rcoef, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, s));
        count(nin + nout);
        if (h->prec == ED_FP64)
            launch_restart_combine<double>((const double *const *)w.vp + nlock, w.rcoef, nin, nout, h->D, w.partials,
                                           w.nblk, s);
        else
            launch_restart_combine<float>((const float *const *)w.vp + nlock, w.rcoef, nin, nout, h->D, w.partials,
                                          w.nblk, s);
        ED_LAUNCH_CHECK();
        k_finalize_dots_par<<<1, 256, 0, s>>>(w.partials, w.nblk, nullptr, w.raw, nullptr, nullptr, 0);
        ED_LAUNCH_CHECK();
        double n2 = 0.0;
        ED_HIP(hipMemcpyAsync(&n2, w.raw, sizeof(double), hipMemcpyDeviceToHost, s));
        ED_HIP(hipStreamSynchronize(s));
        std::vector<double> na((size_t)m + 2, 0.0), nbv((size_t)m + 2, 0.0), ns((size_t)m + 1, 0.0);
        for (int i = 0; i < k; ++i) {
            na[i] = a2[i];
            if (i + 1 < k) nbv[i] = b2[i];
            ns[i] = 1.0;
        }
        const double scale = std::max(1.0, std::fabs(ev[0]));
        if (!(n2 > (64.0 * 2.220446049250313e-16 * scale) * (64.0 * 2.220446049250313e-16 * scale)))
            *breakdown = true;
        nbv[k - 1] = *breakdown ? 0.0 : std::sqrt(n2);
        ns[k] = *breakdown ? 0.0 : 1.0 / n2;
        ED_HIP(hipMemcpyAsync(w.alpha, na.data(), na.size() * sizeof(double), hipMemcpyHostToDevice, s));
        ED_HIP(hipMemcpyAsync(w.beta, nbv.data(), nbv.size() * sizeof(double), hipMemcpyHostToDevice, s));
        ED_HIP(hipMemcpyAsync(w.sig2 + nlock, ns.data(), ns.size() * sizeof(double), hipMemcpyHostToDevice, s));
        if (o.reorth == 3 && nlock == 0) {
            std::vector<double> G((size_t)(m + 1) * (m + 1), 0.0);
            for (int i = 0; i < k; ++i) G[(size_t)i * (m + 1) + i] = 1.0;
            ED_HIP(hipMemcpyAsync(w.gram, G.data(), G.size() * sizeof(double), hipMemcpyHostToDevice, s));
        }
        ED_HIP(hipStreamSynchronize(s));
        return true;
    }

    // m Lanczos steps from v0 with no restart (the continued-fraction
    // coefficients of a resolvent): alpha_h[0..k), beta_h[0..k) on the host,
    // k <= m steps (fewer when the Krylov space is exhausted, beta_h[k-1] = 0),
    // and ||v0||^2 in *v0n2.  Ground-state style storage: locked vectors none.
    int tridiag(const void *v0, int m, double *alpha_h, double *beta_h, double *v0n2) {
        load_vector(v0, w.slots[0]);
        // basis index i lives in slot i (full reorthogonalisation) or i mod 3
        // (three-term recurrence: only S_{j-1}, S_j and the new vector are read)
        std::vector<void *> kr((size_t)m + 1);
        for (int i = 0; i <= m; ++i) kr[i] = w.slots[(size_t)i % w.slots.size()];
        upload_pointers(kr);
        *v0n2 = norm2_sync(0, kr[0]);
        prepare_start(kr[0]);
        k_zero<<<1, 256, 0, s>>>(w.alpha, m + 2);
        k_zero<<<1, 256, 0, s>>>(w.beta, m + 2);
        ED_LAUNCH_CHECK();
        for (int j = 0; j < m; ++j) {
            void *Y = kr[j + 1];
            apply_launch(h, kr[j], Y, s);
                count(2);
            const int nv = j + 1;
            if (o.reorth == 3) {
                dots_gram(nv, Y, kr[j], w.alpha + j);
                update(0, nv, Y, w.partials, w.sig2 + j);
            } else {
                int vb = 0, nvec = nv;
                if (o.reorth == 0 && j >= 2) {
                    vb = j - 1;
                    nvec = 2;
                }
                const int passes = o.reorth >= 2 ? 2 : 1;
                for (int ps = 0; ps < passes; ++ps) {
                    const bool last_pass = ps == passes - 1;
                    dots(vb, nvec, Y, w.alpha + j, j - vb);
                    update(vb, nvec, Y, last_pass ? w.partials : nullptr, last_pass ? w.sig2 + j : nullptr);
                }
            }
            k_finalize_norm<<<1, 256, 0, s>>>(w.partials, w.nblk, w.sig2, w.beta, j, j);
            ED_LAUNCH_CHECK();
        }
        ED_HIP(hipMemcpyAsync(alpha_h, w.alpha, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
        ED_HIP(hipMemcpyAsync(beta_h, w.beta, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
        ED_HIP(hipStreamSynchronize(s));
        double scale = 1.0;
        for (int j = 0; j < m; ++j) scale = std::max(scale, std::fabs(alpha_h[j]));
        for (int j = 0; j < m; ++j) {
            if (!std::isfinite(alpha_h[j]) || !std::isfinite(beta_h[j]))
                fail(ED_EDEVICE, "non-finite Lanczos coefficients at step %d", j);
            if (!(std::fabs(beta_h[j]) > 64.0 * 2.220446049250313e-16 * scale)) {
                beta_h[j] = 0.0;
                return j + 1;
            }
        }
        return m;
    }

    // Two-sided interval for the eigenvalue just found.  The Rayleigh quotient
    // rq is an upper bound (variational).  The Kato-Temple inequality gives
    // lambda >= rq - r^2 / (eta - rq) for any eta with rq < eta <= the next
    // eigenvalue of the (deflated) operator; eta is taken as the second Ritz
    // value of the last cycle's tridiagonal matrix minus its residual bound
    // |beta_m s_m|, which is a lower bound on the next eigenvalue as long as
    // the iteration has not missed one between the two Ritz values.  NaN when
    // there is no second Ritz value or the gap is not resolved.
    void kato_temple(int m, double rq, double r, ed_info *inf) {
        inf->gap_lower = std::nan("");
        inf->e_lower = std::nan("");
        if (m < 2) return;
        std::vector<double> al((size_t)m), be((size_t)m);
        ED_HIP(hipMemcpyAsync(al.data(), w.alpha, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
        ED_HIP(hipMemcpyAsync(be.data(), w.beta, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
        ED_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < m; ++i)
            if (!std::isfinite(al[i]) || !std::isfinite(be[i])) return;
        const double t2 = tridiag_eig(al, be, m, 1);
        const double z = tridiag_evec_last(al, be, m, t2);
        if (!std::isfinite(z)) return;
        const double eta = t2 - std::fabs(be[m - 1] * z);
        inf->gap_lower = eta;
        if (eta > rq && std::isfinite(r)) inf->e_lower = rq - r * r / (eta - rq);
    }

    ed_status run(const void *v0, void *out, double *E, ed_info *info, int64_t fresh = -1) {
        // cycle length: at most the dimension of the space left after deflation;
        // a cycle that spans all of it has exact Ritz values (up to rounding)
        const int m = (int)std::min<int64_t>(w.m, h->D - nlock);
        const bool spans = (int64_t)m == h->D - nlock && o.reorth >= 2;
        ed_info inf{};
        moved = 0.0;
        if (fresh >= 0) {
            k_fill<<<grid_for(h->D, 256, 1 << 16), 256, 0, s>>>(w.slots[0], h->D, (uint64_t)fresh, 1,
                                                               h->prec == ED_FP32 ? 1 : 0);
            ED_LAUNCH_CHECK();
        } else {
            load_vector(v0, w.slots[0]);
        }
        std::vector<void *> kr(w.slots.begin(), w.slots.end());
        upload_pointers(kr);
        prepare_start(kr[0]);
        int total = 0;
        bool converged = false;
        double theta = 0.0, resid = 0.0;
        int jlast = -1;  // number of steps in the current cycle
        const double eps = 2.220446049250313e-16;
        int jstart = 0;  // first step of the cycle (k after an implicit restart)
        while (true) {
            if (jstart == 0) {
                k_zero<<<1, 256, 0, s>>>(w.alpha, m + 2);
                k_zero<<<1, 256, 0, s>>>(w.beta, m + 2);
                ED_LAUNCH_CHECK();
            }
            int j = jstart;
            bool cycle_done = false;
            for (; j < m; ++j) {
                void *Y = kr[j + 1];
                apply_launch(h, kr[j], Y, s);
                count(2);
                const int nv = nlock + j + 1;
                int vb = 0, nvec = nv;
                if (o.reorth == 0 && j >= 2) {  // three-term recurrence by projection on S_{j-1}, S_j
                    vb = nlock + j - 1;
                    nvec = 2;
                }
                if (o.reorth == 3 && nlock == 0) {
                    // one two-sided multi-dot (Y and S_j) and one update with the
                    // coefficients of both projections; scaled by sigma_j like below
                    dots_gram(nv, Y, kr[j], w.alpha + j);
                    update(0, nv, Y, w.partials, w.sig2 + j);
                } else {
                    const int passes = o.reorth >= 2 ? 2 : 1;
                    for (int ps = 0; ps < passes; ++ps) {
                        const bool last_pass = ps == passes - 1;
                        dots(vb, nvec, Y, w.alpha + j, nlock + j - vb);
                        // the last pass also scales by sigma_j: the stored vector is w''
                        update(vb, nvec, Y, last_pass ? w.partials : nullptr,
                               last_pass ? w.sig2 + nlock + j : nullptr);
                    }
                }
                k_finalize_norm<<<1, 256, 0, s>>>(w.partials, w.nblk, w.sig2, w.beta, nlock + j, j);
                ED_LAUNCH_CHECK();
                ++total;
                const bool full = (j + 1 == m);
                const bool check = j == 0 || ((j + 1) % o.check_every == 0) || full || total >= o.max_iter;
                if (!check) continue;
                k_tridiag_lowest<<<1, 256, 0, s>>>(w.alpha, w.beta, j + 1, 0.0, w.tri, w.triwork);
                ED_LAUNCH_CHECK();
                double tv[3];
                ED_HIP(hipMemcpyAsync(tv, w.tri, sizeof(tv), hipMemcpyDeviceToHost, s));
                ED_HIP(hipStreamSynchronize(s));
                theta = tv[0];
                resid = tv[1];
                jlast = j + 1;
                const double scale = std::max(std::fabs(theta), 1.0);
                const bool brk = std::fabs(tv[2]) <= 64.0 * eps * scale;
                if (!std::isfinite(theta) || !std::isfinite(resid))
                    fail(ED_EDEVICE, "non-finite Lanczos coefficients (alpha/beta) at step %d", total);
                if (resid <= o.tol * scale || brk || (full && spans)) {
                    converged = true;
                    cycle_done = true;
                    break;
                }
                if (total >= o.max_iter || full) {
                    cycle_done = true;
                    break;
                }
            }
            (void)cycle_done;
            inf.basis_used = std::max(inf.basis_used, jlast);
            // Ritz vector of this cycle
            k_ritz_coef<<<1, 256, 0, s>>>(w.tri + 3, w.sig2 + nlock, jlast, w.coef);
            ED_LAUNCH_CHECK();
            if (converged || total >= o.max_iter) {
                combine(nlock, w.coef, jlast, out);
                break;
            }
            bool brk_ir = false;
            if (o.keep > 0 && o.keep < m && jlast == m && implicit_restart(m, o.keep, &brk_ir)) {
                ++inf.restarts;
                jstart = o.keep;
                if (brk_ir) {
                    // the kept vectors span an invariant subspace: finish on them
                    k_tridiag_lowest<<<1, 256, 0, s>>>(w.alpha, w.beta, jstart, 0.0, w.tri, w.triwork);
                    ED_LAUNCH_CHECK();
                    jlast = jstart;
                    converged = true;
                    k_ritz_coef<<<1, 256, 0, s>>>(w.tri + 3, w.sig2 + nlock, jlast, w.coef);
                    ED_LAUNCH_CHECK();
                    double tv[3];
                    ED_HIP(hipMemcpyAsync(tv, w.tri, sizeof(tv), hipMemcpyDeviceToHost, s));
                    ED_HIP(hipStreamSynchronize(s));
                    theta = tv[0];
                    resid = 0.0;
                    combine(nlock, w.coef, jlast, out);
                    break;
                }
                continue;
            }
            jstart = 0;
            // restart: psi -> the spare slot, which becomes the new S_0
            void *spare = kr[m];
            combine(nlock, w.coef, jlast, spare);
            std::rotate(kr.begin(), kr.begin() + m, kr.end());
            upload_pointers(kr);
            prepare_start(kr[0]);
            ++inf.restarts;
        }
        // normalise the output and refine
        ED_HIP(hipStreamSynchronize(s));
        // pointer table slot for `out` at position nlock (Krylov slots are done)
        const void *outp = out;
        ED_HIP(hipMemcpyAsync(w.vp + nlock, &outp, sizeof(void *), hipMemcpyHostToDevice, s));
        ED_HIP(hipStreamSynchronize(s));
        const double n2 = norm2_sync(nlock, out);
        if (!(n2 > 0.0)) fail(ED_EDEVICE, "Ritz vector has zero norm");
        count(2);
        k_scale<<<grid_for(h->D, 256, 1 << 16), 256, 0, s>>>(out, h->D, 1.0 / std::sqrt(n2), h->prec == ED_FP32);
        ED_LAUNCH_CHECK();
        inf.iters = total;
        inf.converged = converged ? 1 : 0;
        inf.ritz = theta;
        double rq = theta, rr = resid;
        if (o.refine) {
            rayleigh_fp64(h, out, &rq, &rr, s);
            count(2);
            inf.residual = rr;
            inf.rq_fp64 = rq;
            *E = rq;
        } else {
            inf.residual = resid;
            inf.rq_fp64 = theta;
            *E = theta;
        }
        ED_HIP(hipStreamSynchronize(s));
        kato_temple(jlast, rq, rr, &inf);
        inf.traffic = moved;
        if (info) *info = inf;
        return converged ? ED_OK : ED_ENOCONV;
    }
};

static size_t ws_needed(const ed_ham_s *h, const ed_lanczos_opts &o, int k, bool locked_in_ws) {
    Work w;
    return layout(w, nullptr, h->D, h->prec == ED_FP64 ? 8 : 4, o.max_basis, k, locked_in_ws);
}

// Smallest usable basis: two vectors, or the kept block of an implicit restart
// plus two.
static int min_basis(const ed_ham_s *h, const ed_lanczos_opts &o) {
    return (int)std::min<int64_t>(std::max(2, o.keep + 2), std::max<int64_t>(h->D, 1));
}

// Memory planner (max_basis = 0): the largest basis, at most kAutoBasisMax
// vectors (and the per-kernel pointer limit), whose workspace fits `budget`
// bytes.  ENOMEM when even the smallest usable basis does not fit.
static int plan_basis(const ed_ham_s *h, ed_lanczos_opts o, int k, bool locked_in_ws, size_t budget) {
    int lo = min_basis(h, o);
    int hi = (int)std::min<int64_t>(std::min(kAutoBasisMax, kMaxVec - 2 - k), std::max<int64_t>(h->D, 1));
    if (hi < lo) hi = lo;
    o.max_basis = lo;
    if (ws_needed(h, o, k, locked_in_ws) > budget)
        fail(ED_ENOMEM, "no Lanczos workspace fits: %d basis vectors of %lld elements need %zu bytes, %zu available",
             lo, (long long)h->D, ws_needed(h, o, k, locked_in_ws), budget);
    while (lo < hi) {  // largest m with ws_needed(m) <= budget
        const int mid = (lo + hi + 1) / 2;
        o.max_basis = mid;
        if (ws_needed(h, o, k, locked_in_ws) <= budget) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Device memory a new workspace may take: what the runtime reports free (or,
// with total = true, the device's capacity), less a reserve for the library's
// own tables and the caller's other buffers.
static size_t device_budget(bool total = false) {
    size_t fr = 0, tot = 0;
    ED_HIP(hipMemGetInfo(&fr, &tot));
    const size_t reserve = std::max<size_t>((size_t)1 << 30, tot / 50);
    const size_t avail = total ? tot : fr;
    return avail > reserve ? avail - reserve : 0;
}

// Options with the basis size resolved: max_basis = 0 is planned against
// `budget` (the free device memory for a size query, the given workspace for a
// solve); an explicit basis is capped by the pointer limit of the kernels.
static ed_lanczos_opts resolve(const ed_ham_s *h, const ed_lanczos_opts *opts, int k, bool locked_in_ws,
                               size_t budget) {
    ed_lanczos_opts o = effective(opts, h->D);
    if (o.max_basis == 0) o.max_basis = plan_basis(h, o, k, locked_in_ws, budget);
    if (o.max_basis > kMaxVec - 2 - k) o.max_basis = kMaxVec - 2 - k;
    if (o.keep >= o.max_basis) o.keep = o.max_basis - 1;
    return o;
}

static size_t tridiag_ws_needed(const ed_ham_s *h, const ed_lanczos_opts &o, int m) {
    Work w;
    return layout(w, nullptr, h->D, h->prec == ED_FP64 ? 8 : 4, m, 1, true, o.reorth == 0 ? std::min(3, m + 1) : m + 1);
}

}  // namespace ed

using namespace ed;

extern "C" void ed_lanczos_defaults(ed_lanczos_opts *opts) {
    if (opts) fill_defaults(*opts);
}

extern "C" ed_status ed_workspace_bytes(ed_ham_t h, const ed_lanczos_opts *opts, int k, size_t *bytes) {
    return guard([&] {
        if (!h || !bytes) fail(ED_EINVAL, "ed_workspace_bytes: NULL argument");
        if (k < 1 || (int64_t)k > h->D) fail(ED_EINVAL, "ed_workspace_bytes: k=%d outside [1, D=%lld]", k, (long long)h->D);
        if (k > 200) fail(ED_EINVAL, "ed_workspace_bytes: k=%d above 200", k);
        DeviceGuard g(h->device);
        // a planned basis must fit the memory free now; an explicit one the device
        const ed_lanczos_opts o = resolve(h, opts, k, true, device_budget());
        *bytes = ws_needed(h, o, k, true);
        const size_t cap = device_budget(true);
        if (*bytes > cap)
            fail(ED_ENOMEM, "workspace of %zu bytes (%d basis vectors of %lld elements) exceeds the %zu bytes "
                 "the device can hold; use a smaller max_basis or max_basis = 0 to plan it",
                 *bytes, o.max_basis, (long long)h->D, cap);
    });
}

extern "C" ed_status ed_tridiag_workspace_bytes(ed_ham_t h, const ed_lanczos_opts *opts, int m, size_t *bytes) {
    return guard([&] {
        if (!h || !bytes) fail(ED_EINVAL, "ed_tridiag_workspace_bytes: NULL argument");
        if (m < 1 || (int64_t)m > h->D || m > kMaxVec - 2)
            fail(ED_EINVAL, "m=%d outside [1, min(D=%lld, %d)]", m, (long long)h->D, kMaxVec - 2);
        const ed_lanczos_opts o = effective(opts, h->D);
        *bytes = tridiag_ws_needed(h, o, m);
    });
}

// k0 > 0: evecs[0..k0) already hold converged, orthonormal eigenvectors (and
// evals[0..k0) their values); they are locked as they are and only the
// eigenpairs k0..k-1 are computed.
static ed_status solve(ed_ham_t h, int k, const ed_lanczos_opts *opts, const void *v0, void *ws, size_t ws_bytes,
                       double *evals, void *evecs, ed_info *info, void *stream, int k0 = 0) {
    ed_status result = ED_OK;
    ed_status st = guard([&] {
        if (!h) fail(ED_EINVAL, "NULL handle");
        if (!v0 || !ws || !evals) fail(ED_EINVAL, "NULL start vector, workspace or output");
        if (k < 1 || (int64_t)k > h->D) fail(ED_EINVAL, "k=%d outside [1, D=%lld]", k, (long long)h->D);
        if (k0 < 0 || k0 >= k || (k0 > 0 && !evecs))
            fail(ED_EINVAL, "k0=%d outside [0, k=%d) or no eigenvector array to continue from", k0, k);
        DeviceGuard g(h->device);
        Solver sv;
        sv.s = (hipStream_t)stream;
        // eigenpair e runs cycles of at most D - e steps (the deflated space)
        if (k > 200) fail(ED_EINVAL, "k=%d above 200", k);
        const bool locked_in_ws = (evecs == nullptr);
        sv.o = resolve(h, opts, k, locked_in_ws, ws_bytes);
        // run on the grouped twin when there is one (same operator, basis
        // order by components of the move graphs); vectors are converted at
        // the boundary
        sv.h = (sv.o.layout == 0 && h->twin) ? h->twin : h;
        if (sv.h != h) sv.flat = h;
        const size_t need = ws_needed(h, sv.o, k, locked_in_ws);
        if (ws_bytes < need) fail(ED_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        layout(sv.w, (char *)ws, h->D, h->prec == ED_FP64 ? 8 : 4, sv.o.max_basis, k, locked_in_ws);
        if (!locked_in_ws)
            for (int i = 0; i < k; ++i) sv.w.locked[i] = (char *)evecs + (size_t)i * h->D * sv.w.elem;
        for (int e = 0; e < k0; ++e) sv.convert_in_place(sv.w.locked[e], 0);  // given vectors
        for (int e = 0; e < k; ++e) {
            if (e < k0) {  // given: lock it as it is
                sv.nlock = e;
                const void *p = sv.w.locked[e];
                ED_HIP(hipMemcpyAsync(sv.w.vp + e, &p, sizeof(void *), hipMemcpyHostToDevice, sv.s));
                ED_HIP(hipStreamSynchronize(sv.s));
                const double n2 = sv.norm2_sync(e, p);
                if (!(n2 > 0.0)) fail(ED_EINVAL, "given eigenvector %d has zero norm", e);
                sv.lock_sig2.push_back(1.0 / n2);
                sv.nlock = e + 1;
                continue;
            }
            double E = 0.0;
            ed_info inf{};
            // A Krylov space built from one start vector holds a single vector per
            // distinct eigenvalue, so after deflating one copy of a repeated
            // eigenvalue the same start vector has no component left on the other
            // copies: every further eigenpair starts from a fresh random vector.
            const ed_status r = sv.run(v0, sv.w.locked[e], &E, &inf, e == 0 ? -1 : (int64_t)(0x5EED0000ull + e));
            if (r != ED_OK) result = r;
            evals[e] = E;
            if (info) info[e] = inf;
            // lock it: sigma^2 = 1 / ||psi||^2 (psi normalised to ~1 in storage precision)
            sv.nlock = e;  // pointer table entries [0, e) are the already-locked vectors
            // recompute the norm of the new locked vector through slot e
            const void *p = sv.w.locked[e];
            ED_HIP(hipMemcpyAsync(sv.w.vp + e, &p, sizeof(void *), hipMemcpyHostToDevice, sv.s));
            ED_HIP(hipStreamSynchronize(sv.s));
            const double n2 = sv.norm2_sync(e, p);
            sv.lock_sig2.push_back(n2 > 0.0 ? 1.0 / n2 : 0.0);
            sv.nlock = e + 1;
        }
        // eigenvalues found one after another on the deflated operator are
        // already ascending up to rounding; report them sorted with vectors kept
        // in discovery order only if no vectors were requested
        if (!evecs) std::sort(evals, evals + k);
        else
            for (int e = 0; e < k; ++e) sv.convert_in_place(sv.w.locked[e], 1);
        ED_HIP(hipStreamSynchronize(sv.s));
    });
    if (st != ED_OK) return st;
    return result;
}

extern "C" ed_status ed_lanczos_ground(ed_ham_t h, const ed_lanczos_opts *opts, const void *v0, void *ws,
                                       size_t ws_bytes, double *E0, void *psi0, ed_info *info, void *stream) {
    return solve(h, 1, opts, v0, ws, ws_bytes, E0, psi0, info, stream);
}

extern "C" ed_status ed_lanczos_tridiag(ed_ham_t h, const ed_lanczos_opts *opts, const void *v0, int m, void *ws,
                                        size_t ws_bytes, double *alpha, double *beta, int *steps, double *v0_norm2,
                                        void *stream) {
    return guard([&] {
        if (!h) fail(ED_EINVAL, "NULL handle");
        if (!v0 || !ws || !alpha || !beta || !steps || !v0_norm2) fail(ED_EINVAL, "NULL argument");
        if (m < 1 || (int64_t)m > h->D || m > kMaxVec - 2)
            fail(ED_EINVAL, "m=%d outside [1, min(D=%lld, %d)]", m, (long long)h->D, kMaxVec - 2);
        DeviceGuard g(h->device);
        Solver sv;
        sv.s = (hipStream_t)stream;
        sv.o = effective(opts, h->D);
        sv.o.max_basis = m;
        sv.o.keep = 0;
        sv.h = (sv.o.layout == 0 && h->twin) ? h->twin : h;
        if (sv.h != h) sv.flat = h;
        const size_t need = tridiag_ws_needed(h, sv.o, m);
        if (ws_bytes < need) fail(ED_EINVAL, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        layout(sv.w, (char *)ws, h->D, h->prec == ED_FP64 ? 8 : 4, m, 1, true,
               sv.o.reorth == 0 ? std::min(3, m + 1) : m + 1);
        *steps = sv.tridiag(v0, m, alpha, beta, v0_norm2);
    });
}

extern "C" ed_status ed_arnoldi_lowest(ed_ham_t h, int k, const ed_lanczos_opts *opts, const void *v0, void *ws,
                                       size_t ws_bytes, double *evals, void *evecs, ed_info *info, void *stream) {
    return solve(h, k, opts, v0, ws, ws_bytes, evals, evecs, info, stream);
}

extern "C" ed_status ed_arnoldi_lowest_more(ed_ham_t h, int k0, int k, const ed_lanczos_opts *opts, const void *v0,
                                            void *ws, size_t ws_bytes, double *evals, void *evecs, ed_info *info,
                                            void *stream) {
    return solve(h, k, opts, v0, ws, ws_bytes, evals, evecs, info, stream, k0);
}
