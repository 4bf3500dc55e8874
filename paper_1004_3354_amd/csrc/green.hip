// Impurity Green function by Lanczos continued fractions (Eq. 3 at low
// temperature): the particle part needs c+_{i sigma} applied to an eigenvector
// of the (N_up, N_dn) sector, the hole part c_{i sigma}; each resulting vector
// starts a Lanczos run in the neighbouring sector whose tridiagonal
// coefficients give <phi|(z -+ (H - E0))^-1|phi> as a continued fraction.
#include <cmath>
#include <complex>

#include "ed_internal.h"

namespace ed {

// y = c+_{site, spin} x (dagger = 1) or c_{site, spin} x (dagger = 0), pulled
// from the destination sector: a destination state s' comes from the source
// state s = s' with the site's bit flipped, the other spin unchanged.  Sign:
// (-1)^(number of occupied fermion modes below the site's mode), with all
// up-spin modes before the down-spin ones.
template <typename TX>
__global__ void k_ladder(const TX *x, TX *y, const uint32_t *dst_states, int64_t ddn_dst, int64_t ddn_src,
                         int64_t D_dst, int ns, int n_src, int spin, int site, int dagger, int nup_src) {
    const uint32_t bit = 1u << site, below = bit - 1u;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < D_dst;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = e / ddn_dst, d = e - u * ddn_dst;
        const uint32_t sp = dst_states[spin == ED_SPIN_UP ? u : d];
        const bool ok = dagger ? (sp & bit) != 0u : (sp & bit) == 0u;
        TX v = (TX)0;
        if (ok) {
            const uint32_t s = sp ^ bit;
            const int64_t r = rank_state(s, ns, n_src);
            const int par = __popc(s & below) + (spin == ED_SPIN_DN ? nup_src : 0);
            const int64_t src = spin == ED_SPIN_UP ? r * ddn_src + d : u * ddn_src + r;
            v = x[src];
            if (par & 1) v = -v;
        }
        y[e] = v;
    }
}

}  // namespace ed

using namespace ed;

extern "C" ed_status ed_apply_ladder(ed_ham_t src, ed_ham_t dst, int spin, int site, int dagger, const void *x,
                                     void *y, void *stream) {
    return guard([&] {
        if (!src || !dst || !x || !y) fail(ED_EINVAL, "ed_apply_ladder: NULL argument");
        if (x == y) fail(ED_EINVAL, "ed_apply_ladder: x and y alias");
        if (spin != ED_SPIN_UP && spin != ED_SPIN_DN) fail(ED_EINVAL, "ed_apply_ladder: spin must be 0 or 1");
        if (src->ns != dst->ns || site < 0 || site >= src->ns)
            fail(ED_EINVAL, "ed_apply_ladder: site %d outside [0, Ns) or different Ns", site);
        if (src->prec != dst->prec || src->device != dst->device)
            fail(ED_EINVAL, "ed_apply_ladder: handles of different precision or device");
        const int dn = dagger ? 1 : -1;
        const int nsrc = spin == ED_SPIN_UP ? src->nup : src->ndn;
        const int ndst = spin == ED_SPIN_UP ? dst->nup : dst->ndn;
        const int osrc = spin == ED_SPIN_UP ? src->ndn : src->nup;
        const int odst = spin == ED_SPIN_UP ? dst->ndn : dst->nup;
        if (ndst != nsrc + dn || osrc != odst)
            fail(ED_EINVAL, "ed_apply_ladder: destination sector must differ by %+d electron of the given spin", dn);
        DeviceGuard g(src->device);
        hipStream_t s = (hipStream_t)stream;
        const uint32_t *st = dst->sp[spin].states.as<uint32_t>();
        const unsigned grid = grid_for(dst->D, 256, 1 << 16);
        if (src->prec == ED_FP64)
            k_ladder<double><<<grid, 256, 0, s>>>((const double *)x, (double *)y, st, dst->ddn, src->ddn, dst->D,
                                                  src->ns, nsrc, spin, site, dagger ? 1 : 0, src->nup);
        else
            k_ladder<float><<<grid, 256, 0, s>>>((const float *)x, (float *)y, st, dst->ddn, src->ddn, dst->D,
                                                 src->ns, nsrc, spin, site, dagger ? 1 : 0, src->nup);
        ED_LAUNCH_CHECK();
    });
}

extern "C" ed_status ed_green_cf(const double *alpha, const double *beta, int k, double norm2, double e0, int sign,
                                 double weight, const double *z_re, const double *z_im, int nz, double *g_re,
                                 double *g_im) {
    return guard([&] {
        if (!alpha || !beta || !z_re || !z_im || !g_re || !g_im) fail(ED_EINVAL, "ed_green_cf: NULL argument");
        if (k < 1 || nz < 0 || (sign != 1 && sign != -1)) fail(ED_EINVAL, "ed_green_cf: bad k, nz or sign");
        if (!std::isfinite(weight) || !std::isfinite(norm2)) fail(ED_EINVAL, "ed_green_cf: non-finite weight");
        const double sg = (double)sign;
        for (int i = 0; i < nz; ++i) {
            const std::complex<double> z(z_re[i], z_im[i]);
            std::complex<double> d = z - sg * (alpha[k - 1] - e0);
            for (int j = k - 2; j >= 0; --j) d = z - sg * (alpha[j] - e0) - beta[j] * beta[j] / d;
            const std::complex<double> g = (weight * norm2) / d;
            g_re[i] += g.real();
            g_im[i] += g.imag();
        }
    });
}

extern "C" ed_status ed_boltzmann_weights(const double *E, int n, double beta, double cutoff, double *w, int *kept) {
    return guard([&] {
        if (!E || !w || !kept) fail(ED_EINVAL, "ed_boltzmann_weights: NULL argument");
        if (n < 1 || !(beta > 0.0) || !std::isfinite(beta) || !(cutoff >= 0.0) || !(cutoff < 1.0))
            fail(ED_EINVAL, "ed_boltzmann_weights: need n >= 1, 0 < beta < inf, 0 <= cutoff < 1");
        double emin = E[0];
        for (int i = 0; i < n; ++i) {
            if (!std::isfinite(E[i])) fail(ED_EINVAL, "ed_boltzmann_weights: non-finite energy %d", i);
            emin = std::min(emin, E[i]);
        }
        // factors relative to the lowest level (no overflow), first pass over all
        // states for the cut, second over the kept ones for the normalisation
        double z = 0.0;
        for (int i = 0; i < n; ++i) z += std::exp(-beta * (E[i] - emin));
        // the lowest levels always stay (with a g-fold degenerate lowest level
        // each has share <= 1/g, which a cut above 1/g would otherwise remove)
        double zk = 0.0;
        int nk = 0;
        for (int i = 0; i < n; ++i) {
            const double f = std::exp(-beta * (E[i] - emin));
            w[i] = (f / z >= cutoff || E[i] == emin) ? f : 0.0;
            if (w[i] > 0.0) {
                zk += w[i];
                ++nk;
            }
        }
        for (int i = 0; i < n; ++i) w[i] /= zk;
        *kept = nk;
    });
}
