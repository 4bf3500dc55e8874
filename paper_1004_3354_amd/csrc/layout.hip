// Vectors in the grouped basis order.  A sector vector in rank order has
// element (r_up, r_dn) at r_up * D_dn + r_dn; in the grouped order of a twin
// handle element (p_up, p_dn) sits at p_up * D_dn + p_dn, p the position of the
// state in that spin's grouped order (ed_ham_s).  Converting is a gather along
// rows: row p_up of the grouped vector is row gperm[0][p_up] of the rank-order
// one with its columns permuted by gperm[1].
#include "ed_internal.h"

namespace ed {

// dir = 0: y (grouped) <- x (rank order); dir = 1: y (rank order) <- x (grouped).
// Workgroup rows stride over the rows; threads over the columns of a row, so
// the grouped side is read or written contiguously.
template <typename TX>
__global__ void k_permute(const TX *x, TX *y, const int32_t *pu, const int32_t *pd, int64_t dup, int64_t ddn,
                          int dir) {
    for (int64_t p = blockIdx.y; p < dup; p += gridDim.y) {
        const int64_t r = pu[p];
        for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ddn;
             q += (int64_t)gridDim.x * blockDim.x) {
            const int64_t gi = p * ddn + q, fi = r * ddn + pd[q];
            if (dir == 0) y[gi] = x[fi];
            else y[fi] = x[gi];
        }
    }
}

void permute_vector(const ed_ham_s *g, const void *x, void *y, int dir, hipStream_t s) {
    if (!g || !g->grouped) fail(ED_EINVAL, "no grouped order");
    const dim3 grid((unsigned)std::min<int64_t>((g->ddn + 255) / 256, 64),
                    (unsigned)std::min<int64_t>(g->dup, 65535));
    const int32_t *pu = g->gperm[0].as<int32_t>(), *pd = g->gperm[1].as<int32_t>();
    if (g->prec == ED_FP64)
        k_permute<double><<<grid, 256, 0, s>>>((const double *)x, (double *)y, pu, pd, g->dup, g->ddn, dir);
    else
        k_permute<float><<<grid, 256, 0, s>>>((const float *)x, (float *)y, pu, pd, g->dup, g->ddn, dir);
    ED_LAUNCH_CHECK();
}

}  // namespace ed

using namespace ed;

extern "C" ed_status ed_ham_grouped(ed_ham_t h, ed_ham_t *grouped) {
    return guard([&] {
        if (!h || !grouped) fail(ED_EINVAL, "ed_ham_grouped: NULL argument");
        *grouped = h->grouped ? h : h->twin;
    });
}

extern "C" ed_status ed_grouped_order(ed_ham_t g, int spin, int32_t *rank_of_position) {
    return guard([&] {
        if (!g || !rank_of_position) fail(ED_EINVAL, "ed_grouped_order: NULL argument");
        if (!g->grouped) fail(ED_EINVAL, "ed_grouped_order: the handle is not in the grouped order");
        if (spin != 0 && spin != 1) fail(ED_EINVAL, "ed_grouped_order: spin must be 0 or 1");
        DeviceGuard dg(g->device);
        const int64_t n = spin == 0 ? g->dup : g->ddn;
        ED_HIP(hipMemcpy(rank_of_position, g->gperm[spin].p, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost));
    });
}

static ed_status permute_call(ed_ham_t h, const void *x, void *y, void *stream, int dir, const char *name) {
    return guard([&] {
        if (!h || !x || !y) fail(ED_EINVAL, "%s: NULL argument", name);
        if (x == y) fail(ED_EINVAL, "%s: x and y must not alias", name);
        const ed_ham_s *g = h->grouped ? h : h->twin;
        if (!g) fail(ED_EINVAL, "%s: the Hamiltonian has no grouped order (connected move graphs)", name);
        DeviceGuard dg(g->device);
        permute_vector(g, x, y, dir, (hipStream_t)stream);
    });
}

extern "C" ed_status ed_to_grouped(ed_ham_t h, const void *x, void *y, void *stream) {
    return permute_call(h, x, y, stream, 0, "ed_to_grouped");
}

extern "C" ed_status ed_from_grouped(ed_ham_t h, const void *x, void *y, void *stream) {
    return permute_call(h, x, y, stream, 1, "ed_from_grouped");
}
