// The K lowest levels over a set of sectors, counted with multiplicity: the
// thermal set that the finite-temperature sum of Eq. 3 runs over.  The paper's
// DMFT iteration at N_s = 12 needs the 300 lowest eigenstates of the impurity
// Hamiltonian (its comparison at the end of Section 3.2).
//
// Search: every sector's lowest level comes from one batched ground-state run;
// then, as long as some sector that still has levels left has its highest
// computed level at or below the K-th lowest level found so far, such sectors
// get more levels (restarted Lanczos with explicit deflation against the
// converged vectors, continuing from them), the few with the lowest highest
// levels at once.  A sector's uncomputed levels all lie above its highest computed one,
// so no level that could belong to the K lowest is skipped.  The vectors of
// the levels found stay in device memory owned by the result handle.
#include <algorithm>
#include <cmath>
#include <exception>
#include <thread>
#include <vector>

#include "ed_internal.h"

struct ed_levels_s {
    int device = 0;
    std::vector<ed_ham_s *> hs;
    std::vector<std::vector<double>> energies;  // per sector, in discovery order (ascending up to rounding)
    std::vector<ed::DevMem *> vecs;             // per sector: [nvec][D] eigenvectors in rank order
    std::vector<int> nvec;
    struct Level {
        double E;
        int s, i;
    };
    std::vector<Level> levels;
    std::vector<int> capped;
    int calls = 0;
    double threshold = INFINITY;
    ~ed_levels_s() {
        for (auto *v : vecs) delete v;
    }
};

namespace ed {

static double kth_lowest(const std::vector<std::vector<double>> &en, int K) {
    std::vector<double> all;
    for (auto &e : en) all.insert(all.end(), e.begin(), e.end());
    if ((int)all.size() < K) return INFINITY;
    std::nth_element(all.begin(), all.begin() + (K - 1), all.end());
    return all[K - 1];
}

static double highest(const std::vector<double> &e) { return *std::max_element(e.begin(), e.end()); }

static void lowest_levels(ed_levels_s *L, int nsec, const ed_ham_t *hs, int K, int kmax,
                          const ed_lanczos_opts *opts, uint64_t seed, hipStream_t s) {
    L->hs.assign(hs, hs + nsec);
    L->energies.assign(nsec, {});
    L->vecs.assign(nsec, nullptr);
    L->nvec.assign(nsec, 0);
    // every sector's lowest level from one batched run
    {
        size_t nb = 0;
        ed_status st = ed_batched_workspace_bytes(nsec, hs, opts, &nb);
        if (st != ED_OK) fail(st, "%s", ed_last_error());
        DevMem bws;
        bws.alloc(nb);
        std::vector<double> e0((size_t)nsec);
        st = ed_lanczos_ground_batched(nsec, hs, opts, nullptr, seed, bws.p, nb, e0.data(), nullptr, s);
        if (st != ED_OK && st != ED_ENOCONV) fail(st, "%s", ed_last_error());
        for (int q = 0; q < nsec; ++q) L->energies[q] = {e0[q]};
    }
    const size_t elem = L->hs[0]->prec == ED_FP64 ? 8 : 4;
    // one extension: sector q from its nvec[q] converged levels to k, on the
    // caller's stream with the caller's start-vector buffer and workspace
    // (buffers are grown with headroom and replaced vectors are freed after the
    // round: a device free waits for the whole device, which would serialise
    // the concurrent extensions)
    auto extend = [&](int q, int k, hipStream_t st, DevMem &v0, DevMem &ws, std::vector<DevMem *> &old) {
        ed_ham_s *h = L->hs[q];
        const int k0 = L->nvec[q];
        if (v0.bytes < (size_t)h->D * elem) v0.alloc((size_t)h->D * elem);
        DevMem *ev = new DevMem();
        try {
            ev->alloc((size_t)k * (size_t)h->D * elem);
            if (k0 > 0)
                ED_HIP(hipMemcpyAsync(ev->p, L->vecs[q]->p, (size_t)k0 * (size_t)h->D * elem, hipMemcpyDeviceToDevice,
                                      st));
            k_fill<<<grid_for(h->D, 256, 1 << 16), 256, 0, st>>>(v0.p, h->D, seed + (uint64_t)q, 1,
                                                                h->prec == ED_FP32 ? 1 : 0);
            ED_LAUNCH_CHECK();
            const ed_lanczos_opts o = resolve(h, opts, k, false, device_budget());
            const size_t need = ws_needed(h, o, k, false);
            if (ws.bytes < need) {  // headroom for later extensions when the device has room for it
                size_t fm = 0, tm = 0;
                if (hipMemGetInfo(&fm, &tm) != hipSuccess) {
                    (void)hipGetLastError();
                    fm = 0;
                }
                ws.alloc(need + need / 2 <= fm / 2 ? need + need / 2 : need);
            }
            std::vector<double> ev_h((size_t)k, 0.0);
            for (int i = 0; i < k0; ++i) ev_h[i] = L->energies[q][i];
            const ed_status r = solve(h, k, &o, v0.p, ws.p, ws.bytes, ev_h.data(), ev->p, nullptr, st, k0);
            if (r != ED_OK && r != ED_ENOCONV)
                fail(r, "sector %d (D = %lld), %d levels: %s", q, (long long)h->D, k, ed_last_error());
            L->energies[q].assign(ev_h.begin(), ev_h.end());
        } catch (...) {
            delete ev;
            throw;
        }
        if (L->vecs[q]) old.push_back(L->vecs[q]);
        L->vecs[q] = ev;
        L->nvec[q] = k;
    };
    // Rounds: every sector that may still hold one of the K lowest levels (its
    // highest computed level at or below the K-th lowest found so far, levels
    // left) is a candidate; the lowest few candidates are extended at once,
    // each on its own stream from its own host thread, so that the small
    // sectors' kernels share the GPU.  Extending more sectors than the one
    // with the lowest highest level can only compute levels that were not
    // needed; no level that could be among the K lowest is skipped.
    constexpr int kPar = 8;
    std::vector<hipStream_t> streams(kPar);
    for (auto &st : streams) ED_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    std::vector<DevMem> v0s(kPar), wss(kPar);
    std::vector<std::vector<DevMem *>> olds(kPar);
    auto free_old = [&]() {
        for (auto &o : olds) {
            for (DevMem *d : o) delete d;
            o.clear();
        }
    };
    std::vector<bool> capped((size_t)nsec, false);
    try {
        while (true) {
            const double T = kth_lowest(L->energies, K);
            std::vector<int> cand;
            for (int q = 0; q < nsec; ++q) {
                const int have = (int)L->energies[q].size();
                const int64_t lim = std::min<int64_t>(L->hs[q]->D, kmax);
                if (highest(L->energies[q]) > T) continue;
                if (have >= lim) {
                    if (have < L->hs[q]->D) capped[q] = true;
                    continue;
                }
                cand.push_back(q);
            }
            if (cand.empty()) break;
            std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) {
                return highest(L->energies[a]) < highest(L->energies[b]);
            });
            // concurrency only among sectors whose runs are small next to the device
            int npar = std::min<int>(kPar, (int)cand.size());
            for (int t = 0; t < npar; ++t)
                if ((double)L->hs[cand[t]]->D * (double)elem * 64.0 > 2e9) {
                    npar = 1;
                    break;
                }
            auto target = [&](int q) {
                const int k = L->nvec[q];
                return (int)std::min<int64_t>(std::min<int64_t>(L->hs[q]->D, kmax), k + std::max(2, k / 4));
            };
            if (npar == 1) {
                extend(cand[0], target(cand[0]), s, v0s[0], wss[0], olds[0]);
                ++L->calls;
                free_old();
                continue;
            }
            std::vector<std::exception_ptr> errs((size_t)npar);
            std::vector<std::thread> pool;
            for (int t = 0; t < npar; ++t)
                pool.emplace_back([&, t] {
                    try {
                        DeviceGuard g(L->device);
                        extend(cand[t], target(cand[t]), streams[t], v0s[t], wss[t], olds[t]);
                    } catch (...) {
                        errs[t] = std::current_exception();
                    }
                });
            for (auto &th : pool) th.join();
            free_old();
            for (auto &e : errs)
                if (e) std::rethrow_exception(e);
            L->calls += npar;
        }
    } catch (...) {
        for (auto &st : streams) (void)hipStreamSynchronize(st);
        for (auto &st : streams) (void)hipStreamDestroy(st);
        free_old();
        throw;
    }
    for (auto &st : streams) ED_HIP(hipStreamSynchronize(st));
    for (auto &st : streams) (void)hipStreamDestroy(st);
    DevMem v0, ws;
    L->threshold = kth_lowest(L->energies, K);
    for (int q = 0; q < nsec; ++q)  // one-level sectors: the energy is known, the vector not yet
        if (L->nvec[q] == 0 && L->energies[q][0] <= L->threshold) {
            extend(q, 1, s, v0, ws, olds[0]);
            ++L->calls;
        }
    free_old();
    for (int q = 0; q < nsec; ++q) {
        if (capped[q]) L->capped.push_back(q);
        for (int i = 0; i < (int)L->energies[q].size(); ++i)
            if (L->energies[q][i] <= L->threshold) L->levels.push_back({L->energies[q][i], q, i});
    }
    std::sort(L->levels.begin(), L->levels.end(), [](const ed_levels_s::Level &a, const ed_levels_s::Level &b) {
        return a.E < b.E || (a.E == b.E && (a.s < b.s || (a.s == b.s && a.i < b.i)));
    });
    ED_HIP(hipStreamSynchronize(s));
}

}  // namespace ed

using namespace ed;

extern "C" ed_status ed_lowest_levels(int nsec, const ed_ham_t *hs, int K, int kmax, const ed_lanczos_opts *opts,
                                      uint64_t seed, ed_levels_t *out, void *stream) {
    return guard([&] {
        if (!out) fail(ED_EINVAL, "ed_lowest_levels: out is NULL");
        *out = nullptr;
        if (nsec < 1 || !hs) fail(ED_EINVAL, "ed_lowest_levels: no sectors");
        if (K < 1 || kmax < 1 || kmax > 200) fail(ED_EINVAL, "ed_lowest_levels: need K >= 1 and 1 <= kmax <= 200");
        for (int q = 0; q < nsec; ++q) {
            if (!hs[q]) fail(ED_EINVAL, "ed_lowest_levels: NULL handle %d", q);
            if (hs[q]->prec != hs[0]->prec || hs[q]->device != hs[0]->device)
                fail(ED_EINVAL, "ed_lowest_levels: sectors must share one precision and one GPU");
        }
        DeviceGuard g(hs[0]->device);
        ed_levels_s *L = new ed_levels_s();
        try {
            L->device = hs[0]->device;
            lowest_levels(L, nsec, hs, K, kmax, opts, seed, (hipStream_t)stream);
        } catch (...) {
            delete L;
            throw;
        }
        *out = L;
    });
}

extern "C" ed_status ed_levels_info(ed_levels_t L, int *nlevels, int *calls, int *ncapped, double *threshold) {
    return guard([&] {
        if (!L) fail(ED_EINVAL, "ed_levels_info: NULL handle");
        if (nlevels) *nlevels = (int)L->levels.size();
        if (calls) *calls = L->calls;
        if (ncapped) *ncapped = (int)L->capped.size();
        if (threshold) *threshold = L->threshold;
    });
}

extern "C" ed_status ed_levels_get(ed_levels_t L, double *E, int32_t *sector, int32_t *index) {
    return guard([&] {
        if (!L) fail(ED_EINVAL, "ed_levels_get: NULL handle");
        for (size_t i = 0; i < L->levels.size(); ++i) {
            if (E) E[i] = L->levels[i].E;
            if (sector) sector[i] = L->levels[i].s;
            if (index) index[i] = L->levels[i].i;
        }
    });
}

extern "C" ed_status ed_levels_capped(ed_levels_t L, int32_t *sectors) {
    return guard([&] {
        if (!L || !sectors) fail(ED_EINVAL, "ed_levels_capped: NULL argument");
        for (size_t i = 0; i < L->capped.size(); ++i) sectors[i] = L->capped[i];
    });
}

extern "C" ed_status ed_levels_vector(ed_levels_t L, int sector, int index, void *dst, void *stream) {
    return guard([&] {
        if (!L || !dst) fail(ED_EINVAL, "ed_levels_vector: NULL argument");
        if (sector < 0 || sector >= (int)L->hs.size() || index < 0 || index >= L->nvec[sector])
            fail(ED_EINVAL, "ed_levels_vector: no vector for level %d of sector %d", index, sector);
        DeviceGuard g(L->device);
        const ed_ham_s *h = L->hs[sector];
        const size_t bytes = (size_t)h->D * (h->prec == ED_FP64 ? 8 : 4);
        ED_HIP(hipMemcpyAsync(dst, (char *)L->vecs[sector]->p + (size_t)index * bytes, bytes, hipMemcpyDeviceToDevice,
                              (hipStream_t)stream));
    });
}

extern "C" void ed_levels_free(ed_levels_t L) {
    if (!L) return;
    try {
        DeviceGuard g(L->device);
        (void)hipDeviceSynchronize();
        delete L;
    } catch (...) {
    }
}
