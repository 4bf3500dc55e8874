// Internal declarations of the HIP exact-diagonalization library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ed.h"

namespace ed {

// ----------------------------------------------------------------- errors --
struct Failure {
    ed_status st;
};
[[noreturn]] void fail(ed_status st, const char *fmt, ...);
[[noreturn]] void throw_hip(hipError_t e, const char *what, const char *file, int line);
void clear_error();

#define ED_HIP(call)                                                   \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) ::ed::throw_hip(e_, #call, __FILE__, __LINE__); \
    } while (0)

#define ED_LAUNCH_CHECK() ED_HIP(hipGetLastError())

// Runs body, translating internal failures into a status code.
template <class F>
ed_status guard(F &&body) {
    try {
        clear_error();
        body();
        return ED_OK;
    } catch (const Failure &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        try { fail(ED_ENOMEM, "host allocation failed"); } catch (const Failure &f) { return f.st; }
    } catch (...) {
        try { fail(ED_EDEVICE, "unexpected C++ exception"); } catch (const Failure &f) { return f.st; }
    }
    return ED_EDEVICE;
}

// Restores the caller's current device on exit.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        ED_HIP(hipGetDevice(&prev));
        if (prev != dev) ED_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

// Owned device allocation (library-internal tables only; vectors belong to the caller).
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() { release(); }
    void alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            fail(ED_ENOMEM, "device allocation of %zu bytes failed (%s)", n, hipGetErrorString(e));
        }
        bytes = n;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

inline unsigned grid_for(int64_t n, int block, int64_t cap = 1 << 20) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// --------------------------------------------------------------- binomials --
// C(n, k) for 0 <= n, k <= 32 on the host (all fit in 32 bits).
uint64_t binom_host(int n, int k);
void ensure_device_binomials();  // uploads the constant table on the current device
int64_t basis_rank_host(uint32_t s, int ns, int n);

// ------------------------------------------------------------------ basis --
struct BasisData {
    int ns = 0, n[2] = {0, 0};
    int64_t dim[2] = {0, 0};
    DevMem states[2];
};

}  // namespace ed

struct ed_basis_s {
    int device = 0;
    ed::BasisData b;
};

namespace ed {

// Plan of the grouped-order tile kernel for one (rows per tile, window size)
// choice: windows of whole down components, a per-window copy of the down hop
// table with window-local targets, and the tile-major work list.
struct TilePlan {
    int64_t key = 0;
    int nwin = 0, wmax = 0, namp = 0;
    int half = 0;      // 1: 16-bit entries (windows of at most 1024 states, at most 64 amplitudes)
    int64_t nitems = 0;
    DevMem win;        // int2 [nwin]: (first position, length)
    DevMem wsl_first;  // int32 [nwin + 1]: first slice of each window
    DevMem wsl_off;    // int32 [nslices + 1]: slice offsets in uint4 units
    DevMem wel4;       // uint4 [(slice, k, lane)]: four consecutive states per lane,
                       // window-local target (bits 0..19) | amplitude index (20..31);
                       // half: uint4 [(slice, pair of hops k, lane)], 16-bit entries
                       // target (bits 0..9) | amplitude index (10..15), words
                       // (hop 2k: states 0|1, 2|3; hop 2k+1: states 0|1, 2|3)
    DevMem amp64, amp32;
    DevMem items;      // int4 [nitems]
};

// ------------------------------------------------------------ spin tables --
// Tables of one spin species.  Arrays suffixed 64/32 hold FP64 / FP32 copies.
struct SpinTab {
    int ns = 0, n = 0;
    int64_t dim = 0, nnz = 0, nslices = 0;
    int max_hops = 0;
    DevMem states;            // uint32 [dim]
    DevMem off;               // int32 [dim+1]   CSR over source ranks
    DevMem tgt;               // int32 [nnz]     target rank, ascending per row
    DevMem sgn;               // int8  [nnz]
    DevMem amp;               // double [nnz]    h_ij (export)
    DevMem sa64, sa32;        // signed amplitude per entry
    DevMem ell_off;           // int32 [nslices+1] start (in entries) of each 64-state slice
    DevMem ell_tgt;           // int32 [ell_off[nslices]]  (slice, hop k, lane) -> target
    DevMem ell_sa64, ell_sa32;
    // packed sliced ELL: target rank (bits 0..19) | index into amp table (bits 20..31);
    // amp[0] = 0 for padding.  Built when dim <= 2^20 and <= 4095 distinct amplitudes.
    bool pk_ok = false;
    int namp = 0;
    DevMem ell_pk;            // uint32 [ell_off[nslices]]
    DevMem amp64, amp32;      // distinct signed amplitudes
    // the same packed entries with four consecutive states per lane (256-state
    // slices): ell4_off [nslices4+1] in uint4 units, ell4 uint4 [(slice, k, lane)]
    int64_t nslices4 = 0;
    DevMem ell4_off, ell4;
    DevMem ediag64, ediag32;  // one-spin diagonal piece: eps n + same-spin density terms
    DevMem cidx;              // uint8 [dim] bits of the state on the cross-term support
    int nmv = 0;              // number of move tables
    DevMem mv;                // int32 [nmv][dim] (target << 1 | sign bit) or -1
    std::vector<int> mv_src, mv_dst;  // move q: electron src -> dst
    // uint32 [nmv]: bit 31 set when move q's validity is a test on the word the
    // tile kernel holds per column (the folded cross-term index, or the state
    // bits without one): source bit (bits 0..7) set, destination bit (8..15) clear
    DevMem mvb;
    // down spin, when every move shifts the rank by -4..3: all moves of a state
    // in one word, 5 bits per move (valid << 4 | sign << 3 | shift + 4)
    bool mvp_ok = false;
    DevMem mvp;                        // uint32 [dim]
};

// Four-fermion term in factorised form: output (u, d) pulls x[up_mv(u), dn_mv(d)].
struct XTerm {
    int32_t up_mv;    // index into the up spin's move tables
    int32_t dn_mv;    // index into the down spin's move tables
    double amp;       // element = amp * s_up * s_dn
};

template <typename TA>
struct XTermDev {
    int32_t up_mv, dn_mv;
    TA amp;
};

// Apply kernel schedule: one of the compiled variants.
struct ApplyPlan {
    int variant = -1;   // index into the variant table; -1 = not tuned yet
};

}  // namespace ed

struct ed_ham_s {
    int device = 0;
    int prec = ED_FP64;
    int ns = 0, nup = 0, ndn = 0;
    int64_t dup = 0, ddn = 0, D = 0;
    ed::SpinTab sp[2];
    // cross term sum_ij w_ud[i][j] n_i,up n_j,dn
    int umode = 0;              // 0: no on-site part, 1: uniform U0 on umask, 2: per-site values
    uint32_t umask = 0;
    double U0 = 0.0;
    ed::DevMem usite64, usite32;  // [32]
    int koff = 0;               // number of sites carrying off-diagonal w_ud entries
    ed::DevMem xtab64, xtab32;  // [4^koff]
    // the whole cross term sum_ij w_ud[i][j] n_i,up n_j,dn as one table when
    // every nonzero w_ud entry lies on at most 4 sites: fk sites, per state the
    // bits on them (fcidx) and the 4^fk values
    int fk = -1;                // -1: no folded table
    std::vector<int> fk_sites;  // bit q of the folded index = occupation of fk_sites[q]
    ed::DevMem fcidx[2];
    ed::DevMem dn_fc32;         // uint32 [ddn]: fcidx[1] widened, four columns per 16-byte load
    ed::DevMem ftab64, ftab32;
    // four-fermion terms
    int nx = 0;
    std::vector<ed::XTerm> xterms;
    ed::DevMem xt64, xt32;      // XTermDev<double>/<float> [nx]
    // per up state: the four-fermion terms whose up move is allowed, as CSR
    // (source up rank, down move table, signed amplitude)
    ed::DevMem xl_off, xl_src, xl_tab, xl_amp64, xl_amp32;
    int xl_max = 0;             // largest list length
    ed::ApplyPlan plan;
    ed::DevMem redbuf;          // small FP64 reduction scratch owned by the handle
    size_t redbuf_doubles = 0;
    std::vector<uint32_t> dn_states_host;           // for the LDS window plan
    std::vector<std::pair<int64_t, ed::DevMem *>> windows;  // (capacity, device int2 list)
    std::vector<int> window_counts;
    // Grouped basis order.  On a handle built in that order (grouped = true)
    // the states of each spin are ordered by connected component of the
    // one-spin move graph (hops and same-spin two-body moves), components by
    // their lowest rank, states within a component by number of hops
    // (descending), then rank; every index of its
    // tables and vectors is a position in that order.  gperm[s][p] = rank of
    // position p, gipos[s][r] = position of rank r, comp_off[s] = component
    // boundaries.  A rank-order handle whose move graphs have several
    // components owns such a twin (`twin`), which the solvers run on.
    bool grouped = false;
    ed::DevMem gperm[2], gipos[2];
    std::vector<int32_t> comp_off[2];
    ed_ham_s *twin = nullptr;
    // tile-major, XCD-partitioned work lists of the grouped schedules:
    // (key, device int4 list of (first row, rows, window or band, 0), count)
    std::vector<std::pair<int64_t, ed::DevMem *>> items;
    std::vector<int64_t> item_counts;
    std::vector<ed::TilePlan *> tplans;
    ~ed_ham_s() {
        for (auto &w : windows) delete w.second;
        for (auto &w : items) delete w.second;
        for (auto *t : tplans) delete t;
        delete twin;
    }
};

namespace ed {

// Arguments of the matrix-free apply: everything by pointer, element type TA.
template <typename TX, typename TA>
struct ApplyArgs {
    const TX *x;
    TX *y;
    int64_t dup, ddn;
    // rows (spin up): CSR, read wave-uniformly
    const int32_t *up_off, *up_tgt;
    const TA *up_sa, *up_e;
    const uint32_t *up_st;
    const uint8_t *up_c;
    const int32_t *up_mv;
    // columns (spin down): sliced ELL and CSR
    const int32_t *dn_ell_off, *dn_ell_tgt;
    const TA *dn_ell_sa, *dn_e;
    const int32_t *dn_off, *dn_tgt;
    const TA *dn_sa;
    int nmv_dn;
    const uint32_t *dn_ell_pk;
    const int32_t *dn_ell4_off;
    const uint4 *dn_ell4;
    const TA *amp_tab;
    int namp;
    const uint32_t *dn_st;
    const uint8_t *dn_c;
    const int32_t *dn_mv;
    const uint32_t *dn_mvp;  // packed down move words, or nullptr
    const uint32_t *dn_mvb;  // per down move: validity test on the column word (SpinTab::mvb)
    // cross term
    int umode;
    uint32_t umask;
    TA U0;
    const TA *usite;
    int koff;
    const TA *xtab;
    // four-fermion terms
    int nx;
    const XTermDev<TA> *xt;
    const int32_t *xl_off, *xl_src, *xl_tab;
    const TA *xl_amp;
    // reductions (Rayleigh quotient / residual epilogues)
    double *partials;
    double theta;
    // down-spin windows staged in LDS: (first rank, length) per window
    const int2 *win;
    int nwin;
    int wmax;
    // optional work list (grouped schedules): workgroup b takes items[b] =
    // (first row, rows, window or band, 0); rows = 0 is an empty item
    const int4 *items;
    // grouped tile kernel: per-window slices of the down hop table
    const int32_t *wsl_first, *wsl_off;
    const uint4 *wel4;
    // folded cross-term table (fk < 0: none)
    int fk;
    const TA *ftab;
    const uint8_t *up_fc, *dn_fc;
    const uint32_t *dn_fc32;
};

// Build all tables of a Hamiltonian handle (tables.hip).
void build_tables(ed_ham_s *h, const ed_params *p, const BasisData &b);

// Launch the apply (apply.hip). mode: 0 = store y, 1 = RQ partials, 2 = residual partials.
void apply_launch(ed_ham_s *h, const void *x, void *y, hipStream_t s);
void apply_launch_variant(ed_ham_s *h, int variant, const void *x, void *y, hipStream_t s);
int apply_variant_count(const ed_ham_s *h);
const char *apply_variant_name(const ed_ham_s *h, int variant);
void rayleigh_fp64(ed_ham_s *h, const void *x, double *rq, double *resid, hipStream_t s);
void prepare_rayleigh(ed_ham_s *h);
int64_t rayleigh_pairs_cached(const ed_ham_s *h);
void rayleigh_on(ed_ham_s *h, const void *x, double *part, int64_t nb, double *rq, double *resid, hipStream_t s);

// Rank order <-> grouped order of a vector (layout.hip): dir 0 = to grouped.
void permute_vector(const ed_ham_s *g, const void *x, void *y, int dir, hipStream_t s);

// Deterministic FP64 reductions (lanczos.hip)
int reduce_blocks(int64_t n);

}  // namespace ed
