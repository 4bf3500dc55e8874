/*
 * ed.h -- C interface of the MI355X exact-diagonalization hot path.
 *
 * The library solves the eigenvalue problem the paper states for the impurity
 * Hamiltonian (Section 2, after Eq. 3: only the lowest eigenstates are needed)
 * by the iterative scheme of Section 3 (repeated multiplication of H by a trial
 * vector inside a Lanczos / Arnoldi iteration), one fixed (N_up, N_dn) sector at
 * a time, with the whole sector held by one GPU.  H is never stored: its
 * elements are evaluated when needed, the alternative the paper proposes at the
 * end of Section 3.2.
 *
 * Conventions
 *  - Ns <= 32 sites.  Spin-up site i is fermion mode i, spin-down site i is mode
 *    Ns+i (all up modes precede all down modes in the Jordan-Wigner order).
 *  - A one-spin basis state is an Ns-bit string with N_sigma bits set.  Its rank
 *    is its position in ascending numeric order (combinatorial number system).
 *  - A sector vector has D = D_up * D_dn elements; element (r_up, r_dn) is at
 *    flat index r_up * D_dn + r_dn (the down index is contiguous).
 *  - Vector element type is set per Hamiltonian: ED_FP64 (double) or ED_FP32
 *    (float storage and arithmetic in H.v; every Lanczos reduction, the
 *    tridiagonal eigenproblem and the final Rayleigh quotient are FP64).
 *
 * Ownership: handles are created and freed by the library.  Every vector and
 * workspace pointer is device memory owned by the caller (e.g. a torch tensor's
 * data pointer); small outputs (dimensions, eigenvalues, info) are host memory.
 * `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *
 * Errors: every call returns an ed_status; nothing is thrown across this
 * interface.  The message of the last failure on the calling thread is returned
 * by ed_last_error().  ED_EINVAL: bad argument (detailed below per call);
 * ED_ENOMEM: tables or workspace do not fit; ED_EDEVICE: a HIP runtime error;
 * ED_ENOCONV: iteration limit reached (best estimates are still written);
 * ED_EUNSUPPORTED: a valid model the library has no kernel for.
 */
#ifndef ED_H
#define ED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ED_OK = 0,
    ED_EINVAL = 1,
    ED_ENOMEM = 2,
    ED_EDEVICE = 3,
    ED_ENOCONV = 4,
    ED_EUNSUPPORTED = 5
} ed_status;

enum { ED_FP64 = 0, ED_FP32 = 1 };
enum { ED_SPIN_UP = 0, ED_SPIN_DN = 1 };
/* Four-fermion impurity terms of the multi-orbital Hamiltonian (Section 4). */
enum { ED_SPIN_FLIP = 1, ED_PAIR_HOP = 2, ED_UD_GENERAL = 3, ED_UU_GENERAL = 4, ED_DD_GENERAL = 5 };

typedef struct ed_basis_s *ed_basis_t;
typedef struct ed_ham_s *ed_ham_t;
typedef struct ed_levels_s *ed_levels_t;

/* Version string of the library build. */
const char *ed_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *ed_last_error(void);

/* ------------------------------------------------------------ sector basis --
 * ed_basis: the (N_up, N_dn) sector of an Ns-site model, the block structure
 * behind every dimension the paper quotes (Introduction; Table 1).  The two
 * one-spin bases are generated on the current GPU by combinatorial unranking.
 * EINVAL: Ns outside [1, 32], Nup or Ndn outside [0, Ns], out NULL.
 * ENOMEM: D_up or D_dn above 2^31 - 1. */
ed_status ed_basis(int Ns, int Nup, int Ndn, ed_basis_t *out);

/* Dimensions D_up = C(Ns, Nup), D_dn = C(Ns, Ndn), D = D_up * D_dn.
 * Any output pointer may be NULL. */
ed_status ed_basis_dims(ed_basis_t b, int64_t *Dup, int64_t *Ddn, int64_t *D);

/* Copy one spin's states (ascending, i.e. in rank order) to HOST memory
 * host_out[D_sigma].  EINVAL: spin not 0/1 or host_out NULL. */
ed_status ed_basis_states(ed_basis_t b, int spin, uint32_t *host_out);

/* Rank n bit strings (DEVICE arrays): ranks[i] = position of states[i] in the
 * spin's ascending basis, or -1 if its popcount is not N_sigma or it has bits
 * at or above Ns.  Asynchronous on stream. */
ed_status ed_basis_rank(ed_basis_t b, int spin, const uint32_t *states, int64_t n,
                        int64_t *ranks, void *stream);

void ed_basis_free(ed_basis_t b);

/* ----------------------------------------------------------- Hamiltonian ----
 * The operator whose matrix-vector product is the hot loop (Section 3.1,
 * Listing 1), given by coefficient arrays that cover Eq. (1) (Hubbard), Eq. (2)
 * (Anderson impurity) and the multi-orbital impurity Hamiltonian of Section 4:
 *
 *   H = sum_{s,i} eps[s*Ns+i] n_is
 *     + sum_{s, i != j} hop[(s*Ns+i)*Ns+j] c+_is c_js
 *     + sum_{i,j} w_ud[i*Ns+j] n_i,up n_j,dn
 *     + sum_{s, i<j} w_ss[(s*Ns+i)*Ns+j] n_is n_js
 *     + sum_t x[t].coef * X_t
 *
 * with X_t the spin-flip string  d+_{m up} d_{m dn} d+_{m' dn} d_{m' up}  or the
 * pair-hopping string  d+_{m up} d+_{m dn} d_{m' up} d_{m' dn}, written exactly
 * as in the paper (so the Kanamori term -J'[...] has coef = -J'), or
 * (ED_UD_GENERAL) the general opposite-spin two-body string
 * c+_{m up} c+_{m' dn} c_{l dn} c_{k up}: the element U_{m m' k l} of a full
 * U-matrix, whose other non-diagonal elements Section 4 closes on, or
 * (ED_UU_GENERAL, ED_DD_GENERAL) the same-spin string c+_{m s} c+_{m' s} c_{l s} c_{k s}.
 * Requirements (else EINVAL): every value finite; hop[s] symmetric with a zero
 * diagonal (on-site energies belong in eps); w_ss zero on and below the
 * diagonal; for x of type ED_SPIN_FLIP or ED_PAIR_HOP: m != m', both < Ns, the
 * list Hermitian (the summed coefficient of (type, m, m') equals that of
 * (type, m', m)); for ED_UD_GENERAL: m, m', k, l < Ns (any may coincide; k = m
 * or l = m' give density-assisted terms) and the summed coefficient of
 * (m, m', k, l) equal to that of (k, l, m, m'); for ED_UU/DD_GENERAL: indices
 * < Ns, m != m', k != l, {m, m'} != {k, l} (density terms belong in w_ss) and
 * the same Hermitian pairing after ordering each pair (a swap is a sign).  Off-diagonal w_ud entries may touch at most 8 sites
 * (else EUNSUPPORTED).  Input arrays are read during the call only.
 */
typedef struct {
    int32_t type;   /* ED_SPIN_FLIP, ED_PAIR_HOP, ED_UD_GENERAL, ED_UU_GENERAL, ED_DD_GENERAL */
    int32_t m;
    int32_t mp;
    double coef;
    int32_t k;      /* general terms only (ignored otherwise) */
    int32_t l;      /* general terms only (ignored otherwise) */
} ed_xterm;

typedef struct {
    int32_t Ns;
    const double *eps;    /* [2*Ns]        */
    const double *hop;    /* [2*Ns*Ns]     */
    const double *w_ud;   /* [Ns*Ns]       */
    const double *w_ss;   /* [2*Ns*Ns]     */
    int32_t n_x;
    const ed_xterm *x;    /* [n_x], may be NULL when n_x == 0 */
} ed_params;

/* Build the per-spin tables of H for sector b on the current GPU (the paper's
 * "setup" phase, T_setup in Table 1, in matrix-free form).  precision is ED_FP64
 * or ED_FP32.  The handle keeps its own copy of the basis dimensions; b may be
 * freed afterwards. */
ed_status ed_ham_create(const ed_params *p, ed_basis_t b, int precision, ed_ham_t *out);

ed_status ed_ham_dims(ed_ham_t h, int64_t *Dup, int64_t *Ddn, int64_t *D);

/* Number of entries of one spin's hop table. */
ed_status ed_hop_table_size(ed_ham_t h, int spin, int64_t *nnz);

/* Export one spin's hop table to HOST arrays, CSR over source ranks:
 * off[D_sigma+1]; entries off[r]..off[r+1]-1 hold the target rank, the fermion
 * sign (+1/-1) and the amplitude h_ij of  h_ij c+_i c_j |r>, in ascending target
 * order.  Any of tgt/sign/amp may be NULL. */
ed_status ed_hop_table(ed_ham_t h, int spin, int64_t *off, int32_t *tgt, int8_t *sign,
                       double *amp);

/* y = H x (overwrite) for DEVICE vectors of D elements of the handle's
 * precision.  Asynchronous on stream.  EINVAL: NULL pointers or x == y. */
ed_status ed_apply_H(ed_ham_t h, const void *x, void *y, void *stream);

/* Schedule control.  The apply has several compiled schedules (rows per
 * workgroup, workgroup size, LDS staging of rows); the first ed_apply_H call on a
 * handle times every one that fits on the caller's x and y (synchronously) and
 * keeps the fastest (the environment variable ED_APPLY_VARIANT=<n> forces one).
 * These calls run or query a given schedule, e.g. to test each against a
 * reference.  ed_apply_H_variant returns EINVAL for a schedule that does not fit. */
int ed_apply_variant_count(void);
const char *ed_apply_variant_name(int variant);
int ed_apply_variant_fits(ed_ham_t h, int variant);
int ed_apply_current_variant(ed_ham_t h);
ed_status ed_apply_H_variant(ed_ham_t h, int variant, const void *x, void *y, void *stream);

/* FP64-accurate Rayleigh quotient and residual of a DEVICE vector x stored in
 * the handle's precision: rq = <x,Hx>/<x,x>, resid = ||Hx - rq x|| / ||x||, with
 * H x evaluated in FP64 arithmetic and never stored.  Synchronous. */
ed_status ed_rayleigh(ed_ham_t h, const void *x, double *rq, double *resid, void *stream);

/* ed_rayleigh for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * result, with the per-workgroup partial sums in a static device array of
 * 2^18 (a, b) pairs (4 MiB per GPU, held until the process ends) instead of a
 * buffer the handle allocates.  The array holds D_up x (number of LDS windows
 * of the down basis) pairs at most: EINVAL beyond that (use ed_rayleigh).  No
 * device memory is allocated or freed.  Every call on one GPU shares that
 * GPU's array, so calls that overlap on one GPU (other threads, other streams)
 * race; the partials are overwritten in full by each call, nothing needs to
 * start at zero.  Synchronous. */
ed_status ed_rayleigh_noalloc(ed_ham_t h, const void *x, double *rq, double *resid, void *stream);

/* Fill a DEVICE vector with n numbers of the counter-based SplitMix64 stream
 * `seed` (element i uses output i, or outputs 2i and 2i+1): dist 0 = uniform on
 * [-1, 1), dist 1 = standard normal (Box-Muller).  precision ED_FP64 or ED_FP32
 * (the FP32 value is the round-to-nearest cast of the FP64 one). */
ed_status ed_fill_random(void *x, int64_t n, uint64_t seed, int dist, int precision,
                         void *stream);

/* Frees h and the grouped twin it owns; a no-op on the twin itself. */
void ed_ham_free(ed_ham_t h);

/* ------------------------------------------------------- grouped order ------
 * The paper's solver distributes H by rows; here the vector stays on one GPU
 * and the work is tiled so that the data a tile reads stays in the caches.
 * When the one-spin move graph of either spin (hops and same-spin two-body
 * moves) has several connected components -- the multi-orbital impurity of
 * Section 4 and the Anderson impurity of Eq. 2 with their bath levels attached
 * to one orbital each -- ed_ham_create also builds the same operator in a
 * grouped basis order: the states of each spin ordered by component
 * (components by their lowest rank); within a component, states with more
 * moves first, then by rank (so the tile kernels' hop-table slices hold states
 * of similar hop counts), or by rank alone when the environment variable
 * ED_GROUP_ORDER=rank is set at ed_ham_create.  Every hop then stays inside an
 * (up component x down component) tile of the vector.
 * The solvers iterate in that order by default (ed_lanczos_opts.layout) and
 * convert their vectors at the boundary; these calls expose it.
 *
 * ed_ham_grouped: *grouped = the twin handle (owned by h: do not free it; it
 * lives as long as h), h itself if h is a twin, or NULL when both move graphs
 * are connected (then the rank order is the only one).  The twin accepts every
 * call a handle does (ed_apply_H, the solvers, ...), with vectors in its order:
 * element (p_up, p_dn) at p_up * D_dn + p_dn, p the position in the grouped
 * order of that spin. */
ed_status ed_ham_grouped(ed_ham_t h, ed_ham_t *grouped);

/* rank_of_position[p] (HOST, D_sigma entries) = combinatorial rank of the state
 * at position p of the grouped order of a twin handle g.  EINVAL: g not a twin,
 * spin not 0/1, NULL. */
ed_status ed_grouped_order(ed_ham_t g, int spin, int32_t *rank_of_position);

/* DEVICE vectors of D elements of the handle's precision: y = x converted from
 * rank order to the grouped order (ed_to_grouped) or back (ed_from_grouped).
 * h: a handle with a twin, or the twin.  Asynchronous on stream.  EINVAL: no
 * grouped order, NULL or aliasing vectors. */
ed_status ed_to_grouped(ed_ham_t h, const void *x, void *y, void *stream);
ed_status ed_from_grouped(ed_ham_t h, const void *x, void *y, void *stream);

/* ------------------------------------------------------------ eigensolvers --
 * Lanczos iteration (Section 3) with full reorthogonalisation against every
 * stored basis vector, FP64 reductions, a tridiagonal eigensolve on the GPU and
 * restarts when the stored basis is full. */
typedef struct {
    int32_t max_iter;     /* total Lanczos steps over all restarts (default 600)    */
    int32_t max_basis;    /* stored basis vectors before a restart; 0 (default) =
                             planned: the largest basis of at most 120 vectors whose
                             workspace fits the free device memory (less a reserve
                             of max(1 GiB, 2 % of the device)) in ed_workspace_bytes,
                             or the given workspace in the solvers                  */
    double tol;           /* stop when |beta_j s_j| <= tol * max(|theta|, 1) (1e-10) */
    int32_t reorth;       /* Gram-Schmidt per step (default 2): 0 = three-term only, 1 = one
                             full pass, 2 = two full passes (CGS2), 3 = the two projections
                             of CGS2 from one read of the basis, the second one's
                             coefficients through the Gram matrix of the stored vectors
                             (ground state; with locked vectors it falls back to 2)    */
    int32_t check_every;  /* steps between convergence tests (default 4)            */
    int32_t refine;       /* 1: report the FP64 Rayleigh quotient of the Ritz vector */
    int32_t keep;         /* restart: 0 = from the current Ritz vector alone (default);
                             k >= 1 = implicit restart keeping k vectors (the unwanted
                             Ritz values applied as exact shifts to the tridiagonal
                             matrix, which stays tridiagonal), for the ground state
                             and for each eigenpair of ed_arnoldi_lowest on its
                             deflated space; k <= 16, k < max_basis <= 256           */
    int32_t layout;       /* 0 (default): iterate in the grouped basis order when the
                             Hamiltonian has one (ed_ham_grouped), converting the
                             start vector and the returned vectors; 1: rank order    */
} ed_lanczos_opts;

typedef struct {
    int32_t iters;        /* Lanczos steps taken (all restarts)                  */
    int32_t restarts;
    int32_t converged;    /* 1 if the residual test was met                     */
    int32_t basis_used;   /* largest number of stored basis vectors             */
    double residual;      /* ||H psi - E psi|| / ||psi|| of the returned vector  */
    double ritz;          /* Ritz value from the tridiagonal matrix             */
    double rq_fp64;       /* FP64 Rayleigh quotient (equals the reported E)     */
    double gap_lower;     /* eta: second Ritz value of the last cycle minus its
                             residual bound, taken as a lower bound on the next
                             eigenvalue (of the deflated operator); NaN if none   */
    double e_lower;       /* Kato-Temple lower bound E - residual^2 / (eta - E);
                             [e_lower, E] holds the eigenvalue when eta is a true
                             lower bound on the next one; NaN if eta <= E         */
    double traffic;       /* algorithmic bytes the run's kernels moved: per H.v x read
                             and y written; per Gram-Schmidt pass the projected
                             vectors read and Y read and written; every restart,
                             Ritz, normalisation and refinement pass likewise      */
} ed_info;

/* Fill opts with the defaults above. */
void ed_lanczos_defaults(ed_lanczos_opts *opts);

/* Bytes of DEVICE workspace ed_lanczos_ground (k = 1) or ed_arnoldi_lowest (k)
 * needs with these options (with max_basis = 0, for the basis planned from the
 * free device memory; the solver called with that workspace plans the same
 * basis from its size).  EINVAL: k < 1 or k > D.  ENOMEM: with max_basis = 0,
 * even the smallest usable basis exceeds the free device memory; with an
 * explicit max_basis, the workspace exceeds the device's capacity. */
ed_status ed_workspace_bytes(ed_ham_t h, const ed_lanczos_opts *opts, int k, size_t *bytes);

/* Lowest eigenvalue of the sector.  v0: DEVICE start vector (D elements, any
 * nonzero norm).  ws: DEVICE workspace of ws_bytes >= ed_workspace_bytes(...,1).
 * psi0: optional DEVICE output for the normalised ground-state vector.  E0 is
 * the FP64 Rayleigh quotient of that vector when opts->refine, else the Ritz
 * value.  Synchronous on stream.  ED_ENOCONV: max_iter reached (E0, psi0 and
 * info still hold the best estimate).  A Krylov breakdown (exact invariant
 * subspace) is a success. */
ed_status ed_lanczos_ground(ed_ham_t h, const ed_lanczos_opts *opts, const void *v0,
                            void *ws, size_t ws_bytes, double *E0, void *psi0,
                            ed_info *info, void *stream);

/* The k lowest eigenvalues, counted with multiplicity, ascending, into HOST
 * evals[k]; optional DEVICE evecs[k][D].  Each eigenpair is found by a restarted
 * Lanczos run on H restricted to the orthogonal complement of the pairs already
 * locked (explicit deflation), which also recovers every copy of a degenerate
 * eigenvalue: the first run starts from v0, every later one from a fresh
 * pseudo-random vector (SplitMix64 normal stream 0x5EED0000 + index), because
 * one start vector's Krylov space holds a single vector per distinct eigenvalue.  info[k] (HOST, may be NULL) per eigenpair. */
ed_status ed_arnoldi_lowest(ed_ham_t h, int k, const ed_lanczos_opts *opts, const void *v0,
                            void *ws, size_t ws_bytes, double *evals, void *evecs,
                            ed_info *info, void *stream);

/* ed_arnoldi_lowest continued: evecs[0..k0) (DEVICE [k][D], required) already
 * hold converged orthonormal eigenvectors of h, e.g. from an earlier call, and
 * evals[0..k0) their values; eigenpairs k0..k-1 are computed on the space
 * orthogonal to them (the same explicit deflation), so a caller can raise k
 * without recomputing the levels it has.  Eigenpairs e >= 1 start from the
 * counter-based random stream, so v0 only has to be a valid vector.
 * info[k0..k) is filled.  With k0 = 0 this is ed_arnoldi_lowest.  EINVAL: k0
 * outside [0, k), evecs NULL with k0 > 0, a given vector of zero norm; the
 * rest as ed_arnoldi_lowest. */
ed_status ed_arnoldi_lowest_more(ed_ham_t h, int k0, int k, const ed_lanczos_opts *opts, const void *v0,
                                 void *ws, size_t ws_bytes, double *evals, void *evecs, ed_info *info,
                                 void *stream);

/* Bytes of DEVICE workspace ed_lanczos_tridiag needs for m steps with these
 * options: m + 1 basis vectors, or 3 with the three-term recurrence
 * (reorth = 0), which only ever holds the two latest vectors and the new one.
 * EINVAL: m outside [1, min(D, 1022)]. */
ed_status ed_tridiag_workspace_bytes(ed_ham_t h, const ed_lanczos_opts *opts, int m, size_t *bytes);

/* Tridiagonal Lanczos coefficients of the Krylov space of v0 (no restart):
 * m steps with the reorthogonalisation of opts->reorth (opts->max_basis and
 * keep are ignored).  alpha[0..m), beta[0..m) HOST outputs with beta[j] the
 * coupling of steps j and j+1; *steps = k <= m (fewer when the Krylov space is
 * exhausted; then beta[k-1] = 0); *v0_norm2 = ||v0||^2.  These are the
 * continued-fraction coefficients of <v0|(z - H)^-1|v0>, the form in which the
 * impurity Green function of Eq. 3 is evaluated.  ws: DEVICE workspace of at
 * least ed_tridiag_workspace_bytes(h, opts, m).  Synchronous.
 * EINVAL: m outside [1, min(D, 1022)], NULL arguments, v0 zero. */
ed_status ed_lanczos_tridiag(ed_ham_t h, const ed_lanczos_opts *opts, const void *v0, int m, void *ws,
                             size_t ws_bytes, double *alpha, double *beta, int *steps, double *v0_norm2,
                             void *stream);

/* y = c+_{site,spin} x (dagger = 1) or c_{site,spin} x (dagger = 0): x is a
 * DEVICE vector of sector src, y of sector dst, which must hold one electron
 * more (dagger) or less of that spin and the same number of the other spin,
 * with the same Ns and precision.  The fermion sign follows the mode order of
 * the Conventions (all up modes first).  These are the matrix elements
 * <mu|c+_sigma|nu> of Eq. 3.  Asynchronous on stream.  EINVAL: sectors that do
 * not match, site outside [0, Ns), NULL or aliasing vectors. */
ed_status ed_apply_ladder(ed_ham_t src, ed_ham_t dst, int spin, int site, int dagger, const void *x, void *y,
                          void *stream);

/* Continued fraction on the host, ACCUMULATED into g: g(z) += weight * norm2 /
 * (z - s(alpha_0 - e0) - beta_0^2 / (z - s(alpha_1 - e0) - ...)) over k levels,
 * for nz complex z (z_re, z_im HOST arrays), s = +1 for the particle part
 * <phi|(z - (H - e0))^-1|phi> and -1 for the hole part <phi|(z + (H - e0))^-1|phi>.
 * g_re, g_im: HOST [nz], zeroed by the caller before the first term.  EINVAL:
 * NULL arrays, k < 1, sign not +-1, non-finite weight or norm2. */
ed_status ed_green_cf(const double *alpha, const double *beta, int k, double norm2, double e0, int sign,
                      double weight, const double *z_re, const double *z_im, int nz, double *g_re, double *g_im);

/* Boltzmann weights of Eq. 3 on the host: w[i] = exp(-beta (E[i] - E_min)) / Z
 * for the n computed levels E[0..n) (any sectors), where levels whose share
 * falls below cutoff get w = 0 and Z sums the kept ones, so the kept weights
 * add to 1 and the Green function keeps its total spectral weight.  The levels
 * at E_min are always kept (a g-fold degenerate lowest level has shares of
 * 1/g or less, which a cut above that would otherwise remove).  *kept:
 * number of nonzero weights.  The temperature Green function is then
 * sum_i w[i] G_i(z), each G_i the zero-temperature one of level i.  EINVAL:
 * NULL arrays, n < 1, beta not in (0, inf), cutoff not in [0, 1), E non-finite. */
ed_status ed_boltzmann_weights(const double *E, int n, double beta, double cutoff, double *w, int *kept);

/* ---------------------------------------------------- lowest levels --------
 * The K lowest levels over nsec sectors, counted with multiplicity: the
 * thermal set the finite-temperature sum of Eq. 3 runs over (the paper's DMFT
 * iteration at N_s = 12 needs the 300 lowest states, end of Section 3.2).
 * Every sector's lowest level comes from one ed_lanczos_ground_batched run;
 * then, in rounds, while some sector with levels left has its highest computed
 * level at or below the K-th lowest found so far, the (up to 8) such sectors
 * whose highest computed levels are lowest get more (k -> k + max(2, k/4), at
 * most min(D, kmax)) by ed_arnoldi_lowest_more on top of their converged
 * vectors, concurrently on streams of their own (one at a time when a sector is
 * large).  A sector's uncomputed levels lie above its highest computed one, so
 * no level that could be among the K lowest is skipped.  Sector q's start vectors come from the
 * SplitMix64 normal stream seed + q.  hs: nsec handles of one precision on one
 * GPU; opts: the Lanczos options of every run (max_basis = 0 plans each run
 * against the free device memory).  *out: a result handle that owns the
 * eigenvectors it found (device memory the library allocates; ed_levels_free
 * releases it).  Synchronous.  EINVAL: nsec < 1, K < 1, kmax outside
 * [1, 200], NULL or mismatched handles. */
ed_status ed_lowest_levels(int nsec, const ed_ham_t *hs, int K, int kmax, const ed_lanczos_opts *opts,
                           uint64_t seed, ed_levels_t *out, void *stream);

/* Counts of a result: levels at or below the threshold (the K-th lowest; more
 * than K when a multiplet straddles it), calls of the eigensolver, sectors
 * stopped at kmax while their highest level was still at or below the
 * threshold (they may hold more levels), and the threshold itself (+inf when
 * fewer than K levels exist).  Any output may be NULL. */
ed_status ed_levels_info(ed_levels_t L, int *nlevels, int *calls, int *ncapped, double *threshold);

/* The levels, ascending: energy, sector (index into hs) and index of the level
 * within its sector (discovery order), HOST arrays of nlevels; any may be NULL. */
ed_status ed_levels_get(ed_levels_t L, double *E, int32_t *sector, int32_t *index);

/* Sector indices of the capped sectors, HOST [ncapped]. */
ed_status ed_levels_capped(ed_levels_t L, int32_t *sectors);

/* Copy the normalised eigenvector of level `index` of `sector` (rank order,
 * D elements of the sector's precision) to DEVICE memory dst.  Asynchronous on
 * stream.  EINVAL: no vector for that level. */
ed_status ed_levels_vector(ed_levels_t L, int sector, int index, void *dst, void *stream);

void ed_levels_free(ed_levels_t L);

/* ------------------------------------------------------- sector batching ----
 * All sectors of one impurity problem at once (the paper's solver treats the
 * sectors of the block structure one after another, and its closing remarks
 * of Section 3.2 trace the load imbalance of equal-size splits of the matrix to
 * rows with unequal work: here each sector's share of every batched kernel is
 * sized by its own dimension and row work): one restarted Lanczos per
 * sector, every running sector advanced by the same replayed step -- a fixed
 * sequence of batched kernels captured once in a hipGraph -- while each
 * sector keeps its own step index, so sectors converge (masked off on the
 * device), fill their basis and restart independently.  A sector whose basis
 * is full waits until the host restarts it (at most check_every steps later):
 * implicitly with opts->keep vectors when keep > 0 (exact shifts, as
 * ed_lanczos_ground), else from its Ritz vector; all waiting sectors restart in
 * one batched combination.  opts->reorth 0..3 as for ed_lanczos_ground.  The
 * apply runs over row tiles of about T output elements per workgroup, T picked
 * on the first step by timing candidates (ED_BATCH_TILE=<T> forces one); the
 * vector kernels run over chunks of at most 8192 elements of one sector.
 * hs: nsec handles of one precision on one GPU, each with D < 2^31.  v0s:
 * optional HOST array of nsec DEVICE start vectors (NULL: sector i starts from
 * the SplitMix64 normal stream seed + i).  E0: HOST [nsec] lowest eigenvalue per
 * sector (FP64 Rayleigh quotient of the Ritz vector when opts->refine).  info:
 * HOST [nsec] or NULL (iters: steps of that sector; gap_lower, e_lower: NaN).  ws: DEVICE
 * workspace of at least ed_batched_workspace_bytes.  max_basis = 0 gives 60
 * vectors per sector (at most 1000; keep is used with at most 256).  max_iter
 * bounds the replayed steps.  Synchronous.  ED_ENOCONV if some sector was
 * still unconverged at max_iter (all E0 still written). */
ed_status ed_batched_workspace_bytes(int nsec, const ed_ham_t *hs, const ed_lanczos_opts *opts,
                                     size_t *bytes);
ed_status ed_lanczos_ground_batched(int nsec, const ed_ham_t *hs, const ed_lanczos_opts *opts,
                                    const void *const *v0s, uint64_t seed, void *ws, size_t ws_bytes,
                                    double *E0, ed_info *info, void *stream);
int64_t ed_batched_last_tile(void);
/* Figures of the last batched run in this process (not thread-safe): steps =
 * replayed graph steps, restart_events = batched restart launches, bytes =
 * algorithmic bytes moved (per step and sector: x read, y written, and per
 * projection pass the nv projected vectors read twice plus Y read twice and
 * written once; per restart the inputs read and outputs written).  Any output
 * may be NULL. */
void ed_batched_last_stats(int64_t *steps, int64_t *restart_events, double *bytes);

#ifdef __cplusplus
}
#endif

#endif /* ED_H */
