/*
 * ed_oracle.c -- plain, slow, literal FP64 reference for the exact-diagonalization
 * hot path.  TEST INFRASTRUCTURE ONLY: nothing in the product library links this
 * file; only tests/, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * What it computes, and where the paper defines it:
 *  - the many-electron basis of a fixed (N_up, N_dn) sector, as bit strings in
 *    ascending integer order (the sector decomposition behind the dimensions quoted
 *    in the Introduction and Table 1);
 *  - the Hamiltonian matrix of an arbitrary list of fermionic operator strings
 *    (Eq. 1 Hubbard, Eq. 2 Anderson impurity, the multi-orbital impurity Hamiltonian
 *    of Section 4), built by applying each string literally to every basis state
 *    with Jordan-Wigner signs;
 *  - the compressed-sparse-row format of Section 3.1 / Fig. 1 (row_ind of length
 *    nrows+1, col_ind and H_values of length nnz) from unsorted (row, col, value)
 *    triplets;
 *  - the CSR matrix-vector product of Listing 1 (rows split over OpenMP threads);
 *  - matrix-free generation of single rows, the alternative to storing the matrix
 *    that the paper names in its discussion of improvements (end of Section 3.2).
 *
 * Conventions (the paper does not fix them): fermion mode p < 2*Ns; spin-up site i
 * is mode i, spin-down site i is mode Ns+i, so all up modes precede all down modes.
 * A basis state is |w> = prod_{p ascending} (c+_p)^{n_p} |0>, hence
 *   c_p |w>  = (-1)^{#occupied modes below p} |w - p>,
 *   c+_p |w> = (-1)^{#occupied modes below p} |w + p>.
 * The flat index of (up rank r_u, down rank r_d) is r_u * D_dn + r_d.
 *
 * No blocking, fusion or reordering: every loop is the definition written out.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int popcount64(uint64_t x) { return __builtin_popcountll(x); }

/* ---------------------------------------------------------------- basis ---- */

/* All ns-bit strings with exactly n bits set, in ascending numeric order
 * (Gosper's hack: the next larger integer with the same popcount).
 * Writes them to out (if not NULL) and returns how many there are. */
int64_t orc_enumerate(int ns, int n, uint32_t *out)
{
    if (ns < 0 || ns > 32 || n < 0 || n > ns) return -1;
    if (n == 0) { if (out) out[0] = 0u; return 1; }
    uint64_t s = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    const uint64_t lim = 1ull << ns;
    int64_t c = 0;
    while (s < lim) {
        if (out) out[c] = (uint32_t)s;
        c++;
        uint64_t low = s & (~s + 1ull);
        uint64_t ripple = s + low;
        s = ripple | (((ripple ^ s) / low) >> 2);
    }
    return c;
}

/* Position of state s in the ascending list, or -1. Plain binary search. */
static int64_t find_state(const uint32_t *list, int64_t n, uint32_t s)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (list[mid] == s) return mid;
        if (list[mid] < s) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------- operator strings -- */

/* Apply the operator string op[0] op[1] ... op[nops-1] to |w> (the rightmost
 * operator acts first).  dag[q] != 0 means creation.  Returns 0 if the result is
 * the zero vector, else 1 with the new word and the accumulated sign. */
static int apply_string(uint64_t w, int nops, const int32_t *mode, const int8_t *dag,
                        uint64_t *w_out, int *sign_out)
{
    int sign = 1;
    for (int q = nops - 1; q >= 0; --q) {
        const uint64_t bit = 1ull << mode[q];
        const int occupied = (w & bit) != 0;
        if (dag[q]) { if (occupied) return 0; }
        else        { if (!occupied) return 0; }
        if (popcount64(w & (bit - 1ull)) & 1) sign = -sign;
        w ^= bit;
    }
    *w_out = w;
    *sign_out = sign;
    return 1;
}

/* Public wrapper so tests can exercise the Jordan-Wigner rule on its own. */
int orc_apply_string(uint64_t w, int nops, const int32_t *mode, const int8_t *dag,
                     uint64_t *w_out, int32_t *sign_out)
{
    int s = 0;
    int ok = apply_string(w, nops, mode, dag, w_out, &s);
    *sign_out = s;
    return ok;
}

typedef struct {
    int nterms;
    const double *coef;     /* [nterms] */
    const int64_t *op_off;  /* [nterms+1] offsets into mode/dag */
    const int32_t *mode;
    const int8_t *dag;
} terms_t;

/* ------------------------------------------------------------- H build ---- */

/* Forward application: column I of H is  sum_t coef_t * T_t |I>.
 * Pass 1 (out == NULL): returns the number of (row, col, value) triplets.
 * Pass 2: writes them, column by column, in term order.  Returns -2 if some
 * term leaves the sector (does not conserve N_up and N_dn). */
int64_t orc_build_coo(int ns,
                      int64_t dup, const uint32_t *up, int64_t ddn, const uint32_t *dn,
                      int nterms, const double *coef, const int64_t *op_off,
                      const int32_t *mode, const int8_t *dag,
                      int64_t *row, int64_t *col, double *val)
{
    const int64_t D = dup * ddn;
    const uint64_t mask = (ns == 32) ? 0xffffffffull : ((1ull << ns) - 1ull);
    int64_t *count = (int64_t *)calloc((size_t)D + 1, sizeof(int64_t));
    if (!count) return -3;
    int bad = 0;

    #pragma omp parallel for schedule(dynamic, 1024) reduction(|:bad)
    for (int64_t I = 0; I < D; ++I) {
        const uint64_t w = (uint64_t)up[I / ddn] | ((uint64_t)dn[I % ddn] << ns);
        int64_t c = 0;
        for (int t = 0; t < nterms; ++t) {
            uint64_t w2; int sg;
            const int64_t o = op_off[t];
            if (!apply_string(w, (int)(op_off[t + 1] - o), mode + o, dag + o, &w2, &sg)) continue;
            const int64_t ru = find_state(up, dup, (uint32_t)(w2 & mask));
            const int64_t rd = find_state(dn, ddn, (uint32_t)(w2 >> ns));
            if (ru < 0 || rd < 0) { bad = 1; continue; }
            c++;
        }
        count[I + 1] = c;
    }
    if (bad) { free(count); return -2; }
    for (int64_t I = 0; I < D; ++I) count[I + 1] += count[I];
    const int64_t total = count[D];
    if (!row) { free(count); return total; }

    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t I = 0; I < D; ++I) {
        const uint64_t w = (uint64_t)up[I / ddn] | ((uint64_t)dn[I % ddn] << ns);
        int64_t k = count[I];
        for (int t = 0; t < nterms; ++t) {
            uint64_t w2; int sg;
            const int64_t o = op_off[t];
            if (!apply_string(w, (int)(op_off[t + 1] - o), mode + o, dag + o, &w2, &sg)) continue;
            const int64_t ru = find_state(up, dup, (uint32_t)(w2 & mask));
            const int64_t rd = find_state(dn, ddn, (uint32_t)(w2 >> ns));
            row[k] = ru * ddn + rd;   /* <J| T |I>  is the (J, I) element */
            col[k] = I;
            val[k] = coef[t] * (double)sg;
            k++;
        }
    }
    free(count);
    return total;
}

/* COO -> CSR in the layout of Fig. 1: entries of row i occupy
 * [row_ind[i], row_ind[i+1]), sorted by column; duplicates are summed and exact
 * zeros that result are dropped.  row_ind has nrows+1 entries; col_ind and H
 * must hold nnz entries.  Returns the final number of nonzeros. */
int64_t orc_coo_to_csr(int64_t nrows, int64_t nnz,
                       const int64_t *row, const int64_t *col, const double *val,
                       int64_t *row_ind, int64_t *col_ind, double *H)
{
    int64_t *start = (int64_t *)calloc((size_t)nrows + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)malloc(((size_t)nrows + 1) * sizeof(int64_t));
    if (!start || !fill) { free(start); free(fill); return -3; }
    for (int64_t k = 0; k < nnz; ++k) start[row[k] + 1]++;
    for (int64_t i = 0; i < nrows; ++i) start[i + 1] += start[i];
    memcpy(fill, start, ((size_t)nrows + 1) * sizeof(int64_t));
    for (int64_t k = 0; k < nnz; ++k) {           /* bucket by row */
        const int64_t p = fill[row[k]]++;
        col_ind[p] = col[k];
        H[p] = val[k];
    }
    /* within each row: insertion sort by column, then merge equal columns */
    int64_t *kept = fill;                          /* reuse: kept[i] = merged count */
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < nrows; ++i) {
        const int64_t a = start[i], b = start[i + 1];
        for (int64_t p = a + 1; p < b; ++p) {
            const int64_t c = col_ind[p]; const double v = H[p];
            int64_t q = p - 1;
            while (q >= a && col_ind[q] > c) { col_ind[q + 1] = col_ind[q]; H[q + 1] = H[q]; --q; }
            col_ind[q + 1] = c; H[q + 1] = v;
        }
        int64_t out = a;
        for (int64_t p = a; p < b; ) {
            const int64_t c = col_ind[p];
            double s = 0.0;
            while (p < b && col_ind[p] == c) { s += H[p]; ++p; }
            if (s != 0.0) { col_ind[out] = c; H[out] = s; ++out; }
        }
        kept[i] = out - a;
    }
    /* compact rows to the front */
    int64_t w = 0;
    for (int64_t i = 0; i < nrows; ++i) {
        const int64_t a = start[i];
        const int64_t n = kept[i];
        if (w != a) {
            memmove(col_ind + w, col_ind + a, (size_t)n * sizeof(int64_t));
            memmove(H + w, H + a, (size_t)n * sizeof(double));
        }
        row_ind[i] = w;
        w += n;
    }
    row_ind[nrows] = w;
    free(start); free(fill);
    return w;
}

/* Listing 1: y[i] += H[j] * v[col_ind[j]] over the entries of row i.
 * y is cleared first, so the result is y = H v.  Rows are shared out over
 * OpenMP threads; each row is summed in its stored order. */
void orc_spmv(int64_t nrows, const int64_t *row_ind, const int64_t *col_ind,
              const double *H, const double *v, double *y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nrows; ++i) {
        y[i] = 0.0;
        for (int64_t j = row_ind[i]; j < row_ind[i + 1]; ++j)
            y[i] += H[j] * v[col_ind[j]];
    }
}

/* ----------------------------------------------------- matrix-free rows ---- */

/* Entries of row J, generated without storing H: since all coefficients are
 * real, <J| T |I> = <I| T^dagger |J>, and T^dagger is the string reversed with
 * every operator daggered.  Writes up to cap (column, value) pairs in term order
 * (duplicates not merged) and returns how many there are (or a negative error). */
int64_t orc_row_entries(int ns,
                        int64_t dup, const uint32_t *up, int64_t ddn, const uint32_t *dn,
                        int nterms, const double *coef, const int64_t *op_off,
                        const int32_t *mode, const int8_t *dag,
                        int64_t J, int64_t cap, int64_t *cols, double *vals)
{
    const uint64_t mask = (ns == 32) ? 0xffffffffull : ((1ull << ns) - 1ull);
    const uint64_t w = (uint64_t)up[J / ddn] | ((uint64_t)dn[J % ddn] << ns);
    int64_t k = 0;
    int32_t amode[64];
    int8_t adag[64];
    for (int t = 0; t < nterms; ++t) {
        const int64_t o = op_off[t];
        const int n = (int)(op_off[t + 1] - o);
        if (n > 64) return -4;
        for (int q = 0; q < n; ++q) {              /* adjoint: reverse and dagger */
            amode[q] = mode[o + n - 1 - q];
            adag[q] = (int8_t)!dag[o + n - 1 - q];
        }
        uint64_t w2; int sg;
        if (!apply_string(w, n, amode, adag, &w2, &sg)) continue;
        const int64_t ru = find_state(up, dup, (uint32_t)(w2 & mask));
        const int64_t rd = find_state(dn, ddn, (uint32_t)(w2 >> ns));
        if (ru < 0 || rd < 0) return -2;
        if (k < cap) { cols[k] = ru * ddn + rd; vals[k] = coef[t] * (double)sg; }
        k++;
    }
    return k;
}

/* y_J = sum_I H_JI x_I for a list of rows, each generated on the fly.
 * x is given through the columns it is needed at: for row list[r] the caller
 * first obtains the columns with orc_row_entries.  This helper does the common
 * case where the whole x is in memory. */
int orc_rows_apply(int ns,
                   int64_t dup, const uint32_t *up, int64_t ddn, const uint32_t *dn,
                   int nterms, const double *coef, const int64_t *op_off,
                   const int32_t *mode, const int8_t *dag,
                   int64_t nrows, const int64_t *rows, const double *x, double *y)
{
    int err = 0;
    #pragma omp parallel for schedule(dynamic, 64) reduction(|:err)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t cols[512]; double vals[512];
        int64_t n = orc_row_entries(ns, dup, up, ddn, dn, nterms, coef, op_off, mode, dag,
                                    rows[r], 512, cols, vals);
        if (n < 0 || n > 512) { err = 1; continue; }
        double s = 0.0;
        for (int64_t k = 0; k < n; ++k) s += vals[k] * x[cols[k]];
        y[r] = s;
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------- one-spin hop elements ---- */

/* For one spin species on its own (ns modes, n electrons): for every state r
 * (ascending order) and every ordered pair (i, j), i != j, with h[i*ns+j] != 0,
 * the element of  h_ij c+_i c_j  applied literally to that state.  Output is CSR
 * over source states: off[r]..off[r+1] hold (target rank, sign, amplitude) sorted
 * by target rank.  Pass 1 (tgt == NULL) returns the entry count. */
int64_t orc_onebody_table(int ns, int64_t dim, const uint32_t *states, const double *h,
                          int64_t *off, int64_t *tgt, int8_t *sgn, double *amp)
{
    int64_t total = 0;
    if (off) off[0] = 0;
    for (int64_t r = 0; r < dim; ++r) {
        const int64_t first = total;
        for (int i = 0; i < ns; ++i) {
            for (int j = 0; j < ns; ++j) {
                if (i == j || h[i * ns + j] == 0.0) continue;
                const int32_t md[2] = { i, j };
                const int8_t dg[2] = { 1, 0 };
                uint64_t w2; int sg;
                if (!apply_string(states[r], 2, md, dg, &w2, &sg)) continue;
                if (tgt) {
                    const int64_t t = find_state(states, dim, (uint32_t)w2);
                    if (t < 0) return -2;
                    tgt[total] = t; sgn[total] = (int8_t)sg; amp[total] = h[i * ns + j];
                }
                total++;
            }
        }
        if (tgt) {   /* insertion sort of this row by target rank */
            for (int64_t p = first + 1; p < total; ++p) {
                int64_t t = tgt[p]; int8_t s = sgn[p]; double a = amp[p];
                int64_t q = p - 1;
                while (q >= first && tgt[q] > t) { tgt[q+1] = tgt[q]; sgn[q+1] = sgn[q]; amp[q+1] = amp[q]; --q; }
                tgt[q+1] = t; sgn[q+1] = s; amp[q+1] = a;
            }
        }
        if (off) off[r + 1] = total;
    }
    return total;
}
