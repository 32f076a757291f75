/*
 * Plain FP64 CPU oracle for RgCSR sparse matrix-vector multiplication.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP path.
 *
 * Every routine is the plain definition of what it computes, written for
 * checking by eye against the paper (Oberhuber, Suzuki, Vacata, "New
 * Row-grouped CSR format for storing the sparse matrices on GPU with
 * implementation in CUDA"):
 *   - CSR storage and its serial SpMV            : Section 3.1 (first listing)
 *   - Row-grouped CSR (RgCSR) layout and kernel   : Section 3.4 (Figure 5 text,
 *                                                   second listing)
 *   - Hybrid ELLPACK + COO                        : Section 3.3
 *   - Krylov consumer (CG)                        : Section 1 (SpMV dominates CG)
 * Readings where the paper is silent (ghost index, pad value, long-row split,
 * lanes per row, sort window, Hybrid K1 rule) are the project's documented
 * readings; each routine states the one it uses.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math, no
 * FMA contraction, so a*b+c is two roundings exactly as written; OpenMP only
 * in orc_csr_spmv_par).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------ */
/* CSR                                                                      */
/* ------------------------------------------------------------------------ */

/* Serial CSR SpMV of Section 3.1: Ax[i] starts at 0.0 and accumulates
 * values[j] * x[columns[j]] for j = rowPointers[i] .. rowPointers[i+1]-1 in
 * ascending order.  FP64, one multiply and one add per nonzero. */
void orc_csr_spmv(int64_t n_rows, const int64_t *rp, const int32_t *col,
                  const double *val, const double *x, double *y)
{
    for (int64_t i = 0; i < n_rows; i++) {
        double acc = 0.0;
        for (int64_t j = rp[i]; j < rp[i + 1]; j++)
            acc += val[j] * x[col[j]];
        y[i] = acc;
    }
}

/* The same serial sum with the rows split into n_threads contiguous ranges
 * of equal row count (a static partition), one OpenMP thread each: every row
 * is still summed by one thread in ascending order, so y is bit-identical to
 * orc_csr_spmv.  Used only to time the oracle on every host core. */
void orc_csr_spmv_par(int64_t n_rows, const int64_t *rp, const int32_t *col,
                      const double *val, const double *x, double *y, int n_threads)
{
#pragma omp parallel for schedule(static) num_threads(n_threads)
    for (int64_t i = 0; i < n_rows; i++) {
        double acc = 0.0;
        for (int64_t j = rp[i]; j < rp[i + 1]; j++)
            acc += val[j] * x[col[j]];
        y[i] = acc;
    }
}

/* s_i = sum_j |a_ij| * |x_j|, the scale of the tolerance on floating-point
 * SpMV results. */
void orc_csr_absmv(int64_t n_rows, const int64_t *rp, const int32_t *col,
                   const double *val, const double *x, double *s)
{
    for (int64_t i = 0; i < n_rows; i++) {
        double acc = 0.0;
        for (int64_t j = rp[i]; j < rp[i + 1]; j++)
            acc += fabs(val[j]) * fabs(x[col[j]]);
        s[i] = acc;
    }
}

/* Y = A X for k right-hand sides, computed column by column with the serial
 * CSR SpMV.  X is n_cols x k and Y is n_rows x k, both row-major. */
void orc_csr_spmm(int64_t n_rows, int64_t n_cols, int64_t k, const int64_t *rp,
                  const int32_t *col, const double *val, const double *X, double *Y)
{
    double *xc = (double *)malloc(sizeof(double) * (size_t)(n_cols > 0 ? n_cols : 1));
    double *yc = (double *)malloc(sizeof(double) * (size_t)(n_rows > 0 ? n_rows : 1));
    for (int64_t c = 0; c < k; c++) {
        for (int64_t j = 0; j < n_cols; j++) xc[j] = X[j * k + c];
        orc_csr_spmv(n_rows, rp, col, val, xc, yc);
        for (int64_t i = 0; i < n_rows; i++) Y[i * k + c] = yc[i];
    }
    free(xc);
    free(yc);
}

/* Validation of the CSR convention of Section 3.1.  Returns 0 when valid:
 *   1  rp[0] != 0          2  rp decreases          3  rp[n] != nnz
 *   4  column out of range 5  columns not strictly ascending within a row */
int orc_csr_check(int64_t n_rows, int64_t n_cols, int64_t nnz,
                  const int64_t *rp, const int32_t *col)
{
    if (rp[0] != 0) return 1;
    for (int64_t i = 0; i < n_rows; i++)
        if (rp[i + 1] < rp[i]) return 2;
    if (rp[n_rows] != nnz) return 3;
    for (int64_t i = 0; i < n_rows; i++) {
        for (int64_t j = rp[i]; j < rp[i + 1]; j++) {
            if (col[j] < 0 || (int64_t)col[j] >= n_cols) return 4;
            if (j > rp[i] && col[j] <= col[j - 1]) return 5;
        }
    }
    return 0;
}

/* A^T in CSR by counting: row c of A^T lists, in ascending original row
 * order, the entries (i, c) of A. */
void orc_csr_transpose(int64_t n_rows, int64_t n_cols, const int64_t *rp,
                       const int32_t *col, const double *val,
                       int64_t *rpT, int32_t *colT, double *valT)
{
    for (int64_t c = 0; c <= n_cols; c++) rpT[c] = 0;
    for (int64_t j = 0; j < rp[n_rows]; j++) rpT[col[j] + 1]++;
    for (int64_t c = 0; c < n_cols; c++) rpT[c + 1] += rpT[c];
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_cols > 0 ? n_cols : 1));
    for (int64_t c = 0; c < n_cols; c++) next[c] = rpT[c];
    for (int64_t i = 0; i < n_rows; i++) {
        for (int64_t j = rp[i]; j < rp[i + 1]; j++) {
            int64_t d = next[col[j]]++;
            colT[d] = (int32_t)i;
            valT[d] = val[j];
        }
    }
    free(next);
}

/* Gradient of L = 1/2 ||A(theta) x - b||^2 (plain calculus):
 *   r = A x - b, dL/dx = A^T r (serial scatter over CSR),
 *   dL/dtheta_k = r[row(k)] * x[col(k)]. */
void orc_adjoint(int64_t n_rows, int64_t n_cols, const int64_t *rp, const int32_t *col,
                 const double *val, const double *x, const double *b,
                 double *r, double *dx, double *dval)
{
    orc_csr_spmv(n_rows, rp, col, val, x, r);
    for (int64_t i = 0; i < n_rows; i++) r[i] -= b[i];
    for (int64_t c = 0; c < n_cols; c++) dx[c] = 0.0;
    for (int64_t i = 0; i < n_rows; i++) {
        for (int64_t j = rp[i]; j < rp[i + 1]; j++) {
            dx[col[j]] += val[j] * r[i];
            dval[j] = r[i] * x[col[j]];
        }
    }
}

/* Plain conjugate gradients in FP64 (textbook Hestenes-Stiefel form), the
 * Krylov consumer of SpMV named in Section 1.  Starts from the x passed in.
 * Stops when ||b - A x||_2 / ||b||_2 <= tol (recursive residual) or after
 * maxit iterations.  Returns the iteration count; *relres gets the final
 * relative residual recomputed from scratch. */
int64_t orc_cg(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
               const double *b, double *x, double tol, int64_t maxit, double *relres)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    orc_csr_spmv(n, rp, col, val, x, q);
    double bb = 0.0, rr = 0.0;
    for (int64_t i = 0; i < n; i++) {
        r[i] = b[i] - q[i];
        p[i] = r[i];
        bb += b[i] * b[i];
        rr += r[i] * r[i];
    }
    double bn = sqrt(bb);
    if (bn == 0.0) bn = 1.0;
    int64_t it = 0;
    while (it < maxit && sqrt(rr) / bn > tol) {
        orc_csr_spmv(n, rp, col, val, p, q);
        double pq = 0.0;
        for (int64_t i = 0; i < n; i++) pq += p[i] * q[i];
        double alpha = rr / pq;
        double rr_new = 0.0;
        for (int64_t i = 0; i < n; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            rr_new += r[i] * r[i];
        }
        double beta = rr_new / rr;
        rr = rr_new;
        for (int64_t i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
        it++;
    }
    orc_csr_spmv(n, rp, col, val, x, q);
    double res = 0.0;
    for (int64_t i = 0; i < n; i++) res += (b[i] - q[i]) * (b[i] - q[i]);
    *relres = sqrt(res) / bn;
    free(r);
    free(p);
    free(q);
    return it;
}

/* ------------------------------------------------------------------------ */
/* RgCSR layout (Section 3.4)                                               */
/* ------------------------------------------------------------------------ */
/*
 * Parameters: group size G >= 1, lanes per row T >= 1, sort window
 * sigma >= 1, long-row threshold tau (tau < 0: no split).
 *
 * 1. Row order.  Inside each window of sigma consecutive rows the rows are
 *    sorted by length, longest first, ties kept in original order (the
 *    descending ordering of Section 4.4.2; sigma = 1 keeps the paper's order).
 * 2. Split.  Walking rows in that order, rows longer than tau go to the long
 *    list, all others to the short list (tau < 0: every row is short).
 * 3. Groups.  The short list is cut into consecutive groups of G rows; the
 *    last group holds the remainder (its true size s_g, as the paper's kernel
 *    uses the remainder as the stride of the last group).
 * 4. Width.  w_g = longest row of the group, rounded up to a multiple of T.
 *    groupPointers: gp[0] = 0, gp[g+1] = gp[g] + s_g * w_g.
 * 5. Placement.  Nonzero j (0-based, CSR order) of local row t of group g
 *    sits at gp[g] + (j / T) * (s_g * T) + t * T + (j % T).  With T = 1 this
 *    is the paper's "first nonzero of every row, then the second, ...".
 *    Slots of a row past its length are artificial zeros: value bits all
 *    zero, column = the row's last column (0 for an empty row) as ghost index.
 * 6. Long rows keep CSR order.  The long list is ordered longest first,
 *    ties by original row, and the rows are concatenated in that order.
 */

typedef struct { int64_t len; int64_t idx; } orc_row_key;

static int orc_cmp_desc(const void *a, const void *b)
{
    const orc_row_key *u = (const orc_row_key *)a, *v = (const orc_row_key *)b;
    if (u->len != v->len) return u->len > v->len ? -1 : 1;
    if (u->idx != v->idx) return u->idx < v->idx ? -1 : 1;
    return 0;
}

/* order[p] = original row placed at position p after step 1. */
static void orc_row_order(int64_t n, const int64_t *rp, int64_t sigma, int64_t *order)
{
    orc_row_key *k = (orc_row_key *)malloc(sizeof(orc_row_key) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        k[i].len = rp[i + 1] - rp[i];
        k[i].idx = i;
    }
    if (sigma > 1) {
        for (int64_t w0 = 0; w0 < n; w0 += sigma) {
            int64_t m = (n - w0 < sigma) ? n - w0 : sigma;
            qsort(k + w0, (size_t)m, sizeof(orc_row_key), orc_cmp_desc);
        }
    }
    for (int64_t i = 0; i < n; i++) order[i] = k[i].idx;
    free(k);
}

/* Sizes: out[0] groups, out[1] short rows, out[2] long rows, out[3] grouped
 * slots (gp[groups]), out[4] long nonzeros. */
void orc_rgcsr_sizes(int64_t n, const int64_t *rp, int64_t G, int64_t T,
                     int64_t sigma, int64_t tau, int64_t *out)
{
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    orc_row_order(n, rp, sigma, order);
    int64_t ns = 0, nl = 0, lnnz = 0, slots = 0, ng = 0;
    int64_t in_group = 0, wmax = 0;
    for (int64_t p = 0; p < n; p++) {
        int64_t r = order[p], len = rp[r + 1] - rp[r];
        if (tau >= 0 && len > tau) {
            nl++;
            lnnz += len;
            continue;
        }
        ns++;
        in_group++;
        if (len > wmax) wmax = len;
        if (in_group == G) {
            int64_t w = (wmax + T - 1) / T * T;
            slots += in_group * w;
            ng++;
            in_group = 0;
            wmax = 0;
        }
    }
    if (in_group > 0) {
        int64_t w = (wmax + T - 1) / T * T;
        slots += in_group * w;
        ng++;
    }
    out[0] = ng; out[1] = ns; out[2] = nl; out[3] = slots; out[4] = lnnz;
    free(order);
}

/* Fill every layout array.  Values are moved as raw bytes of width esz, so
 * the layout is bit-exact for any value type.  Array sizes come from
 * orc_rgcsr_sizes: gp[ng+1], short_len[ns], short_row[ns], slot_val[slots*esz],
 * slot_col[slots], long_row[nl], long_ptr[nl+1], long_val[lnnz*esz],
 * long_col[lnnz]. */
void orc_rgcsr_build(int64_t n, const int64_t *rp, const int32_t *col, const uint8_t *val,
                     int64_t esz, int64_t G, int64_t T, int64_t sigma, int64_t tau,
                     int64_t *gp, int32_t *short_len, int32_t *short_row,
                     uint8_t *slot_val, int32_t *slot_col,
                     int32_t *long_row, int64_t *long_ptr, uint8_t *long_val, int32_t *long_col)
{
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    orc_row_order(n, rp, sigma, order);
    /* step 2: split */
    int64_t ns = 0, nl = 0;
    orc_row_key *lk = (orc_row_key *)malloc(sizeof(orc_row_key) * (size_t)(n > 0 ? n : 1));
    for (int64_t p = 0; p < n; p++) {
        int64_t r = order[p], len = rp[r + 1] - rp[r];
        if (tau >= 0 && len > tau) {
            lk[nl].len = len;
            lk[nl].idx = r;
            nl++;
        } else {
            short_row[ns] = (int32_t)r;
            short_len[ns] = (int32_t)len;
            ns++;
        }
    }
    /* step 6: long list longest first, ties by original row */
    qsort(lk, (size_t)nl, sizeof(orc_row_key), orc_cmp_desc);
    long_ptr[0] = 0;
    for (int64_t i = 0; i < nl; i++) {
        int64_t r = lk[i].idx, len = lk[i].len;
        long_row[i] = (int32_t)r;
        for (int64_t j = 0; j < len; j++) {
            memcpy(long_val + (long_ptr[i] + j) * esz, val + (rp[r] + j) * esz, (size_t)esz);
            long_col[long_ptr[i] + j] = col[rp[r] + j];
        }
        long_ptr[i + 1] = long_ptr[i] + len;
    }
    free(lk);
    /* steps 3-5: groups, widths, placement */
    int64_t ng = (ns + G - 1) / G;
    gp[0] = 0;
    for (int64_t g = 0; g < ng; g++) {
        int64_t first = g * G;
        int64_t sg = (ns - first < G) ? ns - first : G;
        int64_t w = 0;
        for (int64_t t = 0; t < sg; t++)
            if (short_len[first + t] > w) w = short_len[first + t];
        w = (w + T - 1) / T * T;
        gp[g + 1] = gp[g] + sg * w;
        for (int64_t t = 0; t < sg; t++) {
            int64_t r = short_row[first + t];
            int64_t len = short_len[first + t];
            int32_t ghost = len > 0 ? col[rp[r] + len - 1] : 0;
            for (int64_t j = 0; j < w; j++) {
                int64_t s = gp[g] + (j / T) * (sg * T) + t * T + (j % T);
                if (j < len) {
                    memcpy(slot_val + s * esz, val + (rp[r] + j) * esz, (size_t)esz);
                    slot_col[s] = col[rp[r] + j];
                } else {
                    memset(slot_val + s * esz, 0, (size_t)esz);
                    slot_col[s] = ghost;
                }
            }
        }
    }
    free(order);
}

/* Inverse of orc_rgcsr_build: recover CSR (row pointers, columns, value
 * bytes) from the layout arrays alone. */
void orc_rgcsr_decode(int64_t n, int64_t G, int64_t T, int64_t ns, int64_t nl,
                      const int64_t *gp, const int32_t *short_len, const int32_t *short_row,
                      const uint8_t *slot_val, const int32_t *slot_col,
                      const int32_t *long_row, const int64_t *long_ptr,
                      const uint8_t *long_val, const int32_t *long_col, int64_t esz,
                      int64_t *rp, int32_t *col, uint8_t *val)
{
    int64_t *len = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    for (int64_t i = 0; i < ns; i++) len[short_row[i]] = short_len[i];
    for (int64_t i = 0; i < nl; i++) len[long_row[i]] = long_ptr[i + 1] - long_ptr[i];
    rp[0] = 0;
    for (int64_t r = 0; r < n; r++) rp[r + 1] = rp[r] + len[r];
    for (int64_t i = 0; i < ns; i++) {
        int64_t g = i / G, t = i % G;
        int64_t sg = (ns - g * G < G) ? ns - g * G : G;
        int64_t r = short_row[i];
        for (int64_t j = 0; j < short_len[i]; j++) {
            int64_t s = gp[g] + (j / T) * (sg * T) + t * T + (j % T);
            col[rp[r] + j] = slot_col[s];
            memcpy(val + (rp[r] + j) * esz, slot_val + s * esz, (size_t)esz);
        }
    }
    for (int64_t i = 0; i < nl; i++) {
        int64_t r = long_row[i];
        for (int64_t j = 0; j < long_ptr[i + 1] - long_ptr[i]; j++) {
            col[rp[r] + j] = long_col[long_ptr[i] + j];
            memcpy(val + (rp[r] + j) * esz, long_val + (long_ptr[i] + j) * esz, (size_t)esz);
        }
    }
    free(len);
}

/* SpMV on the layout, one "thread" per row exactly as the RgCSR kernel of
 * Section 3.4 walks it: start at the row's first slot, add the stride of its
 * group, stop after rowLength steps (padding is never multiplied).  FP64 with
 * FP64 values (the caller upcasts).  The per-row order equals the serial CSR
 * order, so the result is bit-identical to orc_csr_spmv. */
void orc_rgcsr_spmv(int64_t n, int64_t G, int64_t T, int64_t ns, int64_t nl,
                    const int64_t *gp, const int32_t *short_len, const int32_t *short_row,
                    const double *slot_val, const int32_t *slot_col,
                    const int32_t *long_row, const int64_t *long_ptr,
                    const double *long_val, const int32_t *long_col,
                    const double *x, double *y)
{
    for (int64_t r = 0; r < n; r++) y[r] = 0.0;
    for (int64_t i = 0; i < ns; i++) {
        int64_t g = i / G, t = i % G;
        int64_t sg = (ns - g * G < G) ? ns - g * G : G;
        double acc = 0.0;
        for (int64_t j = 0; j < short_len[i]; j++) {
            int64_t s = gp[g] + (j / T) * (sg * T) + t * T + (j % T);
            acc += slot_val[s] * x[slot_col[s]];
        }
        y[short_row[i]] = acc;
    }
    for (int64_t i = 0; i < nl; i++) {
        double acc = 0.0;
        for (int64_t k = long_ptr[i]; k < long_ptr[i + 1]; k++)
            acc += long_val[k] * x[long_col[k]];
        y[long_row[i]] = acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Hybrid ELLPACK + COO (Section 3.3)                                       */
/* ------------------------------------------------------------------------ */
/*
 * The paper stresses that the ELL width K1 < K must be chosen well but does
 * not give a rule.  Project rule: K1 minimises
 *     k * n_pad * (s_v + 4)  +  c * (s_v + 8) * sum_i max(0, len_i - k)
 * over k in [0, max_i len_i] (ties: smallest k), with n_pad = n rounded up to
 * a multiple of 64 and c the assumed cost ratio of a COO entry to an ELL slot.
 * ELL is column-major n_pad x K1 (entry (i, j) at j * n_pad + i) holding the
 * first min(len_i, K1) nonzeros of row i; padding has column -1 and value
 * bits zero.  COO holds the remaining nonzeros in (row, column) order.
 */
int64_t orc_hyb_k1(int64_t n, const int64_t *rp, int64_t s_v, int64_t c)
{
    int64_t kmax = 0;
    for (int64_t i = 0; i < n; i++)
        if (rp[i + 1] - rp[i] > kmax) kmax = rp[i + 1] - rp[i];
    int64_t n_pad = (n + 63) / 64 * 64;
    int64_t *hist = (int64_t *)calloc((size_t)(kmax + 1), sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) hist[rp[i + 1] - rp[i]]++;
    int64_t best_k = 0, best_cost = -1;
    for (int64_t k = 0; k <= kmax; k++) {
        int64_t excess = 0;
        for (int64_t L = k + 1; L <= kmax; L++) excess += hist[L] * (L - k);
        int64_t cost = k * n_pad * (s_v + 4) + c * (s_v + 8) * excess;
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best_k = k;
        }
    }
    free(hist);
    return best_k;
}

/* Number of COO entries for a given K1. */
int64_t orc_hyb_coo_count(int64_t n, const int64_t *rp, int64_t K1)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t len = rp[i + 1] - rp[i];
        if (len > K1) m += len - K1;
    }
    return m;
}

void orc_hyb_build(int64_t n, const int64_t *rp, const int32_t *col, const uint8_t *val,
                   int64_t esz, int64_t K1, int64_t n_pad,
                   int32_t *ell_col, uint8_t *ell_val,
                   int32_t *coo_row, int32_t *coo_col, uint8_t *coo_val)
{
    for (int64_t j = 0; j < K1; j++) {
        for (int64_t i = 0; i < n_pad; i++) {
            int64_t e = j * n_pad + i;
            int64_t len = i < n ? rp[i + 1] - rp[i] : 0;
            if (j < len) {
                ell_col[e] = col[rp[i] + j];
                memcpy(ell_val + e * esz, val + (rp[i] + j) * esz, (size_t)esz);
            } else {
                ell_col[e] = -1;
                memset(ell_val + e * esz, 0, (size_t)esz);
            }
        }
    }
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        for (int64_t j = rp[i] + K1; j < rp[i + 1]; j++) {
            coo_row[m] = (int32_t)i;
            coo_col[m] = col[j];
            memcpy(coo_val + m * esz, val + j * esz, (size_t)esz);
            m++;
        }
    }
}

/* Hybrid SpMV in FP64, ELL step then COO step, each row summed in CSR order
 * (ELL part of the row first, then its COO entries), so the result is
 * bit-identical to orc_csr_spmv. */
void orc_hyb_spmv(int64_t n, int64_t K1, int64_t n_pad, const int32_t *ell_col,
                  const double *ell_val, int64_t m, const int32_t *coo_row,
                  const int32_t *coo_col, const double *coo_val,
                  const double *x, double *y)
{
    for (int64_t i = 0; i < n; i++) {
        double acc = 0.0;
        for (int64_t j = 0; j < K1; j++) {
            int32_t c = ell_col[j * n_pad + i];
            if (c >= 0) acc += ell_val[j * n_pad + i] * x[c];
        }
        y[i] = acc;
    }
    for (int64_t e = 0; e < m; e++)
        y[coo_row[e]] += coo_val[e] * x[coo_col[e]];
}
