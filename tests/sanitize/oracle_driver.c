/* Sanitizer driver for the CPU oracle (built with -fsanitize=address,undefined
 * together with oracle/oracle.c).  Runs every oracle routine on seeded random
 * CSR matrices and checks the facts that tie them together (layout round trip,
 * layout walk and Hybrid equal to the serial sum bit for bit, row-split sum
 * equal to the serial one, transpose twice is the identity, CG converges on a
 * diagonally dominant system).  Exit status 0 when every check holds and the
 * sanitizers report nothing. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_csr_spmv(int64_t, const int64_t *, const int32_t *, const double *, const double *, double *);
void orc_csr_spmv_par(int64_t, const int64_t *, const int32_t *, const double *, const double *, double *, int);
void orc_csr_absmv(int64_t, const int64_t *, const int32_t *, const double *, const double *, double *);
void orc_csr_spmm(int64_t, int64_t, int64_t, const int64_t *, const int32_t *, const double *, const double *,
                  double *);
int orc_csr_check(int64_t, int64_t, int64_t, const int64_t *, const int32_t *);
void orc_csr_transpose(int64_t, int64_t, const int64_t *, const int32_t *, const double *, int64_t *, int32_t *,
                       double *);
void orc_adjoint(int64_t, int64_t, const int64_t *, const int32_t *, const double *, const double *,
                 const double *, double *, double *, double *);
int64_t orc_cg(int64_t, const int64_t *, const int32_t *, const double *, const double *, double *, double,
               int64_t, double *);
void orc_rgcsr_sizes(int64_t, const int64_t *, int64_t, int64_t, int64_t, int64_t, int64_t *);
void orc_rgcsr_build(int64_t, const int64_t *, const int32_t *, const uint8_t *, int64_t, int64_t, int64_t,
                     int64_t, int64_t, int64_t *, int32_t *, int32_t *, uint8_t *, int32_t *, int32_t *, int64_t *,
                     uint8_t *, int32_t *);
void orc_rgcsr_decode(int64_t, int64_t, int64_t, int64_t, int64_t, const int64_t *, const int32_t *,
                      const int32_t *, const uint8_t *, const int32_t *, const int32_t *, const int64_t *,
                      const uint8_t *, const int32_t *, int64_t, int64_t *, int32_t *, uint8_t *);
void orc_rgcsr_spmv(int64_t, int64_t, int64_t, int64_t, int64_t, const int64_t *, const int32_t *,
                    const int32_t *, const double *, const int32_t *, const int32_t *, const int64_t *,
                    const double *, const int32_t *, const double *, double *);
int64_t orc_hyb_k1(int64_t, const int64_t *, int64_t, int64_t);
int64_t orc_hyb_coo_count(int64_t, const int64_t *, int64_t);
void orc_hyb_build(int64_t, const int64_t *, const int32_t *, const uint8_t *, int64_t, int64_t, int64_t,
                   int32_t *, uint8_t *, int32_t *, int32_t *, uint8_t *);
void orc_hyb_spmv(int64_t, int64_t, int64_t, const int32_t *, const double *, int64_t, const int32_t *,
                  const int32_t *, const double *, const double *, double *);

static int failures = 0;
#define CHECK(c, msg)                                                    \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, msg); \
            failures++;                                                  \
        }                                                                \
    } while (0)

static uint64_t rng_state = 88172645463325252ull;
static uint64_t next_u64(void) { /* xorshift64 */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}
static double next_unit(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

typedef struct {
    int64_t n, m, nnz;
    int64_t *rp;
    int32_t *col;
    double *val;
} csr;

/* random CSR with ascending distinct columns per row; the first long_rows
 * rows hold three quarters of the columns */
static csr random_csr(int64_t n, int64_t m, int max_len, int long_rows) {
    csr A;
    A.n = n;
    A.m = m;
    A.rp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t cap = 16, nnz = 0;
    A.col = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    A.val = (double *)malloc(sizeof(double) * (size_t)cap);
    A.rp[0] = 0;
    for (int64_t r = 0; r < n; r++) {
        int64_t len = (int64_t)(next_u64() % (uint64_t)(max_len + 1));
        if (r < long_rows) len = m * 3 / 4;
        if (len > m) len = m;
        for (int64_t c = 0, k = 0; c < m && k < len; c++) {
            /* pick column c with probability (len - k) / (m - c): ascending, distinct */
            if ((int64_t)(next_u64() % (uint64_t)(m - c)) < len - k) {
                if (nnz == cap) {
                    cap *= 2;
                    A.col = (int32_t *)realloc(A.col, sizeof(int32_t) * (size_t)cap);
                    A.val = (double *)realloc(A.val, sizeof(double) * (size_t)cap);
                }
                A.col[nnz] = (int32_t)c;
                A.val[nnz] = 2.0 * next_unit() - 1.0;
                nnz++;
                k++;
            }
        }
        A.rp[r + 1] = nnz;
    }
    A.nnz = nnz;
    return A;
}

static void free_csr(csr *A) {
    free(A->rp);
    free(A->col);
    free(A->val);
}

static void check_layouts(const csr *A, const double *x, const double *y_ref) {
    const int64_t Gs[] = {1, 3, 4, 64}, Ts[] = {1, 2, 8}, sigmas[] = {1, 5, 1 << 30}, taus[] = {-1, 0, 7};
    for (int gi = 0; gi < 4; gi++)
        for (int ti = 0; ti < 3; ti++)
            for (int si = 0; si < 3; si++)
                for (int ui = 0; ui < 3; ui++) {
                    const int64_t G = Gs[gi], T = Ts[ti], sigma = sigmas[si], tau = taus[ui];
                    int64_t sz[5];
                    orc_rgcsr_sizes(A->n, A->rp, G, T, sigma, tau, sz);
                    const int64_t ng = sz[0], ns = sz[1], nl = sz[2], slots = sz[3], lnnz = sz[4];
                    int64_t *gp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ng + 1));
                    int32_t *slen = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ns + 1));
                    int32_t *srow = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ns + 1));
                    double *sval = (double *)malloc(sizeof(double) * (size_t)(slots + 1));
                    int32_t *scol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(slots + 1));
                    int32_t *lrow = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nl + 1));
                    int64_t *lptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nl + 1));
                    double *lval = (double *)malloc(sizeof(double) * (size_t)(lnnz + 1));
                    int32_t *lcol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lnnz + 1));
                    orc_rgcsr_build(A->n, A->rp, A->col, (const uint8_t *)A->val, 8, G, T, sigma, tau, gp, slen,
                                    srow, (uint8_t *)sval, scol, lrow, lptr, (uint8_t *)lval, lcol);
                    int64_t *rp2 = (int64_t *)malloc(sizeof(int64_t) * (size_t)(A->n + 1));
                    int32_t *col2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(A->nnz + 1));
                    double *val2 = (double *)malloc(sizeof(double) * (size_t)(A->nnz + 1));
                    orc_rgcsr_decode(A->n, G, T, ns, nl, gp, slen, srow, (const uint8_t *)sval, scol, lrow, lptr,
                                     (const uint8_t *)lval, lcol, 8, rp2, col2, (uint8_t *)val2);
                    CHECK(memcmp(rp2, A->rp, sizeof(int64_t) * (size_t)(A->n + 1)) == 0, "decode row pointers");
                    CHECK(memcmp(col2, A->col, sizeof(int32_t) * (size_t)A->nnz) == 0, "decode columns");
                    CHECK(memcmp(val2, A->val, sizeof(double) * (size_t)A->nnz) == 0, "decode values");
                    double *y = (double *)malloc(sizeof(double) * (size_t)(A->n + 1));
                    orc_rgcsr_spmv(A->n, G, T, ns, nl, gp, slen, srow, sval, scol, lrow, lptr, lval, lcol, x, y);
                    CHECK(memcmp(y, y_ref, sizeof(double) * (size_t)A->n) == 0, "layout walk equals serial sum");
                    free(gp); free(slen); free(srow); free(sval); free(scol);
                    free(lrow); free(lptr); free(lval); free(lcol);
                    free(rp2); free(col2); free(val2); free(y);
                }
}

static void check_hybrid(const csr *A, const double *x, const double *y_ref) {
    const int64_t K1 = orc_hyb_k1(A->n, A->rp, 4, 3);
    const int64_t n_pad = (A->n + 63) / 64 * 64;
    const int64_t m = orc_hyb_coo_count(A->n, A->rp, K1);
    int32_t *ecol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K1 * n_pad + 1));
    double *eval = (double *)malloc(sizeof(double) * (size_t)(K1 * n_pad + 1));
    int32_t *crow = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
    int32_t *ccol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
    double *cval = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    orc_hyb_build(A->n, A->rp, A->col, (const uint8_t *)A->val, 8, K1, n_pad, ecol, (uint8_t *)eval, crow, ccol,
                  (uint8_t *)cval);
    double *y = (double *)malloc(sizeof(double) * (size_t)(A->n + 1));
    orc_hyb_spmv(A->n, K1, n_pad, ecol, eval, m, crow, ccol, cval, x, y);
    CHECK(memcmp(y, y_ref, sizeof(double) * (size_t)A->n) == 0, "Hybrid equals serial sum");
    free(ecol); free(eval); free(crow); free(ccol); free(cval); free(y);
}

int main(void) {
    const int64_t shapes[][4] = {{0, 0, 0, 0}, {1, 1, 1, 0}, {9, 7, 4, 1}, {130, 90, 12, 2}, {257, 257, 20, 3}};
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); s++) {
        csr A = random_csr(shapes[s][0], shapes[s][1], (int)shapes[s][2], (int)shapes[s][3]);
        CHECK(orc_csr_check(A.n, A.m, A.nnz, A.rp, A.col) == 0, "generated CSR is valid");
        double *x = (double *)malloc(sizeof(double) * (size_t)(A.m + 1));
        for (int64_t i = 0; i < A.m; i++) x[i] = 2.0 * next_unit() - 1.0;
        double *y = (double *)malloc(sizeof(double) * (size_t)(A.n + 1));
        double *y2 = (double *)malloc(sizeof(double) * (size_t)(A.n + 1));
        orc_csr_spmv(A.n, A.rp, A.col, A.val, x, y);
        orc_csr_spmv_par(A.n, A.rp, A.col, A.val, x, y2, 3);
        CHECK(memcmp(y, y2, sizeof(double) * (size_t)A.n) == 0, "row-split sum equals serial sum");
        orc_csr_absmv(A.n, A.rp, A.col, A.val, x, y2);
        for (int64_t i = 0; i < A.n; i++) CHECK(y2[i] >= fabs(y[i]) - 1e-12, "|A||x| bounds |Ax|");
        /* SpMM with k = 3 columns, column 0 = x */
        double *X = (double *)malloc(sizeof(double) * (size_t)(A.m * 3 + 1));
        double *Y = (double *)malloc(sizeof(double) * (size_t)(A.n * 3 + 1));
        for (int64_t i = 0; i < A.m; i++) {
            X[i * 3] = x[i];
            X[i * 3 + 1] = 1.0;
            X[i * 3 + 2] = -x[i];
        }
        orc_csr_spmm(A.n, A.m, 3, A.rp, A.col, A.val, X, Y);
        for (int64_t i = 0; i < A.n; i++) CHECK(Y[i * 3] == y[i], "SpMM column 0 equals SpMV");
        check_layouts(&A, x, y);
        check_hybrid(&A, x, y);
        /* transpose twice is the identity */
        int64_t *rpT = (int64_t *)malloc(sizeof(int64_t) * (size_t)(A.m + 1));
        int32_t *colT = (int32_t *)malloc(sizeof(int32_t) * (size_t)(A.nnz + 1));
        double *valT = (double *)malloc(sizeof(double) * (size_t)(A.nnz + 1));
        int64_t *rpTT = (int64_t *)malloc(sizeof(int64_t) * (size_t)(A.n + 1));
        int32_t *colTT = (int32_t *)malloc(sizeof(int32_t) * (size_t)(A.nnz + 1));
        double *valTT = (double *)malloc(sizeof(double) * (size_t)(A.nnz + 1));
        orc_csr_transpose(A.n, A.m, A.rp, A.col, A.val, rpT, colT, valT);
        orc_csr_transpose(A.m, A.n, rpT, colT, valT, rpTT, colTT, valTT);
        CHECK(memcmp(rpTT, A.rp, sizeof(int64_t) * (size_t)(A.n + 1)) == 0, "transpose twice: row pointers");
        CHECK(memcmp(colTT, A.col, sizeof(int32_t) * (size_t)A.nnz) == 0, "transpose twice: columns");
        CHECK(memcmp(valTT, A.val, sizeof(double) * (size_t)A.nnz) == 0, "transpose twice: values");
        /* adjoint */
        double *b = (double *)malloc(sizeof(double) * (size_t)(A.n + 1));
        double *r = (double *)malloc(sizeof(double) * (size_t)(A.n + 1));
        double *dx = (double *)malloc(sizeof(double) * (size_t)(A.m + 1));
        double *dv = (double *)malloc(sizeof(double) * (size_t)(A.nnz + 1));
        for (int64_t i = 0; i < A.n; i++) b[i] = next_unit();
        orc_adjoint(A.n, A.m, A.rp, A.col, A.val, x, b, r, dx, dv);
        for (int64_t i = 0; i < A.n; i++) CHECK(r[i] == y[i] - b[i], "adjoint residual");
        free(X); free(Y); free(rpT); free(colT); free(valT); free(rpTT); free(colTT); free(valTT);
        free(b); free(r); free(dx); free(dv);
        /* CG on a diagonal system of the same size: x = 1 */
        if (A.n == A.m && A.n > 0) {
            int64_t *rpd = (int64_t *)malloc(sizeof(int64_t) * (size_t)(A.n + 1));
            int32_t *cd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(A.n + 1));
            double *vd = (double *)malloc(sizeof(double) * (size_t)(A.n + 1));
            double *bd = (double *)malloc(sizeof(double) * (size_t)(A.n + 1));
            double *xd = (double *)calloc((size_t)(A.n + 1), sizeof(double));
            for (int64_t i = 0; i <= A.n; i++) rpd[i] = i;
            for (int64_t i = 0; i < A.n; i++) {
                cd[i] = (int32_t)i;
                vd[i] = 1.0 + (double)(i % 7);
                bd[i] = vd[i];
            }
            double rel = 1.0;
            orc_cg(A.n, rpd, cd, vd, bd, xd, 1e-12, 100, &rel);
            CHECK(rel <= 1e-12, "CG on a diagonal system");
            for (int64_t i = 0; i < A.n; i++) CHECK(fabs(xd[i] - 1.0) <= 1e-12, "CG solution");
            free(rpd); free(cd); free(vd); free(bd); free(xd);
        }
        free(x); free(y); free(y2);
        free_csr(&A);
    }
    printf("oracle checks done, failures: %d\n", failures);
    return failures == 0 ? 0 : 1;
}
