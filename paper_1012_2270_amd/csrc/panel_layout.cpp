// Column panels of one CSR matrix (host).
//
// Every nonzero gathers x at its column; for a matrix whose columns are
// spread over all of x (random or power-law sparsity), the gathers of one
// XCD touch all of x and its L2 keeps only a part of it.  Split by column
// into panels, each XCD multiplies one panel at a time and keeps that
// panel's slice of x in its own L2 -- the reuse of x through a cache that
// Section 4.3 studies with the texture cache, arranged for eight L2s.  Rows
// of at most `whole_max` nonzeros are not split (a row of a few nonzeros
// gains little from a cached slice and would pay for a sum per piece): they
// form one more matrix of whole rows, whose work goes to every XCD.  The
// panels and the whole rows are laid out with the same row groups, sort
// windows and long-row split as the whole matrix (Sections 3.2 and 4.4.2).
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace rg {

void check_panels(int32_t P) {
    if (P != 0 && (P < kPanelXcds || P > kPanelMax || P % kPanelXcds != 0))
        fail(RGCSR_EINVAL, "col_panels must be 0 or a multiple of 8 from 8 to 64");
}

void build_panels(PanelBuilt &B, const LayoutParams &p, int vdt, int32_t P, int64_t whole_max, int64_t n_rows,
                  int64_t n_cols, const int64_t *rp, const int32_t *col, const uint8_t *vals) {
    if (P < 1 || P > kPanelMax) fail(RGCSR_EINVAL, "bad panel count");
    const int esz = dtype_size(vdt);
    const int64_t nnz = rp[n_rows];
    if (nnz > INT32_MAX || n_rows + nnz > INT32_MAX) fail(RGCSR_EOVERFLOW, "column panels need nnz + rows < 2^31");
    // value-initialized with (): a braced temporary of an aggregate whose
    // members allocate is not cleaned up by GCC before 13 when one of them
    // throws (the members built before it leak)
    B = PanelBuilt();
    B.P = P;
    // bounds: cb[q] is the first column at which the nonzeros of the columns
    // before it reach q * nnz / P (nondecreasing; empty panels are allowed)
    std::vector<int64_t> ccount((size_t)n_cols + 1, 0);
    for (int64_t k = 0; k < nnz; k++) ccount[(size_t)col[k] + 1]++;
    for (int64_t c = 0; c < n_cols; c++) ccount[c + 1] += ccount[c];
    B.cb.assign((size_t)P + 1, 0);
    for (int32_t q = 1; q < P; q++) {
        const int64_t target = (nnz * q + P - 1) / P;
        B.cb[q] = std::lower_bound(ccount.begin(), ccount.end(), target) - ccount.begin();
        B.cb[q] = std::max(B.cb[q - 1], std::min(B.cb[q], n_cols));
    }
    B.cb[P] = n_cols;
    auto panel_of = [&](int32_t c) {
        return (int32_t)(std::upper_bound(B.cb.begin() + 1, B.cb.end(), (int64_t)c) - (B.cb.begin() + 1));
    };
    // whole rows (empty ones included) are matrix P; the entries of split rows
    // carry their panel
    auto whole = [&](int64_t r) { return rp[r + 1] - rp[r] <= whole_max; };
    std::vector<int32_t> pan((size_t)nnz);
    for (int64_t r = 0; r < n_rows; r++)
        for (int64_t k = rp[r]; k < rp[r + 1]; k++) pan[k] = whole(r) ? P : panel_of(col[k]);

    // split rows and their pieces per panel; whole rows one piece each
    std::vector<int64_t> rows_in((size_t)P + 1, 0);
    B.cptr.assign(1, 0);
    {
        std::vector<int32_t> seen((size_t)P, -1);
        for (int64_t r = 0; r < n_rows; r++) {
            if (whole(r)) {
                rows_in[P]++;
                continue;
            }
            int32_t n = 0;
            for (int64_t k = rp[r]; k < rp[r + 1]; k++)
                if (seen[pan[k]] != (int32_t)r) {
                    seen[pan[k]] = (int32_t)r;
                    rows_in[pan[k]]++;
                    n++;
                }
            B.crow.push_back((int32_t)r);
            B.cptr.push_back(B.cptr.back() + n);
        }
    }
    std::vector<int64_t> piece0((size_t)P + 2, 0);  // first piece of each panel, then of the whole rows
    for (int32_t q = 0; q <= P; q++) piece0[q + 1] = piece0[q] + rows_in[q];
    B.split_pieces = piece0[P];
    B.vidx.assign((size_t)B.cptr.back(), 0);

    B.LP = HostLayout();
    B.LP.G = p.G; B.LP.T = p.T; B.LP.sigma = p.sigma; B.LP.tau = p.tau; B.LP.vdt = vdt; B.LP.esz = esz;
    B.LP.n_matrices = 0;
    B.LPmap = B.LP;
    B.LPmap.esz = 4;
    B.grp_off.assign(1, 0);
    B.long_off.assign(1, 0);
    std::vector<int64_t> prp;
    std::vector<int32_t> pcol, pmap, whole_rows;
    std::vector<uint8_t> pval;
    // append_layout treats a null value pointer as "sizes only": keep the
    // value buffers allocated even for a panel without entries
    pmap.reserve(1);
    pval.reserve((size_t)esz);
    std::vector<int32_t> next(B.cptr.begin(), B.cptr.end() - 1);  // next piece slot of each split row in vidx
    for (int32_t q = 0; q <= P; q++) {
        // panel q as a row-compressed CSR matrix with panel-local columns;
        // q = P: the whole rows, with all columns (append_layout adds the
        // columns of the panels before, so theirs are shifted back by n_cols)
        const int64_t c0 = q < P ? B.cb[q] : n_cols;
        prp.assign(1, 0);
        pcol.clear();
        pmap.clear();
        pval.clear();
        int64_t piece = piece0[q], split = 0;
        for (int64_t r = 0; r < n_rows; r++) {
            const bool w = whole(r);
            if (w != (q == P)) {
                split += !w;
                continue;
            }
            const int64_t before = (int64_t)pcol.size();
            for (int64_t k = rp[r]; k < rp[r + 1]; k++)
                if (pan[k] == q) {
                    pcol.push_back((int32_t)(col[k] - c0));
                    pmap.push_back((int32_t)k);
                    if (vals) pval.insert(pval.end(), vals + (size_t)k * esz, vals + (size_t)(k + 1) * esz);
                }
            if (w) {
                prp.push_back((int64_t)pcol.size());
                whole_rows.push_back((int32_t)r);
                piece++;
            } else {
                if ((int64_t)pcol.size() > before) {
                    prp.push_back((int64_t)pcol.size());
                    B.vidx[next[split]++] = (int32_t)piece++;
                }
                split++;
            }
        }
        const int64_t nr = (int64_t)prp.size() - 1, nc = q < P ? B.cb[q + 1] - B.cb[q] : 0;
        append_layout(B.LP, p, nr, nc, prp.data(), pcol.data(), vals ? pval.data() : nullptr, esz, 0);
        append_layout(B.LPmap, p, nr, nc, prp.data(), pcol.data(), (const uint8_t *)pmap.data(), 4, 0xff);
        B.grp_off.push_back(B.LP.ng);
        B.long_off.push_back(B.LP.nl);
    }
    // output codes: a whole row writes its row of y; piece v of a split row
    // writes slot v of the per-piece sums, coded -1 - v
    auto code = [&](int32_t v) { return v < B.split_pieces ? -1 - v : whole_rows[v - B.split_pieces]; };
    for (int32_t &r : B.LP.short_row) r = code(r);
    for (int32_t &r : B.LP.long_row) r = code(r);
    build_long_work(B.LP.long_ptr, B.LP.work);
}

}  // namespace rg
