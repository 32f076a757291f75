// Host-only part of the C ABI of librgcsr (include/rgcsr.h): default
// options, status strings and the thread-local error message, the host
// layout (Section 3.4) and its sizes, the row ordering, and the Hybrid width
// rule (Section 3.3).  No device code and no HIP runtime: these calls run on
// machines without a GPU, and this file builds with a plain C++ compiler.
#include <cstring>
#include <string>
#include <vector>

#include <algorithm>

#include "internal.h"
#include "tiles.h"

namespace rg {

// The last error of this thread: a copied message, or (when set, and always
// after an allocation failure) a string literal.
static thread_local std::string g_last_error;
static thread_local const char *g_last_static = nullptr;

void set_last_error(const std::string &msg) noexcept {
    try {
        g_last_error = msg;
        g_last_static = nullptr;
    } catch (...) {
        g_last_static = "host allocation failed";
    }
}

void set_last_error_static(const char *msg) noexcept { g_last_static = msg; }

}  // namespace rg

using namespace rg;

extern "C" {

void rgcsr_default_opts(rgcsr_opts *o) {
    if (!o) return;
    o->group_size = 64;
    o->lanes_per_row = 1;
    o->sort_window = 1;
    o->long_row_threshold = -1;
    o->value_dtype = RGCSR_F32;
    o->keep_csr_map = 0;
    o->build_transpose = 0;
    o->validate = 1;
    o->rows_per_lane = 0;
    o->pad_loads = -1;
    o->load_policy = 0;
    o->tile_min_len = -1;
    o->col_panels = 0;
}

const char *rgcsr_status_string(rgcsr_status s) {
    switch (s) {
    case RGCSR_OK: return "ok";
    case RGCSR_EINVAL: return "invalid argument";
    case RGCSR_ECSR: return "malformed CSR input";
    case RGCSR_ENOMEM: return "out of memory";
    case RGCSR_EOVERFLOW: return "size overflow";
    case RGCSR_EHIP: return "HIP runtime error";
    case RGCSR_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *rgcsr_last_error(void) { return g_last_static ? g_last_static : g_last_error.c_str(); }

const char *rgcsr_version(void) { return "rgcsr 0.1 gfx950"; }

rgcsr_status rgcsr_rcm_order(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                             int32_t *perm) {
    ABI_TRY
    if (n < 0 || (n > 0 && (!row_ptr || !perm)) || (nnz > 0 && !col_idx)) fail(RGCSR_EINVAL, "bad argument");
    validate_csr(n, n, nnz, row_ptr, col_idx);
    rcm_order(n, row_ptr, col_idx, perm);
    ABI_CATCH
}

rgcsr_status rgcsr_layout_sizes(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                                const int32_t *col_idx, const rgcsr_opts *opts, rgcsr_info_t *out) {
    ABI_TRY
    if (!out) fail(RGCSR_EINVAL, "out is null");
    const LayoutParams p = resolve_opts(opts);
    const bool validate = opts ? opts->validate != 0 : true;
    if (validate) validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
    else if (!row_ptr) fail(RGCSR_EINVAL, "row_ptr is null");
    std::vector<int64_t> lens;
    int64_t ng, ns, nl, slots, lz;
    layout_sizes(p, n_rows, row_ptr, &ng, &ns, &nl, &slots, &lz, &lens);
    std::vector<int64_t> lp(1, 0);
    for (int64_t l : lens) lp.push_back(lp.back() + l);
    LongWork work;
    build_long_work(lp, work);
    *out = rgcsr_info_t{};
    out->n_rows = n_rows; out->n_cols = n_cols; out->nnz = nnz;
    out->n_groups = ng; out->n_short = ns; out->n_long = nl; out->slots = slots; out->long_nnz = lz;
    out->n_matrices = 1; out->long_work = (int64_t)(work.wave.size() + work.block.size());
    out->partials = work.n_partials;
    out->group_size = p.G; out->lanes_per_row = p.T;
    out->value_dtype = opts ? opts->value_dtype : RGCSR_F32;
    out->sort_window = p.sigma; out->long_row_threshold = p.tau;
    ABI_CATCH
}

rgcsr_status rgcsr_panel_sizes(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                               const int32_t *col_idx, const rgcsr_opts *opts, int64_t *col_bounds, int64_t *pieces,
                               int64_t *split_rows, int64_t *split_pieces, int64_t *slots, int64_t *long_nnz) {
    ABI_TRY
    if (!opts) fail(RGCSR_EINVAL, "opts is null");
    check_panels(opts->col_panels);
    if (opts->col_panels == 0) fail(RGCSR_EINVAL, "col_panels is 0");
    const LayoutParams p = resolve_opts(opts);
    if (opts->validate) validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
    else if (!row_ptr) fail(RGCSR_EINVAL, "row_ptr is null");
    else if (row_ptr[n_rows] != nnz) fail(RGCSR_ECSR, "row_ptr[n_rows] != nnz");
    PanelBuilt B;
    build_panels(B, p, RGCSR_F32, opts->col_panels, p.tau, n_rows, n_cols, row_ptr, col_idx, nullptr);
    if (col_bounds) std::copy(B.cb.begin(), B.cb.end(), col_bounds);
    if (pieces) *pieces = B.LP.n_rows;
    if (split_rows) *split_rows = (int64_t)B.crow.size();
    if (split_pieces) *split_pieces = B.split_pieces;
    if (slots) *slots = B.LP.slots;
    if (long_nnz) *long_nnz = B.LP.long_nnz;
    ABI_CATCH
}

rgcsr_status rgcsr_tile_sizes(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                              const int32_t *col_idx, const rgcsr_opts *opts, int64_t *n_tiles, int64_t *tiled_rows,
                              int64_t *tile_entries, int64_t *units, int64_t *min_len) {
    ABI_TRY
    if (!opts) fail(RGCSR_EINVAL, "opts is null");
    const LayoutParams p = resolve_opts(opts);
    check_dtype(opts->value_dtype, "value_dtype");
    if (opts->validate) validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
    else if (!row_ptr) fail(RGCSR_EINVAL, "row_ptr is null");
    else if (row_ptr[n_rows] != nnz) fail(RGCSR_ECSR, "row_ptr[n_rows] != nnz");
    // the layout's long-row segment (columns only), then the tile selection
    // that a device handle makes from it
    HostLayout L;
    L.G = p.G; L.T = p.T; L.sigma = p.sigma; L.tau = p.tau;
    L.vdt = opts->value_dtype; L.esz = dtype_size(L.vdt);
    append_layout(L, p, n_rows, n_cols, row_ptr, col_idx, nullptr, L.esz, 0);
    HostTiles T;
    build_tiles(L, opts->tile_min_len, T);
    if (n_tiles) *n_tiles = T.n_tiles;
    if (tiled_rows) *tiled_rows = T.n_trows;
    if (tile_entries) *tile_entries = T.n_ent;
    if (units) *units = (int64_t)T.units.size();
    if (min_len) *min_len = T.min_len;
    ABI_CATCH
}

rgcsr_status rgcsr_layout_host(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                               const int32_t *col_idx, const void *vals, rgcsr_dtype vals_dtype,
                               const rgcsr_opts *opts, int64_t *gp, int32_t *short_len, int32_t *short_row,
                               void *slot_val, int32_t *slot_col, int32_t *long_row, int64_t *long_ptr,
                               void *long_val, int32_t *long_col) {
    ABI_TRY
    const LayoutParams p = resolve_opts(opts);
    const int vdt = opts ? opts->value_dtype : RGCSR_F32;
    check_dtype(vdt, "value_dtype");
    check_dtype(vals_dtype, "vals");
    const bool validate = opts ? opts->validate != 0 : true;
    Built B;
    const int64_t *rps[1] = {row_ptr};
    const int32_t *cols[1] = {col_idx};
    const void *vs[1] = {vals};
    (void)nnz;
    if (validate) validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
    build_host(B, p, vdt, 1, &n_rows, &n_cols, rps, cols, vs, vals_dtype, false, false, false);
    const HostLayout &L = B.L;
    auto put = [](auto *dst, const auto &v) {
        if (dst && !v.empty()) memcpy(dst, v.data(), v.size() * sizeof(v[0]));
    };
    put(gp, L.gp);
    put(short_len, L.short_len);
    put(short_row, L.short_row);
    put((uint8_t *)slot_val, L.slot_val);
    put(slot_col, L.slot_col);
    put(long_row, L.long_row);
    put(long_ptr, L.long_ptr);
    put((uint8_t *)long_val, L.long_val);
    put(long_col, L.long_col);
    ABI_CATCH
}

rgcsr_status hyb_choose_width(int64_t n_rows, const int64_t *row_ptr, rgcsr_dtype value_dtype, int64_t *k1) {
    ABI_TRY
    if (!row_ptr || !k1 || n_rows < 0) fail(RGCSR_EINVAL, "bad argument");
    check_dtype(value_dtype, "value_dtype");
    *k1 = hyb_width_rule(n_rows, row_ptr, dtype_size(value_dtype));
    ABI_CATCH
}

}  // extern "C"
