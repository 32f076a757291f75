// Host format library: CSR validation, the RgCSR layout (Section 3.4 plus the
// lanes-per-row, sort-window and long-row readings), long-row work items,
// CSR transpose with a source map, the Hybrid ELL width rule (Section 3.3)
// and value conversion.  Plain C++17; no device code.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>

#include "internal.h"

namespace rg {

[[noreturn]] void fail(rgcsr_status st, const std::string &msg) { throw Error{st, msg}; }

LayoutParams resolve_opts(const rgcsr_opts *opts) {
    rgcsr_opts d;
    rgcsr_default_opts(&d);
    const rgcsr_opts &o = opts ? *opts : d;
    LayoutParams p;
    p.G = o.group_size == 0 ? 64 : o.group_size;
    p.T = o.lanes_per_row == 0 ? 1 : o.lanes_per_row;
    p.sigma = o.sort_window == 0 ? 1 : o.sort_window;
    p.tau = o.long_row_threshold;
    if (p.G < 1) fail(RGCSR_EINVAL, "group_size must be >= 1");
    if (p.T != 1 && p.T != 2 && p.T != 4 && p.T != 8)
        fail(RGCSR_EINVAL, "lanes_per_row must be 1, 2, 4 or 8");
    if (p.sigma < 1) fail(RGCSR_EINVAL, "sort_window must be >= 1");
    if (p.tau < 0) p.tau = -1;
    return p;
}

void validate_csr(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *rp,
                  const int32_t *col) {
    if (n_rows < 0 || n_cols < 0 || nnz < 0) fail(RGCSR_EINVAL, "negative size");
    if (n_rows > INT32_MAX || n_cols > INT32_MAX)
        fail(RGCSR_EOVERFLOW, "n_rows and n_cols must fit int32 column/row indices");
    if (!rp) fail(RGCSR_EINVAL, "row_ptr is null");
    if (nnz > 0 && !col) fail(RGCSR_EINVAL, "col_idx is null");
    if (rp[0] != 0) fail(RGCSR_ECSR, "row_ptr[0] != 0");
    for (int64_t i = 0; i < n_rows; i++) {
        const int64_t b = rp[i], e = rp[i + 1];
        if (e < b) fail(RGCSR_ECSR, "row_ptr decreases at row " + std::to_string(i));
        if (e > nnz) fail(RGCSR_ECSR, "row_ptr exceeds nnz at row " + std::to_string(i));
        if (e - b > INT32_MAX) fail(RGCSR_EOVERFLOW, "row longer than int32");
        int64_t prev = -1;
        for (int64_t k = b; k < e; k++) {
            const int64_t c = col[k];
            if (c < 0 || c >= n_cols)
                fail(RGCSR_ECSR, "column out of range in row " + std::to_string(i));
            if (c <= prev)
                fail(RGCSR_ECSR, "columns not strictly ascending in row " + std::to_string(i));
            prev = c;
        }
    }
    if (rp[n_rows] != nnz) fail(RGCSR_ECSR, "row_ptr[n_rows] != nnz");
}

bool HostLayout::has_gaps() const {
    for (size_t g = 0; g < gend.size(); g++)
        if (gend[g] != gp[g + 1]) return true;
    return false;
}

bool HostLayout::short_identity() const {
    for (int64_t i = 0; i < ns; i++)
        if (short_row[i] != i) return false;
    return true;
}

// Row order after the sort-window step and the short/long split.
static void order_and_split(const LayoutParams &p, int64_t n_rows, const int64_t *rp,
                            std::vector<int32_t> &shortv, std::vector<int32_t> &longv) {
    std::vector<int32_t> ord(n_rows);
    std::iota(ord.begin(), ord.end(), 0);
    auto longer = [rp](int32_t a, int32_t b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; };
    if (p.sigma > 1) {
        for (int64_t w0 = 0; w0 < n_rows; w0 += p.sigma) {
            const int64_t w1 = std::min<int64_t>(n_rows, w0 + p.sigma);
            std::stable_sort(ord.begin() + w0, ord.begin() + w1, longer);
        }
    }
    shortv.clear();
    longv.clear();
    shortv.reserve(n_rows);
    for (int32_t r : ord) {
        if (p.tau >= 0 && rp[r + 1] - rp[r] > p.tau)
            longv.push_back(r);
        else
            shortv.push_back(r);
    }
    // Equal lengths already appear in ascending original row within the
    // sorted order, so a stable sort gives (length desc, row asc).
    std::stable_sort(longv.begin(), longv.end(), longer);
}

static inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

void short_lengths(const LayoutParams &p, int64_t n_rows, const int64_t *rp, std::vector<int32_t> &lens,
                   int64_t *n_long, int64_t *long_nnz) {
    std::vector<int32_t> sv, lv;
    order_and_split(p, n_rows, rp, sv, lv);
    lens.resize(sv.size());
    for (size_t i = 0; i < sv.size(); i++) lens[i] = (int32_t)(rp[sv[i] + 1] - rp[sv[i]]);
    int64_t lz = 0;
    for (int32_t r : lv) lz += rp[r + 1] - rp[r];
    *n_long = (int64_t)lv.size();
    *long_nnz = lz;
}

int64_t group_slots(const std::vector<int32_t> &lens, int32_t G, int32_t T) {
    int64_t s = 0;
    const int64_t n = (int64_t)lens.size();
    for (int64_t g0 = 0; g0 < n; g0 += G) {
        const int64_t g1 = std::min<int64_t>(n, g0 + G);
        int64_t w = 0;
        for (int64_t i = g0; i < g1; i++) w = std::max<int64_t>(w, lens[i]);
        s += (g1 - g0) * round_up(w, T);
    }
    return s;
}

void layout_sizes(const LayoutParams &p, int64_t n_rows, const int64_t *rp, int64_t *ng,
                  int64_t *ns, int64_t *nl, int64_t *slots, int64_t *long_nnz,
                  std::vector<int64_t> *long_lens_sorted) {
    std::vector<int32_t> sv, lv;
    order_and_split(p, n_rows, rp, sv, lv);
    int64_t s = 0;
    const int64_t n_short = (int64_t)sv.size();
    for (int64_t g0 = 0; g0 < n_short; g0 += p.G) {
        const int64_t g1 = std::min<int64_t>(n_short, g0 + p.G);
        int64_t w = 0;
        for (int64_t i = g0; i < g1; i++) w = std::max<int64_t>(w, rp[sv[i] + 1] - rp[sv[i]]);
        s += (g1 - g0) * round_up(w, p.T);
    }
    int64_t lz = 0;
    if (long_lens_sorted) long_lens_sorted->clear();
    for (int32_t r : lv) {
        lz += rp[r + 1] - rp[r];
        if (long_lens_sorted) long_lens_sorted->push_back(rp[r + 1] - rp[r]);
    }
    *ng = (n_short + p.G - 1) / p.G;
    *ns = n_short;
    *nl = (int64_t)lv.size();
    *slots = s;
    *long_nnz = lz;
}

template <int ESZ>
static inline void copy_elem(uint8_t *dst, const uint8_t *src) {
    memcpy(dst, src, ESZ);
}

void append_layout(HostLayout &L, const LayoutParams &p, int64_t n_rows, int64_t n_cols,
                   const int64_t *rp, const int32_t *col, const uint8_t *vals, int esz,
                   uint8_t pad_byte) {
    const int64_t rbase = L.n_rows, cbase = L.n_cols;
    if (rbase + n_rows > INT32_MAX || cbase + n_cols > INT32_MAX)
        fail(RGCSR_EOVERFLOW, "total rows/columns exceed int32");
    std::vector<int32_t> sv, lv;
    order_and_split(p, n_rows, rp, sv, lv);

    // A matrix after the first starts its groups at a multiple of 64 slots,
    // so that a wavefront's 64 consecutive slots of a step stay within the
    // fewest cache lines: a partial last group of the previous matrix would
    // otherwise shift every later group off that alignment.  The skipped
    // slots belong to no group (zero values, in-range columns).
    if (L.n_matrices > 0 && ((int64_t)p.G * p.T) % 64 == 0 && L.slots % 64 != 0) {
        const int64_t aligned = round_up(L.slots, 64);
        L.slot_col.resize(aligned, (int32_t)cbase > 0 ? (int32_t)(cbase - 1) : 0);
        if (vals) L.slot_val.resize((size_t)aligned * esz, pad_byte);
        L.slots = aligned;
        L.gp.back() = aligned;
    }
    // groups of short rows
    const int64_t ng_before = L.ng;
    const int64_t n_short = (int64_t)sv.size();
    const int64_t slot0 = L.slots;
    std::vector<int64_t> gstart;  // local group starts in sv
    int64_t slots = slot0;
    for (int64_t g0 = 0; g0 < n_short; g0 += p.G) {
        const int64_t g1 = std::min<int64_t>(n_short, g0 + p.G);
        int64_t w = 0;
        for (int64_t i = g0; i < g1; i++) w = std::max<int64_t>(w, rp[sv[i] + 1] - rp[sv[i]]);
        gstart.push_back(g0);
        slots += (g1 - g0) * round_up(w, p.T);
        L.gp.push_back(slots);
        L.gend.push_back(slots);
        L.grp_row0.push_back((int32_t)(L.ns + g1));
        if (L.ns + g1 > INT32_MAX) fail(RGCSR_EOVERFLOW, "short rows exceed int32");
    }
    L.slots = slots;
    L.ng += (int64_t)gstart.size();

    // exact reserve() on every append of a batch would copy the arrays each
    // time; push_back grows them geometrically
    for (int32_t r : sv) {
        L.short_len.push_back((int32_t)(rp[r + 1] - rp[r]));
        L.short_row.push_back((int32_t)(rbase + r));
    }

    // scatter: nonzero j of local row t -> slot gp + (j/T)*(s*T) + t*T + j%T
    L.slot_col.resize(slots);
    if (vals) L.slot_val.resize((size_t)slots * esz);
    const int64_t T = p.T;
    int64_t gbase = slot0;
    for (size_t gi = 0; gi < gstart.size(); gi++) {
        const int64_t g0 = gstart[gi];
        const int64_t s = std::min<int64_t>(n_short, g0 + p.G) - g0;
        const int64_t gend = L.gend[L.gend.size() - gstart.size() + gi];
        const int64_t W = s ? (gend - gbase) / s : 0;
        for (int64_t t = 0; t < s; t++) {
            const int32_t r = sv[g0 + t];
            const int64_t b = rp[r], len = rp[r + 1] - b;
            const int32_t ghost = len ? (int32_t)(col[b + len - 1] + cbase) : (int32_t)cbase;
            for (int64_t j = 0; j < W; j++) {
                const int64_t slot = gbase + (j / T) * (s * T) + t * T + (j % T);
                if (j < len) {
                    L.slot_col[slot] = (int32_t)(col[b + j] + cbase);
                    if (vals) memcpy(&L.slot_val[(size_t)slot * esz], vals + (size_t)(b + j) * esz, esz);
                } else {
                    L.slot_col[slot] = ghost;
                    if (vals) memset(&L.slot_val[(size_t)slot * esz], pad_byte, esz);
                }
            }
        }
        gbase = gend;
    }
    L.ns += n_short;

    // long rows, CSR-contiguous in long-list order
    for (int32_t r : lv) {
        const int64_t b = rp[r], len = rp[r + 1] - b;
        L.long_row.push_back((int32_t)(rbase + r));
        const int64_t at = L.long_nnz;
        L.long_nnz += len;
        L.long_ptr.push_back(L.long_nnz);
        L.long_col.resize(L.long_nnz);
        for (int64_t j = 0; j < len; j++) L.long_col[at + j] = (int32_t)(col[b + j] + cbase);
        if (vals) {
            L.long_val.resize((size_t)L.long_nnz * esz);
            memcpy(&L.long_val[(size_t)at * esz], vals + (size_t)b * esz, (size_t)len * esz);
        }
    }
    L.nl += (int64_t)lv.size();

    L.n_rows += n_rows;
    L.n_cols += n_cols;
    L.nnz += rp[n_rows];
    L.n_matrices++;
    L.row_off.push_back(L.n_rows);
    L.col_off.push_back(L.n_cols);
    // groups are ragged when any group before the last has fewer than G rows;
    // only the previous matrix's last group and this matrix's groups can make
    // it so, the earlier ones were checked by earlier appends
    const int64_t g_check0 = std::max<int64_t>(0, ng_before - 1);
    for (int64_t g = g_check0; g + 1 < L.ng && !L.ragged; g++)
        if (L.grp_row0[g + 1] - L.grp_row0[g] != p.G) L.ragged = true;
}

static int32_t lanes_for(int64_t len) {
    // smallest power of two >= ceil(len / kWaveUnroll), at most 64
    int64_t need = (len + kWaveUnroll - 1) / kWaveUnroll;
    int32_t t = 1;
    while (t < need && t < 64) t <<= 1;
    return t;
}

void build_long_work(const std::vector<int64_t> &long_ptr, LongWork &W) {
    W = LongWork{};
    const int64_t nl = (int64_t)long_ptr.size() - 1;
    int64_t i = 0;
    while (i < nl) {
        const int64_t len = long_ptr[i + 1] - long_ptr[i];
        if (len > kWaveRowMax) {
            const int64_t nch = (len + kBlockChunk - 1) / kBlockChunk;
            if (W.n_partials + nch > INT32_MAX) fail(RGCSR_EOVERFLOW, "too many long-row chunks");
            const int32_t pbase = nch > 1 ? (int32_t)W.n_partials : 0;
            for (int64_t c = 0; c < nch; c++)
                W.block.push_back(LongItem{(int32_t)i, (int32_t)c, (int32_t)nch, pbase});
            if (nch > 1) {
                W.combine.push_back(LongItem{(int32_t)i, 0, (int32_t)nch, pbase});
                W.n_partials += nch;
            }
            i++;
            continue;
        }
        const int32_t T = lanes_for(len);
        const int32_t cap = 64 / T;
        int32_t cnt = 1;
        while (cnt < cap && i + cnt < nl) {
            const int64_t l2 = long_ptr[i + cnt + 1] - long_ptr[i + cnt];
            if (l2 > kWaveRowMax || lanes_for(l2) != T) break;
            cnt++;
        }
        W.wave.push_back(LongItem{(int32_t)i, cnt, T, 0});
        i += cnt;
    }
}

void transpose_csr(int64_t n_rows, int64_t n_cols, const int64_t *rp, const int32_t *col,
                   std::vector<int64_t> &rpT, std::vector<int32_t> &colT,
                   std::vector<int32_t> &srcT) {
    const int64_t nnz = rp[n_rows];
    if (nnz > INT32_MAX) fail(RGCSR_EOVERFLOW, "transpose map needs nnz < 2^31");
    rpT.assign(n_cols + 1, 0);
    for (int64_t k = 0; k < nnz; k++) rpT[col[k] + 1]++;
    std::partial_sum(rpT.begin(), rpT.end(), rpT.begin());
    std::vector<int64_t> fill(rpT.begin(), rpT.end() - 1);
    colT.resize(nnz);
    srcT.resize(nnz);
    for (int64_t r = 0; r < n_rows; r++)
        for (int64_t k = rp[r]; k < rp[r + 1]; k++) {
            const int64_t d = fill[col[k]]++;
            colT[d] = (int32_t)r;
            srcT[d] = (int32_t)k;
        }
}

void check_dtype(int dt, const char *what) {
    if (dtype_size(dt) == 0) fail(RGCSR_EINVAL, std::string("bad dtype for ") + what);
}

void build_host(Built &B, const LayoutParams &p, int vdt, int32_t count, const int64_t *n_rows,
                const int64_t *n_cols, const int64_t *const *rp, const int32_t *const *col,
                const void *const *vals, int vals_dt, bool validate, bool keep_map, bool transpose) {
    const int esz = dtype_size(vdt);
    B.L.G = p.G; B.L.T = p.T; B.L.sigma = p.sigma; B.L.tau = p.tau; B.L.vdt = vdt; B.L.esz = esz;
    B.has_T = transpose;
    if (transpose) {
        B.LT = B.L;
        B.LTmap = B.L;
        B.LTmap.esz = 4;
    }
    if (keep_map || transpose) B.row_ptr.assign(1, 0);
    int64_t nnz_base = 0;
    // append_layout treats a null value pointer as "sizes only", so the value
    // buffers stay allocated for matrices without nonzeros
    std::vector<uint8_t> conv;
    conv.reserve((size_t)esz);
    for (int32_t m = 0; m < count; m++) {
        const int64_t nr = n_rows[m], nc = n_cols[m];
        if (nr < 0 || nc < 0) fail(RGCSR_EINVAL, "negative matrix size");
        if (!rp[m]) fail(RGCSR_EINVAL, "row_ptr is null");
        const int64_t nnz = rp[m][nr];
        if (validate) validate_csr(nr, nc, nnz, rp[m], col[m]);
        if (nnz > 0 && !vals[m]) fail(RGCSR_EINVAL, "vals is null");
        conv.resize((size_t)nnz * esz);
        if (nnz) convert_values(vals[m], vals_dt, conv.data(), vdt, nnz);
        append_layout(B.L, p, nr, nc, rp[m], col[m], conv.data(), esz, 0);
        if (!B.row_ptr.empty())
            for (int64_t r = 0; r < nr; r++) B.row_ptr.push_back(nnz_base + rp[m][r + 1]);
        if (transpose) {
            std::vector<int64_t> rpT;
            std::vector<int32_t> colT, srcT;
            transpose_csr(nr, nc, rp[m], col[m], rpT, colT, srcT);
            std::vector<uint8_t> valsT((size_t)std::max<int64_t>(nnz, 1) * esz);
            for (int64_t k = 0; k < nnz; k++) memcpy(&valsT[(size_t)k * esz], &conv[(size_t)srcT[k] * esz], esz);
            std::vector<int32_t> mapT(std::max<int64_t>(nnz, 1));
            if (nnz_base + nnz > INT32_MAX) fail(RGCSR_EOVERFLOW, "transpose map needs total nnz < 2^31");
            for (int64_t k = 0; k < nnz; k++) mapT[k] = (int32_t)(srcT[k] + nnz_base);
            append_layout(B.LT, p, nc, nr, rpT.data(), colT.data(), valsT.data(), esz, 0);
            append_layout(B.LTmap, p, nc, nr, rpT.data(), colT.data(), (const uint8_t *)mapT.data(), 4, 0xff);
        }
        nnz_base += nnz;
    }
    build_long_work(B.L.long_ptr, B.L.work);
    if (transpose) build_long_work(B.LT.long_ptr, B.LT.work);
}

int64_t hyb_width_rule(int64_t n_rows, const int64_t *rp, int s_v) {
    // cost(k) = k * n_pad * (s_v + 4) + 3 * (s_v + 8) * excess(k),
    // excess(k) = sum_i max(0, len_i - k), updated incrementally.
    int64_t kmax = 0;
    for (int64_t i = 0; i < n_rows; i++) kmax = std::max(kmax, rp[i + 1] - rp[i]);
    std::vector<int64_t> hist(kmax + 2, 0);
    for (int64_t i = 0; i < n_rows; i++) hist[rp[i + 1] - rp[i]]++;
    const int64_t n_pad = round_up(n_rows, 64);
    int64_t longer = n_rows - hist[0];  // rows with len > k, at k = 0
    int64_t excess = rp[n_rows];
    int64_t best = 0, best_cost = 3 * (s_v + 8) * excess;
    for (int64_t k = 1; k <= kmax; k++) {
        excess -= longer;
        longer -= hist[k];
        const int64_t cost = k * n_pad * (s_v + 4) + 3 * (s_v + 8) * excess;
        if (cost < best_cost) {
            best_cost = cost;
            best = k;
        }
    }
    return best;
}

void convert_values(const void *src, int sdt, void *dst, int ddt, int64_t n) {
    if (sdt == ddt) {
        memcpy(dst, src, (size_t)n * dtype_size(sdt));
        return;
    }
    auto to_f32 = [&](int64_t i) -> float {
        switch (sdt) {
        case RGCSR_F64: return (float)((const double *)src)[i];
        case RGCSR_F32: return ((const float *)src)[i];
        case RGCSR_BF16: return bf16_to_f32(((const uint16_t *)src)[i]);
        default: {
            // float16 -> float32 exactly
            uint16_t h = ((const uint16_t *)src)[i];
            uint32_t sign = (uint32_t)(h & 0x8000u) << 16, e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
            if (e == 0x1f) return bits_f32(sign | 0x7f800000u | (m << 13));
            if (e == 0) return (sign ? -1.0f : 1.0f) * std::ldexp((float)m, -24);
            return bits_f32(sign | ((e + 112u) << 23) | (m << 13));
        }
        }
    };
    for (int64_t i = 0; i < n; i++) {
        switch (ddt) {
        case RGCSR_F64:
            ((double *)dst)[i] = sdt == RGCSR_F64 ? ((const double *)src)[i] : (double)to_f32(i);
            break;
        case RGCSR_F32: ((float *)dst)[i] = to_f32(i); break;
        case RGCSR_F16: ((uint16_t *)dst)[i] = f32_to_f16_rne(to_f32(i)); break;
        case RGCSR_BF16: ((uint16_t *)dst)[i] = f32_to_bf16_rne(to_f32(i)); break;
        default: fail(RGCSR_EINVAL, "bad dtype");
        }
    }
}

}  // namespace rg
