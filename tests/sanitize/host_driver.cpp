// Sanitizer driver for the host part of librgcsr (built with
// -fsanitize=address,undefined from host_layout.cpp, ordering.cpp,
// tile_layout.cpp, panel_layout.cpp and abi_host.cpp; no device code).  It runs the host-only C entry points on
// seeded random and malformed CSR inputs, then repeats a conversion with the
// n-th host allocation failing for every n until one succeeds: each failing
// call must return RGCSR_ENOMEM, and LeakSanitizer (at exit) must find no
// leak.  Exit status 0 when every check holds.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "../../include/rgcsr.h"

// ---- allocation-failure hook (test only): while armed (inside a library
// call), operator new throws once the countdown reaches zero; -1 never fails
static long g_fail_countdown = -1;
static bool g_armed = false;

static void *counted_alloc(std::size_t n) {
    if (g_armed && g_fail_countdown == 0) throw std::bad_alloc();
    if (g_armed && g_fail_countdown > 0) g_fail_countdown--;
    void *p = std::malloc(n ? n : 1);
    if (!p) throw std::bad_alloc();
    return p;
}
void *operator new(std::size_t n) { return counted_alloc(n); }
void *operator new[](std::size_t n) { return counted_alloc(n); }
void *operator new(std::size_t n, const std::nothrow_t &) noexcept {
    try {
        return counted_alloc(n);
    } catch (...) {
        return nullptr;
    }
}
void *operator new[](std::size_t n, const std::nothrow_t &) noexcept {
    try {
        return counted_alloc(n);
    } catch (...) {
        return nullptr;
    }
}
void operator delete(void *p, const std::nothrow_t &) noexcept { std::free(p); }
void operator delete[](void *p, const std::nothrow_t &) noexcept { std::free(p); }
void operator delete(void *p) noexcept { std::free(p); }
void operator delete[](void *p) noexcept { std::free(p); }
void operator delete(void *p, std::size_t) noexcept { std::free(p); }
void operator delete[](void *p, std::size_t) noexcept { std::free(p); }

static int g_failures = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);             \
            std::fprintf(stderr, "\n");                    \
            g_failures++;                                  \
        }                                                  \
    } while (0)

struct Csr {
    int64_t n_rows, n_cols;
    std::vector<int64_t> rp;
    std::vector<int32_t> col;
    std::vector<float> val;
};

// seeded random CSR: row lengths up to max_len (a few rows long), ascending
// distinct columns, some empty rows
static Csr random_csr(std::mt19937_64 &rng, int64_t n_rows, int64_t n_cols, int max_len, int n_long, int long_len) {
    Csr A{n_rows, n_cols, {0}, {}, {}};
    std::uniform_int_distribution<int> len_d(0, max_len);
    std::uniform_real_distribution<float> val_d(-1.f, 1.f);
    std::vector<char> used(n_cols, 0);
    for (int64_t r = 0; r < n_rows; r++) {
        int len = (r % 97 < n_long && r < 97 * 4) ? long_len : len_d(rng);
        if (len > n_cols) len = (int)n_cols;
        std::vector<int32_t> cs;
        std::uniform_int_distribution<int64_t> c_d(0, n_cols > 0 ? n_cols - 1 : 0);
        while ((int)cs.size() < len) {
            const int32_t c = (int32_t)c_d(rng);
            if (!used[c]) {
                used[c] = 1;
                cs.push_back(c);
            }
        }
        for (int32_t c : cs) used[c] = 0;
        std::sort(cs.begin(), cs.end());
        for (int32_t c : cs) {
            A.col.push_back(c);
            A.val.push_back(val_d(rng));
        }
        A.rp.push_back((int64_t)A.col.size());
    }
    return A;
}

static rgcsr_status layout_all(const Csr &A, const rgcsr_opts &o) {
    rgcsr_info_t info;
    const int64_t nnz = A.rp.back();
    g_armed = true;
    rgcsr_status s = rgcsr_layout_sizes(A.n_rows, A.n_cols, nnz, A.rp.data(), A.col.data(), &o, &info);
    g_armed = false;
    if (s != RGCSR_OK) return s;
    const int esz = o.value_dtype == RGCSR_F64 ? 8 : (o.value_dtype == RGCSR_F32 ? 4 : 2);
    std::vector<int64_t> gp(info.n_groups + 1), long_ptr(info.n_long + 1);
    std::vector<int32_t> short_len(info.n_short), short_row(info.n_short), slot_col(info.slots);
    std::vector<int32_t> long_row(info.n_long), long_col(info.long_nnz);
    std::vector<uint8_t> slot_val((size_t)info.slots * esz), long_val((size_t)info.long_nnz * esz);
    g_armed = true;
    s = rgcsr_layout_host(A.n_rows, A.n_cols, nnz, A.rp.data(), A.col.data(), A.val.data(), RGCSR_F32, &o,
                          gp.data(), short_len.data(), short_row.data(), slot_val.data(), slot_col.data(),
                          long_row.data(), long_ptr.data(), long_val.data(), long_col.data());
    g_armed = false;
    if (s != RGCSR_OK) return s;
    // every nonzero lands exactly once: grouped lengths plus long lengths
    int64_t total = long_ptr.back();
    for (int32_t l : short_len) total += l;
    CHECK(total == nnz, "layout holds %lld of %lld nonzeros", (long long)total, (long long)nnz);
    CHECK(gp.back() == info.slots, "last group pointer");
    return s;
}

// Column-panel sizes: bounds nondecreasing from 0 to n_cols, every split
// row with at least one piece, every whole row one piece.
static rgcsr_status panels_all(const Csr &A, rgcsr_opts o, int32_t P) {
    o.col_panels = P;
    std::vector<int64_t> cb((size_t)P + 1, -1);
    int64_t pieces = -1, split_rows = -1, split_pieces = -1, slots = -1, long_nnz = -1;
    g_armed = true;
    const rgcsr_status s = rgcsr_panel_sizes(A.n_rows, A.n_cols, A.rp.back(), A.rp.data(), A.col.data(), &o,
                                             cb.data(), &pieces, &split_rows, &split_pieces, &slots, &long_nnz);
    g_armed = false;
    if (s != RGCSR_OK) return s;
    CHECK(cb[0] == 0 && cb[P] == A.n_cols, "panel bounds end points");
    for (int32_t q = 0; q < P; q++) CHECK(cb[q] <= cb[q + 1], "panel bounds decrease");
    int64_t whole = 0, split = 0;
    for (int64_t r = 0; r < A.n_rows; r++) (A.rp[r + 1] - A.rp[r] > o.long_row_threshold ? split : whole)++;
    CHECK(split_rows == split, "split rows %lld, expected %lld", (long long)split_rows, (long long)split);
    CHECK(pieces == whole + split_pieces, "pieces %lld", (long long)pieces);
    CHECK(split_pieces >= split - [&] {
        int64_t empty = 0;
        for (int64_t r = 0; r < A.n_rows; r++) empty += A.rp[r + 1] == A.rp[r] && o.long_row_threshold < 0;
        return empty;
    }(), "a split row without pieces");
    CHECK(slots >= 0 && long_nnz >= 0 && long_nnz <= A.rp.back(), "copy sizes");
    return s;
}

// Column-tile sizes: no more tiled entries than long-row entries, a tile
// count that covers the columns, units only when rows are tiled.
static rgcsr_status tiles_all(const Csr &A, rgcsr_opts o, int32_t min_len) {
    o.tile_min_len = min_len;
    int64_t n_tiles = -1, rows = -1, entries = -1, units = -1, thr = -1;
    g_armed = true;
    const rgcsr_status s = rgcsr_tile_sizes(A.n_rows, A.n_cols, A.rp.back(), A.rp.data(), A.col.data(), &o,
                                            &n_tiles, &rows, &entries, &units, &thr);
    g_armed = false;
    if (s != RGCSR_OK) return s;
    const int64_t cols = o.value_dtype == RGCSR_F64 ? 4096 : 8192;
    CHECK(entries >= 0 && entries <= A.rp.back(), "tile entries %lld", (long long)entries);
    CHECK(rows == 0 ? (n_tiles == 0 && units == 0 && entries == 0)
                    : (n_tiles == (A.n_cols + cols - 1) / cols && units > 0 && thr >= 1),
          "tile sizes: %lld rows, %lld tiles, %lld units", (long long)rows, (long long)n_tiles, (long long)units);
    return s;
}

int main() {
    std::mt19937_64 rng(20101012);
    const int shapes[][5] = {{0, 0, 0, 0, 0},     {1, 1, 1, 0, 0},       {7, 5, 4, 0, 0},
                             {300, 200, 12, 2, 150}, {1000, 3000, 40, 3, 2500}, {129, 64, 64, 1, 64}};
    const int dtypes[] = {RGCSR_F64, RGCSR_F32, RGCSR_F16, RGCSR_BF16};
    int cases = 0;
    for (const auto &sh : shapes) {
        Csr A = random_csr(rng, sh[0], sh[1], sh[2], sh[3], sh[4]);
        for (int G : {1, 3, 64, 128})
            for (int T : {1, 2, 8})
                for (int64_t sigma : {(int64_t)1, (int64_t)5, (int64_t)1 << 40})
                    for (int64_t tau : {(int64_t)-1, (int64_t)0, (int64_t)16})
                        for (int dt : dtypes) {
                            rgcsr_opts o;
                            rgcsr_default_opts(&o);
                            o.group_size = G;
                            o.lanes_per_row = T;
                            o.sort_window = sigma;
                            o.long_row_threshold = tau;
                            o.value_dtype = dt;
                            const rgcsr_status s = layout_all(A, o);
                            CHECK(s == RGCSR_OK, "layout status %d: %s", (int)s, rgcsr_last_error());
                            cases++;
                        }
        for (int dt : {RGCSR_F32, RGCSR_F64})
            for (int32_t min_len : {-1, 0, 1, 64})
                for (int64_t tau : {(int64_t)-1, (int64_t)0, (int64_t)16}) {
                    rgcsr_opts o;
                    rgcsr_default_opts(&o);
                    o.sort_window = 5;
                    o.long_row_threshold = tau;
                    o.value_dtype = dt;
                    const rgcsr_status s = tiles_all(A, o, min_len);
                    CHECK(s == RGCSR_OK, "tile sizes status %d: %s", (int)s, rgcsr_last_error());
                    cases++;
                }
        for (int32_t P : {8, 16, 64})
            for (int64_t tau : {(int64_t)-1, (int64_t)0, (int64_t)16}) {
                rgcsr_opts o;
                rgcsr_default_opts(&o);
                o.sort_window = 5;
                o.long_row_threshold = tau;
                const rgcsr_status s = panels_all(A, o, P);
                CHECK(s == RGCSR_OK, "panel sizes status %d: %s", (int)s, rgcsr_last_error());
                cases++;
            }
        int64_t k1 = -1;
        CHECK(hyb_choose_width(A.n_rows, A.rp.data(), RGCSR_F32, &k1) == RGCSR_OK && k1 >= 0, "hyb width");
        if (A.n_rows == A.n_cols) {
            std::vector<int32_t> perm(A.n_rows);
            CHECK(rgcsr_rcm_order(A.n_rows, A.rp.back(), A.rp.data(), A.col.data(), perm.data()) == RGCSR_OK,
                  "rcm: %s", rgcsr_last_error());
            std::vector<char> seen(A.n_rows, 0);
            for (int32_t p : perm) seen[p] = 1;
            for (char c : seen) CHECK(c == 1, "rcm is not a permutation");
        }
    }
    // malformed inputs are refused with RGCSR_ECSR and touch nothing beyond
    // the arrays they describe
    {
        Csr A = random_csr(rng, 50, 40, 6, 0, 0);
        rgcsr_opts o;
        rgcsr_default_opts(&o);
        rgcsr_info_t info;
        Csr B = A;
        B.rp[10] = B.rp[11] + 1;  // decreasing row pointers
        CHECK(rgcsr_layout_sizes(B.n_rows, B.n_cols, B.rp.back(), B.rp.data(), B.col.data(), &o, &info) == RGCSR_ECSR,
              "decreasing row pointers");
        B = A;
        if (!B.col.empty()) B.col[0] = (int32_t)B.n_cols;  // column out of range
        CHECK(rgcsr_layout_sizes(B.n_rows, B.n_cols, B.rp.back(), B.rp.data(), B.col.data(), &o, &info) == RGCSR_ECSR,
              "column out of range");
        B = A;
        for (int64_t r = 0; r < B.n_rows; r++)
            if (B.rp[r + 1] - B.rp[r] >= 2) {
                B.col[B.rp[r] + 1] = B.col[B.rp[r]];  // duplicate column
                break;
            }
        CHECK(rgcsr_layout_sizes(B.n_rows, B.n_cols, B.rp.back(), B.rp.data(), B.col.data(), &o, &info) == RGCSR_ECSR,
              "duplicate column");
        CHECK(rgcsr_layout_sizes(A.n_rows, A.n_cols, A.rp.back() + 1, A.rp.data(), A.col.data(), &o, &info) == RGCSR_ECSR,
              "nnz does not match the last row pointer");
        CHECK(rgcsr_layout_sizes(A.n_rows, A.n_cols, 0, nullptr, nullptr, &o, &info) != RGCSR_OK, "null row pointers");
        o.lanes_per_row = 3;
        CHECK(rgcsr_layout_sizes(A.n_rows, A.n_cols, A.rp.back(), A.rp.data(), A.col.data(), &o, &info) == RGCSR_EINVAL,
              "lanes_per_row 3");
    }
    // allocation failures: the n-th host allocation of a conversion fails,
    // for n = 0, 1, 2, ... until the conversion gets through
    {
        Csr A = random_csr(rng, 2000, 1500, 30, 3, 1200);
        rgcsr_opts o;
        rgcsr_default_opts(&o);
        o.sort_window = 256;
        o.long_row_threshold = 16;
        o.lanes_per_row = 2;
        int enomem = 0;
        for (long n = 0;; n++) {
            g_fail_countdown = n;
            const rgcsr_status s = layout_all(A, o);
            g_fail_countdown = -1;
            if (s == RGCSR_OK) break;
            CHECK(s == RGCSR_ENOMEM, "allocation %ld failing gave status %d: %s", n, (int)s, rgcsr_last_error());
            enomem++;
            if (n > 100000) {
                CHECK(false, "conversion never got through");
                break;
            }
        }
        CHECK(enomem > 10, "only %d allocations were failed", enomem);
        int enomem_panels = 0;
        for (long n = 0;; n++) {
            g_fail_countdown = n;
            const rgcsr_status s = panels_all(A, o, 8);
            g_fail_countdown = -1;
            if (s == RGCSR_OK) break;
            CHECK(s == RGCSR_ENOMEM, "panel sizes: allocation %ld failing gave status %d: %s", n, (int)s,
                  rgcsr_last_error());
            enomem_panels++;
            if (n > 100000) {
                CHECK(false, "panel sizes never got through");
                break;
            }
        }
        CHECK(enomem_panels > 10, "only %d panel allocations were failed", enomem_panels);
        enomem += enomem_panels;
        int enomem_tiles = 0;
        o.value_dtype = RGCSR_F64;
        for (long n = 0;; n++) {
            g_fail_countdown = n;
            const rgcsr_status s = tiles_all(A, o, 64);
            g_fail_countdown = -1;
            if (s == RGCSR_OK) break;
            CHECK(s == RGCSR_ENOMEM, "tile sizes: allocation %ld failing gave status %d: %s", n, (int)s,
                  rgcsr_last_error());
            enomem_tiles++;
            if (n > 100000) {
                CHECK(false, "tile sizes never got through");
                break;
            }
        }
        CHECK(enomem_tiles > 10, "only %d tile allocations were failed", enomem_tiles);
        enomem += enomem_tiles;
        std::printf("allocation failures injected: %d, each returned RGCSR_ENOMEM\n", enomem);
    }
    std::printf("layout cases: %d, failures: %d\n", cases, g_failures);
    return g_failures == 0 ? 0 : 1;
}
