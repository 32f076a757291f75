// Autotuner: pick the RgCSR layout (group size G, lanes per row T, sort window
// sigma, long-row threshold tau) for one matrix or a batch by a cost-model
// prefilter and then timing the best candidates on the device.  The paper
// sweeps the group size by hand (Table 4, Section 4.3); here the candidates
// come from the row-length statistics and the bytes each layout would move.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <string>
#include <vector>

#include "internal.h"

namespace rg {

namespace {

struct Mat {
    int64_t n_rows;
    const int64_t *rp;
};

struct Cand {
    rgcsr_opts o;
    double est;         // modelled bytes of one SpMV
    bool loads_padding;  // the default schedule would load padding slots
};

// Grouped-row lengths of every matrix in layout order under one (sigma, tau).
struct Ordered {
    std::vector<std::vector<int32_t>> lens;
    int64_t short_nnz = 0, long_nnz = 0, n_long = 0, n_short = 0;
};

Ordered order_all(const std::vector<Mat> &mats, int64_t sigma, int64_t tau) {
    Ordered o;
    o.lens.resize(mats.size());
    const LayoutParams p{64, 1, sigma, tau};
    for (size_t m = 0; m < mats.size(); m++) {
        int64_t nl = 0, lz = 0;
        short_lengths(p, mats[m].n_rows, mats[m].rp, o.lens[m], &nl, &lz);
        o.long_nnz += lz;
        o.n_long += nl;
        o.n_short += (int64_t)o.lens[m].size();
        for (int32_t v : o.lens[m]) o.short_nnz += v;
    }
    return o;
}

// Cost model: value and column bytes (over the group width when the default
// schedule loads padding, which it does when padding is at most the grouped
// nonzeros), the long rows with their pointers, one row length per grouped
// row, one output index per grouped row when rows are reordered, and the
// group pointers.
double est_bytes(const Ordered &o, int32_t G, int32_t T, int s_v, bool reordered, bool *loads_padding) {
    int64_t slots = 0, groups = 0;
    for (const auto &l : o.lens) {
        slots += group_slots(l, G, T);
        groups += ((int64_t)l.size() + G - 1) / G;
    }
    const bool over_width = slots - o.short_nnz <= o.short_nnz;
    if (loads_padding) *loads_padding = over_width && slots > o.short_nnz;
    const int64_t loads = over_width ? slots : o.short_nnz;
    return (double)(loads + o.long_nnz) * (s_v + 4) + (double)o.n_long * 16.0 +
           (double)o.n_short * (reordered ? 8.0 : 4.0) + (double)groups * 8.0;
}

// For every (sigma, tau) the (G, T) with the fewest modelled bytes.  Order:
// the paper layout (64, 1, 1, no split), the cheapest layout of each sort
// window, then the rest by modelled bytes; each is tried with the default
// schedule and, when that schedule would load padding, also with loads that
// stop at the row length, until max_cands are taken.
std::vector<Cand> candidates(const std::vector<Mat> &mats, const rgcsr_opts &base, int32_t max_cands,
                             bool batch) {
    int64_t max_len = 0, max_rows = 1;
    for (const Mat &m : mats) {
        max_rows = std::max(max_rows, m.n_rows);
        for (int64_t i = 0; i < m.n_rows; i++) max_len = std::max(max_len, m.rp[i + 1] - m.rp[i]);
    }
    const int s_v = std::max(1, dtype_size(base.value_dtype));
    std::vector<int64_t> sigmas{1};
    for (int64_t s : batch ? std::vector<int64_t>{256, 1024, max_rows}
                           : std::vector<int64_t>{256, 512, 4096, 65536, max_rows})
        if (s > 1 && s <= max_rows && std::find(sigmas.begin(), sigmas.end(), s) == sigmas.end()) sigmas.push_back(s);
    std::vector<int64_t> taus{-1};
    for (int64_t t : batch ? std::vector<int64_t>{64, 256} : std::vector<int64_t>{16, 32, 64, 256, 1024})
        if (t < max_len) taus.push_back(t);
    auto make = [&](int32_t G, int32_t T, int64_t sigma, int64_t tau, double est, bool lp) {
        rgcsr_opts o = base;
        o.group_size = G;
        o.lanes_per_row = T;
        o.sort_window = sigma;
        o.long_row_threshold = tau;
        o.rows_per_lane = 0;
        o.pad_loads = -1;
        if (T != 1) o.load_policy = 0;
        return Cand{o, est, lp};
    };
    std::vector<Cand> layouts;
    Cand paper{};
    for (int64_t sigma : sigmas)
        for (int64_t tau : taus) {
            const Ordered o = order_all(mats, sigma, tau);
            const bool reordered = sigma > 1 || tau >= 0;
            double best = -1.0;
            bool best_lp = false;
            int32_t bG = 64, bT = 1;
            for (int32_t G : {64, 128, 256, 512})
                for (int32_t T : {1, 2, 4, 8}) {
                    bool lp = false;
                    const double e = est_bytes(o, G, T, s_v, reordered, &lp);
                    if (best < 0 || e < best * 0.999) {  // ties keep the smaller G and T
                        best = e;
                        bG = G;
                        bT = T;
                        best_lp = lp;
                    }
                    if (G == 64 && T == 1 && sigma == 1 && tau < 0) paper = make(64, 1, 1, -1, e, lp);
                }
            layouts.push_back(make(bG, bT, sigma, tau, best, best_lp));
        }
    std::stable_sort(layouts.begin(), layouts.end(), [](const Cand &a, const Cand &b) { return a.est < b.est; });
    auto is_paper = [](const Cand &c) {
        return c.o.group_size == 64 && c.o.lanes_per_row == 1 && c.o.sort_window == 1 && c.o.long_row_threshold < 0;
    };
    // the cheapest layout of every sort window first (the cost model cannot
    // see x locality, which small windows keep), then the rest by bytes; the
    // paper layout leads
    std::vector<Cand> firsts, rest;
    for (const Cand &c : layouts) {
        const bool seen = std::any_of(firsts.begin(), firsts.end(),
                                      [&](const Cand &f) { return f.o.sort_window == c.o.sort_window; });
        (seen ? rest : firsts).push_back(c);
    }
    layouts = firsts;
    layouts.insert(layouts.end(), rest.begin(), rest.end());
    if (std::none_of(layouts.begin(), layouts.end(), is_paper)) layouts.insert(layouts.begin(), paper);
    else std::stable_partition(layouts.begin(), layouts.end(), is_paper);
    std::vector<Cand> out;
    for (const Cand &c : layouts) {
        if ((int32_t)out.size() >= max_cands) break;
        out.push_back(c);
        if (c.loads_padding && (int32_t)out.size() < max_cands) {
            Cand z = c;
            z.o.pad_loads = 0;
            out.push_back(z);
        }
    }
    return out;
}

// Build every candidate, time `reps` launches of y = A x after one warm-up,
// keep the fastest.
void tune(const std::vector<Cand> &list, const std::function<rgcsr_status(const rgcsr_opts &, rgcsr_handle *)> &build,
          const void *x, void *y, rgcsr_dtype vec_dtype, int32_t reps, rgcsr_opts *cands, double *times_us,
          int32_t *n_tried, rgcsr_opts *best, int32_t validate, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) fail(RGCSR_EHIP, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        fail(RGCSR_EHIP, "hipEventCreate failed");
    }
    double best_t = -1.0;
    int32_t tried = 0;
    rgcsr_status err = RGCSR_OK;
    for (const Cand &c : list) {
        rgcsr_opts o = c.o;
        o.validate = 0;  // validated once by the caller
        rgcsr_handle h = nullptr;
        rgcsr_status s = build(o, &h);
        if (s != RGCSR_OK) {
            err = s;
            continue;
        }
        double t = -1.0;
        s = rgcsr_spmv(h, x, y, vec_dtype, stream);  // warm-up
        if (s == RGCSR_OK) {
            (void)hipEventRecord(e0, st);
            for (int32_t r = 0; r < reps && s == RGCSR_OK; r++) s = rgcsr_spmv(h, x, y, vec_dtype, stream);
            (void)hipEventRecord(e1, st);
            float ms = 0.f;
            if (s == RGCSR_OK && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
                t = 1e3 * ms / reps;
        }
        rgcsr_destroy(h);
        if (s != RGCSR_OK || t < 0) {
            err = s != RGCSR_OK ? s : RGCSR_EHIP;
            continue;
        }
        if (cands) cands[tried] = c.o;
        if (times_us) times_us[tried] = t;
        tried++;
        if (best_t < 0 || t < best_t) {
            best_t = t;
            *best = c.o;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_tried) *n_tried = tried;
    if (tried == 0) fail(err == RGCSR_OK ? RGCSR_EUNSUPPORTED : err, "no candidate layout could be timed");
    best->validate = validate;
}

template <class F> rgcsr_status guarded(F f) {
    try {
        f();
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.st;
    } catch (const std::bad_alloc &) {
        set_last_error_static("host allocation failed");
        return RGCSR_ENOMEM;
    } catch (...) {
        set_last_error_static("unexpected internal error");
        return RGCSR_EINVAL;
    }
    return RGCSR_OK;
}

}  // namespace

}  // namespace rg

using namespace rg;

extern "C" rgcsr_status rgcsr_autotune(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                                       const int32_t *col_idx, const void *vals, rgcsr_dtype vals_dtype,
                                       const rgcsr_opts *base, const void *x, void *y, rgcsr_dtype vec_dtype,
                                       int32_t max_candidates, int32_t reps, rgcsr_opts *cands, double *times_us,
                                       int32_t *n_tried, rgcsr_opts *best, void *stream) {
    return guarded([&] {
        if (!row_ptr || !best || !x || !y || max_candidates < 1 || reps < 1) fail(RGCSR_EINVAL, "bad argument");
        rgcsr_opts b;
        if (base) b = *base;
        else rgcsr_default_opts(&b);
        if (b.validate) validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
        const std::vector<Cand> list = candidates({Mat{n_rows, row_ptr}}, b, max_candidates, false);
        tune(
            list,
            [&](const rgcsr_opts &o, rgcsr_handle *h) {
                return rgcsr_from_csr(n_rows, n_cols, nnz, row_ptr, col_idx, vals, vals_dtype, &o, 0, stream, h);
            },
            x, y, vec_dtype, reps, cands, times_us, n_tried, best, b.validate, stream);
    });
}

extern "C" rgcsr_status rgcsr_autotune_batch(int32_t count, const int64_t *n_rows, const int64_t *n_cols,
                                             const int64_t *const *row_ptr, const int32_t *const *col_idx,
                                             const void *const *vals, rgcsr_dtype vals_dtype, const rgcsr_opts *base,
                                             const void *x, void *y, rgcsr_dtype vec_dtype, int32_t max_candidates,
                                             int32_t reps, rgcsr_opts *cands, double *times_us, int32_t *n_tried,
                                             rgcsr_opts *best, void *stream) {
    return guarded([&] {
        if (count < 1 || !n_rows || !n_cols || !row_ptr || !col_idx || !best || !x || !y || max_candidates < 1 ||
            reps < 1)
            fail(RGCSR_EINVAL, "bad argument");
        rgcsr_opts b;
        if (base) b = *base;
        else rgcsr_default_opts(&b);
        std::vector<Mat> mats(count);
        for (int32_t m = 0; m < count; m++) {
            if (!row_ptr[m] || n_rows[m] < 0) fail(RGCSR_EINVAL, "bad matrix in batch");
            if (b.validate) validate_csr(n_rows[m], n_cols[m], row_ptr[m][n_rows[m]], row_ptr[m], col_idx[m]);
            mats[m] = Mat{n_rows[m], row_ptr[m]};
        }
        const std::vector<Cand> list = candidates(mats, b, max_candidates, true);
        tune(
            list,
            [&](const rgcsr_opts &o, rgcsr_handle *h) {
                return rgcsr_from_csr_batch(count, n_rows, n_cols, row_ptr, col_idx, vals, vals_dtype, &o, stream, h);
            },
            x, y, vec_dtype, reps, cands, times_us, n_tried, best, b.validate, stream);
    });
}
