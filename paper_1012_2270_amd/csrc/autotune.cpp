// Autotuner: pick the RgCSR layout (group size, sort window, long-row
// threshold) and kernel schedule (rows per lane) for one matrix by timing a
// short list of candidates on the device.  The paper sweeps the group size by
// hand (Table 4, Section 4.3); here the candidates come from the row-length
// statistics and the padding each layout would need.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace rg {

namespace {

struct Cand {
    rgcsr_opts o;
};

int64_t padded_slots(const LayoutParams &p, int64_t n_rows, const int64_t *rp, int64_t *long_nnz) {
    int64_t ng, ns, nl, slots, lz;
    layout_sizes(p, n_rows, rp, &ng, &ns, &nl, &slots, &lz, nullptr);
    *long_nnz = lz;
    return slots;
}

// Candidate list, most promising first.  Long-row thresholds are only tried
// below the longest row; sort windows only when they cut padding noticeably.
std::vector<Cand> candidates(int64_t n_rows, const int64_t *rp, const rgcsr_opts &base, int32_t max_cands) {
    int64_t max_len = 0, nnz = rp[n_rows];
    for (int64_t i = 0; i < n_rows; i++) max_len = std::max(max_len, rp[i + 1] - rp[i]);
    std::vector<Cand> out;
    auto add = [&](int64_t sigma, int64_t tau, int32_t R) {
        rgcsr_opts o = base;
        o.group_size = 64;
        o.lanes_per_row = 1;
        o.sort_window = sigma;
        o.long_row_threshold = tau;
        o.rows_per_lane = R;
        o.pad_loads = -1;
        for (const Cand &c : out)
            if (c.o.sort_window == sigma && c.o.long_row_threshold == tau && c.o.rows_per_lane == R) return;
        out.push_back(Cand{o});
    };
    // the paper's layout with the automatic schedule, and explicit schedules
    add(1, -1, 0);
    const LayoutParams paper{64, 1, 1, -1};
    int64_t lz = 0;
    const int64_t paper_slots = padded_slots(paper, n_rows, rp, &lz);
    const double paper_fill = nnz ? (double)(paper_slots - nnz) / (double)nnz : 0.0;
    if (paper_fill < 0.25) {
        add(1, -1, 1);
        add(1, -1, 2);
        add(1, -1, 4);
    }
    // long-row split and descending order in windows for skewed rows
    for (int64_t tau : {16, 32, 64, 256}) {
        if (tau >= max_len) continue;
        for (int64_t sigma : {int64_t(1), int64_t(512), int64_t(4096), std::max<int64_t>(1, n_rows)}) {
            const LayoutParams p{64, 1, sigma, tau};
            int64_t l2 = 0;
            const int64_t s = padded_slots(p, n_rows, rp, &l2);
            const double fill = (nnz - l2) ? (double)(s - (nnz - l2)) / (double)(nnz - l2) : 0.0;
            if (sigma > 1 && fill > 0.9 * paper_fill && paper_fill > 0) continue;  // sorting buys nothing
            add(sigma, tau, 0);
            add(sigma, tau, 2);
        }
    }
    if ((int32_t)out.size() > max_cands) out.resize(max_cands);
    return out;
}

}  // namespace

}  // namespace rg

using namespace rg;

extern "C" rgcsr_status rgcsr_autotune(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                                       const int32_t *col_idx, const void *vals, rgcsr_dtype vals_dtype,
                                       const rgcsr_opts *base, const void *x, void *y, rgcsr_dtype vec_dtype,
                                       int32_t max_candidates, int32_t reps, rgcsr_opts *cands, double *times_us,
                                       int32_t *n_tried, rgcsr_opts *best, void *stream) {
    try {
        if (!row_ptr || !best || !x || !y || max_candidates < 1 || reps < 1) fail(RGCSR_EINVAL, "bad argument");
        rgcsr_opts b;
        if (base) b = *base;
        else rgcsr_default_opts(&b);
        if (b.validate) validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
        hipStream_t st = (hipStream_t)stream;
        const std::vector<Cand> list = candidates(n_rows, row_ptr, b, max_candidates);
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            fail(RGCSR_EHIP, "hipEventCreate failed");
        double best_t = -1.0;
        int32_t tried = 0;
        rgcsr_status err = RGCSR_OK;
        for (const Cand &c : list) {
            rgcsr_opts o = c.o;
            o.validate = 0;  // validated once above
            rgcsr_handle h = nullptr;
            rgcsr_status s = rgcsr_from_csr(n_rows, n_cols, nnz, row_ptr, col_idx, vals, vals_dtype, &o, 0, stream, &h);
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
                if (s == RGCSR_OK && hipEventSynchronize(e1) == hipSuccess &&
                    hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
                    t = 1e3 * ms / reps;
            }
            rgcsr_destroy(h);
            if (s != RGCSR_OK) {
                err = s;
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
        best->validate = b.validate;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.st;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return RGCSR_ENOMEM;
    } catch (...) {
        set_last_error("unexpected internal error");
        return RGCSR_EINVAL;
    }
    return RGCSR_OK;
}
