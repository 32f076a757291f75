// Device-side CSR -> RgCSR conversion (convert.hip), used by rgcsr_from_csr
// when the CSR arrays are in device memory.  It produces the same arrays as
// the host converter (host_layout.cpp) bit for bit, for one matrix.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <vector>

#include "internal.h"

namespace rg {

// Device scratch of one conversion; freed by the destructor.
struct DevScratch {
    std::vector<void *> bufs;
    hipStream_t st = nullptr;  // work on it finishes before the buffers are freed
    void *get(size_t bytes);
    ~DevScratch();
};

// Plan: the row order (sort windows, long-row split), group widths and
// offsets, and every size the device handle needs, computed on the device;
// the sizes and the small index arrays the host schedule reads are copied
// back (gp: ng + 1 entries, long_ptr: nl + 1 entries).
struct DevPlan {
    int64_t n_rows = 0, n_cols = 0, nnz = 0;
    int64_t ns = 0, nl = 0, ng = 0, slots = 0, long_nnz = 0;
    bool perm = false;       // grouped rows are not rows 0.. ns-1 in order
    bool no_empty = true;    // no grouped row is empty
    std::vector<int64_t> gp_host, long_ptr_host;
    // device arrays owned by scratch
    const int32_t *sv = nullptr;     // [ns] grouped rows in layout order
    const int32_t *lv = nullptr;     // [nl] long rows in long-list order
    const int32_t *lens_s = nullptr; // [ns] their lengths
    const int64_t *gp = nullptr;     // [ng + 1]
    const int64_t *long_ptr = nullptr;  // [nl + 1]
    DevScratch scratch;
};

// Validates the device CSR when asked (RGCSR_ECSR on malformed input) and
// computes the plan.  Synchronises the stream.
void device_plan(DevPlan &P, const LayoutParams &p, int64_t n_rows, int64_t n_cols, int64_t nnz,
                 const int64_t *rp, const int32_t *col, bool validate, hipStream_t st);

// Writes the layout arrays (device pointers of the handle; short_row only
// when P.perm) from the device CSR, values converted from vals_dt to vdt.
void device_fill(const DevPlan &P, const LayoutParams &p, const int64_t *rp, const int32_t *col, const void *vals,
                 int vals_dt, int vdt, int64_t *gp, int32_t *short_len, int32_t *short_row, void *slot_val,
                 int32_t *slot_col, int32_t *long_row, int64_t *long_ptr, void *long_val, int32_t *long_col,
                 hipStream_t st);

}  // namespace rg
