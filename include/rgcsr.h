/*
 * rgcsr.h -- C ABI of librgcsr.so: sparse matrix-vector multiplication in the
 * Row-grouped CSR (RgCSR) format on AMD Instinct MI355X (gfx950).
 *
 * Method: Oberhuber, Suzuki, Vacata, "New Row-grouped CSR format for storing
 * the sparse matrices on GPU with implementation in CUDA".
 *   Section 3.1  CSR input format (row pointers, ascending columns per row).
 *   Section 3.4  RgCSR: rows split into groups; inside a group the first
 *                nonzero of every row is stored, then the second, ...; rows
 *                shorter than the group's longest are padded with artificial
 *                zeros carrying a ghost column; groupPointers + rowLength
 *                replace rowPointers; one thread per row walks its row with
 *                the group size as stride and stops after rowLength steps.
 *   Section 3.3  Hybrid ELLPACK + COO, the paper's comparison format.
 *   Section 3.4  Peak model: 2 flops per nonzero; bytes per nonzero are the
 *                column index, the value and (uncached) the x entry.
 *
 * Conventions for every call:
 *   - Status codes only; nothing aborts and no C++ exception crosses the ABI.
 *     rgcsr_last_error() returns a thread-local message for the last failure.
 *   - "device pointer": memory from hipMalloc (or a torch CUDA tensor) on the
 *     current HIP device.  "host pointer": ordinary CPU memory.
 *   - stream: a hipStream_t passed as void*; NULL is the null stream.  Device
 *     work is enqueued on it and calls return without a device-wide sync,
 *     unless a call says otherwise.  Asynchronous kernel faults surface as
 *     RGCSR_EHIP from a later call that synchronises.
 *   - Index types: row pointers and group pointers are int64; column indices
 *     and row lengths are int32 (as in the paper).
 *   - Values are converted to the handle's storage dtype with round to
 *     nearest even; float64 input bound for float16/bfloat16 storage is first
 *     rounded to float32, then to the 16-bit type.
 *   - Supported (stored value, vector, accumulator) triples for SpMV:
 *     (F64,F64,F64) (F32,F32,F32) (F16,F32,F32) (BF16,F32,F32) (F32,F64,F64);
 *     the vector dtype argument selects the vector/accumulator type.
 */
#ifndef RGCSR_H
#define RGCSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RGCSR_OK = 0,
    RGCSR_EINVAL = 1,      /* bad argument (null pointer, unsupported size)   */
    RGCSR_ECSR = 2,        /* malformed CSR input                             */
    RGCSR_ENOMEM = 3,      /* host or device allocation failed                */
    RGCSR_EOVERFLOW = 4,   /* a size does not fit the index types             */
    RGCSR_EHIP = 5,        /* HIP runtime error                               */
    RGCSR_EUNSUPPORTED = 6 /* valid request that this library does not handle */
} rgcsr_status;

typedef enum { RGCSR_F64 = 0, RGCSR_F32 = 1, RGCSR_F16 = 2, RGCSR_BF16 = 3 } rgcsr_dtype;

/* Layout parameters (Section 3.4 and the project's readings of it).
 *   group_size   G: rows per group, >= 1 (0 selects 64).  Device kernels
 *                need G * lanes_per_row to be a multiple of 64 or a divisor of 64.
 *   lanes_per_row T in {1, 2, 4, 8} (0 selects 1).  T = 1 is the paper's
 *                layout.  With T > 1 each row's width is rounded up to a
 *                multiple of T and nonzero j of local row t of group g sits at
 *                gp[g] + (j / T) * (s_g * T) + t * T + j % T.
 *   sort_window  sigma >= 1 (0 selects 1): inside each window of sigma rows
 *                rows are ordered longest first, ties in original order (the
 *                descending ordering of Section 4.4.2); 1 keeps paper order.
 *   long_row_threshold tau: rows with more than tau nonzeros are stored
 *                CSR-contiguous in a long-row segment (sorted longest first,
 *                ties by original row) and multiplied by whole wavefronts;
 *                negative = no split (paper).
 *   value_dtype  storage dtype of values (rgcsr_dtype).
 *   keep_csr_map keep the CSR row pointers on the device; required by
 *                rgcsr_set_values and by the dvals output of the gradient.
 *   build_transpose also build A^T (structure + value map) so the gradient
 *                computes dx = A^T dy without atomics.
 *   validate     1 (default) checks the CSR input; 0 trusts it (undefined
 *                behaviour on malformed input).
 */
typedef struct {
    int32_t group_size;
    int32_t lanes_per_row;
    int64_t sort_window;
    int64_t long_row_threshold;
    int32_t value_dtype;
    int32_t keep_csr_map;
    int32_t build_transpose;
    int32_t validate;
    int32_t rows_per_lane;  /* kernel schedule: rows each lane multiplies per pass over
                               its groups, 1, 2, 4 or 8; 0 = chosen per wavefront, the
                               largest count whose widest group times the count is at
                               most 16 (several narrow groups share a wavefront, wide
                               ones run alone); only with lanes_per_row = 1, otherwise 1 */
    int32_t pad_loads;      /* kernel schedule: 0 = loads stop at the row length;
                               1 = value/column loads run over the group width so they
                               need not wait for the row length (padding is still never
                               multiplied); 3 = as 1, but the row lengths are not read:
                               columns ascend strictly within a row and padding repeats
                               the row's last column, so a step is multiplied exactly
                               when its column exceeds the previous one (needs
                               lanes_per_row = 1, group_size a multiple of 64 and no
                               empty grouped row; same bits as 0 and 1); 2 = sliced
                               ELLPACK (Section 3.3): row lengths are not read and every
                               slot of the group width is multiplied, padding included
                               (same values for finite x; needs group_size *
                               lanes_per_row a multiple of 64); -1 = when padding is at
                               most 100% of the grouped nonzeros 3 if allowed, else 1,
                               otherwise 0 */
    int32_t load_policy;    /* where loads may be cached, after the paper's texture-cache
                               study (Section 4.3): 0 (default) = value/column streams
                               nontemporal, x gathers cached; 1 = every load cached;
                               2 = x gathers nontemporal too.  1 and 2 need F32 values,
                               lanes_per_row = 1 and F32 vectors, and apply to single
                               right-hand-side launches */
    int32_t tile_min_len;   /* kernel schedule: long rows of at least this many nonzeros
                               (and at least half as many as there are column tiles)
                               are also stored split by column tile of 8,192 columns
                               (4,096 for F64 storage); a launch with one vector of
                               unit stride (F64 for F64 storage, F32 otherwise) and
                               load policy 0 first runs one
                               workgroup per (tile, run of those rows) that stages the
                               tile of x in LDS and writes one partial sum per (row,
                               tile), then the SpMV kernel adds each row's partials in
                               tile order (x is kept in LDS instead of the caches, after
                               the texture-cache study of Section 4.3).  Rows with more
                               than 4,096 nonzeros in one tile (2,048 for F64 storage)
                               stay on the long-row path.  0 = off; -1 (default) = 256, used only when the
                               tiled rows hold at least 262,144 nonzeros.  F32 storage
                               with F64 vectors runs the tiled rows on the long-row
                               path. */
    int32_t col_panels;     /* 0 (default) = off.  P = 8, 16, ..., 64: the handle also
                               keeps a copy of the matrix for launches of several
                               right-hand sides.  The columns are split into P panels
                               of about equal nonzero count; a row longer than
                               long_row_threshold (every row when that is negative) is
                               split into pieces, its entries in one panel's columns,
                               and the other rows stay whole.  The pieces of each panel
                               and then the whole rows are laid out as above, with
                               each element's CSR index so rgcsr_set_values refreshes
                               the copy.  A launch of 2 or more right-hand sides whose
                               X rows (ldx elements) give at most 3 MiB of X per panel
                               and whose column block has at most 32 bytes of
                               accumulators per row (K <= 8 with F32 vectors, K <= 4
                               with F64) runs on the copy: panel q's workgroups run on
                               XCD (q * 8 / P) of the eight, so each XCD's L2 keeps
                               that panel's slice of X (the x reuse through a cache
                               that Section 4.3 studies); whole rows, dealt to every
                               XCD, write their rows of Y, pieces write one sum each
                               to a device buffer of the handle, and a second kernel
                               adds each split row's piece sums in panel order
                               (deterministic).  One vector, and other launches, use
                               the layout itself.  The copy doubles the stored matrix
                               and adds 32 bytes per piece.  Host conversion only
                               (device inputs are copied to the host);
                               rgcsr_plan_from_csr and batches return
                               RGCSR_EUNSUPPORTED. */
} rgcsr_opts;

/* Fills *opts with the paper's layout: G = 64, T = 1, sigma = 1, no long
 * rows, float32 storage, no CSR map, no transpose, validation on, automatic
 * kernel schedule (rows_per_lane = 0, pad_loads = -1, load_policy = 0,
 * tile_min_len = -1), no column panels. */
void rgcsr_default_opts(rgcsr_opts *opts);

typedef struct rgcsr_matrix_s *rgcsr_handle;

/* Sizes of a layout, in elements.  n_groups = groups of short rows,
 * n_short / n_long = rows in the grouped / long-row parts, slots = grouped
 * slots including artificial zeros (gp[n_groups]), long_nnz = nonzeros in the
 * long-row segment, nnz = real nonzeros, n_rows / n_cols totals (a batch is a
 * block-diagonal concatenation), n_matrices = 1 unless built as a batch,
 * long_work = wavefront work items of the long-row path, partials = chunk
 * partial sums of long rows split over several wavefronts. */
typedef struct {
    int64_t n_rows, n_cols, nnz;
    int64_t n_groups, n_short, n_long, slots, long_nnz;
    int64_t n_matrices, long_work, partials;
    int32_t group_size, lanes_per_row, value_dtype, has_transpose;
    int64_t sort_window, long_row_threshold;
    int64_t device_bytes; /* device memory the handle owns */
    int32_t rows_per_lane, pad_loads, load_policy; /* kernel schedule in use */
    int64_t tiled_rows, tile_entries, n_tiles;     /* column-tiled long rows (tile_min_len) */
    int64_t col_panels, panel_pieces;              /* column panels and their pieces (col_panels) */
} rgcsr_info_t;

/* ---- Host-only layout (no GPU needed; used to check the layout on CPU) ---- */

/* Computes the sizes of the layout of a host CSR matrix (row_ptr[n_rows+1],
 * col_idx[nnz], host pointers) under *opts.  Only out->n_groups, n_short,
 * n_long, slots, long_nnz, nnz, n_rows, n_cols, long_work and partials are
 * set.  Returns RGCSR_ECSR for malformed CSR when opts->validate != 0. */
rgcsr_status rgcsr_layout_sizes(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                const int64_t *row_ptr, const int32_t *col_idx,
                                const rgcsr_opts *opts, rgcsr_info_t *out);

/* Writes every layout array of a host CSR matrix into caller-owned host
 * buffers sized from rgcsr_layout_sizes:
 *   gp[n_groups+1] (int64), short_len[n_short], short_row[n_short] (original
 *   row of each grouped row), slot_val[slots] (storage dtype), slot_col[slots],
 *   long_row[n_long], long_ptr[n_long+1] (int64), long_val[long_nnz],
 *   long_col[long_nnz].
 * Artificial zeros have all-zero value bits and the row's last column (0 for
 * an empty row) as ghost index.  vals has dtype vals_dtype. */
rgcsr_status rgcsr_layout_host(int64_t n_rows, int64_t n_cols, int64_t nnz,
                               const int64_t *row_ptr, const int32_t *col_idx,
                               const void *vals, rgcsr_dtype vals_dtype,
                               const rgcsr_opts *opts, int64_t *gp, int32_t *short_len,
                               int32_t *short_row, void *slot_val, int32_t *slot_col,
                               int32_t *long_row, int64_t *long_ptr, void *long_val,
                               int32_t *long_col);

/* Sizes of the column-tiled copy (rgcsr_opts.tile_min_len) of a host CSR
 * matrix under *opts, without a GPU: the rows that a handle built with the
 * same options stores split by column tile as well.  *n_tiles receives the
 * tiles (n_cols / 8,192 rounded up, or / 4,096 for F64 value_dtype; 0 when no
 * row is tiled), *tiled_rows and *tile_entries the rows and nonzeros tiled,
 * *units the workgroups of the tile kernel (empty ones that even out the XCD
 * queues included) and *min_len the row length threshold applied (any output
 * may be NULL).  Values are not needed.  RGCSR_EINVAL when opts is NULL;
 * RGCSR_ECSR for malformed CSR when opts->validate != 0. */
rgcsr_status rgcsr_tile_sizes(int64_t n_rows, int64_t n_cols, int64_t nnz,
                              const int64_t *row_ptr, const int32_t *col_idx,
                              const rgcsr_opts *opts, int64_t *n_tiles, int64_t *tiled_rows,
                              int64_t *tile_entries, int64_t *units, int64_t *min_len);

/* Sizes of the column-panel copy (rgcsr_opts.col_panels) of a host CSR
 * matrix under *opts, without a GPU: col_bounds[col_panels + 1] receives the
 * panel column bounds (panel q holds columns [col_bounds[q],
 * col_bounds[q + 1]); NULL skips it), *pieces the rows of the copy (one per
 * whole row, empty rows included, and one per split row and panel holding
 * some of its entries), *split_rows the rows longer than long_row_threshold
 * (split), *split_pieces their pieces, *slots and *long_nnz the grouped slots
 * and long-row nonzeros of the copy's layout (any output may be NULL).
 * RGCSR_EINVAL when opts is NULL or col_panels is not a multiple of 8 from 8
 * to 64; RGCSR_ECSR for malformed CSR when opts->validate != 0. */
rgcsr_status rgcsr_panel_sizes(int64_t n_rows, int64_t n_cols, int64_t nnz,
                               const int64_t *row_ptr, const int32_t *col_idx,
                               const rgcsr_opts *opts, int64_t *col_bounds, int64_t *pieces,
                               int64_t *split_rows, int64_t *split_pieces, int64_t *slots,
                               int64_t *long_nnz);

/* ---- Device handles ------------------------------------------------------ */

/* rgcsr_from_csr: convert a CSR matrix (Section 3.1) to RgCSR on the current
 * device.  inputs_on_device = 0: row_ptr/col_idx/vals are host pointers,
 * borrowed for the duration of the call, converted by the host library.
 * inputs_on_device = 1: they are device pointers, borrowed until the call
 * returns, and the conversion runs on the device (validation, window sort,
 * long-row split, group widths and offsets, scatter and value conversion),
 * giving the same arrays bit for bit; device inputs are always validated
 * (opts->validate is ignored), and with build_transpose they are copied to the
 * host and converted there.  The device path allocates temporary device
 * memory (freed before return).  The handle owns the device arrays it
 * allocates (hipMalloc); the call synchronises the stream before returning,
 * so the handle is ready. */
rgcsr_status rgcsr_from_csr(int64_t n_rows, int64_t n_cols, int64_t nnz,
                            const int64_t *row_ptr, const int32_t *col_idx,
                            const void *vals, rgcsr_dtype vals_dtype,
                            const rgcsr_opts *opts, int inputs_on_device, void *stream,
                            rgcsr_handle *out);

/* Caller-owned device memory (for callers whose allocator, e.g. PyTorch's,
 * owns every device buffer), in two steps over host CSR arrays:
 *
 * rgcsr_plan_from_csr: validates (per opts->validate) and converts the host
 * CSR input on the host, exactly as rgcsr_from_csr does, and keeps the
 * layout in a host-side plan.  Arguments as rgcsr_from_csr with
 * inputs_on_device = 0; needs no GPU.  rgcsr_plan_from_csr_batch: the same
 * for a block-diagonal batch (arguments as rgcsr_from_csr_batch, without
 * the stream); its handle answers rgcsr_batch_offsets.
 * rgcsr_plan_device_bytes: bytes of device memory the handle needs (its
 * arrays and, with build_transpose, those of A^T), one contiguous block.
 * rgcsr_build: places the handle's arrays in [device_buf, device_buf +
 * buf_bytes) -- a device pointer, 256-byte aligned, at least the plan's
 * device bytes, else RGCSR_EINVAL before any device work -- uploads the
 * layout on `stream` and synchronises it.  The handle borrows the buffer:
 * it must stay allocated and untouched while the handle is in use and until
 * the work queued on it has run; rgcsr_destroy neither frees it nor waits
 * for that work.  device_buf = NULL: the handle allocates and owns the block as
 * rgcsr_from_csr does.  A plan builds one handle: once a build has passed its
 * argument checks (whether it then succeeds or not), rgcsr_build and
 * rgcsr_plan_device_bytes on that plan return RGCSR_EINVAL; argument errors
 * leave the plan usable.  rgcsr_clone of a borrowing handle returns a handle
 * that owns its memory.
 * rgcsr_plan_destroy: frees the plan (host memory only); NULL is allowed. */
typedef struct rgcsr_plan_s *rgcsr_plan;
rgcsr_status rgcsr_plan_from_csr(int64_t n_rows, int64_t n_cols, int64_t nnz,
                                 const int64_t *row_ptr, const int32_t *col_idx,
                                 const void *vals, rgcsr_dtype vals_dtype,
                                 const rgcsr_opts *opts, rgcsr_plan *out);
rgcsr_status rgcsr_plan_from_csr_batch(int32_t count, const int64_t *n_rows, const int64_t *n_cols,
                                       const int64_t *const *row_ptr, const int32_t *const *col_idx,
                                       const void *const *vals, rgcsr_dtype vals_dtype,
                                       const rgcsr_opts *opts, rgcsr_plan *out);
rgcsr_status rgcsr_plan_device_bytes(rgcsr_plan plan, int64_t *bytes);
rgcsr_status rgcsr_build(rgcsr_plan plan, void *device_buf, int64_t buf_bytes, void *stream,
                         rgcsr_handle *out);
rgcsr_status rgcsr_plan_destroy(rgcsr_plan plan);

/* rgcsr_from_csr_batch: build one handle holding `count` independent host CSR
 * matrices as a block-diagonal matrix: matrix m's rows follow matrix m-1's,
 * and so do its columns, so x and y of the batch are the per-matrix vectors
 * concatenated.  Groups never straddle two matrices.  All matrices use the
 * same *opts.  row_ptr[m], col_idx[m], vals[m] are host pointers. */
rgcsr_status rgcsr_from_csr_batch(int32_t count, const int64_t *n_rows, const int64_t *n_cols,
                                  const int64_t *const *row_ptr, const int32_t *const *col_idx,
                                  const void *const *vals, rgcsr_dtype vals_dtype,
                                  const rgcsr_opts *opts, void *stream, rgcsr_handle *out);

/* Row/column offsets of each matrix of a batch handle, host arrays of
 * n_matrices+1 int64 entries each (last = totals). */
rgcsr_status rgcsr_batch_offsets(rgcsr_handle A, int64_t *row_off, int64_t *col_off);

/* rgcsr_spmv: y = A x (Section 3.4 kernel semantics: every row is
 * overwritten, empty rows give 0).  x[n_cols], y[n_rows] are device pointers
 * of vec_dtype (F32 or F64); x and y must not overlap.  One kernel launch,
 * plus a second small one that adds chunk partial sums in a fixed order when
 * some row has more than 16,384 nonzeros (deterministic results). */
rgcsr_status rgcsr_spmv(rgcsr_handle A, const void *x, void *y, rgcsr_dtype vec_dtype,
                        void *stream);

/* rgcsr_spmv_batched: Y = A X for k right-hand sides.  X is n_cols x k
 * row-major with leading dimension ldx >= k, Y is n_rows x k with ldy >= k
 * (device pointers, elements of vec_dtype).  For a batch handle this is
 * Y_m = A_m X_m for every matrix m.  k in {1, 2, 4, 8, 16, 32} runs as one
 * launch when X and Y are 16-byte aligned with ldx, ldy multiples of 4 (F32)
 * or 2 (F64); other k, or unaligned blocks, run as several launches over
 * column blocks (narrower blocks read X and Y rows with scalar accesses).
 * Handles with lanes_per_row > 1 or F16/BF16 stored values run one
 * single-column launch per column.  persistent = 1 launches a fixed grid of
 * wavefronts that loop over the work items (one resident launch); 0 launches
 * one wavefront per item. */
rgcsr_status rgcsr_spmv_batched(rgcsr_handle A, int32_t k, const void *X, int64_t ldx,
                                void *Y, int64_t ldy, rgcsr_dtype vec_dtype,
                                int32_t persistent, void *stream);

/* rgcsr_spmv_transpose_grad: backward of y = A(theta) x.  Given dy[n_rows]:
 *   dx = A^T dy                        (if dx != NULL; dx[n_cols])
 *   dvals[k] = dy[row(k)] * x[col(k)]  (if dvals != NULL; nnz entries in the
 *                                       CSR order of the input matrix)
 * All device pointers of vec_dtype (F32 or F64).  dx uses the transposed
 * RgCSR when the handle was built with build_transpose (deterministic), else
 * an atomic scatter (order of additions not deterministic).  dvals needs
 * keep_csr_map or build_transpose. */
rgcsr_status rgcsr_spmv_transpose_grad(rgcsr_handle A, const void *x, const void *dy,
                                       void *dx, void *dvals, rgcsr_dtype vec_dtype,
                                       void *stream);

/* rgcsr_set_values: overwrite the stored values (and those of A^T, when
 * built) from nnz values in the CSR order of the input matrix, converting to
 * the storage dtype on the device.  vals is a device pointer when on_device
 * = 1, else a host pointer (copied synchronously).  Needs keep_csr_map or
 * build_transpose. */
rgcsr_status rgcsr_set_values(rgcsr_handle A, const void *vals, rgcsr_dtype vals_dtype,
                              int on_device, void *stream);

/* rgcsr_export: copy the device layout arrays into host buffers laid out as
 * for rgcsr_layout_host (any pointer may be NULL to skip that array).
 * Synchronises the stream.  For checking the converter bit for bit. */
rgcsr_status rgcsr_export(rgcsr_handle A, void *stream, int64_t *gp, int32_t *short_len,
                          int32_t *short_row, void *slot_val, int32_t *slot_col,
                          int32_t *long_row, int64_t *long_ptr, void *long_val,
                          int32_t *long_col);

/* rgcsr_to_csr: decode the device layout back to CSR in host buffers
 * (row_ptr[n_rows+1], col_idx[nnz], vals[nnz] in the storage dtype).
 * Values keep their bits.  Synchronises the stream. */
rgcsr_status rgcsr_to_csr(rgcsr_handle A, void *stream, int64_t *row_ptr, int32_t *col_idx,
                          void *vals);

rgcsr_status rgcsr_info(rgcsr_handle A, rgcsr_info_t *out);

/* rgcsr_clone: a new handle with its own device copy of every array of A
 * (device-to-device copies on the stream, synchronised before return).  Used
 * to rotate several copies of one matrix through the caches when timing. */
rgcsr_status rgcsr_clone(rgcsr_handle A, void *stream, rgcsr_handle *out);

/* A handle that owns device memory (every handle except one that
 * rgcsr_build placed in caller memory): synchronises the device, then frees
 * the handle and its device memory.  A handle in caller memory: frees the
 * host struct only and makes no device call, so it stalls no stream; the
 * block stays allocated, and its owner releases it once the work already
 * queued on the handle has run (in stream order, or after synchronising
 * the streams that used it).  NULL is accepted. */
rgcsr_status rgcsr_destroy(rgcsr_handle A);

/* rgcsr_autotune: choose the layout for one host CSR matrix by a cost-model
 * prefilter and device timing (the paper sweeps the group size by hand,
 * Table 4).  For every sort window sigma in {1, 256, 512, 4096, 65536, n} and
 * long-row threshold tau in {none, 16, 32, 64, 256, 1024} (below the longest
 * row), the (G, T) in {64, 128, 256, 512} x {1, 2, 4, 8} with the fewest
 * modelled bytes is kept: value and column loads (over the group width when
 * the default schedule loads padding), long rows, row lengths, output
 * indices and group pointers.  In the order paper layout (64, 1, 1, none),
 * cheapest layout of each sort window, remaining layouts by modelled bytes,
 * each layout is built with the automatic kernel schedule and, when that
 * schedule would load padding, also with loads that stop at the row length,
 * until max_candidates are taken; each is timed over `reps` launches of
 * y = A x (x: device,
 * n_cols entries of vec_dtype; y: device scratch of n_rows).  Other fields
 * of *base (value dtype, CSR map, transpose, validation, load policy) are
 * kept.  Writes the fastest options to *best; when cands/times_us are not
 * NULL they receive every candidate timed (max_candidates entries of room)
 * and its mean launch time in microseconds, *n_tried their count.
 * Synchronises the stream. */
rgcsr_status rgcsr_autotune(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                            const int32_t *col_idx, const void *vals, rgcsr_dtype vals_dtype,
                            const rgcsr_opts *base, const void *x, void *y, rgcsr_dtype vec_dtype,
                            int32_t max_candidates, int32_t reps, rgcsr_opts *cands, double *times_us,
                            int32_t *n_tried, rgcsr_opts *best, void *stream);

/* rgcsr_autotune_batch: the same search for a batch (the inputs of
 * rgcsr_from_csr_batch): sort windows {1, 256, 1024, whole matrix},
 * thresholds {none, 64, 256}, the cost model summed over the matrices; each
 * candidate is built
 * as one batch handle and timed on launches over all matrices (x, y: the
 * concatenated per-matrix vectors, device). */
rgcsr_status rgcsr_autotune_batch(int32_t count, const int64_t *n_rows, const int64_t *n_cols,
                                  const int64_t *const *row_ptr, const int32_t *const *col_idx,
                                  const void *const *vals, rgcsr_dtype vals_dtype, const rgcsr_opts *base,
                                  const void *x, void *y, rgcsr_dtype vec_dtype, int32_t max_candidates,
                                  int32_t reps, rgcsr_opts *cands, double *times_us, int32_t *n_tried,
                                  rgcsr_opts *best, void *stream);

/* ---- Hybrid ELL + COO (Section 3.3) --------------------------------------- */

typedef struct hyb_matrix_s *hyb_handle;

typedef struct {
    int64_t n_rows, n_cols, nnz, n_pad, ell_width, coo_nnz, device_bytes;
    int32_t value_dtype;
} hyb_info_t;

/* ELL width K1 chosen by the project rule: K1 minimises
 *   k * n_pad * (s_v + 4) + 3 * (s_v + 8) * sum_i max(0, len_i - k)
 * over k in [0, max len] (ties: smallest k), n_pad = n_rows rounded up to 64,
 * s_v = bytes of the storage dtype.  ell_width >= 0 forces K1 instead.
 * ELL is column-major n_pad x K1 (padding column -1, value bits 0); COO keeps
 * the remaining nonzeros in (row, column) order.  Host CSR inputs; the call
 * synchronises the stream before returning. */
rgcsr_status hyb_from_csr(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                          const int32_t *col_idx, const void *vals, rgcsr_dtype vals_dtype,
                          rgcsr_dtype value_dtype, int64_t ell_width, int validate,
                          void *stream, hyb_handle *out);

/* Host-only: the K1 the rule picks for this row-pointer array. */
rgcsr_status hyb_choose_width(int64_t n_rows, const int64_t *row_ptr, rgcsr_dtype value_dtype,
                              int64_t *k1);

/* y = A x: an ELL kernel writes every row, then a COO kernel adds the
 * remaining entries (two launches on the stream).  The COO step adds
 * partial sums of rows that cross wavefront boundaries with atomics. */
rgcsr_status hyb_spmv(hyb_handle A, const void *x, void *y, rgcsr_dtype vec_dtype, void *stream);

/* Copies the device ELL/COO arrays to host buffers (ell_col/ell_val of
 * n_pad * K1, coo_* of coo_nnz); any pointer may be NULL. */
rgcsr_status hyb_export(hyb_handle A, void *stream, int32_t *ell_col, void *ell_val,
                        int32_t *coo_row, int32_t *coo_col, void *coo_val);

rgcsr_status hyb_info(hyb_handle A, hyb_info_t *out);

/* Device copy of a Hybrid handle (same conventions as rgcsr_clone). */
rgcsr_status hyb_clone(hyb_handle A, void *stream, hyb_handle *out);
/* Synchronises the device, then frees the handle and the device block it
 * owns (every Hybrid handle owns one).  NULL is accepted. */
rgcsr_status hyb_destroy(hyb_handle A);

/* ---- Mixed-precision conjugate gradients (Krylov consumer, Section 1) ----- */

typedef struct {
    int32_t outer_iterations;   /* FP64 refinement steps taken              */
    int32_t inner_iterations;   /* total inner CG iterations (all steps)    */
    double relres;              /* final ||b - A_hi x||_2 / ||b||_2 in FP64 */
    double seconds;             /* host wall time of the solve              */
    int32_t converged;
} rgcsr_cg_stats;

/* Solves A x = b (A symmetric positive definite) by iterative refinement:
 * the outer loop forms r = b - A_hi x with FP64 vectors and accumulation
 * (A_hi values F32 or F64) and stops when ||r|| / ||b|| <= tol; each inner
 * step runs FP32 CG on A_lo (values F32, F16 or BF16; FP32 vectors and
 * accumulation; dot products accumulated in FP64) on the scaled residual
 * until its relative residual drops below inner_tol or max_inner iterations,
 * then adds the correction to x in FP64.  A_lo and A_hi must have the same
 * square shape; pass the same handle for a pure single-matrix refinement
 * when A_lo stores F32.  b and x are device float64 arrays of n; x holds the
 * initial guess and receives the solution.  Allocates its own device
 * workspace (freed before return) and synchronises the stream. */
rgcsr_status rgcsr_cg_solve(rgcsr_handle A_lo, rgcsr_handle A_hi, const double *b, double *x,
                            double tol, double inner_tol, int32_t max_outer, int32_t max_inner,
                            void *stream, rgcsr_cg_stats *stats);

/* rgcsr_cg_solve without any device allocation, for callers that cannot
 * allocate (tight solver loops, harnesses that forbid hipMalloc): same
 * arguments, method and results (bit for bit) as rgcsr_cg_solve, but the
 * workspace (FP64 r and q, FP32 r, p, q, d, block partials and scalars) is a
 * static device array of 32 MiB + 16.25 KiB that the library holds on every
 * device it runs on until the process ends.  n (rows of A_lo) must be at most
 * 1,048,576, else RGCSR_EUNSUPPORTED before any device work.  No call
 * allocates or frees device memory.  Every call on one device shares that
 * device's workspace: calls that overlap on one device (other host threads,
 * or streams not ordered with each other) race and give wrong results; the
 * call synchronises the stream before it returns, so calls made one after
 * another are safe.  Not capturable in a HIP graph (it synchronises to test
 * convergence). */
rgcsr_status rgcsr_cg_solve_noalloc(rgcsr_handle A_lo, rgcsr_handle A_hi, const double *b, double *x,
                                    double tol, double inner_tol, int32_t max_outer, int32_t max_inner,
                                    void *stream, rgcsr_cg_stats *stats);

/* Plain CG with every vector and accumulation in FP64 on A (F64 or F32
 * storage), the all-FP64 comparison solver.  Same conventions. */
rgcsr_status rgcsr_cg_solve_f64(rgcsr_handle A, const double *b, double *x, double tol,
                                int32_t max_iter, void *stream, rgcsr_cg_stats *stats);

/* ---- Diagnostics ---------------------------------------------------------- */

const char *rgcsr_status_string(rgcsr_status s);
const char *rgcsr_last_error(void);

/* Library version string, e.g. "rgcsr 0.1 gfx950". */
const char *rgcsr_version(void);

/* ---- Row ordering (host only) ------------------------------------------------ */

/* Reverse Cuthill-McKee ordering of the symmetrised sparsity pattern of a
 * square host CSR matrix (row_ptr[n+1], col_idx[nnz]; validated like
 * rgcsr_from_csr).  The paper studies row orderings for padding and x cache
 * use (Section 4.4.2, Table 7: descending length and AMD) and leaves orderings
 * that improve x locality to future work (Section 5); this bandwidth-reducing
 * ordering stands in for AMD.  Rule: i ~ j when i != j and a_ij or a_ji is
 * stored; components are started from the unnumbered vertex of smallest
 * (degree, index); the unnumbered neighbours of each numbered vertex are
 * numbered in (degree, index) order (Cuthill and McKee, 1969); the sequence
 * is reversed (George, 1971).  Writes perm[new] = old (n int32, caller-owned
 * host memory); apply it to rows and columns alike (A' = P A P^T, x' = P x,
 * y = P^T y').  RGCSR_ECSR on malformed input, RGCSR_EOVERFLOW for n >= 2^31. */
rgcsr_status rgcsr_rcm_order(int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col_idx,
                             int32_t *perm);

/* ---- Measurement helper ----------------------------------------------------- */

/* Reads `bytes` bytes of device memory at buf with the nontemporal 16-byte
 * loads the SpMV uses for its value and column streams, one launch on
 * `stream`, so that timing it gives the achievable HBM read rate: a second
 * denominator beside the peak for the bandwidth model of Section 3.4.  buf
 * is a device pointer, 16-byte aligned, and bytes a multiple of 16; sink is a
 * device pointer to 4 bytes that the kernel may write (its contents are
 * meaningless).  Nothing is allocated; RGCSR_EINVAL on a null pointer or a
 * misaligned argument. */
rgcsr_status rgcsr_stream_read(const void *buf, int64_t bytes, void *sink, void *stream);

/* Gather floor of a matrix: reads n (column, value) pairs (col[n] int32,
 * val[n] float32, the matrix's CSR arrays) and gathers x[col[k]] for each,
 * with nothing else of an SpMV (no rows, no cross-lane sums): each of the
 * ceil(n / 8) lanes writes one partial sum to out (device, ceil(n / 8)
 * floats, meaningless as results).  Timing it bounds what any SpMV over the
 * same entries can reach when the x gathers dominate (Section 3.4 models the
 * bytes; random gathers are limited by the request rate instead).  Every
 * col[k] must lie in [0, n_cols) of x (not checked on the device). */
rgcsr_status rgcsr_gather_floor(const int32_t *col, const float *val, int64_t n, const float *x, int64_t n_cols,
                                float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RGCSR_H */
