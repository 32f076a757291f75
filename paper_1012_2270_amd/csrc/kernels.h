// Kernel launch interface used by the C ABI (abi.cpp).  Internal.
#pragma once

#include <hip/hip_runtime_api.h>

#include "internal.h"
#include "tiles.h"

namespace rg {

// Everything one SpMV launch reads.  Device pointers.
struct SpmvParams {
    // grouped (short) rows
    const int64_t *gp;         // [ng+1] group pointers (slot offsets)
    const int64_t *gend;       // [ng] group ends, or null when group g ends at gp[g+1]
    const int32_t *grp_row0;   // [ng+1] first short row of each group (ragged only)
    const int32_t *short_len;  // [ns] row lengths
    const int32_t *short_row;  // [ns] output row of each short row (perm only)
    const void *slot_val;      // [slots] storage dtype
    const int32_t *slot_col;   // [slots]
    int64_t ng, ns;
    int32_t G;
    int32_t wpg;               // wavefronts per group when G*T >= 64, else 0
    int32_t gpw;               // groups per wavefront when G*T < 64, else 0
    int32_t ragged, perm;
    int32_t pad;               // value/column loads run over the group width
    const int32_t *short_items;  // [waves] runs of wave items (rows-per-lane chosen per wavefront)
    // long rows
    const LongItem *wave_work;   // [n_wave_long] wave items
    const LongItem *block_work;  // [n_block_items] block items
    const int32_t *long_row;
    const int64_t *long_ptr;
    const void *long_val;
    const int32_t *long_col;
    void *partial;               // chunk partial sums (accumulator type, K per chunk)
    int32_t n_block_items;       // units [0, n_block_items) are block items
    int32_t n_wave_long;         // wave items [0, n_wave_long) are long-row wave items
    int32_t n_wave_items;        // all wave items (long-row wave items, then row groups)
    int32_t total_units;         // n_block_items + ceil(n_wave_items / kBlockWaves)
    int32_t n_long_units;        // units holding long-row work: n_block_items + ceil(n_wave_long / kBlockWaves)
    // setval/grad: their row-group wavefronts (one row per lane) number
    // total_waves - n_long_waves (n_long_waves = long rows)
    int32_t n_long_waves;
    int32_t total_waves;
    // column-tiled long rows (one right-hand side, FP64 vectors for F64
    // storage, else FP32): the tile kernel has written one partial sum per
    // (tile, tiled row) in the vector type; units [0, n_comb_units) of the
    // launch add them, 64 rows each
    const void *tile_partial;    // [n_tiles * n_trows]
    const int32_t *tile_orow;    // [n_trows] output row of each tiled row
    int32_t n_comb_units, n_tiles, n_trows;
    // value updates: position of each long-row element in the tiled copy
    // (-1 when its row is not tiled) and the tiled values; null without tiles
    const int32_t *tile_dst;     // [long_nnz]
    void *tile_vals;             // [tile entries] storage dtype
    // column panels: workgroup (or, in a persistent launch, table entry) j
    // runs unit unit_map[j], none when -1; null = the usual unit order.  A
    // negative output row code -1 - s (short_row, long_row) names slot s of
    // pan_y (pan_ld elements per slot) instead of a row of y.
    const int32_t *unit_map;     // [n_map]
    int32_t n_map;
    void *pan_y;
    int64_t pan_ld;
    // vectors
    const void *x;
    void *y;
    int64_t ldx, ldy;
};

struct HybParams {
    int64_t n, n_pad, m;
    int32_t K1;
    const int32_t *ell_col;
    const void *ell_val;
    const int32_t *coo_row, *coo_col;
    const void *coo_val;
};

// CG scalar slots and finishing modes.
enum { kRR = 0, kRR0 = 1, kPQ = 2, kAlpha = 3, kBeta = 4, kOut = 5, kNumScal = 8 };
enum { kScalPQ = 0, kScalRRNew = 1, kScalRRInit = 2, kScalOut = 3 };

// Several right-hand sides take the runs of rows per lane (R = 0) up to this
// many accumulator bytes per row (F32 K <= 4, F64 K <= 2); wider, one row per lane.
constexpr int kRunsRowBytes = 16;
hipError_t launch_spmv(const SpmvParams &P, int vdt, int vec_f64, int T, int K, int R, int load_policy, int nwg,
                       hipStream_t st);
// Split rows of a column-panel copy: Y[crow[i]] = sum of the piece sums
// yv[vidx[s]] (K values each) for s in [cptr[i], cptr[i + 1]), in that order
// (0 for a row without pieces).
hipError_t launch_panel_combine(const int32_t *crow, const int32_t *cptr, int64_t n, const int32_t *vidx,
                                const void *yv, void *Y, int64_t ldy, int vec_f64, int K, hipStream_t st);
hipError_t launch_combine(const LongItem *items, int32_t n, const int32_t *long_row, const void *partial, void *Y,
                          int64_t ldy, void *pan_y, int64_t pan_ld, int vec_f64, int K, hipStream_t st);
hipError_t launch_setval(const SpmvParams &P, int vdt, int T, const void *theta, int theta_f64,
                         const int64_t *row_ptr, hipStream_t st);
hipError_t launch_gather_map(int64_t n, int vdt, const int32_t *map, const void *theta, int theta_f64,
                             void *dst, hipStream_t st);
hipError_t launch_grad(const SpmvParams &P, int vdt, int vec_f64, int T, const void *dy, void *dvals, void *dx,
                       const int64_t *row_ptr, bool want_dvals, bool atomic_dx, hipStream_t st);
hipError_t launch_hyb(const HybParams &H, int vdt, int vec_f64, const void *x, void *y, hipStream_t st);

hipError_t launch_dot(int64_t n, const void *a, const void *b, int f64, double *part, int nb, hipStream_t st);
hipError_t launch_scalar(const double *part, int nb, double *scal, int mode, hipStream_t st);
hipError_t launch_cg_xr(int64_t n, void *x, void *r, const void *p, const void *q, int f64, const double *scal,
                        double *part, int nb, hipStream_t st);
hipError_t launch_cg_p(int64_t n, void *p, const void *r, int f64, const double *scal, int nb, hipStream_t st);
hipError_t launch_resid(int64_t n, const double *b, const double *q, double *r, double *part, int nb,
                        hipStream_t st);
hipError_t launch_refine_start(int64_t n, const double *r64, double s, float *r, float *d, float *p,
                               double *part, int nb, hipStream_t st);
hipError_t launch_refine_add(int64_t n, double *x, const float *d, double inv_s, int nb, hipStream_t st);
hipError_t launch_copy(int64_t n, const void *a, void *b, int f64, int nb, hipStream_t st);
hipError_t launch_stream_read(const void *a, int64_t n16, int32_t *sink, int nb, hipStream_t st);
hipError_t launch_gather_floor(const int32_t *col, const float *val, int64_t n, const float *x, float *out,
                               hipStream_t st);
hipError_t launch_zero(int64_t n, void *a, int esz, int nb, hipStream_t st);
// Tile kernel: one workgroup per unit, partial[t * n_trows + row] for the
// rows of every unit.
struct TileParams {
    const TileUnit *units;
    const int32_t *ptr;      // [n_tiles * (n_trows + 1)]
    const uint16_t *lcol;    // [n_ent] column within the tile
    const void *val;         // [n_ent] storage dtype
    const void *x;           // FP64 for F64 storage, else FP32
    void *partial;           // [n_tiles * n_trows], the type of x
    int64_t n_cols;
    int32_t n_trows;
    int32_t x_aligned;       // x is 16-byte aligned (vector loads of a tile)
};
hipError_t launch_tile_spmv(const TileParams &P, int vdt, int n_units, hipStream_t st);
// tile_val[dst[q]] = long_val[q] for the n long-row elements whose row is
// tiled (dst[q] >= 0)
hipError_t launch_tile_values(int64_t n, const int32_t *dst, const void *long_val, void *tile_val, int esz,
                              hipStream_t st);

// Static device workspace of the allocation-free mixed-precision CG
// (rgcsr_cg_solve_noalloc): FP64 r and q, FP32 r, p, q, d for up to
// kNoAllocCgMaxRows rows, then the block partials and the scalar slots, at
// fixed 256-byte aligned offsets.  noalloc_cg_workspace returns its address on
// the current device (looked up once per device and kept).
constexpr int64_t kNoAllocCgMaxRows = int64_t(1) << 20;
constexpr int64_t kNoAllocCgMaxBlocks = 2048;
constexpr size_t kNoAllocOffQ64 = 8 * kNoAllocCgMaxRows;
constexpr size_t kNoAllocOffR = 16 * kNoAllocCgMaxRows;
constexpr size_t kNoAllocOffP = 20 * kNoAllocCgMaxRows;
constexpr size_t kNoAllocOffQ = 24 * kNoAllocCgMaxRows;
constexpr size_t kNoAllocOffD = 28 * kNoAllocCgMaxRows;
constexpr size_t kNoAllocOffPart = 32 * kNoAllocCgMaxRows;
constexpr size_t kNoAllocOffScal = kNoAllocOffPart + 8 * kNoAllocCgMaxBlocks;
constexpr size_t kNoAllocCgBytes = kNoAllocOffScal + 256;
static_assert(8 * kNumScal <= 256, "scalar slots fit their region");
hipError_t noalloc_cg_workspace(void **base);

}  // namespace rg
