// Column tiles of the longest rows: x staged in LDS.  Internal.
//
// Rows of the long-row segment with at least `min_len` nonzeros are also
// stored split by column tile (tile_cols(vdt) columns per tile).  A tile kernel
// runs first: each workgroup stages a tile of x in LDS with coalesced loads,
// streams the tile's entries of a range of those rows, multiplies them
// against x read from LDS and writes one partial sum per (row, tile).  The
// SpMV kernel that follows adds each row's partial sums in a fixed order
// (its first units), beside its other work.  The random x gathers of these rows thus move
// from the L2/Infinity-Cache path into LDS (the paper's texture-cache study,
// Section 4.3, asks where x is kept; its Table 6 shows the long rows as the
// case the row-grouped kernel handles worst).
#pragma once

#include <cstdint>
#include <vector>

#include "internal.h"

namespace rg {

constexpr int kTileCols = 8192;      // x columns per tile: 32 KB of FP32 in LDS
constexpr int kTileCols64 = 4096;    // F64 storage (FP64 x): 32 KB of FP64 in LDS
constexpr int kTileUnitMax = 4096;   // entries per unit: 16 KB of FP32 products in LDS
constexpr int kTileUnitMax64 = 2048; // F64 storage: 16 KB of FP64 products in LDS
constexpr int kTileThreads = 512;    // one workgroup per unit, three per CU (48 KB of LDS each)
// Columns per tile and entries per unit of a layout with stored value type vdt.
constexpr int tile_cols(int vdt) { return vdt == RGCSR_F64 ? kTileCols64 : kTileCols; }
constexpr int tile_unit_max(int vdt) { return vdt == RGCSR_F64 ? kTileUnitMax64 : kTileUnitMax; }
constexpr int kTilePasses = 4;       // passes over a unit's rows (512 / lanes rows per pass)
constexpr int kTileLaneSteps = 16;   // products a lane adds per row segment, at most
constexpr int64_t kTileMinEntries = int64_t(1) << 18;  // automatic choice: tile only this many entries or more

// One unit of the tile kernel (a workgroup): tile t, tiled rows [r0, r1),
// `lanes` lanes per row (a power of two, at most 64, so that no lane adds
// more than kTileLaneSteps products of a segment, and the rows fit
// kTilePasses passes); t < 0 marks an empty unit.  The unit carries its
// entry range, so its entry loads need no dependent read of the row
// pointers.
struct TileUnit {
    int32_t t, r0, r1, lanes;
    int32_t e0, e1;  // the unit's entries [e0, e1) of the tile-major arrays
};

struct HostTiles {
    int64_t n_tiles = 0, n_trows = 0, n_ent = 0;
    int64_t min_len = 0;               // threshold that selected the rows
    std::vector<int32_t> trow;         // [n_trows] long-list index of each tiled row
    std::vector<int32_t> ptr;          // [n_tiles * (n_trows + 1)] first entry of (tile, row)
    std::vector<uint16_t> lcol;        // [n_ent] column - tile * kTileCols
    std::vector<int32_t> src;          // [n_ent] position of the entry in the long-row segment
    std::vector<int32_t> dst;          // [long_nnz] inverse: position in the tiled copy, -1 if not tiled
    std::vector<TileUnit> units;
    std::vector<uint8_t> tiled;        // [nl] 1 when long row i is tiled
    LongWork rest;                     // long-row work of the rows that are not tiled
    bool active() const { return n_trows > 0; }
};

// Selects the tiled rows of layout L (long rows of at least
// max(min_len, tiles / 2) nonzeros, so the partial sums never outnumber the
// entries twice over, and at most tile_unit_max(vdt) nonzeros in any one
// tile, so a row's segment fits a unit;
// min_len < 0 picks 256 and keeps the tiles only when they hold at least
// kTileMinEntries entries; 0 disables) and builds their index arrays and
// units (values are copied on the device through src).  Needs L.long_ptr and
// L.long_col.
void build_tiles(const HostLayout &L, int64_t min_len, HostTiles &T);

// Long-row work items of the rows not tiled (the tiled ones skipped).
void build_long_work_except(const std::vector<int64_t> &long_ptr, const std::vector<uint8_t> &skip, LongWork &W);

}  // namespace rg
