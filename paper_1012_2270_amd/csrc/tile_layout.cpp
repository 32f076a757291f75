// Host side of the column-tiled long rows (tiles.h): row selection, the
// tile-major entry arrays, the per-XCD unit queues, and the long-row work of
// the remaining rows.  Plain C++17; no device code.
#include <algorithm>
#include <cstring>

#include "tiles.h"

namespace rg {

static int32_t lanes_for_len(int64_t len) {
    int64_t need = (len + kWaveUnroll - 1) / kWaveUnroll;
    int32_t t = 1;
    while (t < need && t < 64) t <<= 1;
    return t;
}

void build_long_work_except(const std::vector<int64_t> &long_ptr, const std::vector<uint8_t> &skip, LongWork &W) {
    W = LongWork{};
    const int64_t nl = (int64_t)long_ptr.size() - 1;
    int64_t i = 0;
    while (i < nl) {
        if (!skip.empty() && skip[i]) {
            i++;
            continue;
        }
        const int64_t len = long_ptr[i + 1] - long_ptr[i];
        if (len > kWaveRowMax) {
            const int64_t nch = (len + kBlockChunk - 1) / kBlockChunk;
            if (W.n_partials + nch > INT32_MAX) fail(RGCSR_EOVERFLOW, "too many long-row chunks");
            const int32_t pbase = nch > 1 ? (int32_t)W.n_partials : 0;
            for (int64_t c = 0; c < nch; c++) W.block.push_back(LongItem{(int32_t)i, (int32_t)c, (int32_t)nch, pbase});
            if (nch > 1) {
                W.combine.push_back(LongItem{(int32_t)i, 0, (int32_t)nch, pbase});
                W.n_partials += nch;
            }
            i++;
            continue;
        }
        // consecutive rows of one lane count share a wavefront item
        const int32_t T = lanes_for_len(len);
        const int32_t cap = 64 / T;
        int32_t cnt = 1;
        while (cnt < cap && i + cnt < nl && (skip.empty() || !skip[i + cnt])) {
            const int64_t l2 = long_ptr[i + cnt + 1] - long_ptr[i + cnt];
            if (l2 > kWaveRowMax || lanes_for_len(l2) != T) break;
            cnt++;
        }
        W.wave.push_back(LongItem{(int32_t)i, cnt, T, 0});
        i += cnt;
    }
}

void build_tiles(const HostLayout &L, int64_t min_len, HostTiles &T) {
    T = HostTiles{};
    if (min_len == 0 || L.nl == 0 || L.n_cols == 0) return;
    const bool automatic = min_len < 0;
    const int64_t C = tile_cols(L.vdt);
    const int64_t UM = tile_unit_max(L.vdt);
    const int64_t n_tiles = (L.n_cols + C - 1) / C;
    const int64_t thr = std::max<int64_t>(automatic ? 256 : min_len, (n_tiles + 1) / 2);
    // a row's segment in one tile must fit a unit: a row with more than UM
    // entries in some tile stays on the long-row path (columns
    // ascend within a row, so a segment is a run of consecutive entries)
    auto longest_segment = [&](int64_t i) {
        int64_t best = 0, run = 0, prev = -1;
        for (int64_t q = L.long_ptr[i]; q < L.long_ptr[i + 1]; q++) {
            const int64_t t = L.long_col[q] / C;
            run = t == prev ? run + 1 : 1;
            prev = t;
            best = std::max(best, run);
        }
        return best;
    };
    T.tiled.assign(L.nl, 0);
    int64_t n_ent = 0;
    for (int64_t i = 0; i < L.nl; i++) {
        const int64_t len = L.long_ptr[i + 1] - L.long_ptr[i];
        if (len < thr || (len > UM && longest_segment(i) > UM)) continue;
        T.tiled[i] = 1;
        T.trow.push_back((int32_t)i);
        n_ent += len;
    }
    if (T.trow.empty() || (automatic && n_ent < kTileMinEntries) || n_ent > INT32_MAX || L.long_nnz > INT32_MAX ||
        n_tiles * ((int64_t)T.trow.size() + 1) > INT32_MAX) {
        T = HostTiles{};
        return;
    }
    T.n_tiles = n_tiles;
    T.n_trows = (int64_t)T.trow.size();
    T.n_ent = n_ent;
    T.min_len = thr;
    const int64_t nt = T.n_trows;
    // counts per (tile, row), then tile-major offsets
    T.ptr.assign(n_tiles * (nt + 1), 0);
    for (int64_t k = 0; k < nt; k++) {
        const int64_t i = T.trow[k];
        for (int64_t q = L.long_ptr[i]; q < L.long_ptr[i + 1]; q++) T.ptr[(L.long_col[q] / C) * (nt + 1) + k]++;
    }
    int64_t run = 0;
    for (int64_t t = 0; t < n_tiles; t++) {
        int32_t *p = &T.ptr[t * (nt + 1)];
        for (int64_t k = 0; k <= nt; k++) {
            const int64_t c = k < nt ? p[k] : 0;
            p[k] = (int32_t)run;
            run += c;
        }
    }
    T.lcol.resize(n_ent);
    T.src.resize(n_ent);
    T.dst.assign((size_t)L.long_nnz, -1);
    std::vector<int32_t> fill(T.ptr);
    for (int64_t k = 0; k < nt; k++) {
        const int64_t i = T.trow[k];
        for (int64_t q = L.long_ptr[i]; q < L.long_ptr[i + 1]; q++) {
            const int64_t t = L.long_col[q] / C;
            const int32_t d = fill[t * (nt + 1) + k]++;
            T.lcol[d] = (uint16_t)(L.long_col[q] - t * C);
            T.src[d] = (int32_t)q;
            T.dst[q] = d;
        }
    }
    // units: consecutive rows of one tile, at most UM entries; the
    // longest segment sets the lanes per row, and the rows must fit
    // kTilePasses passes of kTileThreads / lanes rows
    auto lanes_for_seg = [](int64_t seg) {
        int32_t l = 1;
        while (l < 64 && (seg + l - 1) / l > kTileLaneSteps) l <<= 1;
        return l;
    };
    std::vector<std::vector<TileUnit>> per_tile(n_tiles);
    std::vector<int64_t> tile_cost(n_tiles, 0);
    for (int64_t t = 0; t < n_tiles; t++) {
        const int32_t *p = &T.ptr[t * (nt + 1)];
        int64_t r0 = 0;
        while (r0 < nt) {
            int64_t r1 = r0 + 1, seg = p[r0 + 1] - p[r0];
            while (r1 < nt && p[r1 + 1] - p[r0] <= UM) {
                const int64_t s2 = std::max<int64_t>(seg, p[r1 + 1] - p[r1]);
                if (r1 + 1 - r0 > (int64_t)kTilePasses * (kTileThreads / lanes_for_seg(s2))) break;
                seg = s2;
                r1++;
            }
            per_tile[t].push_back(TileUnit{(int32_t)t, (int32_t)r0, (int32_t)r1, lanes_for_seg(seg), p[r0], p[r1]});
            // a unit streams its entries and stages a tile of x (32 KB in
            // either precision, about as much as 4,096 entries of value and
            // column)
            tile_cost[t] += (p[r1] - p[r0]) + 4096;
            r0 = r1;
        }
    }
    // Workgroups go to the 8 XCDs round robin (workgroup b to XCD b % 8):
    // tiles are dealt to the least loaded XCD, largest first, and the queues
    // interleaved, the shorter ones padded with empty units, so each XCD's L2
    // serves only its own tiles of x.
    std::vector<int64_t> order(n_tiles);
    for (int64_t t = 0; t < n_tiles; t++) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return tile_cost[a] > tile_cost[b]; });
    std::vector<std::vector<TileUnit>> q(8);
    std::vector<int64_t> load(8, 0);
    for (int64_t t : order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += tile_cost[t];
        for (const TileUnit &u : per_tile[t]) q[x].push_back(u);
    }
    size_t depth = 0;
    for (auto &v : q) depth = std::max(depth, v.size());
    for (size_t d = 0; d < depth; d++)
        for (int x = 0; x < 8; x++) T.units.push_back(d < q[x].size() ? q[x][d] : TileUnit{-1, 0, 0, 1, 0, 0});
    while (!T.units.empty() && T.units.back().t < 0) T.units.pop_back();
    build_long_work_except(L.long_ptr, T.tiled, T.rest);
}

}  // namespace rg
