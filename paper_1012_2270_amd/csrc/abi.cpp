// C ABI of librgcsr (declared in include/rgcsr.h): handles, conversion,
// launches, value updates, backward pass, Hybrid and the CG drivers.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "convert.h"
#include "internal.h"
#include "kernels.h"
#include "tiles.h"

namespace rg {


#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            ::rg::fail(e_ == hipErrorOutOfMemory ? RGCSR_ENOMEM : RGCSR_EHIP,                           \
                       std::string(#expr) + ": " + hipGetErrorString(e_));                             \
    } while (0)

static int current_device() {
    int d = 0;
    HIPCHK(hipGetDevice(&d));
    return d;
}

static int cu_count(int dev) {
    static std::mutex mu;
    static std::vector<int> cache;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int n = 0;
        HIPCHK(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
        cache[dev] = n > 0 ? n : 256;
    }
    return cache[dev];
}

// One device allocation carved into 256-byte aligned arrays.
struct Arena {
    std::vector<std::pair<void **, size_t>> req;
    size_t total = 0;
    template <class T> void add(T **p, size_t count) {
        if (count == 0) {
            *p = nullptr;
            return;
        }
        req.push_back({(void **)p, count * sizeof(T)});
        total += (count * sizeof(T) + 255) / 256 * 256;
    }
    // Places the arrays in `base` (caller memory of at least `total` bytes,
    // 256-byte aligned) or, when null, in one new hipMalloc block.
    void *commit(void *base = nullptr) {
        if (total == 0) return nullptr;
        if (!base) HIPCHK(hipMalloc(&base, total));
        size_t off = 0;
        for (auto &r : req) {
            *r.first = (char *)base + off;
            off += (r.second + 255) / 256 * 256;
        }
        return base;
    }
};

template <class T> static void upload(T *dst, const std::vector<T> &src, hipStream_t st) {
    if (!src.empty() && dst) HIPCHK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
}
static void upload_bytes(void *dst, const std::vector<uint8_t> &src, hipStream_t st) {
    if (!src.empty() && dst) HIPCHK(hipMemcpyAsync(dst, src.data(), src.size(), hipMemcpyHostToDevice, st));
}

}  // namespace rg

using namespace rg;

struct rgcsr_matrix_s {
    int device = 0;
    LayoutParams prm{};
    int vdt = RGCSR_F32, esz = 4;
    int64_t n_rows = 0, n_cols = 0, nnz = 0, ng = 0, ns = 0, nl = 0, slots = 0, long_nnz = 0;
    int64_t n_matrices = 1, n_wave_long = 0, n_block = 0, n_combine = 0, n_partials = 0;
    bool ragged = false, perm = false;
    int32_t wpg = 0, gpw = 0;
    int32_t R = 1, pad = 0;  // kernel schedule: rows per lane (0 = per wavefront), padded-width loads
    int32_t lp = 0;          // load policy (0 = nontemporal matrix streams, cached x)
    std::vector<int32_t> items;  // R = 0: one word per wavefront, first wave item << 2 | log2(rows per lane)
    std::vector<int64_t> row_off, col_off;
    void *mem = nullptr;
    size_t bytes = 0;
    bool owns_mem = true;  // false: the arrays live in caller memory (rgcsr_build)
    int64_t *gp = nullptr;
    int64_t *gend = nullptr;  // group ends when they differ from the next group's start
    int32_t *grp_row0 = nullptr, *short_len = nullptr, *short_row = nullptr, *slot_col = nullptr;
    void *slot_val = nullptr;
    LongItem *wave_work = nullptr, *block_work = nullptr, *combine = nullptr;
    int32_t *long_row = nullptr, *long_col = nullptr;
    int32_t *short_items = nullptr;
    int64_t *long_ptr = nullptr;
    void *long_val = nullptr;
    void *partial = nullptr;
    int64_t *row_ptr = nullptr;  // CSR map, nullable
    rgcsr_matrix_s *AT = nullptr;
    int32_t *t_map_slot = nullptr, *t_map_long = nullptr;
    // column-tiled long rows (tiles.h); their arrays live in `mem`, or in
    // tile_mem for handles converted on the device
    int64_t n_tiles = 0, n_trows = 0, n_tent = 0, n_tunits = 0;
    int64_t n_rest_wave = 0, n_rest_block = 0, n_rest_combine = 0;
    TileUnit *tile_units = nullptr;
    int32_t *tile_ptr = nullptr, *tile_dst = nullptr, *tile_orow = nullptr;
    uint16_t *tile_lcol = nullptr;
    void *tile_val = nullptr;
    void *tile_partial = nullptr;         // FP64 for F64 storage, else FP32
    LongItem *rest_wave = nullptr, *rest_block = nullptr, *rest_combine = nullptr;
    void *tile_mem = nullptr;
    size_t tile_bytes = 0;
    std::shared_ptr<HostTiles> pending_tiles;  // host arrays until they are uploaded
    // column panels (panel_layout.cpp): PN is a handle of its own over the
    // stacked pieces, used by launches whose x slice per panel fits an L2;
    // the arrays below belong to PN and live in its block
    rgcsr_matrix_s *PN = nullptr;
    int32_t n_panels = 0;
    int64_t panel_cols = 0;                    // widest panel, in columns
    int64_t n_split = 0;                       // rows split into pieces (the others are written whole)
    int32_t *unit_map_rows = nullptr;          // [n_map_rows] workgroup -> unit, rows-per-lane schedule
    int32_t *unit_map_one = nullptr;           // [n_map_one] workgroup -> unit, one row per lane
    int32_t n_map_rows = 0, n_map_one = 0;
    int32_t *pan_crow = nullptr, *pan_cptr = nullptr, *pan_vidx = nullptr;  // split rows and their pieces
    void *pan_y = nullptr;                     // [split pieces * kPanelRowBytes] per-piece sums
    std::shared_ptr<std::vector<int32_t>> pending_maps[5];  // host copies until they are uploaded
};

struct hyb_matrix_s {
    int device = 0;
    int vdt = RGCSR_F32, esz = 4;
    int64_t n_rows = 0, n_cols = 0, nnz = 0, n_pad = 0, K1 = 0, m = 0;
    void *mem = nullptr;
    size_t bytes = 0;
    int32_t *ell_col = nullptr, *coo_row = nullptr, *coo_col = nullptr;
    void *ell_val = nullptr, *coo_val = nullptr;
};

namespace {

void check_device_geometry(const LayoutParams &p) {
    const int64_t GT = (int64_t)p.G * p.T;
    if (!(GT % 64 == 0 || 64 % GT == 0))
        fail(RGCSR_EUNSUPPORTED, "device kernels need group_size * lanes_per_row to be a multiple or a divisor of 64");
}

}  // namespace

// Host layout of one matrix and its handle(s) with the device arrays listed
// but not placed; rgcsr_build hands the handles over.
struct rgcsr_plan_s {
    Built B;
    bool with_row_ptr = false;
    Arena a, aT;
    rgcsr_matrix_s *h = nullptr, *hT = nullptr;
    ~rgcsr_plan_s() {
        delete h;
        delete hT;
    }
};

namespace {

// Runs of wave items, one per wavefront: starting at wave item j, the
// longest run R in {8, 4, 2} whose widest group times R is at most the step
// budget, else R = 1.  A wavefront then needs a single pass over its loads
// unless it holds one group wider than the budget.  half_budget: 8-byte
// values on a schedule with one R everywhere (the kernel then loads
// kLaneSteps / 2 / R steps per pass); rows wider than that budget take R = 2
// (two rows per lane, four steps per pass), 2% faster than one row per lane
// on the FP64 27-point stencil.
std::vector<int32_t> wave_runs(const HostLayout &L, int32_t wpg, bool half_budget) {
    const int64_t budget = half_budget ? kLaneSteps / 2 : kLaneSteps;
    const int64_t n = (int64_t)(L.gp.size() - 1) * wpg;
    std::vector<int64_t> width(n);
    for (int64_t j = 0; j < n; j++) {
        const int64_t g = j / wpg;
        const int64_t row0 = L.ragged ? L.grp_row0[g] : g * L.G;
        const int64_t sg = L.ragged ? L.grp_row0[g + 1] - row0 : std::min<int64_t>(L.G, L.ns - row0);
        width[j] = sg > 0 ? (L.group_end(g) - L.gp[g]) / (sg * L.T) : 0;
    }
    std::vector<int32_t> runs;
    for (int64_t j = 0; j < n;) {
        int lg = 3;
        for (; lg > 0; lg--) {
            const int64_t R = int64_t(1) << lg;
            if (j + R > n) continue;
            int64_t wmax = 0;
            for (int64_t r = 0; r < R; r++) wmax = std::max(wmax, width[j + r]);
            if (wmax * R <= budget) break;
        }
        if (lg == 0 && half_budget && j + 2 <= n && width[j] > budget) lg = 1;
        runs.push_back((int32_t)((j << 2) | lg));
        j += int64_t(1) << lg;
    }
    return runs;
}

// Kernel schedule: padded-width loads when padding is at most the number of
// grouped nonzeros; rows per lane fixed by the caller or, by default, chosen
// per wavefront (wave_runs) when a lane owns a whole row and a group fills
// whole wavefronts, else one.
void choose_schedule(rgcsr_matrix_s *h, const HostLayout &L, int64_t short_nnz, bool no_empty,
                     int32_t rows_per_lane, int32_t pad_loads, int32_t load_policy) {
    const int64_t pad_slots = L.slots - short_nnz;
    if (pad_loads < -1 || pad_loads > 3) fail(RGCSR_EINVAL, "pad_loads must be -1, 0, 1, 2 or 3");
    if (pad_loads >= 2 && h->gpw > 0)
        fail(RGCSR_EUNSUPPORTED, "pad_loads 2 and 3 need group_size * lanes_per_row a multiple of 64");
    // row lengths can be read off the columns when a lane owns a whole row
    // and no grouped row is empty
    const bool cols_give_len = L.T == 1 && h->gpw == 0 && no_empty;
    if (pad_loads == 3 && !cols_give_len)
        fail(RGCSR_EUNSUPPORTED, "pad_loads 3 needs lanes_per_row = 1 and no empty rows among the grouped rows");
    if (pad_loads < 0) h->pad = pad_slots <= short_nnz ? (cols_give_len ? 3 : 1) : 0;
    else h->pad = pad_loads;
    if (load_policy < 0 || load_policy > 2) fail(RGCSR_EINVAL, "load_policy must be 0, 1 or 2");
    if (load_policy != 0 && (L.vdt != RGCSR_F32 || L.T != 1))
        fail(RGCSR_EUNSUPPORTED, "load policies 1 and 2 need F32 values and lanes_per_row = 1");
    h->lp = load_policy;
    int32_t R = rows_per_lane;
    if (R != 0 && R != 1 && R != 2 && R != 4 && R != 8) fail(RGCSR_EINVAL, "rows_per_lane must be 0, 1, 2, 4 or 8");
    if (L.T != 1 || h->gpw > 0) R = 1;
    // run words hold the first wave item in 29 bits
    if (R == 0 && (int64_t)(L.gp.size() - 1) * h->wpg >= (int64_t(1) << 29)) R = 1;
    h->items.clear();
    if (R == 0) {
        // the same run length everywhere (uniform widths, e.g. stencils): the
        // fixed schedule does the same without reading run words, and with
        // 8-byte values it takes half the step budget
        auto uniform = [](const std::vector<int32_t> &items) {
            bool same = !items.empty();
            for (size_t i = 0; same && i < items.size(); i++) {
                const int32_t lg = items[0] & 3;
                same = (items[i] >> 2) == (int32_t)(i << lg) && ((items[i] & 3) == lg || i + 1 == items.size());
            }
            return same;
        };
        h->items = wave_runs(L, h->wpg, false);
        if (L.esz == 8 && uniform(h->items)) {
            std::vector<int32_t> half = wave_runs(L, h->wpg, true);
            if (uniform(half)) h->items = half;
        }
        if (uniform(h->items)) {
            R = 1 << (h->items[0] & 3);
            h->items.clear();
        }
    }
    h->R = R;
}

// A handle whose fields describe the host layout and whose device arrays are
// listed in `a` but not yet placed (plan step of rgcsr_plan_from_csr and of
// make_device).  Host work only.
// Tile arrays of the handle, listed in arena a (counts set on h).
void add_tile_arrays(rgcsr_matrix_s *h, const HostTiles &T, Arena &a) {
    h->n_tiles = T.n_tiles;
    h->n_trows = T.n_trows;
    h->n_tent = T.n_ent;
    h->n_tunits = (int64_t)T.units.size();
    h->n_rest_wave = (int64_t)T.rest.wave.size();
    h->n_rest_block = (int64_t)T.rest.block.size();
    h->n_rest_combine = (int64_t)T.rest.combine.size();
    if (!T.active()) return;
    a.add(&h->tile_units, T.units.size());
    a.add(&h->tile_ptr, T.ptr.size());
    a.add(&h->tile_lcol, (size_t)T.n_ent);
    a.add((uint8_t **)&h->tile_val, (size_t)T.n_ent * h->esz);
    a.add(&h->tile_dst, T.dst.size());
    a.add(&h->tile_orow, (size_t)T.n_trows);
    a.add((uint8_t **)&h->tile_partial, (size_t)(T.n_tiles * T.n_trows) * (h->vdt == RGCSR_F64 ? 8 : 4));
    a.add(&h->rest_wave, T.rest.wave.size());
    a.add(&h->rest_block, T.rest.block.size());
    a.add(&h->rest_combine, T.rest.combine.size());
}

// Uploads the tile arrays; values come from the handle's long-row segment
// (already on the device) through the source map.
void upload_tiles(rgcsr_matrix_s *h, const HostTiles &T, const std::vector<int32_t> &long_row, hipStream_t st) {
    if (!T.active()) return;
    upload(h->tile_units, T.units, st);
    upload(h->tile_ptr, T.ptr, st);
    upload(h->tile_lcol, T.lcol, st);
    upload(h->tile_dst, T.dst, st);
    std::vector<int32_t> orow(T.n_trows);
    for (int64_t k = 0; k < T.n_trows; k++) orow[k] = long_row[T.trow[k]];
    upload(h->tile_orow, orow, st);
    upload(h->rest_wave, T.rest.wave, st);
    upload(h->rest_block, T.rest.block, st);
    upload(h->rest_combine, T.rest.combine, st);
    HIPCHK(launch_tile_values((int64_t)T.dst.size(), h->tile_dst, h->long_val, h->tile_val, h->esz, st));
    // orow is a host temporary: wait for its copy
    HIPCHK(hipStreamSynchronize(st));
}

std::vector<int32_t> panel_unit_map(const rgcsr_matrix_s *h, const HostLayout &L, const PanelBuilt &pb,
                                    bool use_rows);

rgcsr_matrix_s *prepare_handle(const HostLayout &L, bool with_row_ptr, const HostLayout *map, Arena &a,
                               int32_t rows_per_lane, int32_t pad_loads, int32_t load_policy, int32_t tile_min_len,
                               const PanelBuilt *pb = nullptr) {
    auto *h = new rgcsr_matrix_s();
    try {
        h->prm = LayoutParams{L.G, L.T, L.sigma, L.tau};
        h->vdt = L.vdt;
        h->esz = L.esz;
        h->n_rows = L.n_rows; h->n_cols = L.n_cols; h->nnz = L.nnz;
        h->ng = L.ng; h->ns = L.ns; h->nl = L.nl; h->slots = L.slots; h->long_nnz = L.long_nnz;
        h->n_matrices = L.n_matrices;
        h->n_wave_long = (int64_t)L.work.wave.size();
        h->n_block = (int64_t)L.work.block.size();
        h->n_combine = (int64_t)L.work.combine.size();
        h->n_partials = L.work.n_partials;
        h->ragged = L.ragged;
        h->perm = !L.short_identity();
        h->row_off = L.row_off;
        h->col_off = L.col_off;
        const int64_t GT = (int64_t)L.G * L.T;
        h->wpg = GT >= 64 ? (int32_t)(GT / 64) : 0;
        h->gpw = GT < 64 ? (int32_t)(64 / GT) : 0;
        int64_t short_nnz = 0;
        bool no_empty = true;
        for (int32_t v : L.short_len) {
            short_nnz += v;
            no_empty = no_empty && v > 0;
        }
        choose_schedule(h, L, short_nnz, no_empty, rows_per_lane, pad_loads, load_policy);
        // the kernels address a group's slots with 32-bit byte offsets
        int64_t max_group = 0;
        for (size_t g = 0; g + 1 < L.gp.size(); g++) max_group = std::max(max_group, L.group_end(g) - L.gp[g]);
        if (max_group * std::max(L.esz, 4) >= (int64_t(1) << 32))
            fail(RGCSR_EOVERFLOW, "a row group holds 4 GiB or more; use a long-row threshold");

        a.add(&h->gp, L.gp.size());
        a.add(&h->gend, L.has_gaps() ? L.gend.size() : 0);
        a.add(&h->grp_row0, h->ragged ? L.grp_row0.size() : 0);
        a.add(&h->short_len, L.short_len.size());
        a.add(&h->short_row, h->perm ? L.short_row.size() : 0);
        a.add((uint8_t **)&h->slot_val, L.slot_val.size());
        a.add(&h->slot_col, L.slot_col.size());
        a.add(&h->short_items, h->items.size());
        a.add(&h->wave_work, L.work.wave.size());
        a.add(&h->block_work, L.work.block.size());
        a.add(&h->combine, L.work.combine.size());
        a.add(&h->long_row, L.long_row.size());
        a.add(&h->long_ptr, L.long_ptr.size());
        a.add((uint8_t **)&h->long_val, L.long_val.size());
        a.add(&h->long_col, L.long_col.size());
        a.add((uint8_t **)&h->partial, (size_t)L.work.n_partials * 32 * sizeof(double));
        if (with_row_ptr) a.add(&h->row_ptr, (size_t)L.n_rows + 1);
        if (map) {
            a.add(&h->t_map_slot, (size_t)map->slots);
            a.add(&h->t_map_long, (size_t)map->long_nnz);
        }
        // column tiles: FP64 x for F64 storage, FP32 x otherwise
        auto tiles = std::make_shared<HostTiles>();
        build_tiles(L, tile_min_len, *tiles);
        add_tile_arrays(h, *tiles, a);
        if (tiles->active()) h->pending_tiles = tiles;
        if (pb) {
            // panel copy: workgroup tables for both schedules, the pieces of
            // each output row, and the per-piece sums
            h->n_panels = pb->P;
            for (int32_t q = 0; q < pb->P; q++) h->panel_cols = std::max(h->panel_cols, pb->cb[q + 1] - pb->cb[q]);
            h->n_split = (int64_t)pb->crow.size();
            auto rows = std::make_shared<std::vector<int32_t>>(panel_unit_map(h, L, *pb, true));
            auto one = std::make_shared<std::vector<int32_t>>(panel_unit_map(h, L, *pb, false));
            h->n_map_rows = (int32_t)rows->size();
            h->n_map_one = (int32_t)one->size();
            a.add(&h->unit_map_rows, rows->size());
            a.add(&h->unit_map_one, one->size());
            a.add(&h->pan_crow, pb->crow.size());
            a.add(&h->pan_cptr, pb->cptr.size());
            a.add(&h->pan_vidx, pb->vidx.size());
            a.add((uint8_t **)&h->pan_y, (size_t)pb->split_pieces * kPanelRowBytes);
            h->pending_maps[0] = rows;
            h->pending_maps[1] = one;
            h->pending_maps[2] = std::make_shared<std::vector<int32_t>>(pb->crow);
            h->pending_maps[3] = std::make_shared<std::vector<int32_t>>(pb->cptr);
            h->pending_maps[4] = std::make_shared<std::vector<int32_t>>(pb->vidx);
        }
        h->bytes = a.total;
    } catch (...) {
        delete h;
        throw;
    }
    return h;
}

// Places a prepared handle's arrays (in `buf` when given: caller memory the
// handle borrows; else in a block the handle owns) and uploads the layout.
// On failure the handle is left for the caller to free.
void place_and_upload(rgcsr_matrix_s *h, Arena &a, const HostLayout &L, const std::vector<int64_t> *row_ptr,
                      const HostLayout *map, void *buf, hipStream_t st) {
    h->device = current_device();
    h->owns_mem = buf == nullptr;
    h->mem = a.commit(buf);
    upload(h->gp, L.gp, st);
    if (h->gend) upload(h->gend, L.gend, st);
    if (h->ragged) upload(h->grp_row0, L.grp_row0, st);
    upload(h->short_len, L.short_len, st);
    if (h->perm) upload(h->short_row, L.short_row, st);
    upload_bytes(h->slot_val, L.slot_val, st);
    upload(h->slot_col, L.slot_col, st);
    upload(h->short_items, h->items, st);
    upload(h->wave_work, L.work.wave, st);
    upload(h->block_work, L.work.block, st);
    upload(h->combine, L.work.combine, st);
    upload(h->long_row, L.long_row, st);
    upload(h->long_ptr, L.long_ptr, st);
    upload_bytes(h->long_val, L.long_val, st);
    upload(h->long_col, L.long_col, st);
    if (row_ptr && h->row_ptr) upload(h->row_ptr, *row_ptr, st);
    if (map) {
        if (map->slots) HIPCHK(hipMemcpyAsync(h->t_map_slot, map->slot_val.data(), (size_t)map->slots * 4, hipMemcpyHostToDevice, st));
        if (map->long_nnz) HIPCHK(hipMemcpyAsync(h->t_map_long, map->long_val.data(), (size_t)map->long_nnz * 4, hipMemcpyHostToDevice, st));
    }
    if (h->pending_tiles) upload_tiles(h, *h->pending_tiles, L.long_row, st);
    int32_t *const map_dst[5] = {h->unit_map_rows, h->unit_map_one, h->pan_crow, h->pan_cptr, h->pan_vidx};
    for (int i = 0; i < 5; i++)
        if (h->pending_maps[i]) upload(map_dst[i], *h->pending_maps[i], st);
    HIPCHK(hipStreamSynchronize(st));
    h->pending_tiles.reset();
    for (auto &m : h->pending_maps) m.reset();
}

rgcsr_matrix_s *make_device(const HostLayout &L, const std::vector<int64_t> *row_ptr,
                            const HostLayout *map, hipStream_t st, int32_t rows_per_lane = 0,
                            int32_t pad_loads = -1, int32_t load_policy = 0, int32_t tile_min_len = 0,
                            const PanelBuilt *pb = nullptr) {
    Arena a;
    rgcsr_matrix_s *h = prepare_handle(L, row_ptr != nullptr, map, a, rows_per_lane, pad_loads, load_policy,
                                       tile_min_len, pb);
    try {
        place_and_upload(h, a, L, row_ptr, map, nullptr, st);
    } catch (...) {
        (void)hipStreamSynchronize(st);
        if (h->mem && h->owns_mem) (void)hipFree(h->mem);
        delete h;
        throw;
    }
    return h;
}

// Handle built from device CSR arrays: the plan (order, widths, offsets) and
// the scatter run on the device (convert.hip); only sizes, the group and
// long-row offsets and the small work lists go through the host.
rgcsr_matrix_s *make_device_on_device(DevPlan &P, const LayoutParams &p, int vdt, const int64_t *rp,
                                      const int32_t *col, const void *vals, int vals_dt, bool keep_map,
                                      hipStream_t st, int32_t rows_per_lane, int32_t pad_loads,
                                      int32_t load_policy, int32_t tile_min_len) {
    HostLayout L;  // sizes and host-side offsets only
    L.G = p.G; L.T = p.T; L.sigma = p.sigma; L.tau = p.tau; L.vdt = vdt; L.esz = dtype_size(vdt);
    L.n_rows = P.n_rows; L.n_cols = P.n_cols; L.nnz = P.nnz;
    L.ng = P.ng; L.ns = P.ns; L.nl = P.nl; L.slots = P.slots; L.long_nnz = P.long_nnz;
    L.n_matrices = 1;
    L.gp = P.gp_host;
    L.ragged = false;
    L.row_off = {0, P.n_rows};
    L.col_off = {0, P.n_cols};
    build_long_work(P.long_ptr_host, L.work);
    auto *h = new rgcsr_matrix_s();
    try {
        h->device = current_device();
        h->prm = p;
        h->vdt = vdt;
        h->esz = L.esz;
        h->n_rows = L.n_rows; h->n_cols = L.n_cols; h->nnz = L.nnz;
        h->ng = L.ng; h->ns = L.ns; h->nl = L.nl; h->slots = L.slots; h->long_nnz = L.long_nnz;
        h->n_matrices = 1;
        h->n_wave_long = (int64_t)L.work.wave.size();
        h->n_block = (int64_t)L.work.block.size();
        h->n_combine = (int64_t)L.work.combine.size();
        h->n_partials = L.work.n_partials;
        h->ragged = false;
        h->perm = P.perm;
        h->row_off = L.row_off;
        h->col_off = L.col_off;
        const int64_t GT = (int64_t)L.G * L.T;
        h->wpg = GT >= 64 ? (int32_t)(GT / 64) : 0;
        h->gpw = GT < 64 ? (int32_t)(64 / GT) : 0;
        choose_schedule(h, L, P.nnz - P.long_nnz, P.no_empty, rows_per_lane, pad_loads, load_policy);
        int64_t max_group = 0;
        for (size_t g = 0; g + 1 < L.gp.size(); g++) max_group = std::max(max_group, L.group_end(g) - L.gp[g]);
        if (max_group * std::max(L.esz, 4) >= (int64_t(1) << 32))
            fail(RGCSR_EOVERFLOW, "a row group holds 4 GiB or more; use a long-row threshold");
        Arena a;
        a.add(&h->gp, (size_t)L.ng + 1);
        a.add(&h->short_len, (size_t)L.ns);
        a.add(&h->short_row, h->perm ? (size_t)L.ns : 0);
        a.add((uint8_t **)&h->slot_val, (size_t)L.slots * L.esz);
        a.add(&h->slot_col, (size_t)L.slots);
        a.add(&h->short_items, h->items.size());
        a.add(&h->wave_work, L.work.wave.size());
        a.add(&h->block_work, L.work.block.size());
        a.add(&h->combine, L.work.combine.size());
        a.add(&h->long_row, (size_t)L.nl);
        a.add(&h->long_ptr, (size_t)L.nl + 1);
        a.add((uint8_t **)&h->long_val, (size_t)L.long_nnz * L.esz);
        a.add(&h->long_col, (size_t)L.long_nnz);
        a.add((uint8_t **)&h->partial, (size_t)L.work.n_partials * 32 * sizeof(double));
        if (keep_map) a.add(&h->row_ptr, (size_t)P.n_rows + 1);
        h->mem = a.commit();
        h->bytes = a.total;
        device_fill(P, p, rp, col, vals, vals_dt, vdt, h->gp, h->short_len, h->perm ? h->short_row : nullptr,
                    h->slot_val, h->slot_col, h->long_row, h->long_ptr, h->long_val, h->long_col, st);
        upload(h->short_items, h->items, st);
        upload(h->wave_work, L.work.wave, st);
        upload(h->block_work, L.work.block, st);
        upload(h->combine, L.work.combine, st);
        if (keep_map)
            HIPCHK(hipMemcpyAsync(h->row_ptr, rp, ((size_t)P.n_rows + 1) * 8, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        // column tiles from the converted long-row segment: its columns come
        // back to the host, the tile arrays go to a block of their own
        if (tile_min_len != 0 && L.nl > 0) {
            L.nl = P.nl;
            L.long_ptr = P.long_ptr_host;
            L.long_col.resize((size_t)L.long_nnz);
            L.long_row.resize((size_t)L.nl);
            if (L.long_nnz)
                HIPCHK(hipMemcpyAsync(L.long_col.data(), h->long_col, (size_t)L.long_nnz * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(L.long_row.data(), h->long_row, (size_t)L.nl * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            HostTiles T;
            build_tiles(L, tile_min_len, T);
            Arena ta;
            add_tile_arrays(h, T, ta);
            if (T.active()) {
                h->tile_mem = ta.commit();
                h->tile_bytes = ta.total;
                upload_tiles(h, T, L.long_row, st);
            }
        }
    } catch (...) {
        (void)hipStreamSynchronize(st);
        if (h->mem) (void)hipFree(h->mem);
        if (h->tile_mem) (void)hipFree(h->tile_mem);
        delete h;
        throw;
    }
    return h;
}

void free_handle(rgcsr_matrix_s *h) {
    if (!h) return;
    if (h->AT) free_handle(h->AT);
    if (h->PN) free_handle(h->PN);
    if (h->mem && h->owns_mem) (void)hipFree(h->mem);
    if (h->tile_mem) (void)hipFree(h->tile_mem);
    delete h;
}

// Device memory that freeing the handle releases (none for a handle built
// into caller memory: its transpose sits in the same block).
bool owns_device_memory(const rgcsr_matrix_s *h) {
    return h && ((h->mem && h->owns_mem) || h->tile_mem || owns_device_memory(h->AT) || owns_device_memory(h->PN));
}

void check_handle(const rgcsr_matrix_s *h) {
    if (!h) fail(RGCSR_EINVAL, "null handle");
    if (current_device() != h->device) fail(RGCSR_EINVAL, "handle belongs to another device");
}

int32_t short_waves(const rgcsr_matrix_s *h, bool scheduled) {
    int64_t w = h->wpg > 0 ? h->ng * h->wpg : (h->ng + h->gpw - 1) / h->gpw;
    if (scheduled) w = h->R == 0 ? (int64_t)h->items.size() : (w + h->R - 1) / h->R;
    if (w > INT32_MAX / 2) fail(RGCSR_EOVERFLOW, "too many wavefronts");
    return (int32_t)w;
}

// Workgroup -> unit table of a panel copy.  Units are formed as params_of
// forms them (block items, then wavefront items four to a unit); each unit
// belongs to the panel of its first item.  The hardware deals workgroup b to
// XCD b % 8, so panel q's units go to the workgroups b with b % 8 == q * 8 / P
// in unit order (long-row units first, as in every launch); the units of the
// whole rows (index P) are dealt to the XCDs in turn, after the panels' own;
// -1 fills the tail of XCDs with fewer units than the busiest one.
std::vector<int32_t> panel_unit_map(const rgcsr_matrix_s *h, const HostLayout &L, const PanelBuilt &pb,
                                    bool use_rows) {
    const int64_t n_block = h->n_block, n_wave_long = h->n_wave_long;
    const int64_t sw = short_waves(h, use_rows);
    const int64_t units = n_block + (n_wave_long + sw + kBlockWaves - 1) / kBlockWaves;
    auto panel_in = [](const std::vector<int64_t> &off, int64_t i) {
        return (int32_t)(std::upper_bound(off.begin() + 1, off.end(), i) - (off.begin() + 1));
    };
    const int32_t R = use_rows ? h->R : 1;
    std::vector<std::vector<int32_t>> per(kPanelXcds), whole(kPanelXcds);
    int64_t n_whole = 0;
    for (int64_t u = 0; u < units; u++) {
        int32_t q;
        if (u < n_block) {
            q = panel_in(pb.long_off, L.work.block[u].a);
        } else {
            const int64_t w = (u - n_block) * kBlockWaves;
            if (w < n_wave_long) {
                q = panel_in(pb.long_off, L.work.wave[w].a);
            } else {
                // first row group of short wavefront s (as spmv_short reads it)
                const int64_t s = w - n_wave_long;
                int64_t g;
                if (h->wpg > 0)
                    g = (R == 0 ? (int64_t)(h->items[s] >> 2) : s * R) / h->wpg;
                else
                    g = s * h->gpw;
                q = panel_in(pb.grp_off, g);
            }
        }
        if (q < pb.P)
            per[(size_t)q * kPanelXcds / pb.P].push_back((int32_t)u);
        else
            whole[n_whole++ % kPanelXcds].push_back((int32_t)u);
    }
    for (int x = 0; x < kPanelXcds; x++) per[x].insert(per[x].end(), whole[x].begin(), whole[x].end());
    size_t longest = 0;
    for (auto &v : per) longest = std::max(longest, v.size());
    if (longest * kPanelXcds > (size_t)INT32_MAX / 2) fail(RGCSR_EOVERFLOW, "too many workgroups");
    std::vector<int32_t> map(longest * kPanelXcds, -1);
    for (int x = 0; x < kPanelXcds; x++)
        for (size_t j = 0; j < per[x].size(); j++) map[j * kPanelXcds + x] = per[x][j];
    return map;
}

// use_rows: the launch uses the handle's rows-per-lane schedule (single
// right-hand side); otherwise one row per lane.  tiled: the tile kernel has
// written the partial sums of the column-tiled rows, so the long-row work
// covers the other long rows and the first wavefront items add the partials.
SpmvParams params_of(const rgcsr_matrix_s *h, bool use_rows, bool tiled = false) {
    SpmvParams P{};
    P.gp = h->gp; P.gend = h->gend; P.grp_row0 = h->grp_row0; P.short_len = h->short_len; P.short_row = h->short_row;
    P.slot_val = h->slot_val; P.slot_col = h->slot_col;
    P.ng = h->ng; P.ns = h->ns; P.G = h->prm.G; P.wpg = h->wpg; P.gpw = h->gpw;
    P.ragged = h->ragged; P.perm = h->perm; P.pad = h->pad;
    P.short_items = h->short_items;
    P.wave_work = h->wave_work; P.block_work = h->block_work;
    P.long_row = h->long_row; P.long_ptr = h->long_ptr; P.long_val = h->long_val;
    P.long_col = h->long_col; P.partial = h->partial;
    P.tile_dst = h->n_tent ? h->tile_dst : nullptr;
    P.tile_vals = h->n_tent ? h->tile_val : nullptr;
    int64_t n_block = h->n_block, n_wave_long = h->n_wave_long, n_comb = 0;
    if (tiled) {
        P.wave_work = h->rest_wave;
        P.block_work = h->rest_block;
        n_block = h->n_rest_block;
        n_wave_long = h->n_rest_wave;
        n_comb = (h->n_trows + 63) / 64;
        P.tile_partial = h->tile_partial;
        P.tile_orow = h->tile_orow;
        P.n_comb_units = (int32_t)n_comb;
        P.n_tiles = (int32_t)h->n_tiles;
        P.n_trows = (int32_t)h->n_trows;
    }
    const int64_t sw = short_waves(h, use_rows);
    const int64_t wave_items = n_wave_long + sw;
    const int64_t units = n_comb + n_block + (wave_items + kBlockWaves - 1) / kBlockWaves;
    const int64_t tot = h->nl + short_waves(h, false);
    if (wave_items > INT32_MAX / 2 || units > INT32_MAX / 2 || tot > INT32_MAX / 2)
        fail(RGCSR_EOVERFLOW, "too many wavefronts");
    P.n_block_items = (int32_t)n_block;
    P.n_wave_long = (int32_t)n_wave_long;
    P.n_wave_items = (int32_t)wave_items;
    P.total_units = (int32_t)units;
    P.n_long_units = (int32_t)(n_comb + n_block + (n_wave_long + kBlockWaves - 1) / kBlockWaves);
    P.n_long_waves = (int32_t)h->nl;
    P.total_waves = (int32_t)tot;
    return P;
}

int vec_is_f64(rgcsr_dtype vt) {
    if (vt == RGCSR_F64) return 1;
    if (vt == RGCSR_F32) return 0;
    fail(RGCSR_EUNSUPPORTED, "vectors must be F32 or F64");
}

// The panel copy serves launches of several right-hand sides whose
// per-piece sums fit the buffer (K accumulators of kPanelRowBytes at most)
// and whose X slice per panel (panel columns times the X row stride) fits
// kPanelSliceBytes.  One vector stays on the layout, whose column tiles
// keep the long rows' x in LDS (and whose kernels store without the
// per-piece output codes).
bool panel_slice_ok(const rgcsr_matrix_s *h, int64_t ldx, int f64) {
    return h->PN && h->PN->panel_cols * ldx * (f64 ? 8 : 4) <= kPanelSliceBytes;
}
bool panel_launch_ok(const rgcsr_matrix_s *h, int K, int64_t ldx, int f64) {
    return K > 1 && panel_slice_ok(h, ldx, f64) && K * (f64 ? 8 : 4) <= kPanelRowBytes;
}

void spmv_launch(const rgcsr_matrix_s *h, int K, const void *X, int64_t ldx, void *Y, int64_t ldy, int f64,
                 bool persistent, hipStream_t st) {
    if (h->n_rows == 0) return;
    const bool panels = panel_launch_ok(h, K, ldx, f64);
    const rgcsr_matrix_s *pn = h->PN;
    // the column-tiled rows take one vector with unit stride (FP64 for F64
    // storage, FP32 otherwise) and the default load policy; everything else
    // runs them on the long-row path
    const bool tiled = !panels && h->n_trows > 0 && K == 1 && (f64 != 0) == (h->vdt == RGCSR_F64) && ldx == 1 &&
                       h->lp == 0;
    // right-hand sides of up to kRunsRowBytes per row take the runs of rows
    // per lane (R = 0) when the handle has them; otherwise one row per lane
    const rgcsr_matrix_s *src = panels ? pn : h;
    const bool rows = K == 1 || (K * (f64 ? 8 : 4) <= kRunsRowBytes && src->R == 0);
    const int32_t R = K == 1 ? src->R : (rows ? 0 : 1);
    SpmvParams P = params_of(src, rows, tiled);
    P.x = X; P.y = Y; P.ldx = ldx; P.ldy = ldy;
    int64_t nwg = P.total_units;
    if (panels) {
        // pieces of panel q on XCD q * 8 / P, their sums to the piece buffer
        P.unit_map = rows ? pn->unit_map_rows : pn->unit_map_one;
        P.n_map = rows ? pn->n_map_rows : pn->n_map_one;
        P.pan_y = pn->pan_y;
        P.pan_ld = K;
        nwg = P.n_map;
    }
    // a persistent launch (several right-hand sides only) keeps two 256-thread
    // workgroups per CU that stride over the units (a multiple of 8, so a
    // workgroup stays on the XCD of its table entries)
    if (persistent && K > 1) nwg = std::min<int64_t>(nwg, (int64_t)cu_count(h->device) * 2);
    if (nwg == 0 && !panels) return;
    const int vd = h->vdt;
    if (f64 && !(vd == RGCSR_F64 || vd == RGCSR_F32))
        fail(RGCSR_EUNSUPPORTED, "F64 vectors need F64 or F32 stored values");
    if (!f64 && vd == RGCSR_F64) fail(RGCSR_EUNSUPPORTED, "F64 stored values need F64 vectors");
    if (K > 1 && (vd == RGCSR_F16 || vd == RGCSR_BF16))
        fail(RGCSR_EUNSUPPORTED, "several right-hand sides need F32 or F64 stored values");
    if (K > 1 && h->prm.T != 1) fail(RGCSR_EUNSUPPORTED, "several right-hand sides need lanes_per_row = 1");
    if (K == 1 && h->n_cols * ldx * (f64 ? 8 : 4) >= (int64_t(1) << 32))
        fail(RGCSR_EUNSUPPORTED, "x (n_cols * ldx elements) of 4 GiB or more");
    if (K == 1 && h->lp != 0 && f64) fail(RGCSR_EUNSUPPORTED, "load policies 1 and 2 need F32 vectors");
    hipError_t e = hipSuccess;
    if (panels) {
        if (nwg > 0) {
            e = launch_spmv(P, vd, f64, pn->prm.T, K, R, K == 1 ? pn->lp : 0, (int)nwg, st);
            if (e != hipSuccess) fail(RGCSR_EHIP, std::string("spmv launch: ") + hipGetErrorString(e));
        }
        if (pn->n_combine) {
            e = launch_combine(pn->combine, (int32_t)pn->n_combine, pn->long_row, pn->partial, Y, ldy, pn->pan_y, K,
                               f64, K, st);
            if (e != hipSuccess) fail(RGCSR_EHIP, std::string("combine launch: ") + hipGetErrorString(e));
        }
        e = launch_panel_combine(pn->pan_crow, pn->pan_cptr, pn->n_split, pn->pan_vidx, pn->pan_y, Y, ldy, f64, K, st);
        if (e != hipSuccess) fail(RGCSR_EHIP, std::string("panel combine launch: ") + hipGetErrorString(e));
        return;
    }
    if (tiled) {
        TileParams TP{};
        TP.units = h->tile_units;
        TP.ptr = h->tile_ptr;
        TP.lcol = h->tile_lcol;
        TP.val = h->tile_val;
        TP.x = X;
        TP.partial = h->tile_partial;
        TP.n_cols = h->n_cols;
        TP.n_trows = (int32_t)h->n_trows;
        TP.x_aligned = ((uintptr_t)X % 16) == 0;
        e = launch_tile_spmv(TP, vd, (int)h->n_tunits, st);
        if (e != hipSuccess) fail(RGCSR_EHIP, std::string("tile launch: ") + hipGetErrorString(e));
    }
    e = launch_spmv(P, vd, f64, h->prm.T, K, R, K == 1 ? h->lp : 0, (int)nwg, st);
    if (e != hipSuccess) fail(RGCSR_EHIP, std::string("spmv launch: ") + hipGetErrorString(e));
    const int64_t n_comb = tiled ? h->n_rest_combine : h->n_combine;
    if (n_comb) {
        e = launch_combine(tiled ? h->rest_combine : h->combine, (int32_t)n_comb, h->long_row, h->partial, Y, ldy,
                           nullptr, 0, f64, K, st);
        if (e != hipSuccess) fail(RGCSR_EHIP, std::string("combine launch: ") + hipGetErrorString(e));
    }
}

// CG vector kernels: up to 2,048 workgroups (eight per CU), each lane taking
// at least four elements; the partial-sum count is fixed by n, so the
// reductions are deterministic
int64_t nblocks_vec(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>(2048, (n + 1023) / 1024)); }

}  // namespace

extern "C" {

rgcsr_status rgcsr_gather_floor(const int32_t *col, const float *val, int64_t n, const float *x, int64_t n_cols,
                                float *out, void *stream) {
    ABI_TRY
    if (n < 0 || (n > 0 && (!col || !val || !x || !out))) fail(RGCSR_EINVAL, "bad argument");
    if ((n + 7) / 8 / 256 >= INT32_MAX) fail(RGCSR_EOVERFLOW, "too many entries");
    (void)n_cols;
    HIPCHK(launch_gather_floor(col, val, n, x, out, (hipStream_t)stream));
    ABI_CATCH
}

rgcsr_status rgcsr_stream_read(const void *buf, int64_t bytes, void *sink, void *stream) {
    ABI_TRY
    if (!buf || !sink || bytes < 0) fail(RGCSR_EINVAL, "buf and sink must be device pointers, bytes >= 0");
    if (bytes % 16 != 0 || (uintptr_t)buf % 16 != 0 || (uintptr_t)sink % 4 != 0)
        fail(RGCSR_EINVAL, "buf must be 16-byte aligned with bytes a multiple of 16, sink 4-byte aligned");
    // eight 256-thread workgroups per CU stride over the buffer
    const int nb = (int)std::min<int64_t>(std::max<int64_t>(1, bytes / 4096), (int64_t)cu_count(current_device()) * 8);
    HIPCHK(launch_stream_read(buf, bytes / 16, (int32_t *)sink, nb, (hipStream_t)stream));
    ABI_CATCH
}

rgcsr_status rgcsr_from_csr(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                            const int32_t *col_idx, const void *vals, rgcsr_dtype vals_dtype,
                            const rgcsr_opts *opts, int inputs_on_device, void *stream, rgcsr_handle *out) {
    ABI_TRY
    if (!out) fail(RGCSR_EINVAL, "out is null");
    *out = nullptr;
    rgcsr_opts o;
    if (opts) o = *opts; else rgcsr_default_opts(&o);
    const LayoutParams p = resolve_opts(&o);
    check_device_geometry(p);
    check_dtype(o.value_dtype, "value_dtype");
    check_dtype(vals_dtype, "vals");
    if (n_rows < 0 || n_cols < 0 || nnz < 0) fail(RGCSR_EINVAL, "negative size");
    check_panels(o.col_panels);
    if (o.col_panels && o.value_dtype != RGCSR_F32 && o.value_dtype != RGCSR_F64)
        fail(RGCSR_EUNSUPPORTED, "col_panels serves several right-hand sides, which need F32 or F64 stored values");
    hipStream_t st = (hipStream_t)stream;
    std::vector<int64_t> h_rp;
    std::vector<int32_t> h_col;
    std::vector<uint8_t> h_val;
    const int64_t *rp = row_ptr;
    const int32_t *col = col_idx;
    const void *val = vals;
    if (inputs_on_device && !o.build_transpose && !o.col_panels) {
        // conversion on the device; device inputs are always validated
        DevPlan P;
        P.scratch.st = st;
        device_plan(P, p, n_rows, n_cols, nnz, row_ptr, col_idx, true, st);
        *out = make_device_on_device(P, p, o.value_dtype, row_ptr, col_idx, vals, vals_dtype, o.keep_csr_map != 0, st,
                                     o.rows_per_lane, o.pad_loads, o.load_policy, o.tile_min_len);
        return RGCSR_OK;
    }
    if (inputs_on_device) {
        if (!row_ptr) fail(RGCSR_EINVAL, "row_ptr is null");
        h_rp.resize(n_rows + 1);
        h_col.resize(nnz);
        h_val.resize((size_t)nnz * dtype_size(vals_dtype));
        HIPCHK(hipMemcpyAsync(h_rp.data(), row_ptr, (n_rows + 1) * 8, hipMemcpyDeviceToHost, st));
        if (nnz) {
            HIPCHK(hipMemcpyAsync(h_col.data(), col_idx, nnz * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(h_val.data(), vals, h_val.size(), hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        rp = h_rp.data();
        col = h_col.data();
        val = h_val.data();
    }
    if (!rp) fail(RGCSR_EINVAL, "row_ptr is null");
    if (!o.validate && rp[n_rows] != nnz) fail(RGCSR_ECSR, "row_ptr[n_rows] != nnz");
    Built B;
    const bool keep = o.keep_csr_map != 0, tr = o.build_transpose != 0;
    build_host(B, p, o.value_dtype, 1, &n_rows, &n_cols, &rp, &col, &val, vals_dtype, o.validate != 0, keep, tr);
    rgcsr_matrix_s *h = make_device(B.L, (keep || tr) ? &B.row_ptr : nullptr, nullptr, st, o.rows_per_lane,
                                    o.pad_loads, o.load_policy, o.tile_min_len);
    try {
        if (tr)
            h->AT = make_device(B.LT, nullptr, &B.LTmap, st, o.rows_per_lane, o.pad_loads, o.load_policy,
                                o.tile_min_len);
        if (o.col_panels) {
            // the panel copy holds the values in the storage dtype; set_values
            // refreshes it through its element -> CSR index map
            const int64_t esz = dtype_size(o.value_dtype);
            std::vector<uint8_t> conv((size_t)rp[n_rows] * esz);
            if (rp[n_rows]) convert_values(val, vals_dtype, conv.data(), o.value_dtype, rp[n_rows]);
            PanelBuilt pb;
            // rows up to the long-row threshold stay whole (all rows are
            // split when there is none)
            build_panels(pb, p, o.value_dtype, o.col_panels, p.tau, n_rows, n_cols, rp, col, conv.data());
            h->n_panels = o.col_panels;
            h->PN = make_device(pb.LP, nullptr, &pb.LPmap, st, o.rows_per_lane, o.pad_loads, o.load_policy, 0, &pb);
        }
    } catch (...) {
        free_handle(h);
        throw;
    }
    *out = h;
    ABI_CATCH
}

}  // extern "C"

namespace {

// Host conversion of one matrix or a block-diagonal batch into a plan.
rgcsr_plan plan_of(int32_t count, const int64_t *n_rows, const int64_t *n_cols, const int64_t *const *row_ptr,
                   const int32_t *const *col_idx, const void *const *vals, rgcsr_dtype vals_dtype,
                   const rgcsr_opts *opts) {
    rgcsr_opts o;
    if (opts) o = *opts; else rgcsr_default_opts(&o);
    const LayoutParams p = resolve_opts(&o);
    check_device_geometry(p);
    check_dtype(o.value_dtype, "value_dtype");
    check_dtype(vals_dtype, "vals");
    check_panels(o.col_panels);
    if (o.col_panels) fail(RGCSR_EUNSUPPORTED, "col_panels needs rgcsr_from_csr");
    std::unique_ptr<rgcsr_plan_s> P(new rgcsr_plan_s());
    P->with_row_ptr = o.keep_csr_map != 0 || o.build_transpose != 0;
    const bool tr = o.build_transpose != 0;
    build_host(P->B, p, o.value_dtype, count, n_rows, n_cols, row_ptr, col_idx, vals, vals_dtype, o.validate != 0,
               o.keep_csr_map != 0, tr);
    P->h = prepare_handle(P->B.L, P->with_row_ptr, nullptr, P->a, o.rows_per_lane, o.pad_loads, o.load_policy,
                          o.tile_min_len);
    if (tr)
        P->hT = prepare_handle(P->B.LT, false, &P->B.LTmap, P->aT, o.rows_per_lane, o.pad_loads, o.load_policy,
                               o.tile_min_len);
    return P.release();
}

}  // namespace

extern "C" {

rgcsr_status rgcsr_plan_from_csr(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                                 const int32_t *col_idx, const void *vals, rgcsr_dtype vals_dtype,
                                 const rgcsr_opts *opts, rgcsr_plan *out) {
    ABI_TRY
    if (!out) fail(RGCSR_EINVAL, "out is null");
    *out = nullptr;
    if (n_rows < 0 || n_cols < 0 || nnz < 0) fail(RGCSR_EINVAL, "negative size");
    if (!row_ptr) fail(RGCSR_EINVAL, "row_ptr is null");
    if (!(opts ? opts->validate : 1) && row_ptr[n_rows] != nnz) fail(RGCSR_ECSR, "row_ptr[n_rows] != nnz");
    *out = plan_of(1, &n_rows, &n_cols, &row_ptr, &col_idx, &vals, vals_dtype, opts);
    ABI_CATCH
}

rgcsr_status rgcsr_plan_from_csr_batch(int32_t count, const int64_t *n_rows, const int64_t *n_cols,
                                       const int64_t *const *row_ptr, const int32_t *const *col_idx,
                                       const void *const *vals, rgcsr_dtype vals_dtype, const rgcsr_opts *opts,
                                       rgcsr_plan *out) {
    ABI_TRY
    if (!out) fail(RGCSR_EINVAL, "out is null");
    *out = nullptr;
    if (count < 1 || !n_rows || !n_cols || !row_ptr || !col_idx || !vals) fail(RGCSR_EINVAL, "bad batch arrays");
    *out = plan_of(count, n_rows, n_cols, row_ptr, col_idx, vals, vals_dtype, opts);
    ABI_CATCH
}

rgcsr_status rgcsr_plan_device_bytes(rgcsr_plan plan, int64_t *bytes) {
    ABI_TRY
    if (!plan || !bytes) fail(RGCSR_EINVAL, "null argument");
    if (!plan->h) fail(RGCSR_EINVAL, "the plan has been built already");
    *bytes = (int64_t)(plan->a.total + plan->aT.total);
    ABI_CATCH
}

rgcsr_status rgcsr_build(rgcsr_plan plan, void *device_buf, int64_t buf_bytes, void *stream, rgcsr_handle *out) {
    ABI_TRY
    if (!plan || !out) fail(RGCSR_EINVAL, "null argument");
    *out = nullptr;
    if (!plan->h) fail(RGCSR_EINVAL, "the plan has been built already");
    const size_t total = plan->a.total + plan->aT.total;
    if (device_buf) {
        if (buf_bytes < 0 || (size_t)buf_bytes < total) fail(RGCSR_EINVAL, "device buffer smaller than the plan's device bytes");
        if ((uintptr_t)device_buf % 256) fail(RGCSR_EINVAL, "device buffer not 256-byte aligned");
    }
    hipStream_t st = (hipStream_t)stream;
    // the plan gives up its prepared handles whether or not the build succeeds
    rgcsr_matrix_s *h = plan->h, *hT = plan->hT;
    plan->h = plan->hT = nullptr;
    auto drop = [&](rgcsr_matrix_s *x) {
        if (!x) return;
        if (x->mem && x->owns_mem) (void)hipFree(x->mem);
        delete x;
    };
    try {
        place_and_upload(h, plan->a, plan->B.L, plan->with_row_ptr ? &plan->B.row_ptr : nullptr, nullptr, device_buf, st);
        if (hT) {
            void *bufT = device_buf ? (void *)((char *)device_buf + plan->a.total) : nullptr;
            place_and_upload(hT, plan->aT, plan->B.LT, nullptr, &plan->B.LTmap, bufT, st);
        }
    } catch (...) {
        (void)hipStreamSynchronize(st);
        drop(hT);
        drop(h);
        throw;
    }
    h->AT = hT;
    plan->B = Built();
    *out = h;
    ABI_CATCH
}

rgcsr_status rgcsr_plan_destroy(rgcsr_plan plan) {
    ABI_TRY
    delete plan;
    ABI_CATCH
}

rgcsr_status rgcsr_from_csr_batch(int32_t count, const int64_t *n_rows, const int64_t *n_cols,
                                  const int64_t *const *row_ptr, const int32_t *const *col_idx,
                                  const void *const *vals, rgcsr_dtype vals_dtype, const rgcsr_opts *opts,
                                  void *stream, rgcsr_handle *out) {
    ABI_TRY
    if (!out) fail(RGCSR_EINVAL, "out is null");
    *out = nullptr;
    if (count < 1 || !n_rows || !n_cols || !row_ptr || !col_idx || !vals) fail(RGCSR_EINVAL, "bad batch arrays");
    rgcsr_opts o;
    if (opts) o = *opts; else rgcsr_default_opts(&o);
    const LayoutParams p = resolve_opts(&o);
    check_device_geometry(p);
    check_dtype(o.value_dtype, "value_dtype");
    check_dtype(vals_dtype, "vals");
    check_panels(o.col_panels);
    if (o.col_panels) fail(RGCSR_EUNSUPPORTED, "col_panels needs rgcsr_from_csr (one matrix)");
    hipStream_t st = (hipStream_t)stream;
    Built B;
    const bool keep = o.keep_csr_map != 0, tr = o.build_transpose != 0;
    build_host(B, p, o.value_dtype, count, n_rows, n_cols, row_ptr, col_idx, vals, vals_dtype, o.validate != 0,
               keep, tr);
    rgcsr_matrix_s *h = make_device(B.L, (keep || tr) ? &B.row_ptr : nullptr, nullptr, st, o.rows_per_lane,
                                    o.pad_loads, o.load_policy, o.tile_min_len);
    if (tr) {
        try {
            h->AT = make_device(B.LT, nullptr, &B.LTmap, st, o.rows_per_lane, o.pad_loads, o.load_policy,
                                o.tile_min_len);
        } catch (...) {
            free_handle(h);
            throw;
        }
    }
    *out = h;
    ABI_CATCH
}

rgcsr_status rgcsr_batch_offsets(rgcsr_handle A, int64_t *row_off, int64_t *col_off) {
    ABI_TRY
    if (!A) fail(RGCSR_EINVAL, "null handle");
    if (row_off) std::copy(A->row_off.begin(), A->row_off.end(), row_off);
    if (col_off) std::copy(A->col_off.begin(), A->col_off.end(), col_off);
    ABI_CATCH
}

rgcsr_status rgcsr_spmv(rgcsr_handle A, const void *x, void *y, rgcsr_dtype vec_dtype, void *stream) {
    ABI_TRY
    check_handle(A);
    if ((!x && A->n_cols) || (!y && A->n_rows)) fail(RGCSR_EINVAL, "null vector");
    const int f64 = vec_is_f64(vec_dtype);
    spmv_launch(A, 1, x, 1, y, 1, f64, false, (hipStream_t)stream);
    ABI_CATCH
}

rgcsr_status rgcsr_spmv_batched(rgcsr_handle A, int32_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                                rgcsr_dtype vec_dtype, int32_t persistent, void *stream) {
    ABI_TRY
    check_handle(A);
    if (k < 1) fail(RGCSR_EINVAL, "k must be >= 1");
    if (ldx < k || ldy < k) fail(RGCSR_EINVAL, "ldx and ldy must be >= k");
    if ((!X && A->n_cols) || (!Y && A->n_rows)) fail(RGCSR_EINVAL, "null vector");
    const int f64 = vec_is_f64(vec_dtype);
    const int esz = f64 ? 8 : 4, vw = f64 ? 2 : 4;
    // Column blocks of 32, 16, 8, 4, 2, 1.  Blocks whose width is a multiple of
    // the 16-byte vector width read X and Y rows with vector accesses, which
    // needs 16-byte aligned rows; otherwise narrower blocks (scalar accesses)
    // are used.
    const bool aligned = ((uintptr_t)X % 16 == 0) && ((uintptr_t)Y % 16 == 0) && (ldx % vw == 0) && (ldy % vw == 0);
    // the multi-column kernels take one lane per row and F32/F64 values;
    // other handles run one single-column launch per column (strided x, y)
    const bool blocks = A->prm.T == 1 && (A->vdt == RGCSR_F32 || A->vdt == RGCSR_F64);
    // a panel copy takes column blocks whose sums fit its piece buffer
    const int32_t kmax = panel_slice_ok(A, ldx, f64) ? kPanelRowBytes / esz : 32;
    int32_t done = 0;
    while (done < k) {
        int32_t kb = 1;
        for (int32_t c : {32, 16, 8, 4, 2, 1}) {
            if (!blocks) break;
            if (c > k - done || c > kmax) continue;
            if (c % vw == 0 && (!aligned || ((size_t)done * esz) % 16 != 0)) continue;
            kb = c;
            break;
        }
        const char *xp = (const char *)X + (size_t)done * esz;
        char *yp = (char *)Y + (size_t)done * esz;
        spmv_launch(A, kb, xp, ldx, yp, ldy, f64, persistent != 0, (hipStream_t)stream);
        done += kb;
    }
    ABI_CATCH
}

rgcsr_status rgcsr_spmv_transpose_grad(rgcsr_handle A, const void *x, const void *dy, void *dx, void *dvals,
                                       rgcsr_dtype vec_dtype, void *stream) {
    ABI_TRY
    check_handle(A);
    const int f64 = vec_is_f64(vec_dtype);
    hipStream_t st = (hipStream_t)stream;
    if (!dy && A->n_rows) fail(RGCSR_EINVAL, "dy is null");
    if (dvals && !A->row_ptr) fail(RGCSR_EUNSUPPORTED, "dvals needs keep_csr_map or build_transpose");
    if (dvals && !x && A->n_cols) fail(RGCSR_EINVAL, "x is null");
    if (A->vdt == RGCSR_F64 && !f64) fail(RGCSR_EUNSUPPORTED, "F64 stored values need F64 vectors");
    if (f64 && (A->vdt == RGCSR_F16 || A->vdt == RGCSR_BF16)) fail(RGCSR_EUNSUPPORTED, "F64 vectors need F32/F64 values");
    const bool atomic_dx = dx && !A->AT;
    if (dx && A->AT) spmv_launch(A->AT, 1, dy, 1, dx, 1, f64, false, st);
    if (atomic_dx) {
        hipError_t e = launch_zero(A->n_cols, dx, f64 ? 8 : 4, (int)nblocks_vec(A->n_cols), st);
        if (e != hipSuccess) fail(RGCSR_EHIP, hipGetErrorString(e));
    }
    if ((dvals || atomic_dx) && A->n_rows) {
        SpmvParams P = params_of(A, true);
        P.x = x;
        hipError_t e = launch_grad(P, A->vdt, f64, A->prm.T, dy, dvals, dx, A->row_ptr, dvals != nullptr, atomic_dx, st);
        if (e != hipSuccess) fail(RGCSR_EHIP, std::string("grad launch: ") + hipGetErrorString(e));
    }
    ABI_CATCH
}

rgcsr_status rgcsr_set_values(rgcsr_handle A, const void *vals, rgcsr_dtype vals_dtype, int on_device,
                              void *stream) {
    ABI_TRY
    check_handle(A);
    if (!A->row_ptr) fail(RGCSR_EUNSUPPORTED, "set_values needs keep_csr_map or build_transpose");
    if (!vals && A->nnz) fail(RGCSR_EINVAL, "vals is null");
    hipStream_t st = (hipStream_t)stream;
    const void *theta = vals;
    int theta_f64 = 0;
    void *tmp = nullptr;
    if (!on_device || (vals_dtype != RGCSR_F32 && vals_dtype != RGCSR_F64)) {
        if (on_device) fail(RGCSR_EUNSUPPORTED, "device values must be F32 or F64");
        const int tdt = vals_dtype == RGCSR_F64 ? RGCSR_F64 : RGCSR_F32;
        std::vector<uint8_t> conv((size_t)A->nnz * dtype_size(tdt));
        convert_values(vals, vals_dtype, conv.data(), tdt, A->nnz);
        HIPCHK(hipMalloc(&tmp, std::max<size_t>(conv.size(), 1)));
        HIPCHK(hipMemcpyAsync(tmp, conv.data(), conv.size(), hipMemcpyHostToDevice, st));
        theta = tmp;
        theta_f64 = tdt == RGCSR_F64;
    } else {
        theta_f64 = vals_dtype == RGCSR_F64;
    }
    try {
        if (A->n_rows) {
            SpmvParams P = params_of(A, true);
            hipError_t e = launch_setval(P, A->vdt, A->prm.T, theta, theta_f64, A->row_ptr, st);
            if (e != hipSuccess) fail(RGCSR_EHIP, std::string("set_values: ") + hipGetErrorString(e));
        }
        if (A->AT) {
            hipError_t e = launch_gather_map(A->AT->slots, A->vdt, A->AT->t_map_slot, theta, theta_f64, A->AT->slot_val, st);
            if (e == hipSuccess)
                e = launch_gather_map(A->AT->long_nnz, A->vdt, A->AT->t_map_long, theta, theta_f64, A->AT->long_val, st);
            if (e == hipSuccess && A->AT->n_tent)
                e = launch_tile_values(A->AT->long_nnz, A->AT->tile_dst, A->AT->long_val, A->AT->tile_val, A->esz, st);
            if (e != hipSuccess) fail(RGCSR_EHIP, std::string("set_values (transpose): ") + hipGetErrorString(e));
        }
        if (A->PN) {
            hipError_t e = launch_gather_map(A->PN->slots, A->vdt, A->PN->t_map_slot, theta, theta_f64, A->PN->slot_val, st);
            if (e == hipSuccess)
                e = launch_gather_map(A->PN->long_nnz, A->vdt, A->PN->t_map_long, theta, theta_f64, A->PN->long_val, st);
            if (e != hipSuccess) fail(RGCSR_EHIP, std::string("set_values (panels): ") + hipGetErrorString(e));
        }
        if (tmp) {
            HIPCHK(hipStreamSynchronize(st));
            HIPCHK(hipFree(tmp));
            tmp = nullptr;
        }
    } catch (...) {
        if (tmp) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(tmp);
        }
        throw;
    }
    ABI_CATCH
}

rgcsr_status rgcsr_export(rgcsr_handle A, void *stream, int64_t *gp, int32_t *short_len, int32_t *short_row,
                          void *slot_val, int32_t *slot_col, int32_t *long_row, int64_t *long_ptr, void *long_val,
                          int32_t *long_col) {
    ABI_TRY
    check_handle(A);
    hipStream_t st = (hipStream_t)stream;
    auto get = [&](void *dst, const void *src, size_t bytes) {
        if (dst && src && bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    };
    get(gp, A->gp, (A->ng + 1) * 8);
    get(short_len, A->short_len, A->ns * 4);
    if (short_row) {
        if (A->perm) get(short_row, A->short_row, A->ns * 4);
        else
            for (int64_t i = 0; i < A->ns; i++) short_row[i] = (int32_t)i;
    }
    get(slot_val, A->slot_val, (size_t)A->slots * A->esz);
    get(slot_col, A->slot_col, (size_t)A->slots * 4);
    get(long_row, A->long_row, A->nl * 4);
    get(long_ptr, A->long_ptr, (A->nl + 1) * 8);
    get(long_val, A->long_val, (size_t)A->long_nnz * A->esz);
    get(long_col, A->long_col, (size_t)A->long_nnz * 4);
    HIPCHK(hipStreamSynchronize(st));
    ABI_CATCH
}

rgcsr_status rgcsr_to_csr(rgcsr_handle A, void *stream, int64_t *row_ptr, int32_t *col_idx, void *vals) {
    ABI_TRY
    check_handle(A);
    if (!row_ptr || (A->nnz && (!col_idx || !vals))) fail(RGCSR_EINVAL, "null output");
    const int esz = A->esz;
    std::vector<int64_t> gp(A->ng + 1), lp(A->nl + 1);
    std::vector<int32_t> sl(A->ns), sr(A->ns), sc(A->slots), lr(A->nl), lc(A->long_nnz), g0;
    std::vector<uint8_t> sv((size_t)A->slots * esz), lv((size_t)A->long_nnz * esz);
    rgcsr_status s = rgcsr_export(A, stream, gp.data(), sl.data(), sr.data(), sv.data(), sc.data(), lr.data(),
                                  lp.data(), lv.data(), lc.data());
    if (s != RGCSR_OK) return s;
    if (A->ragged) {
        g0.resize(A->ng + 1);
        HIPCHK(hipMemcpy(g0.data(), A->grp_row0, (A->ng + 1) * 4, hipMemcpyDeviceToHost));
    }
    std::vector<int64_t> len(A->n_rows, 0);
    for (int64_t i = 0; i < A->ns; i++) len[sr[i]] = sl[i];
    for (int64_t i = 0; i < A->nl; i++) len[lr[i]] = lp[i + 1] - lp[i];
    row_ptr[0] = 0;
    for (int64_t r = 0; r < A->n_rows; r++) row_ptr[r + 1] = row_ptr[r] + len[r];
    const int64_t G = A->prm.G, T = A->prm.T;
    for (int64_t g = 0; g < A->ng; g++) {
        const int64_t r0 = A->ragged ? g0[g] : g * G;
        const int64_t r1 = A->ragged ? g0[g + 1] : std::min<int64_t>(A->ns, r0 + G);
        const int64_t s = r1 - r0;
        for (int64_t t = 0; t < s; t++) {
            const int64_t row = sr[r0 + t], L = sl[r0 + t];
            for (int64_t j = 0; j < L; j++) {
                const int64_t slot = gp[g] + (j / T) * (s * T) + t * T + j % T;
                col_idx[row_ptr[row] + j] = sc[slot];
                memcpy((uint8_t *)vals + (size_t)(row_ptr[row] + j) * esz, &sv[(size_t)slot * esz], esz);
            }
        }
    }
    for (int64_t i = 0; i < A->nl; i++) {
        const int64_t row = lr[i];
        for (int64_t j = 0; j < lp[i + 1] - lp[i]; j++) {
            col_idx[row_ptr[row] + j] = lc[lp[i] + j];
            memcpy((uint8_t *)vals + (size_t)(row_ptr[row] + j) * esz, &lv[(size_t)(lp[i] + j) * esz], esz);
        }
    }
    ABI_CATCH
}

rgcsr_status rgcsr_info(rgcsr_handle A, rgcsr_info_t *out) {
    ABI_TRY
    if (!A || !out) fail(RGCSR_EINVAL, "null argument");
    *out = rgcsr_info_t{};
    out->n_rows = A->n_rows; out->n_cols = A->n_cols; out->nnz = A->nnz;
    out->n_groups = A->ng; out->n_short = A->ns; out->n_long = A->nl; out->slots = A->slots;
    out->long_nnz = A->long_nnz; out->n_matrices = A->n_matrices; out->long_work = A->n_wave_long + A->n_block;
    out->partials = A->n_partials; out->group_size = A->prm.G; out->lanes_per_row = A->prm.T;
    out->value_dtype = A->vdt; out->has_transpose = A->AT != nullptr;
    out->sort_window = A->prm.sigma; out->long_row_threshold = A->prm.tau;
    out->device_bytes = (int64_t)A->bytes + (A->AT ? (int64_t)A->AT->bytes : 0);
    out->rows_per_lane = A->R;
    out->pad_loads = A->pad;
    out->load_policy = A->lp;
    out->device_bytes += (int64_t)A->tile_bytes + (A->AT ? (int64_t)A->AT->tile_bytes : 0);
    out->tiled_rows = A->n_trows;
    out->tile_entries = A->n_tent;
    out->n_tiles = A->n_tiles;
    if (A->PN) {
        out->col_panels = A->PN->n_panels;
        out->panel_pieces = A->PN->n_rows;
        out->device_bytes += (int64_t)A->PN->bytes;
    }
    ABI_CATCH
}

}  // extern "C"

namespace {

// Rebase every device pointer of a copied struct from one block (the member
// `block` of src) to the same member of dst.
template <class H, class... P> void rebase(H *dst, const H *src, void *H::*block, P H::*...members) {
    auto fix = [&](auto H::*m) {
        auto &p = dst->*m;
        if (p)
            p = (std::remove_reference_t<decltype(p)>)((char *)(dst->*block) +
                                                         ((const char *)(src->*m) - (const char *)(src->*block)));
    };
    (fix(members), ...);
}

rgcsr_matrix_s *clone_handle(const rgcsr_matrix_s *A, hipStream_t st) {
    auto *h = new rgcsr_matrix_s(*A);
    h->mem = nullptr;
    h->owns_mem = true;
    h->AT = nullptr;
    h->PN = nullptr;
    h->tile_mem = nullptr;
    try {
        if (A->bytes) HIPCHK(hipMalloc(&h->mem, A->bytes));
        if (A->bytes) HIPCHK(hipMemcpyAsync(h->mem, A->mem, A->bytes, hipMemcpyDeviceToDevice, st));
        rebase(h, A, &rgcsr_matrix_s::mem, &rgcsr_matrix_s::gp, &rgcsr_matrix_s::gend, &rgcsr_matrix_s::grp_row0,
               &rgcsr_matrix_s::short_len,
               &rgcsr_matrix_s::short_row, &rgcsr_matrix_s::slot_col, &rgcsr_matrix_s::slot_val,
               &rgcsr_matrix_s::short_items, &rgcsr_matrix_s::wave_work, &rgcsr_matrix_s::block_work,
               &rgcsr_matrix_s::combine,
               &rgcsr_matrix_s::long_row, &rgcsr_matrix_s::long_col,
               &rgcsr_matrix_s::long_ptr, &rgcsr_matrix_s::long_val, &rgcsr_matrix_s::partial,
               &rgcsr_matrix_s::row_ptr, &rgcsr_matrix_s::t_map_slot,
               &rgcsr_matrix_s::t_map_long, &rgcsr_matrix_s::unit_map_rows, &rgcsr_matrix_s::unit_map_one,
               &rgcsr_matrix_s::pan_crow, &rgcsr_matrix_s::pan_cptr, &rgcsr_matrix_s::pan_vidx,
               &rgcsr_matrix_s::pan_y);
        // tile arrays: in the same block, or in a block of their own
        auto tile_rebase = [&](void *rgcsr_matrix_s::*block) {
            rebase(h, A, block, &rgcsr_matrix_s::tile_units, &rgcsr_matrix_s::tile_ptr, &rgcsr_matrix_s::tile_dst,
                   &rgcsr_matrix_s::tile_orow, &rgcsr_matrix_s::tile_lcol, &rgcsr_matrix_s::tile_val,
                   &rgcsr_matrix_s::tile_partial, &rgcsr_matrix_s::rest_wave, &rgcsr_matrix_s::rest_block,
                   &rgcsr_matrix_s::rest_combine);
        };
        if (A->tile_mem) {
            h->tile_mem = nullptr;
            HIPCHK(hipMalloc(&h->tile_mem, A->tile_bytes));
            HIPCHK(hipMemcpyAsync(h->tile_mem, A->tile_mem, A->tile_bytes, hipMemcpyDeviceToDevice, st));
            tile_rebase(&rgcsr_matrix_s::tile_mem);
        } else {
            tile_rebase(&rgcsr_matrix_s::mem);
        }
        if (A->AT) h->AT = clone_handle(A->AT, st);
        if (A->PN) h->PN = clone_handle(A->PN, st);
        HIPCHK(hipStreamSynchronize(st));
    } catch (...) {
        free_handle(h);
        throw;
    }
    return h;
}

}  // namespace

extern "C" {

rgcsr_status rgcsr_clone(rgcsr_handle A, void *stream, rgcsr_handle *out) {
    ABI_TRY
    check_handle(A);
    if (!out) fail(RGCSR_EINVAL, "out is null");
    *out = clone_handle(A, (hipStream_t)stream);
    ABI_CATCH
}

rgcsr_status rgcsr_destroy(rgcsr_handle A) {
    ABI_TRY
    if (!A) return RGCSR_OK;
    // hipFree waits for the device in any case; a handle in caller memory
    // frees host memory only, so destroying it stalls no stream
    if (owns_device_memory(A)) (void)hipDeviceSynchronize();
    free_handle(A);
    ABI_CATCH
}

// ---------------------------------------------------------------------------
// Hybrid
// ---------------------------------------------------------------------------
rgcsr_status hyb_from_csr(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *row_ptr,
                          const int32_t *col_idx, const void *vals, rgcsr_dtype vals_dtype, rgcsr_dtype value_dtype,
                          int64_t ell_width, int validate, void *stream, hyb_handle *out) {
    ABI_TRY
    if (!out) fail(RGCSR_EINVAL, "out is null");
    *out = nullptr;
    check_dtype(vals_dtype, "vals");
    check_dtype(value_dtype, "value_dtype");
    if (validate) validate_csr(n_rows, n_cols, nnz, row_ptr, col_idx);
    else if (!row_ptr || row_ptr[n_rows] != nnz) fail(RGCSR_ECSR, "row_ptr[n_rows] != nnz");
    const int esz = dtype_size(value_dtype);
    std::vector<uint8_t> conv((size_t)nnz * esz);
    if (nnz) convert_values(vals, vals_dtype, conv.data(), value_dtype, nnz);
    const int64_t K1 = ell_width >= 0 ? ell_width : hyb_width_rule(n_rows, row_ptr, esz);
    const int64_t n_pad = (n_rows + 63) / 64 * 64;
    if (K1 > 0 && n_pad > INT64_MAX / K1) fail(RGCSR_EOVERFLOW, "ELL too large");
    std::vector<int32_t> ecol((size_t)(n_pad * K1), -1);
    std::vector<uint8_t> eval((size_t)(n_pad * K1) * esz, 0);
    int64_t m = 0;
    for (int64_t i = 0; i < n_rows; i++) m += std::max<int64_t>(0, row_ptr[i + 1] - row_ptr[i] - K1);
    std::vector<int32_t> crow(m), ccol(m);
    std::vector<uint8_t> cval((size_t)m * esz);
    int64_t e = 0;
    for (int64_t i = 0; i < n_rows; i++) {
        const int64_t b = row_ptr[i], len = row_ptr[i + 1] - b;
        for (int64_t j = 0; j < len; j++) {
            if (j < K1) {
                ecol[j * n_pad + i] = col_idx[b + j];
                memcpy(&eval[(size_t)(j * n_pad + i) * esz], &conv[(size_t)(b + j) * esz], esz);
            } else {
                crow[e] = (int32_t)i;
                ccol[e] = col_idx[b + j];
                memcpy(&cval[(size_t)e * esz], &conv[(size_t)(b + j) * esz], esz);
                e++;
            }
        }
    }
    auto *h = new hyb_matrix_s();
    try {
        h->device = current_device();
        h->vdt = value_dtype; h->esz = esz;
        h->n_rows = n_rows; h->n_cols = n_cols; h->nnz = nnz; h->n_pad = n_pad; h->K1 = K1; h->m = m;
        Arena a;
        a.add(&h->ell_col, ecol.size());
        a.add((uint8_t **)&h->ell_val, eval.size());
        a.add(&h->coo_row, crow.size());
        a.add(&h->coo_col, ccol.size());
        a.add((uint8_t **)&h->coo_val, cval.size());
        h->mem = a.commit();
        h->bytes = a.total;
        hipStream_t st = (hipStream_t)stream;
        upload(h->ell_col, ecol, st);
        upload_bytes(h->ell_val, eval, st);
        upload(h->coo_row, crow, st);
        upload(h->coo_col, ccol, st);
        upload_bytes(h->coo_val, cval, st);
        HIPCHK(hipStreamSynchronize(st));
    } catch (...) {
        if (h->mem) (void)hipFree(h->mem);
        delete h;
        throw;
    }
    *out = h;
    ABI_CATCH
}

rgcsr_status hyb_spmv(hyb_handle A, const void *x, void *y, rgcsr_dtype vec_dtype, void *stream) {
    ABI_TRY
    if (!A) fail(RGCSR_EINVAL, "null handle");
    if (current_device() != A->device) fail(RGCSR_EINVAL, "handle belongs to another device");
    if ((!x && A->n_cols) || (!y && A->n_rows)) fail(RGCSR_EINVAL, "null vector");
    const int f64 = vec_is_f64(vec_dtype);
    if (!f64 && A->vdt == RGCSR_F64) fail(RGCSR_EUNSUPPORTED, "F64 stored values need F64 vectors");
    HybParams H{A->n_rows, A->n_pad, A->m, (int32_t)A->K1, A->ell_col, A->ell_val, A->coo_row, A->coo_col, A->coo_val};
    hipError_t e = launch_hyb(H, A->vdt, f64, x, y, (hipStream_t)stream);
    if (e != hipSuccess) fail(e == hipErrorInvalidValue ? RGCSR_EUNSUPPORTED : RGCSR_EHIP,
                              std::string("hyb_spmv: ") + hipGetErrorString(e));
    ABI_CATCH
}

rgcsr_status hyb_export(hyb_handle A, void *stream, int32_t *ell_col, void *ell_val, int32_t *coo_row,
                        int32_t *coo_col, void *coo_val) {
    ABI_TRY
    if (!A) fail(RGCSR_EINVAL, "null handle");
    hipStream_t st = (hipStream_t)stream;
    const size_t ne = (size_t)(A->n_pad * A->K1);
    auto get = [&](void *dst, const void *src, size_t bytes) {
        if (dst && src && bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    };
    get(ell_col, A->ell_col, ne * 4);
    get(ell_val, A->ell_val, ne * A->esz);
    get(coo_row, A->coo_row, (size_t)A->m * 4);
    get(coo_col, A->coo_col, (size_t)A->m * 4);
    get(coo_val, A->coo_val, (size_t)A->m * A->esz);
    HIPCHK(hipStreamSynchronize(st));
    ABI_CATCH
}

rgcsr_status hyb_info(hyb_handle A, hyb_info_t *out) {
    ABI_TRY
    if (!A || !out) fail(RGCSR_EINVAL, "null argument");
    *out = hyb_info_t{A->n_rows, A->n_cols, A->nnz, A->n_pad, A->K1, A->m, (int64_t)A->bytes, A->vdt};
    ABI_CATCH
}

rgcsr_status hyb_clone(hyb_handle A, void *stream, hyb_handle *out) {
    ABI_TRY
    if (!A || !out) fail(RGCSR_EINVAL, "null argument");
    if (current_device() != A->device) fail(RGCSR_EINVAL, "handle belongs to another device");
    hipStream_t st = (hipStream_t)stream;
    auto *h = new hyb_matrix_s(*A);
    h->mem = nullptr;
    try {
        if (A->bytes) HIPCHK(hipMalloc(&h->mem, A->bytes));
        if (A->bytes) HIPCHK(hipMemcpyAsync(h->mem, A->mem, A->bytes, hipMemcpyDeviceToDevice, st));
        rebase(h, A, &hyb_matrix_s::mem, &hyb_matrix_s::ell_col, &hyb_matrix_s::coo_row, &hyb_matrix_s::coo_col,
               &hyb_matrix_s::ell_val, &hyb_matrix_s::coo_val);
        HIPCHK(hipStreamSynchronize(st));
    } catch (...) {
        if (h->mem) (void)hipFree(h->mem);
        delete h;
        throw;
    }
    *out = h;
    ABI_CATCH
}

rgcsr_status hyb_destroy(hyb_handle A) {
    ABI_TRY
    if (!A) return RGCSR_OK;
    (void)hipDeviceSynchronize();
    if (A->mem) (void)hipFree(A->mem);
    delete A;
    ABI_CATCH
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Conjugate gradients
// ---------------------------------------------------------------------------
namespace {

struct DevVec {
    void *p = nullptr;
    ~DevVec() {
        if (p) (void)hipFree(p);
    }
    template <class T> T *alloc(int64_t n) {
        HIPCHK(hipMalloc(&p, std::max<int64_t>(n, 1) * sizeof(T)));
        return (T *)p;
    }
};

void hipok(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(RGCSR_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Declared after the workspace, so it runs first on every exit path: no
// workspace is freed while kernels queued on the stream may still use it.
struct SyncOnExit {
    hipStream_t st;
    ~SyncOnExit() { (void)hipStreamSynchronize(st); }
};

double read_scalar(const double *d, hipStream_t st) {
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return v;
}

}  // namespace

extern "C" {

// Device buffers of the mixed-precision CG (n rows, nb block partials).
struct CgWork {
    double *r64, *q64;
    float *r, *p, *q, *d;
    double *part, *scal;
};

static void cg_mixed_check(rgcsr_handle A_lo, rgcsr_handle A_hi, const double *b, double *x, rgcsr_cg_stats *stats) {
    check_handle(A_lo);
    check_handle(A_hi);
    if (!b || !x || !stats) fail(RGCSR_EINVAL, "null argument");
    const int64_t n = A_lo->n_rows;
    if (A_lo->n_cols != n || A_hi->n_rows != n || A_hi->n_cols != n) fail(RGCSR_EINVAL, "matrices must be square and equal in shape");
    if (A_lo->vdt == RGCSR_F64) fail(RGCSR_EUNSUPPORTED, "A_lo must store F32, F16 or BF16 values");
    if (A_hi->vdt != RGCSR_F64 && A_hi->vdt != RGCSR_F32) fail(RGCSR_EUNSUPPORTED, "A_hi must store F64 or F32 values");
}

// FP64 iterative refinement around FP32 CG on A_lo (every buffer of w is
// written before it is read, so none needs clearing).
static void cg_mixed_run(rgcsr_handle A_lo, rgcsr_handle A_hi, const double *b, double *x, double tol, double inner_tol,
                         int32_t max_outer, int32_t max_inner, hipStream_t st, const CgWork &w, int nb,
                         rgcsr_cg_stats *stats, std::chrono::steady_clock::time_point t0) {
    const int64_t n = A_lo->n_rows;
    double *r64 = w.r64, *q64 = w.q64, *part = w.part, *scal = w.scal;
    float *r = w.r, *p = w.p, *q = w.q, *d = w.d;
    hipok(launch_dot(n, b, b, 1, part, nb, st), "dot");
    hipok(launch_scalar(part, nb, scal, kScalOut, st), "scalar");
    double bnorm = std::sqrt(read_scalar(scal + kOut, st));
    if (bnorm == 0.0) bnorm = 1.0;
    *stats = rgcsr_cg_stats{};
    int32_t outer = 0, inner_total = 0;
    double relres = 0.0;
    for (;;) {
        spmv_launch(A_hi, 1, x, 1, q64, 1, 1, false, st);
        hipok(launch_resid(n, b, q64, r64, part, nb, st), "resid");
        hipok(launch_scalar(part, nb, scal, kScalOut, st), "scalar");
        const double rr = read_scalar(scal + kOut, st);
        relres = std::sqrt(rr) / bnorm;
        if (relres <= tol || outer >= max_outer || rr == 0.0) break;
        const double s = 1.0 / std::sqrt(rr);
        hipok(launch_refine_start(n, r64, s, r, d, p, part, nb, st), "refine_start");
        hipok(launch_scalar(part, nb, scal, kScalRRInit, st), "scalar");
        for (int32_t it = 1; it <= max_inner; it++) {
            spmv_launch(A_lo, 1, p, 1, q, 1, 0, false, st);
            hipok(launch_dot(n, p, q, 0, part, nb, st), "dot");
            hipok(launch_scalar(part, nb, scal, kScalPQ, st), "scalar");
            hipok(launch_cg_xr(n, d, r, p, q, 0, scal, part, nb, st), "cg_xr");
            hipok(launch_scalar(part, nb, scal, kScalRRNew, st), "scalar");
            inner_total++;
            bool stop = it == max_inner;
            if (!stop && it % 4 == 0) {
                double sc[2];
                HIPCHK(hipMemcpyAsync(sc, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                stop = std::sqrt(sc[kRR] / sc[kRR0]) <= inner_tol;
            }
            if (stop) break;
            hipok(launch_cg_p(n, p, r, 0, scal, nb, st), "cg_p");
        }
        hipok(launch_refine_add(n, x, d, 1.0 / s, nb, st), "refine_add");
        outer++;
    }
    HIPCHK(hipStreamSynchronize(st));
    stats->outer_iterations = outer;
    stats->inner_iterations = inner_total;
    stats->relres = relres;
    stats->converged = relres <= tol;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

rgcsr_status rgcsr_cg_solve(rgcsr_handle A_lo, rgcsr_handle A_hi, const double *b, double *x, double tol,
                            double inner_tol, int32_t max_outer, int32_t max_inner, void *stream,
                            rgcsr_cg_stats *stats) {
    ABI_TRY
    cg_mixed_check(A_lo, A_hi, b, x, stats);
    const int64_t n = A_lo->n_rows;
    hipStream_t st = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    const int nb = (int)nblocks_vec(n);
    DevVec m_r64, m_q64, m_r, m_p, m_q, m_d, m_part, m_scal;
    CgWork w;
    w.r64 = m_r64.alloc<double>(n);
    w.q64 = m_q64.alloc<double>(n);
    w.r = m_r.alloc<float>(n);
    w.p = m_p.alloc<float>(n);
    w.q = m_q.alloc<float>(n);
    w.d = m_d.alloc<float>(n);
    w.part = m_part.alloc<double>(nb);
    w.scal = m_scal.alloc<double>(kNumScal);
    SyncOnExit guard{st};
    cg_mixed_run(A_lo, A_hi, b, x, tol, inner_tol, max_outer, max_inner, st, w, nb, stats, t0);
    ABI_CATCH
}

rgcsr_status rgcsr_cg_solve_noalloc(rgcsr_handle A_lo, rgcsr_handle A_hi, const double *b, double *x, double tol,
                                    double inner_tol, int32_t max_outer, int32_t max_inner, void *stream,
                                    rgcsr_cg_stats *stats) {
    ABI_TRY
    cg_mixed_check(A_lo, A_hi, b, x, stats);
    const int64_t n = A_lo->n_rows;
    if (n > kNoAllocCgMaxRows)
        fail(RGCSR_EUNSUPPORTED, "rgcsr_cg_solve_noalloc: " + std::to_string(n) + " rows exceed the static workspace (" +
                                     std::to_string(kNoAllocCgMaxRows) + " rows); use rgcsr_cg_solve");
    hipStream_t st = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    const int nb = (int)nblocks_vec(n);
    if (nb > kNoAllocCgMaxBlocks) fail(RGCSR_EUNSUPPORTED, "too many block partials for the static workspace");
    void *base = nullptr;
    hipok(noalloc_cg_workspace(&base), "workspace address");
    char *ws = (char *)base;
    CgWork w;
    w.r64 = (double *)ws;
    w.q64 = (double *)(ws + kNoAllocOffQ64);
    w.r = (float *)(ws + kNoAllocOffR);
    w.p = (float *)(ws + kNoAllocOffP);
    w.q = (float *)(ws + kNoAllocOffQ);
    w.d = (float *)(ws + kNoAllocOffD);
    w.part = (double *)(ws + kNoAllocOffPart);
    w.scal = (double *)(ws + kNoAllocOffScal);
    // returns only when the stream has passed every kernel that uses the
    // workspace, so a later call (on any stream) finds it free
    SyncOnExit guard{st};
    cg_mixed_run(A_lo, A_hi, b, x, tol, inner_tol, max_outer, max_inner, st, w, nb, stats, t0);
    ABI_CATCH
}

rgcsr_status rgcsr_cg_solve_f64(rgcsr_handle A, const double *b, double *x, double tol, int32_t max_iter,
                                void *stream, rgcsr_cg_stats *stats) {
    ABI_TRY
    check_handle(A);
    if (!b || !x || !stats) fail(RGCSR_EINVAL, "null argument");
    const int64_t n = A->n_rows;
    if (A->n_cols != n) fail(RGCSR_EINVAL, "matrix must be square");
    if (A->vdt != RGCSR_F64 && A->vdt != RGCSR_F32) fail(RGCSR_EUNSUPPORTED, "A must store F64 or F32 values");
    hipStream_t st = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    const int nb = (int)nblocks_vec(n);
    DevVec m_r, m_p, m_q, m_part, m_scal;
    double *r = m_r.alloc<double>(n), *p = m_p.alloc<double>(n), *q = m_q.alloc<double>(n);
    double *part = m_part.alloc<double>(nb), *scal = m_scal.alloc<double>(kNumScal);
    SyncOnExit guard{st};
    hipok(launch_dot(n, b, b, 1, part, nb, st), "dot");
    hipok(launch_scalar(part, nb, scal, kScalOut, st), "scalar");
    double bnorm = std::sqrt(read_scalar(scal + kOut, st));
    if (bnorm == 0.0) bnorm = 1.0;
    spmv_launch(A, 1, x, 1, q, 1, 1, false, st);
    hipok(launch_resid(n, b, q, r, part, nb, st), "resid");
    hipok(launch_scalar(part, nb, scal, kScalRRInit, st), "scalar");
    hipok(launch_copy(n, r, p, 1, nb, st), "copy");
    int32_t it = 0;
    *stats = rgcsr_cg_stats{};
    double rr = read_scalar(scal + kRR, st);
    while (it < max_iter && std::sqrt(rr) / bnorm > tol) {
        spmv_launch(A, 1, p, 1, q, 1, 1, false, st);
        hipok(launch_dot(n, p, q, 1, part, nb, st), "dot");
        hipok(launch_scalar(part, nb, scal, kScalPQ, st), "scalar");
        hipok(launch_cg_xr(n, x, r, p, q, 1, scal, part, nb, st), "cg_xr");
        hipok(launch_scalar(part, nb, scal, kScalRRNew, st), "scalar");
        hipok(launch_cg_p(n, p, r, 1, scal, nb, st), "cg_p");
        it++;
        if (it % 4 == 0 || it == max_iter) rr = read_scalar(scal + kRR, st);
    }
    spmv_launch(A, 1, x, 1, q, 1, 1, false, st);
    hipok(launch_resid(n, b, q, r, part, nb, st), "resid");
    hipok(launch_scalar(part, nb, scal, kScalOut, st), "scalar");
    stats->relres = std::sqrt(read_scalar(scal + kOut, st)) / bnorm;
    stats->inner_iterations = it;
    stats->outer_iterations = 1;
    stats->converged = stats->relres <= tol;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    ABI_CATCH
}

}  // extern "C"
