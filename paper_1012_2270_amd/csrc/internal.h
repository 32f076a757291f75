// Internal declarations shared by the host format library, the kernels and
// the C ABI of librgcsr.  Nothing here is part of the public interface.
#pragma once

#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/rgcsr.h"

#if defined(__HIPCC__)
#define RG_HD __host__ __device__
#else
#define RG_HD
#endif

namespace rg {

// ---------------------------------------------------------------------------
// Errors: internal code throws rg::Error; every ABI entry point catches it and
// turns it into a status code plus the thread-local message.
// ---------------------------------------------------------------------------
struct Error {
    rgcsr_status st;
    std::string msg;
};
[[noreturn]] void fail(rgcsr_status st, const std::string &msg);
// Both never throw: when copying msg fails for lack of memory, the message
// becomes a fixed string.  The second keeps a pointer to a string literal.
void set_last_error(const std::string &msg) noexcept;
void set_last_error_static(const char *msg) noexcept;

inline int dtype_size(int dt) {
    switch (dt) {
    case RGCSR_F64: return 8;
    case RGCSR_F32: return 4;
    case RGCSR_F16: return 2;
    case RGCSR_BF16: return 2;
    default: return 0;
    }
}

// ---------------------------------------------------------------------------
// Round-to-nearest-even conversions to the 16-bit storage types (bit level so
// host and device give identical bits).  A NaN stays a NaN with its sign and
// the leading payload bits, quiet bit set.
// ---------------------------------------------------------------------------
RG_HD inline uint32_t f32_bits(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    return u;
}
RG_HD inline float bits_f32(uint32_t u) {
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

RG_HD inline uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = f32_bits(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

RG_HD inline uint16_t f32_to_f16_rne(float f) {
    uint32_t u = f32_bits(f);
    uint32_t sign = (u >> 16) & 0x8000u;
    uint32_t a = u & 0x7fffffffu;
    if (a > 0x7f800000u) return (uint16_t)(sign | 0x7e00u | ((a >> 13) & 0x3ffu));  // NaN
    if (a >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);  // rounds to +-inf
    if (a >= 0x38800000u) {                                   // normal half
        uint32_t h = (a - 0x38000000u) >> 13;
        uint32_t rem = a & 0x1fffu;
        if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) h++;
        return (uint16_t)(sign | h);
    }
    if (a <= 0x33000000u) return (uint16_t)sign;  // |f| <= 2^-25 rounds to 0
    // subnormal half: value = m * 2^(e-150), unit 2^-24 -> shift by 126-e
    uint32_t e = a >> 23;
    uint32_t m = (a & 0x7fffffu) | 0x800000u;
    uint32_t s = 126u - e;
    uint32_t h = m >> s;
    uint32_t rem = m & ((1u << s) - 1u);
    uint32_t half = 1u << (s - 1u);
    if (rem > half || (rem == half && (h & 1u))) h++;
    return (uint16_t)(sign | h);
}

RG_HD inline float bf16_to_f32(uint16_t b) { return bits_f32((uint32_t)b << 16); }

// Convert n values from src dtype to dst dtype (host).  float64 to a 16-bit
// type goes through float32 first.
void convert_values(const void *src, int src_dt, void *dst, int dst_dt, int64_t n);

// ---------------------------------------------------------------------------
// Long-row work of the SpMV kernel (rows of the long-row segment).
//   wave item  : rows a .. a+b-1 of the long list, c lanes per row (a power of
//                two <= 64, b <= 64 / c); each row has at most kWaveRowMax
//                nonzeros, so every lane multiplies at most kWaveUnroll of them.
//   block item : chunk b of the c chunks of row a, kBlockChunk nonzeros per
//                chunk, one whole workgroup; when c > 1, d is the row's first
//                partial-sum slot.
//   combine    : row a has c > 1 chunks whose partial sums start at slot d.
// ---------------------------------------------------------------------------
struct LongItem {
    int32_t a, b, c, d;
};
constexpr int kWaveUnroll = 16;                                  // nonzeros per lane, wave items
constexpr int kWaveRowMax = 64 * kWaveUnroll;                    // 1024
constexpr int kBlockThreads = 256;                               // SpMV workgroup
constexpr int kBlockWaves = kBlockThreads / 64;                  // 4
constexpr int kBlockUnroll = 64;                                 // nonzeros per lane, block items
constexpr int64_t kBlockChunk = (int64_t)kBlockThreads * kBlockUnroll;  // 16384
constexpr int kLaneSteps = 16;  // loads in flight per lane that the rows-per-lane choice aims at

struct LongWork {
    std::vector<LongItem> wave, block, combine;
    int64_t n_partials = 0;
};

// ---------------------------------------------------------------------------
// Host layout of one matrix or of a block-diagonal batch.
// ---------------------------------------------------------------------------
struct HostLayout {
    int64_t n_rows = 0, n_cols = 0, nnz = 0;
    int32_t G = 64, T = 1;
    int64_t sigma = 1, tau = -1;
    int vdt = RGCSR_F32, esz = 4;
    int64_t ng = 0, ns = 0, nl = 0, slots = 0, long_nnz = 0;
    int64_t n_matrices = 0;
    bool ragged = false;  // some group other than the last has fewer than G rows
    std::vector<int64_t> gp{0};       // gp[g]: first slot of group g; gp[ng]: slot count
    std::vector<int64_t> gend;        // end slot of each group (a batch pads the slots
                                      // before each matrix to a multiple of 64)
    std::vector<int32_t> grp_row0{0};
    std::vector<int32_t> short_len, short_row;
    std::vector<uint8_t> slot_val;
    std::vector<int32_t> slot_col;
    std::vector<int32_t> long_row;
    std::vector<int64_t> long_ptr{0};
    std::vector<uint8_t> long_val;
    std::vector<int32_t> long_col;
    LongWork work;
    std::vector<int64_t> row_off{0}, col_off{0};  // per-matrix offsets (batch)
    bool short_identity() const;
    int64_t group_end(int64_t g) const { return gend.empty() ? gp[g + 1] : gend[g]; }
    bool has_gaps() const;  // some group ends before the next one starts
};

struct LayoutParams {
    int32_t G, T;
    int64_t sigma, tau;
};

LayoutParams resolve_opts(const rgcsr_opts *opts);

// Checks the CSR convention of Section 3.1; throws RGCSR_ECSR with the
// offending row on failure.
void validate_csr(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t *rp,
                  const int32_t *col);

// Reverse Cuthill-McKee order of the symmetrised pattern of a square CSR
// matrix, perm[new] = old (ordering.cpp).
void rcm_order(int64_t n, const int64_t *rp, const int32_t *col, int32_t *perm);

// Appends the layout of one CSR matrix (values already in the storage dtype,
// esz bytes each; pad_bytes fills artificial zeros) to L, offsetting rows by
// L.n_rows and columns by L.n_cols.  When vals is null only sizes and index
// arrays are produced.
void append_layout(HostLayout &L, const LayoutParams &p, int64_t n_rows, int64_t n_cols,
                   const int64_t *rp, const int32_t *col, const uint8_t *vals, int esz,
                   uint8_t pad_byte);

// Lengths of the grouped rows in layout order under (sigma, tau) of p, and
// the count and nonzeros of the long rows; slots of those rows in groups of
// G rows with widths rounded up to T.  Cost model of the autotuner.
void short_lengths(const LayoutParams &p, int64_t n_rows, const int64_t *rp, std::vector<int32_t> &lens,
                   int64_t *n_long, int64_t *long_nnz);
int64_t group_slots(const std::vector<int32_t> &lens, int32_t G, int32_t T);

// Sizes only (no arrays), for rgcsr_layout_sizes.
void layout_sizes(const LayoutParams &p, int64_t n_rows, const int64_t *rp, int64_t *ng,
                  int64_t *ns, int64_t *nl, int64_t *slots, int64_t *long_nnz,
                  std::vector<int64_t> *long_lens_sorted);

// Work items of the long-row path from the long list's row lengths.
void build_long_work(const std::vector<int64_t> &long_ptr, LongWork &work);

// Transpose of a CSR pattern with, for every entry of A^T, the index of the
// entry of A it came from.
void transpose_csr(int64_t n_rows, int64_t n_cols, const int64_t *rp, const int32_t *col,
                   std::vector<int64_t> &rpT, std::vector<int32_t> &colT,
                   std::vector<int32_t> &srcT);

// Hybrid ELL width rule and arrays.
int64_t hyb_width_rule(int64_t n_rows, const int64_t *rp, int s_v);

// Throws RGCSR_EINVAL for a dtype code outside rgcsr_dtype.
void check_dtype(int dt, const char *what);

// Host layout (+ transposed layout) for one or more CSR matrices.
struct Built {
    HostLayout L;
    bool has_T = false;
    HostLayout LT;       // layout of A^T with values
    HostLayout LTmap;    // layout of A^T whose "values" are source indices
    std::vector<int64_t> row_ptr;  // global CSR row pointers
};

// ---------------------------------------------------------------------------
// Column panels (panel_layout.cpp): the matrix split by column into P panels
// of about equal nonzero count, panel q holding columns [cb[q], cb[q+1]).
// The panels are stacked as P row-compressed matrices: piece v of panel q is
// the entries of one row in the panel's columns (in CSR order), pieces of a
// panel in ascending row order, panel after panel; rows of at most whole_max
// nonzeros (empty rows included) are not split but form a last matrix
// (index P) of whole rows, one piece each, with all columns.  LP lays the
// stack out like any matrix (each panel appended as one matrix of a batch,
// so groups and the long-row list never mix panels and columns stay
// global); its output row codes are the row itself for a whole row and
// -1 - v for piece v of a split row (a slot of the per-piece sums, pieces in
// panel order).  LPmap is the same layout whose "values" are the CSR index
// of each element (-1 for padding).  Split row crow[i] is the sum of its
// pieces vidx[cptr[i] .. cptr[i + 1]) in panel order.
// ---------------------------------------------------------------------------
struct PanelBuilt {
    int32_t P = 0;
    std::vector<int64_t> cb;        // [P+1] panel column bounds
    HostLayout LP, LPmap;
    std::vector<int64_t> grp_off;   // [P+2] first row group of each panel (then of the whole rows) in LP
    std::vector<int64_t> long_off;  // [P+2] first long row of each panel (then of the whole rows) in LP
    std::vector<int32_t> crow;      // [split rows] row of each split row
    std::vector<int32_t> cptr;      // [split rows + 1] its pieces in vidx
    std::vector<int32_t> vidx;      // [pieces of split rows] piece index (row of LP)
    int64_t split_pieces = 0;       // pieces of split rows: LP rows [0, split_pieces)
};

constexpr int kPanelMax = 64;            // panels per handle
constexpr int kPanelXcds = 8;            // XCDs the panels are dealt to (P a multiple of this)
constexpr int kPanelRowBytes = 32;       // per-piece sums buffer: K * accumulator bytes per piece
constexpr int64_t kPanelSliceBytes = 3 << 20;  // x slice of one panel that one L2 is asked to hold

// Throws RGCSR_EINVAL unless P is 0 or a multiple of kPanelXcds up to kPanelMax.
void check_panels(int32_t P);

// Builds the panel layouts of one CSR matrix whose values are already in the
// storage dtype (esz bytes each; vals null: sizes and indices only); throws
// RGCSR_EOVERFLOW when the pieces or the nonzeros do not fit 32-bit indices.
void build_panels(PanelBuilt &B, const LayoutParams &p, int vdt, int32_t P, int64_t whole_max, int64_t n_rows,
                  int64_t n_cols, const int64_t *rp, const int32_t *col, const uint8_t *vals);

// Host layout of `count` CSR matrices (a block-diagonal batch when count > 1)
// with values converted to vdt; the CSR row pointers when keep_map or
// transpose, and the layouts of A^T (values, and source indices) when
// transpose.  Validates each matrix when validate is set.
void build_host(Built &B, const LayoutParams &p, int vdt, int32_t count, const int64_t *n_rows,
                const int64_t *n_cols, const int64_t *const *rp, const int32_t *const *col,
                const void *const *vals, int vals_dt, bool validate, bool keep_map, bool transpose);

}  // namespace rg

// Every C entry point runs its body between ABI_TRY and ABI_CATCH: internal
// errors become a status code and the thread-local message, allocation
// failures RGCSR_ENOMEM, and nothing else escapes.
#define ABI_TRY try {
#define ABI_CATCH                                                                                      \
    }                                                                                                  \
    catch (const rg::Error &e) {                                                                       \
        rg::set_last_error(e.msg);                                                                     \
        return e.st;                                                                                   \
    }                                                                                                  \
    catch (const std::bad_alloc &) {                                                                   \
        rg::set_last_error_static("host allocation failed");                                           \
        return RGCSR_ENOMEM;                                                                           \
    }                                                                                                  \
    catch (...) {                                                                                      \
        rg::set_last_error_static("unexpected internal error");                                        \
        return RGCSR_EINVAL;                                                                           \
    }                                                                                                  \
    return RGCSR_OK;

