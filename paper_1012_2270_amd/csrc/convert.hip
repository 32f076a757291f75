// Device-side CSR -> RgCSR conversion for gfx950: the layout of Section 3.4
// with the sort-window, long-row and lanes-per-row readings, built where the
// CSR arrays already live.  Ordering and offsets use rocPRIM primitives
// (stable radix sort, stable selection, scans); the scatter writes each
// group's slots with consecutive lanes on consecutive rows, so a wavefront
// writes 64 consecutive slots per step.  The result equals the host
// converter's arrays bit for bit.
#include <hip/hip_runtime.h>

#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include "convert.h"

namespace rg {

void *DevScratch::get(size_t bytes) {
    void *p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) fail(RGCSR_ENOMEM, "device scratch allocation failed");
    bufs.push_back(p);
    return p;
}

DevScratch::~DevScratch() {
    (void)hipStreamSynchronize(st);
    for (void *p : bufs) (void)hipFree(p);
}

namespace {

#define CHK(x)                                                                                             \
    do {                                                                                                   \
        hipError_t e_ = (x);                                                                               \
        if (e_ != hipSuccess) fail(RGCSR_EHIP, std::string("device conversion: ") + hipGetErrorString(e_)); \
    } while (0)

int nblocks(int64_t n, int per = 256) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 65536)); }

// bit 0: row_ptr[0] != 0; bit 1: decreasing or beyond nnz; bit 2: column out
// of range; bit 3: columns not strictly ascending; bit 4: row_ptr[n] != nnz;
// bit 5: a row longer than int32
__global__ void validate_k(const int64_t *rp, const int32_t *col, int64_t n, int64_t n_cols, int64_t nnz,
                           int32_t *err) {
    int32_t e = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int64_t b = rp[i], en = rp[i + 1];
        if (b < 0 || en < b || en > nnz) {
            e |= 2;
            continue;
        }
        if (en - b > INT32_MAX) e |= 32;
        int64_t prev = -1;
        for (int64_t k = b; k < en; k++) {
            const int64_t c = col[k];
            if (c < 0 || c >= n_cols) e |= 4;
            if (c <= prev) e |= 8;
            prev = c;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (rp[0] != 0) e |= 1;
        if (rp[n] != nnz) e |= 16;
    }
    if (e) atomicOr(err, e);
}

// lengths and the sort keys of the window step: (window, longest first),
// row index as the value; rows of equal key keep their order (stable sort)
__global__ void keys_k(const int64_t *rp, int64_t n, int64_t sigma, int32_t *len, uint64_t *key, int32_t *row) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t l = (int32_t)(rp[i + 1] - rp[i]);
        len[i] = l;
        row[i] = (int32_t)i;
        if (key) key[i] = ((uint64_t)(i / sigma) << 31) | (uint64_t)(0x7fffffffu - (uint32_t)l);
    }
}

// flags of the long-row split over rows in window order
__global__ void split_k(const int32_t *ord, const int32_t *len, int64_t n, int64_t tau, uint8_t *is_short,
                        uint8_t *is_long) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const bool lg = tau >= 0 && len[ord[i]] > tau;
        is_short[i] = lg ? 0 : 1;
        is_long[i] = lg ? 1 : 0;
    }
}

// lengths of the listed rows; long-list keys (longest first); flags for the
// plan: bit 0 = some grouped row is out of place, bit 1 = some grouped row is
// empty
__global__ void gather_len_k(const int32_t *rows, const int32_t *len, int64_t n, int32_t *out, uint32_t *key,
                             int32_t *flags) {
    int32_t f = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t l = len[rows[i]];
        if (out) out[i] = l;
        if (key) key[i] = 0x7fffffffu - (uint32_t)l;
        if (flags) {
            if (rows[i] != i) f |= 1;
            if (l == 0) f |= 2;
        }
    }
    if (flags && f) atomicOr(flags, f);
}

// slots of each group: rows x (widest row rounded up to T)
__global__ void group_slots_k(const int32_t *lens_s, int64_t ns, int32_t G, int32_t T, int64_t ng, int64_t *cnt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += stride) {
        const int64_t r0 = g * G, r1 = std::min<int64_t>(ns, r0 + G);
        int64_t w = 0;
        for (int64_t r = r0; r < r1; r++) w = std::max<int64_t>(w, lens_s[r]);
        w = (w + T - 1) / T * T;
        cnt[g] = (r1 - r0) * w;
    }
}

__global__ void long_len_k(const int32_t *lv, const int32_t *len, int64_t nl, int64_t *out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += stride) out[i] = len[lv[i]];
}

// ---- value conversion, same rules as the host (convert_values) ------------
__device__ __forceinline__ float f16_to_f32_exact(uint16_t h) {
    const uint32_t sign = (uint32_t)(h & 0x8000u) << 16, e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
    if (e == 0x1f) return bits_f32(sign | 0x7f800000u | (m << 13));
    if (e == 0) return (sign ? -1.0f : 1.0f) * ((float)m * 0x1p-24f);
    return bits_f32(sign | ((e + 112u) << 23) | (m << 13));
}

template <int SD> struct In;
template <> struct In<RGCSR_F64> { using T = double; __device__ static float f32(T v) { return (float)v; } };
template <> struct In<RGCSR_F32> { using T = float; __device__ static float f32(T v) { return v; } };
template <> struct In<RGCSR_F16> { using T = uint16_t; __device__ static float f32(T v) { return f16_to_f32_exact(v); } };
template <> struct In<RGCSR_BF16> { using T = uint16_t; __device__ static float f32(T v) { return bf16_to_f32(v); } };

template <int DD> struct Out;
template <> struct Out<RGCSR_F64> { using T = double; };
template <> struct Out<RGCSR_F32> { using T = float; };
template <> struct Out<RGCSR_F16> { using T = uint16_t; };
template <> struct Out<RGCSR_BF16> { using T = uint16_t; };

template <int SD, int DD> __device__ __forceinline__ typename Out<DD>::T cvt(typename In<SD>::T v) {
    if constexpr (SD == DD) return v;
    else if constexpr (DD == RGCSR_F64) return (double)In<SD>::f32(v);
    else if constexpr (DD == RGCSR_F32) return In<SD>::f32(v);
    else if constexpr (DD == RGCSR_F16) return f32_to_f16_rne(In<SD>::f32(v));
    else return f32_to_bf16_rne(In<SD>::f32(v));
}

// one lane per grouped row: nonzero j of local row t of group g goes to
// gp[g] + (j/T)*(s*T) + t*T + j%T; slots past the row's length are padding
// (value bits 0, the row's last column, or 0 for an empty row)
template <int SD, int DD>
__global__ void scatter_k(const int32_t *sv, const int32_t *lens_s, const int64_t *rp, const int32_t *col,
                          const typename In<SD>::T *vals, const int64_t *gp, int64_t ns, int32_t G, int32_t T,
                          int32_t *short_len, int32_t *short_row, int32_t *slot_col, typename Out<DD>::T *slot_val) {
    using O = typename Out<DD>::T;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < ns; s += stride) {
        const int64_t g = s / G, t = s - g * G;
        const int64_t sg = std::min<int64_t>(G, ns - g * G);
        const int64_t g0 = gp[g], W = (gp[g + 1] - g0) / sg;
        const int32_t r = sv[s];
        const int64_t b = rp[r];
        const int64_t len = lens_s[s];
        short_len[s] = (int32_t)len;
        if (short_row) short_row[s] = r;
        const int32_t ghost = len ? col[b + len - 1] : 0;
        for (int64_t j = 0; j < W; j++) {
            const int64_t slot = g0 + (j / T) * (sg * T) + t * T + (j % T);
            if (j < len) {
                slot_col[slot] = col[b + j];
                slot_val[slot] = cvt<SD, DD>(vals[b + j]);
            } else {
                slot_col[slot] = ghost;
                slot_val[slot] = (O)0;
            }
        }
    }
}

// one wavefront per long row: contiguous copy into the long-row segment
template <int SD, int DD>
__global__ void long_copy_k(const int32_t *lv, const int64_t *lp, const int64_t *rp, const int32_t *col,
                            const typename In<SD>::T *vals, int64_t nl, int32_t *long_row, int32_t *long_col,
                            typename Out<DD>::T *long_val) {
    const int lane = threadIdx.x & 63;
    const int64_t wstride = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < nl; i += wstride) {
        const int32_t r = lv[i];
        const int64_t b = rp[r], o = lp[i], len = lp[i + 1] - o;
        if (lane == 0) long_row[i] = r;
        for (int64_t j = lane; j < len; j += 64) {
            long_col[o + j] = col[b + j];
            long_val[o + j] = cvt<SD, DD>(vals[b + j]);
        }
    }
}

// ---- rocPRIM calls with scratch from DevScratch ------------------------------
template <class F> void with_temp(DevScratch &S, F f) {
    size_t bytes = 0;
    CHK(f(nullptr, bytes));
    void *tmp = S.get(bytes);
    CHK(f(tmp, bytes));
}

}  // namespace

void device_plan(DevPlan &P, const LayoutParams &p, int64_t n_rows, int64_t n_cols, int64_t nnz,
                 const int64_t *rp, const int32_t *col, bool validate, hipStream_t st) {
    if (n_rows < 0 || n_cols < 0 || nnz < 0) fail(RGCSR_EINVAL, "negative size");
    if (n_rows > INT32_MAX || n_cols > INT32_MAX)
        fail(RGCSR_EOVERFLOW, "n_rows and n_cols must fit int32 column/row indices");
    if (!rp || (nnz > 0 && !col)) fail(RGCSR_EINVAL, "null CSR array");
    P.n_rows = n_rows;
    P.n_cols = n_cols;
    P.nnz = nnz;
    DevScratch &S = P.scratch;
    const int64_t n = n_rows;
    int32_t *flags = (int32_t *)S.get(8);
    CHK(hipMemsetAsync(flags, 0, 8, st));
    if (validate) {
        hipLaunchKernelGGL(validate_k, dim3(nblocks(n)), dim3(256), 0, st, rp, col, n, n_cols, nnz, flags);
        CHK(hipGetLastError());
        int32_t e = 0;
        CHK(hipMemcpyAsync(&e, flags, 4, hipMemcpyDeviceToHost, st));
        CHK(hipStreamSynchronize(st));
        if (e & 32) fail(RGCSR_EOVERFLOW, "row longer than int32");
        if (e & 1) fail(RGCSR_ECSR, "row_ptr[0] != 0");
        if (e & 2) fail(RGCSR_ECSR, "row_ptr decreases or exceeds nnz");
        if (e & 4) fail(RGCSR_ECSR, "column out of range");
        if (e & 8) fail(RGCSR_ECSR, "columns not strictly ascending");
        if (e & 16) fail(RGCSR_ECSR, "row_ptr[n_rows] != nnz");
    }
    if (n == 0) {
        P.gp_host.assign(1, 0);
        P.long_ptr_host.assign(1, 0);
        P.gp = (const int64_t *)S.get(8);
        CHK(hipMemsetAsync((void *)P.gp, 0, 8, st));
        P.long_ptr = P.gp;
        CHK(hipStreamSynchronize(st));
        return;
    }
    // window order: stable radix sort of (window, longest first)
    int32_t *len = (int32_t *)S.get(n * 4);
    int32_t *ord = (int32_t *)S.get(n * 4);
    uint64_t *key = nullptr;
    if (p.sigma > 1 && p.sigma < n) {
        key = (uint64_t *)S.get(n * 8);
    } else if (p.sigma >= n) {
        key = (uint64_t *)S.get(n * 8);  // one window: the key is the length alone
    }
    int32_t *row_tmp = key ? (int32_t *)S.get(n * 4) : ord;
    hipLaunchKernelGGL(keys_k, dim3(nblocks(n)), dim3(256), 0, st, rp, n, std::max<int64_t>(1, p.sigma), len, key,
                       row_tmp);
    CHK(hipGetLastError());
    if (key) {
        uint64_t *key_out = (uint64_t *)S.get(n * 8);
        const int64_t windows = (n + p.sigma - 1) / p.sigma;
        unsigned int wbits = 0;
        while (wbits < 32 && (int64_t(1) << wbits) < windows) wbits++;
        const unsigned int end_bit = 31 + wbits;
        with_temp(S, [&](void *t, size_t &b) {
            return rocprim::radix_sort_pairs(t, b, key, key_out, row_tmp, ord, (size_t)n, 0u, end_bit, st);
        });
    }
    // long-row split, both lists in window order
    uint8_t *fs = (uint8_t *)S.get(n), *fl = (uint8_t *)S.get(n);
    hipLaunchKernelGGL(split_k, dim3(nblocks(n)), dim3(256), 0, st, ord, len, n, p.tau, fs, fl);
    CHK(hipGetLastError());
    int32_t *sv = (int32_t *)S.get(n * 4);
    int32_t *lv0 = (int32_t *)S.get(n * 4);
    size_t *counts = (size_t *)S.get(2 * sizeof(size_t));
    with_temp(S, [&](void *t, size_t &b) { return rocprim::select(t, b, ord, fs, sv, counts, (size_t)n, st); });
    with_temp(S, [&](void *t, size_t &b) { return rocprim::select(t, b, ord, fl, lv0, counts + 1, (size_t)n, st); });
    size_t hc[2];
    CHK(hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    P.ns = (int64_t)hc[0];
    P.nl = (int64_t)hc[1];
    const int64_t ns = P.ns, nl = P.nl;
    // grouped rows: lengths, order and emptiness flags, group widths, offsets
    int32_t *lens_s = (int32_t *)S.get(std::max<int64_t>(1, ns) * 4);
    if (ns) {
        hipLaunchKernelGGL(gather_len_k, dim3(nblocks(ns)), dim3(256), 0, st, sv, len, ns, lens_s, (uint32_t *)nullptr,
                           flags + 1);
        CHK(hipGetLastError());
    }
    P.ng = (ns + p.G - 1) / p.G;
    int64_t *gp = (int64_t *)S.get((P.ng + 1) * 8);
    CHK(hipMemsetAsync(gp, 0, 8, st));
    if (P.ng) {
        int64_t *cnt = (int64_t *)S.get(P.ng * 8);
        hipLaunchKernelGGL(group_slots_k, dim3(nblocks(P.ng)), dim3(256), 0, st, lens_s, ns, p.G, p.T, P.ng, cnt);
        CHK(hipGetLastError());
        with_temp(S, [&](void *t, size_t &b) {
            return rocprim::inclusive_scan(t, b, cnt, gp + 1, (size_t)P.ng, rocprim::plus<int64_t>(), st);
        });
    }
    // long rows: longest first, ties in window order; their offsets
    int32_t *lv = lv0;
    int64_t *lp = (int64_t *)S.get((nl + 1) * 8);
    CHK(hipMemsetAsync(lp, 0, 8, st));
    if (nl) {
        uint32_t *lk = (uint32_t *)S.get(nl * 4), *lk2 = (uint32_t *)S.get(nl * 4);
        hipLaunchKernelGGL(gather_len_k, dim3(nblocks(nl)), dim3(256), 0, st, lv0, len, nl, (int32_t *)nullptr, lk,
                           (int32_t *)nullptr);
        CHK(hipGetLastError());
        lv = (int32_t *)S.get(nl * 4);
        with_temp(S, [&](void *t, size_t &b) {
            return rocprim::radix_sort_pairs(t, b, lk, lk2, lv0, lv, (size_t)nl, 0u, 31u, st);
        });
        int64_t *ll = (int64_t *)S.get(nl * 8);
        hipLaunchKernelGGL(long_len_k, dim3(nblocks(nl)), dim3(256), 0, st, lv, len, nl, ll);
        CHK(hipGetLastError());
        with_temp(S, [&](void *t, size_t &b) {
            return rocprim::inclusive_scan(t, b, ll, lp + 1, (size_t)nl, rocprim::plus<int64_t>(), st);
        });
    }
    P.gp_host.resize(P.ng + 1);
    P.long_ptr_host.resize(nl + 1);
    int32_t hf = 0;
    CHK(hipMemcpyAsync(P.gp_host.data(), gp, (P.ng + 1) * 8, hipMemcpyDeviceToHost, st));
    CHK(hipMemcpyAsync(P.long_ptr_host.data(), lp, (nl + 1) * 8, hipMemcpyDeviceToHost, st));
    CHK(hipMemcpyAsync(&hf, flags + 1, 4, hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    P.slots = P.gp_host[P.ng];
    P.long_nnz = P.long_ptr_host[nl];
    P.perm = (hf & 1) != 0;
    P.no_empty = (hf & 2) == 0;
    P.sv = sv;
    P.lv = lv;
    P.lens_s = lens_s;
    P.gp = gp;
    P.long_ptr = lp;
}

namespace {

template <int SD, int DD>
void fill_t(const DevPlan &P, const LayoutParams &p, const int64_t *rp, const int32_t *col, const void *vals,
            int32_t *short_len, int32_t *short_row, void *slot_val, int32_t *slot_col, int32_t *long_row,
            void *long_val, int32_t *long_col, hipStream_t st) {
    using IT = typename In<SD>::T;
    using OT = typename Out<DD>::T;
    if (P.ns) {
        hipLaunchKernelGGL((scatter_k<SD, DD>), dim3(nblocks(P.ns)), dim3(256), 0, st, P.sv, P.lens_s, rp, col,
                           (const IT *)vals, P.gp, P.ns, p.G, p.T, short_len, short_row, slot_col, (OT *)slot_val);
        CHK(hipGetLastError());
    }
    if (P.nl) {
        hipLaunchKernelGGL((long_copy_k<SD, DD>), dim3(nblocks(P.nl, 4)), dim3(256), 0, st, P.lv, P.long_ptr, rp, col,
                           (const IT *)vals, P.nl, long_row, long_col, (OT *)long_val);
        CHK(hipGetLastError());
    }
}

template <int SD>
void fill_s(int vdt, const DevPlan &P, const LayoutParams &p, const int64_t *rp, const int32_t *col, const void *vals,
            int32_t *short_len, int32_t *short_row, void *slot_val, int32_t *slot_col, int32_t *long_row,
            void *long_val, int32_t *long_col, hipStream_t st) {
    switch (vdt) {
    case RGCSR_F64: return fill_t<SD, RGCSR_F64>(P, p, rp, col, vals, short_len, short_row, slot_val, slot_col, long_row, long_val, long_col, st);
    case RGCSR_F32: return fill_t<SD, RGCSR_F32>(P, p, rp, col, vals, short_len, short_row, slot_val, slot_col, long_row, long_val, long_col, st);
    case RGCSR_F16: return fill_t<SD, RGCSR_F16>(P, p, rp, col, vals, short_len, short_row, slot_val, slot_col, long_row, long_val, long_col, st);
    case RGCSR_BF16: return fill_t<SD, RGCSR_BF16>(P, p, rp, col, vals, short_len, short_row, slot_val, slot_col, long_row, long_val, long_col, st);
    }
    fail(RGCSR_EINVAL, "bad value dtype");
}

}  // namespace

void device_fill(const DevPlan &P, const LayoutParams &p, const int64_t *rp, const int32_t *col, const void *vals,
                 int vals_dt, int vdt, int64_t *gp, int32_t *short_len, int32_t *short_row, void *slot_val,
                 int32_t *slot_col, int32_t *long_row, int64_t *long_ptr, void *long_val, int32_t *long_col,
                 hipStream_t st) {
    if (P.nnz > 0 && !vals) fail(RGCSR_EINVAL, "vals is null");
    CHK(hipMemcpyAsync(gp, P.gp, (P.ng + 1) * 8, hipMemcpyDeviceToDevice, st));
    CHK(hipMemcpyAsync(long_ptr, P.long_ptr, (P.nl + 1) * 8, hipMemcpyDeviceToDevice, st));
    switch (vals_dt) {
    case RGCSR_F64: return fill_s<RGCSR_F64>(vdt, P, p, rp, col, vals, short_len, short_row, slot_val, slot_col, long_row, long_val, long_col, st);
    case RGCSR_F32: return fill_s<RGCSR_F32>(vdt, P, p, rp, col, vals, short_len, short_row, slot_val, slot_col, long_row, long_val, long_col, st);
    case RGCSR_F16: return fill_s<RGCSR_F16>(vdt, P, p, rp, col, vals, short_len, short_row, slot_val, slot_col, long_row, long_val, long_col, st);
    case RGCSR_BF16: return fill_s<RGCSR_BF16>(vdt, P, p, rp, col, vals, short_len, short_row, slot_val, slot_col, long_row, long_val, long_col, st);
    }
    fail(RGCSR_EINVAL, "bad input dtype");
}

}  // namespace rg
