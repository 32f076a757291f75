// Column-tiled long rows (tiles.h): the tile kernel, and the value copy after
// an update.  The partial sums are added by the SpMV kernel (kernels.hip).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "tiles.h"

namespace rg {

// Stored value type S and the type A of x, the products and the partial
// sums (FP64 for F64 storage, else FP32).
template <int VD> struct TileVal;
template <> struct TileVal<RGCSR_F64> {
    using S = double;
    using A = double;
    __device__ static double cvt(S v) { return v; }
};
template <> struct TileVal<RGCSR_F32> {
    using S = float;
    using A = float;
    __device__ static float cvt(S v) { return v; }
};
template <> struct TileVal<RGCSR_F16> {
    using S = uint16_t;
    using A = float;
    __device__ static float cvt(S v) { return (float)__builtin_bit_cast(_Float16, v); }
};
template <> struct TileVal<RGCSR_BF16> {
    using S = uint16_t;
    using A = float;
    __device__ static float cvt(S v) { return bf16_to_f32(v); }
};

// One unit per workgroup: tile t of x and the unit's products in LDS.  Every
// load of the unit -- its entries element-parallel, the x tile as 16-byte
// vectors, the row bounds of its kTilePasses passes -- is issued before the
// first barrier; then each entry is multiplied against x from LDS into the
// product buffer, and `lanes` lanes per row add the row's products
// (lane-strided, then a butterfly within the lane group) into
// partial[t][row].
template <int VD>
__global__ __launch_bounds__(kTileThreads) void tile_spmv_k(TileParams P) {
    using V = TileVal<VD>;
    using S = typename V::S;
    using A = typename V::A;
    constexpr int C = tile_cols(VD);
    constexpr int UM = tile_unit_max(VD);
    constexpr int EU = UM / kTileThreads;
    __shared__ A xs[C];
    __shared__ A prod[UM];
    const TileUnit u = P.units[blockIdx.x];
    if (u.t < 0) return;
    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)u.t * C;
    const int nc = (int)min((int64_t)C, P.n_cols - c0);
    const int32_t *ptr = P.ptr + (int64_t)u.t * (P.n_trows + 1);
    const int32_t e0 = u.e0;
    const int32_t n = u.e1 - e0;
    const S *val = (const S *)P.val + e0;
    const uint16_t *lc = P.lcol + e0;
    S v[EU];
    uint16_t c[EU];
#pragma unroll
    for (int k = 0; k < EU; k++) {
        // a unit may hold no entries (rows without nonzeros in this tile)
        const int i = tid + k * kTileThreads;
        if (i < n) {
            v[k] = __builtin_nontemporal_load(val + i);
            c[k] = __builtin_nontemporal_load(lc + i);
        } else {
            v[k] = S(0);
            c[k] = 0;
        }
    }
    const A *xt = (const A *)P.x + c0;
    // the tile (32 KB in either precision) as 16-byte vectors
    constexpr int X4 = C * (int)sizeof(A) / 16 / kTileThreads;
    // assigned on every path, so the array stays in registers
    float4 x4[X4];
    const bool vec = P.x_aligned && nc == C;
#pragma unroll
    for (int k = 0; k < X4; k++)
        x4[k] = vec ? reinterpret_cast<const float4 *>(xt)[tid + k * kTileThreads] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int L = u.lanes;
    const int sh = 31 - __builtin_clz(L);
    const int q = tid & (L - 1);
    const int per = kTileThreads >> sh;
    int32_t b0[kTilePasses], b1[kTilePasses];
#pragma unroll
    for (int j = 0; j < kTilePasses; j++) {
        const int r = u.r0 + j * per + (tid >> sh);
        b0[j] = r < u.r1 ? ptr[r] - e0 : 0;
        b1[j] = r < u.r1 ? ptr[r + 1] - e0 : 0;
    }
    if (vec) {
#pragma unroll
        for (int k = 0; k < X4; k++) reinterpret_cast<float4 *>(xs)[tid + k * kTileThreads] = x4[k];
    } else {
        for (int i = tid; i < nc; i += kTileThreads) xs[i] = xt[i];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < EU; k++) {
        const int i = tid + k * kTileThreads;
        if (i < n) prod[i] = V::cvt(v[k]) * xs[c[k]];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kTilePasses; j++) {
        const int r = j * per + (tid >> sh);
        A acc = A(0);
        for (int32_t p = b0[j] + q; p < b1[j]; p += L) acc += prod[p];
        for (int off = L >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (u.r0 + r < u.r1 && q == 0) ((A *)P.partial)[(int64_t)u.t * P.n_trows + u.r0 + r] = acc;
    }
}

hipError_t launch_tile_spmv(const TileParams &P, int vdt, int n_units, hipStream_t st) {
    if (n_units == 0) return hipSuccess;
    switch (vdt) {
    case RGCSR_F64: hipLaunchKernelGGL(tile_spmv_k<RGCSR_F64>, dim3(n_units), dim3(kTileThreads), 0, st, P); break;
    case RGCSR_F32: hipLaunchKernelGGL(tile_spmv_k<RGCSR_F32>, dim3(n_units), dim3(kTileThreads), 0, st, P); break;
    case RGCSR_F16: hipLaunchKernelGGL(tile_spmv_k<RGCSR_F16>, dim3(n_units), dim3(kTileThreads), 0, st, P); break;
    case RGCSR_BF16: hipLaunchKernelGGL(tile_spmv_k<RGCSR_BF16>, dim3(n_units), dim3(kTileThreads), 0, st, P); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class E>
__global__ __launch_bounds__(256) void tile_values_k(int64_t n, const int32_t *dst, const E *lv, E *tv) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t d = dst[i];
    if (d >= 0) tv[d] = lv[i];
}

hipError_t launch_tile_values(int64_t n, const int32_t *dst, const void *long_val, void *tile_val, int esz,
                              hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int nb = (int)((n + 255) / 256);
    if (esz == 8)
        hipLaunchKernelGGL(tile_values_k<uint64_t>, dim3(nb), dim3(256), 0, st, n, dst, (const uint64_t *)long_val,
                           (uint64_t *)tile_val);
    else if (esz == 4)
        hipLaunchKernelGGL(tile_values_k<uint32_t>, dim3(nb), dim3(256), 0, st, n, dst, (const uint32_t *)long_val,
                           (uint32_t *)tile_val);
    else if (esz == 2)
        hipLaunchKernelGGL(tile_values_k<uint16_t>, dim3(nb), dim3(256), 0, st, n, dst, (const uint16_t *)long_val,
                           (uint16_t *)tile_val);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace rg
