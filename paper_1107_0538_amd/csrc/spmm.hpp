// Row-block sparse products over row-major N x s blocks (s <= 64), shared by
// the multi-RHS and block forms: lane j of a wave owns column j, so a
// gathered row of X is one coalesced s * 8-byte load and a CSR value/index is
// a wave-uniform (scalar) load.  Every column's row sum runs in stored order
// with separate multiply and add, so column j equals the sequential CSR
// product.
#pragma once

#include "context.hpp"

namespace jpcg {

__device__ __forceinline__ int mr_logical(int G) { return xcd_logical_block((int)blockIdx.x, G); }


// Nonzeros of a row whose gathers a wave issues together: 16 with one
// column per lane, 32 (16 per half-wave) with two (mr_row_x2).
constexpr int kMrBatch = 16;
constexpr int kMrBatch2 = 32;

// One wave: y_lane = sum_k a_ik x[col_k][lane] for row i in stored order,
// without contraction, so each column is the sequential CSR row sum.
template <typename T, typename Gather>
__device__ __forceinline__ T mr_row(const int* __restrict__ rowptr, const int* __restrict__ col,
                                    const T* __restrict__ val, int i, Gather gather)
{
#pragma clang fp contract(off)
    // Batches of kMrBatch nonzeros: the (wave-uniform) indices and values
    // are loaded, then all the batch's gathers are in flight together; the
    // tail batch reads past the row's end (into the next row or the arrays'
    // zero pad of kCsrPad entries) and skips those slots, so a 27-entry row
    // takes two gather round trips.
    constexpr int B = kMrBatch;
    static_assert(B <= kCsrPad, "batch reads must stay within the padded arrays");
    // The row is the same in every lane: make that explicit so that the
    // row's indices and values come through the scalar cache.
    i = __builtin_amdgcn_readfirstlane(i);
    const int k0 = __builtin_amdgcn_readfirstlane(rowptr[i]), k1 = __builtin_amdgcn_readfirstlane(rowptr[i + 1]);
    T acc = T(0);
    for (int k = k0; k < k1; k += B) {
        T v[B], g[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            v[u] = val[k + u];
            g[u] = gather(col[k + u]);
        }
#pragma unroll
        for (int u = 0; u < B; ++u)
            if (k + u < k1) acc = acc + v[u] * g[u];
    }
    return acc;
}

// The same row product with two nonzeros per gather instruction (FP64, s
// even): lane l takes columns 2 (l mod 32) and 2 (l mod 32) + 1 of the
// nonzeros at even (lower half) or odd (upper half) positions of each batch,
// so one 16-byte load per lane fetches two nonzeros' rows of X.  This
// gather-heavy product is limited by the per-CU address path, which handles a
// 16-byte lane as fast as an 8-byte one, not by bytes.  Products are rounded
// on their own; the upper half hands its products to the lower half, which
// adds them in stored order, so both columns are the sequential CSR row sums
// bitwise (as mr_row).  The sums are valid in the lower half's lanes.
template <typename Gather2>
__device__ __forceinline__ double2 mr_row_x2(const int* __restrict__ rowptr, const int* __restrict__ col,
                                             const double* __restrict__ val, int i, Gather2 gather2)
{
#pragma clang fp contract(off)
    constexpr int B = kMrBatch2;  // nonzeros per batch, half of them per half-wave
    static_assert(B <= kCsrPad, "batch reads must stay within the padded arrays");
    i = __builtin_amdgcn_readfirstlane(i);
    const int k0 = __builtin_amdgcn_readfirstlane(rowptr[i]), k1 = __builtin_amdgcn_readfirstlane(rowptr[i + 1]);
    const bool upper = (threadIdx.x & 32) != 0;
    double a0 = 0.0, a1 = 0.0;
    for (int k = k0; k < k1; k += B) {
        double v[B / 2];
        double2 g[B / 2];
#pragma unroll
        for (int u = 0; u < B / 2; ++u) {
            const int ke = k + 2 * u;
            const double ve = val[ke], vo = val[ke + 1];
            const int ce = col[ke], co = col[ke + 1];
            v[u] = upper ? vo : ve;
            g[u] = gather2(upper ? co : ce);
        }
#pragma unroll
        for (int u = 0; u < B / 2; ++u) {
            const double p0 = v[u] * g[u].x, p1 = v[u] * g[u].y;
            const double q0 = __shfl_xor(p0, 32), q1 = __shfl_xor(p1, 32);  // the other half's products
            if (k + 2 * u < k1) {
                a0 = a0 + p0;
                a1 = a1 + p1;
            }
            if (k + 2 * u + 1 < k1) {
                a0 = a0 + q0;
                a1 = a1 + q1;
            }
        }
    }
    return make_double2(a0, a1);
}

// Y = A X (row-major N x s), lane = column.
template <int BS, typename T>
__global__ __launch_bounds__(BS) void k_spmm(int n, int s, const int* __restrict__ rowptr,
                                             const int* __restrict__ col, const T* __restrict__ val,
                                             const T* __restrict__ X, T* __restrict__ Y, int rows_per_block, int G)
{
    const int L = mr_logical(G);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int rs = min(L * rows_per_block, n), re = min(rs + rows_per_block, n);
    const int cl = lane < s ? lane : 0;
    if constexpr (sizeof(T) == 8) {
        if (s % 2 == 0) {  // two nonzeros per gather (see mr_row_x2)
            const int c2 = 2 * (lane & 31);
            const bool pair = lane < 32 && c2 < s;
            const int cp = c2 < s ? c2 : 0;
            for (int i = rs + w; i < re; i += BS / kWave) {
                const double2 y = mr_row_x2(rowptr, col, val, i, [&](int j) {
                    return *(const double2*)(X + (size_t)j * s + cp);
                });
                if (pair) *(double2*)(Y + (size_t)i * s + cp) = y;
            }
            return;
        }
    }
    for (int i = rs + w; i < re; i += BS / kWave) {
        const T y = mr_row<T>(rowptr, col, val, i, [&](int j) { return X[(size_t)j * s + cl]; });
        if (lane < s) Y[(size_t)i * s + lane] = y;
    }
}

}  // namespace jpcg
