// CSR-stream sparse products over "tiles" of whole rows.
//
// A tile is a run of consecutive rows whose nonzeros fit 64 * NPL slots (or a
// single longer row).  One wave owns a tile at a time:
//   1. each lane loads NPL (value, column) pairs at stride 64 -- every load is
//      coalesced and all of them are independent, so a lane has 2 NPL loads
//      plus NPL gathers in flight instead of a dependent chain per row;
//   2. the products a_ij * x_j go to the wave's slice of LDS;
//   3. one lane per row adds its row's products in stored column order.
// Step 3 adds in the same order as a sequential CSR row sum and the products
// are rounded on their own, so y = A x is bitwise the plain sequential result.
// Rows longer than a tile take a vector path: the whole wave strides over the
// row and reduces with a butterfly.
//
// Workgroups own equal, contiguous runs of tiles.
#pragma once

#include <vector>

#include "common.hpp"

namespace jpcg {

// A tile: rows [r0, r1) holding nonzeros [k0, k1).  Workgroup L owns tiles
// [L * per_block, (L + 1) * per_block) -- an arithmetic map, so finding a
// tile costs one 16-byte load and no index chase.
//
// Narrow column indices: when every column of a tile lies within 32 Ki of
// the tile's first row (true of any banded ordering of a mesh operator up to
// a bandwidth of about 32 Ki), col16[k] = col[k] - r0 + kCol16Bias is read
// instead of col[k]: 10 bytes per nonzero instead of 12 for an FP64 product,
// the same columns, the same sums.  col16 is null where it does not fit.
constexpr int kCol16Bias = 32768;

struct TileMap {
    const int4* tiles;
    int T;
    int per_block;
    const unsigned short* col16;
};

// Host: cut rows into tiles of at most `cap` nonzeros (a longer row forms a
// tile of its own).
inline void build_tiles(const std::vector<int>& rowptr, int cap, std::vector<int4>& tiles)
{
    const int n = (int)rowptr.size() - 1;
    tiles.clear();
    int r = 0;
    while (r < n) {
        const int k0 = rowptr[r];
        int e = r + 1;
        if (rowptr[e] - k0 <= cap) {
            while (e < n && rowptr[e + 1] - k0 <= cap) ++e;
        }
        tiles.push_back(int4{r, e, k0, rowptr[e]});
        r = e;
    }
}

// One workgroup per tile: col16[k] = col[k] - r0 + kCol16Bias for the tile's
// nonzeros; *wide = 1 if an offset does not fit 16 bits.
static __global__ void col16_kernel(const int4* __restrict__ tiles, const int* __restrict__ col,
                                    unsigned short* __restrict__ col16, int* wide)
{
    const int4 d = tiles[blockIdx.x];
    for (int k = d.z + (int)threadIdx.x; k < d.w; k += blockDim.x) {
        const int off = col[k] - d.x + kCol16Bias;
        if (off < 0 || off > 0xffff) {
            *wide = 1;
        } else {
            col16[k] = (unsigned short)off;
        }
    }
}

// Narrow column indices (device) for T device tiles over the device column
// array col[nnz], or null when some column lies too far from its tile's first
// row.  Synchronises the stream.
static unsigned short* make_col16(hipStream_t stream, const int4* tiles, int T, const int* col, int64_t nnz)
{
    if (T <= 0 || nnz <= 0) return nullptr;
    unsigned short* col16 = nullptr;
    int* wide = nullptr;
    int hwide = 0;
    try {
        JPCG_HIP(hipMalloc(&col16, sizeof(unsigned short) * nnz));
        JPCG_HIP(hipMalloc(&wide, sizeof(int)));
        JPCG_HIP(hipMemsetAsync(wide, 0, sizeof(int), stream));
        col16_kernel<<<T, 256, 0, stream>>>(tiles, col, col16, wide);
        JPCG_HIP(hipGetLastError());
        JPCG_HIP(hipMemcpyAsync(&hwide, wide, sizeof(int), hipMemcpyDeviceToHost, stream));
        JPCG_HIP(hipStreamSynchronize(stream));
    } catch (...) {
        if (col16) (void)hipFree(col16);
        if (wide) (void)hipFree(wide);
        throw;
    }
    (void)hipFree(wide);
    if (hwide) {
        (void)hipFree(col16);
        return nullptr;
    }
    return col16;
}

// Sum prod[a..b) in order; eight LDS reads are issued per batch.
template <typename T>
__device__ __forceinline__ T lds_row_sum(const T* prod, int a, int b)
{
    T s = T(0);
    int k = a;
    for (; k + 8 <= b; k += 8) {
        T t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = prod[k + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += t[u];
    }
    for (; k < b; ++k) s += prod[k];
    return s;
}

// The row-sum-preserving row sum: sum of prod[k] * (px[k] - xi) over [a, b)
// in order, with eight of each LDS array read per batch.
template <typename T>
__device__ __forceinline__ T lds_row_sum_diff(const T* prod, const T* px, int a, int b, T xi)
{
    T s = T(0);
    int k = a;
    for (; k + 8 <= b; k += 8) {
        T t[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            t[u] = prod[k + u];
            y[u] = px[k + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s += t[u] * (y[u] - xi);
    }
    for (; k < b; ++k) s += prod[k] * (px[k] - xi);
    return s;
}

// Visit every row of the workgroup's tiles.
//   gather(j)       raw operand(s) of column j (type GV), loaded per nonzero
//   value(g)        the vector entry x_j from the raw operands (may use scalars
//                   that the prologue sets)
//   pre(i)          raw operand(s) of row i for the row step (type PV)
//   row(i, y, pv)   consumes y_i = (A x)_i; called by one lane per row
//   prologue()      runs once per wave after the wave's first gathers are
//                   issued (or at the end if the wave has no tile); it may
//                   load and reduce scalars that value/row depend on, so that
//                   latency overlaps the gathers.  Returning false ends the
//                   wave's work.
// With DIFF the product is evaluated in row-sum-preserving form,
//   y_i = sum_{j != i} a_ij (x_j - x_i) + s_i x_i,   s_i = sum_j a_ij,
// with self(pv) giving the row's own x_i and rowsum[i] = s_i (computed in
// double, stored in T).  A constant vector then costs no cancellation, which
// keeps a float product accurate on the smooth near-null modes of a
// Neumann-plus-mass operator.  `prod` is this wave's LDS slice of 64 * NPL
// values (twice that with DIFF).
// VT is the type of the stored values (T, or float for an FP64 product that
// streams FP32 values); products and sums are in T.
template <int NPL, typename T, bool DIFF = false, typename VT = T, typename Gather, typename Value, typename Pre,
          typename Self, typename Row, typename Prologue>
__device__ __forceinline__ void tile_rows_x(const int* __restrict__ rowptr, const int* __restrict__ col,
                                            const VT* __restrict__ val, const T* __restrict__ rowsum,
                                            const TileMap& tm, int L, T* prod, Gather gather, Value value, Pre pre,
                                            Self self, Row row, Prologue prologue)
{
    constexpr int CAP = kWave * NPL;
    using GV = decltype(gather(0));
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    const int tb = L * tm.per_block;
    const int t1 = min(tb + tm.per_block, tm.T);
    T* px = prod + CAP;  // DIFF: gathered entries next to the values
    const unsigned short* __restrict__ c16 = tm.col16;
    bool ready = false;
    for (int t = tb + wave; t < t1; t += nwaves) {
        const int4 d = tm.tiles[t];
        const int r0 = d.x, r1 = d.y, k0 = d.z, k1 = d.w;
        if (k1 - k0 <= CAP) {
            // Branch-free: every slot loads (slots past the tile read entry 0 and
            // are zeroed), so all 2*NPL streaming loads issue before the first
            // gather and all NPL gathers issue before the first product.
            const int i0 = r0 + lane;
            const bool has_row = i0 < r1;
            const int ic = has_row ? i0 : r0;
            const int ra = rowptr[ic], rb = rowptr[ic + 1];
            const auto pv = pre(ic);
            T v[NPL];
            GV g[NPL];
            int c[NPL];
            if (c16) {
                const int base = r0 - kCol16Bias;
#pragma unroll
                for (int j = 0; j < NPL; ++j) {
                    const int k = k0 + lane + kWave * j;
                    const int kk = k < k1 ? k : 0;
                    v[j] = (T)val[kk];
                    c[j] = base + (int)c16[kk];
                }
            } else {
#pragma unroll
                for (int j = 0; j < NPL; ++j) {
                    const int k = k0 + lane + kWave * j;
                    const int kk = k < k1 ? k : 0;
                    v[j] = (T)val[kk];
                    c[j] = col[kk];
                }
            }
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
                const bool in = k0 + lane + kWave * j < k1;
                c[j] = in ? c[j] : 0;
                v[j] = in ? v[j] : T(0);
            }
#pragma unroll
            for (int j = 0; j < NPL; ++j) g[j] = gather(c[j]);
            if (!ready) {
                if (!prologue()) return;
                ready = true;
            }
            if constexpr (DIFF) {
#pragma unroll
                for (int j = 0; j < NPL; ++j) {
                    prod[lane + kWave * j] = v[j];
                    px[lane + kWave * j] = value(g[j]);
                }
            } else {
#pragma unroll
                for (int j = 0; j < NPL; ++j) prod[lane + kWave * j] = v[j] * value(g[j]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int i = i0; i < r1; i += kWave) {  // more than 64 rows only in tiny-row tiles
                const auto pvi = i == i0 ? pv : pre(i);
                const int a = (i == i0 ? ra : rowptr[i]) - k0, b = (i == i0 ? rb : rowptr[i + 1]) - k0;
                if constexpr (DIFF) {
                    const T xi = self(pvi);
                    const T s = lds_row_sum_diff(prod, px, a, b, xi);
                    row(i, s + rowsum[i] * xi, pvi);
                } else {
                    row(i, lds_row_sum(prod, a, b), pvi);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            // One row longer than a tile (r1 == r0 + 1).
            if (!ready) {
                if (!prologue()) return;
                ready = true;
            }
            const auto pvi = pre(r0);
            T acc = T(0);
            auto colk = [&](int k) { return c16 ? r0 - kCol16Bias + (int)c16[k] : col[k]; };
            if constexpr (DIFF) {
                const T xi = self(pvi);
                for (int k = k0 + lane; k < k1; k += kWave) acc += (T)val[k] * (value(gather(colk(k))) - xi);
            } else {
                for (int k = k0 + lane; k < k1; k += kWave) acc += (T)val[k] * value(gather(colk(k)));
            }
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
            if constexpr (DIFF) acc += rowsum[r0] * self(pvi);
            if (lane == 0) row(r0, acc, pvi);
        }
    }
    if (!ready) prologue();
}

struct NoSelf {
    template <typename P>
    __device__ __forceinline__ int operator()(const P&) const { return 0; }
};

// The plain (non-DIFF) walk.
template <int NPL, typename T, typename Gather, typename Value, typename Pre, typename Row, typename Prologue>
__device__ __forceinline__ void tile_rows(const int* __restrict__ rowptr, const int* __restrict__ col,
                                          const T* __restrict__ val, const TileMap& tm, int L, T* prod,
                                          Gather gather, Value value, Pre pre, Row row, Prologue prologue)
{
    tile_rows_x<NPL, T, false>(rowptr, col, val, (const T*)nullptr, tm, L, prod, gather, value, pre, NoSelf{}, row,
                               prologue);
}

struct Pair2 {
    double a, b;
};

struct NoPre {
    __device__ __forceinline__ int operator()(int) const { return 0; }
};

struct NoPrologue {
    __device__ __forceinline__ bool operator()() const { return true; }
};

template <typename T>
struct Ident {
    __device__ __forceinline__ T operator()(T g) const { return g; }
};

}  // namespace jpcg
