// Dense FP64 kernels of the learned warm start: the snapshot Gram matrix of
// the proper orthogonal decomposition (method of snapshots), the products
// that form the modes and decode coefficients, and the projections.
//
// Both are tall-skinny: n (grid rows, ~1e5) is large, the other dimensions
// are at most a few hundred.
//   dense_gram  C = A' B  (ka x kb): 64 x 64 output tiles, the n rows split in
//               fixed chunks, per-chunk partials summed in chunk order by a
//               second kernel (deterministic).
//   dense_gemm  C = A W   (n x m): 64 x 64 output tiles, the short k dimension
//               staged through LDS.
// Each thread owns a 4 x 4 block of outputs; operands are staged through LDS.
#include <algorithm>
#include <cstdint>
#include <mutex>

#include "context.hpp"

namespace jpcg {

constexpr int kT = 64;   // output tile
constexpr int kKT = 16;  // rows (gram) or k (gemm) per LDS stage

// Partial C_z = A[rows of chunk z]' B[rows of chunk z] for one 64 x 64 tile.
__global__ __launch_bounds__(256) void k_gram_partial(const double* __restrict__ A, int64_t n, int ka, int64_t lda,
                                                      const double* __restrict__ B, int kb, int64_t ldb,
                                                      double* __restrict__ part, int64_t chunk)
{
    __shared__ double As[kKT][kT];
    __shared__ double Bs[kKT][kT];
    const int ta = blockIdx.x, tb = blockIdx.y, z = blockIdx.z;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t r0 = (int64_t)z * chunk, r1 = std::min<int64_t>(n, r0 + chunk);
    double acc[4][4] = {};
    for (int64_t r = r0; r < r1; r += kKT) {
        // Stage kKT rows x 64 columns of A and of B (zero outside).
        for (int e = threadIdx.x; e < kKT * kT; e += 256) {
            const int rr = e / kT, cc = e % kT;
            const int64_t row = r + rr;
            const int ca = ta * kT + cc, cb = tb * kT + cc;
            As[rr][cc] = (row < r1 && ca < ka) ? A[row * lda + ca] : 0.0;
            Bs[rr][cc] = (row < r1 && cb < kb) ? B[row * ldb + cb] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < kKT; ++rr) {
            double av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = As[rr][ty * 4 + u];
                bv[u] = Bs[rr][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
        }
        __syncthreads();
    }
    double* out = part + (size_t)z * ka * kb;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = ta * kT + ty * 4 + u;
        if (i >= ka) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = tb * kT + tx * 4 + v;
            if (j < kb) out[(size_t)i * kb + j] = acc[u][v];
        }
    }
}

__global__ void k_sum_partials(const double* __restrict__ part, int nparts, int64_t count, double* __restrict__ C)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int z = 0; z < nparts; ++z) s += part[(size_t)z * count + e];
        C[e] = s;
    }
}

// C (n x m, ldc) = A (n x k, lda) W (k x m, row-major).
__global__ __launch_bounds__(256) void k_gemm_tall(const double* __restrict__ A, int64_t n, int k, int64_t lda,
                                                   const double* __restrict__ W, int m, double* __restrict__ C,
                                                   int64_t ldc)
{
    __shared__ double As[kT][kKT + 1];
    __shared__ double Ws[kKT][kT];
    const int64_t rb = (int64_t)blockIdx.x * kT;
    const int cb = blockIdx.y * kT;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < k; k0 += kKT) {
        for (int e = threadIdx.x; e < kT * kKT; e += 256) {
            const int rr = e / kKT, kk = e % kKT;
            const int64_t row = rb + rr;
            As[rr][kk] = (row < n && k0 + kk < k) ? A[row * lda + k0 + kk] : 0.0;
            const int wk = e / kT, wc = e % kT;
            Ws[wk][wc] = (k0 + wk < k && cb + wc < m) ? W[(size_t)(k0 + wk) * m + cb + wc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKT; ++kk) {
            double av[4], wv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = As[ty * 4 + u][kk];
                wv[u] = Ws[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], wv[v], acc[u][v]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t row = rb + ty * 4 + u;
        if (row >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int col = cb + tx * 4 + v;
            if (col < m) C[row * ldc + col] = acc[u][v];
        }
    }
}

// X (n x nb, row-major) = Phi (n x k, ldphi) c' with c_jl = scale_l coef_jl +
// shift_l (FP64; coef nb x k FP32 row-major): one thread per row, the
// coefficients staged in LDS.
__global__ __launch_bounds__(256) void k_decode(const double* __restrict__ Phi, int64_t n, int k, int64_t ldphi,
                                                const float* __restrict__ coef, int nb,
                                                const double* __restrict__ scale, const double* __restrict__ shift,
                                                double* __restrict__ X)
{
    extern __shared__ double cs[];  // nb x k
    for (int e = threadIdx.x; e < nb * k; e += blockDim.x) {
        const int l = e % k;
        double c = (double)coef[e];
        if (scale) c *= scale[l];
        if (shift) c += shift[l];
        cs[e] = c;
    }
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double* row = Phi + i * ldphi;
        for (int j = 0; j < nb; ++j) {
            double s = 0.0;
            for (int l = 0; l < k; ++l) s = fma(row[l], cs[j * k + l], s);
            X[i * nb + j] = s;
        }
    }
}

// Fixed scratch of the no-allocation Gram (the per-chunk partials): one copy
// per device, held until the process ends.  Host code never passes this name
// to a kernel; it uses the address hipGetSymbolAddress returns on the device.
constexpr size_t kGramScratchDoubles = (size_t)4 << 20;  // 32 MiB
static __device__ __align__(256) double scratch[kGramScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (which must be current),
// looked up once per device.
int scratch_address(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return CG_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CG_EHIP;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

constexpr int64_t kGramChunk = 2048;

int64_t gram_parts(int64_t n) { return std::max<int64_t>(1, (n + kGramChunk - 1) / kGramChunk); }

// C = A' B through the partials buffer `part` (gram_parts(n) * ka * kb doubles).
void gram_launch(const double* A, int64_t n, int ka, int64_t lda, const double* B, int kb, int64_t ldb,
                 double* C, double* part, hipStream_t st)
{
    const int nparts = (int)gram_parts(n);
    dim3 grid((ka + kT - 1) / kT, (kb + kT - 1) / kT, nparts);
    k_gram_partial<<<grid, 256, 0, st>>>(A, n, ka, lda, B, kb, ldb, part, kGramChunk);
    JPCG_HIP(hipGetLastError());
    const int64_t count = (int64_t)ka * kb;
    k_sum_partials<<<(int)std::min<int64_t>(4096, (count + 255) / 256), 256, 0, st>>>(part, nparts, count, C);
    JPCG_HIP(hipGetLastError());
}

}  // namespace jpcg

using namespace jpcg;

extern "C" {

int dense_gram(const double* A, int64_t n, int32_t ka, int64_t lda, const double* B, int32_t kb, int64_t ldb,
               double* C, void* stream)
{
    if (!A || !B || !C || n < 0 || ka <= 0 || kb <= 0 || lda < ka || ldb < kb) return CG_EINVAL;
    try {
        hipStream_t st = (hipStream_t)stream;
        double* part = nullptr;
        JPCG_HIP(hipMallocAsync((void**)&part, sizeof(double) * (size_t)gram_parts(n) * ka * kb, st));
        gram_launch(A, n, ka, lda, B, kb, ldb, C, part, st);
        JPCG_HIP(hipFreeAsync(part, st));
        return 0;
    } catch (const HipError& e) {
        return e.code == hipErrorOutOfMemory ? CG_ENOMEM : CG_EHIP;
    }
}

int dense_gram_noalloc(const double* A, int64_t n, int32_t ka, int64_t lda, const double* B, int32_t kb,
                       int64_t ldb, double* C, void* stream)
{
    if (!A || !B || !C || n < 0 || ka <= 0 || kb <= 0 || lda < ka || ldb < kb) return CG_EINVAL;
    if ((uint64_t)gram_parts(n) * (uint64_t)ka * (uint64_t)kb > kGramScratchDoubles) return CG_ESCRATCH;
    try {
        hipStream_t st = (hipStream_t)stream;
        int dev = -1;
        JPCG_HIP(hipGetDevice(&dev));
        if (st) {
            int sdev = -1;
            JPCG_HIP(hipStreamGetDevice(st, &sdev));
            if (sdev != dev) return CG_EINVAL;
        }
        double* part = nullptr;
        const int rc = scratch_address(dev, &part);
        if (rc) return rc;
        gram_launch(A, n, ka, lda, B, kb, ldb, C, part, st);
        return 0;
    } catch (const HipError&) {
        return CG_EHIP;
    }
}

int dense_gemm(const double* A, int64_t n, int32_t k, int64_t lda, const double* W, int32_t m, double* C,
               int64_t ldc, void* stream)
{
    if (!A || !W || !C || n < 0 || k <= 0 || m <= 0 || lda < k || ldc < m) return CG_EINVAL;
    try {
        hipStream_t st = (hipStream_t)stream;
        if (n == 0) return 0;
        dim3 grid((unsigned)((n + kT - 1) / kT), (m + kT - 1) / kT);
        k_gemm_tall<<<grid, 256, 0, st>>>(A, n, k, lda, W, m, C, ldc);
        JPCG_HIP(hipGetLastError());
        return 0;
    } catch (const HipError&) {
        return CG_EHIP;
    }
}

int pod_decode(const double* Phi, int64_t n, int32_t k, int64_t ldphi, const float* coef, int32_t nb,
               const double* scale, const double* shift, double* X, void* stream)
{
    if (!Phi || !coef || !X || n < 0 || k <= 0 || nb <= 0 || ldphi < k || (int64_t)nb * k > 4096) return CG_EINVAL;
    try {
        if (n == 0) return 0;
        const int grid = (int)std::min<int64_t>(4096, (n + 255) / 256);
        k_decode<<<grid, 256, sizeof(double) * nb * k, (hipStream_t)stream>>>(Phi, n, k, ldphi, coef, nb, scale, shift, X);
        JPCG_HIP(hipGetLastError());
        return 0;
    } catch (const HipError&) {
        return CG_EHIP;
    }
}

}  // extern "C"
