// Multi-RHS Jacobi-PCG: s <= 64 independent CG recurrences (one per column of
// a row-major N x s block) sharing one sparse product per iteration.
//
// Each column follows the FP64 oracle's loop exactly; the columns only share
// launches.  Layout: lane j of a wave owns column j, so a gathered row of X is
// one coalesced s * 8-byte load and a CSR value/index is a wave-uniform
// (scalar) load.  Every column's row sum runs in stored order with separate
// multiply and add, so spmm's column j equals the sequential CSR product.
//
// Per iteration (parity P), all captured in hipGraph chunks:
//   k_mr_pnew       p_j = z_j + beta_j p_j (active), z_j (first step) or p_j
//                   carried forward (frozen), elementwise
//   k_mr_direction  q = A p, partials of p_j'q_j (one gathered row of p per
//                   nonzero)
//   k_mr_scalars    one workgroup per column: sigma_j, alpha_j, breakdown
//   k_mr_update     x += alpha p, r -= alpha q, z = M^-1 r, partials of r'z, r'r
//   k_mr_scalars    one workgroup per column: continue-condition, breakdown,
//                   limit, beta
// A column whose recurrence residual passes is frozen (its p is carried
// forward unchanged) and waits; when no column is active the host runs one
// true-residual check for all waiting columns, exactly the oracle's check,
// and resumes replaced ones.  Each column's per-workgroup partials are
// reduced by that column's own workgroup of the scalar kernel, in a fixed
// order; whether any column is still active is read from the 64 statuses by
// every kernel that needs it.
#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <vector>

#include "spmm.hpp"

namespace jpcg {

enum ColStatus : int {
    COL_ACTIVE = 0,
    COL_PENDING = 1,  // recurrence residual passed; true residual not yet checked
    COL_CONVERGED = 2,
    COL_MAXIT = 3,
    COL_BREAKDOWN = 4,
    COL_ZERO = 5,     // b_j = 0
    COL_UNUSED = 6,   // lane >= s
};

constexpr int kCols = 64;

struct MrState {
    int kk;            // iterations completed (the next one is kk + 1, parity (kk + 1) & 1)
    int pad[3];
    int status[kCols];
    int iters[kCols];
    int repl[kCols];
    int first[kCols];  // next direction step is the first for this column (p = z)
    double rho[kCols];
    double alpha[kCols];
    double beta[kCols];
    double nb[kCols];
    double thr[kCols];
    double rr[kCols];
    double rr_true[kCols];
};

template <typename T>
struct MrArgs {
    int n, s;
    const int* __restrict__ rowptr;
    const int* __restrict__ col;
    const T* __restrict__ val;
    const T* __restrict__ dinv;
    const T* B;
    T* X;
    T* R;
    T* Z;
    T* P[2];
    T* Q;
    int G;
    int rows_per_block;
    double* part;  // [G][3][64]
    MrState* st;
    int maxit;
    double tol;
    const T* rowsum;  // FP32 solves: row sums of A (FP64 sums) for the row-sum-preserving product
    int confirm;      // 1: a passed recurrence test is confirmed on b - A x; 0: it ends the column
};

// Block-reduce K per-lane quantities over the waves (lane = column) and write
// them to part[L][k][lane].
template <int BS, int K>
__device__ __forceinline__ void mr_block_partials(double (&v)[K], double* part, int L)
{
    constexpr int NW = BS / kWave;
    __shared__ double lds[NW][K][kWave];
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int k = 0; k < K; ++k) lds[w][k][lane] = v[k];
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < NW; ++j) t += lds[j][k][lane];
            part[((size_t)L * K + k) * kWave + lane] = t;
        }
    }
}

// True in every thread if some column is active (each wave reads the 64
// statuses once).
__device__ __forceinline__ bool mr_any_active(const MrState* st)
{
    const int lane = threadIdx.x & (kWave - 1);
    return __ballot(st->status[lane] == COL_ACTIVE) != 0ull;
}

// Row-sum-preserving form of the same row product for the FP32 inner solve:
// y_i = sum_k a_ik (x_j - x_i) + s_i x_i with s_i the row sum (summed in
// FP64), so the near-constant modes of A are not lost to FP32 cancellation.
template <typename T, typename Gather>
__device__ __forceinline__ T mr_row_diff(const int* __restrict__ rowptr, const int* __restrict__ col,
                                         const T* __restrict__ val, const T* __restrict__ rowsum, int i, T xi,
                                         Gather gather)
{
    constexpr int B = kMrBatch;
    static_assert(B <= kCsrPad, "batch reads must stay within the padded arrays");
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
            if (k + u < k1) acc = fma_t(v[u], g[u] - xi, acc);
    }
    return fma_t(rowsum[i], xi, acc);
}

// Residual R = B - A X with Z = M^-1 R and partials (r'r, r'z, b'b) per column.
// mode 0: setup (every column; clears both P buffers), 1: check (only pending
// columns are rewritten), 2: report (nothing is written but the partials).
template <int BS, typename T>
__global__ __launch_bounds__(BS) void k_mr_residual(MrArgs<T> a, int mode)
{
    const int L = mr_logical(a.G);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int rs = min(L * a.rows_per_block, a.n), re = min(rs + a.rows_per_block, a.n);
    const int s = a.s;
    const bool used = lane < s;
    const int cl = used ? lane : 0;
    const bool write = used && (mode == 0 || (mode == 1 && a.st->status[lane] == COL_PENDING));
    double v[3] = {0.0, 0.0, 0.0};
    const T* __restrict__ X = a.X;
    for (int i = rs + w; i < re; i += BS / kWave) {
        const T ax = mr_row<T>(a.rowptr, a.col, a.val, i, [&](int j) { return X[(size_t)j * s + cl]; });
        const size_t o = (size_t)i * s + cl;
        const T bi = a.B[o];
        const T ri = bi - ax;
        const T zi = a.dinv[i] * ri;
        if (write) {
            a.R[o] = ri;
            a.Z[o] = zi;
        }
        if (mode == 0 && used) {
            a.P[0][o] = T(0);
            a.P[1][o] = T(0);
        }
        if (used) {
            v[0] += (double)ri * (double)ri;
            v[1] += (double)ri * (double)zi;
            v[2] += (double)bi * (double)bi;
        }
    }
    mr_block_partials<BS, 3>(v, a.part, L);
}

// p_new = z + beta p_old (active), z (first step) or p_old (frozen: carried
// forward), elementwise over the block's rows.
template <int BS, typename T>
__global__ __launch_bounds__(BS) void k_mr_pnew(MrArgs<T> a, int P)
{
    const MrState* st = a.st;
    if (!mr_any_active(st)) return;
    const int L = mr_logical(a.G);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int rs = min(L * a.rows_per_block, a.n), re = min(rs + a.rows_per_block, a.n);
    const int s = a.s;
    if (lane >= s) return;
    const int status = st->status[lane];
    const bool active = status == COL_ACTIVE;
    const bool first = active && st->first[lane];
    const T beta = (T)st->beta[lane];
    const T* __restrict__ Z = a.Z;
    const T* __restrict__ pold = a.P[P ^ 1];
    T* __restrict__ pnew = a.P[P];
    for (int i = rs + w; i < re; i += BS / kWave) {
        const size_t o = (size_t)i * s + lane;
        const T po = pold[o];
        pnew[o] = active ? (first ? Z[o] : fma_t(beta, po, Z[o])) : po;
    }
}

// q = A p_new (p_new from k_mr_pnew); partials of p_new'q for active columns.
template <int BS, typename T>
__global__ __launch_bounds__(BS) void k_mr_direction(MrArgs<T> a, int P)
{
    const MrState* st = a.st;
    if (!mr_any_active(st)) return;
    const int L = mr_logical(a.G);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int rs = min(L * a.rows_per_block, a.n), re = min(rs + a.rows_per_block, a.n);
    const int s = a.s;
    const bool used = lane < s;
    const int cl = used ? lane : 0;
    const bool active = used && st->status[lane] == COL_ACTIVE;
    const T* __restrict__ pnew = a.P[P];
    double v[1] = {0.0};
    if constexpr (sizeof(T) == 8) {
        if (s % 2 == 0) {  // two nonzeros per gather; lane = column pair in the lower half
            const int c2 = 2 * (lane & 31);
            const bool pair = lane < 32 && c2 < s;
            const int cp = c2 < s ? c2 : 0;
            const bool act0 = pair && st->status[cp] == COL_ACTIVE, act1 = pair && st->status[cp + 1] == COL_ACTIVE;
            double v0 = 0.0, v1 = 0.0;
            for (int i = rs + w; i < re; i += BS / kWave) {
                const size_t o = (size_t)i * s + cp;
                const double2 qi = mr_row_x2(a.rowptr, a.col, a.val, i, [&](int j) {
                    return *(const double2*)(pnew + (size_t)j * s + cp);
                });
                if (pair) {
                    *(double2*)(a.Q + o) = qi;
                    const double2 pi = *(const double2*)(pnew + o);
                    if (act0) v0 += pi.x * qi.x;
                    if (act1) v1 += pi.y * qi.y;
                }
            }
            // Back to lane = column for the block partials.
            const double w0 = __shfl(v0, lane >> 1), w1 = __shfl(v1, lane >> 1);
            v[0] = (lane & 1) ? w1 : w0;
            mr_block_partials<BS, 1>(v, a.part, L);
            return;
        }
    }
    for (int i = rs + w; i < re; i += BS / kWave) {
        const size_t o = (size_t)i * s + cl;
        auto gather = [&](int j) { return pnew[(size_t)j * s + cl]; };
        T qi;
        if constexpr (sizeof(T) == 4) qi = mr_row_diff<T>(a.rowptr, a.col, a.val, a.rowsum, i, pnew[o], gather);
        else qi = mr_row<T>(a.rowptr, a.col, a.val, i, gather);
        if (used) {
            a.Q[o] = qi;
            if (active) v[0] += (double)pnew[o] * (double)qi;
        }
    }
    mr_block_partials<BS, 1>(v, a.part, L);
}

// x += alpha p, r -= alpha q, z = M^-1 r for active columns; partials of r'z, r'r.
template <int BS, typename T>
__global__ __launch_bounds__(BS) void k_mr_update(MrArgs<T> a, int P)
{
    MrState* st = a.st;
    if (!mr_any_active(st)) return;
    const int L = mr_logical(a.G);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int rs = min(L * a.rows_per_block, a.n), re = min(rs + a.rows_per_block, a.n);
    const int s = a.s;
    const bool active = lane < s && st->status[lane] == COL_ACTIVE;
    if (L == 0 && threadIdx.x == 0) st->kk += 1;  // this iteration is being done
    const T alpha = (T)st->alpha[lane < s ? lane : 0];
    const T* __restrict__ p = a.P[P];
    double v[2] = {0.0, 0.0};
    if (active) {
        for (int i = rs + w; i < re; i += BS / kWave) {
            const size_t o = (size_t)i * s + lane;
            a.X[o] = fma_t(alpha, p[o], a.X[o]);
            const T ri = fma_t(-alpha, a.Q[o], a.R[o]);
            a.R[o] = ri;
            const T zi = a.dinv[i] * ri;
            a.Z[o] = zi;
            v[0] += (double)ri * (double)zi;
            v[1] += (double)ri * (double)ri;
        }
    }
    mr_block_partials<BS, 2>(v, a.part, L);
}

enum MrPhase : int { MR_SETUP = 0, MR_SIGMA = 1, MR_ITER = 2, MR_CHECK = 3, MR_REPORT = 4 };

// Column j's sums of the G per-workgroup partials of K quantities, in a fixed
// order; the totals are returned in every thread.
template <int BS, int K>
__device__ __forceinline__ void mr_column_sum(const double* part, int G, int j, double (&out)[K], double* lds)
{
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = 0.0;
    for (int g = threadIdx.x; g < G; g += BS) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] += part[((size_t)g * K + k) * kWave + j];
    }
    block_sum<BS, K>(out, lds);
}

// The per-column scalar steps: workgroup j owns column j's state.
template <typename T>
__global__ __launch_bounds__(256) void k_mr_scalars(MrArgs<T> a, int phase)
{
    __shared__ double lds[(256 / kWave) * 3];
    MrState* st = a.st;
    const int j = blockIdx.x;
    if (phase == MR_SETUP && j == 0 && threadIdx.x == 0) st->kk = 0;
    if (j >= a.s) {
        if (phase == MR_SETUP && threadIdx.x == 0) st->status[j] = COL_UNUSED;
        return;
    }
    int status = st->status[j];
    if ((phase == MR_SIGMA || phase == MR_ITER) && status != COL_ACTIVE) return;
    if (phase == MR_CHECK && status != COL_PENDING) return;
    double g[3] = {0.0, 0.0, 0.0};
    if (phase == MR_SIGMA) {
        double t[1];
        mr_column_sum<256, 1>(a.part, a.G, j, t, lds);
        g[0] = t[0];
    } else if (phase == MR_ITER) {
        double t[2];
        mr_column_sum<256, 2>(a.part, a.G, j, t, lds);
        g[0] = t[0];
        g[1] = t[1];
    } else {
        mr_column_sum<256, 3>(a.part, a.G, j, g, lds);
    }
    if (threadIdx.x != 0) return;
    if (phase == MR_SETUP) {
        // g = (r'r, r'z, b'b) of r0
        st->repl[j] = 0;
        st->iters[j] = 0;
        st->first[j] = 1;
        st->beta[j] = 0.0;
        st->alpha[j] = 0.0;
        const double nb = sqrt(g[2]);
        st->nb[j] = nb;
        st->thr[j] = a.tol * nb;
        st->rr[j] = g[0];
        st->rho[j] = g[1];
        st->rr_true[j] = -1.0;
        if (nb == 0.0) {
            status = COL_ZERO;
            st->rr_true[j] = 0.0;
        } else if (sqrt(g[0]) <= a.tol * nb) {
            status = COL_CONVERGED;
            st->rr_true[j] = g[0];
        } else {
            status = COL_ACTIVE;
        }
    } else if (phase == MR_SIGMA) {
        const double sigma = g[0];
        if (!(sigma > 0.0) || !isfinite(sigma)) status = COL_BREAKDOWN;
        else st->alpha[j] = st->rho[j] / sigma;
    } else if (phase == MR_ITER) {
        // g = (r'z, r'r) after the update: the oracle's order of tests.
        st->iters[j] += 1;
        st->first[j] = 0;
        st->rr[j] = g[1];
        if (sqrt(g[1]) <= st->thr[j]) {
            status = a.confirm ? COL_PENDING : COL_CONVERGED;
            if (!a.confirm) st->rr_true[j] = g[1];
        } else if (!(g[0] > 0.0) || !isfinite(g[0])) {
            status = COL_BREAKDOWN;
        } else if (st->iters[j] >= a.maxit) {
            status = COL_MAXIT;
        } else {
            st->beta[j] = g[0] / st->rho[j];
            st->rho[j] = g[0];
        }
    } else if (phase == MR_CHECK) {
        // g = (r'r, r'z, b'b) of the true residual; r, z were replaced for pending columns.
        if (sqrt(g[0]) <= st->thr[j]) {
            status = COL_CONVERGED;
            st->rr_true[j] = g[0];
        } else if (!(g[1] > 0.0) || !isfinite(g[1])) {
            status = COL_BREAKDOWN;
        } else if (st->iters[j] >= a.maxit) {
            status = COL_MAXIT;
        } else {
            status = COL_ACTIVE;
            st->repl[j] += 1;
            st->beta[j] = g[1] / st->rho[j];
            st->rho[j] = g[1];
        }
    } else {  // MR_REPORT: true residual of the returned x for every column
        if (status != COL_ZERO) st->rr_true[j] = g[0];
    }
    st->status[j] = status;
}

// Mixed form, outer step: B32 = R64 / ||r_j|| for the columns still active
// in the FP64 state (0 for the others), X32 = 0.
__global__ void k_mr_scale(int n, int s, const double* __restrict__ r64, const MrState* st64,
                           float* __restrict__ b32, float* __restrict__ x32)
{
    const int lane = threadIdx.x & (kWave - 1);
    if (lane >= s) return;
    const bool active = st64->status[lane] == COL_ACTIVE;
    const double nr = sqrt(st64->rr[lane]);
    const double inv = active && nr > 0.0 ? 1.0 / nr : 0.0;
    for (int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < n; i += gridDim.x * (blockDim.x / kWave)) {
        const size_t o = (size_t)i * s + lane;
        b32[o] = (float)(r64[o] * inv);
        x32[o] = 0.0f;
    }
}

// Mixed form: X64 += ||r_j|| X32 for the columns that were active.
__global__ void k_mr_fold(int n, int s, double* __restrict__ x64, const float* __restrict__ x32, const MrState* st64)
{
    const int lane = threadIdx.x & (kWave - 1);
    if (lane >= s || st64->status[lane] != COL_ACTIVE) return;
    const double nr = sqrt(st64->rr[lane]);
    for (int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < n; i += gridDim.x * (blockDim.x / kWave)) {
        const size_t o = (size_t)i * s + lane;
        x64[o] = fma(nr, (double)x32[o], x64[o]);
    }
}

// x_j = 0 for columns with b_j = 0.
template <typename T>
__global__ void k_mr_zero_cols(MrArgs<T> a)
{
    const int lane = threadIdx.x & (kWave - 1);
    if (lane >= a.s || a.st->status[lane] != COL_ZERO) return;
    for (int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < a.n;
         i += gridDim.x * (blockDim.x / kWave))
        a.X[(size_t)i * a.s + lane] = T(0);
}

constexpr int kMrBS = 512;

}  // namespace jpcg

// Multi-RHS solver state hanging off a context, for one block width s and
// one precision (FP64, or the FP32 inner solver of the mixed form).
struct cg_multi {
    int s = 0, G = 0, chunk = 0;
    bool fp32 = false;
    void* work = nullptr;  // R, Z, P0, P1, Q, and the solver's own B, X: 7 N s values
    double* part = nullptr;
    jpcg::MrState* st = nullptr;
    jpcg::MrState* hst = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t ev = nullptr;
    jpcg::MrArgs<double> args{};
    jpcg::MrArgs<float> args32{};
};

namespace jpcg {

static void destroy_multi(cg_multi* m)
{
    if (!m) return;
    for (auto& e : m->exec)
        if (e) (void)hipGraphExecDestroy(e);
    if (m->ev) (void)hipEventDestroy(m->ev);
    if (m->work) (void)hipFree(m->work);
    if (m->part) (void)hipFree(m->part);
    if (m->st) (void)hipFree(m->st);
    if (m->hst) (void)hipHostFree(m->hst);
    delete m;
}

static void mr_launch(const void* fn, int grid, int bs, hipStream_t st, void** args)
{
    JPCG_HIP(hipLaunchKernel(fn, dim3(grid), dim3(bs), args, 0, st));
}

template <typename T>
static MrArgs<T>& margs(cg_multi* m);
template <>
MrArgs<double>& margs<double>(cg_multi* m) { return m->args; }
template <>
MrArgs<float>& margs<float>(cg_multi* m) { return m->args32; }

// The multi-column product's grid: workgroups per CU.  Without autotune the
// default (2); with it, the first use times the 64-column product at 1, 2, 3,
// 4, 6 and 8 workgroups per CU (rows split evenly, XCD-aware order) and keeps
// the fastest.
constexpr int kSpmmDefaultWpc = 2;

int spmm_blocks_per_cu(cg_ctx* c)
{
    if (c->spmm_wpc > 0) return c->spmm_wpc;
    if (!c->opts.autotune) return c->spmm_wpc = kSpmmDefaultWpc;
    const int s = kCols;
    const size_t nb = sizeof(double) * (size_t)c->n * s;
    double *X = nullptr, *Y = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best_w = kSpmmDefaultWpc;
    float best = 1e30f;
    try {
        JPCG_HIP(hipMalloc(&X, nb));
        JPCG_HIP(hipMalloc(&Y, nb));
        JPCG_HIP(hipMemsetAsync(X, 0, nb, c->stream));
        JPCG_HIP(hipEventCreate(&e0));
        JPCG_HIP(hipEventCreate(&e1));
        int n = c->n;
        for (int w : {1, 2, 3, 4, 6, 8}) {
            int G = std::max(8, std::min(c->cus * w, (c->n + 15) / 16) / 8 * 8);
            int rpb = (c->n + G - 1) / G;
            void* args[] = {&n, (void*)&s, &c->rowptr, &c->col, &c->val, &X, &Y, &rpb, &G};
            JPCG_HIP(hipLaunchKernel((const void*)k_spmm<512, double>, dim3(G), dim3(512), args, 0, c->stream));
            JPCG_HIP(hipEventRecord(e0, c->stream));
            constexpr int kReps = 8;
            for (int r = 0; r < kReps; ++r)
                JPCG_HIP(hipLaunchKernel((const void*)k_spmm<512, double>, dim3(G), dim3(512), args, 0, c->stream));
            JPCG_HIP(hipEventRecord(e1, c->stream));
            JPCG_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            JPCG_HIP(hipEventElapsedTime(&ms, e0, e1));
            ms /= kReps;
            if (ms < best) {
                best = ms;
                best_w = w;
            }
        }
    } catch (...) {
        if (X) (void)hipFree(X);
        if (Y) (void)hipFree(Y);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipFree(X);
    (void)hipFree(Y);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tuned_spmm_us = best * 1e3;
    return c->spmm_wpc = best_w;
}

template <typename T>
static cg_multi* make_multi(cg_ctx* c, int s)
{
    const int wpc = spmm_blocks_per_cu(c);
    cg_multi* m = new cg_multi();
    try {
        m->s = s;
        m->fp32 = sizeof(T) == 4;
        m->chunk = 8;
        m->G = std::max(8, std::min(c->cus * wpc, (c->n + 63) / 64) / 8 * 8);
        const size_t ns = (size_t)c->n * s;
        JPCG_HIP(hipMalloc(&m->work, sizeof(T) * ns * 7));
        JPCG_HIP(hipMalloc(&m->part, sizeof(double) * (size_t)m->G * 3 * kWave));
        JPCG_HIP(hipMalloc(&m->st, sizeof(MrState)));
        JPCG_HIP(hipHostMalloc(&m->hst, sizeof(MrState), hipHostMallocDefault));
        JPCG_HIP(hipEventCreateWithFlags(&m->ev, hipEventDisableTiming));
        JPCG_HIP(hipMemsetAsync(m->work, 0, sizeof(T) * ns * 7, c->stream));
        JPCG_HIP(hipMemsetAsync(m->st, 0, sizeof(MrState), c->stream));
        MrArgs<T>& a = margs<T>(m);
        T* w = (T*)m->work;
        a.n = c->n;
        a.s = s;
        a.rowptr = c->rowptr;
        a.col = c->col;
        if constexpr (sizeof(T) == 4) {
            a.val = c->val32;
            a.dinv = c->dinv32;
            a.rowsum = c->rowsum32;
        } else {
            a.val = c->val;
            a.dinv = c->dinv;
            a.rowsum = nullptr;
        }
        a.R = w;
        a.Z = w + ns;
        a.P[0] = w + 2 * ns;
        a.P[1] = w + 3 * ns;
        a.Q = w + 4 * ns;
        a.B = w + 5 * ns;
        a.X = w + 6 * ns;
        a.G = m->G;
        a.rows_per_block = (c->n + m->G - 1) / m->G;
        a.part = m->part;
        a.st = m->st;
        a.maxit = c->n;
        a.tol = 1e-10;
        a.confirm = 1;
        JPCG_HIP(hipStreamSynchronize(c->stream));
        return m;
    } catch (...) {
        destroy_multi(m);
        throw;
    }
}

// (Re)capture the chunk graphs; tol, maxit and confirm are kernel arguments.
template <typename T>
static void capture_multi(cg_multi* m)
{
    for (auto& e : m->exec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    MrArgs<T>& args = margs<T>(m);
    hipStream_t cap;
    JPCG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    for (int par = 0; par < 2; ++par) {
        hipGraph_t graph;
        JPCG_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        for (int it = 0; it < m->chunk; ++it) {
            int P = (par + it) & 1, ph_sig = MR_SIGMA, ph_it = MR_ITER;
            void* a0[] = {&args, &P};
            mr_launch((const void*)k_mr_pnew<kMrBS, T>, m->G, kMrBS, cap, a0);
            mr_launch((const void*)k_mr_direction<kMrBS, T>, m->G, kMrBS, cap, a0);
            void* a1[] = {&args, &ph_sig};
            mr_launch((const void*)k_mr_scalars<T>, kCols, 256, cap, a1);
            mr_launch((const void*)k_mr_update<kMrBS, T>, m->G, kMrBS, cap, a0);
            void* a2[] = {&args, &ph_it};
            mr_launch((const void*)k_mr_scalars<T>, kCols, 256, cap, a2);
        }
        JPCG_HIP(hipStreamEndCapture(cap, &graph));
        hipError_t e = hipGraphInstantiate(&m->exec[par], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        JPCG_HIP(e);
    }
    JPCG_HIP(hipStreamDestroy(cap));
}

void free_multi(cg_ctx* c)
{
    destroy_multi(c->multi);
    c->multi = nullptr;
    destroy_multi(c->multi32);
    c->multi32 = nullptr;
}

static MrState mr_read(cg_ctx* c, cg_multi* m)
{
    JPCG_HIP(hipMemcpyAsync(m->hst, m->st, sizeof(MrState), hipMemcpyDeviceToHost, c->stream));
    JPCG_HIP(hipStreamSynchronize(c->stream));
    return *m->hst;
}

// The context's multi-RHS solver of precision T for block width s, with its
// graphs captured for (tol, maxit, confirm).
template <typename T>
static cg_multi* multi_for(cg_ctx* c, int s, double tol, int maxit, int confirm)
{
    cg_multi*& slot = sizeof(T) == 4 ? c->multi32 : c->multi;
    if (!slot || slot->s != s) {
        destroy_multi(slot);
        slot = nullptr;
        slot = make_multi<T>(c, s);
    }
    MrArgs<T>& a = margs<T>(slot);
    if (!slot->exec[0] || a.tol != tol || a.maxit != maxit || a.confirm != confirm) {
        a.tol = tol;
        a.maxit = maxit;
        a.confirm = confirm;
        capture_multi<T>(slot);
    }
    return slot;
}

// One multi-RHS solve on the solver's own B and X: setup, chunks of
// iterations, true-residual checks of waiting columns (confirm = 1), and the
// final report.  Returns the final state.
template <typename T>
static MrState run_multi(cg_ctx* c, cg_multi* m)
{
    MrArgs<T>& args = margs<T>(m);
    hipStream_t st = c->stream;
    const int s = m->s;
    int mode = 0, ph = MR_SETUP;
    void* ra[] = {&args, &mode};
    mr_launch((const void*)k_mr_residual<kMrBS, T>, m->G, kMrBS, st, ra);
    void* sa[] = {&args, &ph};
    mr_launch((const void*)k_mr_scalars<T>, kCols, 256, st, sa);
    void* za[] = {&args};
    mr_launch((const void*)k_mr_zero_cols<T>, 256, 256, st, za);
    int next = 1;
    const long long guard = 4LL * args.maxit + 64;
    long long launched = 0;
    while (true) {
        MrState h = mr_read(c, m);
        // Iterations after the last column stopped returned early, so the
        // next iteration's parity comes from the device's count, not from
        // the number of iterations launched.
        next = h.kk + 1;
        bool active = false, pending = false;
        for (int j = 0; j < s; ++j) {
            active = active || h.status[j] == COL_ACTIVE;
            pending = pending || h.status[j] == COL_PENDING;
        }
        if (!active) {
            if (!pending) break;
            mode = 1;
            ph = MR_CHECK;
            mr_launch((const void*)k_mr_residual<kMrBS, T>, m->G, kMrBS, st, ra);
            mr_launch((const void*)k_mr_scalars<T>, kCols, 256, st, sa);
            continue;
        }
        if (launched > guard) throw HipError{hipErrorUnknown, "multi-RHS solver did not stop"};
        // Two chunks per poll keep the device busy while the host reads.
        JPCG_HIP(hipGraphLaunch(m->exec[next & 1], st));
        next += m->chunk;
        JPCG_HIP(hipGraphLaunch(m->exec[next & 1], st));
        next += m->chunk;
        launched += 2 * m->chunk;
    }
    if (args.confirm) {
        mode = 2;
        ph = MR_REPORT;
        mr_launch((const void*)k_mr_residual<kMrBS, T>, m->G, kMrBS, st, ra);
        mr_launch((const void*)k_mr_scalars<T>, kCols, 256, st, sa);
    }
    return mr_read(c, m);
}

static int col_code(int status)
{
    if (status == COL_MAXIT) return CG_MAXIT;
    if (status == COL_BREAKDOWN) return CG_BREAKDOWN;
    return CG_CONVERGED;
}

}  // namespace jpcg

using namespace jpcg;

extern "C" {

int spmm(cg_ctx* c, const double* X, double* Y, int32_t s)
{
    if (!c) return CG_EINVAL;
    if (!X || !Y || X == Y || s < 1 || s > kCols) return set_error(c, CG_EINVAL, "spmm: bad arguments");
    try {
        const int wpc = c->opts.autotune ? spmm_blocks_per_cu(c) : 4;
        const int G = std::max(8, std::min(c->cus * wpc, (c->n + 15) / 16) / 8 * 8);
        const int rpb = (c->n + G - 1) / G;
        int n = c->n;
        void* args[] = {&n, &s, &c->rowptr, &c->col, &c->val, &X, &Y, (void*)&rpb, (void*)&G};
        mr_launch((const void*)k_spmm<kMrBS, double>, G, kMrBS, c->stream, args);
        return 0;
    } catch (const HipError& e) {
        return set_error(c, CG_EHIP, std::string("spmm: ") + e.what + ": " + hipGetErrorString(e.code));
    }
}

int cg_solve_multi(cg_ctx* c, const double* B, double* X, int32_t s, double tol, int32_t maxit, cg_info* info)
{
    if (!c) return CG_EINVAL;
    if (!B || !X || B == X || s < 1 || s > kCols || !(tol >= 0.0) || !std::isfinite(tol))
        return set_error(c, CG_EINVAL, "cg_solve_multi: bad arguments");
    if (maxit <= 0) maxit = c->n;
    try {
        cg_multi* m = multi_for<double>(c, s, tol, maxit, 1);
        hipStream_t st = c->stream;
        const size_t nb = sizeof(double) * (size_t)c->n * s;
        JPCG_HIP(hipEventRecord(c->ev0, st));
        JPCG_HIP(hipMemcpyAsync((void*)m->args.B, B, nb, hipMemcpyDeviceToDevice, st));
        JPCG_HIP(hipMemcpyAsync(m->args.X, X, nb, hipMemcpyDeviceToDevice, st));
        const MrState h = run_multi<double>(c, m);
        JPCG_HIP(hipMemcpyAsync(X, m->args.X, nb, hipMemcpyDeviceToDevice, st));
        JPCG_HIP(hipEventRecord(c->ev1, st));
        JPCG_HIP(hipEventSynchronize(c->ev1));
        float ms = 0.f;
        JPCG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        int worst = CG_CONVERGED;
        for (int j = 0; j < s; ++j) {
            const int code = col_code(h.status[j]);
            worst = std::max(worst, code);
            if (info) {
                cg_info& o = info[j];
                o.iters = h.iters[j];
                o.status = code;
                o.replacements = h.repl[j];
                o.outer = 0;
                o.relres_recur = h.nb[j] > 0 ? std::sqrt(h.rr[j]) / h.nb[j] : 0.0;
                o.relres_true = h.nb[j] > 0 ? std::sqrt(h.rr_true[j]) / h.nb[j] : 0.0;
                o.seconds = ms * 1e-3;
            }
        }
        return worst;
    } catch (const HipError& e) {
        return set_error(c, CG_EHIP, std::string("cg_solve_multi: ") + e.what + ": " + hipGetErrorString(e.code));
    }
}

int cg_solve_multi_mixed(cg_ctx* c, const double* B, double* X, int32_t s, double tol, int32_t maxit_outer,
                         double tol_inner, int32_t maxit_inner, cg_info* info)
{
    if (!c) return CG_EINVAL;
    if (!c->val32) return set_error(c, CG_EINVAL, "cg_solve_multi_mixed: the context was created without fp32_copy");
    if (!B || !X || B == X || s < 1 || s > kCols || !(tol >= 0.0) || !std::isfinite(tol) || !(tol_inner >= 0.0) ||
        !std::isfinite(tol_inner))
        return set_error(c, CG_EINVAL, "cg_solve_multi_mixed: bad arguments");
    if (maxit_outer <= 0) maxit_outer = 50;
    if (maxit_inner <= 0) maxit_inner = c->n;
    if (tol_inner == 0.0) tol_inner = 1e-3;
    try {
        // The FP64 solver holds B, X and the outer residual (its setup phase
        // is the FP64 test); the FP32 solver runs the inner solves.
        cg_multi* m64 = multi_for<double>(c, s, tol, c->n, 1);
        cg_multi* m32 = multi_for<float>(c, s, tol_inner, maxit_inner, 0);
        hipStream_t st = c->stream;
        const size_t nb = sizeof(double) * (size_t)c->n * s;
        JPCG_HIP(hipEventRecord(c->ev0, st));
        JPCG_HIP(hipMemcpyAsync((void*)m64->args.B, B, nb, hipMemcpyDeviceToDevice, st));
        JPCG_HIP(hipMemcpyAsync(m64->args.X, X, nb, hipMemcpyDeviceToDevice, st));
        int final_status[kCols];
        int inner_iters[kCols] = {};
        for (int j = 0; j < kCols; ++j) final_status[j] = -1;
        int n = c->n;
        const int eg = std::min(4096, (c->n + 3) / 4);
        MrState h{};
        int outer = 0;
        for (;; ++outer) {
            // r = b - A x in FP64 and the per-column tests.
            int mode = 0, ph = MR_SETUP;
            void* ra[] = {&m64->args, &mode};
            mr_launch((const void*)k_mr_residual<kMrBS, double>, m64->G, kMrBS, st, ra);
            void* sa[] = {&m64->args, &ph};
            mr_launch((const void*)k_mr_scalars<double>, kCols, 256, st, sa);
            if (outer == 0) {  // x_j = 0 for b_j = 0
                void* za[] = {&m64->args};
                mr_launch((const void*)k_mr_zero_cols<double>, 256, 256, st, za);
            }
            h = mr_read(c, m64);
            bool any = false, changed = false;
            for (int j = 0; j < s; ++j) {
                if (final_status[j] >= 0) {  // decided earlier: keep it out of the inner solves
                    if (h.status[j] == COL_ACTIVE) {
                        h.status[j] = final_status[j] == CG_BREAKDOWN ? COL_BREAKDOWN : COL_MAXIT;
                        changed = true;
                    }
                    continue;
                }
                if (!(h.rr[j] == h.rr[j]) || !(h.nb[j] == h.nb[j])) {  // NaN input
                    final_status[j] = CG_BREAKDOWN;
                    h.status[j] = COL_BREAKDOWN;
                    changed = true;
                } else if (h.status[j] != COL_ACTIVE) {
                    final_status[j] = CG_CONVERGED;  // converged (or b_j = 0)
                } else if (outer >= maxit_outer) {
                    final_status[j] = CG_MAXIT;
                    h.status[j] = COL_MAXIT;
                    changed = true;
                } else {
                    any = true;
                }
            }
            if (!any) break;
            if (changed) {
                int* dstatus = (int*)((char*)m64->st + offsetof(MrState, status));
                JPCG_HIP(hipMemcpyAsync(dstatus, h.status, sizeof(int) * kCols, hipMemcpyHostToDevice, st));
            }
            // Scaled residual of the active columns into the FP32 solver.
            const double* r64 = m64->args.R;
            void* ka[] = {&n, &s, &r64, &m64->st, &m32->args32.B, &m32->args32.X};
            mr_launch((const void*)k_mr_scale, eg, 256, st, ka);
            const MrState hi = run_multi<float>(c, m32);
            for (int j = 0; j < s; ++j)
                if (h.status[j] == COL_ACTIVE) inner_iters[j] += hi.iters[j];
            const float* x32 = m32->args32.X;
            void* fa[] = {&n, &s, &m64->args.X, &x32, &m64->st};
            mr_launch((const void*)k_mr_fold, eg, 256, st, fa);
        }
        JPCG_HIP(hipMemcpyAsync(X, m64->args.X, nb, hipMemcpyDeviceToDevice, st));
        JPCG_HIP(hipEventRecord(c->ev1, st));
        JPCG_HIP(hipEventSynchronize(c->ev1));
        float ms = 0.f;
        JPCG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        int worst = CG_CONVERGED;
        for (int j = 0; j < s; ++j) {
            const int code = final_status[j] < 0 ? CG_MAXIT : final_status[j];
            worst = std::max(worst, code);
            if (info) {
                cg_info& o = info[j];
                o.iters = inner_iters[j];
                o.status = code;
                o.replacements = 0;
                o.outer = outer;
                const double rel = h.nb[j] > 0 ? std::sqrt(h.rr[j]) / h.nb[j] : 0.0;
                o.relres_recur = rel;
                o.relres_true = rel;
                o.seconds = ms * 1e-3;
            }
        }
        return worst;
    } catch (const HipError& e) {
        return set_error(c, CG_EHIP,
                         std::string("cg_solve_multi_mixed: ") + e.what + ": " + hipGetErrorString(e.code));
    }
}

}  // extern "C"
