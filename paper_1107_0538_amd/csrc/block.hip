// Block Jacobi-PCG for s <= 64 right-hand sides: O'Leary's block conjugate
// gradients (the paper's CG iteration, Section IV, on a block of vectors) in
// the breakdown-free form of Ji and Li, whose search blocks are
// orthonormalised with rank revelation by shifted Cholesky QR (Fukaya et al.).
//
// Per iteration, on N x 64 row-major FP64 blocks (columns >= s are zero):
//   Q = A P                                  k_bc_spmm (row products, lane = column)
//   Gamma = P'Q, Psi = P'R                   k_bc_gram<2> + k_bc_sum
//   alpha = Gamma^-1 Psi                     k_bc_alpha (one wave: Cholesky over
//                                            the live columns, inverse factor)
//   X += P alpha                             k_bc_gemm<XUP>
//   R -= Q alpha, Z = M^-1 R, ||r_j||^2      k_bc_gemm<RUP> + k_bc_sum
//   Q'Z                                      k_bc_gram<1> + k_bc_sum
//   test, beta = -Gamma^-1 Q'Z               k_bc_beta
//   W = Z + P beta                           k_bc_gemm<DIR>
//   three CholeskyQR passes of W -> P        (k_bc_gram<1>, k_bc_sum, k_bc_orth,
//                                            k_bc_gemm<APPLY>) x 3
// The Gram and block-times-64x64 products are dense contractions: they run on
// the FP64 matrix cores (v_mfma_f64_16x16x4f64), operands straight from
// global memory into the fragment layout.  The 64 x 64 factorisations run in
// one wave of one workgroup, the matrix held in registers.  All kernels of an
// iteration are captured in hipGraph chunks and return at entry once the
// state is no longer RUN; the host confirms a
// passed recurrence test on the true residuals and restarts the block from
// them if a column fails.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>

#include "spmm.hpp"

namespace jpcg {

constexpr int kB = 64;       // block width inside the solver
constexpr int kBB = kB * kB;
typedef double d4 __attribute__((ext_vector_type(4)));

enum BcStatus : int { BC_RUN = 0, BC_PENDING = 1, BC_CONVERGED = 2, BC_MAXIT = 3, BC_BREAKDOWN = 4 };

struct BcState {
    int status;
    int k;         // iterations completed
    int maxit;
    int s;         // caller's block width
    int n;
    int restarts;
    int rank;      // live columns of P
    int pad;
    int live[kB];  // column j of P belongs to the basis
    double tol;
    double tau;    // rank cut-off of the second and third CholeskyQR passes
    double nb[kB];
    double thr2[kB];
    double rr[kB];   // ||r_j||^2 of the recurrence (or of the true residual after a check)
    double G0[kBB];  // reduced Gram matrices
    double G1[kBB];
    double Li[kBB];  // inverse Cholesky factor of Gamma = P'Q over the live columns
    double M[kBB];   // the 64 x 64 matrix the next block pass applies
};

__device__ __forceinline__ bool bc_stopped(const BcState* st, int gate)
{
    return gate && __builtin_amdgcn_readfirstlane(st->status) != BC_RUN;
}

// ---------------------------------------------------------------------------
// Gram products C_o = U' V_o (64 x 64) of N x 64 blocks, one per operand o.
// Fragment layouts of v_mfma_f64_16x16x4f64 (D = A B, A 16 x 4, B 4 x 16):
// lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and D[l / 16 + 4 v][l % 16]
// in slot v.  For C = U'V the reduction index is the row: A[i][k] =
// U[r0 + k][16 ib + i], B[k][j] = V[r0 + k][16 jb + j], so lane l loads
// U[r0 + l / 16][16 ib + l % 16] -- four rows of 128 contiguous bytes per
// block of 16 columns.  Each wave accumulates all 16 output tiles of its
// operand over its rows; waves of a workgroup are added in LDS in wave order
// and each workgroup writes one partial per operand.
// NOP = 2: waves 0, 1 take V0 and waves 2, 3 take V1 (U is read twice, from L2).
// ---------------------------------------------------------------------------
constexpr int kGramBS = 256;

template <int NOP>
__global__ __launch_bounds__(kGramBS, 2) void k_bc_gram(int n, const double* __restrict__ U,
                                                     const double* __restrict__ V0, const double* __restrict__ V1,
                                                     double* __restrict__ part, int rows_per_wg, int G,
                                                     const BcState* st, int gate)
{
    if (bc_stopped(st, gate)) return;
    __shared__ double red[NOP][kBB];
    const int L = xcd_logical_block((int)blockIdx.x, G);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int kWavesPerOp = 4 / NOP;
    const int op = w / kWavesPerOp, sub = w % kWavesPerOp;
    const double* __restrict__ V = op == 0 ? V0 : V1;
    const int rs = min(L * rows_per_wg, n), re = min(rs + rows_per_wg, n);
    d4 acc[4][4];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) acc[ib][jb] = d4{0.0, 0.0, 0.0, 0.0};
    const int rq = lane >> 4, cq = lane & 15;
    // The loads of the next 4-row step are issued before this step's products.
    double a[4], b[4];
    auto fetch = [&](int r0) {
        const int row = r0 + rq;
        const bool ok = row < re;
        const size_t o = (size_t)(ok ? row : rs) * kB + cq;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = ok ? U[o + 16 * q] : 0.0;
            b[q] = ok ? V[o + 16 * q] : 0.0;
        }
    };
    int r0 = rs + 4 * sub;
    if (r0 < re) fetch(r0);
    while (r0 < re) {
        double ca[4], cb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ca[q] = a[q];
            cb[q] = b[q];
        }
        r0 += 4 * kWavesPerOp;
        if (r0 < re) fetch(r0);
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) acc[ib][jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[ib], cb[jb], acc[ib][jb], 0, 0, 0);
    }
    // Add the waves of each operand in wave order.
    for (int t = 0; t < kWavesPerOp; ++t) {
        if (sub == t) {
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int e = (16 * ib + rq + 4 * v) * kB + 16 * jb + cq;
                        const double x = acc[ib][jb][v];
                        red[op][e] = t == 0 ? x : red[op][e] + x;
                    }
        }
        __syncthreads();
    }
    double* out = part + (size_t)L * NOP * kBB;
    for (int e = threadIdx.x; e < NOP * kBB; e += kGramBS) out[e] = red[e / kBB][e % kBB];
}

// dst[e] = sum over g of part[g * count + e] for e < count, in a fixed order:
// a workgroup takes EPB consecutive entries; its 256 / EPB thread groups add
// the partials g = q, q + groups, ... (group q), and the group sums are added
// in group order.  which 0: Gram partials, entries [0, 4096) to st->G0 and
// [4096, 8192) to st->G1; which 1: column norms to st->rr.
template <int EPB>
__global__ __launch_bounds__(256) void k_bc_sum(const double* __restrict__ part, int G, int count, int which,
                                                BcState* st, int gate)
{
    if (bc_stopped(st, gate)) return;
    constexpr int kGroups = 256 / EPB;
    __shared__ double red[kGroups][EPB];
    const int j = threadIdx.x % EPB, q = threadIdx.x / EPB;
    const int e = blockIdx.x * EPB + j;
    double s = 0.0;
    if (e < count) {
        int g = q;
        for (; g + 3 * kGroups < G; g += 4 * kGroups) {
            const double a0 = part[(size_t)g * count + e], a1 = part[(size_t)(g + kGroups) * count + e];
            const double a2 = part[(size_t)(g + 2 * kGroups) * count + e], a3 = part[(size_t)(g + 3 * kGroups) * count + e];
            s += (a0 + a1) + (a2 + a3);
        }
        for (; g < G; g += kGroups) s += part[(size_t)g * count + e];
    }
    red[q][j] = s;
    __syncthreads();
    if (q == 0 && e < count) {
        double t = 0.0;
        for (int k = 0; k < kGroups; ++k) t += red[k][j];
        if (which == 0) (e < kBB ? st->G0[e] : st->G1[e - kBB]) = t;
        else st->rr[e] = t;
    }
}

// ---------------------------------------------------------------------------
// Block times 64 x 64: U M with U N x 64 and M = st->M.  Per wave a tile of
// 16 rows: D (16 x 64) = sum over 16 steps t of A_t B_t with the reduction
// index permuted so that lane l's A values are 16 contiguous entries of one
// row: step t, lane l holds A = U[r0 + l % 16][16 (l / 16) + t] and
// B = M[16 (l / 16) + t][16 jb + l % 16] (read from LDS).
//   BC_XUP:   Y += U M                     (X += P alpha)
//   BC_RUP:   Y -= U M, Z = M^-1 Y, per-column partials of y'y
//                                          (R -= Q alpha, Z, ||r_j||^2)
//   BC_DIR:   Y = Z + U M                  (W = Z + P beta)
//   BC_APPLY: Y = U M
// ---------------------------------------------------------------------------
enum BcGemm : int { BC_XUP = 0, BC_RUP = 1, BC_DIR = 2, BC_APPLY = 3 };
constexpr int kGemmBS = 256;
constexpr int kMPad = 65;  // LDS row pitch of M (doubles)

struct BcGemmArgs {
    int n;
    const double* U;
    double* Y;
    double* Z;          // BC_RUP: written; BC_DIR: read
    const double* dinv;
    double* part;       // BC_RUP: [G][64] partials of y'y
    int G;
};

__device__ __forceinline__ void bc_tile_load(const double* __restrict__ U, int r0, int n, double (&a)[16])
{
    const int lane = threadIdx.x & 63, rq = lane >> 4, cq = lane & 15;
    const int row = r0 + cq;
    const bool ok = row < n;
    const double2* src = (const double2*)(U + (size_t)(ok ? row : 0) * kB + 16 * rq);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const double2 v = ok ? src[t] : make_double2(0.0, 0.0);
        a[2 * t] = v.x;
        a[2 * t + 1] = v.y;
    }
}

__device__ __forceinline__ void bc_tile_product(const double (&a)[16], const double* Ms, d4 (&acc)[4])
{
    const int lane = threadIdx.x & 63, rq = lane >> 4, cq = lane & 15;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) acc[jb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 16; ++t)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
            acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], Ms[(16 * rq + t) * kMPad + 16 * jb + cq], acc[jb], 0, 0, 0);
}

template <int MODE>
__global__ __launch_bounds__(kGemmBS, 2) void k_bc_gemm(BcGemmArgs g, BcState* st, int gate)
{
    if (bc_stopped(st, gate)) return;
    __shared__ double Ms[kB * kMPad];
    __shared__ double red[4][kB];
    for (int e = threadIdx.x; e < kBB; e += kGemmBS) Ms[(e / kB) * kMPad + e % kB] = st->M[e];
    __syncthreads();
    const int L = xcd_logical_block((int)blockIdx.x, g.G);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, rq = lane >> 4, cq = lane & 15;
    const int tiles = (g.n + 15) / 16;
    const int tpw = (tiles + g.G - 1) / g.G;
    const int t0 = min(L * tpw, tiles), t1 = min(t0 + tpw, tiles);
    double nrm[4] = {0.0, 0.0, 0.0, 0.0};
    if (MODE == BC_XUP && L == 0 && threadIdx.x == 0) st->k += 1;
    // The next tile's row loads are issued before this tile's products.
    double a[16];
    int tile = t0 + w;
    if (tile < t1) bc_tile_load(g.U, tile * 16, g.n, a);
    while (tile < t1) {
        const int r0 = tile * 16;
        double ca[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) ca[u] = a[u];
        tile += kGemmBS / 64;
        if (tile < t1) bc_tile_load(g.U, tile * 16, g.n, a);
        d4 acc[4];
        bc_tile_product(ca, Ms, acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = r0 + rq + 4 * v;
            if (row >= g.n) continue;
            double di = 0.0;
            if constexpr (MODE == BC_RUP) di = g.dinv[row];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const size_t o = (size_t)row * kB + 16 * jb + cq;
                if constexpr (MODE == BC_XUP) {
                    g.Y[o] = g.Y[o] + acc[jb][v];
                } else if constexpr (MODE == BC_RUP) {
                    const double r = g.Y[o] - acc[jb][v];
                    g.Y[o] = r;
                    g.Z[o] = di * r;
                    nrm[jb] += r * r;
                } else if constexpr (MODE == BC_DIR) {
                    g.Y[o] = g.Z[o] + acc[jb][v];
                } else {
                    g.Y[o] = acc[jb][v];
                }
            }
        }
    }
    if constexpr (MODE == BC_RUP) {
        // Column 16 jb + cq: lanes cq, cq + 16, cq + 32, cq + 48, then the waves in order.
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            double x = nrm[jb];
            x += __shfl_xor(x, 16);
            x += __shfl_xor(x, 32);
            nrm[jb] = x;
        }
        if (rq == 0) {
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) red[w][16 * jb + cq] = nrm[jb];
        }
        __syncthreads();
        if (threadIdx.x < kB) {
            const int j = threadIdx.x;
            g.part[(size_t)L * kB + j] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
        }
    }
}

// ---------------------------------------------------------------------------
// Row products and residuals.
// ---------------------------------------------------------------------------
constexpr int kBcSpmmBS = 512;

// Y = A X over N x 64 blocks (two nonzeros per gather, see mr_row_x2).
__global__ __launch_bounds__(kBcSpmmBS) void k_bc_spmm(int n, const int* __restrict__ rowptr,
                                                       const int* __restrict__ col, const double* __restrict__ val,
                                                       const double* __restrict__ X, double* __restrict__ Y,
                                                       int rows_per_block, int G, const BcState* st, int gate)
{
    if (bc_stopped(st, gate)) return;
    const int L = xcd_logical_block((int)blockIdx.x, G);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int rs = min(L * rows_per_block, n), re = min(rs + rows_per_block, n);
    const int cp = 2 * (lane & 31);
    for (int i = rs + w; i < re; i += kBcSpmmBS / kWave) {
        const double2 y = mr_row_x2(rowptr, col, val, i, [&](int j) { return *(const double2*)(X + (size_t)j * kB + cp); });
        if (lane < 32) *(double2*)(Y + (size_t)i * kB + cp) = y;
    }
}

// R = B - AX (AX given), Z = M^-1 R, per-workgroup partials of r'r and b'b
// (part[g][0][64], part[g][1][64]); write = 0 only measures.
__global__ __launch_bounds__(256) void k_bc_residual(int n, const double* __restrict__ B,
                                                     const double* __restrict__ AX, const double* __restrict__ dinv,
                                                     double* __restrict__ R, double* __restrict__ Z,
                                                     double* __restrict__ part, int write)
{
    __shared__ double red[2][4][kB];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double rr = 0.0, bb = 0.0;
    for (int i = blockIdx.x * 4 + w; i < n; i += gridDim.x * 4) {
        const size_t o = (size_t)i * kB + lane;
        const double b = B[o], r = b - AX[o];
        if (write) {
            R[o] = r;
            Z[o] = dinv[i] * r;
        }
        rr += r * r;
        bb += b * b;
    }
    red[0][w][lane] = rr;
    red[1][w][lane] = bb;
    __syncthreads();
    if (threadIdx.x < kB) {
        const int j = threadIdx.x;
        part[((size_t)blockIdx.x * 2 + 0) * kB + j] = ((red[0][0][j] + red[0][1][j]) + red[0][2][j]) + red[0][3][j];
        part[((size_t)blockIdx.x * 2 + 1) * kB + j] = ((red[1][0][j] + red[1][1][j]) + red[1][2][j]) + red[1][3][j];
    }
}

// Copy between the caller's n x s block (leading dimension s) and the
// solver's n x 64 block (columns >= s zero).
__global__ void k_bc_pack(int n, int s, const double* __restrict__ src, double* __restrict__ dst, int to_wide)
{
    const int lane = threadIdx.x & 63;
    for (int i = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; i < n; i += gridDim.x * (blockDim.x / 64)) {
        if (to_wide) dst[(size_t)i * kB + lane] = lane < s ? src[(size_t)i * s + lane] : 0.0;
        else if (lane < s) dst[(size_t)i * s + lane] = src[(size_t)i * kB + lane];
    }
}

// ---------------------------------------------------------------------------
// 64 x 64 factorisations, one workgroup of 256 threads, matrices in LDS.
// ---------------------------------------------------------------------------
constexpr int kSmallBS = 256;
constexpr int kSP = 65;  // LDS pitch

// Cholesky factorisation of the symmetric matrix in A (its lower triangle)
// taking columns in order.  mode 0: every column in `use` must have a
// positive pivot (bad = 1 otherwise); mode 1: a column whose pivot is <= tau
// is dropped.  keep[k] is set for the factored columns.  On return row k of A
// holds column k of the factor L (A = L' in its upper triangle, zeros below
// the diagonal; zero rows for dropped or unused columns).  Called by the whole
// workgroup; wave 0 factors alone, without workgroup barriers: lane j holds
// column j of the trailing matrix in registers, updated in both triangles so
// that it stays exactly symmetric (lane i's update of a_ji is the same fused
// product as lane j's of a_ij).  Step k: the pivot is lane k's a_kk; lane i's
// own a_ik scaled by the inverse pivot is l_ik, written to A[k][i]; every lane
// reads that row's entries right of the diagonal as broadcasts and subtracts
// l_ik l_jk from its column.
template <int K>
__device__ __forceinline__ void chol_step(double (&a)[kB], int j, unsigned long long usem, int mode, double tau,
                                          double* A, int* keep, bool& badk)
{
    const double d = read_lane(a[K], K);
    bool kk = ((usem >> K) & 1ull) != 0;
    if (kk) {
        if (mode == 0) {
            if (!(d > 0.0) || !isfinite(d)) {
                badk = true;
                kk = false;
            }
        } else if (!(d > tau)) {
            kk = false;
        }
    }
    if (j == 0) keep[K] = kk ? 1 : 0;
    if (!kk) {
        A[K * kSP + j] = 0.0;
        return;
    }
    const double piv = sqrt(d), ip = 1.0 / piv;
    const double l = j == K ? piv : (j > K ? a[K] * ip : 0.0);
    A[K * kSP + j] = l;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Columns j <= K are final: they subtract l_ik * 0, which leaves a_ij
    // unchanged (the entries are finite).  The row is read in groups of 16,
    // all loads of a group issued before its updates.
    const double lm = j > K ? l : 0.0;
    constexpr int I0 = K + 1, NI = kB - I0;
#pragma unroll
    for (int c = 0; c < NI; c += 16) {
        double li[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (c + u < NI) li[u] = A[K * kSP + I0 + c + u];
        __builtin_amdgcn_sched_barrier(0);  // the group's loads stay ahead of its updates
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (c + u < NI) a[I0 + c + u] = __builtin_fma(-li[u], lm, a[I0 + c + u]);
    }
}

template <int... K>
__device__ __forceinline__ void chol_steps(std::integer_sequence<int, K...>, double (&a)[kB], int j,
                                           unsigned long long usem, int mode, double tau, double* A, int* keep,
                                           bool& badk)
{
    (chol_step<K>(a, j, usem, mode, tau, A, keep, badk), ...);
}

__device__ __forceinline__ void small_cholesky(double* A, const int* use, int mode, double tau, int* keep, int* bad)
{
    if (threadIdx.x < kB) {
        const int j = threadIdx.x;
        const unsigned long long usem = __ballot(use[j] != 0);
        double a[kB];
#pragma unroll
        for (int i = 0; i < kB; ++i) a[i] = A[i >= j ? i * kSP + j : j * kSP + i];
        // Every lane has read its column before row 0 is overwritten.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        bool badk = false;
        chol_steps(std::make_integer_sequence<int, kB>{}, a, j, usem, mode, tau, A, keep, badk);
        if (j == 0 && badk) *bad = 1;
    }
    __syncthreads();
}

// Step M of the forward substitution (M a template parameter): x_M = r_M /
// L[M][M], then r_i -= L[i][M] x_M for the rows below, L's column M read from
// row M of U = L' as broadcasts.
template <int M>
__device__ __forceinline__ void inv_step(double (&r)[kB], unsigned long long km, const double* U)
{
    if (!((km >> M) & 1ull)) {
        r[M] = 0.0;
        return;
    }
    const double xm = r[M] / U[M * kSP + M];
    r[M] = xm;
    // The row is read in groups of 16, all loads of a group issued before
    // its updates.
    constexpr int I0 = M + 1, NI = kB - I0;
#pragma unroll
    for (int c = 0; c < NI; c += 16) {
        double ui[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (c + u < NI) ui[u] = U[M * kSP + I0 + c + u];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (c + u < NI) r[I0 + c + u] = __builtin_fma(-ui[u], xm, r[I0 + c + u]);
    }
}

template <int... M>
__device__ __forceinline__ void inv_steps(std::integer_sequence<int, M...>, double (&r)[kB], unsigned long long km,
                                          const double* U)
{
    (inv_step<M>(r, km, U), ...);
}

// X = Lk^-1 for the factor left in U = L' by small_cholesky, restricted to the
// kept columns (rows and columns not kept are zero in X).  Wave 0 alone: lane j
// forms column j by forward substitution in column order (each x_m, once
// known, updates every row below it, so the updates of a step are
// independent).
__device__ __forceinline__ void small_tri_inverse(const double* U, const int* keep, double* X)
{
    if (threadIdx.x < kB) {
        const int j = threadIdx.x;
        const unsigned long long km = __ballot(keep[j] != 0);
        const bool mine = ((km >> j) & 1ull) != 0;
        double r[kB];
#pragma unroll
        for (int i = 0; i < kB; ++i) r[i] = i == j ? 1.0 : 0.0;
        inv_steps(std::make_integer_sequence<int, kB>{}, r, km, U);
#pragma unroll
        for (int i = 0; i < kB; ++i) X[i * kSP + j] = mine ? r[i] : 0.0;
    }
    __syncthreads();
}

// C = op(A) B for 64 x 64 LDS matrices (op = transpose if ta), written to
// out[e] (global, row-major) scaled by `sign`.  Returns whether every entry
// (of the whole matrix) is finite.
__device__ bool small_matmul_out(const double* A, int ta, const double* B, double sign, double* out)
{
    const int t = threadIdx.x;
    const int r0 = (t >> 4) * 4, c0 = (t & 15) * 4;
    double c[4][4] = {};
    for (int m = 0; m < kB; ++m) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            av[u] = ta ? A[m * kSP + r0 + u] : A[(r0 + u) * kSP + m];
            bv[u] = B[m * kSP + c0 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) c[u][v] += av[u] * bv[v];
    }
    bool finite = true;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            out[(r0 + u) * kB + c0 + v] = sign * c[u][v];
            finite = finite && isfinite(c[u][v]);
        }
    return __syncthreads_and(finite ? 1 : 0) != 0;
}

// The same product into an LDS matrix.
__device__ void small_matmul_lds(const double* A, int ta, const double* B, double* C)
{
    const int t = threadIdx.x;
    const int r0 = (t >> 4) * 4, c0 = (t & 15) * 4;
    double c[4][4] = {};
    for (int m = 0; m < kB; ++m) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            av[u] = ta ? A[m * kSP + r0 + u] : A[(r0 + u) * kSP + m];
            bv[u] = B[m * kSP + c0 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) c[u][v] += av[u] * bv[v];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) C[(r0 + u) * kSP + c0 + v] = c[u][v];
    __syncthreads();
}

__device__ void load_small(const double* src, double* dst)
{
    for (int e = threadIdx.x; e < kBB; e += kSmallBS) dst[(e / kB) * kSP + e % kB] = src[e];
    __syncthreads();
}

// alpha = Gamma^-1 Psi over the live columns (Gamma = G0 = P'Q, Psi = G1 = P'R):
// Cholesky of Gamma, Li = L^-1 kept for beta, M = Li' (Li Psi).
__global__ __launch_bounds__(kSmallBS) void k_bc_alpha(BcState* st, int gate)
{
    if (bc_stopped(st, gate)) return;
    __shared__ double A[kB * kSP], X[kB * kSP], T[kB * kSP];
    __shared__ int use[kB], keep[kB], bad;
    if (threadIdx.x == 0) bad = 0;
    if (threadIdx.x < kB) use[threadIdx.x] = st->live[threadIdx.x];
    load_small(st->G0, A);
    small_cholesky(A, use, 0, 0.0, keep, &bad);
    if (bad) {
        if (threadIdx.x == 0) st->status = BC_BREAKDOWN;
        return;
    }
    small_tri_inverse(A, keep, X);
    for (int e = threadIdx.x; e < kBB; e += kSmallBS) st->Li[e] = X[(e / kB) * kSP + e % kB];
    load_small(st->G1, A);
    small_matmul_lds(X, 0, A, T);                             // T = Li Psi
    const bool finite = small_matmul_out(X, 1, T, 1.0, st->M);  // M = Li' T
    if (!finite && threadIdx.x == 0) st->status = BC_BREAKDOWN;
}

// Apply the stopping tests to the column norms of the updated residual
// (st->rr) and, if the iteration continues, M = beta = -Li' (Li Q'Z) (G0 = Q'Z).
__global__ __launch_bounds__(kSmallBS) void k_bc_beta(BcState* st, int gate)
{
    if (bc_stopped(st, gate)) return;
    __shared__ double A[kB * kSP], X[kB * kSP], T[kB * kSP];
    __shared__ int decide;
    const int t = threadIdx.x;
    if (t < kB) {
        // Lane j tests column j; the ballots give every lane the verdicts.
        const double rj = st->rr[t];
        const bool pass = __ballot(rj <= st->thr2[t]) == ~0ull;
        const bool finite = __ballot(isfinite(rj)) == ~0ull;
        int s = BC_RUN;
        if (!finite) s = BC_BREAKDOWN;
        else if (pass) s = BC_PENDING;
        else if (st->k >= st->maxit) s = BC_MAXIT;
        if (t == 0) {
            st->status = s;
            decide = s;
        }
    }
    __syncthreads();
    if (decide != BC_RUN) return;
    load_small(st->Li, X);
    load_small(st->G0, A);
    small_matmul_lds(X, 0, A, T);
    const bool finite = small_matmul_out(X, 1, T, -1.0, st->M);
    if (!finite && threadIdx.x == 0) st->status = BC_BREAKDOWN;
}

// One CholeskyQR pass on the Gram matrix G0 of the current block W:
// pass 0: columns scaled to unit norm, shift 11 (n s + s (s + 1)) u trace,
// no dropping; passes 1 and 2: columns dropped at a pivot <= tau.  M = the
// inverse transposed factor (times the scaling in pass 0); after pass 2 the
// kept columns are the live columns of the new P.
__global__ __launch_bounds__(kSmallBS) void k_bc_orth(BcState* st, int pass, int gate)
{
    if (bc_stopped(st, gate)) return;
    __shared__ double A[kB * kSP], X[kB * kSP], scale[kB];
    __shared__ int use[kB], keep[kB], bad;
    __shared__ double shift;
    const int t = threadIdx.x;
    load_small(st->G0, A);
    if (t < kB) {
        const double d = A[t * kSP + t];
        scale[t] = pass == 0 ? (d > 0.0 ? 1.0 / sqrt(d) : 0.0) : 1.0;
        use[t] = 1;
    }
    if (t == 0) bad = 0;
    __syncthreads();
    if (pass == 0) {
        for (int e = t; e < kBB; e += kSmallBS) {
            const int i = e / kB, j = e % kB;
            A[i * kSP + j] *= scale[i] * scale[j];
        }
        __syncthreads();
        if (t == 0) {
            double tr = 0.0;
            for (int j = 0; j < kB; ++j) tr += A[j * kSP + j];
            const double s = (double)st->s, n = (double)st->n;
            shift = 11.0 * (n * s + s * (s + 1.0)) * 0x1p-53 * tr;
        }
        __syncthreads();
        if (t < kB) A[t * kSP + t] += shift;
        __syncthreads();
    }
    small_cholesky(A, use, 1, pass == 0 ? 0.0 : st->tau, keep, &bad);
    small_tri_inverse(A, keep, X);
    // M[i][j] = scale_i X[j][i]
    for (int e = t; e < kBB; e += kSmallBS) {
        const int i = e / kB, j = e % kB;
        st->M[e] = scale[i] * X[j * kSP + i];
    }
    if (pass == 2 && t < kB) {
        st->live[t] = keep[t];
        if (t == 0) {
            int r = 0;
            for (int j = 0; j < kB; ++j) r += keep[j];
            st->rank = r;
            if (r == 0) st->status = BC_BREAKDOWN;
        }
    }
}

// Set-up / check scalars from the residual partials (part[g][2][64]):
// mode 0 (set-up): nb, thresholds; status CONVERGED if every column passes,
// BREAKDOWN on a non-finite value, else RUN.  mode 1 (check of a PENDING
// state): CONVERGED if every true residual passes, else RUN and one more
// restart.  mode 2 (report): rr = ||b - A x||^2 only.
__global__ void k_bc_scalars(BcState* st, const double* __restrict__ part, int G, int mode)
{
    __shared__ double rr[kB], bb[kB];
    const int t = threadIdx.x;
    if (t < kB) {
        double a = 0.0, b = 0.0;
        for (int g = 0; g < G; ++g) {
            a += part[((size_t)g * 2 + 0) * kB + t];
            b += part[((size_t)g * 2 + 1) * kB + t];
        }
        rr[t] = a;
        bb[t] = b;
        st->rr[t] = a;
        if (mode == 0) {
            const double nb = sqrt(b);
            st->nb[t] = nb;
            const double thr = st->tol * nb;
            st->thr2[t] = thr * thr;
        }
    }
    __syncthreads();
    if (t == 0 && mode != 2) {
        bool pass = true, finite = true;
        for (int j = 0; j < kB; ++j) {
            pass = pass && rr[j] <= st->thr2[j];
            finite = finite && isfinite(rr[j]) && isfinite(bb[j]);
        }
        if (mode == 0) {
            st->k = 0;
            st->restarts = 0;
            for (int j = 0; j < kB; ++j) st->live[j] = 1;
        }
        if (!finite) st->status = BC_BREAKDOWN;
        else if (pass) st->status = BC_CONVERGED;
        else {
            if (mode == 1) st->restarts += 1;
            st->status = BC_RUN;
        }
    }
}

}  // namespace jpcg

// Block solver state hanging off a context.
struct cg_block {
    int gram_G = 0, gemm_G = 0, spmm_G = 0, spmm_rpb = 0, gram_rpw = 0, res_G = 0, chunk = 4;
    double* work = nullptr;  // B, X, R, Z, P, Q, W: 7 n x 64 blocks
    double* part = nullptr;  // Gram partials [gram_G][2][4096]
    double* part2 = nullptr; // norm / residual partials [max(gemm_G, res_G)][2][64]
    jpcg::BcState* st = nullptr;
    jpcg::BcState* hst = nullptr;
    hipGraphExec_t exec = nullptr;
    double tol = -1.0, tau = -1.0;
    int maxit = -1;
};

namespace jpcg {

struct BcBufs {
    double *B, *X, *R, *Z, *P, *Q, *W;
};

static BcBufs bufs(cg_ctx* c, cg_block* b)
{
    const size_t nb = (size_t)c->n * kB;
    double* w = b->work;
    return {w, w + nb, w + 2 * nb, w + 3 * nb, w + 4 * nb, w + 5 * nb, w + 6 * nb};
}

void free_block(cg_ctx* c)
{
    cg_block* b = c->block;
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->work) (void)hipFree(b->work);
    if (b->part) (void)hipFree(b->part);
    if (b->part2) (void)hipFree(b->part2);
    if (b->st) (void)hipFree(b->st);
    if (b->hst) (void)hipHostFree(b->hst);
    delete b;
    c->block = nullptr;
}

static void launch(const void* fn, int grid, int bs, hipStream_t st, void** args)
{
    JPCG_HIP(hipLaunchKernel(fn, dim3(grid), dim3(bs), args, 0, st));
}

// The kernels of the block operations, enqueued on `st`.
struct BcOps {
    cg_ctx* c;
    cg_block* b;
    BcBufs v;
    hipStream_t st;

    void spmm(const double* X, double* Y, int gate)
    {
        int n = c->n;
        void* a[] = {&n, &c->rowptr, &c->col, &c->val, &X, &Y, &b->spmm_rpb, &b->spmm_G, &b->st, &gate};
        launch((const void*)k_bc_spmm, b->spmm_G, kBcSpmmBS, st, a);
    }
    void gram(const double* U, const double* V0, const double* V1, int gate)
    {
        int n = c->n;
        const int nop = V1 ? 2 : 1;
        void* a[] = {&n, &U, &V0, &V1, &b->part, &b->gram_rpw, &b->gram_G, &b->st, &gate};
        launch(nop == 2 ? (const void*)k_bc_gram<2> : (const void*)k_bc_gram<1>, b->gram_G, kGramBS, st, a);
        int count = nop * kBB, which = 0;
        void* r[] = {&b->part, &b->gram_G, &count, &which, &b->st, &gate};
        launch((const void*)k_bc_sum<32>, count / 32, 256, st, r);
    }
    void norms(int gate)
    {
        int count = kB, which = 1;
        void* r[] = {&b->part2, &b->gemm_G, &count, &which, &b->st, &gate};
        launch((const void*)k_bc_sum<4>, kB / 4, 256, st, r);
    }
    void gemm(int mode, const double* U, double* Y, double* Z, int gate)
    {
        BcGemmArgs g{c->n, U, Y, Z, c->dinv, b->part2, b->gemm_G};
        void* a[] = {&g, &b->st, &gate};
        const void* fn = mode == BC_XUP   ? (const void*)k_bc_gemm<BC_XUP>
                         : mode == BC_RUP ? (const void*)k_bc_gemm<BC_RUP>
                         : mode == BC_DIR ? (const void*)k_bc_gemm<BC_DIR>
                                          : (const void*)k_bc_gemm<BC_APPLY>;
        launch(fn, b->gemm_G, kGemmBS, st, a);
    }
    void orth_pass(int pass, int gate)
    {
        void* a[] = {&b->st, &pass, &gate};
        launch((const void*)k_bc_orth, 1, kSmallBS, st, a);
    }
    // P = orth(W0): three CholeskyQR passes, the blocks in W0 -> Wa -> Wb -> P.
    void orth(double* W0, double* Wa, double* Wb, int gate)
    {
        gram(W0, W0, nullptr, gate);
        orth_pass(0, gate);
        gemm(BC_APPLY, W0, Wa, nullptr, gate);
        gram(Wa, Wa, nullptr, gate);
        orth_pass(1, gate);
        gemm(BC_APPLY, Wa, Wb, nullptr, gate);
        gram(Wb, Wb, nullptr, gate);
        orth_pass(2, gate);
        gemm(BC_APPLY, Wb, v.P, nullptr, gate);
    }
    // R = B - A X, Z = M^-1 R (write), partials of r'r, b'b; then the scalars.
    void residual(int write, int mode)
    {
        spmm(v.X, v.Q, 0);
        int n = c->n;
        void* a[] = {&n, &v.B, &v.Q, &c->dinv, &v.R, &v.Z, &b->part2, &write};
        launch((const void*)k_bc_residual, b->res_G, 256, st, a);
        void* s[] = {&b->st, &b->part2, &b->res_G, &mode};
        launch((const void*)k_bc_scalars, 1, 64, st, s);
    }
    // One gated iteration.
    void iteration()
    {
        spmm(v.P, v.Q, 1);
        gram(v.P, v.Q, v.R, 1);
        int gate = 1;
        void* a[] = {&b->st, &gate};
        launch((const void*)k_bc_alpha, 1, kSmallBS, st, a);
        gemm(BC_XUP, v.P, v.X, nullptr, 1);
        gemm(BC_RUP, v.Q, v.R, v.Z, 1);
        norms(1);
        gram(v.Q, v.Z, nullptr, 1);
        void* bta[] = {&b->st, &gate};
        launch((const void*)k_bc_beta, 1, kSmallBS, st, bta);
        gemm(BC_DIR, v.P, v.W, v.Z, 1);
        // W -> Z -> Q -> P (Z and Q are free until the next iteration's product)
        orth(v.W, v.Z, v.Q, 1);
    }
};

static cg_block* make_block(cg_ctx* c)
{
    cg_block* b = new cg_block();
    try {
        const size_t nb = (size_t)c->n * kB;
        b->gram_G = std::max(8, std::min(c->cus, (c->n + 63) / 64) / 8 * 8);
        b->gram_rpw = (c->n + b->gram_G - 1) / b->gram_G;
        const int tiles = (c->n + 15) / 16;
        b->gemm_G = std::max(8, std::min(c->cus * 2, (tiles + 3) / 4) / 8 * 8);
        const int wpc = c->opts.autotune ? spmm_blocks_per_cu(c) : 4;
        b->spmm_G = std::max(8, std::min(c->cus * wpc, (c->n + 15) / 16) / 8 * 8);
        b->spmm_rpb = (c->n + b->spmm_G - 1) / b->spmm_G;
        b->res_G = std::min(1024, (c->n + 3) / 4);
        JPCG_HIP(hipMalloc(&b->work, sizeof(double) * nb * 7));
        JPCG_HIP(hipMalloc(&b->part, sizeof(double) * (size_t)b->gram_G * 2 * kBB));
        JPCG_HIP(hipMalloc(&b->part2, sizeof(double) * (size_t)std::max(b->gemm_G, b->res_G) * 2 * kB));
        JPCG_HIP(hipMalloc(&b->st, sizeof(BcState)));
        JPCG_HIP(hipHostMalloc(&b->hst, sizeof(BcState), hipHostMallocDefault));
        JPCG_HIP(hipMemsetAsync(b->work, 0, sizeof(double) * nb * 7, c->stream));
        JPCG_HIP(hipMemsetAsync(b->st, 0, sizeof(BcState), c->stream));
        JPCG_HIP(hipStreamSynchronize(c->stream));
        return b;
    } catch (...) {
        if (b->work) (void)hipFree(b->work);
        if (b->part) (void)hipFree(b->part);
        if (b->part2) (void)hipFree(b->part2);
        if (b->st) (void)hipFree(b->st);
        if (b->hst) (void)hipHostFree(b->hst);
        delete b;
        throw;
    }
}

static void capture_block(cg_ctx* c, cg_block* b)
{
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    hipStream_t cap;
    JPCG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    BcOps ops{c, b, bufs(c, b), cap};
    hipGraph_t graph;
    JPCG_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    for (int it = 0; it < b->chunk; ++it) ops.iteration();
    JPCG_HIP(hipStreamEndCapture(cap, &graph));
    hipError_t e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    JPCG_HIP(e);
    JPCG_HIP(hipStreamDestroy(cap));
}

static BcState bc_read(cg_ctx* c, cg_block* b)
{
    JPCG_HIP(hipMemcpyAsync(b->hst, b->st, sizeof(BcState), hipMemcpyDeviceToHost, c->stream));
    JPCG_HIP(hipStreamSynchronize(c->stream));
    return *b->hst;
}

static void bc_set_status(cg_ctx* c, cg_block* b, int status)
{
    b->hst->status = status;
    JPCG_HIP(hipMemcpyAsync(b->st, b->hst, sizeof(int), hipMemcpyHostToDevice, c->stream));
}

}  // namespace jpcg

using namespace jpcg;

extern "C" {

int cg_solve_block(cg_ctx* c, const double* B, double* X, int32_t s, double tol, int32_t maxit, cg_info* info)
{
    if (!c) return CG_EINVAL;
    if (!B || !X || B == X || s < 1 || s > kB || !(tol >= 0.0) || !std::isfinite(tol))
        return set_error(c, CG_EINVAL, "cg_solve_block: bad arguments");
    if (maxit <= 0) maxit = c->n;
    try {
        if (!c->block) c->block = make_block(c);
        cg_block* b = c->block;
        hipStream_t st = c->stream;
        BcOps ops{c, b, bufs(c, b), st};
        // Parameters live in the state block; the graphs read them there.
        JPCG_HIP(hipStreamSynchronize(st));
        b->hst->tol = tol;
        b->hst->tau = 1e-14;
        b->hst->maxit = maxit;
        b->hst->s = s;
        b->hst->n = c->n;
        JPCG_HIP(hipMemcpyAsync(&b->st->tol, &b->hst->tol, sizeof(double) * 2, hipMemcpyHostToDevice, st));
        JPCG_HIP(hipMemcpyAsync(&b->st->maxit, &b->hst->maxit, sizeof(int) * 3, hipMemcpyHostToDevice, st));
        if (!b->exec) capture_block(c, b);
        JPCG_HIP(hipEventRecord(c->ev0, st));
        int n = c->n, one = 1, zero = 0;
        const int pg = std::min(4096, (c->n + 3) / 4);
        void* pb[] = {&n, &s, &B, &ops.v.B, &one};
        launch((const void*)k_bc_pack, pg, 256, st, pb);
        void* px[] = {&n, &s, &X, &ops.v.X, &one};
        launch((const void*)k_bc_pack, pg, 256, st, px);
        ops.residual(1, 0);
        BcState h = bc_read(c, b);
        if (h.status == BC_RUN) {
            ops.orth(ops.v.Z, ops.v.W, ops.v.Q, 0);
            const long long guard = 2LL * maxit + 64;
            long long launched = 0;
            while (true) {
                JPCG_HIP(hipGraphLaunch(b->exec, st));
                JPCG_HIP(hipGraphLaunch(b->exec, st));
                launched += 2 * b->chunk;
                h = bc_read(c, b);
                if (h.status == BC_PENDING) {
                    // Confirm on the true residuals; restart from them if a column fails.
                    ops.residual(1, 1);
                    h = bc_read(c, b);
                    if (h.status == BC_RUN) {
                        if (h.k >= maxit) {
                            bc_set_status(c, b, BC_MAXIT);
                            h.status = BC_MAXIT;
                        } else {
                            for (int j = 0; j < kB; ++j) b->hst->live[j] = 1;
                            JPCG_HIP(hipMemcpyAsync(b->st->live, b->hst->live, sizeof(int) * kB, hipMemcpyHostToDevice, st));
                            ops.orth(ops.v.Z, ops.v.W, ops.v.Q, 0);
                        }
                    }
                }
                if (h.status != BC_RUN) break;
                if (launched > guard) throw HipError{hipErrorUnknown, "block solver did not stop"};
            }
        }
        // True residual of the returned X for every column.
        ops.residual(0, 2);
        void* ux[] = {&n, &s, &ops.v.X, &X, &zero};
        launch((const void*)k_bc_pack, pg, 256, st, ux);
        JPCG_HIP(hipEventRecord(c->ev1, st));
        JPCG_HIP(hipEventSynchronize(c->ev1));
        const BcState f = bc_read(c, b);
        float ms = 0.f;
        JPCG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        const int code = h.status == BC_CONVERGED ? CG_CONVERGED : h.status == BC_MAXIT ? CG_MAXIT : CG_BREAKDOWN;
        if (info) {
            for (int j = 0; j < s; ++j) {
                cg_info& o = info[j];
                o.iters = h.k;
                o.status = code;
                o.replacements = h.restarts;
                o.outer = h.rank;
                o.relres_recur = f.nb[j] > 0 ? std::sqrt(h.rr[j]) / f.nb[j] : 0.0;
                o.relres_true = f.nb[j] > 0 ? std::sqrt(f.rr[j]) / f.nb[j] : 0.0;
                o.seconds = ms * 1e-3;
            }
        }
        return code;
    } catch (const HipError& e) {
        return set_error(c, CG_EHIP, std::string("cg_solve_block: ") + e.what + ": " + hipGetErrorString(e.code));
    }
}

}  // extern "C"
