// Standard-form Jacobi-PCG kernels (two per iteration), templated on the
// value type T of the matrix and vectors: double for the FP64 solve, float
// for the inner solve of the mixed-precision form.  Dot products, partial
// sums and every scalar (alpha, beta, the tests) stay in double.
//
//   A_k  (k_direction)  reduce the previous B's partials of r'z and r'r, apply
//        the continue-condition / breakdown / iteration-limit tests,
//        beta_k = rho_{k-1} / rho_{k-2}; p_k = z + beta_k p_{k-1} formed inside
//        the gather of q = A p_k; partials of p_k' q.
//   B_k  (k_update)  reduce A_k's partials, alpha_k = rho_{k-1} / sigma_k;
//        x += alpha p, r -= alpha q, z = M^-1 r; partials of r'z and r'r.
//
// z and p are stored interleaved, ZPair {z_i, p_i} per row, in two arrays used
// by iteration parity: zp[P] holds {z_k, p_k} once B_k has run (A_k writes p_k
// into zp[P].p, B_k writes z_k into zp[P].z), so A_{k+1} fetches both operands
// of p_{k+1} = z_k + beta p_k for a column with one 2-element load.
//
// Every workgroup reduces the previous kernel's per-workgroup partials itself,
// in a fixed order, so all workgroups reach the same bits and the same
// decision without atomics.  Scalars that must outlive a kernel sit in a small
// state block, double-buffered by iteration parity so that no kernel reads a
// slot it writes.
#pragma once

#include "phases.hpp"
#include "tiles.hpp"

namespace jpcg {

struct CgState {
    int stop;
    int k;  // completed iterations (advanced by B's workgroup 0)
    int maxit;
    int replacements;
    double nb;       // ||b||
    double thr;      // tol * ||b||
    double rho[2];   // rho[k % 2] = r_{k-1}' z_{k-1}, written by A_k
    double rr;       // ||r_k||^2 seen by the last continue-condition test
    double rr_true;  // ||b - A x||^2 of the returned x
    double sigma, alpha, beta;
    double rr_ref;   // ||r||^2 after the last residual replacement (or of r0)
};

template <typename T>
struct CgArgsT {
    SysView<T> s;  // b, x: the solver's own buffers; zp[P] as described above
    const T* rowsum;  // FP32 solves: row sums of A (computed in FP64) for the row-sum-preserving product
    TileMap tm;    // tiles of the sparse products, per workgroup
    int R;         // rows per workgroup of the elementwise update
    int G;
    double* part_setup;    // [G][3]: r'r, r'z, b'b of r0
    double* part_sig;      // [G][1]: p'q
    double* part_iter[2];  // [G][2]: r'z, r'r after B of parity P (or a check)
    double* part_rep;      // [G][1]: ||b - A x||^2 for the report
    CgState* st;
    double* hist;
    const float* val32;    // FP32-matrix form: FP32 values streamed by the direction products
    double drop2;          // > 0: also confirm on the true residual once ||r||^2 <= drop2 rr_ref
};

// FP32 products use the row-sum-preserving evaluation (see tiles.hpp): the
// FP32 copy of A alone would misrepresent the near-constant modes that
// dominate x for these Neumann-plus-mass systems.
// The FP32-matrix form (M32) streams FP32 values into an FP64 product, in
// the same row-sum-preserving evaluation with FP64 row sums.
template <typename T, bool M32 = false>
constexpr bool kDiff = sizeof(T) == 4 || M32;

template <int NPL, int BS, typename T, bool M32 = false>
struct Lds {
    double red[(BS / kWave) * 4];
    T prod[BS * NPL * (kDiff<T, M32> ? 2 : 1)];  // per wave: 64 * NPL products (values and entries when DIFF)
};

template <int NPL, typename T, bool M32 = false>
__device__ __forceinline__ T* wave_prod(T* prod)
{
    return prod + (threadIdx.x / kWave) * (kWave * NPL * (kDiff<T, M32> ? 2 : 1));
}

// The tile walk in the evaluation that suits T (and the FP32-matrix form).
template <int NPL, typename T, bool M32 = false, typename Gather, typename Value, typename Pre, typename Self,
          typename Row, typename Prologue>
__device__ __forceinline__ void walk(const CgArgsT<T>& a, int L, T* prod, Gather gather, Value value, Pre pre,
                                     Self self, Row row, Prologue prologue)
{
    const SysView<T>& s = a.s;
    if constexpr (M32) {
        tile_rows_x<NPL, T, true, float>(s.rowptr, s.col, a.val32, a.rowsum, a.tm, L, wave_prod<NPL, T, true>(prod),
                                         gather, value, pre, self, row, prologue);
    } else {
        tile_rows_x<NPL, T, kDiff<T>>(s.rowptr, s.col, s.val, a.rowsum, a.tm, L, wave_prod<NPL, T>(prod), gather,
                                      value, pre, self, row, prologue);
    }
}

template <typename T>
struct Tri {
    T a, b, c;
};

__device__ __forceinline__ int logical_of(int G) { return xcd_logical_block((int)blockIdx.x, G); }

// r_out = b - A x and (if z_out) z_out[i].z = M^-1 r_out over the workgroup's
// tiles; shares of r'r, r'z, b'b.
template <int NPL, int BS, typename T>
__device__ __forceinline__ void tile_residual(const CgArgsT<T>& a, T* prod, T* r_out, ZPair<T>* z_out, double& rr,
                                              double& rz, double& bb)
{
    const SysView<T>& s = a.s;
    const T* __restrict__ x = s.x;
    walk<NPL, T>(
        a, logical_of(a.G), prod, [&](int j) { return x[j]; }, Ident<T>{},
        [&](int i) { return Tri<T>{s.b[i], s.dinv[i], kDiff<T> ? x[i] : T(0)}; }, [&](const Tri<T>& t) { return t.c; },
        [&](int i, T ax, Tri<T> bd) {
            const T bi = bd.a;
            const T ri = bi - ax;
            r_out[i] = ri;
            rr += (double)ri * (double)ri;
            bb += (double)bi * (double)bi;
            if (z_out) {
                const T zi = bd.b * ri;
                z_out[i].z = zi;
                rz += (double)ri * (double)zi;
            }
        },
        NoPrologue{});
}

template <int NPL, int BS, typename T>
__global__ __launch_bounds__(BS) void k_setup(CgArgsT<T> a)
{
    __shared__ Lds<NPL, BS, T> sh;
    double v[3] = {0.0, 0.0, 0.0};
    tile_residual<NPL, BS, T>(a, sh.prod, a.s.r, a.s.zp[0], v[0], v[1], v[2]);
    block_partials<BS, 3>(v, sh.red, a.part_setup, logical_of(a.G));
}

// A_1: initial tests, then p_1 = z_0 (from zp[0].z), q = A p_1, p_1 into zp[1].p.
template <int NPL, int BS, typename T, bool M32 = false>
__global__ __launch_bounds__(BS) void k_first(CgArgsT<T> a, double tol, int maxit)
{
    __shared__ Lds<NPL, BS, T, M32> sh;
    double g[3];
    wave_grid_sum<3>(a.part_setup, a.G, g);
    const double rr = g[0], rho = g[1], nb = sqrt(g[2]), thr = tol * nb;
    CgState* st = a.st;
    const SysView<T>& s = a.s;
    const int L = logical_of(a.G);
    if (threadIdx.x == 0 && L == 0) {
        st->k = 0;
        st->maxit = maxit;
        st->replacements = 0;
        st->nb = nb;
        st->thr = thr;
        st->rho[1] = rho;
        st->rr = rr;
        st->rr_true = -1.0;
        st->rr_ref = rr;
        if (a.hist) a.hist[0] = nb > 0.0 ? sqrt(rr) / nb : 0.0;
        st->stop = nb == 0.0 ? STOP_ZERO_RHS : (sqrt(rr) <= thr ? STOP_CONV0 : RUNNING);
        if (nb == 0.0) st->rr_true = 0.0;
        else if (sqrt(rr) <= thr) st->rr_true = rr;
    }
    if (nb == 0.0) {
        const int rs = min(L * a.R, s.n), re = min(rs + a.R, s.n);
        for (int i = rs + (int)threadIdx.x; i < re; i += BS) s.x[i] = T(0);
        return;
    }
    if (sqrt(rr) <= thr) return;
    const ZPair<T>* __restrict__ z0 = a.s.zp[0];
    ZPair<T>* __restrict__ p1 = a.s.zp[1];
    double sig = 0.0;
    walk<NPL, T, M32>(
        a, L, sh.prod, [&](int j) { return z0[j].z; }, Ident<T>{}, [&](int i) { return z0[i].z; },
        [&](T zi) { return zi; },
        [&](int i, T qi, T pi) {
            p1[i] = ZPair<T>{T(0), pi};  // whole pair: .z is written by B_1
            s.q[i] = qi;
            sig += (double)pi * (double)qi;
        },
        NoPrologue{});
    double v[1] = {sig};
    block_partials<BS, 1>(v, sh.red, a.part_sig, L);
}

// A_k, k >= 2, parity P = k % 2.  The scalar work (reducing the previous B's
// partials, the tests, beta) runs as the tile walk's prologue, after the
// first gathers are issued, so its memory latency overlaps theirs.
template <int NPL, int BS, typename T, bool M32 = false>
__global__ __launch_bounds__(BS) void k_direction(CgArgsT<T> a, int P)
{
    __shared__ Lds<NPL, BS, T, M32> sh;
    CgState* st = a.st;
    const SysView<T>& s = a.s;
    const ZPair<T>* __restrict__ zpold = a.s.zp[P ^ 1];  // {z_{k-1}, p_{k-1}}
    ZPair<T>* __restrict__ zpnew = a.s.zp[P];
    const int L = logical_of(a.G);
    const bool lead = threadIdx.x == 0 && L == 0;
    T beta = T(0);
    double sig = 0.0;
    bool go = true;
    __shared__ double s_g[2];
    auto prologue = [&]() -> bool {
        const int stop = st->stop, km1 = st->k, maxit = st->maxit;
        const double rr_ref = st->rr_ref;
        const double thr = st->thr, nb = st->nb, rho_prev = st->rho[P ^ 1];
        // Wave 0 reduces the partials for the workgroup and shares them
        // through LDS (every wave calls the prologue exactly once).
        if (threadIdx.x < kWave) {
            double g[2];
            wave_grid_sum<2>(a.part_iter[P ^ 1], a.G, g);
            if (threadIdx.x == 0) {
                s_g[0] = g[0];
                s_g[1] = g[1];
            }
        }
        __syncthreads();
        const double rz = s_g[0], rr = s_g[1];
        go = false;
        if (stop != RUNNING) return false;
        if (lead) {
            st->rr = rr;
            if (a.hist) a.hist[km1] = sqrt(rr) / nb;
        }
        // The oracle's order: continue-condition, breakdown of r'z, iteration limit.
        // With drop2 (the FP32-matrix form), the true residual is also confirmed
        // each time the recurrence residual has fallen by sqrt(drop2) since the
        // last replacement, and replaces r if it does not pass (reliable updates).
        if (sqrt(rr) <= thr || rr <= a.drop2 * rr_ref) {
            if (lead) st->stop = STOP_CHECK;
            return false;
        }
        if (!(rz > 0.0) || !isfinite(rz)) {
            if (lead) st->stop = STOP_BREAKDOWN;
            return false;
        }
        if (km1 >= maxit) {
            if (lead) st->stop = STOP_MAXIT;
            return false;
        }
        const double b = rz / rho_prev;
        beta = (T)b;
        if (lead) {
            st->rho[P] = rz;
            st->beta = b;
        }
        go = true;
        return true;
    };
    walk<NPL, T, M32>(
        a, L, sh.prod, [&](int j) { return zpold[j]; },
        [&](ZPair<T> zp) { return fma_t(beta, zp.p, zp.z); }, [&](int i) { return zpold[i]; },
        [&](ZPair<T> zp) { return fma_t(beta, zp.p, zp.z); },
        [&](int i, T qi, ZPair<T> zp) {
            const T pi = fma_t(beta, zp.p, zp.z);
            zpnew[i] = ZPair<T>{T(0), pi};  // whole pair: .z (z_{k-2}) is dead until B_k
            s.q[i] = qi;
            sig += (double)pi * (double)qi;
        },
        prologue);
    if (!go) return;  // the same decision in every wave of every workgroup
    double v[1] = {sig};
    block_partials<BS, 1>(v, sh.red, a.part_sig, L);
}

// B_k, parity P = k % 2.  Rows are split arithmetically; the state, the row
// operands and the partials of sigma are all requested before any is used.
template <int BS, typename T>
__global__ __launch_bounds__(BS) void k_update(CgArgsT<T> a, int P)
{
    __shared__ Lds<1, BS, T> sh;
    CgState* st = a.st;
    const SysView<T>& s = a.s;
    const int stop = st->stop;
    const double rho = st->rho[P];
    const int L = logical_of(a.G);
    const int rs = min(L * a.R, s.n), re = min(rs + a.R, s.n);
    ZPair<T>* __restrict__ zp = a.s.zp[P];  // p_k in .p; z_k goes to .z
    const int i0 = rs + (int)threadIdx.x;
    const bool h0 = i0 < re;
    const int ic = h0 ? i0 : 0;
    const T p0 = zp[ic].p, q0 = s.q[ic], x0 = s.x[ic], r0 = s.r[ic], d0 = s.dinv[ic];
    // z_k is written with p_k as a whole pair (full 2-element stores).
    // Wave 0 reduces the partials of sigma for the workgroup.
    if (threadIdx.x < kWave) {
        double g[1];
        wave_grid_sum<1>(a.part_sig, a.G, g);
        if (threadIdx.x == 0) sh.red[0] = g[0];
    }
    __syncthreads();
    const double sigma = sh.red[0];
    __syncthreads();  // sh.red is reused by block_partials below
    if (stop != RUNNING) return;
    const bool lead = threadIdx.x == 0 && L == 0;
    if (!(sigma > 0.0) || !isfinite(sigma)) {
        if (lead) st->stop = STOP_BREAKDOWN;
        return;
    }
    const double alpha_d = rho / sigma;
    const T alpha = (T)alpha_d;
    double v[2] = {0.0, 0.0};
    if (h0) {
        s.x[i0] = fma_t(alpha, p0, x0);
        const T ri = fma_t(-alpha, q0, r0);
        s.r[i0] = ri;
        const T zi = d0 * ri;
        zp[i0] = ZPair<T>{zi, p0};
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
    }
    for (int i = i0 + BS; i < re; i += BS) {
        const T pi = zp[i].p;
        s.x[i] = fma_t(alpha, pi, s.x[i]);
        const T ri = fma_t(-alpha, s.q[i], s.r[i]);
        s.r[i] = ri;
        const T zi = s.dinv[i] * ri;
        zp[i] = ZPair<T>{zi, pi};
        v[0] += (double)ri * (double)zi;
        v[1] += (double)ri * (double)ri;
    }
    block_partials<BS, 2>(v, sh.red, a.part_iter[P], L);
    if (lead) {
        st->k = st->k + 1;
        st->sigma = sigma;
        st->alpha = alpha_d;
    }
}

// True residual r = b - A x, z = M^-1 r into zp[P].z, the slot A_{k+1} reads
// (p_k in zp[P].p is kept).
template <int NPL, int BS, typename T>
__global__ __launch_bounds__(BS) void k_check(CgArgsT<T> a, int P)
{
    __shared__ Lds<NPL, BS, T> sh;
    double rr = 0.0, rz = 0.0, bb = 0.0;
    tile_residual<NPL, BS, T>(a, sh.prod, a.s.r, a.s.zp[P], rr, rz, bb);
    double v[2] = {rz, rr};
    block_partials<BS, 2>(v, sh.red, a.part_iter[P], logical_of(a.G));
}

// One workgroup: accept the solve, or resume with the replaced residual.
template <int BS, typename T>
__global__ __launch_bounds__(BS) void k_check_decide(CgArgsT<T> a, int P)
{
    double g[2];
    wave_grid_sum<2>(a.part_iter[P], a.G, g);
    if (threadIdx.x == 0) {
        CgState* st = a.st;
        if (sqrt(g[1]) <= st->thr) {
            st->stop = STOP_CONVERGED;
            st->rr_true = g[1];
        } else {
            st->stop = RUNNING;
            st->replacements += 1;
            st->rr_ref = g[1];
        }
    }
}

// ||b - A x||^2 of the returned x, for solves that end without convergence.
template <int NPL, int BS, typename T>
__global__ __launch_bounds__(BS) void k_report(CgArgsT<T> a)
{
    __shared__ Lds<NPL, BS, T> sh;
    double v[1] = {0.0};
    double rz = 0.0, bb = 0.0;
    tile_residual<NPL, BS, T>(a, sh.prod, a.s.q, (ZPair<T>*)nullptr, v[0], rz, bb);
    block_partials<BS, 1>(v, sh.red, a.part_rep, logical_of(a.G));
}

template <int BS, typename T>
__global__ __launch_bounds__(BS) void k_report_sum(CgArgsT<T> a)
{
    double g[1];
    wave_grid_sum<1>(a.part_rep, a.G, g);
    if (threadIdx.x == 0) a.st->rr_true = g[0];
}

// y = A x over the solver's tiles (rows summed in stored order).
template <int NPL, int BS, typename T>
__global__ __launch_bounds__(BS) void k_spmv(CgArgsT<T> a, const T* __restrict__ x, T* __restrict__ y)
{
    __shared__ Lds<NPL, BS, T> sh;
    walk<NPL, T>(a, logical_of(a.G), sh.prod, [&](int j) { return x[j]; }, Ident<T>{},
                 [&](int i) { return kDiff<T> ? x[i] : T(0); }, [&](T xi) { return xi; }, [&](int i, T v, T) { y[i] = v; },
                 NoPrologue{});
}

}  // namespace jpcg
