// The steps of one Jacobi-PCG solve, as device functions over a block's rows.
//
// A "team" is a set of co-resident workgroups that owns one system: the
// system's rows are cut into product tiles (tiles.hpp), workgroup L of the
// team owns an equal run of tiles (so a contiguous row range), and the team
// meets at grid barriers between steps.  The batched solver runs many teams
// in one launch.  A team of one workgroup synchronises with __syncthreads
// alone.
//
// Per iteration there are two team-wide reductions, so two barriers:
//   step A   q = A p_new, p_new = z + beta p_old formed on the fly (the direction
//            update of the previous iteration is fused into the gather), and the
//            partial of sigma = p_new' q;
//   step B   x += alpha p_new, r -= alpha q, z = M^-1 r, partials of r'z and r'r.
// The continue-condition and the true-residual confirmation (step R,
// r = b - A x) follow the paper's loop-with-constraint structure (Section IV).
//
// Value type T is double (FP64 solve) or float (inner solve of the mixed-
// precision form).  Dot products always accumulate in double.
#pragma once

#include "tiles.hpp"

namespace jpcg {

// Slots of the partial-sum array, each `G` doubles long.  A group of K
// consecutive slots holds the K quantities of one reduction.
enum : int {
    SLOT_SIG = 0,    // p'q
    SLOT_ITER = 1,   // r'z, r'r after step B
    SLOT_SETUP = 3,  // r'r, r'z, b'b of the initial residual
    SLOT_CHECK = 6,  // r'r, r'z of the confirming true residual
    NSLOT = 8
};

// Stop codes of the graph-chunked solvers' device state.
enum StopCode : int {
    RUNNING = 0,
    STOP_ZERO_RHS = 1,   // ||b|| = 0: x = 0
    STOP_CONV0 = 2,      // x0 already satisfies the test
    STOP_CHECK = 3,      // recurrence residual passed: confirm on b - A x
    STOP_MAXIT = 4,
    STOP_BREAKDOWN = 5,
    STOP_CONVERGED = 6,  // confirmed
};

// Device-side result of a solve, copied back by the host.
struct DevInfo {
    int iters;
    int status;
    int replacements;
    int outer;
    double rr_recur;  // ||r||^2 of the recurrence at exit
    double rr_true;   // ||b - A x||^2 of the returned x
    double bb;        // ||b||^2
    double pad;
};

// z and p of the CG loop, stored interleaved per row in two arrays used by
// iteration parity: the product fetches both operands of p_new = z + beta
// p_old for a column with one 2-element load.  Stores write whole pairs
// where they can (a dead half gets 0 or its current value).
template <typename T>
struct alignas(2 * sizeof(T)) ZPair {
    T z, p;
};

template <typename T>
struct SysView {
    int n;
    const int* __restrict__ rowptr;
    const int* __restrict__ col;
    const T* __restrict__ val;
    const T* __restrict__ dinv;  // M^-1 diagonal (all ones for no preconditioner)
    const T* b;
    T* x;
    T* r;
    ZPair<T>* zp[2];  // by parity: {z, p} per row
    T* q;
};

struct Team {
    GridBarrier* bar;
    double* part;  // NSLOT * G doubles
    int G;         // workgroups in the team
    int L;         // this workgroup's index in the team
    unsigned gen;  // thread 0's copy of the barrier generation
    long long limit;
    int* s_flag;   // LDS word used by the barrier

    __device__ __forceinline__ bool sync()
    {
        if (G == 1) {
            __syncthreads();
            return true;
        }
        return grid_barrier(bar, (unsigned)G, gen, limit, s_flag);
    }
    // Base of reduction group s: the group's K quantities, interleaved per block.
    __device__ __forceinline__ double* slot(int s) const { return part + (size_t)s * G; }
};

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c)
{
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c)
{
    return __builtin_fmaf(a, b, c);
}

template <typename T>
struct BD {
    T b, d;
};

// Rows [x, y) of workgroup L's tiles (empty when it owns none).
__device__ __forceinline__ int2 tile_row_range(const TileMap& tm, int L)
{
    const int tb = L * tm.per_block, t1 = min(tb + tm.per_block, tm.T);
    if (tb >= t1) return int2{0, 0};
    return int2{tm.tiles[tb].x, tm.tiles[t1 - 1].y};
}

// Step A: p_new = z + beta p_old (or z on the first step), q = A p_new over the
// workgroup's tiles, p_new formed on the fly in the gather of {z, p_old} from
// `cur` and stored into `nxt` (whose z half is dead until step B).  Returns
// this thread's share of p_new' q.
template <int NPL, typename T>
__device__ __forceinline__ double step_a(const SysView<T>& s, const TileMap& tm, int L, T* prod, bool first, T beta,
                                         const ZPair<T>* __restrict__ cur, ZPair<T>* __restrict__ nxt)
{
    T* __restrict__ q = s.q;
    double sig = 0.0;
    if (first) {
        tile_rows<NPL, T>(
            s.rowptr, s.col, s.val, tm, L, prod, [&](int j) { return cur[j].z; }, Ident<T>{},
            [&](int i) { return cur[i].z; },
            [&](int i, T qi, T pi) {
                nxt[i] = ZPair<T>{T(0), pi};
                q[i] = qi;
                sig += (double)pi * (double)qi;
            },
            NoPrologue{});
    } else {
        tile_rows<NPL, T>(
            s.rowptr, s.col, s.val, tm, L, prod, [&](int j) { return cur[j]; },
            [&](ZPair<T> g) { return fma_t(beta, g.p, g.z); }, [&](int i) { return cur[i]; },
            [&](int i, T qi, ZPair<T> o) {
                const T pi = fma_t(beta, o.p, o.z);
                nxt[i] = ZPair<T>{T(0), pi};
                q[i] = qi;
                sig += (double)pi * (double)qi;
            },
            NoPrologue{});
    }
    return sig;
}

// Step B: x += alpha p, r -= alpha q, z = M^-1 r with p and z in `zp`; shares
// of r'z and r'r.
template <int BS, typename T>
__device__ __forceinline__ void step_b(const SysView<T>& s, int rs, int re, T alpha, ZPair<T>* __restrict__ zp,
                                       double& rz, double& rr)
{
    for (int i = rs + (int)threadIdx.x; i < re; i += BS) {
        const T pi = zp[i].p, qi = s.q[i];
        s.x[i] = fma_t(alpha, pi, s.x[i]);
        const T ri = fma_t(-alpha, qi, s.r[i]);
        s.r[i] = ri;
        const T zi = s.dinv[i] * ri;
        zp[i] = ZPair<T>{zi, pi};
        rz += (double)ri * (double)zi;
        rr += (double)ri * (double)ri;
    }
}

// Step R: rout = b - A x and, if zout, zout[i].z = M^-1 rout over the
// workgroup's tiles; shares of r'r, r'z, b'b.
template <int NPL, typename T>
__device__ __forceinline__ void step_r(const SysView<T>& s, const TileMap& tm, int L, T* prod, T* __restrict__ rout,
                                       ZPair<T>* __restrict__ zout, double& rr, double& rz, double& bb)
{
    const T* __restrict__ x = s.x;
    tile_rows<NPL, T>(
        s.rowptr, s.col, s.val, tm, L, prod, [&](int j) { return x[j]; }, Ident<T>{},
        [&](int i) { return BD<T>{s.b[i], s.dinv[i]}; },
        [&](int i, T ax, BD<T> o) {
            const T ri = o.b - ax;
            rout[i] = ri;
            rr += (double)ri * (double)ri;
            bb += (double)o.b * (double)o.b;
            if (zout) {
                const T zi = o.d * ri;
                zout[i].z = zi;
                rz += (double)ri * (double)zi;
            }
        },
        NoPrologue{});
}

// One full Jacobi-PCG solve of system s by team t, following the loop of the
// FP64 oracle step for step (residual replacement included).  Every decision
// is taken on team-reduced scalars that are bitwise identical in every
// workgroup, so all workgroups leave the loop together.  Returns the status;
// workgroup 0 of the team writes *info (and hist[k] = ||r_k|| / ||b||).
template <int NPL, int BS, typename T>
__device__ int pcg_team(const SysView<T>& s, Team& t, const TileMap& tm, T* prod, double tol, int maxit,
                        double* lds, DevInfo* info, double* hist)
{
    const bool writer = (t.L == 0 && threadIdx.x == 0);
    const int2 rows = tile_row_range(tm, t.L);
    const int rs = rows.x, re = rows.y;
    int status = CG_MAXIT, k = 0, repl = 0;
    double nb = 0.0, rr = 0.0, rrt = -1.0;

    {   // r0 = b - A x0, z0 = M^-1 r0, ||b||^2, ||r0||^2, r0'z0
        double v[3] = {0.0, 0.0, 0.0};
        step_r<NPL, T>(s, tm, t.L, prod, s.r, s.zp[0], v[0], v[1], v[2]);
        block_partials<BS, 3>(v, lds, t.slot(SLOT_SETUP), t.L);
    }
    if (!t.sync()) return CG_ETIMEOUT;
    double rho;
    {
        double g[3];
        grid_sum<BS, 3>(t.slot(SLOT_SETUP), t.G, g, lds);
        rr = g[0];
        rho = g[1];
        nb = sqrt(g[2]);
        if (writer) info->bb = g[2];
    }
    if (nb == 0.0) {
        for (int i = rs + (int)threadIdx.x; i < re; i += BS) s.x[i] = T(0);
        if (writer) {
            *info = DevInfo{0, CG_CONVERGED, 0, 0, 0.0, 0.0, 0.0, 0.0};
            if (hist) hist[0] = 0.0;
        }
        return CG_CONVERGED;
    }
    const double thr = tol * nb;
    if (writer && hist) hist[0] = sqrt(rr) / nb;
    if (sqrt(rr) <= thr) {
        if (writer) {
            info->iters = 0;
            info->status = CG_CONVERGED;
            info->replacements = 0;
            info->rr_recur = rr;
            info->rr_true = rr;
        }
        return CG_CONVERGED;
    }

    double beta = 0.0;
    while (k < maxit) {
        // zp[k & 1] holds {z_k, p_k}; p_{k+1} and then z_{k+1} go to the other.
        const ZPair<T>* cur = (k & 1) ? s.zp[1] : s.zp[0];  // selects, not a dynamic index: s is local
        ZPair<T>* nxt = (k & 1) ? s.zp[0] : s.zp[1];
        {
            double v[1] = {step_a<NPL, T>(s, tm, t.L, prod, k == 0, (T)beta, cur, nxt)};
            block_partials<BS, 1>(v, lds, t.slot(SLOT_SIG), t.L);
        }
        if (!t.sync()) return CG_ETIMEOUT;
        double sigma;
        {
            double g[1];
            grid_sum<BS, 1>(t.slot(SLOT_SIG), t.G, g, lds);
            sigma = g[0];
        }
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            status = CG_BREAKDOWN;
            break;
        }
        const double alpha = rho / sigma;
        {
            double v[2] = {0.0, 0.0};
            step_b<BS, T>(s, rs, re, (T)alpha, nxt, v[0], v[1]);
            block_partials<BS, 2>(v, lds, t.slot(SLOT_ITER), t.L);
        }
        ++k;
        if (!t.sync()) return CG_ETIMEOUT;
        double rz;
        {
            double g[2];
            grid_sum<BS, 2>(t.slot(SLOT_ITER), t.G, g, lds);
            rz = g[0];
            rr = g[1];
        }
        if (writer && hist) hist[k] = sqrt(rr) / nb;
        if (sqrt(rr) <= thr) {
            // Continue-condition met on the recurrence: confirm on b - A x.
            {
                double v[2] = {0.0, 0.0}, unused = 0.0;
                step_r<NPL, T>(s, tm, t.L, prod, s.r, (k & 1) ? s.zp[1] : s.zp[0], v[0], v[1], unused);
                block_partials<BS, 2>(v, lds, t.slot(SLOT_CHECK), t.L);
            }
            if (!t.sync()) return CG_ETIMEOUT;
            double g[2];
            grid_sum<BS, 2>(t.slot(SLOT_CHECK), t.G, g, lds);
            if (sqrt(g[0]) <= thr) {
                status = CG_CONVERGED;
                rrt = g[0];
                break;
            }
            ++repl;  // r and z now hold the true residual and its preconditioned form
            rz = g[1];
        }
        if (!(rz > 0.0) || !isfinite(rz)) {
            status = CG_BREAKDOWN;
            break;
        }
        beta = rz / rho;
        rho = rz;
    }

    if (rrt < 0.0) {  // report the true residual of the returned x
        double v[1] = {0.0}, unused0 = 0.0, unused1 = 0.0;
        step_r<NPL, T>(s, tm, t.L, prod, s.q, (ZPair<T>*)nullptr, v[0], unused0, unused1);
        block_partials<BS, 1>(v, lds, t.slot(SLOT_CHECK), t.L);
        if (!t.sync()) return CG_ETIMEOUT;
        double g[1];
        grid_sum<BS, 1>(t.slot(SLOT_CHECK), t.G, g, lds);
        rrt = g[0];
    }
    if (writer) {
        info->iters = k;
        info->status = status;
        info->replacements = repl;
        info->rr_recur = rr;
        info->rr_true = rrt;
    }
    return status;
}

}  // namespace jpcg
