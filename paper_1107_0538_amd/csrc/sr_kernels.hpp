// Single-reduction Jacobi-PCG (Chronopoulos and Gear's form of the same
// iteration: s = A p carried by a recurrence): one kernel per iteration.
//
// Iteration k (the oracle's single-reduction loop, same symbols):
//   sigma_k = p_{k-1}' s_{k-1},  alpha_k = gamma_{k-1} / sigma_k, where
//     p_{k-1} = u_{k-1} + beta_{k-1} p_{k-2},  s_{k-1} = w_{k-1} + beta_{k-1} s_{k-2}
//   x_k = x_{k-1} + alpha_k p_{k-1},  r_k = r_{k-1} - alpha_k s_{k-1},  u_k = M^-1 r_k
//   w_k = A u_k;  one reduction of
//     gamma_k = r_k'u_k, delta_k = w_k'u_k, ||r_k||^2,
//     e_k = u_k's_{k-1} + p_{k-1}'w_k, f_k = p_{k-1}'s_{k-1}
// so that the next kernel obtains p_k's_k without a second reduction:
//     sigma_{k+1} = delta_k + beta_k e_k + beta_k^2 f_k,  beta_k = gamma_k / gamma_{k-1}.
// (Chronopoulos and Gear's scalar recurrence sigma = delta - beta gamma / alpha
// assumes r_k'u_{k-1} = 0, which a residual replacement near the attainable
// accuracy destroys; it then turns negative for an SPD matrix.)
// Kernel K_k reduces the previous kernel's partials in its prologue, applies
// the continue-condition to r_{k-1}, and forms every gathered u_k(j) on the
// fly from r_{k-1}, w_{k-1}, s_{k-2} and M^-1 of column j with exactly the
// expressions the owning row lane uses, so w_k = A u_k for the u_k that the
// row lanes store implicitly.  The gathered vectors r, w and s and the Jacobi
// diagonal are stored together, SrQuad {r, w, s, d} per row, in two arrays
// used by iteration parity (one 32-byte gather per nonzero; kernels store
// whole quads where they can); p and x update in place (no other row reads
// them).
//
// After a residual replacement the auxiliary vectors are recomputed from
// their definitions (the replacement strategy for these forms analysed by
// Cools, Yetkin, Agullo, Giraud and Vanroose, 2018): the restart kernel forms
// w = A u for the replaced r and s = A p_{k-1}, with the same five partials,
// and the next kernel proceeds as after any other iteration.
#pragma once

#include "tiles.hpp"

namespace jpcg {

struct SrState {
    int stop;
    int kk[2];   // kk[P] = iterations done after the kernel of parity P
    int k_done;  // iterations done when a kernel raised the stop flag
    int maxit;
    int replacements;
    double nb, thr;
    double gam[2];    // gam[P] = gamma_{k-1}, written by K_k (P = k % 2)
    double rr;        // ||r||^2 at the last continue-condition test
    double rr_true;   // ||b - A x||^2 of the returned x
};

// Partials per workgroup and iteration: gamma, delta, ||r||^2, e, f.
constexpr int kSrPart = 5;

struct alignas(32) SrQuad {
    double r, w, s, d;
};

struct SrArgs {
    int n;
    const int* __restrict__ rowptr;
    const int* __restrict__ col;
    const double* __restrict__ val;
    const double* __restrict__ dinv;
    const double* b;
    double* x;
    SrQuad* qd[2];  // by parity: {r, w, s, d} per row
    double* p;
    TileMap tm;
    int G;
    double* part[2];     // [G][kSrPart]: gamma, delta, r'r, e, f from the kernel of parity P
    double* part_setup;  // [G][2]: r'r, b'b of r0
    double* part_chk;    // [G][1]: ||b - A x||^2 (check and report)
    SrState* st;
    double* hist;
};

template <int NPL, int BS>
struct SrLds {
    double red[(BS / kWave) * 4];
    double prod[BS * NPL];
};

__device__ __forceinline__ int sr_logical(const SrArgs& a) { return xcd_logical_block((int)blockIdx.x, a.G); }
__device__ __forceinline__ bool sr_leader(const SrArgs& a) { return threadIdx.x == 0 && sr_logical(a) == 0; }

struct Six {
    SrQuad q;
    double p, x;
};

// qd[0] = {r0 = b - A x0, 0, 0, d}; clears p (s and p are read with a zero
// beta on the first iteration); partials of r'r and b'b.
template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_sr_setup(SrArgs a)
{
    __shared__ SrLds<NPL, BS> sh;
    double v[2] = {0.0, 0.0};
    const double* __restrict__ x = a.x;
    tile_rows<NPL, double>(
        a.rowptr, a.col, a.val, a.tm, sr_logical(a), sh.prod + (threadIdx.x / kWave) * (kWave * NPL),
        [&](int j) { return x[j]; }, Ident<double>{}, [&](int i) { return Pair2{a.b[i], a.dinv[i]}; },
        [&](int i, double ax, Pair2 bd) {
            const double bi = bd.a;
            const double ri = bi - ax;
            a.qd[0][i] = SrQuad{ri, 0.0, 0.0, bd.b};
            a.p[i] = 0.0;
            v[0] += ri * ri;
            v[1] += bi * bi;
        },
        NoPrologue{});
    block_partials<BS, 2>(v, sh.red, a.part_setup, sr_logical(a));
}

// Initial tests, then w0 = A u0 into qd[0].w with the partials of (gamma0,
// delta0, ||r0||^2) in part[0].
template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_sr_first(SrArgs a, double tol, int maxit)
{
    __shared__ SrLds<NPL, BS> sh;
    double g[2];
    wave_grid_sum<2>(a.part_setup, a.G, g);
    const double rr = g[0], nb = sqrt(g[1]), thr = tol * nb;
    SrState* st = a.st;
    if (sr_leader(a)) {
        st->kk[0] = 0;
        st->kk[1] = 0;
        st->k_done = 0;
        st->maxit = maxit;
        st->replacements = 0;
        st->nb = nb;
        st->thr = thr;
        st->rr = rr;
        st->rr_true = -1.0;
        if (a.hist) a.hist[0] = nb > 0.0 ? sqrt(rr) / nb : 0.0;
        st->stop = nb == 0.0 ? STOP_ZERO_RHS : (sqrt(rr) <= thr ? STOP_CONV0 : RUNNING);
        if (nb == 0.0) st->rr_true = 0.0;
        else if (sqrt(rr) <= thr) st->rr_true = rr;
    }
    if (nb == 0.0) {
        // x = 0 over this workgroup's tile rows.
        const int tb = sr_logical(a) * a.tm.per_block, t1 = min(tb + a.tm.per_block, a.tm.T);
        if (tb < t1) {
            const int rs = a.tm.tiles[tb].x, re = a.tm.tiles[t1 - 1].y;
            for (int i = rs + (int)threadIdx.x; i < re; i += BS) a.x[i] = 0.0;
        }
        return;
    }
    if (sqrt(rr) <= thr) return;
    SrQuad* __restrict__ q0 = a.qd[0];
    // p and s start at zero, so e = f = 0 and sigma_1 = delta_0.
    double v[kSrPart] = {0.0, 0.0, 0.0, 0.0, 0.0};
    tile_rows<NPL, double>(
        a.rowptr, a.col, a.val, a.tm, sr_logical(a), sh.prod + (threadIdx.x / kWave) * (kWave * NPL),
        // Gathers read only the r and d halves; row steps write only w.
        [&](int j) { return Pair2{q0[j].r, q0[j].d}; }, [&](Pair2 rd) { return rd.b * rd.a; },
        [&](int i) { return Pair2{q0[i].r, q0[i].d}; },
        [&](int i, double wi, Pair2 rd) {
            const double ui = rd.b * rd.a;
            q0[i].w = wi;
            v[0] += rd.a * ui;
            v[1] += wi * ui;
            v[2] += rd.a * rd.a;
        },
        NoPrologue{});
    block_partials<BS, kSrPart>(v, sh.red, a.part[0], sr_logical(a));
}

// K_k, parity P = k % 2.
template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_sr_iter(SrArgs a, int P)
{
    __shared__ SrLds<NPL, BS> sh;
    SrState* st = a.st;
    const int Q = P ^ 1;
    const SrQuad* __restrict__ qold = a.qd[Q];  // {r_{k-1}, w_{k-1}, s_{k-2}, d}
    SrQuad* __restrict__ qnew = a.qd[P];        // {r_k, w_k, s_{k-1}, d}
    const bool lead = sr_leader(a);
    double alpha = 0.0, beta = 0.0, gam_prev = 0.0;
    int km1 = 0;
    bool go = false;
    __shared__ double s_g[kSrPart];
    auto prologue = [&]() -> bool {
        const int stop = st->stop, maxit = st->maxit;
        km1 = st->kk[Q];
        const double thr = st->thr, nb = st->nb, gam2 = st->gam[Q];
        // Wave 0 reduces the partials for the workgroup (every wave calls the
        // prologue exactly once, so the barrier is met by all of them).
        if (threadIdx.x < kWave) {
            double g0[kSrPart];
            wave_grid_sum<kSrPart>(a.part[Q], a.G, g0);
            if (threadIdx.x == 0) {
#pragma unroll
                for (int j = 0; j < kSrPart; ++j) s_g[j] = g0[j];
            }
        }
        __syncthreads();
        const double gam = s_g[0], delta = s_g[1], rr = s_g[2];
        if (stop != RUNNING) return false;
        if (lead) {
            st->rr = rr;
            if (a.hist) a.hist[km1] = sqrt(rr) / nb;
        }
        // The oracle's order: continue-condition, breakdown of gamma, iteration
        // limit, then breakdown of sigma at the top of the next iteration.
        int code = RUNNING;
        double sigma = delta;
        if (sqrt(rr) <= thr) code = STOP_CHECK;
        else if (!(gam > 0.0) || !isfinite(gam)) code = STOP_BREAKDOWN;
        else if (km1 >= maxit) code = STOP_MAXIT;
        else {
            if (km1 > 0) {
                beta = gam / gam2;
                // p's with p = u + beta p_old, s = w + beta s_old, expanded.
                sigma = delta + beta * s_g[3] + beta * beta * s_g[4];
            }
            if (!(sigma > 0.0) || !isfinite(sigma)) code = STOP_BREAKDOWN;
        }
        if (code != RUNNING) {
            if (lead) {
                st->k_done = km1;
                st->stop = code;
            }
            return false;
        }
        alpha = gam / sigma;
        gam_prev = gam;
        go = true;
        return true;
    };
    double v[kSrPart] = {0.0, 0.0, 0.0, 0.0, 0.0};
    tile_rows<NPL, double>(
        a.rowptr, a.col, a.val, a.tm, sr_logical(a), sh.prod + (threadIdx.x / kWave) * (kWave * NPL),
        [&](int j) { return qold[j]; },
        [&](SrQuad q) {
            const double s1 = __builtin_fma(beta, q.s, q.w);
            return q.d * __builtin_fma(-alpha, s1, q.r);
        },
        [&](int i) { return Six{qold[i], a.p[i], a.x[i]}; },
        [&](int i, double wi, Six o) {
            const double u0 = o.q.d * o.q.r;
            const double pi = __builtin_fma(beta, o.p, u0);
            const double si = __builtin_fma(beta, o.q.s, o.q.w);
            const double ri = __builtin_fma(-alpha, si, o.q.r);
            const double ui = o.q.d * ri;
            a.p[i] = pi;
            a.x[i] = __builtin_fma(alpha, pi, o.x);
            qnew[i] = SrQuad{ri, wi, si, o.q.d};
            v[0] += ri * ui;
            v[1] += wi * ui;
            v[2] += ri * ri;
            v[3] += ui * si + pi * wi;
            v[4] += pi * si;
        },
        prologue);
    if (!go) return;  // the same decision in every wave of every workgroup
    block_partials<BS, kSrPart>(v, sh.red, a.part[P], sr_logical(a));
    if (lead) {
        st->kk[P] = km1 + 1;
        st->gam[P] = gam_prev;
    }
}

// ||b - A x||^2 into part_chk; with replace, the true residual replaces qd[P].r.
template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_sr_residual(SrArgs a, int P, int replace)
{
    __shared__ SrLds<NPL, BS> sh;
    double v[1] = {0.0};
    const double* __restrict__ x = a.x;
    SrQuad* __restrict__ qout = a.qd[P];
    tile_rows<NPL, double>(
        a.rowptr, a.col, a.val, a.tm, sr_logical(a), sh.prod + (threadIdx.x / kWave) * (kWave * NPL),
        [&](int j) { return x[j]; }, Ident<double>{}, [&](int i) { return a.b[i]; },
        [&](int i, double ax, double bi) {
            const double ri = bi - ax;
            if (replace) qout[i].r = ri;
            v[0] += ri * ri;
        },
        NoPrologue{});
    block_partials<BS, 1>(v, sh.red, a.part_chk, sr_logical(a));
}

// One workgroup: accept (CONVERGED) or resume after replacement; with
// report != 0 only record ||b - A x||^2.
template <int BS>
__global__ __launch_bounds__(BS) void k_sr_decide(SrArgs a, int report)
{
    double g[1];
    wave_grid_sum<1>(a.part_chk, a.G, g);
    if (threadIdx.x == 0) {
        SrState* st = a.st;
        if (report) {
            st->rr_true = g[0];
        } else if (sqrt(g[0]) <= st->thr) {
            st->stop = STOP_CONVERGED;
            st->rr_true = g[0];
        } else {
            st->stop = RUNNING;
            st->replacements += 1;
        }
    }
}

// After a replacement at iteration k (parity P): w_k = A M^-1 r_k for the
// replaced r in qd[P].w and s = A p_{k-1} in qd[P].s, with the five partials
// of the iteration kernel (gamma, delta, r'r, u'(A p) + p'w, p'(A p)) in
// part[P], so the next kernel continues as after an ordinary iteration.
struct Rdp {
    double r, d, p;
};

template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_sr_restart(SrArgs a, int P)
{
    __shared__ SrLds<NPL, BS> sh;
    SrQuad* __restrict__ q = a.qd[P];
    const double* __restrict__ p = a.p;
    double* prod = sh.prod + (threadIdx.x / kWave) * (kWave * NPL);
    double v[kSrPart] = {0.0, 0.0, 0.0, 0.0, 0.0};
    tile_rows<NPL, double>(
        a.rowptr, a.col, a.val, a.tm, sr_logical(a), prod,
        [&](int j) { return Pair2{q[j].r, q[j].d}; }, [&](Pair2 rd) { return rd.b * rd.a; },
        [&](int i) { return Rdp{q[i].r, q[i].d, p[i]}; },
        [&](int i, double wi, Rdp o) {
            const double ui = o.d * o.r;
            q[i].w = wi;
            v[0] += o.r * ui;
            v[1] += wi * ui;
            v[2] += o.r * o.r;
            v[3] += o.p * wi;
        },
        NoPrologue{});
    // The second product's gathers read only p, and its row steps write only
    // the s half of the quads, so the first product's w stores cannot race.
    tile_rows<NPL, double>(
        a.rowptr, a.col, a.val, a.tm, sr_logical(a), prod, [&](int j) { return p[j]; }, Ident<double>{},
        [&](int i) { return Pair2{p[i], q[i].d * q[i].r}; },
        [&](int i, double si, Pair2 pu) {
            q[i].s = si;
            v[3] += pu.b * si;
            v[4] += pu.a * si;
        },
        NoPrologue{});
    block_partials<BS, kSrPart>(v, sh.red, a.part[P], sr_logical(a));
}

}  // namespace jpcg
