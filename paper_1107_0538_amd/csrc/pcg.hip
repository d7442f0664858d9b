// Single-system Jacobi-PCG on one MI355X: create, solve, spmv.
//
// The paper's case study (Section IV) runs the CG loop on the host and the
// repetitive vector and matrix work on the GPU, crossing the bus every
// iteration.  Here the scalars (alpha, beta, the continue-condition) never
// leave the device.  Each iteration is two kernels:
//
//   A_k  (direction + SpMV + dot)  reduce the previous B's partials of r'z and
//        r'r, apply the continue-condition / breakdown / iteration-limit
//        tests, beta_k = rho_{k-1} / rho_{k-2}; p_k = z + beta_k p_{k-1} formed
//        on the fly inside the product q = A p_k; partials of p_k' q.
//   B_k  (update)  reduce A_k's partials, alpha_k = rho_{k-1} / sigma_k;
//        x += alpha p, r -= alpha q, z = M^-1 r; partials of r'z and r'r.
//
// Every workgroup reduces the previous kernel's per-workgroup partials itself,
// in a fixed order, so all workgroups reach the same bits and the same
// decision without atomics (measured on MI355X, a last-workgroup ticket costs
// far more than the redundant reduction).  Scalars that must outlive a kernel
// sit in a small state block, double-buffered by iteration parity so that no
// kernel reads a slot it writes.  Iterations are launched in hipGraph chunks;
// once a kernel raises the stop flag the rest of the chunk returns at once.
// When the recurrence residual passes the test the host runs the true-
// residual check (and the residual replacement, if the check fails) between
// chunks, exactly where the FP64 oracle does.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "context.hpp"
#include "tiles.hpp"

namespace jpcg {

enum StopCode : int {
    RUNNING = 0,
    STOP_ZERO_RHS = 1,   // ||b|| = 0: x = 0
    STOP_CONV0 = 2,      // x0 already satisfies the test
    STOP_CHECK = 3,      // recurrence residual passed: confirm on b - A x
    STOP_MAXIT = 4,
    STOP_BREAKDOWN = 5,
    STOP_CONVERGED = 6,  // confirmed
};

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
};

struct CgArgs {
    SysView<double> s;  // b, x are the context's copies; p0/p1 alternate by parity
    TileMap tm;         // tiles of the sparse products, per workgroup
    int R;              // rows per workgroup of the elementwise update
    int G;
    double* part_setup;    // [G][3]: r'r, r'z, b'b of r0
    double* part_sig;      // [G][1]: p'q
    double* part_iter[2];  // [G][2]: r'z, r'r after B of parity P (or a check)
    double* part_rep;      // [G][1]: ||b - A x||^2 for the report
    CgState* st;
    double* hist;
};

template <int NPL, int BS>
struct Lds {
    double red[(BS / kWave) * 4];
    double prod[BS * NPL];  // per wave: 64 * NPL products
};

template <int NPL>
__device__ __forceinline__ double* wave_prod(double* prod)
{
    return prod + (threadIdx.x / kWave) * (kWave * NPL);
}

__device__ __forceinline__ int logical(const CgArgs& a) { return xcd_logical_block((int)blockIdx.x, a.G); }

__device__ __forceinline__ bool leader(const CgArgs& a) { return threadIdx.x == 0 && logical(a) == 0; }

struct Pair {
    double a, b;
};

// r_out = b - A x and (if z_out) z_out = M^-1 r_out over the workgroup's tiles;
// shares of r'r, r'z, b'b.
template <int NPL, int BS>
__device__ __forceinline__ void tile_residual(const CgArgs& a, double* prod, double* r_out, double* z_out,
                                              double& rr, double& rz, double& bb)
{
    const SysView<double>& s = a.s;
    const double* __restrict__ x = s.x;
    tile_rows<NPL, double>(
        s.rowptr, s.col, s.val, a.tm, logical(a), wave_prod<NPL>(prod), [&](int j) { return x[j]; }, Mul<double>{},
        [&](int i) { return Pair{s.b[i], s.dinv[i]}; },
        [&](int i, double ax, Pair bd) {
            const double bi = bd.a;
            const double ri = bi - ax;
            r_out[i] = ri;
            rr += ri * ri;
            bb += bi * bi;
            if (z_out) {
                const double zi = bd.b * ri;
                z_out[i] = zi;
                rz += ri * zi;
            }
        },
        NoPrologue{});
}

template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_setup(CgArgs a)
{
    __shared__ Lds<NPL, BS> sh;
    double v[3] = {0.0, 0.0, 0.0};
    tile_residual<NPL, BS>(a, sh.prod, a.s.r, a.s.z, v[0], v[1], v[2]);
    block_partials<BS, 3>(v, sh.red, a.part_setup, logical(a));
}

// A_1: initial tests, then p_1 = z_0, q = A p_1.
template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_first(CgArgs a, double tol, int maxit)
{
    __shared__ Lds<NPL, BS> sh;
    double g[3];
    wave_grid_sum<3>(a.part_setup, a.G, g);
    const double rr = g[0], rho = g[1], nb = sqrt(g[2]), thr = tol * nb;
    CgState* st = a.st;
    const SysView<double>& s = a.s;
    if (leader(a)) {
        st->k = 0;
        st->maxit = maxit;
        st->replacements = 0;
        st->nb = nb;
        st->thr = thr;
        st->rho[1] = rho;
        st->rr = rr;
        st->rr_true = -1.0;
        if (a.hist) a.hist[0] = nb > 0.0 ? sqrt(rr) / nb : 0.0;
        st->stop = nb == 0.0 ? STOP_ZERO_RHS : (sqrt(rr) <= thr ? STOP_CONV0 : RUNNING);
        if (nb == 0.0) st->rr_true = 0.0;
        else if (sqrt(rr) <= thr) st->rr_true = rr;
    }
    if (nb == 0.0) {
        const int L = logical(a);
        const int rs = min(L * a.R, s.n), re = min(rs + a.R, s.n);
        for (int i = rs + (int)threadIdx.x; i < re; i += BS) s.x[i] = 0.0;
        return;
    }
    if (sqrt(rr) <= thr) return;
    const double* __restrict__ z = s.z;
    double sig = 0.0;
    tile_rows<NPL, double>(
        s.rowptr, s.col, s.val, a.tm, logical(a), wave_prod<NPL>(sh.prod), [&](int j) { return z[j]; },
        Mul<double>{}, [&](int i) { return z[i]; },
        [&](int i, double qi, double pi) {
            s.p1[i] = pi;
            s.q[i] = qi;
            sig += pi * qi;
        },
        NoPrologue{});
    double v[1] = {sig};
    block_partials<BS, 1>(v, sh.red, a.part_sig, logical(a));
}

// A_k, k >= 2, parity P = k % 2.  The scalar work (reducing the previous B's
// partials, the tests, beta) runs as the tile walk's prologue, after the
// first gathers are issued, so its memory latency overlaps theirs.
template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_direction(CgArgs a, int P)
{
    __shared__ Lds<NPL, BS> sh;
    CgState* st = a.st;
    const SysView<double>& s = a.s;
    const double* __restrict__ z = s.z;
    const double* __restrict__ pold = P ? s.p0 : s.p1;
    double* __restrict__ pnew = P ? s.p1 : s.p0;
    const bool lead = leader(a);
    double beta = 0.0, sig = 0.0;
    bool go = true;
    auto prologue = [&]() -> bool {
        const int stop = st->stop, km1 = st->k, maxit = st->maxit;
        const double thr = st->thr, nb = st->nb, rho_prev = st->rho[P ^ 1];
        double g[2];
        wave_grid_sum<2>(a.part_iter[P ^ 1], a.G, g);
        const double rz = g[0], rr = g[1];
        go = false;
        if (stop != RUNNING) return false;
        if (lead) {
            st->rr = rr;
            if (a.hist) a.hist[km1] = sqrt(rr) / nb;
        }
        // The oracle's order: continue-condition, breakdown of r'z, iteration limit.
        if (sqrt(rr) <= thr) {
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
        beta = rz / rho_prev;
        if (lead) {
            st->rho[P] = rz;
            st->beta = beta;
        }
        go = true;
        return true;
    };
    tile_rows<NPL, double>(
        s.rowptr, s.col, s.val, a.tm, logical(a), wave_prod<NPL>(sh.prod),
        [&](int j) { return Pair{z[j], pold[j]}; },
        [&](double v, Pair zp) { return v * __builtin_fma(beta, zp.b, zp.a); },
        [&](int i) { return Pair{z[i], pold[i]}; },
        [&](int i, double qi, Pair zp) {
            const double pi = __builtin_fma(beta, zp.b, zp.a);
            pnew[i] = pi;
            s.q[i] = qi;
            sig += pi * qi;
        },
        prologue);
    if (!go) return;  // the same decision in every wave of every workgroup
    double v[1] = {sig};
    block_partials<BS, 1>(v, sh.red, a.part_sig, logical(a));
}

// B_k, parity P = k % 2.  Rows are split arithmetically; the state, the row
// operands and the partials of sigma are all requested before any is used.
template <int BS>
__global__ __launch_bounds__(BS) void k_update(CgArgs a, int P)
{
    __shared__ Lds<1, BS> sh;
    CgState* st = a.st;
    const SysView<double>& s = a.s;
    const int stop = st->stop;
    const double rho = st->rho[P];
    const int L = logical(a);
    const int rs = min(L * a.R, s.n), re = min(rs + a.R, s.n);
    const double* __restrict__ p = P ? s.p1 : s.p0;
    const int i0 = rs + (int)threadIdx.x;
    const bool h0 = i0 < re;
    const int ic = h0 ? i0 : 0;
    const double p0 = p[ic], q0 = s.q[ic], x0 = s.x[ic], r0 = s.r[ic], d0 = s.dinv[ic];
    double g[1];
    wave_grid_sum<1>(a.part_sig, a.G, g);
    const double sigma = g[0];
    if (stop != RUNNING) return;
    const bool lead = leader(a);
    if (!(sigma > 0.0) || !isfinite(sigma)) {
        if (lead) st->stop = STOP_BREAKDOWN;
        return;
    }
    const double alpha = rho / sigma;
    double v[2] = {0.0, 0.0};
    if (h0) {
        s.x[i0] = __builtin_fma(alpha, p0, x0);
        const double ri = __builtin_fma(-alpha, q0, r0);
        s.r[i0] = ri;
        const double zi = d0 * ri;
        s.z[i0] = zi;
        v[0] += ri * zi;
        v[1] += ri * ri;
    }
    for (int i = i0 + BS; i < re; i += BS) {
        s.x[i] = __builtin_fma(alpha, p[i], s.x[i]);
        const double ri = __builtin_fma(-alpha, s.q[i], s.r[i]);
        s.r[i] = ri;
        const double zi = s.dinv[i] * ri;
        s.z[i] = zi;
        v[0] += ri * zi;
        v[1] += ri * ri;
    }
    block_partials<BS, 2>(v, sh.red, a.part_iter[P], L);
    if (lead) {
        st->k = st->k + 1;
        st->sigma = sigma;
        st->alpha = alpha;
    }
}

// True residual r = b - A x, z = M^-1 r into the slot the next A_{k+1} reads.
template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_check(CgArgs a, int P)
{
    __shared__ Lds<NPL, BS> sh;
    double rr = 0.0, rz = 0.0, bb = 0.0;
    tile_residual<NPL, BS>(a, sh.prod, a.s.r, a.s.z, rr, rz, bb);
    double v[2] = {rz, rr};
    block_partials<BS, 2>(v, sh.red, a.part_iter[P], logical(a));
}

// One workgroup: accept the solve, or resume with the replaced residual.
template <int BS>
__global__ __launch_bounds__(BS) void k_check_decide(CgArgs a, int P)
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
        }
    }
}

// ||b - A x||^2 of the returned x, for solves that end without convergence.
template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_report(CgArgs a)
{
    __shared__ Lds<NPL, BS> sh;
    double v[1] = {0.0};
    double rz = 0.0, bb = 0.0;
    tile_residual<NPL, BS>(a, sh.prod, a.s.q, (double*)nullptr, v[0], rz, bb);
    block_partials<BS, 1>(v, sh.red, a.part_rep, logical(a));
}

template <int BS>
__global__ __launch_bounds__(BS) void k_report_sum(CgArgs a)
{
    double g[1];
    wave_grid_sum<1>(a.part_rep, a.G, g);
    if (threadIdx.x == 0) a.st->rr_true = g[0];
}

// y = A x over the solver's tiles (rows summed in stored order).
template <int NPL, int BS>
__global__ __launch_bounds__(BS) void k_spmv(CgArgs a, const double* __restrict__ x, double* __restrict__ y)
{
    __shared__ Lds<NPL, BS> sh;
    tile_rows<NPL, double>(a.s.rowptr, a.s.col, a.s.val, a.tm, logical(a), wave_prod<NPL>(sh.prod),
                           [&](int j) { return x[j]; }, Mul<double>{}, NoPre{},
                           [&](int i, double v, int) { y[i] = v; }, NoPrologue{});
}

// dinv_i = 1 / a_ii (Jacobi) or 1 (no preconditioner); flags a missing or
// non-positive diagonal.
__global__ void jacobi_kernel(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                              const double* __restrict__ val, int jacobi, double* __restrict__ dinv,
                              float* __restrict__ dinv32, int* __restrict__ bad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double inv = 1.0;
    if (jacobi) {
        double d = 0.0;
        int found = 0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i) {
                d += val[k];
                found = 1;
            }
        if (!found || !(d > 0.0)) atomicOr(bad, 1);
        inv = 1.0 / d;
    }
    dinv[i] = inv;
    if (dinv32) dinv32[i] = (float)inv;
}

__global__ void cast_f32_kernel(int64_t n, const double* __restrict__ in, float* __restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

// ---------------------------------------------------------------------------
// Kernel tables per launch shape
// ---------------------------------------------------------------------------
struct CgKernels {
    const void* spmv;
    const void* setup;
    const void* first;
    const void* direction;
    const void* update;
    const void* check;
    const void* check_decide;
    const void* report;
    const void* report_sum;
};

template <int NPL, int BS>
static CgKernels kernels_for()
{
    return CgKernels{(const void*)k_spmv<NPL, BS>,      (const void*)k_setup<NPL, BS>,
                     (const void*)k_first<NPL, BS>,     (const void*)k_direction<NPL, BS>,
                     (const void*)k_update<BS>,         (const void*)k_check<NPL, BS>,
                     (const void*)k_check_decide<BS>,   (const void*)k_report<NPL, BS>,
                     (const void*)k_report_sum<BS>};
}

// Tile shapes: NPL nonzeros per lane, BS threads; LDS for products is
// BS * NPL * 8 bytes, kept within 64 KiB.
static bool kernels(int npl, int bs, CgKernels& k)
{
    if (npl == 4 && bs == 256) { k = kernels_for<4, 256>(); return true; }
    if (npl == 8 && bs == 256) { k = kernels_for<8, 256>(); return true; }
    if (npl == 16 && bs == 256) { k = kernels_for<16, 256>(); return true; }
    if (npl == 4 && bs == 512) { k = kernels_for<4, 512>(); return true; }
    if (npl == 8 && bs == 512) { k = kernels_for<8, 512>(); return true; }
    if (npl == 16 && bs == 512) { k = kernels_for<16, 512>(); return true; }
    if (npl == 4 && bs == 1024) { k = kernels_for<4, 1024>(); return true; }
    if (npl == 8 && bs == 1024) { k = kernels_for<8, 1024>(); return true; }
    return false;
}

static bool valid_npl(int l) { return l == 4 || l == 8 || l == 16; }
static bool valid_bs(int b) { return b == 256 || b == 512 || b == 1024; }

static void launch(const void* fn, int grid, int bs, hipStream_t st, void** args)
{
    JPCG_HIP(hipLaunchKernel(fn, dim3(grid), dim3(bs), args, 0, st));
}

void partition_rows(const std::vector<int>& rowptr, int G, std::vector<int>& out)
{
    const int n = (int)rowptr.size() - 1;
    const int64_t nnz = rowptr[n];
    out.assign(G + 1, 0);
    for (int L = 1; L < G; ++L) {
        // Balance rows plus nonzeros so empty rows still spread out.
        const int64_t target = (int64_t)((double)L * (double)(nnz + n) / (double)G);
        int lo = out[L - 1], hi = n;
        while (lo < hi) {
            const int mid = lo + (hi - lo) / 2;
            if ((int64_t)rowptr[mid] + mid < target) lo = mid + 1; else hi = mid;
        }
        out[L] = lo;
    }
    out[G] = n;
}

int set_error(cg_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

// Per-grid device buffers: partials and tiles.
struct GridBufs {
    int G = 0;
    int T = 0;
    int4* tiles = nullptr;   // [T]
    double* part = nullptr;  // setup 3G + sig G + iter 2*2G + rep G = 9G
};

}  // namespace jpcg

// The graph-chunked solver state that hangs off a context.
struct cg_graphs {
    jpcg::CgKernels kern{};
    int npl = 0, bs = 0, G = 0, chunk = 0;
    jpcg::GridBufs gb;
    jpcg::CgState* st = nullptr;
    jpcg::CgState* hst = nullptr;  // pinned, 4 slots
    double* cb = nullptr;          // context-owned b and x: graphs bind fixed addresses
    double* cx = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t evs[4] = {nullptr, nullptr, nullptr, nullptr};
    jpcg::CgArgs args{};
};

namespace jpcg {

static void destroy_graphs(cg_graphs* g)
{
    if (!g) return;
    for (auto& e : g->exec)
        if (e) (void)hipGraphExecDestroy(e);
    for (auto& e : g->evs)
        if (e) (void)hipEventDestroy(e);
    void* ptrs[] = {g->gb.tiles, g->gb.part, g->st, g->cb, g->cx};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (g->hst) (void)hipHostFree(g->hst);
    delete g;
}

// Build the kernels' arguments and capture the two chunk graphs (first A of
// parity 0 or 1) for one launch shape.
static cg_graphs* make_graphs(cg_ctx* c, int npl, int bs, int G, int chunk)
{
    cg_graphs* g = new cg_graphs();
    try {
        if (!kernels(npl, bs, g->kern)) throw HipError{hipErrorInvalidValue, "launch shape"};
        g->npl = npl;
        g->bs = bs;
        g->G = G;
        g->chunk = chunk;
        std::vector<int4> tiles;
        build_tiles(c->h_rowptr, kWave * npl, tiles);
        const int T = (int)tiles.size();
        g->gb.G = G;
        g->gb.T = T;
        JPCG_HIP(hipMalloc(&g->gb.tiles, sizeof(int4) * std::max(T, 1)));
        JPCG_HIP(hipMalloc(&g->gb.part, sizeof(double) * 9 * (size_t)G));
        JPCG_HIP(hipMalloc(&g->st, sizeof(CgState)));
        JPCG_HIP(hipHostMalloc(&g->hst, sizeof(CgState) * 4, hipHostMallocDefault));
        JPCG_HIP(hipMalloc(&g->cb, sizeof(double) * c->n));
        JPCG_HIP(hipMalloc(&g->cx, sizeof(double) * c->n));
        for (auto& e : g->evs) JPCG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        if (T) JPCG_HIP(hipMemcpyAsync(g->gb.tiles, tiles.data(), sizeof(int4) * T, hipMemcpyHostToDevice, c->stream));
        JPCG_HIP(hipMemsetAsync(g->st, 0, sizeof(CgState), c->stream));
        CgArgs& a = g->args;
        a.s = SysView<double>{c->n, c->rowptr, c->col, c->val, c->dinv, g->cb, g->cx, c->r, c->z, c->p0, c->p1, c->q};
        a.tm = TileMap{g->gb.tiles, T, (T + G - 1) / G};
        a.R = (c->n + G - 1) / G;
        a.G = G;
        a.part_setup = g->gb.part;
        a.part_sig = g->gb.part + 3 * (size_t)G;
        a.part_iter[0] = g->gb.part + 4 * (size_t)G;
        a.part_iter[1] = g->gb.part + 6 * (size_t)G;
        a.part_rep = g->gb.part + 8 * (size_t)G;
        a.st = g->st;
        a.hist = nullptr;
        JPCG_HIP(hipStreamSynchronize(c->stream));
        hipStream_t cap;
        JPCG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        for (int par = 0; par < 2; ++par) {
            hipGraph_t graph;
            JPCG_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            for (int it = 0; it < chunk; ++it) {
                int P = (par + it) & 1;
                void* args[] = {&a, &P};
                launch(g->kern.direction, G, bs, cap, args);
                launch(g->kern.update, G, bs, cap, args);
            }
            JPCG_HIP(hipStreamEndCapture(cap, &graph));
            hipError_t e = hipGraphInstantiate(&g->exec[par], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            JPCG_HIP(e);
        }
        JPCG_HIP(hipStreamDestroy(cap));
        return g;
    } catch (...) {
        destroy_graphs(g);
        throw;
    }
}

static void launch_spmv(cg_ctx* c, const double* x, double* y)
{
    cg_graphs* g = c->graphs;
    void* args[] = {&g->args, &x, &y};
    launch(g->kern.spmv, g->G, g->bs, c->stream, args);
}

// One solve through the graph path.  b, x are caller device pointers.
static void run_solve(cg_ctx* c, cg_graphs* g, const double* b, double* x, double tol, int maxit, double* hist,
                      CgState& out)
{
    hipStream_t s = c->stream;
    const size_t vb = sizeof(double) * c->n;
    JPCG_HIP(hipMemcpyAsync(g->cb, b, vb, hipMemcpyDeviceToDevice, s));
    JPCG_HIP(hipMemcpyAsync(g->cx, x, vb, hipMemcpyDeviceToDevice, s));
    CgArgs a = g->args;
    a.hist = hist;
    // The chunk graphs were captured without the history pointer; a solve that
    // records history launches the same kernels one by one instead.
    const bool use_graph = hist == nullptr;
    {
        void* args0[] = {&a};
        launch(g->kern.setup, g->G, g->bs, s, args0);
        void* args1[] = {&a, &tol, &maxit};
        launch(g->kern.first, g->G, g->bs, s, args1);
        int P = 1;
        void* args2[] = {&a, &P};
        launch(g->kern.update, g->G, g->bs, s, args2);
    }
    int next_k = 2;  // index of the next A to launch
    int slot = 0, pending = 0;
    const long long guard = (long long)maxit + 8LL * g->chunk + 64;
    long long launched = 1;
    auto launch_chunk = [&](int k0) {
        if (use_graph) {
            JPCG_HIP(hipGraphLaunch(g->exec[k0 & 1], s));
        } else {
            for (int it = 0; it < g->chunk; ++it) {
                int P = (k0 + it) & 1;
                void* args[] = {&a, &P};
                launch(g->kern.direction, g->G, g->bs, s, args);
                launch(g->kern.update, g->G, g->bs, s, args);
            }
        }
        JPCG_HIP(hipMemcpyAsync(&g->hst[slot], g->st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        JPCG_HIP(hipEventRecord(g->evs[slot], s));
    };
    while (true) {
        // Keep two chunks in flight; inspect the older one's state.
        launch_chunk(next_k);
        next_k += g->chunk;
        launched += g->chunk;
        slot = (slot + 1) & 3;
        ++pending;
        if (pending < 2) continue;
        const int old = (slot + 2) & 3;  // the chunk launched before the newest
        JPCG_HIP(hipEventSynchronize(g->evs[old]));
        --pending;
        const CgState& hs = g->hst[old];
        if (hs.stop == RUNNING) {
            if (launched > guard) throw HipError{hipErrorUnknown, "solver did not stop"};
            continue;
        }
        // Drain, then read the settled state.
        JPCG_HIP(hipMemcpyAsync(&g->hst[slot], g->st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        JPCG_HIP(hipStreamSynchronize(s));
        pending = 0;
        CgState st = g->hst[slot];
        if (st.stop == STOP_CHECK) {
            int P = st.k & 1;
            void* args[] = {&a, &P};
            launch(g->kern.check, g->G, g->bs, s, args);
            launch(g->kern.check_decide, 1, g->bs, s, args);
            JPCG_HIP(hipMemcpyAsync(&g->hst[slot], g->st, sizeof(CgState), hipMemcpyDeviceToHost, s));
            JPCG_HIP(hipStreamSynchronize(s));
            st = g->hst[slot];
            if (st.stop == RUNNING) {  // replaced residual: resume at A_{k+1}
                next_k = st.k + 1;
                continue;
            }
        }
        if (st.stop == STOP_MAXIT || st.stop == STOP_BREAKDOWN) {
            void* args[] = {&a};
            launch(g->kern.report, g->G, g->bs, s, args);
            launch(g->kern.report_sum, 1, g->bs, s, args);
        }
        break;
    }
    JPCG_HIP(hipMemcpyAsync(x, g->cx, vb, hipMemcpyDeviceToDevice, s));
    JPCG_HIP(hipMemcpyAsync(&g->hst[0], g->st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    JPCG_HIP(hipStreamSynchronize(s));
    out = g->hst[0];
}

static int status_of(const CgState& st)
{
    switch (st.stop) {
        case STOP_ZERO_RHS:
        case STOP_CONV0:
        case STOP_CONVERGED: return CG_CONVERGED;
        case STOP_MAXIT: return CG_MAXIT;
        case STOP_BREAKDOWN: return CG_BREAKDOWN;
        default: return CG_EHIP;
    }
}

static int default_grid(cg_ctx* c, int npl, int bs, int blocks_per_cu)
{
    int G = c->cus * std::max(1, blocks_per_cu);
    // At least about one tile per wave.
    const int64_t tiles = (c->nnz + (int64_t)kWave * npl - 1) / ((int64_t)kWave * npl) + 1;
    const int64_t need = (tiles + bs / kWave - 1) / (bs / kWave);
    G = (int)std::min<int64_t>(G, std::max<int64_t>(8, (need + 7) / 8 * 8));
    return std::max(8, G / 8 * 8);
}

// Time short solves over tile shapes (nonzeros per lane, block size,
// workgroups per CU) and keep the fastest; record its standalone product time.
static void autotune(cg_ctx* c)
{
    double *xb = nullptr, *yb = nullptr;
    JPCG_HIP(hipMalloc(&xb, sizeof(double) * c->n));
    JPCG_HIP(hipMalloc(&yb, sizeof(double) * c->n));
    std::vector<double> ones(c->n, 1.0);
    JPCG_HIP(hipMemcpyAsync(yb, ones.data(), sizeof(double) * c->n, hipMemcpyHostToDevice, c->stream));
    JPCG_HIP(hipMemsetAsync(xb, 0, sizeof(double) * c->n, c->stream));
    hipEvent_t e0, e1;
    JPCG_HIP(hipEventCreate(&e0));
    JPCG_HIP(hipEventCreate(&e1));
    float ms = 0.f, best = 1e30f;
    const int iters = std::max(16, std::min(64, c->n));
    cg_graphs* keep = nullptr;
    const int shapes[][2] = {{4, 256}, {8, 256}, {16, 256}, {4, 512}, {8, 512}, {16, 512}, {4, 1024}, {8, 1024}};
    for (const auto& sh : shapes) {
        for (int bpc : {1, 2, 4}) {
            const int G = default_grid(c, sh[0], sh[1], bpc);
            cg_graphs* g = nullptr;
            try {
                g = make_graphs(c, sh[0], sh[1], G, c->chunk);
                CgState st;
                JPCG_HIP(hipMemsetAsync(xb, 0, sizeof(double) * c->n, c->stream));
                run_solve(c, g, yb, xb, 0.0, 4, nullptr, st);  // warm
                JPCG_HIP(hipEventRecord(e0, c->stream));
                run_solve(c, g, yb, xb, 0.0, iters, nullptr, st);
                JPCG_HIP(hipEventRecord(e1, c->stream));
                JPCG_HIP(hipEventSynchronize(e1));
                JPCG_HIP(hipEventElapsedTime(&ms, e0, e1));
            } catch (const HipError&) {
                // A shape this device cannot launch (e.g. its LDS need): skip it.
                (void)hipGetLastError();
                destroy_graphs(g);
                continue;
            }
            if (ms < best) {
                best = ms;
                destroy_graphs(keep);
                keep = g;
            } else {
                destroy_graphs(g);
            }
            if (c->n < 4096) break;  // small systems: the shape hardly matters
        }
    }
    if (!keep) throw HipError{hipErrorInvalidConfiguration, "no launch shape could run"};
    c->tuned_iter_us = best * 1e3 / iters;
    destroy_graphs(c->graphs);
    c->graphs = keep;
    c->npl = keep->npl;
    c->bs = keep->bs;
    c->grid = keep->G;
    // Standalone product with the chosen shape.
    const int reps = 20;
    launch_spmv(c, yb, xb);
    JPCG_HIP(hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps; ++r) launch_spmv(c, yb, xb);
    JPCG_HIP(hipEventRecord(e1, c->stream));
    JPCG_HIP(hipEventSynchronize(e1));
    JPCG_HIP(hipEventElapsedTime(&ms, e0, e1));
    c->tuned_spmv_us = ms * 1e3 / reps;
    JPCG_HIP(hipEventDestroy(e0));
    JPCG_HIP(hipEventDestroy(e1));
    JPCG_HIP(hipFree(xb));
    JPCG_HIP(hipFree(yb));
}

static void free_ctx(cg_ctx* c)
{
    if (!c) return;
    destroy_graphs(c->graphs);
    void* ptrs[] = {c->rowptr, c->col, c->val, c->dinv, c->val32, c->dinv32, c->r, c->z, c->p0, c->p1, c->q, c->hist};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}

}  // namespace jpcg

using namespace jpcg;

extern "C" {

void cg_opts_default(cg_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precond = CG_PRECOND_JACOBI;
}

const char* cg_strerror(int code)
{
    switch (code) {
        case CG_CONVERGED: return "converged";
        case CG_MAXIT: return "iteration limit reached";
        case CG_BREAKDOWN: return "breakdown: matrix or preconditioner not SPD, or non-finite input";
        case CG_EINVAL: return "invalid argument";
        case CG_EDIAG: return "diagonal entry missing or not positive";
        case CG_ENOMEM: return "out of memory";
        case CG_EHIP: return "HIP runtime error";
        case CG_ETIMEOUT: return "device wait timed out";
        case CG_EUNSUPPORTED: return "unsupported option";
        default: return "unknown status";
    }
}

const char* cg_last_error(const cg_ctx* c) { return c ? c->err.c_str() : ""; }

int cg_create(const cg_csr* A, const cg_opts* opts, void* hip_stream, cg_ctx** out)
{
    if (!out) return CG_EINVAL;
    *out = nullptr;
    if (!A || A->n <= 0 || A->nnz < 0 || A->nnz > 0x7fffffffLL || !A->rowptr || (A->nnz > 0 && (!A->col || !A->val)) ||
        (A->mem != CG_MEM_HOST && A->mem != CG_MEM_DEVICE))
        return CG_EINVAL;
    cg_ctx* c = nullptr;
    try {
        c = new cg_ctx();
        if (opts) c->opts = *opts; else cg_opts_default(&c->opts);
        if (c->opts.precond == CG_PRECOND_DEFAULT) c->opts.precond = CG_PRECOND_JACOBI;
        if ((c->opts.precond != CG_PRECOND_JACOBI && c->opts.precond != CG_PRECOND_NONE) ||
            (c->opts.nnz_per_lane && !valid_npl(c->opts.nnz_per_lane)) ||
            (c->opts.block_size && !valid_bs(c->opts.block_size)) || c->opts.chunk < 0 || c->opts.blocks_per_cu < 0) {
            free_ctx(c);
            return CG_EINVAL;
        }
        c->stream = (hipStream_t)hip_stream;
        c->n = A->n;
        c->nnz = A->nnz;
        JPCG_HIP(hipGetDevice(&c->device));
        JPCG_HIP(hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device));
        int wall_khz = 0;
        JPCG_HIP(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, c->device));
        c->limit_ticks = (long long)std::max(wall_khz, 1000) * 1000LL * 4;  // 4 s of device wall clock

        // Host copy for validation and row partitioning.
        const int n = A->n;
        const int64_t nnz = A->nnz;
        c->h_rowptr.resize(n + 1);
        std::vector<int> hcol(nnz);
        std::vector<double> hval(nnz);
        if (A->mem == CG_MEM_HOST) {
            std::memcpy(c->h_rowptr.data(), A->rowptr, sizeof(int) * (n + 1));
            if (nnz) std::memcpy(hcol.data(), A->col, sizeof(int) * nnz);
            if (nnz) std::memcpy(hval.data(), A->val, sizeof(double) * nnz);
        } else {
            JPCG_HIP(hipMemcpy(c->h_rowptr.data(), A->rowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
            if (nnz) JPCG_HIP(hipMemcpy(hcol.data(), A->col, sizeof(int) * nnz, hipMemcpyDeviceToHost));
            if (nnz) JPCG_HIP(hipMemcpy(hval.data(), A->val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
        }
        const std::vector<int>& rp = c->h_rowptr;
        bool ok = rp[0] == 0 && rp[n] == nnz;
        for (int i = 0; ok && i < n; ++i) ok = rp[i + 1] >= rp[i];
        for (int64_t k = 0; ok && k < nnz; ++k) ok = hcol[k] >= 0 && hcol[k] < n;
        if (!ok) {
            free_ctx(c);
            return CG_EINVAL;
        }

        JPCG_HIP(hipMalloc(&c->rowptr, sizeof(int) * (n + 1)));
        JPCG_HIP(hipMalloc(&c->col, sizeof(int) * std::max<int64_t>(nnz, 1)));
        JPCG_HIP(hipMalloc(&c->val, sizeof(double) * std::max<int64_t>(nnz, 1)));
        JPCG_HIP(hipMalloc(&c->dinv, sizeof(double) * n));
        for (double** v : {&c->r, &c->z, &c->p0, &c->p1, &c->q}) JPCG_HIP(hipMalloc(v, sizeof(double) * n));
        JPCG_HIP(hipEventCreate(&c->ev0));
        JPCG_HIP(hipEventCreate(&c->ev1));
        JPCG_HIP(hipMemcpyAsync(c->rowptr, rp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, c->stream));
        if (nnz) {
            JPCG_HIP(hipMemcpyAsync(c->col, hcol.data(), sizeof(int) * nnz, hipMemcpyHostToDevice, c->stream));
            JPCG_HIP(hipMemcpyAsync(c->val, hval.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, c->stream));
        }
        if (c->opts.fp32_copy) {
            JPCG_HIP(hipMalloc(&c->val32, sizeof(float) * std::max<int64_t>(nnz, 1)));
            JPCG_HIP(hipMalloc(&c->dinv32, sizeof(float) * n));
            if (nnz) cast_f32_kernel<<<1024, 256, 0, c->stream>>>(nnz, c->val, c->val32);
            JPCG_HIP(hipGetLastError());
        }
        int* bad = nullptr;
        JPCG_HIP(hipMalloc(&bad, sizeof(int)));
        JPCG_HIP(hipMemsetAsync(bad, 0, sizeof(int), c->stream));
        jacobi_kernel<<<(n + 255) / 256, 256, 0, c->stream>>>(n, c->rowptr, c->col, c->val,
                                                              c->opts.precond == CG_PRECOND_JACOBI, c->dinv,
                                                              c->dinv32, bad);
        JPCG_HIP(hipGetLastError());
        int hbad = 0;
        JPCG_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        JPCG_HIP(hipStreamSynchronize(c->stream));
        JPCG_HIP(hipFree(bad));
        if (hbad) {
            free_ctx(c);
            return CG_EDIAG;
        }

        // Launch shape: defaults, explicit options, or the autotuner.
        c->chunk = c->opts.chunk ? c->opts.chunk : 16;
        c->npl = c->opts.nnz_per_lane ? c->opts.nnz_per_lane : 8;
        c->bs = c->opts.block_size ? c->opts.block_size : 512;
        if (c->npl == 16 && c->bs == 1024) c->bs = 512;  // product tiles must fit 64 KiB of LDS
        c->grid = default_grid(c, c->npl, c->bs, c->opts.blocks_per_cu ? c->opts.blocks_per_cu : 1);
        if (c->opts.autotune) {
            autotune(c);
        } else {
            c->graphs = make_graphs(c, c->npl, c->bs, c->grid, c->chunk);
        }
        *out = c;
        return 0;
    } catch (const HipError& e) {
        free_ctx(c);
        return e.code == hipErrorOutOfMemory ? CG_ENOMEM : CG_EHIP;
    } catch (const std::bad_alloc&) {
        free_ctx(c);
        return CG_ENOMEM;
    }
}

void cg_destroy(cg_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
}

int cg_solve(cg_ctx* c, const double* b, double* x, double tol, int32_t maxit, cg_info* info)
{
    if (!c) return CG_EINVAL;
    if (!b || !x || b == x || !(tol >= 0.0) || !std::isfinite(tol))
        return set_error(c, CG_EINVAL, "cg_solve: b and x must be distinct device pointers and tol finite >= 0");
    if (maxit <= 0) maxit = c->n;
    try {
        double* hist = nullptr;
        if (c->opts.history) {
            if (c->hist_cap < maxit + 1) {
                if (c->hist) JPCG_HIP(hipFree(c->hist));
                c->hist = nullptr;
                JPCG_HIP(hipMalloc(&c->hist, sizeof(double) * ((size_t)maxit + 1)));
                c->hist_cap = maxit + 1;
            }
            hist = c->hist;
        }
        CgState st;
        JPCG_HIP(hipEventRecord(c->ev0, c->stream));
        run_solve(c, c->graphs, b, x, tol, maxit, hist, st);
        JPCG_HIP(hipEventRecord(c->ev1, c->stream));
        JPCG_HIP(hipEventSynchronize(c->ev1));
        float ms = 0.f;
        JPCG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        const int status = status_of(st);
        c->hist_len = hist ? st.k + 1 : 0;
        if (info) {
            info->iters = st.k;
            info->status = status;
            info->replacements = st.replacements;
            info->outer = 0;
            info->relres_recur = st.nb > 0 ? std::sqrt(st.rr) / st.nb : 0.0;
            info->relres_true = st.nb > 0 ? std::sqrt(st.rr_true) / st.nb : 0.0;
            info->seconds = ms * 1e-3;
        }
        return status;
    } catch (const HipError& e) {
        return set_error(c, CG_EHIP, std::string("cg_solve: ") + e.what + ": " + hipGetErrorString(e.code));
    }
}

int spmv(cg_ctx* c, const double* x, double* y)
{
    if (!c) return CG_EINVAL;
    if (!x || !y || x == y) return set_error(c, CG_EINVAL, "spmv: x and y must be distinct device pointers");
    try {
        launch_spmv(c, x, y);
        return 0;
    } catch (const HipError& e) {
        return set_error(c, CG_EHIP, std::string("spmv: ") + e.what + ": " + hipGetErrorString(e.code));
    }
}

int cg_get_history(cg_ctx* c, double* host_out, int32_t cap)
{
    if (!c || !host_out || cap < 0) return CG_EINVAL;
    if (!c->opts.history) return set_error(c, CG_EUNSUPPORTED, "history was not enabled at create");
    const int m = std::min(cap, c->hist_len);
    try {
        if (m > 0) JPCG_HIP(hipMemcpy(host_out, c->hist, sizeof(double) * m, hipMemcpyDeviceToHost));
    } catch (const HipError& e) {
        return set_error(c, CG_EHIP, e.what);
    }
    return m;
}

int cg_get_config(cg_ctx* c, cg_config* cfg)
{
    if (!c || !cfg) return CG_EINVAL;
    cfg->nnz_per_lane = c->npl;
    cfg->block_size = c->bs;
    cfg->grid = c->grid;
    cfg->tiles = c->graphs ? c->graphs->gb.T : 0;
    cfg->chunk = c->chunk;
    cfg->spmv_us = c->tuned_spmv_us;
    cfg->iter_us = c->tuned_iter_us;
    return 0;
}

}  // extern "C"
