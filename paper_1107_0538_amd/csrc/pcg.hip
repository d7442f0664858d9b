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
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstring>
#include <new>

#include "context.hpp"
#include "sr_kernels.hpp"
#include "std_kernels.hpp"
#include "tiles.hpp"

namespace jpcg {

// Per-workgroup partial sums of a solver context, in doubles per workgroup:
// standard form 9 (setup 3, p'q 1, two parities of 2, report 1), single-
// reduction form 2 * kSrPart + 3 (two parities, setup 2, check 1).
constexpr int kPartPerWg = 16;
static_assert(2 * kSrPart + 3 <= kPartPerWg && 9 <= kPartPerWg, "partials layout");

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

// s_i = sum_j a_ij in FP64, stored in FP32, for the row-sum-preserving FP32 product.
__global__ void rowsum_kernel(int n, const int* __restrict__ rowptr, const double* __restrict__ val,
                              float* __restrict__ rs, double* __restrict__ rs64)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k];
    rs[i] = (float)s;
    rs64[i] = s;
}

__global__ void cast_f32_kernel(int64_t n, const double* __restrict__ in, float* __restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

// ---------------------------------------------------------------------------
// Kernel tables per launch shape
// ---------------------------------------------------------------------------
// FP64 refinement step of the mixed-precision form: every workgroup reduces
// the partials of r'r and b'b of r = b - A x (FP64) and scales the residual
// into the FP32 right-hand side, b32 = r / ||r||, clearing x32.
struct MixedState {
    double rr, bb, scale;
};

template <int BS>
__global__ __launch_bounds__(BS) void k_mixed_scale(int n, const double* __restrict__ r, const double* part, int G,
                                                    float* __restrict__ b32, float* __restrict__ x32,
                                                    MixedState* ms)
{
    double g[3];
    wave_grid_sum<3>(part, G, g);  // r'r, r'z, b'b of the FP64 residual
    const double nr = sqrt(g[0]);
    const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ms->rr = g[0];
        ms->bb = g[2];
        ms->scale = nr;
    }
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) {
        b32[i] = (float)(r[i] * inv);
        x32[i] = 0.0f;
    }
}

// x64 += ||r|| * x32: the FP64 refinement update.
template <int BS>
__global__ __launch_bounds__(BS) void k_mixed_update(int n, double* __restrict__ x, const float* __restrict__ x32,
                                                     const MixedState* ms)
{
    const double sc = ms->scale;
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) x[i] = fma(sc, (double)x32[i], x[i]);
}

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
    // single-reduction form (FP64 only)
    const void* sr_setup;
    const void* sr_first;
    const void* sr_iter;
    const void* sr_residual;
    const void* sr_decide;
    const void* sr_restart;
};

// M32: the FP32-matrix form's products (FP32 values, FP64 vectors, row-sum-
// preserving) for the iteration; set-up, checks and reports keep FP64 values.
template <int NPL, int BS, typename T, bool M32 = false>
static CgKernels kernels_for()
{
    CgKernels k{};
    k.spmv = (const void*)k_spmv<NPL, BS, T>;
    k.setup = (const void*)k_setup<NPL, BS, T>;
    k.first = (const void*)k_first<NPL, BS, T, M32>;
    k.direction = (const void*)k_direction<NPL, BS, T, M32>;
    k.update = (const void*)k_update<BS, T>;
    k.check = (const void*)k_check<NPL, BS, T>;
    k.check_decide = (const void*)k_check_decide<BS, T>;
    k.report = (const void*)k_report<NPL, BS, T>;
    k.report_sum = (const void*)k_report_sum<BS, T>;
    if constexpr (sizeof(T) == 8) {
        k.sr_setup = (const void*)k_sr_setup<NPL, BS>;
        k.sr_first = (const void*)k_sr_first<NPL, BS>;
        k.sr_iter = (const void*)k_sr_iter<NPL, BS>;
        k.sr_residual = (const void*)k_sr_residual<NPL, BS>;
        k.sr_decide = (const void*)k_sr_decide<BS>;
        k.sr_restart = (const void*)k_sr_restart<NPL, BS>;
    }
    return k;
}

// Tile shapes: NPL nonzeros per lane, BS threads; LDS for products is
// BS * NPL * sizeof(T) bytes.
template <typename T, bool M32 = false>
static bool kernels_t(int npl, int bs, CgKernels& k)
{
    if (npl == 4 && bs == 256) { k = kernels_for<4, 256, T, M32>(); return true; }
    if (npl == 8 && bs == 256) { k = kernels_for<8, 256, T, M32>(); return true; }
    if (npl == 16 && bs == 256) { k = kernels_for<16, 256, T, M32>(); return true; }
    if (npl == 4 && bs == 512) { k = kernels_for<4, 512, T, M32>(); return true; }
    if (npl == 8 && bs == 512) { k = kernels_for<8, 512, T, M32>(); return true; }
    if (npl == 16 && bs == 512) { k = kernels_for<16, 512, T, M32>(); return true; }
    if (npl == 4 && bs == 1024) { k = kernels_for<4, 1024, T, M32>(); return true; }
    if (npl == 8 && bs == 1024) { k = kernels_for<8, 1024, T, M32>(); return true; }
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

// What a solve leaves behind, for either form.
struct SolveResult {
    int stop = 0;
    int iters = 0;
    int replacements = 0;
    double nb = 0.0, rr = 0.0, rr_true = 0.0;
};

}  // namespace jpcg

// The graph-chunked solver state that hangs off a context: one form, one
// precision (FP64, or the FP32 inner solver of the mixed form), one launch
// shape.
struct cg_graphs {
    jpcg::CgKernels kern{};
    int form = CG_FORM_STANDARD;
    bool fp32 = false;
    int npl = 0, bs = 0, G = 0, T = 0, chunk = 0;
    int4* tiles = nullptr;
    unsigned short* col16 = nullptr;  // narrow column indices of these tiles (null: 32-bit)
    double* part = nullptr;  // kPartPerWg * G doubles, laid out per form
    void* st = nullptr;      // CgState or SrState
    void* hst = nullptr;     // pinned, 4 slots
    size_t st_bytes = 0;
    void* cb = nullptr;      // the solver's own b and x: graphs bind fixed addresses
    void* cx = nullptr;
    void* work32 = nullptr;  // FP32 work vectors: r, two {z, p} pair arrays, q (6 strides)
    // exec[P][q]: a chunk whose first iteration has parity P, ending with the
    // copy of the state block into pinned slot q (the host reads slot q after
    // the chunk's event; four slots so that two chunks can be in flight).
    hipGraphExec_t exec[2][4] = {};
    hipEvent_t evs[4] = {nullptr, nullptr, nullptr, nullptr};
    jpcg::CgArgsT<double> args{};
    jpcg::CgArgsT<float> args32{};
    jpcg::SrArgs sargs{};
};

namespace jpcg {

static void destroy_graphs(cg_graphs* g)
{
    if (!g) return;
    for (auto& row : g->exec)
        for (auto& e : row)
            if (e) (void)hipGraphExecDestroy(e);
    for (auto& e : g->evs)
        if (e) (void)hipEventDestroy(e);
    void* ptrs[] = {g->tiles, g->col16, g->part, g->st, g->cb, g->cx, g->work32};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (g->hst) (void)hipHostFree(g->hst);
    delete g;
}

template <typename T>
static void fill_args(CgArgsT<T>& a, const SysView<T>& s, const TileMap& tm, int n, int G, double* part, void* st)
{
    a.s = s;
    a.tm = tm;
    a.R = (n + G - 1) / G;
    a.G = G;
    a.part_setup = part;
    a.part_sig = part + 3 * (size_t)G;
    a.part_iter[0] = part + 4 * (size_t)G;
    a.part_iter[1] = part + 6 * (size_t)G;
    a.part_rep = part + 8 * (size_t)G;
    a.st = (CgState*)st;
    a.hist = nullptr;
    a.rowsum = nullptr;
    a.val32 = nullptr;
    a.drop2 = 0.0;
}

// Build the kernels' arguments and capture the two chunk graphs (first
// iteration of parity 0 or 1) for one form, precision and launch shape.
// mat32: the FP32-matrix form (FP64 standard form whose iteration products
// stream the FP32 values), confirming on the FP64 true residual each time the
// recurrence residual has fallen by `drop` since the last replacement.
static cg_graphs* make_graphs(cg_ctx* c, int form, bool fp32, int npl, int bs, int G, int chunk, bool mat32 = false,
                              double drop = 0.0)
{
    cg_graphs* g = new cg_graphs();
    try {
        const bool ok = fp32 ? kernels_t<float>(npl, bs, g->kern)
                        : mat32 ? kernels_t<double, true>(npl, bs, g->kern)
                                : kernels_t<double>(npl, bs, g->kern);
        if (!ok || ((fp32 || mat32) && form != CG_FORM_STANDARD)) throw HipError{hipErrorInvalidValue, "launch shape"};
        g->form = form;
        g->fp32 = fp32;
        g->npl = npl;
        g->bs = bs;
        g->G = G;
        g->chunk = chunk;
        std::vector<int4> tiles;
        build_tiles(c->h_rowptr, kWave * npl, tiles);
        const int T = (int)tiles.size();
        g->T = T;
        g->st_bytes = std::max(sizeof(CgState), sizeof(SrState));
        const size_t eb = fp32 ? sizeof(float) : sizeof(double);
        JPCG_HIP(hipMalloc(&g->tiles, sizeof(int4) * std::max(T, 1)));
        JPCG_HIP(hipMalloc(&g->part, sizeof(double) * kPartPerWg * (size_t)G));
        JPCG_HIP(hipMalloc(&g->st, g->st_bytes));
        JPCG_HIP(hipHostMalloc(&g->hst, g->st_bytes * 4, hipHostMallocDefault));
        JPCG_HIP(hipMalloc(&g->cb, eb * c->n));
        JPCG_HIP(hipMalloc(&g->cx, eb * c->n));
        for (auto& e : g->evs) JPCG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        if (T) JPCG_HIP(hipMemcpyAsync(g->tiles, tiles.data(), sizeof(int4) * T, hipMemcpyHostToDevice, c->stream));
        JPCG_HIP(hipMemsetAsync(g->st, 0, g->st_bytes, c->stream));
        if (c->opts.col_bits != 32) g->col16 = make_col16(c->stream, g->tiles, T, c->col, c->nnz);
        const TileMap tm{g->tiles, T, (T + G - 1) / G, g->col16};
        if (fp32) {
            const size_t n = c->work_stride;
            JPCG_HIP(hipMalloc(&g->work32, sizeof(float) * 6 * n));
            JPCG_HIP(hipMemsetAsync(g->work32, 0, sizeof(float) * 6 * n, c->stream));
            float* w = (float*)g->work32;
            fill_args(g->args32,
                      SysView<float>{c->n, c->rowptr, c->col, c->val32, c->dinv32, (float*)g->cb, (float*)g->cx, w,
                                     {(ZPair<float>*)(w + n), (ZPair<float>*)(w + 3 * n)}, w + 5 * n},
                      tm, c->n, G, g->part, g->st);
            g->args32.rowsum = c->rowsum32;
        } else {
            double* const* w = c->work;
            fill_args(g->args,
                      SysView<double>{c->n, c->rowptr, c->col, c->val, c->dinv, (double*)g->cb, (double*)g->cx, w[0],
                                      {(ZPair<double>*)w[1], (ZPair<double>*)w[3]},  // spanning w[1..2], w[3..4]
                                      w[5]},
                      tm, c->n, G, g->part, g->st);
            if (mat32) {
                g->args.rowsum = c->rowsum64;
                g->args.val32 = c->val32;
                g->args.drop2 = drop * drop;
            }
            SrArgs& sa = g->sargs;
            sa.n = c->n;
            sa.rowptr = c->rowptr;
            sa.col = c->col;
            sa.val = c->val;
            sa.dinv = c->dinv;
            sa.b = (double*)g->cb;
            sa.x = (double*)g->cx;
            sa.qd[0] = (SrQuad*)w[0];  // spans w[0..3]
            sa.qd[1] = (SrQuad*)w[4];  // spans w[4..7]
            sa.p = w[8];
            sa.tm = tm;
            sa.G = G;
            sa.part[0] = g->part;
            sa.part[1] = g->part + kSrPart * (size_t)G;
            sa.part_setup = g->part + 2 * kSrPart * (size_t)G;
            sa.part_chk = g->part + (2 * kSrPart + 2) * (size_t)G;
            sa.st = (SrState*)g->st;
            sa.hist = nullptr;
        }
        JPCG_HIP(hipStreamSynchronize(c->stream));
        hipStream_t cap;
        JPCG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        for (int pq = 0; pq < 8; ++pq) {
            const int par = pq >> 2, q = pq & 3;
            hipGraph_t graph;
            JPCG_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            for (int it = 0; it < chunk; ++it) {
                int P = (par + it) & 1;
                if (form == CG_FORM_SINGLE_REDUCTION) {
                    void* args[] = {&g->sargs, &P};
                    launch(g->kern.sr_iter, G, bs, cap, args);
                } else {
                    void* args[] = {fp32 ? (void*)&g->args32 : (void*)&g->args, &P};
                    launch(g->kern.direction, G, bs, cap, args);
                    launch(g->kern.update, G, bs, cap, args);
                }
            }
            JPCG_HIP(hipMemcpyAsync((char*)g->hst + q * g->st_bytes, g->st, g->st_bytes, hipMemcpyDeviceToHost, cap));
            JPCG_HIP(hipStreamEndCapture(cap, &graph));
            hipError_t e = hipGraphInstantiate(&g->exec[par][q], graph, nullptr, nullptr, 0);
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

}  // namespace jpcg

// The standalone product (spmv) has its own tiling and grid: it carries no
// partial sums, so its grid is not tied to the solver's, and the product
// alone runs best with more, smaller tiles in flight (tile width 8, two
// workgroups of 512 per CU at 51^3) than the solver kernels, whose reduction
// of the previous kernel's partials grows with the grid.
struct cg_spmv_plan {
    int npl = 0, bs = 0, G = 0, T = 0;
    int4* tiles = nullptr;
    unsigned short* col16 = nullptr;
    const void* kern = nullptr;
    jpcg::CgArgsT<double> args{};
};

namespace jpcg {

static void destroy_spmv_plan(cg_spmv_plan* p)
{
    if (!p) return;
    if (p->tiles) (void)hipFree(p->tiles);
    if (p->col16) (void)hipFree(p->col16);
    delete p;
}

static cg_spmv_plan* make_spmv_plan(cg_ctx* c, int npl, int bs, int G)
{
    cg_spmv_plan* p = new cg_spmv_plan();
    try {
        CgKernels k{};
        if (!kernels_t<double>(npl, bs, k)) throw HipError{hipErrorInvalidValue, "launch shape"};
        p->npl = npl;
        p->bs = bs;
        p->G = G;
        p->kern = k.spmv;
        std::vector<int4> tiles;
        build_tiles(c->h_rowptr, kWave * npl, tiles);
        p->T = (int)tiles.size();
        JPCG_HIP(hipMalloc(&p->tiles, sizeof(int4) * std::max(p->T, 1)));
        if (p->T)
            JPCG_HIP(hipMemcpyAsync(p->tiles, tiles.data(), sizeof(int4) * p->T, hipMemcpyHostToDevice, c->stream));
        if (c->opts.col_bits != 32) p->col16 = make_col16(c->stream, p->tiles, p->T, c->col, c->nnz);
        JPCG_HIP(hipStreamSynchronize(c->stream));
        CgArgsT<double>& a = p->args;
        a.s = SysView<double>{c->n, c->rowptr, c->col, c->val, c->dinv, nullptr, nullptr, nullptr,
                              {nullptr, nullptr}, nullptr};
        a.rowsum = nullptr;
        a.tm = TileMap{p->tiles, p->T, (p->T + G - 1) / G, p->col16};
        a.R = (c->n + G - 1) / G;
        a.G = G;
        return p;
    } catch (...) {
        destroy_spmv_plan(p);
        throw;
    }
}

static void launch_spmv(cg_ctx* c, const double* x, double* y)
{
    cg_spmv_plan* p = c->spmv;
    void* args[] = {&p->args, &x, &y};
    launch(p->kern, p->G, p->bs, c->stream, args);
}

// The chunk loop shared by both forms: two chunks in flight; the state block
// of the older one is inspected while the newer runs.  `iteration` launches
// one iteration without a graph (used when history is recorded), `stopped`
// handles a raised stop flag and returns the next iteration index to resume
// at, or -1 when the solve is over.
template <typename Iter, typename Stopped>
static void chunk_loop(cg_ctx* c, cg_graphs* g, int first_k, int maxit, bool use_graph, Iter iteration,
                       Stopped stopped)
{
    hipStream_t s = c->stream;
    int next_k = first_k, slot = 0, pending = 0;
    const long long guard = (long long)maxit + 8LL * g->chunk + 64;
    long long launched = 0;
    char* hst = (char*)g->hst;
    while (true) {
        if (use_graph) {
            JPCG_HIP(hipGraphLaunch(g->exec[next_k & 1][slot], s));  // copies the state into slot
        } else {
            for (int it = 0; it < g->chunk; ++it) iteration((next_k + it) & 1);
            JPCG_HIP(hipMemcpyAsync(hst + slot * g->st_bytes, g->st, g->st_bytes, hipMemcpyDeviceToHost, s));
        }
        JPCG_HIP(hipEventRecord(g->evs[slot], s));
        next_k += g->chunk;
        launched += g->chunk;
        slot = (slot + 1) & 3;
        ++pending;
        if (pending < 2) continue;
        const int old = (slot + 2) & 3;  // the chunk launched before the newest
        JPCG_HIP(hipEventSynchronize(g->evs[old]));
        --pending;
        if (*(const int*)(hst + old * g->st_bytes) == RUNNING) {
            if (launched > guard) throw HipError{hipErrorUnknown, "solver did not stop"};
            continue;
        }
        JPCG_HIP(hipStreamSynchronize(s));  // drain the chunk still in flight
        pending = 0;
        const int resume = stopped();
        if (resume < 0) return;
        next_k = resume;
        launched = resume - first_k;  // iterations done on the device, not launched

    }
}

template <typename State>
static State read_state(cg_ctx* c, cg_graphs* g)
{
    State* h = (State*)g->hst;
    JPCG_HIP(hipMemcpyAsync(h, g->st, sizeof(State), hipMemcpyDeviceToHost, c->stream));
    JPCG_HIP(hipStreamSynchronize(c->stream));
    return *h;
}

// Standard form on the graphs' own b and x.  With confirm == false (the
// FP32 inner solve of the mixed form) a passed continue-condition ends the
// solve without the true-residual check.
template <typename T>
static SolveResult run_standard(cg_ctx* c, cg_graphs* g, CgArgsT<T> a, double tol, int maxit, double* hist,
                                bool confirm)
{
    hipStream_t s = c->stream;
    a.hist = hist;
    {
        void* args0[] = {&a};
        launch(g->kern.setup, g->G, g->bs, s, args0);
        void* args1[] = {&a, &tol, &maxit};
        launch(g->kern.first, g->G, g->bs, s, args1);
        int P = 1;
        void* args2[] = {&a, &P};
        launch(g->kern.update, g->G, g->bs, s, args2);
    }
    auto iteration = [&](int P) {
        void* args[] = {&a, &P};
        launch(g->kern.direction, g->G, g->bs, s, args);
        launch(g->kern.update, g->G, g->bs, s, args);
    };
    auto stopped = [&]() -> int {
        CgState st = read_state<CgState>(c, g);
        if (st.stop == STOP_CHECK && confirm) {
            int P = st.k & 1;
            void* args[] = {&a, &P};
            launch(g->kern.check, g->G, g->bs, s, args);
            launch(g->kern.check_decide, 1, g->bs, s, args);
            st = read_state<CgState>(c, g);
            if (st.stop == RUNNING) return st.k + 1;  // replaced residual: resume at A_{k+1}
        }
        if (confirm && (st.stop == STOP_MAXIT || st.stop == STOP_BREAKDOWN)) {
            void* args[] = {&a};
            launch(g->kern.report, g->G, g->bs, s, args);
            launch(g->kern.report_sum, 1, g->bs, s, args);
        }
        return -1;
    };
    chunk_loop(c, g, 2, maxit, hist == nullptr, iteration, stopped);
    const CgState st = read_state<CgState>(c, g);
    SolveResult r;
    r.stop = st.stop;
    r.iters = st.k;
    r.replacements = st.replacements;
    r.nb = st.nb;
    r.rr = st.rr;
    r.rr_true = st.rr_true;
    return r;
}

static SolveResult run_single(cg_ctx* c, cg_graphs* g, double tol, int maxit, double* hist)
{
    hipStream_t s = c->stream;
    SrArgs a = g->sargs;
    a.hist = hist;
    {
        void* args0[] = {&a};
        launch(g->kern.sr_setup, g->G, g->bs, s, args0);
        void* args1[] = {&a, &tol, &maxit};
        launch(g->kern.sr_first, g->G, g->bs, s, args1);
    }
    auto iteration = [&](int P) {
        void* args[] = {&a, &P};
        launch(g->kern.sr_iter, g->G, g->bs, s, args);
    };
    auto stopped = [&]() -> int {
        SrState st = read_state<SrState>(c, g);
        if (st.stop == STOP_CHECK) {
            int P = st.k_done & 1, replace = 1, report = 0;
            void* args[] = {&a, &P, &replace};
            launch(g->kern.sr_residual, g->G, g->bs, s, args);
            void* dargs[] = {&a, &report};
            launch(g->kern.sr_decide, 1, g->bs, s, dargs);
            st = read_state<SrState>(c, g);
            if (st.stop == RUNNING) {  // replaced residual: w = A M^-1 r, then resume
                void* rargs[] = {&a, &P};
                launch(g->kern.sr_restart, g->G, g->bs, s, rargs);
                return st.k_done + 1;
            }
        }
        if (st.stop == STOP_MAXIT || st.stop == STOP_BREAKDOWN) {
            int P = 0, replace = 0, report = 1;
            void* args[] = {&a, &P, &replace};
            launch(g->kern.sr_residual, g->G, g->bs, s, args);
            void* dargs[] = {&a, &report};
            launch(g->kern.sr_decide, 1, g->bs, s, dargs);
        }
        return -1;
    };
    chunk_loop(c, g, 1, maxit, hist == nullptr, iteration, stopped);
    const SrState st = read_state<SrState>(c, g);
    SolveResult r;
    r.stop = st.stop;
    r.iters = st.k_done;
    r.replacements = st.replacements;
    r.nb = st.nb;
    r.rr = st.rr;
    r.rr_true = st.rr_true;
    return r;
}

// One FP64 solve through the graph path.  b, x are caller device pointers.
static SolveResult run_solve(cg_ctx* c, cg_graphs* g, const double* b, double* x, double tol, int maxit,
                             double* hist)
{
    hipStream_t s = c->stream;
    const size_t vb = sizeof(double) * c->n;
    JPCG_HIP(hipMemcpyAsync(g->cb, b, vb, hipMemcpyDeviceToDevice, s));
    JPCG_HIP(hipMemcpyAsync(g->cx, x, vb, hipMemcpyDeviceToDevice, s));
    const SolveResult r = g->form == CG_FORM_SINGLE_REDUCTION
                              ? run_single(c, g, tol, maxit, hist)
                              : run_standard<double>(c, g, g->args, tol, maxit, hist, true);
    JPCG_HIP(hipMemcpyAsync(x, g->cx, vb, hipMemcpyDeviceToDevice, s));
    JPCG_HIP(hipStreamSynchronize(s));
    return r;
}

// Mixed precision: FP64 outer residual, scaling, refinement update and final
// test; FP32 inner Jacobi-PCG on the FP32 copy of A.
struct MixedResult {
    int status = CG_MAXIT;
    int outer = 0;
    int inner_iters = 0;
    double nb = 0.0, rr = 0.0;
};

static MixedResult run_mixed(cg_ctx* c, const double* b, double* x, double tol, int max_outer, double tol_in,
                             int maxit_in)
{
    hipStream_t s = c->stream;
    cg_graphs* g64 = c->graphs_std;
    cg_graphs* g32 = c->graphs32;
    const size_t vb = sizeof(double) * c->n;
    JPCG_HIP(hipMemcpyAsync(g64->cb, b, vb, hipMemcpyDeviceToDevice, s));
    JPCG_HIP(hipMemcpyAsync(g64->cx, x, vb, hipMemcpyDeviceToDevice, s));
    CgArgsT<double> a64 = g64->args;
    MixedResult res;
    MixedState* hms = (MixedState*)c->mixed_host;
    const int eg = std::min(4096, (c->n + 255) / 256);
    for (int outer = 0;; ++outer) {
        void* args0[] = {&a64};
        launch(g64->kern.setup, g64->G, g64->bs, s, args0);  // r = b - A x in FP64
        int n = c->n;
        void* sargs[] = {&n, &a64.s.r, &a64.part_setup, &a64.G, &g32->cb, &g32->cx, &c->mixed_dev};
        launch((const void*)k_mixed_scale<256>, eg, 256, s, sargs);
        JPCG_HIP(hipMemcpyAsync(hms, c->mixed_dev, sizeof(MixedState), hipMemcpyDeviceToHost, s));
        JPCG_HIP(hipStreamSynchronize(s));
        res.outer = outer;
        res.nb = std::sqrt(hms->bb);
        res.rr = hms->rr;
        if (!(res.rr == res.rr) || !(hms->bb == hms->bb)) {  // NaN input
            res.status = CG_BREAKDOWN;
            break;
        }
        if (res.nb == 0.0 || std::sqrt(res.rr) <= tol * res.nb) {
            res.status = CG_CONVERGED;
            if (res.nb == 0.0) JPCG_HIP(hipMemsetAsync(g64->cx, 0, vb, s));
            break;
        }
        if (outer >= max_outer) {
            res.status = CG_MAXIT;
            break;
        }
        const SolveResult in = run_standard<float>(c, g32, g32->args32, tol_in, maxit_in, nullptr, false);
        res.inner_iters += in.iters;
        void* uargs[] = {&n, &a64.s.x, &g32->cx, &c->mixed_dev};
        launch((const void*)k_mixed_update<256>, eg, 256, s, uargs);
    }
    JPCG_HIP(hipMemcpyAsync(x, g64->cx, vb, hipMemcpyDeviceToDevice, s));
    JPCG_HIP(hipStreamSynchronize(s));
    return res;
}

static int status_of(int stop)
{
    switch (stop) {
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
// Tuned shapes, kept for the life of the process and reused by later
// contexts whose matrix has the same size and row-length profile.
struct TuneKey {
    int device, n, maxrow, form, chunk;
    int64_t nnz;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(device, n, maxrow, form, chunk, nnz) < std::tie(o.device, o.n, o.maxrow, o.form, o.chunk, o.nnz);
    }
};
struct TuneResult {
    int npl, bs, G;
    double iter_us, spmv_us;
    int spmv_npl, spmv_bs, spmv_G;
};
static std::mutex g_tune_mutex;
static std::map<TuneKey, TuneResult> g_tune_cache;

static TuneKey tune_key(const cg_ctx* c)
{
    int maxrow = 0;
    for (int i = 0; i < c->n; ++i) maxrow = std::max(maxrow, c->h_rowptr[i + 1] - c->h_rowptr[i]);
    return TuneKey{c->device, c->n, maxrow, c->form, c->chunk, c->nnz};
}

static void autotune(cg_ctx* c)
{
    const TuneKey key = tune_key(c);
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            const TuneResult& r = it->second;
            cg_graphs* g = make_graphs(c, c->form, false, r.npl, r.bs, r.G, c->chunk);
            destroy_graphs(c->graphs);
            c->graphs = g;
            c->npl = r.npl;
            c->bs = r.bs;
            c->grid = r.G;
            c->tuned_iter_us = r.iter_us;
            c->tuned_spmv_us = r.spmv_us;
            c->spmv = make_spmv_plan(c, r.spmv_npl, r.spmv_bs, r.spmv_G);
            c->tune_cached = true;
            return;
        }
    }
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
                g = make_graphs(c, c->form, false, sh[0], sh[1], G, c->chunk);
                JPCG_HIP(hipMemsetAsync(xb, 0, sizeof(double) * c->n, c->stream));
                run_solve(c, g, yb, xb, 0.0, 4, nullptr);  // warm
                JPCG_HIP(hipEventRecord(e0, c->stream));
                run_solve(c, g, yb, xb, 0.0, iters, nullptr);
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
    // The standalone product's own shape: time each tiling and grid.
    const int reps = 20;
    float best_spmv = 1e30f;
    const int pshapes[][2] = {{4, 512}, {8, 256}, {8, 512}, {16, 256}, {16, 512}};
    for (const auto& sh : pshapes) {
        for (int bpc : {1, 2, 4}) {
            // The candidate is made current for timing; afterwards the better
            // of it and the best so far stays in c->spmv, the other is freed.
            cg_spmv_plan* p = nullptr;
            bool current = false;
            try {
                p = make_spmv_plan(c, sh[0], sh[1], default_grid(c, sh[0], sh[1], bpc));
                std::swap(p, c->spmv);  // p: the best so far (or none)
                current = true;
                launch_spmv(c, yb, xb);
                JPCG_HIP(hipEventRecord(e0, c->stream));
                for (int r = 0; r < reps; ++r) launch_spmv(c, yb, xb);
                JPCG_HIP(hipEventRecord(e1, c->stream));
                JPCG_HIP(hipEventSynchronize(e1));
                JPCG_HIP(hipEventElapsedTime(&ms, e0, e1));
            } catch (const HipError&) {
                (void)hipGetLastError();  // a shape this device cannot launch
                ms = 1e30f;
            }
            if (!current) continue;  // the candidate was never made
            if (ms < best_spmv) {
                best_spmv = ms;
                destroy_spmv_plan(p);
            } else {
                std::swap(p, c->spmv);
                destroy_spmv_plan(p);
            }
            if (c->n < 4096) break;
        }
    }
    if (!c->spmv) throw HipError{hipErrorInvalidConfiguration, "no product shape could run"};
    c->tuned_spmv_us = best_spmv * 1e3 / reps;
    JPCG_HIP(hipEventDestroy(e0));
    JPCG_HIP(hipEventDestroy(e1));
    JPCG_HIP(hipFree(xb));
    JPCG_HIP(hipFree(yb));
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[key] = TuneResult{c->npl,          c->bs,          c->grid,     c->tuned_iter_us, c->tuned_spmv_us,
                                   c->spmv->npl, c->spmv->bs, c->spmv->G};
}

static void free_ctx(cg_ctx* c)
{
    if (!c) return;
    if (c->graphs_std != c->graphs) destroy_graphs(c->graphs_std);
    destroy_graphs(c->graphs);
    destroy_graphs(c->graphs32);
    destroy_graphs(c->graphs_m32);
    destroy_spmv_plan(c->spmv);
    free_multi(c);
    free_block(c);
    if (c->mixed_dev) (void)hipFree(c->mixed_dev);
    if (c->mixed_host) (void)hipHostFree(c->mixed_host);
    void* ptrs[] = {c->rowptr, c->col, c->val, c->dinv, c->val32, c->dinv32, c->rowsum32, c->rowsum64, c->work[0],
                    c->hist};
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
        case CG_ESCRATCH: return "request exceeds the fixed scratch buffer of a no-allocation call";
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
            (c->opts.block_size && !valid_bs(c->opts.block_size)) || c->opts.chunk < 0 || c->opts.blocks_per_cu < 0 ||
            (c->opts.form != CG_FORM_STANDARD && c->opts.form != CG_FORM_SINGLE_REDUCTION) ||
            (c->opts.col_bits != 0 && c->opts.col_bits != 32)) {
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
        // kCsrPad zero entries after the last nonzero: batched loads of a
        // row's entries may run past its end (the extra slots are ignored).
        JPCG_HIP(hipMalloc(&c->col, sizeof(int) * (nnz + kCsrPad)));
        JPCG_HIP(hipMalloc(&c->val, sizeof(double) * (nnz + kCsrPad)));
        JPCG_HIP(hipMemsetAsync(c->col + nnz, 0, sizeof(int) * kCsrPad, c->stream));
        JPCG_HIP(hipMemsetAsync(c->val + nnz, 0, sizeof(double) * kCsrPad, c->stream));
        JPCG_HIP(hipMalloc(&c->dinv, sizeof(double) * n));
        c->work_stride = ((size_t)n + 63) / 64 * 64;
        JPCG_HIP(hipMalloc(&c->work[0], sizeof(double) * c->work_stride * cg_ctx::kWorkVecs));
        for (int v = 1; v < cg_ctx::kWorkVecs; ++v) c->work[v] = c->work[0] + (size_t)v * c->work_stride;
        JPCG_HIP(hipMemsetAsync(c->work[0], 0, sizeof(double) * c->work_stride * cg_ctx::kWorkVecs, c->stream));
        JPCG_HIP(hipEventCreate(&c->ev0));
        JPCG_HIP(hipEventCreate(&c->ev1));
        JPCG_HIP(hipMemcpyAsync(c->rowptr, rp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, c->stream));
        if (nnz) {
            JPCG_HIP(hipMemcpyAsync(c->col, hcol.data(), sizeof(int) * nnz, hipMemcpyHostToDevice, c->stream));
            JPCG_HIP(hipMemcpyAsync(c->val, hval.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, c->stream));
        }
        if (c->opts.fp32_copy) {
            JPCG_HIP(hipMalloc(&c->val32, sizeof(float) * (nnz + kCsrPad)));
            JPCG_HIP(hipMemsetAsync(c->val32 + nnz, 0, sizeof(float) * kCsrPad, c->stream));
            JPCG_HIP(hipMalloc(&c->dinv32, sizeof(float) * n));
            JPCG_HIP(hipMalloc(&c->rowsum32, sizeof(float) * n));
            JPCG_HIP(hipMalloc(&c->rowsum64, sizeof(double) * n));
            if (nnz) cast_f32_kernel<<<1024, 256, 0, c->stream>>>(nnz, c->val, c->val32);
            rowsum_kernel<<<(n + 255) / 256, 256, 0, c->stream>>>(n, c->rowptr, c->val, c->rowsum32, c->rowsum64);
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
        c->form = c->opts.form;
        // Default tile width: the fastest measured at the paper's size and at
        // 128^3 in both forms (fewer, fuller tiles amortise each tile's
        // load-gather-sum latency chain).
        c->npl = c->opts.nnz_per_lane ? c->opts.nnz_per_lane : 16;
        c->bs = c->opts.block_size ? c->opts.block_size : 512;
        if (c->npl == 16 && c->bs == 1024) c->bs = 512;  // product tiles must fit 64 KiB of LDS
        c->grid = default_grid(c, c->npl, c->bs, c->opts.blocks_per_cu ? c->opts.blocks_per_cu : 1);
        if (c->opts.autotune) {
            autotune(c);
        } else {
            c->graphs = make_graphs(c, c->form, false, c->npl, c->bs, c->grid, c->chunk);
            // The standalone product: the solver's shape if the caller chose
            // one, else tile width 8, block 512, two workgroups per CU.
            const bool explicit_shape = c->opts.nnz_per_lane || c->opts.block_size || c->opts.blocks_per_cu;
            c->spmv = explicit_shape ? make_spmv_plan(c, c->npl, c->bs, c->grid)
                                     : make_spmv_plan(c, 8, 512, default_grid(c, 8, 512, 2));
        }
        // The mixed form needs the standard FP64 graphs (outer residual) and
        // FP32 standard graphs (inner solve) with the same tile shape.
        if (c->opts.fp32_copy) {
            c->graphs_std = c->form == CG_FORM_STANDARD
                                ? c->graphs
                                : make_graphs(c, CG_FORM_STANDARD, false, c->npl, c->bs, c->grid, c->chunk);
            c->graphs32 = make_graphs(c, CG_FORM_STANDARD, true, c->npl, c->bs, c->grid, c->chunk);
            JPCG_HIP(hipMalloc(&c->mixed_dev, 64));
            JPCG_HIP(hipHostMalloc(&c->mixed_host, 64, hipHostMallocDefault));
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
        JPCG_HIP(hipEventRecord(c->ev0, c->stream));
        const SolveResult st = run_solve(c, c->graphs, b, x, tol, maxit, hist);
        JPCG_HIP(hipEventRecord(c->ev1, c->stream));
        JPCG_HIP(hipEventSynchronize(c->ev1));
        float ms = 0.f;
        JPCG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        const int status = status_of(st.stop);
        c->hist_len = hist ? st.iters + 1 : 0;
        if (info) {
            info->iters = st.iters;
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

int cg_solve_mixed(cg_ctx* c, const double* b, double* x, double tol, int32_t maxit_outer, double tol_inner,
                   int32_t maxit_inner, cg_info* info)
{
    if (!c) return CG_EINVAL;
    if (!c->graphs32) return set_error(c, CG_EINVAL, "cg_solve_mixed: the context was created without fp32_copy");
    if (!b || !x || b == x || !(tol >= 0.0) || !std::isfinite(tol) || !(tol_inner >= 0.0) || !std::isfinite(tol_inner))
        return set_error(c, CG_EINVAL, "cg_solve_mixed: bad arguments");
    if (maxit_outer <= 0) maxit_outer = 50;
    if (maxit_inner <= 0) maxit_inner = c->n;
    if (tol_inner == 0.0) tol_inner = 1e-3;
    try {
        JPCG_HIP(hipEventRecord(c->ev0, c->stream));
        const MixedResult r = run_mixed(c, b, x, tol, maxit_outer, tol_inner, maxit_inner);
        JPCG_HIP(hipEventRecord(c->ev1, c->stream));
        JPCG_HIP(hipEventSynchronize(c->ev1));
        float ms = 0.f;
        JPCG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        if (info) {
            info->iters = r.inner_iters;
            info->status = r.status;
            info->replacements = 0;
            info->outer = r.outer;
            const double rel = r.nb > 0 ? std::sqrt(r.rr) / r.nb : 0.0;
            info->relres_recur = rel;
            info->relres_true = rel;
            info->seconds = ms * 1e-3;
        }
        return r.status;
    } catch (const HipError& e) {
        return set_error(c, CG_EHIP, std::string("cg_solve_mixed: ") + e.what + ": " + hipGetErrorString(e.code));
    }
}

int cg_solve_mixed_matrix(cg_ctx* c, const double* b, double* x, double tol, int32_t maxit, double drop,
                          cg_info* info)
{
    if (!c) return CG_EINVAL;
    if (!c->val32) return set_error(c, CG_EINVAL, "cg_solve_mixed_matrix: the context was created without fp32_copy");
    if (!b || !x || b == x || !(tol >= 0.0) || !std::isfinite(tol) || !(drop >= 0.0 && drop < 1.0))
        return set_error(c, CG_EINVAL, "cg_solve_mixed_matrix: bad arguments");
    if (maxit <= 0) maxit = c->n;
    if (drop == 0.0) drop = 1e-2;
    try {
        if (!c->graphs_m32 || c->graphs_m32->args.drop2 != drop * drop) {
            destroy_graphs(c->graphs_m32);
            c->graphs_m32 = nullptr;
            // Each reliable update drains the chunk in flight, so this form
            // takes chunks of 8 unless the caller chose a length (at 51^3:
            // 8.25 ms against 8.42 ms at 16; unchanged at 128^3).
            const int chunk = c->opts.chunk ? c->chunk : std::min(c->chunk, 8);
            c->graphs_m32 = make_graphs(c, CG_FORM_STANDARD, false, c->npl, c->bs, c->grid, chunk, true, drop);
        }
        JPCG_HIP(hipEventRecord(c->ev0, c->stream));
        const SolveResult st = run_solve(c, c->graphs_m32, b, x, tol, maxit, nullptr);
        JPCG_HIP(hipEventRecord(c->ev1, c->stream));
        JPCG_HIP(hipEventSynchronize(c->ev1));
        float ms = 0.f;
        JPCG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        const int status = status_of(st.stop);
        if (info) {
            info->iters = st.iters;
            info->status = status;
            info->replacements = st.replacements;
            info->outer = 0;
            info->relres_recur = st.nb > 0 ? std::sqrt(st.rr) / st.nb : 0.0;
            info->relres_true = st.nb > 0 ? std::sqrt(st.rr_true) / st.nb : 0.0;
            info->seconds = ms * 1e-3;
        }
        return status;
    } catch (const HipError& e) {
        return set_error(c, CG_EHIP, std::string("cg_solve_mixed_matrix: ") + e.what + ": " + hipGetErrorString(e.code));
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
    cfg->tiles = c->graphs ? c->graphs->T : 0;
    cfg->chunk = c->chunk;
    cfg->form = c->form;
    cfg->tune_cached = c->tune_cached ? 1 : 0;
    cfg->col_bits = c->graphs && c->graphs->col16 ? 16 : 32;
    cfg->spmv_nnz_per_lane = c->spmv ? c->spmv->npl : 0;
    cfg->spmv_block_size = c->spmv ? c->spmv->bs : 0;
    cfg->spmv_grid = c->spmv ? c->spmv->G : 0;
    cfg->spmv_us = c->tuned_spmv_us;
    cfg->iter_us = c->tuned_iter_us;
    cfg->spmm_blocks_per_cu = c->spmm_wpc;
    cfg->spmm_pad = 0;
    cfg->spmm_us = c->tuned_spmm_us;
    return 0;
}

}  // extern "C"
