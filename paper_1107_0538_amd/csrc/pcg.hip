// Single-system Jacobi-PCG on one MI355X: create, solve, spmv.
//
// The CG loop of the paper's case study (Section IV) runs as ONE persistent,
// cooperatively launched kernel: the scalars the paper computed on the host
// (alpha, beta, the continue-condition) are reduced on the device and every
// workgroup takes the same decision, so no host round trip happens inside the
// loop.  The sparse product the paper calls "DGEMV(sparse)" is a vector-CSR
// kernel: LPR lanes of a wave share one row, stream its column indices and
// values with coalesced loads and gather x through L1/L2.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "context.hpp"

namespace jpcg {

constexpr int kBS = 256;

struct SolveParams {
    SysView<double> s;
    const int* blk_row;
    GridBarrier* bar;
    double* part;
    DevInfo* info;
    double* hist;
    double tol;
    int maxit;
    int G;
    long long limit;
};

template <int LPR, int BS>
__global__ __launch_bounds__(BS) void pcg_solve_kernel(SolveParams a)
{
    __shared__ double lds[(BS / kWave) * 4];
    __shared__ int s_flag;
    Team t;
    t.bar = a.bar;
    t.part = a.part;
    t.G = a.G;
    t.L = xcd_logical_block((int)blockIdx.x, a.G);
    t.gen = threadIdx.x == 0 ? barrier_gen(a.bar) : 0u;
    t.limit = a.limit;
    t.s_flag = &s_flag;
    const int rs = a.blk_row[t.L], re = a.blk_row[t.L + 1];
    pcg_team<LPR, BS, double>(a.s, t, rs, re, a.tol, a.maxit, lds, a.info, a.hist);
}

// y = A x, one row per group of LPR lanes.
template <int LPR, int BS, typename T>
__global__ __launch_bounds__(BS) void spmv_kernel(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                                                  const T* __restrict__ val, const T* __restrict__ x, T* __restrict__ y)
{
    const int b = xcd_logical_block((int)blockIdx.x, (int)gridDim.x);
    const int i = b * (BS / LPR) + (int)threadIdx.x / LPR;
    const int lane = threadIdx.x & (LPR - 1);
    T acc = T(0);
    if (i < n) {
        const int k1 = rowptr[i + 1];
        for (int k = rowptr[i] + lane; k < k1; k += LPR) acc = fma_t(val[k], x[col[k]], acc);
    }
    acc = group_sum<LPR>(acc);
    if (lane == 0 && i < n) y[i] = acc;
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

static const void* solve_kernel(int lpr)
{
    switch (lpr) {
        case 4: return (const void*)pcg_solve_kernel<4, kBS>;
        case 8: return (const void*)pcg_solve_kernel<8, kBS>;
        case 16: return (const void*)pcg_solve_kernel<16, kBS>;
        case 32: return (const void*)pcg_solve_kernel<32, kBS>;
        case 64: return (const void*)pcg_solve_kernel<64, kBS>;
        default: return nullptr;
    }
}

static bool valid_lpr(int l) { return l == 4 || l == 8 || l == 16 || l == 32 || l == 64; }

static void launch_spmv(hipStream_t st, int lpr, int n, const int* rowptr, const int* col, const double* val,
                        const double* x, double* y)
{
    const int rows_per_block = kBS / lpr;
    int grid = (n + rows_per_block - 1) / rows_per_block;
    grid = (grid + 7) / 8 * 8;  // whole XCD rounds for the logical remap
    switch (lpr) {
        case 4: spmv_kernel<4, kBS, double><<<grid, kBS, 0, st>>>(n, rowptr, col, val, x, y); break;
        case 8: spmv_kernel<8, kBS, double><<<grid, kBS, 0, st>>>(n, rowptr, col, val, x, y); break;
        case 16: spmv_kernel<16, kBS, double><<<grid, kBS, 0, st>>>(n, rowptr, col, val, x, y); break;
        case 32: spmv_kernel<32, kBS, double><<<grid, kBS, 0, st>>>(n, rowptr, col, val, x, y); break;
        default: spmv_kernel<64, kBS, double><<<grid, kBS, 0, st>>>(n, rowptr, col, val, x, y); break;
    }
    JPCG_HIP(hipGetLastError());
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

int max_coop_grid(cg_ctx* c, int lpr)
{
    int per_cu = 0;
    JPCG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, solve_kernel(lpr), kBS, 0));
    return std::max(per_cu, 0) * c->cus;
}

void ensure_grid(cg_ctx* c, int G)
{
    if (G > c->grid_cap) {
        if (c->part) JPCG_HIP(hipFree(c->part));
        if (c->blk_row) JPCG_HIP(hipFree(c->blk_row));
        c->part = nullptr;
        c->blk_row = nullptr;
        JPCG_HIP(hipMalloc(&c->part, sizeof(double) * NSLOT * (size_t)G));
        JPCG_HIP(hipMalloc(&c->blk_row, sizeof(int) * ((size_t)G + 1)));
        c->grid_cap = G;
        c->blk_row_grid = 0;
    }
    if (c->blk_row_grid != G) {
        std::vector<int> rows;
        partition_rows(c->h_rowptr, G, rows);
        JPCG_HIP(hipMemcpyAsync(c->blk_row, rows.data(), sizeof(int) * rows.size(), hipMemcpyHostToDevice, c->stream));
        JPCG_HIP(hipStreamSynchronize(c->stream));
        c->blk_row_grid = G;
    }
}

bool barrier_aborted(hipStream_t stream, GridBarrier* bar)
{
    unsigned ab = 0;
    JPCG_HIP(hipMemcpyAsync(&ab, &bar->abort, sizeof(unsigned), hipMemcpyDeviceToHost, stream));
    JPCG_HIP(hipStreamSynchronize(stream));
    if (ab) {
        JPCG_HIP(hipMemsetAsync(bar, 0, sizeof(GridBarrier), stream));
        JPCG_HIP(hipStreamSynchronize(stream));
    }
    return ab != 0;
}

// Grid for a given LPR: persistent workgroups per CU, capped by occupancy
// and by the amount of work (at least one row group per workgroup).
static int pick_grid(cg_ctx* c, int lpr, int blocks_per_cu)
{
    const int cap = max_coop_grid(c, lpr);
    int G = c->cus * std::max(1, blocks_per_cu);
    G = std::min(G, cap);
    const int rows_per_pass = kBS / lpr;
    const int need = (c->n + rows_per_pass - 1) / rows_per_pass;
    G = std::min(G, std::max(8, (need + 7) / 8 * 8));
    if (G >= 8) G = G / 8 * 8;
    return std::max(G, 1);
}

static void launch_solve(cg_ctx* c, int lpr, int G, const double* b, double* x, double tol, int maxit, double* hist)
{
    ensure_grid(c, G);
    SolveParams a;
    a.s = SysView<double>{c->n, c->rowptr, c->col, c->val, c->dinv, b, x, c->r, c->z, c->p0, c->p1, c->q};
    a.blk_row = c->blk_row;
    a.bar = c->bar;
    a.part = c->part;
    a.info = c->dinfo;
    a.hist = hist;
    a.tol = tol;
    a.maxit = maxit;
    a.G = G;
    a.limit = c->limit_ticks;
    void* args[] = {&a};
    JPCG_HIP(hipLaunchCooperativeKernel(solve_kernel(lpr), dim3(G), dim3(kBS), args, 0, c->stream));
}

// Time `reps` standalone products with each LPR and a short solve with each
// (LPR, workgroups per CU); keep the fastest of each.
static void autotune(cg_ctx* c)
{
    double *xb = nullptr, *yb = nullptr;
    JPCG_HIP(hipMalloc(&xb, sizeof(double) * c->n));
    JPCG_HIP(hipMalloc(&yb, sizeof(double) * c->n));
    std::vector<double> ones(c->n, 1.0);
    JPCG_HIP(hipMemcpyAsync(yb, ones.data(), sizeof(double) * c->n, hipMemcpyHostToDevice, c->stream));
    JPCG_HIP(hipMemsetAsync(xb, 0, sizeof(double) * c->n, c->stream));
    const int lprs[] = {4, 8, 16, 32, 64};
    float best = 1e30f, ms = 0.f;
    for (int l : lprs) {
        launch_spmv(c->stream, l, c->n, c->rowptr, c->col, c->val, yb, xb);
        const int reps = 20;
        JPCG_HIP(hipEventRecord(c->ev0, c->stream));
        for (int r = 0; r < reps; ++r) launch_spmv(c->stream, l, c->n, c->rowptr, c->col, c->val, yb, xb);
        JPCG_HIP(hipEventRecord(c->ev1, c->stream));
        JPCG_HIP(hipEventSynchronize(c->ev1));
        JPCG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        if (ms / reps < best) {
            best = ms / reps;
            c->spmv_lpr = l;
        }
    }
    c->tuned_spmv_us = best * 1e3;
    // Solver: fixed iteration count from x = 0 with b = 1 (tol 0 forces maxit).
    const int iters = std::min(40, std::max(4, c->n));
    best = 1e30f;
    for (int l : lprs) {
        const int cap = max_coop_grid(c, l) / std::max(c->cus, 1);
        for (int bpc = 1; bpc <= std::min(cap, 8); bpc *= 2) {
            const int G = pick_grid(c, l, bpc);
            JPCG_HIP(hipMemsetAsync(xb, 0, sizeof(double) * c->n, c->stream));
            JPCG_HIP(hipEventRecord(c->ev0, c->stream));
            launch_solve(c, l, G, yb, xb, 0.0, iters, nullptr);
            JPCG_HIP(hipEventRecord(c->ev1, c->stream));
            JPCG_HIP(hipEventSynchronize(c->ev1));
            JPCG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
            if (barrier_aborted(c->stream, c->bar)) throw HipError{hipErrorLaunchTimeOut, "autotune solve timed out"};
            if (ms < best) {
                best = ms;
                c->lpr = l;
                c->grid = G;
            }
        }
    }
    c->tuned_iter_us = best * 1e3 / iters;
    JPCG_HIP(hipFree(xb));
    JPCG_HIP(hipFree(yb));
}

static void free_ctx(cg_ctx* c)
{
    if (!c) return;
    void* ptrs[] = {c->rowptr, c->col, c->val, c->dinv, c->val32, c->dinv32, c->r, c->z, c->p0, c->p1,
                    c->q, c->part, c->blk_row, c->bar, c->dinfo, c->hist};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (c->hinfo) (void)hipHostFree(c->hinfo);
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
        if (c->opts.precond != CG_PRECOND_JACOBI && c->opts.precond != CG_PRECOND_NONE) {
            free_ctx(c);
            return CG_EINVAL;
        }
        if (c->opts.lanes_per_row && !valid_lpr(c->opts.lanes_per_row)) {
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
        if (rp[0] != 0 || rp[n] != nnz) {
            int rc = set_error(c, CG_EINVAL, "rowptr[0] must be 0 and rowptr[n] must equal nnz");
            free_ctx(c);
            return rc;
        }
        for (int i = 0; i < n; ++i)
            if (rp[i + 1] < rp[i]) {
                free_ctx(c);
                return CG_EINVAL;
            }
        for (int64_t k = 0; k < nnz; ++k)
            if (hcol[k] < 0 || hcol[k] >= n) {
                free_ctx(c);
                return CG_EINVAL;
            }

        JPCG_HIP(hipMalloc(&c->rowptr, sizeof(int) * (n + 1)));
        JPCG_HIP(hipMalloc(&c->col, sizeof(int) * std::max<int64_t>(nnz, 1)));
        JPCG_HIP(hipMalloc(&c->val, sizeof(double) * std::max<int64_t>(nnz, 1)));
        JPCG_HIP(hipMalloc(&c->dinv, sizeof(double) * n));
        for (double** v : {&c->r, &c->z, &c->p0, &c->p1, &c->q}) JPCG_HIP(hipMalloc(v, sizeof(double) * n));
        JPCG_HIP(hipMalloc(&c->bar, sizeof(GridBarrier)));
        JPCG_HIP(hipMalloc(&c->dinfo, sizeof(DevInfo)));
        JPCG_HIP(hipHostMalloc(&c->hinfo, sizeof(DevInfo), hipHostMallocDefault));
        JPCG_HIP(hipEventCreate(&c->ev0));
        JPCG_HIP(hipEventCreate(&c->ev1));
        JPCG_HIP(hipMemcpyAsync(c->rowptr, rp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, c->stream));
        if (nnz) {
            JPCG_HIP(hipMemcpyAsync(c->col, hcol.data(), sizeof(int) * nnz, hipMemcpyHostToDevice, c->stream));
            JPCG_HIP(hipMemcpyAsync(c->val, hval.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, c->stream));
        }
        JPCG_HIP(hipMemsetAsync(c->bar, 0, sizeof(GridBarrier), c->stream));
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
        c->lpr = c->opts.lanes_per_row ? c->opts.lanes_per_row : 32;
        c->spmv_lpr = c->lpr;
        c->grid = pick_grid(c, c->lpr, c->opts.blocks_per_cu ? c->opts.blocks_per_cu : 2);
        if (c->opts.autotune) autotune(c);
        ensure_grid(c, c->grid);
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
        launch_solve(c, c->lpr, c->grid, b, x, tol, maxit, hist);
        JPCG_HIP(hipEventRecord(c->ev1, c->stream));
        JPCG_HIP(hipMemcpyAsync(c->hinfo, c->dinfo, sizeof(DevInfo), hipMemcpyDeviceToHost, c->stream));
        JPCG_HIP(hipStreamSynchronize(c->stream));
        if (barrier_aborted(c->stream, c->bar)) {
            if (info) info->status = CG_ETIMEOUT;
            return set_error(c, CG_ETIMEOUT, "cg_solve: a grid barrier timed out");
        }
        float ms = 0.f;
        JPCG_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        const DevInfo& d = *c->hinfo;
        c->hist_len = hist ? d.iters + 1 : 0;
        if (info) {
            const double nb = std::sqrt(d.bb);
            info->iters = d.iters;
            info->status = d.status;
            info->replacements = d.replacements;
            info->outer = 0;
            info->relres_recur = nb > 0 ? std::sqrt(d.rr_recur) / nb : 0.0;
            info->relres_true = nb > 0 ? std::sqrt(d.rr_true) / nb : 0.0;
            info->seconds = ms * 1e-3;
        }
        return d.status;
    } catch (const HipError& e) {
        return set_error(c, CG_EHIP, std::string("cg_solve: ") + e.what + ": " + hipGetErrorString(e.code));
    }
}

int spmv(cg_ctx* c, const double* x, double* y)
{
    if (!c) return CG_EINVAL;
    if (!x || !y || x == y) return set_error(c, CG_EINVAL, "spmv: x and y must be distinct device pointers");
    try {
        launch_spmv(c->stream, c->spmv_lpr, c->n, c->rowptr, c->col, c->val, x, y);
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
    cfg->lanes_per_row = c->lpr;
    cfg->block_size = kBS;
    cfg->grid = c->grid;
    cfg->spmv_lanes = c->spmv_lpr;
    cfg->spmv_us = c->tuned_spmv_us;
    cfg->iter_us = c->tuned_iter_us;
    return 0;
}

}  // extern "C"
