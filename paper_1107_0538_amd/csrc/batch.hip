// Batched Jacobi-PCG: many independent SPD systems in one persistent launch.
//
// The systems are concatenated into one block-diagonal CSR (global row and
// column indices, int32) and each system's rows are cut into product tiles
// (tiles.hpp).  System s is owned by a team of workgroups sized in proportion
// to its expected work (nonzeros times an iteration count that grows with the
// grid size); member L of a team owns an equal run of the system's tiles.
// Every team runs the full solve of the FP64 oracle's loop (pcg_team,
// residual replacement included) on its own rows, meeting at its own grid
// barrier between steps -- a team of one workgroup needs only __syncthreads.  The launch is captured in a hipGraph together
// with the kernel that clears the barriers, so one graph launch solves the
// whole batch.  All teams are co-resident (the grid stays within the
// occupancy limit) and every barrier wait is bounded.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <queue>
#include <vector>

#include "context.hpp"

namespace jpcg {

struct BatchArgs {
    const int* __restrict__ rowptr;  // global, N_total + 1
    const int* __restrict__ col;     // global column indices
    const double* __restrict__ val;
    const double* __restrict__ dinv;
    const double* b;
    double* x;
    double* r;
    ZPair<double>* zp[2];  // {z, p} per row by iteration parity
    double* q;
    const int2* block_team;  // per workgroup: (system, member)
    const int* team_size;    // per system
    const int* part_off;     // per system: offset of its NSLOT * team_size partials
    const int4* tiles;       // every system's product tiles, global rows and nonzeros
    const unsigned short* col16;  // narrow column indices of those tiles, or null
    const int* tile_off;     // per system: first tile; last entry = total tiles
    const int* sys_rows;     // per system: number of rows
    GridBarrier* bar;        // per system
    double* part;
    DevInfo* info;           // per system
    double tol;
    int maxit;               // <= 0: each system's own n
    long long limit;
};

// At least three waves per SIMD: at tile width 16 the kernel would otherwise
// take a few more registers than that allows and run two workgroups per CU
// instead of three (about 8 % slower on the 256-system batch).
template <int NPL, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(3))) void k_batch(BatchArgs a)
{
    __shared__ double lds[(BS / kWave) * 4];
    __shared__ double prod[BS * NPL];
    __shared__ int s_flag;
    const int2 bt = a.block_team[blockIdx.x];
    const int sys = bt.x;
    Team t;
    t.bar = a.bar + sys;
    t.part = a.part + a.part_off[sys];
    t.G = a.team_size[sys];
    t.L = bt.y;
    t.gen = threadIdx.x == 0 ? barrier_gen(t.bar) : 0u;
    t.limit = a.limit;
    t.s_flag = &s_flag;
    const int t0 = a.tile_off[sys], nt = a.tile_off[sys + 1] - t0;
    const TileMap tm{a.tiles + t0, nt, (nt + t.G - 1) / t.G, a.col16};
    SysView<double> v{0, a.rowptr, a.col, a.val, a.dinv, a.b, a.x, a.r, {a.zp[0], a.zp[1]}, a.q};
    const int maxit = a.maxit > 0 ? a.maxit : a.sys_rows[sys];
    double* wprod = prod + (threadIdx.x / kWave) * (kWave * NPL);
    const int st = pcg_team<NPL, BS, double>(v, t, tm, wprod, a.tol, maxit, lds, a.info + sys, nullptr);
    if (st == CG_ETIMEOUT && threadIdx.x == 0 && t.L == 0) a.info[sys].status = CG_ETIMEOUT;
}

// Zero the barrier words (a kernel, not a memset: the graph replays it).
__global__ void k_batch_clear(unsigned* words, int count)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) words[i] = 0u;
}

__global__ void k_batch_jacobi(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                               const double* __restrict__ val, int jacobi, double* __restrict__ dinv,
                               int* __restrict__ bad)
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
}

constexpr int kBatchBS = 256;

}  // namespace jpcg

struct cg_batch {
    hipStream_t stream = nullptr;
    int nsys = 0;
    int64_t n_total = 0;
    int64_t nnz_total = 0;
    int npl = 8;
    int grid = 0;
    std::vector<int64_t> row_off;  // nsys + 1
    std::vector<int> team;         // team sizes
    int* rowptr = nullptr;
    int* col = nullptr;
    double* val = nullptr;
    double* dinv = nullptr;
    double* vec = nullptr;  // b, x, r, {z, p} pairs (two), q: 8 strides of N_total rounded up to 64
    int2* block_team = nullptr;
    int4* tiles = nullptr;
    unsigned short* col16 = nullptr;
    int* ints = nullptr;    // team_size, part_off, sys_rows, tile_off
    jpcg::GridBarrier* bar = nullptr;
    double* part = nullptr;
    jpcg::DevInfo* info = nullptr;
    jpcg::DevInfo* hinfo = nullptr;
    hipGraphExec_t exec = nullptr;
    double graph_tol = -1.0;
    int graph_maxit = -2;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    jpcg::BatchArgs args{};
    long long limit = 0;
    std::string err;
};

namespace jpcg {

static void free_batch(cg_batch* b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    void* ptrs[] = {b->rowptr, b->col, b->val, b->dinv, b->vec, b->block_team, b->tiles, b->col16, b->ints, b->bar,
                    b->part, b->info};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (b->hinfo) (void)hipHostFree(b->hinfo);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    delete b;
}

static const void* batch_kernel(int npl)
{
    switch (npl) {
        case 4: return (const void*)k_batch<4, kBatchBS>;
        case 8: return (const void*)k_batch<8, kBatchBS>;
        case 16: return (const void*)k_batch<16, kBatchBS>;
        default: return nullptr;
    }
}

static void capture_batch(cg_batch* b, double tol, int maxit)
{
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    b->args.tol = tol;
    b->args.maxit = maxit;
    hipStream_t cap;
    JPCG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph;
    JPCG_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    unsigned* words = (unsigned*)b->bar;
    int count = (int)(sizeof(GridBarrier) / sizeof(unsigned)) * b->nsys;
    void* cargs[] = {&words, &count};
    JPCG_HIP(hipLaunchKernel((const void*)k_batch_clear, dim3(std::min(1024, (count + 255) / 256)), dim3(256), cargs,
                             0, cap));
    void* kargs[] = {&b->args};
    JPCG_HIP(hipLaunchKernel(batch_kernel(b->npl), dim3(b->grid), dim3(kBatchBS), kargs, 0, cap));
    JPCG_HIP(hipStreamEndCapture(cap, &graph));
    hipError_t e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    JPCG_HIP(hipStreamDestroy(cap));
    JPCG_HIP(e);
    b->graph_tol = tol;
    b->graph_maxit = maxit;
}

}  // namespace jpcg

using namespace jpcg;

extern "C" {

int cg_batch_create(int32_t nsys, const cg_csr* systems, const cg_opts* opts, void* hip_stream, cg_batch** out)
{
    if (!out) return CG_EINVAL;
    *out = nullptr;
    if (nsys <= 0 || !systems) return CG_EINVAL;
    cg_opts o;
    if (opts) o = *opts; else cg_opts_default(&o);
    if (o.precond == CG_PRECOND_DEFAULT) o.precond = CG_PRECOND_JACOBI;
    if (o.precond != CG_PRECOND_JACOBI && o.precond != CG_PRECOND_NONE) return CG_EINVAL;
    if (o.col_bits != 0 && o.col_bits != 32) return CG_EINVAL;
    if (o.autotune) {
        // Build the batch at each tile width, time 20 iterations of every
        // system (tol 0, b = 1) and keep the fastest.
        cg_batch* best = nullptr;
        double best_s = 1e300;
        int last_rc = CG_EINVAL;
        for (int npl : {4, 8, 16}) {
            cg_opts o2 = o;
            o2.autotune = 0;
            o2.nnz_per_lane = npl;
            cg_batch* cand = nullptr;
            last_rc = cg_batch_create(nsys, systems, &o2, hip_stream, &cand);
            if (last_rc != 0) {
                if (last_rc == CG_EINVAL || last_rc == CG_EDIAG) return last_rc;  // input errors
                continue;
            }
            double t = 1e300;
            double *bv = nullptr, *xv = nullptr;
            std::vector<cg_info> info(nsys);
            try {
                const size_t bytes = sizeof(double) * (size_t)cand->n_total;
                JPCG_HIP(hipMalloc(&bv, bytes));
                JPCG_HIP(hipMalloc(&xv, bytes));
                std::vector<double> ones(cand->n_total, 1.0);
                JPCG_HIP(hipMemcpyAsync(bv, ones.data(), bytes, hipMemcpyHostToDevice, cand->stream));
                JPCG_HIP(hipMemsetAsync(xv, 0, bytes, cand->stream));
                if (cg_batch_solve(cand, bv, xv, 0.0, 20, info.data()) >= 0) t = info[0].seconds;
            } catch (const HipError&) {
                t = 1e300;
            }
            if (bv) (void)hipFree(bv);
            if (xv) (void)hipFree(xv);
            if (t < best_s) {
                cg_batch_destroy(best);
                best = cand;
                best_s = t;
            } else {
                cg_batch_destroy(cand);
            }
        }
        if (!best) return last_rc != 0 ? last_rc : CG_EHIP;
        *out = best;
        return 0;
    }
    cg_batch* b = nullptr;
    try {
        b = new cg_batch();
        b->stream = (hipStream_t)hip_stream;
        b->nsys = nsys;
        b->npl = o.nnz_per_lane ? o.nnz_per_lane : 16;
        if (!batch_kernel(b->npl)) {
            free_batch(b);
            return CG_EINVAL;
        }
        // Validate and concatenate on the host.
        b->row_off.assign(nsys + 1, 0);
        std::vector<int64_t> nnz_off(nsys + 1, 0);
        for (int s = 0; s < nsys; ++s) {
            const cg_csr& A = systems[s];
            if (A.n <= 0 || A.nnz < 0 || !A.rowptr || (A.nnz > 0 && (!A.col || !A.val)) || A.mem != CG_MEM_HOST) {
                free_batch(b);
                return CG_EINVAL;
            }
            b->row_off[s + 1] = b->row_off[s] + A.n;
            nnz_off[s + 1] = nnz_off[s] + A.nnz;
        }
        b->n_total = b->row_off[nsys];
        b->nnz_total = nnz_off[nsys];
        if (b->n_total >= 0x7fffffffLL || b->nnz_total >= 0x7fffffffLL) {
            free_batch(b);
            return CG_EINVAL;
        }
        const int N = (int)b->n_total;
        std::vector<int> rowptr(N + 1);
        std::vector<int> col(b->nnz_total);
        for (int s = 0; s < nsys; ++s) {
            const cg_csr& A = systems[s];
            const int ro = (int)b->row_off[s], ko = (int)nnz_off[s];
            if (A.rowptr[0] != 0 || A.rowptr[A.n] != A.nnz) {
                free_batch(b);
                return CG_EINVAL;
            }
            for (int i = 0; i < A.n; ++i) {
                if (A.rowptr[i + 1] < A.rowptr[i]) {
                    free_batch(b);
                    return CG_EINVAL;
                }
                rowptr[ro + i] = ko + A.rowptr[i];
            }
            for (int64_t k = 0; k < A.nnz; ++k) {
                if (A.col[k] < 0 || A.col[k] >= A.n) {
                    free_batch(b);
                    return CG_EINVAL;
                }
                col[ko + k] = ro + A.col[k];
            }
        }
        rowptr[N] = (int)b->nnz_total;

        // Product tiles of every system (global rows and nonzeros).
        const int cap = kWave * b->npl;
        std::vector<int4> tiles;
        std::vector<int> tile_off(nsys + 1, 0);
        for (int s = 0; s < nsys; ++s) {
            const cg_csr& A = systems[s];
            std::vector<int> local_rp(A.rowptr, A.rowptr + A.n + 1);
            std::vector<int4> ts;
            build_tiles(local_rp, cap, ts);
            const int ro = (int)b->row_off[s], ko = (int)nnz_off[s];
            for (const int4& t : ts) tiles.push_back(int4{t.x + ro, t.y + ro, t.z + ko, t.w + ko});
            tile_off[s + 1] = (int)tiles.size();
        }

        // Teams: workgroups per system in proportion to nnz times rows^(1/3)
        // (CG iterations grow with the grid edge), at most one per tile,
        // within the co-resident capacity (the occupancy limit unless
        // opts->blocks_per_cu asks for fewer per CU).  The product streams
        // the whole batch's matrices from HBM every iteration, so it wants as
        // many waves in flight as fit.
        int dev = 0, cus = 0, per_cu = 0, wall_khz = 0;
        JPCG_HIP(hipGetDevice(&dev));
        JPCG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        JPCG_HIP(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
        JPCG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel(b->npl), kBatchBS, 0));
        b->limit = (long long)std::max(wall_khz, 1000) * 1000LL * 8;  // 8 s of device wall clock
        const int bpc = o.blocks_per_cu > 0 ? std::min(o.blocks_per_cu, per_cu) : 0;
        const int capacity = std::max(nsys, std::max(1, (bpc > 0 ? bpc : per_cu) * cus));
        if (nsys > per_cu * cus) {  // one workgroup per system must still be co-resident
            free_batch(b);
            return CG_EINVAL;
        }
        std::vector<double> work(nsys);
        double total = 0.0;
        for (int s = 0; s < nsys; ++s) {
            const double n_s = (double)systems[s].n, z_s = (double)systems[s].nnz;
            work[s] = (z_s + n_s) * std::cbrt(n_s);
            total += work[s];
        }
        // The batch ends when its slowest team does, and a team's time goes
        // as its work over its size: hand out the workgroups one at a time,
        // each to the team with the largest work per member (which minimises
        // the largest of those ratios), a team never larger than its tiles.
        (void)total;
        b->team.assign(nsys, 1);
        int used = nsys;
        std::priority_queue<std::pair<double, int>> queue;
        for (int s = 0; s < nsys; ++s) queue.push({work[s], s});
        while (used < capacity && !queue.empty()) {
            const int s = queue.top().second;
            queue.pop();
            if (b->team[s] >= std::max(1, tile_off[s + 1] - tile_off[s])) continue;  // no tile left to give
            b->team[s] += 1;
            used += 1;
            queue.push({work[s] / b->team[s], s});
        }
        b->grid = used;
        // Per-workgroup tables.
        std::vector<int2> block_team(used);
        std::vector<int> team_size(nsys), part_off(nsys), sys_rows(nsys);
        int blk = 0, poff = 0;
        for (int s = 0; s < nsys; ++s) {
            const int T = b->team[s];
            team_size[s] = T;
            part_off[s] = poff;
            poff += NSLOT * T;
            sys_rows[s] = systems[s].n;
            for (int L = 0; L < T; ++L) block_team[blk++] = int2{s, L};
        }
        const int ntile_total = (int)tiles.size();

        // Device copies.
        JPCG_HIP(hipMalloc(&b->rowptr, sizeof(int) * (N + 1)));
        JPCG_HIP(hipMalloc(&b->col, sizeof(int) * std::max<int64_t>(b->nnz_total, 1)));
        JPCG_HIP(hipMalloc(&b->val, sizeof(double) * std::max<int64_t>(b->nnz_total, 1)));
        JPCG_HIP(hipMalloc(&b->dinv, sizeof(double) * N));
        const size_t NP = ((size_t)N + 63) / 64 * 64;
        JPCG_HIP(hipMalloc(&b->vec, sizeof(double) * 8 * NP));
        JPCG_HIP(hipMalloc(&b->block_team, sizeof(int2) * used));
        JPCG_HIP(hipMalloc(&b->tiles, sizeof(int4) * std::max(ntile_total, 1)));
        JPCG_HIP(hipMalloc(&b->ints, sizeof(int) * (4 * (size_t)nsys + 1)));
        JPCG_HIP(hipMalloc(&b->bar, sizeof(GridBarrier) * nsys));
        JPCG_HIP(hipMalloc(&b->part, sizeof(double) * std::max(poff, 1)));
        JPCG_HIP(hipMalloc(&b->info, sizeof(DevInfo) * nsys));
        JPCG_HIP(hipHostMalloc(&b->hinfo, sizeof(DevInfo) * nsys, hipHostMallocDefault));
        JPCG_HIP(hipEventCreate(&b->ev0));
        JPCG_HIP(hipEventCreate(&b->ev1));
        hipStream_t st = b->stream;
        JPCG_HIP(hipMemcpyAsync(b->rowptr, rowptr.data(), sizeof(int) * (N + 1), hipMemcpyHostToDevice, st));
        JPCG_HIP(hipMemcpyAsync(b->col, col.data(), sizeof(int) * b->nnz_total, hipMemcpyHostToDevice, st));
        for (int s = 0; s < nsys; ++s)
            JPCG_HIP(hipMemcpyAsync(b->val + nnz_off[s], systems[s].val, sizeof(double) * systems[s].nnz,
                                    hipMemcpyHostToDevice, st));
        JPCG_HIP(hipMemsetAsync(b->vec, 0, sizeof(double) * 8 * NP, st));
        JPCG_HIP(hipMemcpyAsync(b->block_team, block_team.data(), sizeof(int2) * used, hipMemcpyHostToDevice, st));
        int* d_team = b->ints;
        int* d_poff = d_team + nsys;
        int* d_rows = d_poff + nsys;
        int* d_toff = d_rows + nsys;
        JPCG_HIP(hipMemcpyAsync(d_team, team_size.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st));
        JPCG_HIP(hipMemcpyAsync(d_poff, part_off.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st));
        JPCG_HIP(hipMemcpyAsync(d_rows, sys_rows.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st));
        JPCG_HIP(hipMemcpyAsync(d_toff, tile_off.data(), sizeof(int) * (nsys + 1), hipMemcpyHostToDevice, st));
        if (ntile_total > 0)
            JPCG_HIP(hipMemcpyAsync(b->tiles, tiles.data(), sizeof(int4) * ntile_total, hipMemcpyHostToDevice, st));
        int* bad = nullptr;
        JPCG_HIP(hipMalloc(&bad, sizeof(int)));
        JPCG_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
        k_batch_jacobi<<<(N + 255) / 256, 256, 0, st>>>(N, b->rowptr, b->col, b->val, o.precond == CG_PRECOND_JACOBI,
                                                       b->dinv, bad);
        JPCG_HIP(hipGetLastError());
        int hbad = 0;
        JPCG_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        JPCG_HIP(hipStreamSynchronize(st));
        JPCG_HIP(hipFree(bad));
        if (hbad) {
            free_batch(b);
            return CG_EDIAG;
        }
        if (o.col_bits != 32) b->col16 = make_col16(st, b->tiles, ntile_total, b->col, b->nnz_total);
        double* v = b->vec;
        BatchArgs& a = b->args;
        a.rowptr = b->rowptr;
        a.col = b->col;
        a.val = b->val;
        a.dinv = b->dinv;
        a.b = v;
        a.x = v + NP;
        a.r = v + 2 * NP;
        a.zp[0] = (ZPair<double>*)(v + 3 * NP);  // spans strides 3 and 4
        a.zp[1] = (ZPair<double>*)(v + 5 * NP);  // spans strides 5 and 6
        a.q = v + 7 * NP;
        a.block_team = b->block_team;
        a.team_size = d_team;
        a.part_off = d_poff;
        a.tiles = b->tiles;
        a.col16 = b->col16;
        a.tile_off = d_toff;
        a.sys_rows = d_rows;
        a.bar = b->bar;
        a.part = b->part;
        a.info = b->info;
        a.limit = b->limit;
        *out = b;
        return 0;
    } catch (const HipError& e) {
        free_batch(b);
        return e.code == hipErrorOutOfMemory ? CG_ENOMEM : CG_EHIP;
    } catch (const std::bad_alloc&) {
        free_batch(b);
        return CG_ENOMEM;
    }
}

int cg_batch_solve(cg_batch* b, const double* b_cat, double* x_cat, double tol, int32_t maxit, cg_info* info)
{
    if (!b) return CG_EINVAL;
    if (!b_cat || !x_cat || b_cat == x_cat || !(tol >= 0.0) || !std::isfinite(tol)) return CG_EINVAL;
    try {
        if (!b->exec || b->graph_tol != tol || b->graph_maxit != maxit) capture_batch(b, tol, maxit);
        hipStream_t st = b->stream;
        const size_t vb = sizeof(double) * (size_t)b->n_total;
        JPCG_HIP(hipEventRecord(b->ev0, st));
        JPCG_HIP(hipMemcpyAsync((void*)b->args.b, b_cat, vb, hipMemcpyDeviceToDevice, st));
        JPCG_HIP(hipMemcpyAsync(b->args.x, x_cat, vb, hipMemcpyDeviceToDevice, st));
        JPCG_HIP(hipGraphLaunch(b->exec, st));
        JPCG_HIP(hipMemcpyAsync(x_cat, b->args.x, vb, hipMemcpyDeviceToDevice, st));
        JPCG_HIP(hipEventRecord(b->ev1, st));
        JPCG_HIP(hipMemcpyAsync(b->hinfo, b->info, sizeof(DevInfo) * b->nsys, hipMemcpyDeviceToHost, st));
        JPCG_HIP(hipStreamSynchronize(st));
        float ms = 0.f;
        JPCG_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
        int worst = CG_CONVERGED;
        bool timeout = false;
        for (int s = 0; s < b->nsys; ++s) {
            const DevInfo& d = b->hinfo[s];
            if (d.status == CG_ETIMEOUT) timeout = true;
            else worst = std::max(worst, d.status);
            if (info) {
                const double nb = std::sqrt(d.bb);
                info[s].iters = d.iters;
                info[s].status = d.status;
                info[s].replacements = d.replacements;
                info[s].outer = 0;
                info[s].relres_recur = nb > 0 ? std::sqrt(d.rr_recur) / nb : 0.0;
                info[s].relres_true = nb > 0 ? std::sqrt(d.rr_true) / nb : 0.0;
                info[s].seconds = ms * 1e-3;
            }
        }
        if (timeout) {
            b->err = "a team barrier timed out";
            return CG_ETIMEOUT;
        }
        return worst;
    } catch (const HipError& e) {
        b->err = std::string("cg_batch_solve: ") + e.what + ": " + hipGetErrorString(e.code);
        return CG_EHIP;
    }
}

int64_t cg_batch_offset(const cg_batch* b, int32_t s)
{
    if (!b || s < 0 || s > b->nsys) return CG_EINVAL;
    return b->row_off[s];
}

int cg_batch_teams(const cg_batch* b, int32_t* team_sizes)
{
    if (!b || !team_sizes) return CG_EINVAL;
    for (int s = 0; s < b->nsys; ++s) team_sizes[s] = b->team[s];
    return b->grid;
}

const char* cg_batch_last_error(const cg_batch* b) { return b ? b->err.c_str() : ""; }

void cg_batch_destroy(cg_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    free_batch(b);
}

}  // extern "C"
