// The solver context behind the opaque cg_ctx handle, shared by the
// translation units that implement the single-system and form entry points.
#pragma once

#include <string>
#include <vector>

#include "phases.hpp"

namespace jpcg {
// Zero entries after the last nonzero of the context's col and val arrays
// (the multi-RHS row products read batches of up to 32 past a row's start).
constexpr int kCsrPad = 32;
}  // namespace jpcg

struct cg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n = 0;
    int64_t nnz = 0;
    cg_opts opts{};

    // Library-owned copy of A and the preconditioner.
    int* rowptr = nullptr;
    int* col = nullptr;
    double* val = nullptr;
    double* dinv = nullptr;
    float* val32 = nullptr;   // fp32_copy
    float* dinv32 = nullptr;  // fp32_copy
    float* rowsum32 = nullptr;  // fp32_copy: row sums of A (FP64 sums, FP32 storage)
    double* rowsum64 = nullptr; // fp32_copy: the same row sums in FP64 (FP32-matrix form)
    std::vector<int> h_rowptr;

    // Work vectors for single-RHS solves (one allocation, each vector at a
    // stride of n rounded up to 64 entries, so every vector starts 512-byte
    // aligned): the standard form uses r, two interleaved {z, p} pair arrays
    // of two vectors each, and q; the single-reduction form uses two
    // {r, w, s, d} quad arrays of four vectors each, and p.
    static constexpr int kWorkVecs = 9;
    double* work[kWorkVecs] = {};
    size_t work_stride = 0;

    // Graph-chunked solver for the chosen launch shape.
    struct cg_graphs* graphs = nullptr;      // the context's form, FP64
    struct cg_graphs* graphs_std = nullptr;  // standard form FP64 (mixed-form outer residual)
    struct cg_graphs* graphs32 = nullptr;    // standard form FP32 (mixed-form inner solve)
    struct cg_graphs* graphs_m32 = nullptr;  // standard form FP64 with the FP32 matrix stream
    void* mixed_dev = nullptr;
    void* mixed_host = nullptr;
    struct cg_spmv_plan* spmv = nullptr;     // the standalone product's tiling and grid
    struct cg_multi* multi = nullptr;        // multi-RHS solver for one block width
    struct cg_multi* multi32 = nullptr;      // FP32 multi-RHS inner solver (mixed form)
    struct cg_block* block = nullptr;        // block CG solver (up to 64 right-hand sides)
    double* hist = nullptr;
    int hist_cap = 0;
    int hist_len = 0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int cus = 0;
    long long limit_ticks = 0;

    // Launch shape.
    int form = CG_FORM_STANDARD;
    int npl = 8;   // nonzeros per lane of a product tile
    int bs = 512;
    int grid = 0;
    int chunk = 16;
    int spmm_wpc = 0;            // workgroups per CU of the multi-column product (0: not chosen yet)
    double tuned_spmm_us = 0.0;
    double tuned_spmv_us = 0.0;
    double tuned_iter_us = 0.0;
    bool tune_cached = false;  // the tuned shape came from an earlier context

    std::string err;
};

namespace jpcg {

// Row boundaries of G workgroups with about (nnz + n) / G rows-plus-nonzeros each.
void partition_rows(const std::vector<int>& rowptr, int G, std::vector<int>& out);

int set_error(cg_ctx* c, int code, const std::string& msg);

// Free the multi-RHS solver state of a context (multi.hip).
void free_multi(cg_ctx* c);

// Workgroups per CU of the multi-column row products, chosen at first use
// (timed when the context was created with autotune) (multi.hip).
int spmm_blocks_per_cu(cg_ctx* c);

// Free the block solver state of a context (block.hip).
void free_block(cg_ctx* c);

}  // namespace jpcg
