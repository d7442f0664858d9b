// The solver context behind the opaque cg_ctx handle, shared by the
// translation units that implement the single-system and form entry points.
#pragma once

#include <string>
#include <vector>

#include "phases.hpp"

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
    std::vector<int> h_rowptr;

    // Work vectors for single-RHS solves (n each).
    double* r = nullptr;
    double* z = nullptr;
    double* p0 = nullptr;
    double* p1 = nullptr;
    double* q = nullptr;

    // Persistent-grid state.
    double* part = nullptr;  // NSLOT * grid_cap
    int* blk_row = nullptr;  // grid_cap + 1
    int grid_cap = 0;
    int blk_row_grid = 0;    // grid the current blk_row was built for
    jpcg::GridBarrier* bar = nullptr;
    jpcg::DevInfo* dinfo = nullptr;
    jpcg::DevInfo* hinfo = nullptr;  // pinned
    double* hist = nullptr;
    int hist_cap = 0;
    int hist_len = 0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int cus = 0;
    long long limit_ticks = 0;

    // Launch shape.
    int lpr = 32;
    int spmv_lpr = 32;
    int grid = 0;
    double tuned_spmv_us = 0.0;
    double tuned_iter_us = 0.0;

    std::string err;
};

namespace jpcg {

// Row boundaries of G workgroups with about nnz / G nonzeros each.
void partition_rows(const std::vector<int>& rowptr, int G, std::vector<int>& out);

// Ensure the context's persistent-grid buffers fit `G` workgroups and the
// row partition matches it.
void ensure_grid(cg_ctx* c, int G);

// Largest cooperative grid for the FP64 solver at `lpr`.
int max_coop_grid(cg_ctx* c, int lpr);

// Read back the barrier's abort word; reset the barrier if it was raised.
bool barrier_aborted(hipStream_t stream, GridBarrier* bar);

int set_error(cg_ctx* c, int code, const std::string& msg);

}  // namespace jpcg
