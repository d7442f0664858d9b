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

    // Graph-chunked solver for the chosen launch shape.
    struct cg_graphs* graphs = nullptr;
    double* hist = nullptr;
    int hist_cap = 0;
    int hist_len = 0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int cus = 0;
    long long limit_ticks = 0;

    // Launch shape.
    int npl = 8;   // nonzeros per lane of a product tile
    int bs = 512;
    int grid = 0;
    int chunk = 16;
    double tuned_spmv_us = 0.0;
    double tuned_iter_us = 0.0;

    std::string err;
};

namespace jpcg {

// Row boundaries of G workgroups with about (nnz + n) / G rows-plus-nonzeros each.
void partition_rows(const std::vector<int>& rowptr, int G, std::vector<int>& out);

int set_error(cg_ctx* c, int code, const std::string& msg);

}  // namespace jpcg
