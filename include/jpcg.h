/*
 * jpcg -- Jacobi-preconditioned conjugate gradients for CSR finite-element
 * systems on AMD MI355X (gfx950).
 *
 * The operation is the one the paper parallelises (Section IV): the conjugate-
 * gradient method for a symmetric positive-definite matrix stored in CSR, run
 * to a relative residual of 1e-10 (Table I caption) within at most N
 * iterations.  Its repetitive work -- the sparse matrix-vector product the
 * paper calls "DGEMV(sparse)" and the vector updates and dot products around
 * it -- runs in hand-written HIP kernels.  The scalar steps the paper kept on
 * the host (alpha, beta, the continue-condition) stay on the device here.
 *
 * Conventions for every call:
 *   - Matrices are square CSR: int32 rowptr[n+1] (rowptr[0] = 0, non-
 *     decreasing, rowptr[n] = nnz), int32 col[nnz] in [0, n), float64
 *     val[nnz].  Columns need not be sorted; the Jacobi preconditioner needs
 *     every diagonal entry present and positive.
 *   - Vectors passed to solve/apply calls are DEVICE pointers on the
 *     context's device; matrices passed to create calls may be host or
 *     device memory (cg_csr.mem).  The library copies matrices into memory it
 *     owns, so the caller may free its arrays once create returns.
 *   - Work is enqueued on the HIP stream given at create.  Calls that return
 *     a status (solves) synchronise that stream before returning; calls that
 *     only compute (spmv, spmm) return after enqueueing.
 *   - Return codes: >= 0 is a solver status (CG_CONVERGED, CG_MAXIT,
 *     CG_BREAKDOWN); < 0 is an API error, with text from cg_strerror() and,
 *     where a context exists, detail from cg_last_error().
 *   - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef JPCG_H
#define JPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Solver statuses (>= 0) and API errors (< 0). */
enum {
    CG_CONVERGED = 0,    /* ||b - A x|| <= tol ||b||, confirmed on the true residual  */
    CG_MAXIT = 1,        /* maxit iterations done; x holds the last iterate          */
    CG_BREAKDOWN = 2,    /* p'Ap <= 0, r'z <= 0 or a non-finite scalar: not SPD / NaN */
    CG_EINVAL = -1,      /* bad argument or malformed CSR                            */
    CG_EDIAG = -2,       /* Jacobi requested but a diagonal entry is missing or <= 0 */
    CG_ENOMEM = -3,      /* device or host allocation failed                         */
    CG_EHIP = -4,        /* a HIP runtime call failed                                */
    CG_ETIMEOUT = -5,    /* a device-side wait exceeded its limit; the kernel left   */
    CG_EUNSUPPORTED = -6, /* option not available for this context                   */
    CG_ESCRATCH = -7     /* request larger than a no-allocation call's fixed scratch */
};

enum { CG_MEM_HOST = 0, CG_MEM_DEVICE = 1 };
/* Preconditioner choice; 0 in cg_opts.precond selects the default (Jacobi). */
enum { CG_PRECOND_DEFAULT = 0, CG_PRECOND_JACOBI = 1, CG_PRECOND_NONE = 2 };

/* Form of the iteration.  Both compute the same Krylov iterates in exact
 * arithmetic and stop by the same rules; the single-reduction form
 * (Chronopoulos and Gear) carries s = A p by a recurrence so that each
 * iteration needs one product, one reduction and one kernel. */
enum { CG_FORM_STANDARD = 0, CG_FORM_SINGLE_REDUCTION = 1 };

/* A square CSR matrix (see the conventions above). */
typedef struct {
    int32_t n;
    int32_t mem; /* CG_MEM_HOST or CG_MEM_DEVICE */
    int64_t nnz;
    const int32_t *rowptr;
    const int32_t *col;
    const double *val;
} cg_csr;

/* Options for cg_create.  Zero-initialised fields take the defaults. */
typedef struct {
    int32_t precond;       /* CG_PRECOND_JACOBI (default) or CG_PRECOND_NONE (M = I)    */
    int32_t fp32_copy;     /* 1: also keep an FP32 copy of the values (mixed form)       */
    int32_t autotune;      /* 1: time launch shapes at create and keep the fastest       */
                           /* (cg_create: reused for later matrices of the same size    */
                           /* and row profile; cg_batch_create: the tile width)         */
    int32_t nnz_per_lane;  /* 4, 8 or 16: a product tile holds 64x that; 0 = 16       */
    int32_t blocks_per_cu; /* 0 = default; workgroups per compute unit of the grid      */
    int32_t history;       /* 1: record ||r_k|| / ||b|| for every iteration            */
    int32_t block_size;    /* 0 = default; else 256, 512 or 1024 threads per workgroup  */
    int32_t chunk;         /* 0 = default; CG iterations per launched hipGraph chunk    */
    int32_t form;          /* CG_FORM_STANDARD (default) or CG_FORM_SINGLE_REDUCTION    */
    int32_t col_bits;      /* 0 = default: the products read 16-bit column offsets from */
                           /* each tile's first row where every one fits (10 bytes per  */
                           /* FP64 nonzero instead of 12; same sums), else 32-bit       */
                           /* columns; 32 = always 32-bit columns                       */
    int32_t reserved[6];   /* must be zero                                               */
} cg_opts;

/* Result of a solve. */
typedef struct {
    int32_t iters;        /* products A p inside the CG loop                          */
    int32_t status;       /* CG_CONVERGED, CG_MAXIT, CG_BREAKDOWN or an API error     */
    int32_t replacements; /* times r was replaced by the true residual                */
    int32_t outer;        /* refinement steps (mixed-precision form), else 0          */
    double relres_recur;  /* ||r_k|| / ||b|| from the recurrence at exit             */
    double relres_true;   /* ||b - A x|| / ||b|| of the returned x, in FP64           */
    double seconds;       /* device time of the solve, HIP events around the kernels */
} cg_info;

/* The launch shape a context uses (after autotuning, if requested). */
typedef struct {
    int32_t nnz_per_lane;  /* a product tile holds up to 64 * nnz_per_lane nonzeros */
    int32_t block_size;
    int32_t grid;          /* workgroups of every solver kernel                   */
    int32_t tiles;         /* product tiles (runs of whole rows) of the matrix    */
    int32_t chunk;         /* iterations per hipGraph chunk                       */
    int32_t form;          /* CG_FORM_STANDARD or CG_FORM_SINGLE_REDUCTION        */
    int32_t tune_cached;   /* 1: the autotuner reused the shape it chose earlier in
                              this process for a matrix of the same size and
                              row-length profile (no timing at this create)     */
    int32_t col_bits;      /* 16 or 32: column index width the products read      */
    int32_t spmv_nnz_per_lane; /* spmv's own tiling, block size and grid: the       */
    int32_t spmv_block_size;   /* solver's shape if opts gave one, else tile width */
    int32_t spmv_grid;         /* 8, block 512, two workgroups per CU (autotuned   */
                               /* separately when opts->autotune is set)           */
    double spmv_us;        /* autotuner's best spmv time, 0 if not tuned          */
    double iter_us;        /* autotuner's best solver time per iteration, or 0    */
    int32_t spmm_blocks_per_cu; /* workgroups per CU of the multi-column product   */
                                /* (spmm, cg_solve_multi, cg_solve_block): 0 until  */
                                /* first used; timed at first use with autotune     */
    int32_t spmm_pad;
    double spmm_us;        /* autotuner's best 64-column product time, or 0       */
} cg_config;

typedef struct cg_ctx cg_ctx;
typedef struct cg_batch cg_batch;

/* Fill *opts with defaults: Jacobi, no FP32 copy, no autotune, no history. */
void cg_opts_default(cg_opts *opts);

/*
 * Create a solver context for A on the current HIP device (Section IV: the
 * setup step that reads the CSR data and prepares the loop).
 *   A          : the matrix; copied, validated (rowptr monotone, rowptr[0]=0,
 *                rowptr[n]=nnz, 0 <= col < n, nnz < 2^31), then the Jacobi
 *                inverse diagonal is extracted on the device.
 *   opts       : NULL for defaults.
 *   hip_stream : a hipStream_t (NULL = the null stream), e.g. torch's
 *                torch.cuda.current_stream().cuda_stream.
 *   out        : receives the context; free it with cg_destroy.
 * Returns 0, CG_EINVAL, CG_EDIAG, CG_ENOMEM or CG_EHIP.  On error *out is NULL.
 */
int cg_create(const cg_csr *A, const cg_opts *opts, void *hip_stream, cg_ctx **out);

/*
 * Solve A x = b by Jacobi-preconditioned CG (Section IV; tolerance as in the
 * Table I caption).  b and x are device pointers to float64[n]; x holds x0 on
 * entry (zero it for the default start) and the result on exit; x must not
 * alias b.  Stops when the recurrence residual satisfies ||r|| <= tol ||b||
 * and the true residual b - A x confirms it (otherwise r is replaced by the
 * true residual and the loop continues).  maxit <= 0 means n.  ||b|| = 0
 * gives x = 0 and 0 iterations.  Iterations run as two kernels each,
 * launched in hipGraph chunks; every scalar stays on the device.  The call
 * synchronises the context's stream.
 * info may be NULL.  Returns the status (>= 0) or an API error (< 0).
 */
int cg_solve(cg_ctx *ctx, const double *b, double *x, double tol, int32_t maxit, cg_info *info);

/*
 * Mixed-precision solve (FP32 inner Jacobi-PCG, FP64 refinement): repeat
 *   r = b - A x in FP64;  stop if ||r|| <= tol ||b|| (FP64 test);
 *   solve A d = r / ||r|| with FP32 Jacobi-PCG on the FP32 copy of A (FP64
 *     dot products) from d = 0 until its recurrence residual is <= tol_inner;
 *   x += ||r|| d in FP64,
 * at most maxit_outer times (<= 0: 50); each inner solve runs at most
 * maxit_inner iterations (<= 0: n); tol_inner = 0 means 1e-3.  Requires a
 * context created with fp32_copy = 1, else CG_EINVAL.  b, x as in cg_solve.
 * info->iters counts inner iterations, info->outer refinement steps, and
 * info->relres_true is the FP64 ||b - A x|| / ||b|| of the returned x.
 * Returns CG_CONVERGED, CG_MAXIT (outer limit), CG_BREAKDOWN (non-finite
 * residual) or an API error.
 */
int cg_solve_mixed(cg_ctx *ctx, const double *b, double *x, double tol, int32_t maxit_outer,
                   double tol_inner, int32_t maxit_inner, cg_info *info);

/*
 * Mixed precision that keeps the FP64 iteration: the iteration's sparse
 * products stream the FP32 copy of the values (4 instead of 8 bytes per
 * nonzero) in the row-sum-preserving evaluation
 *     (A p)_i ~ sum_j fl32(a_ij) (p_j - p_i) + s_i p_i,   s_i = sum_j a_ij in FP64,
 * while every vector, dot product and scalar stays FP64 (cg_solve's standard
 * form).  The perturbation fl32(a_ij) - a_ij leaves A 1 exact, so the near-
 * constant modes of these systems are not disturbed; the drift of the
 * recurrence residual from b - A x that the rest of it causes is removed by
 * reliable updates (Sleijpen and van der Vorst): whenever the recurrence
 * residual has fallen by the factor drop since the last replacement (0 =
 * 1e-2; 0 < drop < 1), and at the continue-condition, the FP64 true residual
 * either confirms convergence or replaces r, and the iteration continues.
 * Requires fp32_copy.  Same arguments, statuses and info as cg_solve
 * (replacements counts every replaced residual).  Every replacement drains
 * the graph chunk in flight, so unless opts.chunk was set this form launches
 * chunks of at most 8 iterations.
 */
int cg_solve_mixed_matrix(cg_ctx *ctx, const double *b, double *x, double tol, int32_t maxit, double drop,
                          cg_info *info);

/* y = A x (the paper's "DGEMV(sparse)").  Device pointers to float64[n], x != y.
 * Rows are summed in stored order (bitwise the sequential CSR product), with
 * the product's own tiling and grid (cg_config.spmv_*).  Asynchronous on the
 * context's stream.  Returns 0 or an API error. */
int spmv(cg_ctx *ctx, const double *x, double *y);

/*
 * Y = A X for a row-major n x s block (1 <= s <= 64), device pointers,
 * X != Y.  Column j of Y is the sequential CSR product of column j of X (each
 * row summed in stored order).  Asynchronous on the context's stream.
 */
int spmm(cg_ctx *ctx, const double *X, double *Y, int32_t s);

/*
 * Solve A X = B for s right-hand sides (1 <= s <= 64; row-major n x s device
 * blocks; X holds X0 on entry).  Each column runs its own Jacobi-PCG
 * recurrence with cg_solve's stopping rules (continue-condition, true-
 * residual confirmation, replacement); the columns share one sparse product,
 * one update and the scalar steps per iteration.  info, if not NULL, points
 * to s cg_info records (one per column; seconds is the whole call).  Returns
 * CG_CONVERGED if every column converged, else the largest column status
 * (CG_MAXIT, CG_BREAKDOWN), or an API error.  Synchronises the stream.
 */
int cg_solve_multi(cg_ctx *ctx, const double *B, double *X, int32_t s, double tol, int32_t maxit,
                   cg_info *info);

/*
 * Multi-RHS mixed-precision solve: cg_solve_mixed's scheme applied to the
 * columns of B together.  Repeat: R = B - A X in FP64 and the per-column FP64
 * test; for the columns not yet converged, solve A D = R / ||r_j|| with the
 * FP32 multi-RHS Jacobi-PCG on the FP32 copy of A (row-sum-preserving
 * product, FP64 dot products) until each column's recurrence residual is
 * <= tol_inner; X += ||r_j|| D.  At most maxit_outer rounds (<= 0: 50); each
 * inner solve at most maxit_inner iterations (<= 0: n); tol_inner = 0 means
 * 1e-3.  Requires fp32_copy = 1 (else CG_EINVAL).  B, X, s as in
 * cg_solve_multi; info[j].iters counts column j's FP32 iterations,
 * info[j].outer the rounds, info[j].relres_true its FP64 relative residual.
 * Returns CG_CONVERGED if every column converged, else the largest column
 * status (CG_MAXIT, CG_BREAKDOWN for non-finite input), or an API error.
 */
int cg_solve_multi_mixed(cg_ctx *ctx, const double *B, double *X, int32_t s, double tol, int32_t maxit_outer,
                         double tol_inner, int32_t maxit_inner, cg_info *info);

/*
 * Block conjugate gradients for s right-hand sides at once: O'Leary's block
 * method (the paper's CG iteration, Section IV, applied to a block of
 * vectors) in the breakdown-free form of Ji and Li.  Each iteration makes one
 * block product Q = A P of the N x s search block, takes s x s matrices
 * alpha = (P'Q)^-1 P'R and beta = -(P'Q)^-1 Q'Z in place of CG's scalars, and
 * orthonormalises the next search block Z + P beta by three CholeskyQR passes
 * (the first shifted, as Fukaya, Kannan, Nakatsukasa, Zhang and Yamamoto
 * describe; columns scaled to unit norm; columns whose pivot after the
 * shifted pass is <= 1e-14 are dropped as dependent).  The Krylov space grows
 * by up to s directions per iteration, so the columns need fewer iterations
 * than s separate solves; the iterates differ from cg_solve's by design.
 * B and X: device, row-major n x s (leading dimension s), 1 <= s <= 64; X
 * holds X0 on input and the solution on output; B and X must not alias.
 * Stops when every column passes ||b_j - A x_j|| <= tol ||b_j||, tested on
 * the recurrence residuals and confirmed on the true residuals; if a column
 * fails the confirmation the block restarts from the true residuals.
 * maxit <= 0 means n (counted in block products).  info (s entries): iters =
 * block iterations (the same for every column), status, replacements =
 * restarts, outer = rank of the last search block, relres_recur, relres_true
 * (of the returned x_j), seconds.  Columns with b_j = 0 return x_j = 0.
 * Synchronous.  Returns CG_CONVERGED, CG_MAXIT, CG_BREAKDOWN (P'AP not
 * positive definite on the live directions, or a non-finite value), or an
 * API error.
 */
int cg_solve_block(cg_ctx *ctx, const double *B, double *X, int32_t s, double tol, int32_t maxit, cg_info *info);

/*
 * Batched solves: nsys independent SPD systems solved together in one
 * persistent kernel launch (captured in a hipGraph).  systems[s] must be in
 * host memory (mem = CG_MEM_HOST) and is validated like cg_create's input;
 * the systems are copied into one block-diagonal device CSR.  Each system is
 * solved by a team of workgroups sized in proportion to its expected work,
 * with cg_solve's algorithm and stopping rules; its rows are cut into
 * product tiles and each workgroup of the team owns an equal run of them.
 * opts->precond applies to every system; opts->nnz_per_lane picks the tile
 * width (4, 8 or 16 nonzeros per lane, 0 = 16); opts->blocks_per_cu bounds the
 * workgroups per compute unit (0 = the occupancy limit, the most that can be
 * co-resident; larger values are clamped to it); opts->col_bits as for
 * cg_create (the 16-bit form is used only if it fits every system's tiles).
 * Teams wait for each
 * other at bounded barriers, so a device shared with other work while the
 * batch runs can end the solve with CG_ETIMEOUT.  At most one system per
 * co-resident workgroup slot (else CG_EINVAL).
 * Returns 0, CG_EINVAL, CG_EDIAG (some system lacks a positive diagonal),
 * CG_ENOMEM or CG_EHIP.
 */
int cg_batch_create(int32_t nsys, const cg_csr *systems, const cg_opts *opts, void *hip_stream,
                    cg_batch **out);

/*
 * Solve every system: b_cat and x_cat are device vectors holding the systems'
 * right-hand sides / initial guesses concatenated in system order (system s
 * starts at cg_batch_offset(batch, s)); x_cat receives the solutions.  maxit
 * <= 0 means each system's own n.  info, if not NULL, receives nsys records.
 * Returns CG_CONVERGED if all converged, else the largest system status, or
 * CG_ETIMEOUT if a team wait exceeded its limit.  Synchronises the stream.
 */
int cg_batch_solve(cg_batch *batch, const double *b_cat, double *x_cat, double tol, int32_t maxit,
                   cg_info *info);

/* Row offset of system s in the concatenated vectors (s = nsys gives the total). */
int64_t cg_batch_offset(const cg_batch *batch, int32_t s);

/* Workgroups per system (team_sizes[nsys]); returns the total grid. */
int cg_batch_teams(const cg_batch *batch, int32_t *team_sizes);

/* Detail of the last error on this batch ("" if none). */
const char *cg_batch_last_error(const cg_batch *batch);

/* Free the batch.  NULL is ignored. */
void cg_batch_destroy(cg_batch *batch);

/*
 * Dense FP64 products of the learned warm start (proper orthogonal
 * decomposition by the method of snapshots, and decoding coefficients into a
 * start vector).  All pointers are device memory, row-major with the given
 * leading dimensions; the call is asynchronous on hip_stream (NULL = default
 * stream).  Returns 0, CG_EINVAL (NULL pointer, n < 0, a width <= 0, or a
 * leading dimension smaller than its width), CG_ENOMEM or CG_EHIP.
 *
 * dense_gram:  C (ka x kb, row-major, leading dimension kb) = A' B with
 *              A n x ka (lda), B n x kb (ldb).  The n rows are summed in
 *              fixed chunks and the chunk partials in chunk order, so the
 *              result is deterministic.  Uses stream-ordered scratch.
 * dense_gemm:  C (n x m, ldc) = A W with A n x k (lda), W k x m (row-major).
 */
int dense_gram(const double *A, int64_t n, int32_t ka, int64_t lda, const double *B, int32_t kb, int64_t ldb,
               double *C, void *hip_stream);
int dense_gemm(const double *A, int64_t n, int32_t k, int64_t lda, const double *W, int32_t m, double *C,
               int64_t ldc, void *hip_stream);
/* dense_gram_noalloc: dense_gram for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and result (bitwise equal to
 * dense_gram); the chunk partials live in a fixed 32 MiB device buffer that
 * the library holds on each device it runs on until the process ends, and the
 * call allocates nothing.  Limit: ceil(n / 2048) * ka * kb <= 4194304
 * (e.g. ka = kb = 64 up to n = 2097152); larger requests return CG_ESCRATCH
 * before any work is enqueued.  Runs on the current device, which must own
 * hip_stream (else CG_EINVAL).  Every call on a device shares that buffer:
 * calls that overlap on one device (other streams, other threads) race and
 * must be serialised by the caller.  Asynchronous; returns 0, CG_EINVAL,
 * CG_ESCRATCH, CG_EUNSUPPORTED (device index >= 64) or CG_EHIP. */
int dense_gram_noalloc(const double *A, int64_t n, int32_t ka, int64_t lda, const double *B, int32_t kb,
                       int64_t ldb, double *C, void *hip_stream);
/* Decode POD coefficients into start vectors: X (n x nb, row-major) = Phi c'
 * with Phi n x k (ldphi, FP64), coef nb x k (row-major, FP32: the network's
 * output layout) and c_jl = scale[l] * coef_jl + shift[l] in FP64 (scale and
 * shift are k-vectors, either may be NULL: 1 and 0); nb * k <= 4096.  Device
 * memory, asynchronous.  Returns 0, CG_EINVAL or CG_EHIP. */
int pod_decode(const double *Phi, int64_t n, int32_t k, int64_t ldphi, const float *coef, int32_t nb,
               const double *scale, const double *shift, double *X, void *hip_stream);

/*
 * The Q1 hexahedral operator of the finite-element case study (Section IV)
 * on a structured grid, built from the element coefficients on the device:
 * -div(sigma grad u) + c u discretised with trilinear hexahedra on the unit
 * cube, n_edge nodes per edge (N = n_edge^3, h = 1 / (n_edge - 1)), one
 * coefficient per element.  Nodes are numbered x + n y + n^2 z (x fastest),
 * elements the same with n_edge - 1; every node is kept (no boundary rows
 * removed), so the 27-point pattern has (3 n_edge - 2)^3 entries.  Between
 * two nodes that differ in d coordinates an element adds
 * sigma_e h Khat(d) + c h^3 Mhat(d), Khat = (1/3, 0, -1/12, -1/12),
 * Mhat(d) = (1/3)^(3-d) (1/6)^d; a_ij sums this over the elements holding
 * both nodes, in ascending element order.
 * sigma: device FP64 array of (n_edge - 1)^3 element coefficients; c >= 0;
 * 2 <= n_edge and (3 n_edge - 2)^3 < 2^31.  Asynchronous on hip_stream.
 * Returns 0, CG_EINVAL or CG_EHIP.
 *
 * q1_apply:    y = A x without forming A (device x, y of N entries, x != y).
 *              Reads x, sigma and writes y: about 24 N bytes against the
 *              12 nnz + 4 (N + 1) + 16 N of the CSR product.  Each row adds
 *              its 27 products in ascending column order, so the result is
 *              bitwise the sequential product of the matrix q1_assemble
 *              writes.
 * q1_assemble: the same A in CSR: rowptr int32[N + 1], col int32[nnz]
 *              (ascending per row, diagonal included), val FP64[nnz], all
 *              device memory owned by the caller (nnz = (3 n_edge - 2)^3).
 *              The arrays can be passed to cg_create with CG_MEM_DEVICE.
 */
int q1_apply(int32_t n_edge, double c, const double *sigma, const double *x, double *y, void *hip_stream);
int q1_assemble(int32_t n_edge, double c, const double *sigma, int32_t *rowptr, int32_t *col, double *val,
                void *hip_stream);

/*
 * Multilayer perceptron of the learned warm start (maps source parameters to
 * POD coefficients): nlayers affine layers with dims[0..nlayers] widths,
 * SiLU after every hidden layer, linear output, loss = mean squared error
 * sum((Y - T)^2) / (batch * dims[nlayers]), Adam with bias correction.
 * Parameters are one flat FP32 vector, per layer W (dims[l+1] x dims[l],
 * row-major) then b (dims[l+1]).
 * precision 0: FP32 throughout.  precision 1: BF16 weights and hidden
 * activations (round to nearest even from FP32 master weights), products
 * accumulated in FP32, gradients and Adam state FP32.
 * Batches X (batch x dims[0]), T and Y (batch x dims[nlayers]) are FP32,
 * row-major, device memory; 1 <= batch <= max_batch.  Calls are ordered on
 * hip_stream; mlp_forward and mlp_train_step with loss == NULL do not
 * synchronise.  Returns 0, CG_EINVAL, CG_ENOMEM or CG_EHIP.
 */
typedef struct mlp_net mlp_net;
int mlp_create(int32_t nlayers, const int32_t *dims, int32_t precision, int32_t max_batch, void *hip_stream,
               mlp_net **out);
/* Number of parameters (or CG_EINVAL for NULL). */
int64_t mlp_param_count(const mlp_net *net);
/* Load parameters from host memory (FP32, flat order above); resets Adam. */
int mlp_set_params(mlp_net *net, const float *host_params);
/* Copy the FP32 master parameters to host memory. */
int mlp_get_params(mlp_net *net, float *host_params);
/* Y = network(X). */
int mlp_forward(mlp_net *net, const float *X, int32_t batch, float *Y);
/* Gradient of the loss at (X, T) into host memory (flat order, may be NULL);
 * *loss (may be NULL) receives the loss in FP64.  Synchronises the stream. */
int mlp_gradients(mlp_net *net, const float *X, const float *T, int32_t batch, float *host_grads, double *loss);
/* One Adam step on the gradient at (X, T); *loss as in mlp_gradients. */
int mlp_train_step(mlp_net *net, const float *X, const float *T, int32_t batch, float lr, float beta1, float beta2,
                   float eps, double *loss);
/* Free the network.  NULL is ignored. */
void mlp_destroy(mlp_net *net);

/* Copy up to `cap` entries of the last solve's residual history
 * (||r_k|| / ||b||, k = 0..iters) into host memory; returns the count
 * written, or an API error if history was not enabled at create. */
int cg_get_history(cg_ctx *ctx, double *host_out, int32_t cap);

/* The launch shape in use. */
int cg_get_config(cg_ctx *ctx, cg_config *cfg);

/* Free the context and all device memory it owns.  NULL is ignored. */
void cg_destroy(cg_ctx *ctx);

/* Static text for a status or error code. */
const char *cg_strerror(int code);

/* Detail of the last error on this context ("" if none). */
const char *cg_last_error(const cg_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* JPCG_H */
