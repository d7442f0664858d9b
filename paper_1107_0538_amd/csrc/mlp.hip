// Multilayer perceptron of the learned warm start: forward, backward and Adam
// on the GPU with hand-written kernels.
//
// Network: hidden layers h = silu(W h_prev + b), linear output, loss =
// sum((Y - T)^2) / (B * out), Adam with bias correction.  W_l is (out x in)
// row-major; batches are (B x features) row-major.  Two precisions:
//   FP32  every operand FP32;
//   BF16  weights and hidden activations held as BF16 copies (FP32 master
//         weights updated by Adam), products accumulated in FP32, gradients
//         FP32.
// The products are one tiled GEMM kernel (64 x 64 output tiles, 16-deep LDS
// stages, 4 x 4 outputs per thread, FP32 accumulation) with optional
// transposed operands and a split of the reduction dimension whose partials
// are summed in fixed order (weight gradients reduce over the batch).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "context.hpp"

namespace jpcg {

using bf16 = uint16_t;

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(bf16 v) { return __uint_as_float((uint32_t)v << 16); }

// Round to nearest even (ties to even), NaN kept quiet.
__device__ __forceinline__ bf16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16)0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16)(u >> 16);
}
template <typename T>
__device__ __forceinline__ T from_f(float v);
template <>
__device__ __forceinline__ float from_f<float>(float v) { return v; }
template <>
__device__ __forceinline__ bf16 from_f<bf16>(float v) { return f2bf(v); }

constexpr int GT = 64, GK = 16;

// C_z (M x N, row-major, ldc) = sum over k in split z of A(m,k) B(k,n).
// A(m,k) = TA ? A[k*lda + m] : A[m*lda + k];  B(k,n) = TB ? B[n*ldb + k] : B[k*ldb + n].
template <typename XA, typename XB, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_mgemm(int M, int N, int K, const XA* __restrict__ A, int lda,
                                               const XB* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
                                               int kchunk)
{
    __shared__ float As[GK][GT + 1];
    __shared__ float Bs[GK][GT + 1];
    const int mb = blockIdx.x * GT, nb = blockIdx.y * GT, z = blockIdx.z;
    const int k_lo = z * kchunk, k_hi = min(K, k_lo + kchunk);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    float acc[4][4] = {};
    for (int k0 = k_lo; k0 < k_hi; k0 += GK) {
        for (int e = threadIdx.x; e < GT * GK; e += 256) {
            const int kk = e / GT, mm = e % GT;
            const int m = mb + mm, k = k0 + kk;
            float av = 0.f;
            if (m < M && k < k_hi) av = to_f(TA ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k]);
            As[kk][mm] = av;
            const int n = nb + mm;
            float bv = 0.f;
            if (n < N && k < k_hi) bv = to_f(TB ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n]);
            Bs[kk][mm] = bv;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            float av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = As[kk][ty * 4 + u];
                bv[u] = Bs[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = __builtin_fmaf(av[u], bv[v], acc[u][v]);
        }
        __syncthreads();
    }
    float* out = C + (size_t)z * M * ldc;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int m = mb + ty * 4 + u;
        if (m >= M) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int n = nb + tx * 4 + v;
            if (n < N) out[(size_t)m * ldc + n] = acc[u][v];
        }
    }
}

__global__ void k_sum_splits(const float* __restrict__ part, int splits, int64_t count, float* __restrict__ out)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < splits; ++z) s += part[(size_t)z * count + e];
        out[e] = s;
    }
}

__device__ __forceinline__ float sigmoidf_(float u) { return 1.f / (1.f + __expf(-u)); }

// U = C + bias (pre-activation, FP32); H = silu(U) (hidden) or U (output).
template <typename TH>
__global__ void k_bias_act(int Bn, int N, const float* __restrict__ C, const float* __restrict__ bias,
                           float* __restrict__ U, TH* __restrict__ H, int act)
{
    const int64_t count = (int64_t)Bn * N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const float u = C[e] + bias[e % N];
        U[e] = u;
        H[e] = from_f<TH>(act ? u * sigmoidf_(u) : u);
    }
}

// D = 2 (Y - T) / (B * m); per-block partial sums of (Y - T)^2.
__global__ void k_mse(int64_t count, const float* __restrict__ Y, const float* __restrict__ T, float scale,
                      float* __restrict__ D, double* __restrict__ loss_part)
{
    __shared__ double red[256];
    double l = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const float d = Y[e] - T[e];
        D[e] = 2.f * d * scale;
        l += (double)d * (double)d;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) s += red[i];
        loss_part[blockIdx.x] = s;
    }
}

// D_out = D_in * silu'(U).
__global__ void k_silu_back(int64_t count, const float* __restrict__ Din, const float* __restrict__ U,
                            float* __restrict__ Dout)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        const float u = U[e], s = sigmoidf_(u);
        Dout[e] = Din[e] * (s * (1.f + u * (1.f - s)));
    }
}

// db[o] = sum over the batch of D[b, o], in batch order.
__global__ void k_colsum(int Bn, int N, const float* __restrict__ D, float* __restrict__ db)
{
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= N) return;
    float s = 0.f;
    for (int b = 0; b < Bn; ++b) s += D[(size_t)b * N + o];
    db[o] = s;
}

// Adam on the FP32 master parameters; refresh the BF16 copies.
__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2,
                       bf16* __restrict__ pb)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        if (pb) pb[i] = f2bf(pi);
    }
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ in, bf16* __restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = f2bf(in[i]);
}

static int grid_for(int64_t count) { return (int)std::min<int64_t>(2048, std::max<int64_t>(1, (count + 255) / 256)); }

}  // namespace jpcg

struct mlp_net {
    hipStream_t stream = nullptr;
    int L = 0;                  // layers
    std::vector<int> dims;      // L + 1
    int precision = 0;          // 0 FP32, 1 BF16
    int max_batch = 0;
    int64_t nparam = 0;
    std::vector<int64_t> woff;  // offset of W_l in the flat parameter vector (b_l follows)
    float* p = nullptr;         // FP32 master parameters
    float* g = nullptr;         // gradients
    float* m = nullptr;         // Adam moments
    float* v = nullptr;
    jpcg::bf16* pb = nullptr;   // BF16 copies (BF16 mode)
    std::vector<void*> H;       // activations per layer input (L + 1): FP32 or BF16 (input and hidden), FP32 output
    std::vector<float*> U;      // pre-activations per layer
    float* D0 = nullptr;        // gradient buffers (max_batch x max width)
    float* D1 = nullptr;
    float* C = nullptr;         // GEMM output / split partials
    size_t c_cap = 0;
    double* loss_part = nullptr;
    double* hloss = nullptr;
    int t = 0;                  // Adam step count
};

namespace jpcg {

static void free_mlp(mlp_net* n)
{
    if (!n) return;
    void* ptrs[] = {n->p, n->g, n->m, n->v, n->pb, n->D0, n->D1, n->C, n->loss_part};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    for (void* q : n->H)
        if (q) (void)hipFree(q);
    for (float* q : n->U)
        if (q) (void)hipFree(q);
    if (n->hloss) (void)hipHostFree(n->hloss);
    delete n;
}

// C = op(A) op(B) with the reduction split in `splits` fixed chunks.
template <typename XA, typename XB, bool TA, bool TB>
static void gemm(mlp_net* n, int M, int N, int K, const XA* A, int lda, const XB* B, int ldb, float* out, int splits)
{
    const int kchunk = (K + splits - 1) / splits;
    splits = (K + kchunk - 1) / kchunk;
    float* dst = splits > 1 ? n->C : out;
    if (splits > 1 && (size_t)splits * M * N > n->c_cap) throw HipError{hipErrorInvalidValue, "gemm scratch"};
    dim3 grid((M + GT - 1) / GT, (N + GT - 1) / GT, splits);
    k_mgemm<XA, XB, TA, TB><<<grid, 256, 0, n->stream>>>(M, N, K, A, lda, B, ldb, dst, N, kchunk);
    JPCG_HIP(hipGetLastError());
    if (splits > 1) {
        const int64_t count = (int64_t)M * N;
        k_sum_splits<<<grid_for(count), 256, 0, n->stream>>>(n->C, splits, count, out);
        JPCG_HIP(hipGetLastError());
    }
}

template <typename TW>
static const TW* weights(mlp_net* n, int l);
template <>
const float* weights<float>(mlp_net* n, int l) { return n->p + n->woff[l]; }
template <>
const bf16* weights<bf16>(mlp_net* n, int l) { return n->pb + n->woff[l]; }

template <typename TW>
static void forward_t(mlp_net* n, const float* X, int Bn, float* Y)
{
    hipStream_t st = n->stream;
    const int64_t in0 = (int64_t)Bn * n->dims[0];
    if constexpr (sizeof(TW) == 2) {
        k_to_bf16<<<grid_for(in0), 256, 0, st>>>(in0, X, (bf16*)n->H[0]);
    } else {
        JPCG_HIP(hipMemcpyAsync(n->H[0], X, sizeof(float) * in0, hipMemcpyDeviceToDevice, st));
    }
    for (int l = 0; l < n->L; ++l) {
        const int in = n->dims[l], out = n->dims[l + 1];
        const bool last = l == n->L - 1;
        gemm<TW, TW, false, true>(n, Bn, out, in, (const TW*)n->H[l], in, weights<TW>(n, l), in, n->C, 1);
        const float* bias = n->p + n->woff[l] + (int64_t)out * in;
        const int64_t count = (int64_t)Bn * out;
        if (last) {
            k_bias_act<float><<<grid_for(count), 256, 0, st>>>(Bn, out, n->C, bias, n->U[l], (float*)n->H[l + 1], 0);
        } else {
            k_bias_act<TW><<<grid_for(count), 256, 0, st>>>(Bn, out, n->C, bias, n->U[l], (TW*)n->H[l + 1], 1);
        }
        JPCG_HIP(hipGetLastError());
    }
    if (Y) {
        JPCG_HIP(hipMemcpyAsync(Y, n->H[n->L], sizeof(float) * (int64_t)Bn * n->dims[n->L], hipMemcpyDeviceToDevice,
                                st));
    }
}

// Forward, loss, and gradients into n->g; returns the loss (host, after sync if want_loss).
template <typename TW>
static double backward_t(mlp_net* n, const float* X, const float* T, int Bn, bool want_loss)
{
    hipStream_t st = n->stream;
    forward_t<TW>(n, X, Bn, nullptr);
    const int L = n->L;
    const int m = n->dims[L];
    const int64_t cnt = (int64_t)Bn * m;
    const int lg = grid_for(cnt);
    k_mse<<<lg, 256, 0, st>>>(cnt, (const float*)n->H[L], T, 1.f / (float)cnt, n->D0, n->loss_part);
    JPCG_HIP(hipGetLastError());
    float* D = n->D0;
    float* Dn = n->D1;
    for (int l = L - 1; l >= 0; --l) {
        const int in = n->dims[l], out = n->dims[l + 1];
        float* gW = n->g + n->woff[l];
        float* gb = gW + (int64_t)out * in;
        // dW = D' H_l (out x in), reduced over the batch in fixed chunks.
        const int splits = std::max(1, std::min(16, Bn / 128));
        gemm<float, TW, true, false>(n, out, in, Bn, D, out, (const TW*)n->H[l], in, gW, splits);
        k_colsum<<<(out + 255) / 256, 256, 0, st>>>(Bn, out, D, gb);
        JPCG_HIP(hipGetLastError());
        if (l > 0) {
            // dH = D W_l (B x in), then through the SiLU of layer l-1.
            gemm<float, TW, false, false>(n, Bn, in, out, D, out, weights<TW>(n, l), in, Dn, 1);
            const int64_t c2 = (int64_t)Bn * in;
            k_silu_back<<<grid_for(c2), 256, 0, st>>>(c2, Dn, n->U[l - 1], Dn);
            JPCG_HIP(hipGetLastError());
            std::swap(D, Dn);
        }
    }
    if (!want_loss) return 0.0;
    JPCG_HIP(hipMemcpyAsync(n->hloss, n->loss_part, sizeof(double) * lg, hipMemcpyDeviceToHost, st));
    JPCG_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (int i = 0; i < lg; ++i) s += n->hloss[i];
    return s / (double)cnt;
}

}  // namespace jpcg

using namespace jpcg;

extern "C" {

int mlp_create(int32_t nlayers, const int32_t* dims, int32_t precision, int32_t max_batch, void* stream,
               mlp_net** out)
{
    if (!out) return CG_EINVAL;
    *out = nullptr;
    if (nlayers < 1 || !dims || (precision != 0 && precision != 1) || max_batch < 1) return CG_EINVAL;
    for (int l = 0; l <= nlayers; ++l)
        if (dims[l] < 1) return CG_EINVAL;
    mlp_net* n = nullptr;
    try {
        n = new mlp_net();
        n->stream = (hipStream_t)stream;
        n->L = nlayers;
        n->dims.assign(dims, dims + nlayers + 1);
        n->precision = precision;
        n->max_batch = max_batch;
        int64_t o = 0;
        int wmax = 0;
        for (int l = 0; l < nlayers; ++l) {
            n->woff.push_back(o);
            o += (int64_t)dims[l] * dims[l + 1] + dims[l + 1];
        }
        for (int l = 0; l <= nlayers; ++l) wmax = std::max(wmax, dims[l]);
        n->nparam = o;
        for (float** q : {&n->p, &n->g, &n->m, &n->v}) JPCG_HIP(hipMalloc((void**)q, sizeof(float) * o));
        JPCG_HIP(hipMemsetAsync(n->p, 0, sizeof(float) * o, n->stream));
        JPCG_HIP(hipMemsetAsync(n->m, 0, sizeof(float) * o, n->stream));
        JPCG_HIP(hipMemsetAsync(n->v, 0, sizeof(float) * o, n->stream));
        if (precision == 1) {
            JPCG_HIP(hipMalloc((void**)&n->pb, sizeof(bf16) * o));
            JPCG_HIP(hipMemsetAsync(n->pb, 0, sizeof(bf16) * o, n->stream));
        }
        const size_t act_bytes = precision == 1 ? sizeof(bf16) : sizeof(float);
        n->H.assign(nlayers + 1, nullptr);
        n->U.assign(nlayers, nullptr);
        for (int l = 0; l <= nlayers; ++l) {
            const size_t eb = l == nlayers ? sizeof(float) : act_bytes;
            JPCG_HIP(hipMalloc(&n->H[l], eb * (size_t)max_batch * dims[l]));
        }
        for (int l = 0; l < nlayers; ++l) JPCG_HIP(hipMalloc((void**)&n->U[l], sizeof(float) * (size_t)max_batch * dims[l + 1]));
        JPCG_HIP(hipMalloc((void**)&n->D0, sizeof(float) * (size_t)max_batch * wmax));
        JPCG_HIP(hipMalloc((void**)&n->D1, sizeof(float) * (size_t)max_batch * wmax));
        n->c_cap = std::max<size_t>((size_t)max_batch * wmax, (size_t)16 * wmax * wmax);
        JPCG_HIP(hipMalloc((void**)&n->C, sizeof(float) * n->c_cap));
        JPCG_HIP(hipMalloc((void**)&n->loss_part, sizeof(double) * 2048));
        JPCG_HIP(hipHostMalloc((void**)&n->hloss, sizeof(double) * 2048, hipHostMallocDefault));
        JPCG_HIP(hipStreamSynchronize(n->stream));
        *out = n;
        return 0;
    } catch (const HipError& e) {
        free_mlp(n);
        return e.code == hipErrorOutOfMemory ? CG_ENOMEM : CG_EHIP;
    } catch (const std::bad_alloc&) {
        free_mlp(n);
        return CG_ENOMEM;
    }
}

int64_t mlp_param_count(const mlp_net* n) { return n ? n->nparam : CG_EINVAL; }

int mlp_set_params(mlp_net* n, const float* host)
{
    if (!n || !host) return CG_EINVAL;
    try {
        JPCG_HIP(hipMemcpyAsync(n->p, host, sizeof(float) * n->nparam, hipMemcpyHostToDevice, n->stream));
        if (n->pb) k_to_bf16<<<grid_for(n->nparam), 256, 0, n->stream>>>(n->nparam, n->p, n->pb);
        JPCG_HIP(hipMemsetAsync(n->m, 0, sizeof(float) * n->nparam, n->stream));
        JPCG_HIP(hipMemsetAsync(n->v, 0, sizeof(float) * n->nparam, n->stream));
        JPCG_HIP(hipStreamSynchronize(n->stream));
        n->t = 0;
        return 0;
    } catch (const HipError&) {
        return CG_EHIP;
    }
}

int mlp_get_params(mlp_net* n, float* host)
{
    if (!n || !host) return CG_EINVAL;
    try {
        JPCG_HIP(hipMemcpyAsync(host, n->p, sizeof(float) * n->nparam, hipMemcpyDeviceToHost, n->stream));
        JPCG_HIP(hipStreamSynchronize(n->stream));
        return 0;
    } catch (const HipError&) {
        return CG_EHIP;
    }
}

int mlp_forward(mlp_net* n, const float* X, int32_t batch, float* Y)
{
    if (!n || !X || !Y || batch < 1 || batch > n->max_batch) return CG_EINVAL;
    try {
        if (n->precision == 1) forward_t<bf16>(n, X, batch, Y);
        else forward_t<float>(n, X, batch, Y);
        return 0;
    } catch (const HipError&) {
        return CG_EHIP;
    }
}

int mlp_gradients(mlp_net* n, const float* X, const float* T, int32_t batch, float* grads_host, double* loss)
{
    if (!n || !X || !T || batch < 1 || batch > n->max_batch) return CG_EINVAL;
    try {
        const double l = n->precision == 1 ? backward_t<bf16>(n, X, T, batch, true)
                                           : backward_t<float>(n, X, T, batch, true);
        if (loss) *loss = l;
        if (grads_host) {
            JPCG_HIP(hipMemcpyAsync(grads_host, n->g, sizeof(float) * n->nparam, hipMemcpyDeviceToHost, n->stream));
            JPCG_HIP(hipStreamSynchronize(n->stream));
        }
        return 0;
    } catch (const HipError&) {
        return CG_EHIP;
    }
}

int mlp_train_step(mlp_net* n, const float* X, const float* T, int32_t batch, float lr, float beta1, float beta2,
                   float eps, double* loss)
{
    if (!n || !X || !T || batch < 1 || batch > n->max_batch || !(lr > 0.f)) return CG_EINVAL;
    try {
        const double l = n->precision == 1 ? backward_t<bf16>(n, X, T, batch, loss != nullptr)
                                           : backward_t<float>(n, X, T, batch, loss != nullptr);
        if (loss) *loss = l;
        n->t += 1;
        const float c1 = 1.f - std::pow(beta1, (float)n->t), c2 = 1.f - std::pow(beta2, (float)n->t);
        k_adam<<<grid_for(n->nparam), 256, 0, n->stream>>>(n->nparam, n->p, n->g, n->m, n->v, lr, beta1, beta2, eps,
                                                           c1, c2, n->pb);
        JPCG_HIP(hipGetLastError());
        return 0;
    } catch (const HipError&) {
        return CG_EHIP;
    }
}

void mlp_destroy(mlp_net* n)
{
    if (!n) return;
    (void)hipStreamSynchronize(n->stream);
    free_mlp(n);
}

}  // extern "C"
