// The Q1 hexahedral operator of the finite-element case study (Section IV),
// on the structured n^3 grid, computed from the element coefficients on the
// device: a matrix-free product and a device assembly of the same operator
// in CSR.
//
// -div(sigma grad u) + c u with trilinear hexahedra of side h = 1/(n-1), one
// coefficient sigma_e per element.  Between two nodes that differ in d
// coordinates (d = 0..3) an element contributes sigma_e h Khat(d) +
// c h^3 Mhat(d), with Khat = (1/3, 0, -1/12, -1/12) and Mhat(d) =
// (1/3)^(3-d) (1/6)^d (tensor products of the 1-D linear element).  Entry
// a_ij sums these over the elements containing both nodes; node i's 27
// neighbours are the offsets {-1, 0, 1}^3 inside the grid.
//
// Node id = x + n y + n^2 z (x fastest), element id the same with n - 1;
// sigma is an (n-1)^3 FP64 array in element order.  One thread per node (a
// workgroup covers 64 consecutive nodes of an x-line), the 8 surrounding
// coefficients read once per node and the row's 27 entries formed from their
// sub-box sums (q1_row, shared by both kernels); the row's 27 products are
// added in ascending column order (separate multiply and add), the same
// order as the assembled row, so q1_apply equals the sequential product of
// the matrix q1_assemble writes, bit for bit.
#include <cstdint>

#include "context.hpp"

namespace jpcg {

struct Q1Coef {
    double hk[4];   // h Khat(d)
    double chm[4];  // c h^3 Mhat(d)
};

static Q1Coef q1_coef(int n, double c)
{
    const double h = 1.0 / (double)(n - 1);
    const double khat[4] = {1.0 / 3.0, 0.0, -1.0 / 12.0, -1.0 / 12.0};
    const double mhat[4] = {1.0 / 27.0, 1.0 / 54.0, 1.0 / 108.0, 1.0 / 216.0};
    Q1Coef q;
    for (int d = 0; d < 4; ++d) {
        q.hk[d] = h * khat[d];
        q.chm[d] = c * (h * h * h) * mhat[d];
    }
    return q;
}

// Row i's CSR start: rows are z-major, and a node at coordinate t has
// cnt(t) = 3 - [t == 0] - [t == n - 1] neighbours along that axis, so the
// entries before it are C(z) S^2 + cnt(z) (C(y) S + cnt(y) C(x)) with
// S = 3n - 2 and C(t) = sum_{u<t} cnt(u).
__device__ __forceinline__ int q1_cnt(int t, int n) { return 3 - (t == 0) - (t == n - 1); }
__device__ __forceinline__ long long q1_cum(int t, int n) { return t == 0 ? 0 : (t == n ? 3LL * n - 2 : 3LL * t - 1); }

// The 27 entries of node i's row, offset o = 9 (dz + 1) + 3 (dy + 1) + (dx + 1)
// (ascending column order).  Along each axis the neighbour at -1 shares the
// element below the node (slot 0), +1 the one above (slot 1), 0 both; the
// shared elements' coefficient sum and count are sums over a sub-box of the
// 2 x 2 x 2 elements, formed axis by axis once per node, and
// a = h Khat(d) sum(sigma) + c h^3 Mhat(d) count.
__device__ __forceinline__ void q1_row(const double (&sg)[2][2][2], const double (&in)[2][2][2], const Q1Coef& q,
                                       double (&a)[27])
{
#pragma clang fp contract(off)
    double sx[2][2][3], cx[2][2][3];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            sx[u][v][0] = sg[u][v][0];
            sx[u][v][1] = sg[u][v][1];
            sx[u][v][2] = sg[u][v][0] + sg[u][v][1];
            cx[u][v][0] = in[u][v][0];
            cx[u][v][1] = in[u][v][1];
            cx[u][v][2] = in[u][v][0] + in[u][v][1];
        }
    double sy[2][3][3], cy[2][3][3];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            sy[u][0][kx] = sx[u][0][kx];
            sy[u][1][kx] = sx[u][1][kx];
            sy[u][2][kx] = sx[u][0][kx] + sx[u][1][kx];
            cy[u][0][kx] = cx[u][0][kx];
            cy[u][1][kx] = cx[u][1][kx];
            cy[u][2][kx] = cx[u][0][kx] + cx[u][1][kx];
        }
    // Slot choice per offset: -1 -> 0, +1 -> 1, 0 -> 2 (both).
    constexpr int kSlot[3] = {0, 2, 1};
#pragma unroll
    for (int o = 0; o < 27; ++o) {
        const int ix = o % 3, iy = (o / 3) % 3, iz = o / 9;
        const int kx = kSlot[ix], ky = kSlot[iy], kz = kSlot[iz];
        const double ss = kz == 2 ? sy[0][ky][kx] + sy[1][ky][kx] : sy[kz][ky][kx];
        const double cc = kz == 2 ? cy[0][ky][kx] + cy[1][ky][kx] : cy[kz][ky][kx];
        const int d = (ix != 1) + (iy != 1) + (iz != 1);
        a[o] = fma(q.hk[d], ss, q.chm[d] * cc);
    }
}

// Coefficients of the 8 elements around node (x, y, z): sg = sigma (0 outside
// the grid), in = 1 inside, 0 outside.
__device__ __forceinline__ void q1_elements(const double* __restrict__ sigma, int n, int x, int y, int z,
                                            double (&sg)[2][2][2], double (&in)[2][2][2])
{
    const int m = n - 1;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int ez = z - 1 + a, ey = y - 1 + b, ex = x - 1 + e;
                const bool ok = ez >= 0 && ez < m && ey >= 0 && ey < m && ex >= 0 && ex < m;
                sg[a][b][e] = ok ? sigma[((size_t)ez * m + ey) * m + ex] : 0.0;
                in[a][b][e] = ok ? 1.0 : 0.0;
            }
}

// Grid (ceil(n / 64), n, n) of 64-thread workgroups: thread x of workgroup
// (bx, y, z) is node (64 bx + x, y, z), so no index is divided.
constexpr int kQ1X = 64;

__global__ __launch_bounds__(kQ1X) void k_q1_apply(int n, Q1Coef q, const double* __restrict__ sigma,
                                                   const double* __restrict__ xv, double* __restrict__ yv)
{
#pragma clang fp contract(off)
    const int x = blockIdx.x * kQ1X + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= n) return;
    const int nn = n * n;
    const int i = x + n * y + nn * z;
    double sg[2][2][2], in[2][2][2];
    q1_elements(sigma, n, x, y, z, sg, in);
    // Neighbour offsets clamped into the grid (a neighbour outside reads the
    // node itself and its term is selected away), so the 27 loads issue
    // together without branches.
    const int ox[3] = {x > 0 ? -1 : 0, 0, x < n - 1 ? 1 : 0};
    const int oy[3] = {y > 0 ? -n : 0, 0, y < n - 1 ? n : 0};
    const int oz[3] = {z > 0 ? -nn : 0, 0, z < n - 1 ? nn : 0};
    const bool vx[3] = {x > 0, true, x < n - 1}, vy[3] = {y > 0, true, y < n - 1}, vz[3] = {z > 0, true, z < n - 1};
    double xs[27];
#pragma unroll
    for (int o = 0; o < 27; ++o) xs[o] = xv[i + ox[o % 3] + oy[(o / 3) % 3] + oz[o / 9]];
    double a[27];
    q1_row(sg, in, q, a);
    double acc = 0.0;
#pragma unroll
    for (int o = 0; o < 27; ++o) {
        const double t = a[o] * xs[o];
        acc = acc + ((vx[o % 3] && vy[(o / 3) % 3] && vz[o / 9]) ? t : 0.0);
    }
    yv[i] = acc;
}

__global__ __launch_bounds__(kQ1X) void k_q1_assemble(int n, Q1Coef q, const double* __restrict__ sigma,
                                                      int* __restrict__ rowptr, int* __restrict__ col,
                                                      double* __restrict__ val)
{
    const int x = blockIdx.x * kQ1X + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
    if (x >= n) return;
    const int nn = n * n;
    const int i = x + n * y + nn * z;
    const long long S = 3LL * n - 2;
    long long k = q1_cum(z, n) * S * S + q1_cnt(z, n) * (q1_cum(y, n) * S + q1_cnt(y, n) * q1_cum(x, n));
    rowptr[i] = (int)k;
    if (i == n * nn - 1) rowptr[i + 1] = (int)(S * S * S);
    double sg[2][2][2], in[2][2][2];
    q1_elements(sigma, n, x, y, z, sg, in);
    double a[27];
    q1_row(sg, in, q, a);
#pragma unroll
    for (int o = 0; o < 27; ++o) {
        const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
        const int zz = z + dz, yy = y + dy, xx = x + dx;
        if (zz < 0 || zz >= n || yy < 0 || yy >= n || xx < 0 || xx >= n) continue;
        col[k] = i + dx + n * dy + nn * dz;
        val[k] = a[o];
        ++k;
    }
}

static bool q1_size_ok(int n)
{
    if (n < 2) return false;
    const long long S = 3LL * n - 2;
    return S * S * S < (1LL << 31) && (long long)n * n * n < (1LL << 31);
}

}  // namespace jpcg

using namespace jpcg;

extern "C" {

int q1_apply(int32_t n_edge, double c, const double* sigma, const double* x, double* y, void* stream)
{
    if (!sigma || !x || !y || x == y || !jpcg::q1_size_ok(n_edge) || !(c >= 0.0)) return CG_EINVAL;
    try {
        const dim3 grid((n_edge + kQ1X - 1) / kQ1X, n_edge, n_edge);
        k_q1_apply<<<grid, kQ1X, 0, (hipStream_t)stream>>>(n_edge, q1_coef(n_edge, c), sigma, x, y);
        JPCG_HIP(hipGetLastError());
        return 0;
    } catch (const HipError&) {
        return CG_EHIP;
    }
}

int q1_assemble(int32_t n_edge, double c, const double* sigma, int32_t* rowptr, int32_t* col, double* val,
                void* stream)
{
    if (!sigma || !rowptr || !col || !val || !jpcg::q1_size_ok(n_edge) || !(c >= 0.0)) return CG_EINVAL;
    try {
        const dim3 grid((n_edge + kQ1X - 1) / kQ1X, n_edge, n_edge);
        k_q1_assemble<<<grid, kQ1X, 0, (hipStream_t)stream>>>(n_edge, q1_coef(n_edge, c), sigma, rowptr, col, val);
        JPCG_HIP(hipGetLastError());
        return 0;
    } catch (const HipError&) {
        return CG_EHIP;
    }
}

}  // extern "C"
