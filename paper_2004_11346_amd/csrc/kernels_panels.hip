// Panel kernels shared by the plain and the fast ALT paths.
//
// X[task][col][R] holds the coefficients of one (|m|, parity) task as
// R = 4 * batch real right-hand sides per column (column 4f + 2s + c: field f,
// sign s of m, c = re/im); Y[task][row][R] holds half-grid values (row r =
// node 2N-1-r).  pack/scatter move between beta and X, combine/fold between Y
// and the (l, m mod M) grid with the parity split of Section 3.1.2
// (g(x) = E + O, g(-x) = E - O; folding with the weights for the inverse).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "prof.h"

namespace sht {
namespace dev {

namespace {

__device__ __forceinline__ int64_t d_coef_offset(int N, int m) {
    int64_t a = m < 0 ? -(int64_t)m : m;
    int64_t twoN = 2 * (int64_t)N;
    if (a == 0) return 0;
    int64_t off = twoN * (2 * a - 1) - a * (a - 1);
    if (m < 0) off += twoN - a;
    return off;
}

// The coefficient side (beta) and the grid side (g) are the large arrays: the
// thread maps make them contiguous across a wave (consecutive degrees of one
// order, or consecutive orders of one grid row), and put the fields on the
// fastest-varying workgroup index, so that the 32-byte pieces of panel rows
// (4 values per field) written or read by neighbouring workgroups meet in L2.

// beta -> X panels, orders a_lo..a_hi.  grid (ceil(batch / 4), ceil(max_cols / 64),
// orders), block 256 = 4 fields x 64 column pairs.  Thread (f, j) moves the
// degrees k = a + 2j (even task) and a + 2j + 1 (odd task) of orders +a, -a.
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_pack(int N, int batch, int a_lo, const int64_t *__restrict__ x_off,
                                              const B *__restrict__ beta, T *__restrict__ X) {
    const int a = a_lo + blockIdx.z;
    const int f = 4 * blockIdx.x + (threadIdx.x >> 6);
    const int j = 64 * blockIdx.y + (threadIdx.x & 63);
    if (f >= batch) return;
    const int64_t xe = x_off[2 * a], xo = x_off[2 * a + 1];
    const int ce = (int)(xo - xe), co = (int)(x_off[2 * a + 2] - xo);
    if (j >= ce) return;
    const int R = 4 * batch;
    const B *bp = beta + 2 * ((int64_t)f * 4 * N * N + d_coef_offset(N, a) + 2 * j);
    const B *bn = beta + 2 * ((int64_t)f * 4 * N * N + d_coef_offset(N, -a) + 2 * j);
    const bool neg = a > 0;
    T *x0 = X + (xe + j) * R + 4 * f;
    x0[0] = (T)bp[0];
    x0[1] = (T)bp[1];
    x0[2] = neg ? (T)bn[0] : (T)0;
    x0[3] = neg ? (T)bn[1] : (T)0;
    if (j < co) {
        T *x1 = X + (xo + j) * R + 4 * f;
        x1[0] = (T)bp[2];
        x1[1] = (T)bp[3];
        x1[2] = neg ? (T)bn[2] : (T)0;
        x1[3] = neg ? (T)bn[3] : (T)0;
    }
}

// X panels -> beta (transposed direction), same map as k_pack
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_scatter(int N, int batch, int a_lo, const int64_t *__restrict__ x_off,
                                                 const T *__restrict__ X, B *__restrict__ beta) {
    const int a = a_lo + blockIdx.z;
    const int f = 4 * blockIdx.x + (threadIdx.x >> 6);
    const int j = 64 * blockIdx.y + (threadIdx.x & 63);
    if (f >= batch) return;
    const int64_t xe = x_off[2 * a], xo = x_off[2 * a + 1];
    const int ce = (int)(xo - xe), co = (int)(x_off[2 * a + 2] - xo);
    if (j >= ce) return;
    const int R = 4 * batch;
    B *bp = beta + 2 * ((int64_t)f * 4 * N * N + d_coef_offset(N, a) + 2 * j);
    B *bn = beta + 2 * ((int64_t)f * 4 * N * N + d_coef_offset(N, -a) + 2 * j);
    const bool neg = a > 0;
    const T *x0 = X + (xe + j) * R + 4 * f;
    bp[0] = (B)x0[0];
    bp[1] = (B)x0[1];
    if (neg) {
        bn[0] = (B)x0[2];
        bn[1] = (B)x0[3];
    }
    if (j < co) {
        const T *x1 = X + (xo + j) * R + 4 * f;
        bp[2] = (B)x1[0];
        bp[3] = (B)x1[1];
        if (neg) {
            bn[2] = (B)x1[2];
            bn[3] = (B)x1[3];
        }
    }
}

// Y panels -> g columns (parity recombination, Section 3.1.2):
// g(l = 2N-1-r) = E + O, g(l' = r) = E - O.  grid (batch, ceil(orders / 64),
// ceil(N / 4)), block 256 = 4 rows x 64 orders.
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_combine(int N, int M, int batch, int a_lo, int a_hi,
                                                 const T *__restrict__ Y, B *__restrict__ g) {
    const int f = blockIdx.x;
    const int a = a_lo + 64 * blockIdx.y + (threadIdx.x & 63);
    const int r = 4 * blockIdx.z + (threadIdx.x >> 6);
    if (a > a_hi || r >= N) return;
    const int R = 4 * batch, n = 2 * N;
    const T *ye = Y + ((int64_t)(2 * a) * N + r) * R + 4 * f;
    const T *yo = Y + ((int64_t)(2 * a + 1) * N + r) * R + 4 * f;
    T E[4], O[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        E[q] = ye[q];
        O[q] = yo[q];
    }
    B *gb = g + 2 * ((int64_t)f * n * M);
    B *gl = gb + 2 * ((int64_t)(n - 1 - r) * M), *gm = gb + 2 * ((int64_t)r * M);
    gl[2 * a] = (B)(E[0] + O[0]);
    gl[2 * a + 1] = (B)(E[1] + O[1]);
    gm[2 * a] = (B)(E[0] - O[0]);
    gm[2 * a + 1] = (B)(E[1] - O[1]);
    if (a > 0) {
        gl[2 * (M - a)] = (B)(E[2] + O[2]);
        gl[2 * (M - a) + 1] = (B)(E[3] + O[3]);
        gm[2 * (M - a)] = (B)(E[2] - O[2]);
        gm[2 * (M - a) + 1] = (B)(E[3] - O[3]);
    }
}

// g columns -> Y panels: H_even = w (g(l) + g(l')), H_odd = w (g(l) - g(l')).
// grid (ceil(N R / 256), orders), block 256: consecutive threads take
// consecutive panel values, so the panel rows are written whole.
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_fold(int N, int M, int batch, int a_lo, const double *__restrict__ wh,
                                              const B *__restrict__ g, T *__restrict__ Y) {
    const int a = a_lo + blockIdx.y;
    const int R = 4 * batch;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)N * R) return;
    const int r = (int)(e / R), col = (int)(e - (int64_t)r * R);
    const int f = col >> 2, s = (col >> 1) & 1, c = col & 1;
    T u = (T)0, v = (T)0;
    const int n = 2 * N;
    if (!(s == 1 && a == 0)) {
        const int cc = s ? M - a : a;
        const B *gb = g + 2 * ((int64_t)f * n * M);
        u = (T)gb[2 * ((int64_t)(n - 1 - r) * M + cc) + c];
        v = (T)gb[2 * ((int64_t)r * M + cc) + c];
    }
    const T w = wh ? (T)wh[r] : (T)1;
    Y[((int64_t)(2 * a) * N + r) * R + col] = w * (u + v);
    Y[((int64_t)(2 * a + 1) * N + r) * R + col] = w * (u - v);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// dtype: element type of beta / g (0 FP64, 1 FP32); panel64: panels are FP64
// (otherwise they have the element type of beta / g).
hipError_t panel_pack(int dtype, bool panel64, int N, int batch, int a_lo, int a_hi, const int64_t *x_off,
                      int64_t max_cols, const void *beta, void *X, hipStream_t s) {
    prof::Scope ps(s, "k_pack");
    dim3 grid((batch + 3) / 4, (unsigned)((max_cols + 63) / 64), a_hi - a_lo + 1);
    if (dtype == 0)
        hipLaunchKernelGGL((k_pack<double, double>), grid, dim3(256), 0, s, N, batch, a_lo, x_off,
                           (const double *)beta, (double *)X);
    else if (panel64)
        hipLaunchKernelGGL((k_pack<float, double>), grid, dim3(256), 0, s, N, batch, a_lo, x_off, (const float *)beta,
                           (double *)X);
    else
        hipLaunchKernelGGL((k_pack<float, float>), grid, dim3(256), 0, s, N, batch, a_lo, x_off, (const float *)beta,
                           (float *)X);
    return hipGetLastError();
}

hipError_t panel_scatter(int dtype, bool panel64, int N, int batch, int a_lo, int a_hi, const int64_t *x_off,
                         int64_t max_cols, const void *X, void *beta, hipStream_t s) {
    prof::Scope ps(s, "k_scatter");
    dim3 grid((batch + 3) / 4, (unsigned)((max_cols + 63) / 64), a_hi - a_lo + 1);
    if (dtype == 0)
        hipLaunchKernelGGL((k_scatter<double, double>), grid, dim3(256), 0, s, N, batch, a_lo, x_off,
                           (const double *)X, (double *)beta);
    else if (panel64)
        hipLaunchKernelGGL((k_scatter<float, double>), grid, dim3(256), 0, s, N, batch, a_lo, x_off,
                           (const double *)X, (float *)beta);
    else
        hipLaunchKernelGGL((k_scatter<float, float>), grid, dim3(256), 0, s, N, batch, a_lo, x_off,
                           (const float *)X, (float *)beta);
    return hipGetLastError();
}

hipError_t panel_combine(int dtype, bool panel64, int N, int batch, int a_lo, int a_hi, const void *Y, void *g,
                         hipStream_t s) {
    prof::Scope ps(s, "k_combine");
    const int M = 4 * N - 1;
    dim3 grid(batch, (a_hi - a_lo + 64) / 64, (N + 3) / 4);
    if (dtype == 0)
        hipLaunchKernelGGL((k_combine<double, double>), grid, dim3(256), 0, s, N, M, batch, a_lo, a_hi,
                           (const double *)Y, (double *)g);
    else if (panel64)
        hipLaunchKernelGGL((k_combine<float, double>), grid, dim3(256), 0, s, N, M, batch, a_lo, a_hi,
                           (const double *)Y, (float *)g);
    else
        hipLaunchKernelGGL((k_combine<float, float>), grid, dim3(256), 0, s, N, M, batch, a_lo, a_hi, (const float *)Y,
                           (float *)g);
    return hipGetLastError();
}

hipError_t panel_fold(int dtype, bool panel64, int N, int batch, int a_lo, int a_hi, const double *wh,
                      const void *g, void *Y, hipStream_t s) {
    prof::Scope ps(s, "k_fold");
    const int R = 4 * batch, M = 4 * N - 1;
    dim3 grid(blocks_for((int64_t)N * R), a_hi - a_lo + 1);
    if (dtype == 0)
        hipLaunchKernelGGL((k_fold<double, double>), grid, dim3(256), 0, s, N, M, batch, a_lo, wh,
                           (const double *)g, (double *)Y);
    else if (panel64)
        hipLaunchKernelGGL((k_fold<float, double>), grid, dim3(256), 0, s, N, M, batch, a_lo, wh, (const float *)g,
                           (double *)Y);
    else
        hipLaunchKernelGGL((k_fold<float, float>), grid, dim3(256), 0, s, N, M, batch, a_lo, wh, (const float *)g,
                           (float *)Y);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace sht
