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

// beta -> X panels for tasks [t_lo, t_hi] (orders a_lo..a_hi, both parities).
// grid: (ceil(max_cols * R / 256), ntasks), block 256.
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_pack(int N, int batch, int t_lo, const int64_t *__restrict__ x_off,
                                              const B *__restrict__ beta, T *__restrict__ X) {
    const int task = t_lo + blockIdx.y;
    const int a = task >> 1, par = task & 1;
    const int64_t rows = x_off[task + 1] - x_off[task];
    const int R = 4 * batch;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= rows * R) return;
    const int j = (int)(e / R), col = (int)(e - (int64_t)j * R);
    const int f = col >> 2, s = (col >> 1) & 1, c = col & 1;
    const int k = a + par + 2 * j;
    T v = (T)0;
    if (!(s == 1 && a == 0)) v = (T)beta[2 * ((int64_t)f * 4 * N * N + d_coef_offset(N, s ? -a : a) + (k - a)) + c];
    X[(x_off[task] + j) * R + col] = v;
}

// X panels -> beta (transposed direction)
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_scatter(int N, int batch, int t_lo, const int64_t *__restrict__ x_off,
                                                 const T *__restrict__ X, B *__restrict__ beta) {
    const int task = t_lo + blockIdx.y;
    const int a = task >> 1, par = task & 1;
    const int64_t rows = x_off[task + 1] - x_off[task];
    const int R = 4 * batch;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= rows * R) return;
    const int j = (int)(e / R), col = (int)(e - (int64_t)j * R);
    const int f = col >> 2, s = (col >> 1) & 1, c = col & 1;
    if (s == 1 && a == 0) return;
    const int k = a + par + 2 * j;
    beta[2 * ((int64_t)f * 4 * N * N + d_coef_offset(N, s ? -a : a) + (k - a)) + c] = (B)X[(x_off[task] + j) * R + col];
}

// Y panels -> g columns (parity recombination, Section 3.1.2):
// g(l = 2N-1-r) = E + O, g(l' = r) = E - O.  grid: (ceil(N * R / 256), orders).
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_combine(int N, int M, int batch, int a_lo, const T *__restrict__ Y,
                                                 B *__restrict__ g) {
    const int a = a_lo + blockIdx.y;
    const int R = 4 * batch;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)N * R) return;
    const int r = (int)(e / R), col = (int)(e - (int64_t)r * R);
    const int f = col >> 2, s = (col >> 1) & 1, c = col & 1;
    if (s == 1 && a == 0) return;
    const T E = Y[((int64_t)(2 * a) * N + r) * R + col];
    const T O = Y[((int64_t)(2 * a + 1) * N + r) * R + col];
    const int n = 2 * N;
    const int cc = s ? M - a : a;
    B *gb = g + 2 * ((int64_t)f * n * M);
    gb[2 * ((int64_t)(n - 1 - r) * M + cc) + c] = (B)(E + O);
    gb[2 * ((int64_t)r * M + cc) + c] = (B)(E - O);
}

// g columns -> Y panels: H_even = w (g(l) + g(l')), H_odd = w (g(l) - g(l')).
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
    const int R = 4 * batch, t_lo = 2 * a_lo, nt = 2 * (a_hi - a_lo + 1);
    dim3 grid(blocks_for(max_cols * R), nt);
    if (dtype == 0)
        hipLaunchKernelGGL((k_pack<double, double>), grid, dim3(256), 0, s, N, batch, t_lo, x_off,
                           (const double *)beta, (double *)X);
    else if (panel64)
        hipLaunchKernelGGL((k_pack<float, double>), grid, dim3(256), 0, s, N, batch, t_lo, x_off, (const float *)beta,
                           (double *)X);
    else
        hipLaunchKernelGGL((k_pack<float, float>), grid, dim3(256), 0, s, N, batch, t_lo, x_off, (const float *)beta,
                           (float *)X);
    return hipGetLastError();
}

hipError_t panel_scatter(int dtype, bool panel64, int N, int batch, int a_lo, int a_hi, const int64_t *x_off,
                         int64_t max_cols, const void *X, void *beta, hipStream_t s) {
    prof::Scope ps(s, "k_scatter");
    const int R = 4 * batch, t_lo = 2 * a_lo, nt = 2 * (a_hi - a_lo + 1);
    dim3 grid(blocks_for(max_cols * R), nt);
    if (dtype == 0)
        hipLaunchKernelGGL((k_scatter<double, double>), grid, dim3(256), 0, s, N, batch, t_lo, x_off,
                           (const double *)X, (double *)beta);
    else if (panel64)
        hipLaunchKernelGGL((k_scatter<float, double>), grid, dim3(256), 0, s, N, batch, t_lo, x_off,
                           (const double *)X, (float *)beta);
    else
        hipLaunchKernelGGL((k_scatter<float, float>), grid, dim3(256), 0, s, N, batch, t_lo, x_off,
                           (const float *)X, (float *)beta);
    return hipGetLastError();
}

hipError_t panel_combine(int dtype, bool panel64, int N, int batch, int a_lo, int a_hi, const void *Y, void *g,
                         hipStream_t s) {
    prof::Scope ps(s, "k_combine");
    const int R = 4 * batch, M = 4 * N - 1;
    dim3 grid(blocks_for((int64_t)N * R), a_hi - a_lo + 1);
    if (dtype == 0)
        hipLaunchKernelGGL((k_combine<double, double>), grid, dim3(256), 0, s, N, M, batch, a_lo,
                           (const double *)Y, (double *)g);
    else if (panel64)
        hipLaunchKernelGGL((k_combine<float, double>), grid, dim3(256), 0, s, N, M, batch, a_lo,
                           (const double *)Y, (float *)g);
    else
        hipLaunchKernelGGL((k_combine<float, float>), grid, dim3(256), 0, s, N, M, batch, a_lo, (const float *)Y,
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
