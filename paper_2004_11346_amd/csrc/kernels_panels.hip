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

// Every kernel stages a tile in LDS so that both sides move in runs of at
// least 256 bytes: a panel row holds R = 4 batch values (field f at columns
// 4f .. 4f + 3), and the tiles take the fields in chunks of FC = 8 (32 panel
// values, 256 bytes per panel row).
constexpr int FC = 8;
constexpr int kIt = 16;  // tile values per thread: every tile holds 4096 values, 256 threads
// LDS row pitch (doubles) of the pack / scatter tile that keeps a
// half-wave's 64-bit accesses on distinct banks when it reads across the rows
// of 128 complex values (258 doubles = 516 dwords, 4 banks apart)
constexpr int kPS = 258;
static_assert(FC * 2 * 256 == 256 * kIt, "pack / scatter tile: [FC][2][128][2]");
static_assert(2 * 64 * 4 * FC == 256 * kIt, "pack / scatter panel side: 2 parities x 64 rows x 4 FC");
static_assert(2 * 64 * 4 * FC == 256 * kIt, "combine / fold tile: [2][64][4 FC]");
static_assert(FC * 2 * 2 * 64 * 2 == 256 * kIt, "combine / fold grid side: FC x mirror x sign x 64 x re/im");

// beta -> X panels.  grid (ceil(max_cols / 64), orders), block 256.  Tile:
// one order a, column pairs j0 .. j0 + 63 (degrees a + 2j0 .. a + 2j0 + 127 of
// orders +a and -a), FC fields at a time.
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_pack(int N, int batch, int a_lo, const int64_t *__restrict__ x_off,
                                              const B *__restrict__ beta, T *__restrict__ X) {
    __shared__ double tile[FC * 2 * kPS];  // (field, sign) rows of 128 complex values, pitch kPS
    const int a = a_lo + blockIdx.y;
    const int j0 = 64 * blockIdx.x;
    const int64_t xe = x_off[2 * a], xo = x_off[2 * a + 1];
    const int ce = (int)(xo - xe), co = (int)(x_off[2 * a + 2] - xo);
    if (j0 >= ce) return;
    const int R = 4 * batch, n = 2 * N, nk = n - a;  // degrees of order a
    const int k0 = 2 * j0;                           // first degree offset k - a
    const int64_t offp = d_coef_offset(N, a), offn = d_coef_offset(N, -a);
    const int tid = threadIdx.x;
    for (int f0 = 0; f0 < batch; f0 += FC) {
        __syncthreads();
        // read: per (field, sign) 128 consecutive complex values (2 KB); all of
        // a thread's loads are issued before the tile is written
        double v[kIt];
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int fi = e >> 9, sg = (e >> 8) & 1, q = e & 255;  // q: 128 complex x re/im
            const int kk = k0 + (q >> 1), f = f0 + fi;
            v[i] = (f < batch && kk < nk && (sg == 0 || a > 0))
                       ? (double)beta[2 * ((int64_t)f * 4 * N * N + (sg ? offn : offp) + kk) + (q & 1)]
                       : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            tile[(e >> 8) * kPS + (e & 255)] = v[i];
        }
        __syncthreads();
        // write: rows of both parity tasks, 4 FC values each (contiguous runs)
        const int nf = min(FC, batch - f0);
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int par = e / (64 * 4 * FC), rem = e - par * (64 * 4 * FC);
            const int jj = rem / (4 * FC), c = rem - jj * (4 * FC);
            const int fi = c >> 2, sg = (c >> 1) & 1, ri = c & 1;
            const int j = j0 + jj;
            if (fi < nf && j < (par ? co : ce))
                X[((par ? xo : xe) + j) * R + 4 * f0 + c] = (T)tile[(2 * fi + sg) * kPS + 2 * (2 * jj + par) + ri];
        }
    }
}

// X panels -> beta (transposed direction), the same tile read the other way
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_scatter(int N, int batch, int a_lo, const int64_t *__restrict__ x_off,
                                                 const T *__restrict__ X, B *__restrict__ beta) {
    __shared__ double tile[FC * 2 * kPS];
    const int a = a_lo + blockIdx.y;
    const int j0 = 64 * blockIdx.x;
    const int64_t xe = x_off[2 * a], xo = x_off[2 * a + 1];
    const int ce = (int)(xo - xe), co = (int)(x_off[2 * a + 2] - xo);
    if (j0 >= ce) return;
    const int R = 4 * batch, n = 2 * N, nk = n - a;
    const int k0 = 2 * j0;
    const int64_t offp = d_coef_offset(N, a), offn = d_coef_offset(N, -a);
    const int tid = threadIdx.x;
    for (int f0 = 0; f0 < batch; f0 += FC) {
        const int nf = min(FC, batch - f0);
        __syncthreads();
        double v[kIt];
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int par = e / (64 * 4 * FC), rem = e - par * (64 * 4 * FC);
            const int jj = rem / (4 * FC), c = rem - jj * (4 * FC);
            const int j = j0 + jj;
            v[i] = ((c >> 2) < nf && j < (par ? co : ce)) ? (double)X[((par ? xo : xe) + j) * R + 4 * f0 + c] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int par = e / (64 * 4 * FC), rem = e - par * (64 * 4 * FC);
            const int jj = rem / (4 * FC), c = rem - jj * (4 * FC);
            tile[(c >> 1) * kPS + 2 * (2 * jj + par) + (c & 1)] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int fi = e >> 9, sg = (e >> 8) & 1, q = e & 255;
            const int kk = k0 + (q >> 1), f = f0 + fi;
            if (f < batch && kk < nk && (sg == 0 || a > 0))
                beta[2 * ((int64_t)f * 4 * N * N + (sg ? offn : offp) + kk) + (q & 1)] = (B)tile[(e >> 8) * kPS + q];
        }
    }
}

// Y panels -> g columns (parity recombination, Section 3.1.2):
// g(l = 2N-1-r) = E + O, g(l' = r) = E - O.  grid (ceil(orders / 64), N),
// block 256.  Tile: 64 orders x one half-grid row r, FC fields; each grid row
// receives runs of 64 consecutive orders (1 KB) per field and sign.
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_combine(int N, int M, int batch, int a_lo, int a_hi,
                                                 const T *__restrict__ Y, B *__restrict__ g) {
    __shared__ double tile[2][64][4 * FC];  // parity, order, panel value
    const int a0 = a_lo + 64 * blockIdx.x, r = blockIdx.y;
    const int R = 4 * batch, n = 2 * N;
    const int tid = threadIdx.x;
    for (int f0 = 0; f0 < batch; f0 += FC) {
        const int nf = min(FC, batch - f0);
        __syncthreads();
        // read: 128 panel-row pieces of 4 FC values (256 bytes)
        double v[kIt];
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int seg = e / (4 * FC), c = e - seg * (4 * FC);
            const int par = seg >> 6, a = a0 + (seg & 63);
            v[i] = (a <= a_hi && (c >> 2) < nf) ? (double)Y[((int64_t)(2 * a + par) * N + r) * R + 4 * f0 + c] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int seg = e / (4 * FC), c = e - seg * (4 * FC);
            tile[seg >> 6][seg & 63][c] = v[i];
        }
        __syncthreads();
        // write: per (field, mirror row, sign) 64 consecutive orders
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int ri2 = e & 1, ai = (e >> 1) & 63, sg = (e >> 7) & 1, mirror = (e >> 8) & 1, fi = e >> 9;
            const int aj = sg ? 63 - ai : ai, a = a0 + aj;  // mirror 0: node 2N-1-r (E + O), 1: node r (E - O)
            if (fi >= nf || a > a_hi || (sg && a == 0)) continue;
            const int c = 4 * fi + 2 * sg + ri2;
            const double E = tile[0][aj][c], O = tile[1][aj][c];
            const int l = mirror ? r : n - 1 - r, col = sg ? M - a : a;
            g[2 * ((int64_t)(f0 + fi) * n * M + (int64_t)l * M + col) + ri2] = (B)(mirror ? E - O : E + O);
        }
    }
}

// g columns -> Y panels: H_even = w (g(l) + g(l')), H_odd = w (g(l) - g(l')).
// grid (ceil(orders / 64), N), block 256; the tile of k_combine read the
// other way.
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_fold(int N, int M, int batch, int a_lo, int a_hi,
                                              const double *__restrict__ wh, const B *__restrict__ g,
                                              T *__restrict__ Y) {
    __shared__ double tile[2][64][4 * FC];  // mirror (node 2N-1-r, node r), order, value
    const int a0 = a_lo + 64 * blockIdx.x, r = blockIdx.y;
    const int R = 4 * batch, n = 2 * N;
    const int tid = threadIdx.x;
    const double w = wh ? wh[r] : 1.0;
    for (int f0 = 0; f0 < batch; f0 += FC) {
        const int nf = min(FC, batch - f0);
        __syncthreads();
        double v[kIt];
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int ri2 = e & 1, ai = (e >> 1) & 63, sg = (e >> 7) & 1, mirror = (e >> 8) & 1, fi = e >> 9;
            const int a = a0 + (sg ? 63 - ai : ai);
            const int l = mirror ? r : n - 1 - r, col = sg ? M - a : a;
            v[i] = (fi < nf && a <= a_hi && !(sg && a == 0))
                       ? (double)g[2 * ((int64_t)(f0 + fi) * n * M + (int64_t)l * M + col) + ri2]
                       : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int ri2 = e & 1, ai = (e >> 1) & 63, sg = (e >> 7) & 1, mirror = (e >> 8) & 1, fi = e >> 9;
            tile[mirror][sg ? 63 - ai : ai][4 * fi + 2 * sg + ri2] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kIt; ++i) {
            const int e = tid + 256 * i;
            const int seg = e / (4 * FC), c = e - seg * (4 * FC);
            const int par = seg >> 6, ai = seg & 63, a = a0 + ai;
            if (a > a_hi || (c >> 2) >= nf) continue;
            const double u = tile[0][ai][c], v2 = tile[1][ai][c];
            Y[((int64_t)(2 * a + par) * N + r) * R + 4 * f0 + c] = (T)(w * (par ? u - v2 : u + v2));
        }
    }
}

// Direct (untiled) variants for fewer than four fields: one thread per panel
// value, consecutive threads take consecutive panel values.

// beta -> X panels for tasks [t_lo, t_hi] (orders a_lo..a_hi, both parities).
// grid: (ceil(max_cols * R / 256), ntasks), block 256.
template <typename B, typename T>
__global__ __launch_bounds__(256) void k_pack_direct(int N, int batch, int t_lo, const int64_t *__restrict__ x_off,
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
__global__ __launch_bounds__(256) void k_scatter_direct(int N, int batch, int t_lo, const int64_t *__restrict__ x_off,
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
__global__ __launch_bounds__(256) void k_combine_direct(int N, int M, int batch, int a_lo, const T *__restrict__ Y,
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
__global__ __launch_bounds__(256) void k_fold_direct(int N, int M, int batch, int a_lo, const double *__restrict__ wh,
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
    if (batch < 4) {
        const int R = 4 * batch, t_lo = 2 * a_lo, nt = 2 * (a_hi - a_lo + 1);
        dim3 g1(blocks_for(max_cols * R), nt);
        if (dtype == 0)
            hipLaunchKernelGGL((k_pack_direct<double, double>), g1, dim3(256), 0, s, N, batch, t_lo, x_off,
                               (const double *)beta, (double *)X);
        else if (panel64)
            hipLaunchKernelGGL((k_pack_direct<float, double>), g1, dim3(256), 0, s, N, batch, t_lo, x_off,
                               (const float *)beta, (double *)X);
        else
            hipLaunchKernelGGL((k_pack_direct<float, float>), g1, dim3(256), 0, s, N, batch, t_lo, x_off,
                               (const float *)beta, (float *)X);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((max_cols + 63) / 64), a_hi - a_lo + 1);
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
    if (batch < 4) {
        const int R = 4 * batch, t_lo = 2 * a_lo, nt = 2 * (a_hi - a_lo + 1);
        dim3 g1(blocks_for(max_cols * R), nt);
        if (dtype == 0)
            hipLaunchKernelGGL((k_scatter_direct<double, double>), g1, dim3(256), 0, s, N, batch, t_lo, x_off,
                               (const double *)X, (double *)beta);
        else if (panel64)
            hipLaunchKernelGGL((k_scatter_direct<float, double>), g1, dim3(256), 0, s, N, batch, t_lo, x_off,
                               (const double *)X, (float *)beta);
        else
            hipLaunchKernelGGL((k_scatter_direct<float, float>), g1, dim3(256), 0, s, N, batch, t_lo, x_off,
                               (const float *)X, (float *)beta);
        return hipGetLastError();
    }
    dim3 grid((unsigned)((max_cols + 63) / 64), a_hi - a_lo + 1);
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
    if (batch < 4) {
        const int R = 4 * batch, M1 = 4 * N - 1;
        dim3 g1(blocks_for((int64_t)N * R), a_hi - a_lo + 1);
        if (dtype == 0)
            hipLaunchKernelGGL((k_combine_direct<double, double>), g1, dim3(256), 0, s, N, M1, batch, a_lo,
                               (const double *)Y, (double *)g);
        else if (panel64)
            hipLaunchKernelGGL((k_combine_direct<float, double>), g1, dim3(256), 0, s, N, M1, batch, a_lo,
                               (const double *)Y, (float *)g);
        else
            hipLaunchKernelGGL((k_combine_direct<float, float>), g1, dim3(256), 0, s, N, M1, batch, a_lo,
                               (const float *)Y, (float *)g);
        return hipGetLastError();
    }
    const int M = 4 * N - 1;
    dim3 grid((a_hi - a_lo + 64) / 64, N);
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
    if (batch < 4) {
        const int R = 4 * batch, M1 = 4 * N - 1;
        dim3 g1(blocks_for((int64_t)N * R), a_hi - a_lo + 1);
        if (dtype == 0)
            hipLaunchKernelGGL((k_fold_direct<double, double>), g1, dim3(256), 0, s, N, M1, batch, a_lo, wh,
                               (const double *)g, (double *)Y);
        else if (panel64)
            hipLaunchKernelGGL((k_fold_direct<float, double>), g1, dim3(256), 0, s, N, M1, batch, a_lo, wh,
                               (const float *)g, (double *)Y);
        else
            hipLaunchKernelGGL((k_fold_direct<float, float>), g1, dim3(256), 0, s, N, M1, batch, a_lo, wh,
                               (const float *)g, (float *)Y);
        return hipGetLastError();
    }
    const int M = 4 * N - 1;
    dim3 grid((a_hi - a_lo + 64) / 64, N);
    if (dtype == 0)
        hipLaunchKernelGGL((k_fold<double, double>), grid, dim3(256), 0, s, N, M, batch, a_lo, a_hi, wh,
                           (const double *)g, (double *)Y);
    else if (panel64)
        hipLaunchKernelGGL((k_fold<float, double>), grid, dim3(256), 0, s, N, M, batch, a_lo, a_hi, wh, (const float *)g,
                           (double *)Y);
    else
        hipLaunchKernelGGL((k_fold<float, float>), grid, dim3(256), 0, s, N, M, batch, a_lo, a_hi, wh, (const float *)g,
                           (float *)Y);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace sht
