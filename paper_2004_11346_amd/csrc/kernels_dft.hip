// Length-M (M = 4N - 1) DFT along phi for every grid row (Section 1, the phi
// sums of eq. `sht_fft`):
//   synthesis  f[l][j] = sum_{m=-(2N-1)}^{2N-1} g[l][m mod M] e^{i m phi_j},
//              phi_j = 2 pi (j + 1/2) / M,
//   analysis   g[l][m mod M] = scale * sum_j f[l][j] e^{-i m phi_j}.
// The half-sample shift of phi_j becomes a twiddle e^{+-i pi m / M} on the
// order side (with the signed order m), leaving a plain length-M DFT.
//
// Three schedules, chosen per M and element type when the plan is built:
//  * rows in LDS: the row held once in LDS, mixed-radix passes over the prime
//    factors of M (largest first, pairs of 3 as radix 9), the digit-reversed
//    result written back through a position table; rows of at most 4096
//    points with small radices run persistently, two workgroups per CU, each
//    loading the next row into registers during the current row's passes,
//    the others one workgroup per row;
//  * Rader (prime M): with a primitive root g of M, the outputs X_k, k != 0,
//    are x_0 plus a cyclic convolution of length M - 1 of the inputs taken in
//    the order x_{g^q} with the phases w^{g^{-q}}; the convolution runs in LDS
//    as a forward mixed-radix transform of length M - 1, a product with the
//    phases' precomputed spectrum and the reverse passes back to natural
//    order, so a prime row costs O(M log M) instead of M^2 products;
//  * four-step (rows larger than LDS): M = M1 M2, n = M2 n1 + n2,
//    k = k1 + M1 k2: a first kernel takes the length-M1 transforms over n1 for
//    a chunk of n2 and multiplies by w_M^{n2 k1}, a second the length-M2
//    transforms over n2 for a chunk of k1; the intermediate rows go through a
//    grid-sized buffer of the plan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dft_device.h"
#include "kernels.h"
#include "prof.h"

namespace sht {
namespace dev {

namespace {

using namespace dft;

constexpr int kThreads = 512;
constexpr size_t kLds = 160 * 1024;
constexpr int kRaderMaxo = 24;  // generic-pass outputs per thread (M - 1 <= 12288)
constexpr int kSegMaxo = 16;    // four-step: at most 8192 elements per workgroup

// Row pointers of grid row l of field (or field pair) b for the I/O mode of
// dft_row: complex rows at [b][l]; real rows of fields 2b and 2b + 1 (the
// second absent when 2b + 1 >= nreal).
template <typename T, int IO>
struct RowPtrs {
    const T *src = nullptr, *src2 = nullptr;
    T *dst = nullptr, *dst2 = nullptr;
    __device__ RowPtrs(int N, int M, int b, int l, int nreal, const T *in, T *out) {
        const int64_t crow = 2 * (((int64_t)b * 2 * N + l) * M);
        const int64_t r1 = ((int64_t)(2 * b) * 2 * N + l) * M, r2 = r1 + (int64_t)2 * N * M;
        const bool two = 2 * b + 1 < nreal;
        if constexpr (IO == 2) {
            src = in + r1;
            src2 = two ? in + r2 : nullptr;
        } else {
            src = in + crow;
        }
        if constexpr (IO == 1) {
            dst = out + r1;
            dst2 = two ? out + r2 : nullptr;
        } else {
            dst = out + crow;
        }
    }
};

// two 512-thread workgroups per CU (an FP64 row up to about 4900 points fills
// half of the LDS) need at most 128 registers per lane: four waves per SIMD
template <typename C, typename T, int MAXO, int IO>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(MAXO == 0 ? 4 : 1, 8))) void k_dft_rows(int N, int M, Passes ps, const double *__restrict__ tab,
                                                       const int *__restrict__ src_pos, int mode, C scale,
                                                       const T *in, T *out, int nreal) {
    extern __shared__ unsigned char smem_raw[];
    typename V2<C>::t *buf = reinterpret_cast<typename V2<C>::t *>(smem_raw);
    const RowPtrs<T, IO> r(N, M, blockIdx.y, blockIdx.x, nreal, in, out);
    dft_row<C, T, MAXO, IO>(N, M, ps, tab, src_pos, mode, scale, r.src, r.src2, r.dst, r.dst2, buf);
}

// rows whose last pass is a prime radix above 13 taken by Rader's
// convolution (the other passes as in k_dft_rows)
template <typename C, typename T, int MAXO, int IO>
__global__ __launch_bounds__(kThreads) void k_dft_rows_rl(int N, int M, Passes ps, const double *__restrict__ tab,
                                                          const int *__restrict__ src_pos, int mode, C scale,
                                                          const T *in, T *out, int nreal, RaderLast rl) {
    extern __shared__ unsigned char smem_raw[];
    typename V2<C>::t *buf = reinterpret_cast<typename V2<C>::t *>(smem_raw);
    const RowPtrs<T, IO> r(N, M, blockIdx.y, blockIdx.x, nreal, in, out);
    dft_row<C, T, MAXO, IO, true>(N, M, ps, tab, src_pos, mode, scale, r.src, r.src2, r.dst, r.dst2, buf, &rl);
}

// Rows in LDS, persistent: workgroup w takes rows w, w + gridDim.x, ... of
// the flattened (field, l) row list.  Rows of at most kUnroll * kThreads
// points whose first pass has a register butterfly of radix up to 13 and
// whose other passes radices up to 9.  Every thread loads its kUnroll points
// of the next row into registers after the first pass of the current row, so
// the loads are in flight during the remaining passes and the stores (the
// larger butterflies stay out of that stretch, which keeps the registers
// within four waves per SIMD); the output slots of its columns, the same for
// every row, are read once.  Same arithmetic as k_dft_rows.
template <typename C, typename T, int IO>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_dft_rows_pipe(
    int N, int M, Passes ps, const double *__restrict__ tab, const int *__restrict__ src_pos, int mode, C scale,
    const T *in, T *out, int nreal, int nrows) {
    typedef typename V2<C>::t c2;
    extern __shared__ unsigned char smem_raw[];
    c2 *buf = reinterpret_cast<c2 *>(smem_raw);
    double2 *t = reinterpret_cast<double2 *>(buf + M + (M & 1));
    const int twoM = 2 * M, n = 2 * N;
    const C sgn = mode == 0 ? (C)1 : (C)-1;
    constexpr int bd = kThreads;  // the launch's block size
    // column j of this thread, clamped so that every load is in bounds and
    // unconditional (a clamped column is loaded and never stored)
    int sp[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) sp[j] = src_pos[min((int)threadIdx.x + j * bd, M - 1)];
    load_tab(tab, M, t);
    c2 v[kUnroll];
    int row = blockIdx.x;
    {
        const RowPtrs<T, IO> r(N, M, row / n, row % n, nreal, in, out);
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) v[j] = ld_in<C, T, IO>(r.src, r.src2, min((int)threadIdx.x + j * bd, M - 1));
    }
    __syncthreads();  // table
    for (; row < nrows; row += gridDim.x) {
        // the thread index as a value the compiler cannot follow across
        // rows: the per-column phase-table addresses are recomputed for each
        // row instead of being hoisted out of the loop (and spilled)
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = tid + j * bd;
            if (c >= M) continue;
            c2 x = v[j];
            if (mode == 0) {
                const int m = signed_order(c, N, M);
                x = cmul<C>(x, tw<C>(t, m < 0 ? m + twoM : m, (C)1));
            }
            buf[c] = x;
        }
        __syncthreads();
        run_pass_range<C, 13, kThreads>(buf, M, ps, 0, 1, t, M, sgn);
        {
            // the last row of a workgroup loads its own row again (unused)
            const int next = row + (int)gridDim.x < nrows ? row + (int)gridDim.x : row;
            const RowPtrs<T, IO> r(N, M, next / n, next % n, nreal, in, out);
#pragma unroll
            for (int j = 0; j < kUnroll; ++j) v[j] = ld_in<C, T, IO>(r.src, r.src2, min(tid + j * bd, M - 1));
        }
        run_pass_range<C, 9, kThreads>(buf, M, ps, 1, ps.n, t, M, sgn);
        const RowPtrs<T, IO> r(N, M, row / n, row % n, nreal, in, out);
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = tid + j * bd;
            if (c >= M) continue;
            c2 x = buf[sp[j]];
            if (mode == 1) {
                const int m = signed_order(c, N, M);
                int q = m < 0 ? -m : twoM - m;  // e^{-i pi m / M}
                if (q == twoM) q = 0;
                x = cmul<C>(x, tw<C>(t, q, (C)1));
                x.x *= scale;
                x.y *= scale;
            }
            st_out<C, T, IO>(r.dst, r.dst2, c, x);
        }
        __syncthreads();  // every read of buf done before the next row lands
    }
}

// prime M by Rader's convolution
template <typename C, typename T, int IO>
__global__ __launch_bounds__(kThreads) void k_dft_rader(int N, int M, Passes pc, const double *__restrict__ tab,
                                                        const double *__restrict__ ctab, const int *__restrict__ inslot,
                                                        const int *__restrict__ outslot, const C *__restrict__ bspec,
                                                        int mode, C scale, const T *in, T *out, int nreal) {
    typedef typename V2<C>::t c2;
    extern __shared__ unsigned char smem_raw[];
    c2 *buf = reinterpret_cast<c2 *>(smem_raw);
    const int L = M - 1;
    double2 *t = reinterpret_cast<double2 *>(buf + L + (L & 1));  // 16-byte aligned after the row
    double2 *tc = t + tab_entries(M);
    c2 *red = reinterpret_cast<c2 *>(tc + tab_entries(L));  // [kThreads / 64 + 1]
    const RowPtrs<T, IO> r(N, M, blockIdx.y, blockIdx.x, nreal, in, out);
    load_tab(tab, M, t);
    load_tab(ctab, L, tc);
    __syncthreads();
    const int twoM = 2 * M;
    const int bd = blockDim.x;
    // inputs: x_n to slot q with g^q = n (n >= 1); x_0 kept aside; total sum
    c2 sum = c2{(C)0, (C)0};
    for (int c0 = 0; c0 < M; c0 += kUnroll * bd) {
        c2 v[kUnroll];
        int q[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = c0 + threadIdx.x + j * bd;
            if (c < M) {
                v[j] = ld_in<C, T, IO>(r.src, r.src2, c);
                q[j] = inslot[c];
            }
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = c0 + threadIdx.x + j * bd;
            if (c >= M) continue;
            c2 x = v[j];
            if (mode == 0) {
                const int m = signed_order(c, N, M);
                x = cmul<C>(x, tw<C>(t, m < 0 ? m + twoM : m, (C)1));
            }
            sum.x += x.x;
            sum.y += x.y;
            if (c == 0)
                red[kThreads / 64] = x;
            else
                buf[q[j]] = x;
        }
    }
    // X_0 = sum of all inputs
    for (int o = 32; o > 0; o >>= 1) {
        sum.x += __shfl_xor(sum.x, o);
        sum.y += __shfl_xor(sum.y, o);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    // cyclic convolution: forward transform (sign -1), spectrum product,
    // reverse passes (the 1/(M-1) is folded into the spectrum)
    run_passes<C, kRaderMaxo>(buf, L, pc, tc, L, (C)-1);
    const C *bs = bspec + (size_t)(mode == 0 ? 0 : 2 * L);
    for (int c0 = 0; c0 < L; c0 += kUnroll * bd) {
        c2 b[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = c0 + threadIdx.x + j * bd;
            if (c < L) b[j] = reinterpret_cast<const c2 *>(bs)[c];
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = c0 + threadIdx.x + j * bd;
            if (c < L) buf[c] = cmul<C>(buf[c], b[j]);
        }
    }
    __syncthreads();
    run_passes_inv<C, kRaderMaxo>(buf, L, pc, tc, L, (C)-1);
    c2 x0 = red[kThreads / 64];
    c2 X0 = c2{(C)0, (C)0};
    for (int w = 0; w < kThreads / 64; ++w) {
        X0.x += red[w].x;
        X0.y += red[w].y;
    }
    for (int c0 = 0; c0 < M; c0 += kUnroll * bd) {
        int sp[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = c0 + threadIdx.x + j * bd;
            sp[j] = (c < M && c > 0) ? outslot[c] : 0;
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = c0 + threadIdx.x + j * bd;
            if (c >= M) continue;
            c2 x;
            if (c == 0) {
                x = X0;
            } else {
                x = buf[sp[j]];
                x.x += x0.x;
                x.y += x0.y;
            }
            if (mode == 1) {
                const int m = signed_order(c, N, M);
                int qq = m < 0 ? -m : twoM - m;
                if (qq == twoM) qq = 0;
                x = cmul<C>(x, tw<C>(t, qq, (C)1));
                x.x *= scale;
                x.y *= scale;
            }
            st_out<C, T, IO>(r.dst, r.dst2, c, x);
        }
    }
}

// four-step, first kernel: for n2 in [n2_0, n2_0 + cnt), the length-M1
// transforms over n1 of x[M2 n1 + n2] (pre-twiddled for synthesis), times
// w_M^{n2 k1}, written to y[k1 M2 + n2]
template <typename C, typename T, int IO>
__global__ __launch_bounds__(kThreads) void k_dft_4s_a(int N, int M, int M1, int M2, int chunk, Passes ps,
                                                       const double *__restrict__ tab, const int *__restrict__ src_pos,
                                                       int mode, const T *in, T *out, int nreal, RaderLast rl) {
    typedef typename V2<C>::t c2;
    extern __shared__ unsigned char smem_raw[];
    c2 *buf = reinterpret_cast<c2 *>(smem_raw);
    const int n2_0 = blockIdx.x * chunk;
    const int cnt = min(chunk, M2 - n2_0);
    const int total = cnt * M1;
    double2 *t = reinterpret_cast<double2 *>(buf + chunk * M1 + ((chunk * M1) & 1));
    double2 *tc = t + tab_entries(M);
    // input rows in the I/O mode (IO 2: two real rows); output: complex
    // intermediate rows
    const RowPtrs<T, IO == 2 ? 2 : 0> r(N, M, blockIdx.z, blockIdx.y, nreal, in, out);
    const T *src = r.src;
    T *dst = out + 2 * (((int64_t)blockIdx.z * 2 * N + blockIdx.y) * M);
    load_tab(tab, M, t);
    if (rl.R > 0) load_tab(rl.ctab, rl.R - 1, tc);
    __syncthreads();
    const int twoM = 2 * M;
    const C sgn = mode == 0 ? (C)1 : (C)-1;
    const int bd = blockDim.x;
    for (int e0 = 0; e0 < total; e0 += kUnroll * bd) {
        c2 v[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int e = e0 + threadIdx.x + j * bd;
            if (e < total) {
                const int n1 = e / cnt, n2l = e - n1 * cnt;
                v[j] = ld_in<C, T, IO == 2 ? 2 : 0>(src, r.src2, M2 * n1 + n2_0 + n2l);
            }
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int e = e0 + threadIdx.x + j * bd;
            if (e >= total) continue;
            const int n1 = e / cnt, n2l = e - n1 * cnt;
            c2 x = v[j];
            if (mode == 0) {
                const int m = signed_order(M2 * n1 + n2_0 + n2l, N, M);
                x = cmul<C>(x, tw<C>(t, m < 0 ? m + twoM : m, (C)1));
            }
            buf[n2l * M1 + n1] = x;
        }
    }
    __syncthreads();
    if (rl.R > 0) {
        run_passes<C, kSegMaxo>(buf, total, ps, t, M, sgn, ps.n - 1);
        c2 *cbuf = reinterpret_cast<c2 *>(tc + tab_entries(rl.R - 1));
        rader_last<C>(buf, cbuf, cbuf + (chunk * M1 / rl.R) * (rl.R - 1), total, rl, tc, sgn);
    } else {
        run_passes<C, kSegMaxo>(buf, total, ps, t, M, sgn);
    }
    for (int e0 = 0; e0 < total; e0 += kUnroll * bd) {
        int sp[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int e = e0 + threadIdx.x + j * bd;
            sp[j] = e < total ? src_pos[e / cnt] : 0;
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int e = e0 + threadIdx.x + j * bd;
            if (e >= total) continue;
            const int k1 = e / cnt, n2l = e - k1 * cnt;
            const int n2 = n2_0 + n2l;
            c2 x = buf[n2l * M1 + sp[j]];
            x = cmul<C>(x, tw<C>(t, (int)((2 * (int64_t)n2 * k1) % twoM), sgn));
            st<C, T>(dst + 2 * ((int64_t)k1 * M2 + n2), x);
        }
    }
}

// four-step, second kernel: for k1 in [k1_0, k1_0 + cnt), the length-M2
// transforms over n2 of y[k1 M2 + n2], written to X[k1 + M1 k2]
// (post-twiddled and scaled for analysis)
template <typename C, typename T, int IO>
__global__ __launch_bounds__(kThreads) void k_dft_4s_b(int N, int M, int M1, int M2, int chunk, Passes ps,
                                                       const double *__restrict__ tab, const int *__restrict__ src_pos,
                                                       int mode, C scale, const T *in, T *out, int nreal,
                                                       RaderLast rl) {
    typedef typename V2<C>::t c2;
    extern __shared__ unsigned char smem_raw[];
    c2 *buf = reinterpret_cast<c2 *>(smem_raw);
    const int k1_0 = blockIdx.x * chunk;
    const int cnt = min(chunk, M1 - k1_0);
    const int total = cnt * M2;
    double2 *t = reinterpret_cast<double2 *>(buf + chunk * M2 + ((chunk * M2) & 1));
    double2 *tc = t + tab_entries(M);
    // input: complex intermediate rows; output rows in the I/O mode (IO 1:
    // two real rows)
    const T *src = in + 2 * (((int64_t)blockIdx.z * 2 * N + blockIdx.y) * M) + 2 * (int64_t)k1_0 * M2;
    const RowPtrs<T, IO == 1 ? 1 : 0> r(N, M, blockIdx.z, blockIdx.y, nreal, in, out);
    load_tab(tab, M, t);
    if (rl.R > 0) load_tab(rl.ctab, rl.R - 1, tc);
    const int twoM = 2 * M;
    const C sgn = mode == 0 ? (C)1 : (C)-1;
    const int bd = blockDim.x;
    for (int e0 = 0; e0 < total; e0 += kUnroll * bd) {
        c2 v[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int e = e0 + threadIdx.x + j * bd;
            if (e < total) v[j] = ld<C, T>(src + 2 * (int64_t)e);
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int e = e0 + threadIdx.x + j * bd;
            if (e < total) buf[e] = v[j];
        }
    }
    __syncthreads();
    if (rl.R > 0) {
        run_passes<C, kSegMaxo>(buf, total, ps, t, M, sgn, ps.n - 1);
        c2 *cbuf = reinterpret_cast<c2 *>(tc + tab_entries(rl.R - 1));
        rader_last<C>(buf, cbuf, cbuf + (chunk * M2 / rl.R) * (rl.R - 1), total, rl, tc, sgn);
    } else {
        run_passes<C, kSegMaxo>(buf, total, ps, t, M, sgn);
    }
    for (int e0 = 0; e0 < total; e0 += kUnroll * bd) {
        int sp[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int e = e0 + threadIdx.x + j * bd;
            sp[j] = e < total ? src_pos[e / cnt] : 0;
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int e = e0 + threadIdx.x + j * bd;
            if (e >= total) continue;
            const int k2 = e / cnt, k1l = e - k2 * cnt;
            const int k = k1_0 + k1l + M1 * k2;
            c2 x = buf[k1l * M2 + sp[j]];
            if (mode == 1) {
                const int m = signed_order(k, N, M);
                int q = m < 0 ? -m : twoM - m;
                if (q == twoM) q = 0;
                x = cmul<C>(x, tw<C>(t, q, (C)1));
                x.x *= scale;
                x.y *= scale;
            }
            st_out<C, T, IO == 1 ? 1 : 0>(r.dst, r.dst2, k, x);
        }
    }
}

Passes to_passes(int n, const int *R, const int *L) {
    Passes ps;
    ps.n = n;
    for (int i = 0; i < 24; ++i) {
        ps.R[i] = i < n ? R[i] : 0;
        ps.L[i] = i < n ? L[i] : 0;
    }
    return ps;
}

int max_radix(int n, const int *R) {
    int m = 0;
    for (int i = 0; i < n; ++i) m = std::max(m, R[i]);
    return m;
}

// compute units of the current device
int cu_count() {
    static int cus[64] = {0};
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= 64) d = 0;
    if (cus[d] <= 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, d) != hipSuccess || n <= 0) n = 256;
        cus[d] = n;
    }
    return cus[d];
}

// device view of the Rader last pass of pass list i (R = 0: none)
RaderLast rader_last_of(const DftPlan &p, int i) {
    RaderLast r;
    std::memset(&r, 0, sizeof r);
    r.R = p.rl_R[i];
    if (r.R > 0) {
        r.pc = to_passes(p.rl_nrad[i], p.rl_radix[i], p.rl_blen[i]);
        r.ctab = p.rl_ctab[i];
        r.inslot = p.rl_inslot[i];
        r.outslot = p.rl_outslot[i];
        r.bspec = p.rl_bspec[i];
        r.bspecf = p.rl_bspecf[i];
    }
    return r;
}

template <typename C, int IO>
hipError_t set_attrs_io() {
    const void *fns[] = {(const void *)&k_dft_rows_pipe<C, C, IO>,
                         (const void *)&k_dft_rows_rl<C, C, 0, IO>, (const void *)&k_dft_rows_rl<C, C, 8, IO>,
                         (const void *)&k_dft_rows<C, C, 0, IO>,  (const void *)&k_dft_rows<C, C, 8, IO>,
                         (const void *)&k_dft_rows<C, C, 16, IO>, (const void *)&k_dft_rows<C, C, 32, IO>,
                         (const void *)&k_dft_rader<C, C, IO>,    (const void *)&k_dft_4s_a<C, C, IO>,
                         (const void *)&k_dft_4s_b<C, C, IO>};
    for (const void *fn : fns) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename C>
hipError_t set_attrs() {
    static bool done = false;
    if (done) return hipSuccess;
    hipError_t e;
    if ((e = set_attrs_io<C, 0>()) != hipSuccess) return e;
    if ((e = set_attrs_io<C, 1>()) != hipSuccess) return e;
    if ((e = set_attrs_io<C, 2>()) != hipSuccess) return e;
    done = true;
    return hipSuccess;
}

// IO: 0 complex rows; 1 synthesis into real field pairs; 2 analysis of real
// field pairs (see dft_row).  nreal: real fields (IO 1 and 2).
template <typename C, typename T, int IO>
hipError_t launch(const DftPlan &p, int batch, int mode, double scale, const void *in, void *out, int nreal,
                  hipStream_t s) {
    typedef typename V2<C>::t c2;
    hipError_t e = set_attrs<C>();
    if (e != hipSuccess) return e;
    const bool f64 = sizeof(C) == 8;
    const double *tab = p.tab;
    const int M = p.M;
    // LDS: the row (padded to 16 bytes), then FP64 phase tables
    auto row_bytes = [](int64_t n) { return sizeof(c2) * (size_t)(n + (n & 1)); };
    prof::Scope sc(s, mode == 0 ? "k_dft_synthesis" : "k_dft_analysis");
    if (p.kind == kDftRows) {
        const Passes ps = to_passes(p.nrad, p.radix, p.blen);
        const size_t lds = row_bytes(M) + 16 * (size_t)tab_entries(M);
        const int maxr = max_radix(p.nrad, p.radix);
        const dim3 grid(2 * p.N, batch);
#define SHT_ROWS(MX)                                                                                        \
    hipLaunchKernelGGL((k_dft_rows<C, T, MX, IO>), grid, dim3(kThreads), lds, s, p.N, M, ps, tab, p.src_pos, \
                       mode, (C)scale, (const T *)in, (T *)out, nreal)
        const int nrows = 2 * p.N * batch;
        if (nrows <= 0) return hipSuccess;
        if (p.rl_R[0] > 0) {
            // the last pass by Rader's convolution; generic passes before it
            // only for radices above 13 (rows of at most 8 kThreads points)
            const RaderLast rl = rader_last_of(p, 0);
            const size_t lrl = lds + rader_last_lds(M, rl.R, sizeof(c2));
            if (max_radix(p.nrad - 1, p.radix) <= 13)
                hipLaunchKernelGGL((k_dft_rows_rl<C, T, 0, IO>), grid, dim3(kThreads), lrl, s, p.N, M, ps, tab,
                                   p.src_pos, mode, (C)scale, (const T *)in, (T *)out, nreal, rl);
            else
                hipLaunchKernelGGL((k_dft_rows_rl<C, T, 8, IO>), grid, dim3(kThreads), lrl, s, p.N, M, ps, tab,
                                   p.src_pos, mode, (C)scale, (const T *)in, (T *)out, nreal, rl);
            return hipGetLastError();
        }
        bool tail9 = p.nrad >= 1;
        for (int i = 1; i < p.nrad; ++i) tail9 = tail9 && p.radix[i] <= 9;
        if (maxr <= 13 && tail9 && M <= kUnroll * kThreads) {
            // two workgroups per CU (LDS of two FP64 rows of up to 4096 points)
            const int wg = std::min(nrows, 2 * cu_count());
            hipLaunchKernelGGL((k_dft_rows_pipe<C, T, IO>), dim3(wg), dim3(kThreads), lds, s, p.N, M, ps, tab,
                               p.src_pos, mode, (C)scale, (const T *)in, (T *)out, nreal, nrows);
        } else if (maxr <= 13)
            SHT_ROWS(0);
        else if (M <= 8 * kThreads)
            SHT_ROWS(8);
        else if (M <= 16 * kThreads)
            SHT_ROWS(16);
        else
            SHT_ROWS(32);
#undef SHT_ROWS
        return hipGetLastError();
    }
    if (p.kind == kDftRader) {
        const Passes pc = to_passes(p.nrad, p.radix, p.blen);
        const size_t lds = row_bytes(M - 1) + 16 * ((size_t)tab_entries(M) + tab_entries(M - 1)) +
                           sizeof(c2) * (kThreads / 64 + 1);
        hipLaunchKernelGGL((k_dft_rader<C, T, IO>), dim3(2 * p.N, batch), dim3(kThreads), lds, s, p.N, M, pc, tab,
                           p.ctab, p.inslot, p.outslot,
                           f64 ? (const C *)p.bspec : (const C *)p.bspecf, mode, (C)scale, (const T *)in, (T *)out,
                           nreal);
        return hipGetLastError();
    }
    if (p.kind == kDftFourStep) {
        if (!p.scratch) return hipErrorInvalidValue;
        const Passes pa = to_passes(p.nrad, p.radix, p.blen);
        const Passes pb = to_passes(p.nrad2, p.radix2, p.blen2);
        const RaderLast rla = rader_last_of(p, 0), rlb = rader_last_of(p, 1);
        const size_t la = row_bytes((int64_t)p.chunk1 * p.M1) + 16 * (size_t)tab_entries(M) +
                          (rla.R ? rader_last_lds(p.chunk1 * p.M1, rla.R, sizeof(c2)) : 0);
        const size_t lb = row_bytes((int64_t)p.chunk2 * p.M2) + 16 * (size_t)tab_entries(M) +
                          (rlb.R ? rader_last_lds(p.chunk2 * p.M2, rlb.R, sizeof(c2)) : 0);
        T *scr = (T *)p.scratch;
        hipLaunchKernelGGL((k_dft_4s_a<C, T, IO>), dim3((p.M2 + p.chunk1 - 1) / p.chunk1, 2 * p.N, batch),
                           dim3(kThreads), la, s, p.N, M, p.M1, p.M2, p.chunk1, pa, tab, p.src_pos, mode,
                           (const T *)in, scr, nreal, rla);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_dft_4s_b<C, T, IO>), dim3((p.M1 + p.chunk2 - 1) / p.chunk2, 2 * p.N, batch),
                           dim3(kThreads), lb, s, p.N, M, p.M1, p.M2, p.chunk2, pb, tab, p.src_pos2, mode, (C)scale,
                           (const T *)scr, (T *)out, nreal, rlb);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------- host tables

std::vector<int> prime_factors(int m) {
    std::vector<int> f;
    for (int p = 2; (long long)p * p <= m; ++p)
        while (m % p == 0) {
            f.push_back(p);
            m /= p;
        }
    if (m > 1) f.push_back(m);
    return f;
}

// radices (largest first; `last`, a prime factor of L, moved to the end when
// given), block lengths and the slot of every output frequency after the DIF
// passes of length L
void passes_of(int L, std::vector<int> &radix, std::vector<int> &blen, std::vector<int> &src_pos, int last = 0) {
    // prime factors, with pairs of 3 merged into radix-9 passes (one pass
    // and one LDS round trip fewer, and fewer products per point than two
    // radix-3 passes)
    radix.clear();
    int threes = 0;
    bool took_last = false;
    for (int p : prime_factors(L)) {
        if (p == last && !took_last)
            took_last = true;
        else if (p == 3)
            ++threes;
        else
            radix.push_back(p);
    }
    for (; threes >= 2; threes -= 2) radix.push_back(9);
    if (threes) radix.push_back(3);
    std::sort(radix.rbegin(), radix.rend());
    if (took_last) radix.push_back(last);
    blen.clear();
    int len = L;
    for (int R : radix) {
        blen.push_back(len);
        len /= R;
    }
    std::vector<int> freq(L);
    struct Rec {
        static void go(std::vector<int> &f, const std::vector<int> &rs, size_t d, int pos0, int len, int mult,
                       int fb) {
            if (d == rs.size()) {
                f[pos0] = fb;
                return;
            }
            const int R = rs[d], Ls = len / R;
            for (int k2 = 0; k2 < R; ++k2) go(f, rs, d + 1, pos0 + Ls * k2, Ls, mult * R, fb + k2 * mult);
        }
    };
    Rec::go(freq, radix, 0, 0, L, 1, 0);
    src_pos.assign(L, 0);
    for (int i = 0; i < L; ++i) src_pos[freq[i]] = i;
}

// two-level table of e^{i pi r / Mt}: lo[j] = e^{i pi j / Mt} (j < 64),
// hi[j] = e^{i pi 64 j / Mt}
void phase_table(int Mt, std::vector<double> &t, std::vector<float> &tf) {
    const int n = tab_entries(Mt);
    t.assign(2 * (size_t)n, 0.0);
    tf.assign(2 * (size_t)n, 0.0f);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        const long long r = i < 64 ? i : 64LL * (i - 64);
        const long double ph = pi * (long double)(r % (2LL * Mt)) / Mt;
        t[2 * i] = (double)cosl(ph);
        t[2 * i + 1] = (double)sinl(ph);
        tf[2 * i] = (float)cosl(ph);
        tf[2 * i + 1] = (float)sinl(ph);
    }
}

long long powmod(long long b, long long e, long long m) {
    long long r = 1 % m;
    b %= m;
    while (e > 0) {
        if (e & 1) r = r * b % m;
        b = b * b % m;
        e >>= 1;
    }
    return r;
}

int primitive_root(int M) {
    const std::vector<int> f = prime_factors(M - 1);
    for (int g = 2; g < M; ++g) {
        bool ok = true;
        for (int p : f)
            if (powmod(g, (M - 1) / p, M) == 1) {
                ok = false;
                break;
            }
        if (ok) return g;
    }
    return 1;
}

// Rader tables of a prime P: the passes of the convolution length P - 1, the
// phase table of base P - 1, the slot of every input n >= 1 (g^q = n for a
// primitive root g), the convolution slot of every output k >= 1, and the
// spectra of b_q = e^{sgn 2 pi i g^{-q} / P} (sgn = +1, then -1) under the
// sign -1 transform of length P - 1, divided by P - 1, in the digit-reversed
// slots of those passes
void rader_tables(int P, std::vector<int> &radix, std::vector<int> &blen, std::vector<int> &src_pos,
                  std::vector<double> &ctab, std::vector<float> &ctabf, std::vector<int> &inslot,
                  std::vector<int> &outslot, std::vector<double> &bspec, std::vector<float> &bspecf) {
    const int L = P - 1;
    passes_of(L, radix, blen, src_pos);
    phase_table(L, ctab, ctabf);
    const int g = primitive_root(P);
    inslot.assign(P, 0);
    outslot.assign(P, 0);
    std::vector<int> gpow(L);
    long long v = 1;
    for (int q = 0; q < L; ++q) {
        gpow[q] = (int)v;
        inslot[(int)v] = q;
        v = v * g % P;
    }
    for (int k = 1; k < P; ++k) outslot[k] = (L - inslot[k]) % L;
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<long double> cr(L), ci(L);
    for (int j = 0; j < L; ++j) {
        cr[j] = cosl(2 * pi * j / L);
        ci[j] = -sinl(2 * pi * j / L);
    }
    bspec.assign(4 * (size_t)L, 0.0);
    bspecf.assign(4 * (size_t)L, 0.0f);
    for (int si = 0; si < 2; ++si) {
        const long double sgn = si == 0 ? 1.0L : -1.0L;
        std::vector<long double> br(L), bi(L);
        for (int q = 0; q < L; ++q) {
            const int e = gpow[(L - q) % L];  // g^{-q}
            br[q] = cosl(2 * pi * e / P);
            bi[q] = sgn * sinl(2 * pi * e / P);
        }
        for (int j = 0; j < L; ++j) {
            long double sr = 0, sim = 0;
            long long idx = 0;
            for (int q = 0; q < L; ++q) {
                sr += br[q] * cr[idx] - bi[q] * ci[idx];
                sim += br[q] * ci[idx] + bi[q] * cr[idx];
                idx += j;
                if (idx >= L) idx -= L;
            }
            const size_t o = 2 * ((size_t)si * L + src_pos[j]);
            bspec[o] = (double)(sr / L);
            bspec[o + 1] = (double)(sim / L);
            bspecf[o] = (float)(sr / L);
            bspecf[o + 1] = (float)(sim / L);
        }
    }
}

// the largest prime factor P of L with minp <= P <= 4097 whose P - 1 has
// register radices only, or 0.  Smaller primes keep the direct P-term sums of
// the generic pass, which cost less than the convolution's extra passes:
// measured at N = 64 to 4096, in the four-step kernels (thousands of points
// per workgroup) Rader's form wins from 43 on and loses at 17 and 31; in
// rows of a few hundred points it loses at 73 and wins at 89.
constexpr int kRaderLastMin = 41;      // four-step kernels
constexpr int kRaderLastRowsMin = 80;  // rows in LDS
int rader_last_prime(int L, int minp = kRaderLastMin) {
    int best = 0;
    for (int p : prime_factors(L)) {
        if (p < minp || p > 4097 || p <= best) continue;
        bool smooth = true;
        for (int q : prime_factors(p - 1)) smooth = smooth && q <= 13;
        if (smooth) best = p;
    }
    return best;
}

// fill the Rader-last tables of pass list i for prime P
void set_rader_last(DftHost &h, int i, int P) {
    h.rl_R[i] = P;
    rader_tables(P, h.rl_radix[i], h.rl_blen[i], h.rl_src_pos[i], h.rl_ctab[i], h.rl_ctabf[i], h.rl_inslot[i],
                 h.rl_outslot[i], h.rl_bspec[i], h.rl_bspecf[i]);
}

// the largest prime factor of L left to a generic pass (above 13) once
// `rl` (0: none) runs as the Rader last pass
int generic_prime(int L, int rl) {
    int g = 0;
    bool took = false;
    for (int p : prime_factors(L)) {
        if (p == rl && !took) {
            took = true;
            continue;
        }
        if (p > 13) g = std::max(g, p);
    }
    return g;
}

bool fits_rows(int M, size_t elt) {
    const std::vector<int> f = prime_factors(M);
    const int maxp = f.empty() ? 1 : *std::max_element(f.begin(), f.end());
    return elt * ((size_t)M + 1) + 16 * (size_t)tab_entries(M) <= kLds && (maxp <= 13 || M <= 32 * kThreads);
}

bool fits_rader(int M, size_t elt) {
    const std::vector<int> f = prime_factors(M - 1);
    const int maxp = f.empty() ? 1 : *std::max_element(f.begin(), f.end());
    return elt * ((size_t)M + kThreads / 64 + 1) + 16 * ((size_t)tab_entries(M) + tab_entries(M - 1)) <= kLds &&
           (maxp <= 13 || M - 1 <= kRaderMaxo * kThreads);
}

// four-step split with the smallest larger factor whose segments fit
bool four_step_split(int M, size_t elt, int &M1, int &M2, int &c1, int &c2, bool rader_last) {
    int best = -1;
    for (int d = 2; (long long)d * d <= M; ++d) {
        if (M % d) continue;
        const int a = d, b = M / d;
        // each workgroup holds chunk x length <= 8192 elements (the generic
        // pass holds 16 outputs per thread) plus the table
        if (b > 16 * kThreads) continue;
        if (elt * ((size_t)b + 1) + 16 * (size_t)tab_entries(M) > kLds) continue;
        if (best < 0 || b < M / best) best = a;
    }
    if (best < 0) return false;
    M2 = best;  // length of the second pass's transforms
    M1 = M / best;
    // chunks: about 4096 elements (FP64; 8192 FP32) so that two workgroups fit
    // a CU where possible; half that where a Rader last pass needs its
    // convolution buffer beside the rows
    const int p1 = rader_last ? rader_last_prime(M1) : 0, p2 = rader_last ? rader_last_prime(M2) : 0;
    const int target1 = (elt == 16 ? 4096 : 8192) / (p1 ? 2 : 1), target2 = (elt == 16 ? 4096 : 8192) / (p2 ? 2 : 1);
    c1 = std::max(1, std::min(M2, target1 / M1));
    c2 = std::max(1, std::min(M1, target2 / M2));
    auto lds = [&](int c, int Ml, int p) {
        return elt * ((size_t)c * Ml + 1) + 16 * (size_t)tab_entries(M) + (p ? rader_last_lds(c * Ml, p, elt) : 0);
    };
    while (c1 > 1 && lds(c1, M1, p1) > kLds) --c1;
    while (c2 > 1 && lds(c2, M2, p2) > kLds) --c2;
    return lds(c1, M1, p1) <= kLds && lds(c2, M2, p2) <= kLds;
}

}  // namespace

void dft_build(int M, int dtype, DftHost &h, int force, bool rader_last) {
    const size_t elt = dtype == 0 ? 16 : 8;
    h = DftHost();
    h.M = M;
    phase_table(M, h.tab, h.tabf);
    const std::vector<int> pf = prime_factors(M);
    const bool prime = pf.size() == 1 && M > 13;
    // a large prime factor as a last pass of the rows by Rader's convolution
    // where the row, its convolution buffer and the tables fit LDS (rows of at
    // most 8 kThreads points: the generic passes of the others hold 8 outputs
    // per thread)
    int prow = rader_last && !prime ? rader_last_prime(M, kRaderLastRowsMin) : 0;
    if (prow && !(M <= 8 * kThreads &&
                  elt * ((size_t)M + 1) + 16 * (size_t)tab_entries(M) + rader_last_lds(M, prow, elt) <= kLds))
        prow = 0;
    // by length: rows that would keep a generic pass of kRaderLastRowsMin or
    // more (measured: 127 at N = 4096 in FP32) go four-step where its two
    // lengths keep none of kRaderLastMin or more
    bool rows_first = true;
    if (force == 0 && !prime && rader_last && generic_prime(M, prow) >= kRaderLastRowsMin) {
        int M1 = 0, M2 = 0, c1 = 0, c2 = 0;
        if (four_step_split(M, elt, M1, M2, c1, c2, true) &&
            generic_prime(M1, rader_last_prime(M1)) < kRaderLastMin &&
            generic_prime(M2, rader_last_prime(M2)) < kRaderLastMin)
            rows_first = false;
    }
    if (((force == 0 && !prime && rows_first) || force == 1) && fits_rows(M, elt)) {
        h.kind = kDftRows;
        passes_of(M, h.radix, h.blen, h.src_pos, prow);
        if (prow) set_rader_last(h, 0, prow);
        return;
    }
    if ((force == 0 || force == 2) && prime && fits_rader(M, elt)) {
        h.kind = kDftRader;
        rader_tables(M, h.radix, h.blen, h.src_pos, h.ctab, h.ctabf, h.inslot, h.outslot, h.bspec, h.bspecf);
        return;
    }
    int M1 = 0, M2 = 0, c1 = 0, c2 = 0;
    if ((force == 0 || force == 3) && !prime) {
        // with Rader last passes for large prime factors of M1 and M2 where
        // the chunks fit, else the generic passes
        bool rl = rader_last;
        bool ok = four_step_split(M, elt, M1, M2, c1, c2, rl);
        if (!ok && rl) ok = four_step_split(M, elt, M1, M2, c1, c2, rl = false);
        if (ok) {
            h.kind = kDftFourStep;
            h.M1 = M1;
            h.M2 = M2;
            h.chunk1 = c1;
            h.chunk2 = c2;
            const int p1 = rl ? rader_last_prime(M1) : 0, p2 = rl ? rader_last_prime(M2) : 0;
            passes_of(M1, h.radix, h.blen, h.src_pos, p1);
            passes_of(M2, h.radix2, h.blen2, h.src_pos2, p2);
            if (p1) set_rader_last(h, 0, p1);
            if (p2) set_rader_last(h, 1, p2);
            return;
        }
    }
    h.kind = kDftNone;
}

hipError_t dft_init() {
    hipError_t e = set_attrs<double>();
    if (e != hipSuccess) return e;
    return set_attrs<float>();
}

hipError_t dft_synthesis(const DftPlan &p, int dtype, int batch, void *f, hipStream_t s) {
    if (dtype == 0) return launch<double, double, 0>(p, batch, 0, 1.0, f, f, 0, s);
    return launch<float, float, 0>(p, batch, 0, 1.0, f, f, 0, s);
}

hipError_t dft_analysis(const DftPlan &p, int dtype, int batch, double scale, const void *f, void *g,
                        hipStream_t s) {
    if (dtype == 0) return launch<double, double, 0>(p, batch, 1, scale, f, g, 0, s);
    return launch<float, float, 0>(p, batch, 1, scale, f, g, 0, s);
}

hipError_t dft_synthesis_real(const DftPlan &p, int dtype, int pairs, int nreal, const void *z, void *f,
                              hipStream_t s) {
    if (dtype == 0) return launch<double, double, 1>(p, pairs, 0, 1.0, z, f, nreal, s);
    return launch<float, float, 1>(p, pairs, 0, 1.0, z, f, nreal, s);
}

hipError_t dft_analysis_real(const DftPlan &p, int dtype, int pairs, int nreal, double scale, const void *f,
                             void *z, hipStream_t s) {
    if (dtype == 0) return launch<double, double, 2>(p, pairs, 1, scale, f, z, nreal, s);
    return launch<float, float, 2>(p, pairs, 1, scale, f, z, nreal, s);
}

}  // namespace dev
}  // namespace sht
