// Plain (dense) associated Legendre transform on gfx950.
//
// Forward (Section 1, ALT; Section 3.1.1): for every order m and every node
//   g(m, theta_l) = sum_{k=|m|}^{2N-1} beta_{k,m} Pbar_k^{|m|}(x_l),
// evaluated on the N nodes with x > 0 and mirrored with the parity split of
// Section 3.1.2 (g = E + O at x, E - O at -x, E/O the sums over k-|m| even/odd).
// The Legendre values are regenerated in registers by the three-term
// recurrence in k (3 FP64 operations per value); the dense matrices are never
// stored (N^2(2N+1) entries would not fit in HBM at N = 4096).
//
// Lanes are nodes: every lane of a wave walks the same degree k at the same
// time, so the recurrence coefficients and the coefficients beta_{k,+-m} are
// wave-uniform (scalar loads) and each step is a handful of FP64 FMAs.
//
// Values that start below the binary64 range (Pbar_m^m ~ sin^m theta) are
// carried as mantissa * 2^e with a per-lane exponent, rescaled by exact
// powers of two; contributions are mantissa * 2^e (zero once 2^e underflows).
#include <hip/hip_runtime.h>

#include "kernels.h"

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

__device__ __forceinline__ int64_t d_tri_offset(int N, int a) {
    return 2 * (int64_t)N * a - (int64_t)a * (a - 1) / 2;
}

__device__ __forceinline__ double scale_of(int e) {
    return e < -1074 ? 0.0 : ldexp(1.0, e);
}

template <typename T> struct Cplx;
template <> struct Cplx<double> { typedef double2 type; };
template <> struct Cplx<float> { typedef float2 type; };

template <typename T>
__device__ __forceinline__ void ld2(const T *p, double &re, double &im) {
    typedef typename Cplx<T>::type C;
    C v = *reinterpret_cast<const C *>(p);
    re = (double)v.x;
    im = (double)v.y;
}

template <typename T>
__device__ __forceinline__ void st2(T *p, double re, double im) {
    typedef typename Cplx<T>::type C;
    C v;
    v.x = (T)re;
    v.y = (T)im;
    *reinterpret_cast<C *>(p) = v;
}

constexpr double kBig = 0x1p200;
constexpr double kShrink = 0x1p-200;

}  // namespace

// grid: (ceil(N/64), a_hi - a_lo + 1), block 64.  FB fields per pass.
template <typename T, int FB>
__global__ __launch_bounds__(64) void k_alt_dense_fwd(
    int N, int M, int batch, int a_lo, const double *__restrict__ xh,
    const double *__restrict__ dmant, const int *__restrict__ dexp,
    const double *__restrict__ coef, const T *__restrict__ beta, T *__restrict__ g) {
    const int a = a_lo + blockIdx.y;
    const int n = 2 * N;
    const int r = blockIdx.x * 64 + threadIdx.x;
    const bool valid = r < N;
    const int rr = valid ? r : N - 1;
    const double x = xh[rr];
    const double *c = coef + 2 * d_tri_offset(N, a);
    const int64_t offp = d_coef_offset(N, a), offn = d_coef_offset(N, -a);
    const int64_t bstride = 4LL * N * N;   // complex entries per field
    const int64_t gstride = (int64_t)n * M;
    const bool neg = a > 0;

    for (int b0 = 0; b0 < batch; b0 += FB) {
        double Ep[FB][2], Op[FB][2], En[FB][2], On[FB][2];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            Ep[f][0] = Ep[f][1] = Op[f][0] = Op[f][1] = 0.0;
            En[f][0] = En[f][1] = On[f][0] = On[f][1] = 0.0;
        }
        const T *bp[FB];
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            int fb = b0 + f < batch ? b0 + f : batch - 1;
            bp[f] = beta + 2 * (fb * bstride);
        }
        double p1 = dmant[(int64_t)a * N + rr], p0 = 0.0;
        int e = dexp[(int64_t)a * N + rr];
        double sc = scale_of(e);
        // k = a (even part)
        {
            double v = p1 * sc;
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                double br, bi;
                ld2(bp[f] + 2 * offp, br, bi);
                Ep[f][0] = fma(v, br, Ep[f][0]);
                Ep[f][1] = fma(v, bi, Ep[f][1]);
                if (neg) {
                    ld2(bp[f] + 2 * offn, br, bi);
                    En[f][0] = fma(v, br, En[f][0]);
                    En[f][1] = fma(v, bi, En[f][1]);
                }
            }
        }
        for (int k = a + 1; k < n; k += 2) {
            // odd step: k - a odd
            {
                const int j = k - a;
                double p2 = c[2 * j] * (x * p1 - c[2 * j + 1] * p0);
                p0 = p1;
                p1 = p2;
                double v = p1 * sc;
#pragma unroll
                for (int f = 0; f < FB; ++f) {
                    double br, bi;
                    ld2(bp[f] + 2 * (offp + j), br, bi);
                    Op[f][0] = fma(v, br, Op[f][0]);
                    Op[f][1] = fma(v, bi, Op[f][1]);
                    if (neg) {
                        ld2(bp[f] + 2 * (offn + j), br, bi);
                        On[f][0] = fma(v, br, On[f][0]);
                        On[f][1] = fma(v, bi, On[f][1]);
                    }
                }
            }
            if (k + 1 < n) {
                const int j = k + 1 - a;
                double p2 = c[2 * j] * (x * p1 - c[2 * j + 1] * p0);
                p0 = p1;
                p1 = p2;
                double v = p1 * sc;
#pragma unroll
                for (int f = 0; f < FB; ++f) {
                    double br, bi;
                    ld2(bp[f] + 2 * (offp + j), br, bi);
                    Ep[f][0] = fma(v, br, Ep[f][0]);
                    Ep[f][1] = fma(v, bi, Ep[f][1]);
                    if (neg) {
                        ld2(bp[f] + 2 * (offn + j), br, bi);
                        En[f][0] = fma(v, br, En[f][0]);
                        En[f][1] = fma(v, bi, En[f][1]);
                    }
                }
            }
            if (fabs(p1) > kBig) {
                p0 *= kShrink;
                p1 *= kShrink;
                e += 200;
                sc = scale_of(e);
            }
        }
        if (valid) {
            const int l = n - 1 - r, lm = r;  // x_l > 0, x_lm = -x_l
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                if (b0 + f >= batch) break;
                T *gb = g + 2 * ((b0 + f) * gstride);
                st2(gb + 2 * ((int64_t)l * M + a), Ep[f][0] + Op[f][0], Ep[f][1] + Op[f][1]);
                st2(gb + 2 * ((int64_t)lm * M + a), Ep[f][0] - Op[f][0], Ep[f][1] - Op[f][1]);
                if (neg) {
                    st2(gb + 2 * ((int64_t)l * M + (M - a)), En[f][0] + On[f][0], En[f][1] + On[f][1]);
                    st2(gb + 2 * ((int64_t)lm * M + (M - a)), En[f][0] - On[f][0], En[f][1] - On[f][1]);
                }
            }
        }
    }
}

// Fold for the transposed ALT (Section 3.1.1 with the parity split of
// Section 3.1.2): for order a, half-grid node r (l = 2N-1-r, mirror l' = r),
//   H[a][0][r][col] = w_r (g(l) + g(l'))   (even k - a)
//   H[a][1][r][col] = w_r (g(l) - g(l'))   (odd  k - a)
// col = 4 f + 2 s + c: field f, sign s (0: +a, 1: -a), c (0 re, 1 im).
// With w == nullptr the weights are 1 (adjoint).  H is FP64 (dense path) or T.
// grid: (ceil(N/64), a_hi - a_lo + 1), block 64.
template <typename T, typename H>
__global__ __launch_bounds__(64) void k_fold(int N, int M, int batch, int a_lo,
                                             const double *__restrict__ wh,
                                             const T *__restrict__ g, H *__restrict__ hbuf,
                                             int64_t hbuf_order_stride, const int64_t *__restrict__ horder_off) {
    const int a = a_lo + blockIdx.y;
    const int r = blockIdx.x * 64 + threadIdx.x;
    if (r >= N) return;
    const int n = 2 * N, R = 4 * batch;
    const int l = n - 1 - r, lm = r;
    const double w = wh ? wh[r] : 1.0;
    const int64_t gstride = (int64_t)n * M;
    H *he = hbuf + (horder_off ? horder_off[a] : (int64_t)(a - a_lo) * hbuf_order_stride);
    H *ho = he + (int64_t)N * R;
    for (int f = 0; f < batch; ++f) {
        const T *gb = g + 2 * (f * gstride);
        for (int s = 0; s < 2; ++s) {
            double ur, ui, vr, vi;
            if (s == 1 && a == 0) {
                ur = ui = vr = vi = 0.0;
            } else {
                int col = s ? M - a : a;
                ld2(gb + 2 * ((int64_t)l * M + col), ur, ui);
                ld2(gb + 2 * ((int64_t)lm * M + col), vr, vi);
            }
            int c0 = 4 * f + 2 * s;
            he[(int64_t)r * R + c0] = (H)(w * (ur + vr));
            he[(int64_t)r * R + c0 + 1] = (H)(w * (ui + vi));
            ho[(int64_t)r * R + c0] = (H)(w * (ur - vr));
            ho[(int64_t)r * R + c0 + 1] = (H)(w * (ui - vi));
        }
    }
}

// Transposed dense ALT with FP64 MFMA (v_mfma_f64_16x16x4f64):
//   beta_{k, +-a} = sum_r Pbar_k^a(x_r) H[a][par(k)][r][col]
// (Section 3.1.1, B = A^T W with W folded into H).  The sum over nodes is the
// MFMA reduction dimension (4 nodes per instruction); 16 degrees of one
// parity form the rows of a tile and the 16 columns are (field, sign, re/im).
// The lanes first run the recurrence with lane = node for 32 consecutive
// degrees and park the values in LDS split by parity; the MFMA A operands are
// read back from there transposed.  The recurrence state of every 64-node
// group of the chunk lives in LDS between degree tiles.
//
// grid: (nchunks, a_hi - a_lo + 1), block 64 (one wave).  A chunk is up to
// kMaxGroups groups of 64 nodes.  With one chunk the result goes to beta
// directly; otherwise to part[chunk][tri(a) + k - a][R], summed by
// k_reduce_chunks.
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kMaxGroups = 16;

template <typename T, int CB>
__global__ __launch_bounds__(64) void k_alt_dense_adj(
    int N, int M, int batch, int a_lo, const double *__restrict__ xh,
    const double *__restrict__ dmant, const int *__restrict__ dexp,
    const double *__restrict__ coef, const double *__restrict__ hbuf,
    int64_t hbuf_order_stride, T *__restrict__ beta, double *__restrict__ part, int nchunks) {
    constexpr int PAD = 18;  // row stride (doubles) of the LDS tiles
    __shared__ double tileE[64 * PAD];
    __shared__ double tileO[64 * PAD];
    __shared__ double st_p0[kMaxGroups * 64];
    __shared__ double st_p1[kMaxGroups * 64];
    __shared__ int st_e[kMaxGroups * 64];
    const int a = a_lo + blockIdx.y;
    const int chunk = blockIdx.x;
    const int n = 2 * N, R = 4 * batch;
    const int lane = threadIdx.x;
    const double *c = coef + 2 * d_tri_offset(N, a);
    const double *hE = hbuf + (int64_t)(a - a_lo) * hbuf_order_stride;
    const double *hO = hE + (int64_t)N * R;
    const int G = (N + 63) / 64;
    const int g_begin = chunk * kMaxGroups;
    const int ng = min(G - g_begin, kMaxGroups);
    const int nk = n - a;  // number of degrees of this order

    for (int gi = 0; gi < ng; ++gi) {
        int r = (g_begin + gi) * 64 + lane;
        bool ok = r < N;
        int rr = ok ? r : 0;
        st_p1[gi * 64 + lane] = ok ? dmant[(int64_t)a * N + rr] : 0.0;
        st_p0[gi * 64 + lane] = 0.0;
        st_e[gi * 64 + lane] = ok ? dexp[(int64_t)a * N + rr] : -4000;
    }

    for (int kt = 0; kt < nk; kt += 32) {
        d4 accE[CB], accO[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            accE[cb] = d4{0.0, 0.0, 0.0, 0.0};
            accO[cb] = d4{0.0, 0.0, 0.0, 0.0};
        }
        for (int gi = 0; gi < ng; ++gi) {
            const int grp = g_begin + gi;
            const int r = grp * 64 + lane;
            const double x = xh[r < N ? r : 0];
            double p0 = st_p0[gi * 64 + lane], p1 = st_p1[gi * 64 + lane];
            int e = st_e[gi * 64 + lane];
            double sc = scale_of(e);
            __syncthreads();  // previous MFMA reads of the tiles are done
            for (int j = 0; j < 32; ++j) {
                const int kk = kt + j;  // k - a
                double v = 0.0;
                if (kk < nk) {
                    if (kk > 0) {
                        double p2 = c[2 * kk] * (x * p1 - c[2 * kk + 1] * p0);
                        p0 = p1;
                        p1 = p2;
                        if (fabs(p1) > kBig) {
                            p0 *= kShrink;
                            p1 *= kShrink;
                            e += 200;
                            sc = scale_of(e);
                        }
                    }
                    v = p1 * sc;
                }
                if (j & 1)
                    tileO[lane * PAD + (j >> 1)] = v;
                else
                    tileE[lane * PAD + (j >> 1)] = v;
            }
            st_p0[gi * 64 + lane] = p0;
            st_p1[gi * 64 + lane] = p1;
            st_e[gi * 64 + lane] = e;
            __syncthreads();
            // A: rows = 16 degrees (lane % 16), K = 4 nodes (lane / 16)
#pragma unroll 4
            for (int s = 0; s < 16; ++s) {
                const int nig = 4 * s + (lane >> 4);
                const int node = grp * 64 + nig;
                const double aE = tileE[nig * PAD + (lane & 15)];
                const double aO = tileO[nig * PAD + (lane & 15)];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int col = cb * 16 + (lane & 15);
                    const bool okb = node < N && col < R;
                    const double bE = okb ? hE[(int64_t)node * R + col] : 0.0;
                    const double bO = okb ? hO[(int64_t)node * R + col] : 0.0;
                    accE[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aE, bE, accE[cb], 0, 0, 0);
                    accO[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aO, bO, accO[cb], 0, 0, 0);
                }
            }
        }
        // D layout (gfx950): element i of lane l is row l/16 + 4 i, column l%16
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int col = cb * 16 + (lane & 15);
            if (col >= R) continue;
            const int f = col >> 2, s = (col >> 1) & 1, cc = col & 1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = (lane >> 4) + 4 * i;
#pragma unroll
                for (int par = 0; par < 2; ++par) {
                    const int kk = kt + 2 * row + par;
                    if (kk >= nk) continue;
                    const double val = par ? accO[cb][i] : accE[cb][i];
                    if (nchunks == 1) {
                        if (s == 1 && a == 0) continue;
                        int64_t o = (int64_t)f * 4LL * N * N + d_coef_offset(N, s ? -a : a) + kk;
                        beta[2 * o + cc] = (T)val;
                    } else {
                        int64_t tri_total = (int64_t)N * (2 * N + 1);
                        int64_t o = ((int64_t)chunk * tri_total + d_tri_offset(N, a) + kk) * R + col;
                        part[o] = val;
                    }
                }
            }
        }
    }
}

// Sum the chunk partials of k_alt_dense_adj and scatter to beta (type T).
// grid: (ceil(R * (2N - a_lo) / 256), orders), block 256.
template <typename T>
__global__ __launch_bounds__(256) void k_reduce_chunks(int N, int batch, int a_lo, int nchunks,
                                                       const double *__restrict__ part,
                                                       T *__restrict__ beta) {
    const int a = a_lo + blockIdx.y;
    const int R = 4 * batch;
    const int nk = 2 * N - a;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)nk * R) return;
    const int kk = (int)(idx / R), col = (int)(idx % R);
    const int f = col >> 2, s = (col >> 1) & 1, cc = col & 1;
    if (s == 1 && a == 0) return;
    const int64_t tri_total = (int64_t)N * (2 * N + 1);
    double acc = 0.0;
    for (int ch = 0; ch < nchunks; ++ch)
        acc += part[((int64_t)ch * tri_total + d_tri_offset(N, a) + kk) * R + col];
    int64_t o = (int64_t)f * 4LL * N * N + d_coef_offset(N, s ? -a : a) + kk;
    beta[2 * o + cc] = (T)acc;
}

// ------------------------------------------------------------- launchers
template <typename T>
static hipError_t launch_fwd(const DenseTables &t, int batch, int a_lo, int a_hi,
                             const void *beta, void *g, hipStream_t s) {
    dim3 grid((t.N + 63) / 64, a_hi - a_lo + 1);
    const T *b = (const T *)beta;
    T *gg = (T *)g;
    if (batch >= 4)
        hipLaunchKernelGGL((k_alt_dense_fwd<T, 4>), grid, dim3(64), 0, s, t.N, t.M, batch, a_lo, t.xh,
                           t.dmant, t.dexp, t.coef, b, gg);
    else if (batch == 3)
        hipLaunchKernelGGL((k_alt_dense_fwd<T, 3>), grid, dim3(64), 0, s, t.N, t.M, batch, a_lo, t.xh,
                           t.dmant, t.dexp, t.coef, b, gg);
    else if (batch == 2)
        hipLaunchKernelGGL((k_alt_dense_fwd<T, 2>), grid, dim3(64), 0, s, t.N, t.M, batch, a_lo, t.xh,
                           t.dmant, t.dexp, t.coef, b, gg);
    else
        hipLaunchKernelGGL((k_alt_dense_fwd<T, 1>), grid, dim3(64), 0, s, t.N, t.M, batch, a_lo, t.xh,
                           t.dmant, t.dexp, t.coef, b, gg);
    return hipGetLastError();
}

hipError_t alt_dense_forward(const DenseTables &t, int dtype, int batch, int a_lo, int a_hi,
                             const void *beta, void *g, hipStream_t s) {
    if (dtype == 0) return launch_fwd<double>(t, batch, a_lo, a_hi, beta, g, s);
    return launch_fwd<float>(t, batch, a_lo, a_hi, beta, g, s);
}

template <typename T, int CB>
static void launch_adj_cb(const DenseTables &t, int batch, int a_lo, int norders, const double *hbuf,
                          int64_t hstride, T *beta, double *part, int nchunks, hipStream_t s) {
    hipLaunchKernelGGL((k_alt_dense_adj<T, CB>), dim3(nchunks, norders), dim3(64), 0, s, t.N, t.M, batch,
                       a_lo, t.xh, t.dmant, t.dexp, t.coef, hbuf, hstride, beta, part, nchunks);
}

template <typename T>
static hipError_t launch_adj(const DenseTables &t, int batch, int a_lo, int a_hi, bool weights,
                             const void *g, void *beta, double *hbuf, double *part, hipStream_t s) {
    const int N = t.N, R = 4 * batch;
    const int norders = a_hi - a_lo + 1;
    const int64_t hstride = 2LL * N * R;
    dim3 grid_f((N + 63) / 64, norders);
    hipLaunchKernelGGL((k_fold<T, double>), grid_f, dim3(64), 0, s, N, t.M, batch, a_lo,
                       weights ? t.wh : (const double *)nullptr, (const T *)g, hbuf, hstride,
                       (const int64_t *)nullptr);
    const int G = (N + 63) / 64;
    const int nchunks = (G + kMaxGroups - 1) / kMaxGroups;
    const int cb = (R + 15) / 16;
    T *b = (T *)beta;
    switch (cb) {
        case 1: launch_adj_cb<T, 1>(t, batch, a_lo, norders, hbuf, hstride, b, part, nchunks, s); break;
        case 2: launch_adj_cb<T, 2>(t, batch, a_lo, norders, hbuf, hstride, b, part, nchunks, s); break;
        case 3:
        case 4: launch_adj_cb<T, 4>(t, batch, a_lo, norders, hbuf, hstride, b, part, nchunks, s); break;
        default:
            if (cb > 8) return hipErrorInvalidValue;
            launch_adj_cb<T, 8>(t, batch, a_lo, norders, hbuf, hstride, b, part, nchunks, s);
            break;
    }
    if (nchunks > 1) {
        dim3 grid_r((unsigned)((R * 2LL * N + 255) / 256), norders);
        hipLaunchKernelGGL((k_reduce_chunks<T>), grid_r, dim3(256), 0, s, N, batch, a_lo, nchunks,
                           (const double *)part, b);
    }
    return hipGetLastError();
}

hipError_t alt_dense_transpose(const DenseTables &t, int dtype, int batch, int a_lo, int a_hi,
                               bool weights, const void *g, void *beta, double *hbuf, double *part,
                               hipStream_t s) {
    if (dtype == 0) return launch_adj<double>(t, batch, a_lo, a_hi, weights, g, beta, hbuf, part, s);
    return launch_adj<float>(t, batch, a_lo, a_hi, weights, g, beta, hbuf, part, s);
}

size_t dense_part_bytes(int N, int batch) {
    const int G = (N + 63) / 64;
    const int nchunks = (G + kMaxGroups - 1) / kMaxGroups;
    if (nchunks <= 1) return 0;
    return (size_t)nchunks * (size_t)N * (2 * N + 1) * 4 * batch * sizeof(double);
}

}  // namespace dev
}  // namespace sht
