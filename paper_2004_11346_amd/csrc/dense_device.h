// Device bodies of the plain (dense) ALT shared by the per-plan kernels and
// the grouped persistent kernels: the three-term recurrence in the degree with
// the extended exponent, the VALU forward of one node tile and the VALU
// transposed product of one order.  Included by .hip files only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sht {
namespace dev {
namespace dense {

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

__device__ __forceinline__ double scale_of(int e) { return e < -1074 ? 0.0 : ldexp(1.0, e); }

template <typename T> struct Cplx;
template <> struct Cplx<double> { typedef double2 type; };
template <> struct Cplx<float> { typedef float2 type; };

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

// one recurrence step: p0 <- p1, p1 <- a (x p1 - b p0)
__device__ __forceinline__ void rstep(double a, double b, double x, double &p0, double &p1) {
    const double p2 = a * (x * p1 - b * p0);
    p0 = p1;
    p1 = p2;
}

__device__ __forceinline__ void rescale(double &p0, double &p1, int &e, double &sc) {
    if (fabs(p1) > kBig) {
        p0 *= kShrink;
        p1 *= kShrink;
        e += 200;
        sc = scale_of(e);
    }
}

// same-parity step: with (p0, p1) = (Pbar_{k-2}, Pbar_k), the composed
// two-step recurrence Pbar_{k+2} = (alpha x^2 + beta) Pbar_k + gamma Pbar_{k-2}
// (c3 = (alpha, beta, gamma) of degree k + 2); rescaled like rstep
__device__ __forceinline__ void two_step(const double *__restrict__ c3, double x2, double &p0, double &p1, int &e,
                                         double &sc) {
    const double p2 = fma(c3[0], x2, c3[1]) * p1 + c3[2] * p0;
    p0 = p1;
    p1 = p2;
    rescale(p0, p1, e, sc);
}

// n same-parity steps without a column guard (pairs, no register copies),
// values p * 2^e to out[j * stride], one rescale test at the end; scaling by
// 2^-200 is exact, so the values equal those of n two_step calls
template <int n>
__device__ __forceinline__ void two_step_run(const double *__restrict__ c3, double x2, double &p0, double &p1, int &e,
                                             double &sc, double *out, int stride) {
    static_assert(n % 2 == 0, "steps come in pairs");
    double q0 = p0, q1 = p1;
#pragma unroll
    for (int j = 0; j < n; j += 2) {
        const double *c = c3 + 3 * j;
        const double r2 = fma(c[0], x2, c[1]) * q1 + c[2] * q0;
        out[j * stride] = r2 * sc;
        const double r3 = fma(c[3], x2, c[4]) * r2 + c[5] * q1;
        out[(j + 1) * stride] = r3 * sc;
        q0 = r2;
        q1 = r3;
    }
    p0 = q0;
    p1 = q1;
    if (fabs(p1) > kBig || fabs(p0) > kBig) {
        p0 *= kShrink;
        p1 *= kShrink;
        e += 200;
        sc = scale_of(e);
    }
}

typedef double d4v __attribute__((ext_vector_type(4)));


// VALU forward of one order a and one tile of 64 NPL nodes (one wave).
// LDS per buffer: coefficients [64][2] and beta [64][FB][2 signs][2].
// lds: at least fwd_tile_lds(FB) doubles.
__host__ __device__ constexpr int fwd_tile_lds(int FB) { return 2 * 64 * 2 + 2 * 64 * FB * 4; }

template <typename T, int FB, int NPL>
__device__ __forceinline__ void dense_fwd_tile(int N, int M, int batch, int a, int tile,
                                               const double *__restrict__ xh, const double *__restrict__ dmant,
                                               const int *__restrict__ dexp, const double *__restrict__ coef,
                                               const T *__restrict__ beta, T *__restrict__ g, double *lds) {
    constexpr int KC = 64;
    double(*s_c)[KC * 2] = reinterpret_cast<double(*)[KC * 2]>(lds);
    double(*s_b)[KC * FB * 4] = reinterpret_cast<double(*)[KC * FB * 4]>(lds + 2 * KC * 2);
    const int n = 2 * N, nk = n - a;
    const int lane = threadIdx.x;
    const bool neg = a > 0;
    const double *c = coef + 2 * d_tri_offset(N, a);
    const int64_t offp = d_coef_offset(N, a), offn = d_coef_offset(N, -a);
    const int64_t bstride = 4LL * N * N;
    const int64_t gstride = (int64_t)n * M;
    int rr[NPL];
    double x[NPL];
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
        const int r = (tile * NPL + i) * 64 + lane;
        rr[i] = r;
        x[i] = xh[r < N ? r : N - 1];
    }
    for (int b0 = 0; b0 < batch; b0 += FB) {
        double p0[NPL], p1[NPL], sc[NPL];
        int e[NPL];
        double acc[NPL][8 * FB];  // per field: E+ re/im, E- re/im, O+ re/im, O- re/im
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            const int r = rr[i] < N ? rr[i] : N - 1;
            p1[i] = dmant[(int64_t)a * N + r];
            e[i] = rr[i] < N ? dexp[(int64_t)a * N + r] : -4000;
            p0[i] = 0.0;
            sc[i] = scale_of(e[i]);
#pragma unroll
            for (int q = 0; q < 8 * FB; ++q) acc[i][q] = 0.0;
        }
        // chunk loader: lane j fetches degree kc0 + j
        double lc0 = 0, lc1 = 0, lb[FB * 4];
        auto fetch = [&](int kc0) {
            const int j = kc0 + lane;
            const bool ok = j < nk;
            lc0 = ok ? c[2 * j] : 0.0;
            lc1 = ok ? c[2 * j + 1] : 0.0;
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                const int fb = b0 + f < batch ? b0 + f : batch - 1;
                const T *bp = beta + 2 * ((int64_t)fb * bstride);
                lb[4 * f + 0] = ok ? (double)bp[2 * (offp + j)] : 0.0;
                lb[4 * f + 1] = ok ? (double)bp[2 * (offp + j) + 1] : 0.0;
                lb[4 * f + 2] = (ok && neg) ? (double)bp[2 * (offn + j)] : 0.0;
                lb[4 * f + 3] = (ok && neg) ? (double)bp[2 * (offn + j) + 1] : 0.0;
            }
        };
        auto stash = [&](int buf) {
            s_c[buf][2 * lane] = lc0;
            s_c[buf][2 * lane + 1] = lc1;
#pragma unroll
            for (int q = 0; q < 4 * FB; ++q) s_b[buf][lane * 4 * FB + q] = lb[q];
        };
        fetch(0);
        stash(0);
        __syncthreads();
        int buf = 0;
        for (int kc0 = 0; kc0 < nk; kc0 += KC) {
            if (kc0 + KC < nk) fetch(kc0 + KC);
            const int kn = min(KC, nk - kc0);
            for (int kk = 0; kk < kn; kk += 2) {
                {  // even k - a
                    const int j = kc0 + kk;
                    const double ca = s_c[buf][2 * kk], cb = s_c[buf][2 * kk + 1];
                    const double *bv = &s_b[buf][kk * 4 * FB];
#pragma unroll
                    for (int i = 0; i < NPL; ++i) {
                        if (j > 0) rstep(ca, cb, x[i], p0[i], p1[i]);
                        const double v = p1[i] * sc[i];
#pragma unroll
                        for (int f = 0; f < FB; ++f)
#pragma unroll
                            for (int q = 0; q < 4; ++q) acc[i][8 * f + q] = fma(v, bv[4 * f + q], acc[i][8 * f + q]);
                    }
                }
                if (kk + 1 < kn) {  // odd k - a
                    const double ca = s_c[buf][2 * kk + 2], cb = s_c[buf][2 * kk + 3];
                    const double *bv = &s_b[buf][(kk + 1) * 4 * FB];
#pragma unroll
                    for (int i = 0; i < NPL; ++i) {
                        rstep(ca, cb, x[i], p0[i], p1[i]);
                        const double v = p1[i] * sc[i];
#pragma unroll
                        for (int f = 0; f < FB; ++f)
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                acc[i][8 * f + 4 + q] = fma(v, bv[4 * f + q], acc[i][8 * f + 4 + q]);
                        rescale(p0[i], p1[i], e[i], sc[i]);
                    }
                }
            }
            if (kc0 + KC < nk) {
                stash(buf ^ 1);
                __syncthreads();
                buf ^= 1;
            }
        }
#pragma unroll
        for (int i = 0; i < NPL; ++i) {
            const int r = rr[i];
            if (r >= N) continue;
            const int l = n - 1 - r, lm = r;
#pragma unroll
            for (int f = 0; f < FB; ++f) {
                if (b0 + f >= batch) break;
                T *gb = g + 2 * ((b0 + f) * gstride);
                const double *A = &acc[i][8 * f];
                st2(gb + 2 * ((int64_t)l * M + a), A[0] + A[4], A[1] + A[5]);
                st2(gb + 2 * ((int64_t)lm * M + a), A[0] - A[4], A[1] - A[5]);
                if (neg) {
                    st2(gb + 2 * ((int64_t)l * M + (M - a)), A[2] + A[6], A[3] + A[7]);
                    st2(gb + 2 * ((int64_t)lm * M + (M - a)), A[2] - A[6], A[3] - A[7]);
                }
            }
        }
        __syncthreads();
    }
}

// VALU transpose for few right-hand sides.  grid: (orders), block 64 W.
// Lane (wave w, lane l) owns nodes w 64 NR + 64 i + l (i < NR) and keeps their
// folded grid values h_p(r) = w_r (g(2N-1-r) + (-1)^p g(r)) for both parities
// in registers.  The recurrence runs over the degrees; each lane forms the
// 4 FB products of every degree, KB = 8 / FB degrees at a time (32 partial
// sums per lane), and the 32 sums are reduced over the wave's lanes with a
// reduce-scatter (five halving exchange rounds and one final exchange, after
// which lanes 2 i and 2 i + 1 hold sum i); the W waves' sums are added
// through LDS in a fixed order.
template <typename T, int FB, int NR>
__device__ __forceinline__ void dense_adj_order(int N, int M, int batch, int b0, int a, int W,
                                                const double *__restrict__ xh, const double *__restrict__ wh,
                                                const double *__restrict__ dmant, const int *__restrict__ dexp,
                                                const double *__restrict__ coef, const T *__restrict__ g,
                                                T *__restrict__ beta, double *red) {
    constexpr int NQ = 4 * FB;     // per node: field, sign of m, re/im
    constexpr int KB = 32 / NQ;    // degrees per reduction round
    const int n = 2 * N, nk = n - a;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const bool neg = a > 0;
    const int M_ = M;
    const double *c = coef + 2 * d_tri_offset(N, a);
    const int64_t gstride = (int64_t)n * M_;
    double x[NR], p0[NR], p1[NR], sc[NR], he[NR][NQ], ho[NR][NQ];
    int e[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int r = w * 64 * NR + 64 * i + lane;
        const bool ok = r < N;
        const int rr = ok ? r : N - 1;
        x[i] = xh[rr];
        p1[i] = dmant[(int64_t)a * N + rr];
        e[i] = ok ? dexp[(int64_t)a * N + rr] : -4000;
        p0[i] = 0.0;
        sc[i] = scale_of(e[i]);
        const double wt = wh ? wh[rr] : 1.0;
        const int l = n - 1 - rr, lm = rr;
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            const int fb = b0 + f < batch ? b0 + f : batch - 1;
            const T *gb = g + 2 * ((int64_t)fb * gstride);
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                const int col = s2 == 0 ? a : M_ - a;
                const bool use = ok && (s2 == 0 || neg) && (b0 + f < batch);
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                    const double gl = use ? (double)gb[2 * ((int64_t)l * M_ + col) + cc] : 0.0;
                    const double gm = use ? (double)gb[2 * ((int64_t)lm * M_ + col) + cc] : 0.0;
                    he[i][4 * f + 2 * s2 + cc] = wt * (gl + gm);
                    ho[i][4 * f + 2 * s2 + cc] = wt * (gl - gm);
                }
            }
        }
    }
    const int64_t bstride = 4LL * N * N;
    const int64_t offp = d_coef_offset(N, a), offn = d_coef_offset(N, -a);
    for (int j0 = 0; j0 < nk; j0 += KB) {
        double v[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) v[q] = 0.0;
#pragma unroll
        for (int jj = 0; jj < KB; ++jj) {
            const int j = j0 + jj;
            if (j < nk) {
                const double ca = c[2 * j], cb = c[2 * j + 1];
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    if (j > 0) rstep(ca, cb, x[i], p0[i], p1[i]);
                    const double pv = p1[i] * sc[i];
                    if (j & 1) {
#pragma unroll
                        for (int q = 0; q < NQ; ++q) v[jj * NQ + q] = fma(pv, ho[i][q], v[jj * NQ + q]);
                        rescale(p0[i], p1[i], e[i], sc[i]);
                    } else {
#pragma unroll
                        for (int q = 0; q < NQ; ++q) v[jj * NQ + q] = fma(pv, he[i][q], v[jj * NQ + q]);
                    }
                }
            }
        }
        // reduce-scatter over the 64 lanes: after the round with mask m the
        // lane keeps the half of its values selected by (lane & m)
#pragma unroll
        for (int rnd = 0; rnd < 5; ++rnd) {
            const int m = 32 >> rnd, half = 16 >> rnd;
            const bool hi = (lane & m) != 0;
#pragma unroll
            for (int i = 0; i < half; ++i) {
                const double mine = hi ? v[i + half] : v[i];
                const double other = hi ? v[i] : v[i + half];
                v[i] = mine + __shfl_xor(other, m);
            }
        }
        v[0] += __shfl_xor(v[0], 1);
        if (W > 1) {
            red[w * 64 + lane] = v[0];
            __syncthreads();
        }
        if (w == 0) {
            double t = v[0];
            for (int u = 1; u < W; ++u) t += red[u * 64 + lane];
            const int idx = lane >> 1, jj = idx / NQ, q = idx - jj * NQ;
            const int j = j0 + jj;
            const int f = q >> 2, s2 = (q >> 1) & 1, cc = q & 1;
            if ((lane & 1) == 0 && jj < KB && j < nk && b0 + f < batch && (s2 == 0 || neg))
                beta[2 * ((int64_t)(b0 + f) * bstride + (s2 == 0 ? offp : offn) + j) + cc] = (T)t;
        }
        if (W > 1) __syncthreads();
    }
}

}  // namespace dense
}  // namespace dev
}  // namespace sht
