// Device body of the length-M phi DFT of one grid row (shared by the per-plan
// kernel and the grouped persistent kernel).  Included by .hip files only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sht {
namespace dev {
namespace dft {

template <typename C> struct V2;
template <> struct V2<double> { typedef double2 t; };
template <> struct V2<float> { typedef float2 t; };

struct Passes {
    int n;
    int R[24];
    int L[24];  // block length before the pass
};

template <typename C>
__device__ __forceinline__ typename V2<C>::t cmul(typename V2<C>::t a, typename V2<C>::t b) {
    return typename V2<C>::t{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// phase e^{sgn * 2 pi i q / M}: table entry 2q mod 2M, conjugated for sgn < 0
template <typename C>
__device__ __forceinline__ typename V2<C>::t phase(const C *__restrict__ tw2, int idx2, C sgn) {
    return typename V2<C>::t{tw2[2 * idx2], sgn * tw2[2 * idx2 + 1]};
}

// register butterflies of radix R over blocks of length L
template <typename C, int R>
__device__ __forceinline__ void pass_reg(typename V2<C>::t *buf, int M, int L, const C *__restrict__ tw2, C sgn) {
    typedef typename V2<C>::t c2;
    const int Ls = L / R;
    const int twoM = 2 * M;
    c2 wr[R];  // w_R^q = e^{sgn 2 pi i q / R}
#pragma unroll
    for (int q = 0; q < R; ++q) wr[q] = phase<C>(tw2, (2 * q * (M / R)) % twoM, sgn);
    const int unitL = 2 * (M / L);  // table step of w_L
    for (int t = threadIdx.x; t < M / R; t += blockDim.x) {
        const int b = t / Ls, n1 = t - b * Ls;
        const int base = b * L + n1;
        c2 x[R];
#pragma unroll
        for (int n2 = 0; n2 < R; ++n2) x[n2] = buf[base + Ls * n2];
        const int step = (n1 * unitL) % twoM;
        int ti = 0;
#pragma unroll
        for (int k2 = 0; k2 < R; ++k2) {
            c2 y = x[0];
#pragma unroll
            for (int n2 = 1; n2 < R; ++n2) {
                const c2 p = cmul<C>(x[n2], wr[(n2 * k2) % R]);
                y.x += p.x;
                y.y += p.y;
            }
            if (k2 > 0) y = cmul<C>(y, phase<C>(tw2, ti, sgn));
            buf[base + Ls * k2] = y;
            ti += step;
            if (ti >= twoM) ti -= twoM;
        }
    }
}

// any radix: every output is an R-term sum; results held in registers until all
// threads have read the pass's inputs.  At most MAXO outputs per thread.
template <typename C, int MAXO>
__device__ __forceinline__ void pass_sum(typename V2<C>::t *buf, int M, int R, int L, const C *__restrict__ tw2,
                                         C sgn) {
    typedef typename V2<C>::t c2;
    const int Ls = L / R;
    const int twoM = 2 * M;
    const int unitR = 2 * (M / R), unitL = 2 * (M / L);
    c2 out[MAXO];
    int pos[MAXO];
#pragma unroll
    for (int j = 0; j < MAXO; ++j) {
        const int o = threadIdx.x + j * blockDim.x;
        pos[j] = -1;
        if (o >= M) continue;
        // o = base + Ls k2 within block b
        const int b = o / L, rem = o - b * L;
        const int k2 = rem / Ls, n1 = rem - k2 * Ls;
        const int base = b * L + n1;
        const int step = (k2 * unitR) % twoM;
        c2 y = c2{(C)0, (C)0};
        int ti = 0;
        for (int n2 = 0; n2 < R; ++n2) {
            const c2 p = cmul<C>(buf[base + Ls * n2], phase<C>(tw2, ti, sgn));
            y.x += p.x;
            y.y += p.y;
            ti += step;
            if (ti >= twoM) ti -= twoM;
        }
        const int tl = (int)(((long long)n1 * k2 * unitL) % twoM);
        out[j] = cmul<C>(y, phase<C>(tw2, tl, sgn));
        pos[j] = o;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MAXO; ++j)
        if (pos[j] >= 0) buf[pos[j]] = out[j];
}

// mode 0: synthesis (pre-twiddle e^{+i pi m/M}, sign +1)
// mode 1: analysis  (sign -1, post-twiddle scale * e^{-i pi m/M})
// One row by one workgroup: src and dst point at the row (may alias), buf is
// M complex values of LDS.  MAXO: outputs per thread of the generic pass
// (radices above 13); 0 when every radix has a register butterfly, which
// keeps the register budget low enough for two 512-thread rows per CU.
template <typename C, typename T, int MAXO>
__device__ __forceinline__ void dft_row(int N, int M, const Passes &ps, const C *__restrict__ tw2,
                                        const int *__restrict__ src_pos, int mode, C scale, const T *src, T *dst,
                                        typename V2<C>::t *buf) {
    typedef typename V2<C>::t c2;
    const int twoM = 2 * M;
    const C sgn = mode == 0 ? (C)1 : (C)-1;
    for (int c = threadIdx.x; c < M; c += blockDim.x) {
        c2 v = c2{(C)src[2 * c], (C)src[2 * c + 1]};
        if (mode == 0) {
            const int m = c <= 2 * N - 1 ? c : c - M;  // signed order
            v = cmul<C>(v, c2{tw2[2 * (m < 0 ? m + twoM : m)], tw2[2 * (m < 0 ? m + twoM : m) + 1]});
        }
        buf[c] = v;
    }
    __syncthreads();
    for (int p = 0; p < ps.n; ++p) {
        const int R = ps.R[p], L = ps.L[p];
        switch (R) {
            case 2: pass_reg<C, 2>(buf, M, L, tw2, sgn); break;
            case 3: pass_reg<C, 3>(buf, M, L, tw2, sgn); break;
            case 5: pass_reg<C, 5>(buf, M, L, tw2, sgn); break;
            case 7: pass_reg<C, 7>(buf, M, L, tw2, sgn); break;
            case 11: pass_reg<C, 11>(buf, M, L, tw2, sgn); break;
            case 13: pass_reg<C, 13>(buf, M, L, tw2, sgn); break;
            default:
                if constexpr (MAXO > 0) pass_sum<C, MAXO>(buf, M, R, L, tw2, sgn);
                break;
        }
        __syncthreads();
    }
    for (int c = threadIdx.x; c < M; c += blockDim.x) {
        c2 v = buf[src_pos[c]];
        if (mode == 1) {
            const int m = c <= 2 * N - 1 ? c : c - M;
            int q = m < 0 ? -m : twoM - m;  // e^{-i pi m / M}
            if (q == twoM) q = 0;
            v = cmul<C>(v, c2{tw2[2 * q], tw2[2 * q + 1]});
            v.x *= scale;
            v.y *= scale;
        }
        dst[2 * c] = (T)v.x;
        dst[2 * c + 1] = (T)v.y;
    }
}

}  // namespace dft
}  // namespace dev
}  // namespace sht
