// Device bodies of the length-M phi DFT (Section 1, the phi sums of eq.
// `sht_fft`), shared by the per-plan kernels and the grouped persistent
// kernel.  Included by .hip files only.
//
// Building blocks:
//  * a two-level phase table in LDS: e^{i pi r / Mt} = lo[r mod 64] * hi[r / 64]
//    for r in [0, 2 Mt), 64 + ceil(2 Mt / 64) complex entries (a few KB), filled
//    from a global table rounded from long double on the host;
//  * mixed-radix decimation-in-frequency passes over a buffer of `total`
//    elements made of independent segments of length L0 (a whole row, or the
//    sub-rows of a four-step pass): a pass of radix R over blocks of length L
//    splits each block into R interleaved sub-blocks of length L/R with
//      y[n1 + (L/R) k2] = w_L^{n1 k2} sum_{n2} x[n1 + (L/R) n2] w_R^{n2 k2};
//    radices up to 13 (and 9 for a pair of 3s) run as register butterflies,
//    larger primes as R-term sums; after the passes every segment is in
//    digit-reversed order;
//  * global loads and stores issued in unrolled groups, so that a thread's
//    accesses are in flight together.
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

constexpr int kUnroll = 8;  // global accesses in flight per thread and group

template <typename C>
__device__ __forceinline__ typename V2<C>::t cmul(typename V2<C>::t a, typename V2<C>::t b) {
    return typename V2<C>::t{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// entries of the two-level table of base Mt
__host__ __device__ inline int tab_entries(int Mt) { return 64 + (2 * Mt + 63) / 64; }

// e^{sgn i pi r / Mt}, 0 <= r < 2 Mt, from the FP64 table in LDS
__device__ __forceinline__ double2 twd(const double2 *t, int r, double sgn) {
    double2 p = cmul<double>(t[r & 63], t[64 + (r >> 6)]);
    p.y *= sgn;
    return p;
}

template <typename C>
__device__ __forceinline__ typename V2<C>::t tw(const double2 *t, int r, C sgn) {
    const double2 p = twd(t, r, (double)sgn);
    return typename V2<C>::t{(C)p.x, (C)p.y};
}

// copy a table of base Mt from global memory to LDS (FP64 for every element
// type: twiddle powers are formed from it in FP64)
__device__ __forceinline__ void load_tab(const double *__restrict__ g, int Mt, double2 *t) {
    const int n = tab_entries(Mt);
    for (int i = threadIdx.x; i < n; i += blockDim.x) t[i] = reinterpret_cast<const double2 *>(g)[i];
}

// a wave-uniform double moved to scalar registers
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// cos and sin of 2 pi q / R for q = 0 .. (R - 1) / 2 (odd R); the same for
// every lane, so they live in scalar registers.  q = 0 is used by composite
// R, where j k = 0 mod R for some j, k > 0 (j = k = 3 for R = 9).
template <int R>
__device__ __forceinline__ void roots(const double2 *t, int Mt, double (&c)[(R - 1) / 2 + 1],
                                      double (&sn)[(R - 1) / 2 + 1]) {
    c[0] = 1.0;
    sn[0] = 0.0;
#pragma unroll
    for (int q = 1; q <= (R - 1) / 2; ++q) {
        const double2 w = twd(t, 2 * q * (Mt / R), 1.0);
        c[q] = uniform(w.x);
        sn[q] = uniform(w.y);
    }
}

// R-point DFT of x (sign sgn) in place, odd R: with s_j = x_j + x_{R-j} and
// d_j = x_j - x_{R-j}, y_k = x_0 + sum_j s_j cos(2 pi j k / R)
// + i sgn sum_j d_j sin(2 pi j k / R) and y_{R-k} the same with -i: half the
// products of the direct sum and half the roots.
template <typename C, int R>
__device__ __forceinline__ void dft_small(typename V2<C>::t (&x)[R], const double (&c)[(R - 1) / 2 + 1],
                                          const double (&sn)[(R - 1) / 2 + 1], C sgn) {
    typedef typename V2<C>::t c2;
    if constexpr (R == 2) {
        const c2 a = x[0], b = x[1];
        x[0] = c2{a.x + b.x, a.y + b.y};
        x[1] = c2{a.x - b.x, a.y - b.y};
    } else {
        constexpr int H = (R - 1) / 2;
        c2 sj[H + 1], dj[H + 1];
        c2 y0 = x[0];
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            sj[j] = c2{x[j].x + x[R - j].x, x[j].y + x[R - j].y};
            dj[j] = c2{x[j].x - x[R - j].x, x[j].y - x[R - j].y};
            y0.x += sj[j].x;
            y0.y += sj[j].y;
        }
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            c2 a = x[0], b = c2{(C)0, (C)0};
#pragma unroll
            for (int j = 1; j <= H; ++j) {
                const int q = (j * k) % R;
                const C cq = (C)(q <= H ? c[q] : c[R - q]);
                const C sq = (C)(q <= H ? sn[q] : -sn[R - q]);
                a.x += cq * sj[j].x;
                a.y += cq * sj[j].y;
                b.x += sq * dj[j].x;
                b.y += sq * dj[j].y;
            }
            b.x *= sgn;
            b.y *= sgn;
            x[k] = c2{a.x - b.y, a.y + b.x};      // a + i b
            x[R - k] = c2{a.x + b.y, a.y - b.x};  // a - i b
        }
        x[0] = y0;
    }
}

// register butterflies of radix R over blocks of length L (table base Mt,
// L divides Mt), `total` elements.  The twiddles w_L^{n1 k2} of a butterfly
// are powers of w_L^{n1}, formed in FP64 from table lookups of w and w^R; the
// outputs k and R - k are stored as soon as they are formed
// (w^{R-k} = w^R conj(w^k)), which keeps the live registers to the sums and
// differences of the inputs.
// BD > 0: the block size as a compile-time constant (otherwise blockDim.x)
template <typename C, int R, int BD = 0>
__device__ __forceinline__ void pass_reg(typename V2<C>::t *buf, int total, int L, const double2 *t, int Mt,
                                         C sgn) {
    typedef typename V2<C>::t c2;
    constexpr int H = (R - 1) / 2;
    const int Ls = L / R;
    double c[H + 1], sn[H + 1];
    if constexpr (R > 2) roots<R>(t, Mt, c, sn);
    const int unitL = 2 * (Mt / L);
    const int nb = total / R;
    // butterfly b = blk Ls + n1, stepped by the block size without divisions
    const int bd = BD > 0 ? BD : (int)blockDim.x, sdiv = bd / Ls, smod = bd - sdiv * Ls;
    int blk = (int)threadIdx.x / Ls, n1 = (int)threadIdx.x - blk * Ls;
    for (int b = threadIdx.x; b < nb; b += bd) {
        const int base = blk * L + n1;
        const double2 w1 = twd(t, n1 * unitL, (double)sgn);
        if constexpr (R == 2) {
            const c2 x0 = buf[base], x1 = buf[base + Ls];
            buf[base] = c2{x0.x + x1.x, x0.y + x1.y};
            buf[base + Ls] = cmul<C>(c2{x0.x - x1.x, x0.y - x1.y}, c2{(C)w1.x, (C)w1.y});
        } else {
            const c2 x0 = buf[base];
            c2 sj[H + 1], dj[H + 1];
            c2 y0 = x0;
#pragma unroll
            for (int j = 1; j <= H; ++j) {
                const c2 u = buf[base + Ls * j], v = buf[base + Ls * (R - j)];
                sj[j] = c2{u.x + v.x, u.y + v.y};
                dj[j] = c2{u.x - v.x, u.y - v.y};
                y0.x += sj[j].x;
                y0.y += sj[j].y;
            }
            buf[base] = y0;
            // w^R for the conjugate-side twiddles: one more table lookup
            // (n1 R unitL < 2 Mt since n1 < L / R)
            const double2 wR = twd(t, n1 * R * unitL, (double)sgn);
            double2 wk = w1;
#pragma unroll
            for (int k = 1; k <= H; ++k) {
                c2 a = x0, bb = c2{(C)0, (C)0};
#pragma unroll
                for (int j = 1; j <= H; ++j) {
                    const int q = (j * k) % R;
                    const C cq = (C)(q <= H ? c[q] : c[R - q]);
                    const C sq = (C)(q <= H ? sn[q] : -sn[R - q]);
                    a.x += cq * sj[j].x;
                    a.y += cq * sj[j].y;
                    bb.x += sq * dj[j].x;
                    bb.y += sq * dj[j].y;
                }
                bb.x *= sgn;
                bb.y *= sgn;
                const double2 wm = cmul<double>(wR, double2{wk.x, -wk.y});  // w^{R-k}
                buf[base + Ls * k] = cmul<C>(c2{a.x - bb.y, a.y + bb.x}, c2{(C)wk.x, (C)wk.y});
                buf[base + Ls * (R - k)] = cmul<C>(c2{a.x + bb.y, a.y - bb.x}, c2{(C)wm.x, (C)wm.y});
                wk = cmul<double>(wk, w1);
            }
        }
        n1 += smod;
        blk += sdiv;
        if (n1 >= Ls) {
            n1 -= Ls;
            ++blk;
        }
    }
}

// any radix: every output is an R-term sum held in registers until all
// threads have read the pass's inputs.  At most MAXO outputs per thread.
template <typename C, int MAXO>
__device__ __forceinline__ void pass_sum(typename V2<C>::t *buf, int total, int R, int L, const double2 *t, int Mt,
                                         C sgn) {
    typedef typename V2<C>::t c2;
    const int Ls = L / R;
    const int twoM = 2 * Mt;
    const int unitR = 2 * (Mt / R), unitL = 2 * (Mt / L);
    c2 out[MAXO];
#pragma unroll
    for (int j = 0; j < MAXO; ++j) {
        const int o = threadIdx.x + j * blockDim.x;
        if (o >= total) continue;
        const int b = o / L, rem = o - b * L;
        const int k2 = rem / Ls, n1 = rem - k2 * Ls;
        const int base = b * L + n1;
        // phases w_R^{n2 k2}: powers of one table lookup, formed in FP64
        const double2 ws = twd(t, (k2 * unitR) % twoM, (double)sgn);
        double2 w = double2{1.0, 0.0};
        c2 y = c2{(C)0, (C)0};
        for (int n2 = 0; n2 < R; ++n2) {
            const c2 p = cmul<C>(buf[base + Ls * n2], c2{(C)w.x, (C)w.y});
            y.x += p.x;
            y.y += p.y;
            w = cmul<double>(w, ws);
        }
        const int tl = (int)(((long long)n1 * k2 * unitL) % twoM);
        out[j] = cmul<C>(y, tw<C>(t, tl, sgn));
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MAXO; ++j) {
        const int o = threadIdx.x + j * blockDim.x;
        if (o < total) buf[o] = out[j];
    }
}

// the first npass passes of `ps` (all of them when npass < 0) over `total`
// elements (segments of length ps.L[0]); ends with a barrier
template <typename C, int MAXO>
__device__ __forceinline__ void run_passes(typename V2<C>::t *buf, int total, const Passes &ps, const double2 *t,
                                           int Mt, C sgn, int npass = -1) {
    const int np = npass < 0 ? ps.n : npass;
    for (int p = 0; p < np; ++p) {
        const int R = ps.R[p], L = ps.L[p];
        switch (R) {
            case 2: pass_reg<C, 2>(buf, total, L, t, Mt, sgn); break;
            case 3: pass_reg<C, 3>(buf, total, L, t, Mt, sgn); break;
            case 5: pass_reg<C, 5>(buf, total, L, t, Mt, sgn); break;
            case 7: pass_reg<C, 7>(buf, total, L, t, Mt, sgn); break;
            case 9: pass_reg<C, 9>(buf, total, L, t, Mt, sgn); break;
            case 11: pass_reg<C, 11>(buf, total, L, t, Mt, sgn); break;
            case 13: pass_reg<C, 13>(buf, total, L, t, Mt, sgn); break;
            default:
                if constexpr (MAXO > 0) pass_sum<C, MAXO>(buf, total, R, L, t, Mt, sgn);
                break;
        }
        __syncthreads();
    }
}

// passes p0 .. p1 - 1 of `ps`, register butterflies of radix at most MAXR
// only (a smaller MAXR keeps the larger butterflies, and their registers, out
// of the code), BD threads per block; every pass ends with a barrier
template <typename C, int MAXR, int BD>
__device__ __forceinline__ void run_pass_range(typename V2<C>::t *buf, int total, const Passes &ps, int p0, int p1,
                                               const double2 *t, int Mt, C sgn) {
    for (int p = p0; p < p1; ++p) {
        const int R = ps.R[p], L = ps.L[p];
        switch (R) {
            case 2: pass_reg<C, 2, BD>(buf, total, L, t, Mt, sgn); break;
            case 3: pass_reg<C, 3, BD>(buf, total, L, t, Mt, sgn); break;
            case 5: pass_reg<C, 5, BD>(buf, total, L, t, Mt, sgn); break;
            case 7: pass_reg<C, 7, BD>(buf, total, L, t, Mt, sgn); break;
            case 9:
                if constexpr (MAXR >= 9) pass_reg<C, 9, BD>(buf, total, L, t, Mt, sgn);
                break;
            case 11:
                if constexpr (MAXR >= 11) pass_reg<C, 11, BD>(buf, total, L, t, Mt, sgn);
                break;
            case 13:
                if constexpr (MAXR >= 13) pass_reg<C, 13, BD>(buf, total, L, t, Mt, sgn);
                break;
            default: break;
        }
        __syncthreads();
    }
}

// Inverse of a register pass up to the factor R: for each butterfly the
// outputs are first multiplied by the conjugate twiddles w_L^{-n1 k2}, then an
// R-point DFT of the opposite sign gives R times the pass's inputs.  Run over
// the passes in reverse order (run_passes_inv), it takes a digit-reversed
// spectrum back to natural order: M times the inverse transform.
template <typename C, int R>
__device__ __forceinline__ void pass_reg_inv(typename V2<C>::t *buf, int total, int L, const double2 *t, int Mt,
                                             C sgn) {
    typedef typename V2<C>::t c2;
    const int Ls = L / R;
    double c[(R - 1) / 2 + 1], sn[(R - 1) / 2 + 1];
    if constexpr (R > 2) roots<R>(t, Mt, c, sn);
    const int unitL = 2 * (Mt / L);
    const int nb = total / R;
    const int bd = blockDim.x, sdiv = bd / Ls, smod = bd - sdiv * Ls;
    int blk = (int)threadIdx.x / Ls, n1 = (int)threadIdx.x - blk * Ls;
    for (int b = threadIdx.x; b < nb; b += bd) {
        const int base = blk * L + n1;
        const double2 w1 = twd(t, n1 * unitL, -(double)sgn);
        c2 y[R];
        y[0] = buf[base];
        double2 wk = w1;
#pragma unroll
        for (int k2 = 1; k2 < R; ++k2) {
            y[k2] = cmul<C>(buf[base + Ls * k2], c2{(C)wk.x, (C)wk.y});
            if (k2 + 1 < R) wk = cmul<double>(wk, w1);
        }
        dft_small<C, R>(y, c, sn, -sgn);
#pragma unroll
        for (int n2 = 0; n2 < R; ++n2) buf[base + Ls * n2] = y[n2];
        n1 += smod;
        blk += sdiv;
        if (n1 >= Ls) {
            n1 -= Ls;
            ++blk;
        }
    }
}

// generic-radix form of pass_reg_inv (MAXO inputs per thread)
template <typename C, int MAXO>
__device__ __forceinline__ void pass_sum_inv(typename V2<C>::t *buf, int total, int R, int L, const double2 *t,
                                             int Mt, C sgn) {
    typedef typename V2<C>::t c2;
    const int Ls = L / R;
    const int twoM = 2 * Mt;
    const int unitR = 2 * (Mt / R), unitL = 2 * (Mt / L);
    c2 out[MAXO];
#pragma unroll
    for (int j = 0; j < MAXO; ++j) {
        const int o = threadIdx.x + j * blockDim.x;
        if (o >= total) continue;
        const int b = o / L, rem = o - b * L;
        const int n2 = rem / Ls, n1 = rem - n2 * Ls;
        const int base = b * L + n1;
        // x[n2] = sum_k2 w_R^{-n2 k2} w_L^{-n1 k2} y[k2]: powers of one phase
        const double2 ws = twd(t, (int)(((long long)n2 * unitR + (long long)n1 * unitL) % twoM), -(double)sgn);
        double2 w = double2{1.0, 0.0};
        c2 x = c2{(C)0, (C)0};
        for (int k2 = 0; k2 < R; ++k2) {
            const c2 p = cmul<C>(buf[base + Ls * k2], c2{(C)w.x, (C)w.y});
            x.x += p.x;
            x.y += p.y;
            w = cmul<double>(w, ws);
        }
        out[j] = x;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MAXO; ++j) {
        const int o = threadIdx.x + j * blockDim.x;
        if (o < total) buf[o] = out[j];
    }
}

// reverse passes: digit-reversed spectrum (of run_passes with sign sgn) ->
// natural order, times the segment length; ends with a barrier
template <typename C, int MAXO>
__device__ __forceinline__ void run_passes_inv(typename V2<C>::t *buf, int total, const Passes &ps, const double2 *t,
                                               int Mt, C sgn) {
    for (int p = ps.n - 1; p >= 0; --p) {
        const int R = ps.R[p], L = ps.L[p];
        switch (R) {
            case 2: pass_reg_inv<C, 2>(buf, total, L, t, Mt, sgn); break;
            case 3: pass_reg_inv<C, 3>(buf, total, L, t, Mt, sgn); break;
            case 5: pass_reg_inv<C, 5>(buf, total, L, t, Mt, sgn); break;
            case 7: pass_reg_inv<C, 7>(buf, total, L, t, Mt, sgn); break;
            case 9: pass_reg_inv<C, 9>(buf, total, L, t, Mt, sgn); break;
            case 11: pass_reg_inv<C, 11>(buf, total, L, t, Mt, sgn); break;
            case 13: pass_reg_inv<C, 13>(buf, total, L, t, Mt, sgn); break;
            default:
                if constexpr (MAXO > 0) pass_sum_inv<C, MAXO>(buf, total, R, L, t, Mt, sgn);
                break;
        }
        __syncthreads();
    }
}

// Tables of a last pass of prime radix R > 13 taken by Rader's convolution
// (R - 1 a product of radices up to 13).  After the other passes the points
// of every block of R contiguous elements want a plain length-R DFT (the last
// pass has no twiddles); with a primitive root g of R, output g^{-p} is
// x_0 plus the cyclic convolution of a_q = x_{g^q} with b_q = w^{g^{-q}}.
//   inslot[n]: slot q of input n >= 1 (g^q = n); outslot[k]: slot of the
//   convolution that output k >= 1 reads; pc: the passes of length R - 1;
//   bspec: [2][R - 1] complex spectra of b (sign +1, then -1) under the
//   sign -1 transform, divided by R - 1, in the passes' digit-reversed slots;
//   ctab: phase table of base R - 1 (global).
struct RaderLast {
    int R;
    Passes pc;
    const double *ctab;
    const int *inslot, *outslot;
    const double *bspec;
    const float *bspecf;
};

// LDS bytes past the row buffer for a Rader last pass over `total` points:
// its phase table, the convolution buffer and two values per block
__host__ __device__ inline size_t rader_last_lds(int total, int R, size_t elt) {
    const int nblk = total / R;
    return 16 * (size_t)tab_entries(R - 1) + elt * ((size_t)nblk * (R - 1) + 2 * (size_t)nblk);
}

// The last pass of radix rl.R over `total` points of buf (blocks of R
// contiguous points, the transform of sign sgn) by Rader's convolution:
// gather into cbuf, forward transform of the R - 1 slots (sign -1), product
// with the spectrum, reverse passes (natural slot order), outputs back into
// buf.  tc: rl.ctab in LDS; aux: [2 * total / R] values.  Ends with a barrier.
template <typename C>
__device__ __forceinline__ void rader_last(typename V2<C>::t *buf, typename V2<C>::t *cbuf, typename V2<C>::t *aux,
                                           int total, const RaderLast &rl, const double2 *tc, C sgn) {
    typedef typename V2<C>::t c2;
    const int R = rl.R, L = R - 1, nblk = total / R;
    const int bd = blockDim.x;
    for (int i = threadIdx.x; i < total; i += bd) {
        const int b = i / R, n = i - b * R;
        const c2 x = buf[i];
        if (n == 0)
            aux[b] = x;  // x_0 of the block
        else
            cbuf[b * L + rl.inslot[n]] = x;
    }
    __syncthreads();
    run_passes<C, 0>(cbuf, nblk * L, rl.pc, tc, L, (C)-1);
    // frequency 0 of a (the sum of x_n, n >= 1) sits in slot 0
    for (int b = threadIdx.x; b < nblk; b += bd) aux[nblk + b] = cbuf[b * L];
    __syncthreads();
    const c2 *bs = reinterpret_cast<const c2 *>(sizeof(C) == 8 ? (const void *)rl.bspec : (const void *)rl.bspecf) +
                   (sgn > (C)0 ? 0 : L);
    for (int i = threadIdx.x; i < nblk * L; i += bd) {
        const int b = i / L, j = i - b * L;
        cbuf[i] = cmul<C>(cbuf[i], bs[j]);
    }
    __syncthreads();
    run_passes_inv<C, 0>(cbuf, nblk * L, rl.pc, tc, L, (C)-1);
    for (int i = threadIdx.x; i < total; i += bd) {
        const int b = i / R, k = i - b * R;
        const c2 x0 = aux[b];
        const c2 y = k == 0 ? aux[nblk + b] : cbuf[b * L + rl.outslot[k]];
        buf[i] = c2{x0.x + y.x, x0.y + y.y};
    }
    __syncthreads();
}

template <typename C, typename T>
__device__ __forceinline__ typename V2<C>::t ld(const T *p) {
    const typename V2<T>::t v = *reinterpret_cast<const typename V2<T>::t *>(p);
    return typename V2<C>::t{(C)v.x, (C)v.y};
}

template <typename C, typename T>
__device__ __forceinline__ void st(T *p, typename V2<C>::t v) {
    *reinterpret_cast<typename V2<T>::t *>(p) = typename V2<T>::t{(T)v.x, (T)v.y};
}

// Row input/output of the real-field transforms: a complex row z = f1 + i f2
// carries two real rows f1, f2 (two fields of real data; the second may be
// absent, then it reads as zero and is not written).
//   IO = 0: complex rows in and out;
//   IO = 1: complex row in, the real and imaginary parts stored to two real
//           rows (synthesis of two real fields);
//   IO = 2: two real rows in as one complex row, complex row out (analysis).
template <typename C, typename T, int IO>
__device__ __forceinline__ typename V2<C>::t ld_in(const T *src, const T *src2, int c) {
    if constexpr (IO == 2) return typename V2<C>::t{(C)src[c], src2 ? (C)src2[c] : (C)0};
    else return ld<C, T>(src + 2 * c);
}

template <typename C, typename T, int IO>
__device__ __forceinline__ void st_out(T *dst, T *dst2, int c, typename V2<C>::t v) {
    if constexpr (IO == 1) {
        dst[c] = (T)v.x;
        if (dst2) dst2[c] = (T)v.y;
    } else {
        st<C, T>(dst + 2 * c, v);
    }
}

// signed order of grid column c: 0..2N-1, then -(2N-1)..-1
__device__ __forceinline__ int signed_order(int c, int N, int M) { return c <= 2 * N - 1 ? c : c - M; }

// mode 0: synthesis, f[j] = sum_m g[m mod M] e^{i m phi_j}: pre-twiddle
//         e^{+i pi m / M}, sign +1, no scaling;
// mode 1: analysis, g[m mod M] = scale sum_j f[j] e^{-i m phi_j}: sign -1,
//         post-twiddle scale e^{-i pi m / M}.
// One row by one workgroup: src and dst point at the row (may alias), buf is
// M complex values of LDS followed by the phase table (base M).  MAXO:
// outputs per thread of the generic pass (radices above 13); 0 when every
// radix has a register butterfly.  RL: the last pass is taken by Rader's
// convolution (rl; its table, convolution buffer and block values follow
// the phase table in LDS).
template <typename C, typename T, int MAXO, int IO = 0, bool RL = false>
__device__ __forceinline__ void dft_row(int N, int M, const Passes &ps, const double *__restrict__ gtab,
                                        const int *__restrict__ src_pos, int mode, C scale, const T *src,
                                        const T *src2, T *dst, T *dst2, typename V2<C>::t *buf,
                                        const RaderLast *rl = nullptr) {
    typedef typename V2<C>::t c2;
    double2 *t = reinterpret_cast<double2 *>(buf + M + (M & 1));  // 16-byte aligned after the row
    load_tab(gtab, M, t);
    double2 *tc = t + tab_entries(M);
    if constexpr (RL) load_tab(rl->ctab, rl->R - 1, tc);
    const int twoM = 2 * M;
    const C sgn = mode == 0 ? (C)1 : (C)-1;
    const int bd = blockDim.x;
    c2 v[kUnroll];
    __syncthreads();  // table
    for (int c0 = 0; c0 < M; c0 += kUnroll * bd) {
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = c0 + threadIdx.x + j * bd;
            if (c < M) v[j] = ld_in<C, T, IO>(src, src2, c);
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
            buf[c] = x;
        }
    }
    __syncthreads();
    if constexpr (RL) {
        run_passes<C, MAXO>(buf, M, ps, t, M, sgn, ps.n - 1);
        c2 *cbuf = reinterpret_cast<c2 *>(tc + tab_entries(rl->R - 1));
        rader_last<C>(buf, cbuf, cbuf + (M / rl->R) * (rl->R - 1), M, *rl, tc, sgn);
    } else {
        run_passes<C, MAXO>(buf, M, ps, t, M, sgn);
    }
    for (int c0 = 0; c0 < M; c0 += kUnroll * bd) {
        int sp[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = c0 + threadIdx.x + j * bd;
            sp[j] = c < M ? src_pos[c] : 0;
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const int c = c0 + threadIdx.x + j * bd;
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
            st_out<C, T, IO>(dst, dst2, c, x);
        }
    }
}

}  // namespace dft
}  // namespace dev
}  // namespace sht
