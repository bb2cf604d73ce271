// Length-M (M = 4N - 1) DFT along phi for every grid row (Section 1):
//   synthesis  f[l][j] = sum_{m=-(2N-1)}^{2N-1} g[l][m mod M] e^{i m phi_j},
//              phi_j = 2 pi (j + 1/2) / M,
//   analysis   g[l][m mod M] = scale * sum_j f[l][j] e^{-i m phi_j}.
// The half-sample shift of phi_j becomes a twiddle e^{+-i pi m / M} on the
// order side (with the signed order m), leaving a plain length-M DFT.
//
// One workgroup owns one row, held once in LDS.  The DFT is an in-place
// mixed-radix decimation in frequency over the prime factors of M (largest
// first): a pass of radix R over blocks of length L splits each block into R
// interleaved sub-blocks of length L/R with
//   y[n1 + (L/R) k2] = w_L^{n1 k2} sum_{n2} x[n1 + (L/R) n2] w_R^{n2 k2}.
// Small radices run as register butterflies (each thread owns whole
// butterflies, so a pass needs no barrier between its reads and writes);
// large primes (e.g. 89 in 2047 = 23 * 89, 127 in 16383) compute every output
// of the pass as an R-term sum into registers, then write after a barrier.
// After the last pass the spectrum sits in digit-reversed order; a position
// table maps each output index to its LDS slot so the row is written back
// with coalesced stores.  Every phase is looked up in one table of
// e^{i pi r / M}, r in [0, 2M), with indices reduced exactly in integers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "prof.h"

namespace sht {
namespace dev {

namespace {

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
template <typename C, typename T>
__global__ __launch_bounds__(512) void k_dft_rows(int N, int M, Passes ps, const C *__restrict__ tw2,
                                                  const int *__restrict__ src_pos, int mode, C scale, const T *in,
                                                  T *out) {
    typedef typename V2<C>::t c2;
    extern __shared__ unsigned char smem_raw[];
    c2 *buf = reinterpret_cast<c2 *>(smem_raw);
    const int64_t base = 2 * ((int64_t)blockIdx.y * 2 * N * M + (int64_t)blockIdx.x * M);
    const T *src = in + base;
    T *dst = out + base;
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
            default: pass_sum<C, 32>(buf, M, R, L, tw2, sgn); break;
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

template <typename C, typename T>
hipError_t launch_rows(const DftPlan &p, int batch, int mode, double scale, const void *in, void *out,
                       hipStream_t s) {
    Passes ps;
    ps.n = p.nrad;
    for (int i = 0; i < 24; ++i) {
        ps.R[i] = p.radix[i];
        ps.L[i] = p.blen[i];
    }
    const size_t lds = sizeof(typename V2<C>::t) * (size_t)p.M;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)&k_dft_rows<C, T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const C *tw = sizeof(C) == 8 ? (const C *)p.tw2 : (const C *)p.tw2f;
    prof::Scope sc(s, mode == 0 ? "k_dft_synthesis" : "k_dft_analysis");
    hipLaunchKernelGGL((k_dft_rows<C, T>), dim3(2 * p.N, batch), dim3(512), lds, s, p.N, p.M, ps, tw, p.src_pos,
                       mode, (C)scale, (const T *)in, (T *)out);
    return hipGetLastError();
}

}  // namespace

bool dft_supported(int M, int dtype) {
    const size_t elt = dtype == 0 ? 16 : 8;
    // one row in LDS; the generic pass holds at most 32 outputs per thread
    return elt * (size_t)M <= 160 * 1024 && M <= 32 * 512;
}

void dft_passes(int M, std::vector<int> &radix, std::vector<int> &blen, std::vector<int> &src_pos) {
    radix.clear();
    int m = M;
    for (int p = 2; (long long)p * p <= m; ++p)
        while (m % p == 0) {
            radix.push_back(p);
            m /= p;
        }
    if (m > 1) radix.push_back(m);
    std::sort(radix.rbegin(), radix.rend());
    blen.clear();
    int L = M;
    for (int R : radix) {
        blen.push_back(L);
        L /= R;
    }
    // output frequency of every LDS slot after the passes (digit reversal)
    std::vector<int> freq(M);
    struct Rec {
        static void go(std::vector<int> &f, const std::vector<int> &rs, size_t d, int pos0, int L, int mult,
                       int fb) {
            if (d == rs.size()) {
                f[pos0] = fb;
                return;
            }
            const int R = rs[d], Ls = L / R;
            for (int k2 = 0; k2 < R; ++k2) go(f, rs, d + 1, pos0 + Ls * k2, Ls, mult * R, fb + k2 * mult);
        }
    };
    Rec::go(freq, radix, 0, 0, M, 1, 0);
    src_pos.assign(M, 0);
    for (int i = 0; i < M; ++i) src_pos[freq[i]] = i;
}

hipError_t dft_synthesis(const DftPlan &p, int dtype, int batch, void *f, hipStream_t s) {
    if (dtype == 0) return launch_rows<double, double>(p, batch, 0, 1.0, f, f, s);
    return launch_rows<float, float>(p, batch, 0, 1.0, f, f, s);
}

hipError_t dft_analysis(const DftPlan &p, int dtype, int batch, double scale, const void *f, void *g,
                        hipStream_t s) {
    if (dtype == 0) return launch_rows<double, double>(p, batch, 1, scale, f, g, s);
    return launch_rows<float, float>(p, batch, 1, scale, f, g, s);
}

}  // namespace dev
}  // namespace sht
