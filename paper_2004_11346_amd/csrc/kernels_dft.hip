// Length-M (M = 4N - 1) DFT along phi for every grid row (Section 1):
//   synthesis  f[l][j] = sum_{m=-(2N-1)}^{2N-1} g[l][m mod M] e^{i m phi_j},
//              phi_j = 2 pi (j + 1/2) / M,
//   analysis   g[l][m mod M] = scale * sum_j f[l][j] e^{-i m phi_j}.
// The half-sample shift of phi_j becomes a twiddle e^{+-i pi m / M} on the
// order side (with the signed order m), leaving a plain length-M DFT.
//
// One workgroup owns one row, held in LDS (two ping-pong buffers); the DFT is
// a mixed-radix Stockham autosort over the prime factors of M.  Every output
// of a pass is the length-R sum  Y[j + sT] = sum_r X[i + r M/R] w^{r(k + sT)}
// (k = i mod T, j = (i/T) T R + k, w = e^{+-2 pi i / (T R)}), computed by one
// thread with the phase index advanced incrementally, so any radix -- including
// the large primes of M = 2047 = 23 * 89 or 16383 = 3 * 43 * 127 -- uses the
// same code.  All phases are looked up in one table of e^{i pi r / M},
// r in [0, 2M), whose indices are reduced exactly in integers.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sht {
namespace dev {

namespace {

template <typename C> struct V2;
template <> struct V2<double> { typedef double2 t; };
template <> struct V2<float> { typedef float2 t; };

struct Radices {
    int n;
    int r[24];
};

// mode 0: synthesis (pre-twiddle e^{+i pi m/M}, sign +1)
// mode 1: analysis  (sign -1, post-twiddle scale * e^{-i pi m/M})
template <typename C, typename T>
__global__ __launch_bounds__(256) void k_dft_rows(int N, int M, Radices rad,
                                                  const C *__restrict__ tw2, int mode, C scale,
                                                  const T *in, T *out) {
    typedef typename V2<C>::t c2;
    extern __shared__ unsigned char smem_raw[];
    c2 *bufA = reinterpret_cast<c2 *>(smem_raw);
    c2 *bufB = bufA + M;
    const int row = blockIdx.x;
    const int fld = blockIdx.y;
    const int64_t base = 2 * ((int64_t)fld * 2 * N * M + (int64_t)row * M);
    const T *src = in + base;
    T *dst = out + base;
    const int twoM = 2 * M;
    const C sgn = mode == 0 ? (C)1 : (C)-1;

    for (int c = threadIdx.x; c < M; c += blockDim.x) {
        C xr = (C)src[2 * c], xi = (C)src[2 * c + 1];
        if (mode == 0) {
            int m = c <= 2 * N - 1 ? c : c - M;  // signed order
            int q = m < 0 ? m + twoM : m;        // e^{i pi m / M}
            C tr = tw2[2 * q], ti = tw2[2 * q + 1];
            C yr = xr * tr - xi * ti, yi = xr * ti + xi * tr;
            xr = yr;
            xi = yi;
        }
        bufA[c] = c2{xr, xi};
    }
    __syncthreads();

    c2 *X = bufA, *Y = bufB;
    int Tp = 1;
    for (int p = 0; p < rad.n; ++p) {
        const int R = rad.r[p];
        const int MR = M / R;
        const int TR = Tp * R;
        const int unit = 2 * (M / TR);  // table step per phase unit of w
        for (int o = threadIdx.x; o < M; o += blockDim.x) {
            const int i = o % MR, s = o / MR;
            const int k = i % Tp;
            const int step = k + s * Tp;  // < Tp R
            C accr = 0, acci = 0;
            int q = 0;
            for (int r = 0; r < R; ++r) {
                c2 x = X[i + r * MR];
                const int ti = q * unit;  // < 2M
                C wr = tw2[2 * ti], wi = sgn * tw2[2 * ti + 1];
                accr += x.x * wr - x.y * wi;
                acci += x.x * wi + x.y * wr;
                q += step;
                if (q >= TR) q -= TR;
            }
            const int j = (i / Tp) * TR + k;
            Y[j + s * Tp] = c2{accr, acci};
        }
        __syncthreads();
        c2 *tmp = X;
        X = Y;
        Y = tmp;
        Tp = TR;
    }

    for (int c = threadIdx.x; c < M; c += blockDim.x) {
        c2 v = X[c];
        C yr = v.x, yi = v.y;
        if (mode == 1) {
            int m = c <= 2 * N - 1 ? c : c - M;
            int q = m < 0 ? -m : twoM - m;  // e^{-i pi m / M}
            if (q == twoM) q = 0;
            C tr = tw2[2 * q], ti = tw2[2 * q + 1];
            C zr = yr * tr - yi * ti, zi = yr * ti + yi * tr;
            yr = zr * scale;
            yi = zi * scale;
        }
        dst[2 * c] = (T)yr;
        dst[2 * c + 1] = (T)yi;
    }
}

template <typename C, typename T>
hipError_t launch_rows(const DftPlan &p, int batch, int mode, double scale, const void *in, void *out,
                       hipStream_t s) {
    Radices rad;
    rad.n = p.nrad;
    for (int i = 0; i < 24; ++i) rad.r[i] = p.radix[i];
    const size_t lds = 2 * sizeof(typename V2<C>::t) * (size_t)p.M;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)&k_dft_rows<C, T>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const C *tw = sizeof(C) == 8 ? (const C *)p.tw2 : (const C *)p.tw2f;
    hipLaunchKernelGGL((k_dft_rows<C, T>), dim3(2 * p.N, batch), dim3(256), lds, s, p.N, p.M, rad, tw,
                       mode, (C)scale, (const T *)in, (T *)out);
    return hipGetLastError();
}

}  // namespace

bool dft_supported(int M, int dtype) {
    const size_t elt = dtype == 0 ? 16 : 8;
    return 2 * elt * (size_t)M <= 160 * 1024;
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
