// Real fields (Section 1, the expansion of f): a real f has
// beta_{k,-m} = conj(beta_{k,m}) (the same Pbar_k^{|m|} serves both signs),
// so a real field is given by its coefficients of orders m >= 0 only, and two
// real fields f1, f2 travel through the complex transform as z = f1 + i f2:
//   beta^z_{k,m}  = beta1_{k,m} + i beta2_{k,m},
//   beta^z_{k,-m} = conj(beta1_{k,m}) + i conj(beta2_{k,m})          (m > 0),
// and back
//   beta1_{k,m} = (beta^z_{k,m} + conj(beta^z_{k,-m})) / 2,
//   beta2_{k,m} = (beta^z_{k,m} - conj(beta^z_{k,-m})) / (2 i).
// The ALT then runs on 4 real right-hand sides per pair of real fields, half
// of what two complex fields take, and one complex phi DFT serves two real
// rows.
//
// Half layout of a real field's coefficients: orders m = 0 .. 2N-1, inside an
// order the degrees k = m .. 2N-1; order m starts at 2N m - m (m - 1) / 2.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "prof.h"
#include "sht_internal.h"

namespace sht {
namespace dev {

namespace {

__device__ __forceinline__ int64_t full_off(int N, int m) {
    const int64_t a = m < 0 ? -(int64_t)m : m, twoN = 2 * (int64_t)N;
    if (a == 0) return 0;
    int64_t off = twoN * (2 * a - 1) - a * (a - 1);
    if (m < 0) off += twoN - a;
    return off;
}

__device__ __forceinline__ int64_t half_off(int N, int a) { return 2 * (int64_t)N * a - (int64_t)a * (a - 1) / 2; }

// one workgroup per (order a, pair p): fields 2p and 2p + 1 (zero past nreal)
template <typename T>
__global__ __launch_bounds__(256) void k_real_pack(int N, int nreal, const T *__restrict__ half, T *__restrict__ full) {
    const int a = blockIdx.x, p = blockIdx.y;
    const int n = 2 * N - a;
    const int64_t hfield = (int64_t)N * (2 * N + 1), ffield = 4 * (int64_t)N * N;
    const bool has1 = 2 * p < nreal, has2 = 2 * p + 1 < nreal;
    const T *h1 = half + 2 * ((int64_t)(2 * p) * hfield + half_off(N, a));
    const T *h2 = half + 2 * ((int64_t)(2 * p + 1) * hfield + half_off(N, a));
    T *zp = full + 2 * ((int64_t)p * ffield + full_off(N, a));
    T *zm = full + 2 * ((int64_t)p * ffield + full_off(N, -a));
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        T r1 = 0, i1 = 0, r2 = 0, i2 = 0;
        if (has1) {
            r1 = h1[2 * j];
            i1 = h1[2 * j + 1];
        }
        if (has2) {
            r2 = h2[2 * j];
            i2 = h2[2 * j + 1];
        }
        if (a == 0) {  // real coefficients at m = 0 (imaginary parts ignored)
            zp[2 * j] = r1;
            zp[2 * j + 1] = r2;
        } else {
            zp[2 * j] = r1 - i2;
            zp[2 * j + 1] = i1 + r2;
            zm[2 * j] = r1 + i2;
            zm[2 * j + 1] = r2 - i1;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_real_unpack(int N, int nreal, const T *__restrict__ full, T *__restrict__ half) {
    const int a = blockIdx.x, p = blockIdx.y;
    const int n = 2 * N - a;
    const int64_t hfield = (int64_t)N * (2 * N + 1), ffield = 4 * (int64_t)N * N;
    const bool has1 = 2 * p < nreal, has2 = 2 * p + 1 < nreal;
    T *h1 = half + 2 * ((int64_t)(2 * p) * hfield + half_off(N, a));
    T *h2 = half + 2 * ((int64_t)(2 * p + 1) * hfield + half_off(N, a));
    const T *zp = full + 2 * ((int64_t)p * ffield + full_off(N, a));
    const T *zm = full + 2 * ((int64_t)p * ffield + full_off(N, -a));
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const T pr = zp[2 * j], pi = zp[2 * j + 1];
        const T mr = zm[2 * j], mi = zm[2 * j + 1];  // the same slot when a = 0
        if (has1) {
            h1[2 * j] = (T)0.5 * (pr + mr);
            h1[2 * j + 1] = (T)0.5 * (pi - mi);
        }
        if (has2) {
            h2[2 * j] = (T)0.5 * (pi + mi);
            h2[2 * j + 1] = (T)0.5 * (mr - pr);
        }
    }
}

}  // namespace

hipError_t real_pack(int dtype, int N, int pairs, int nreal, const void *half, void *full, hipStream_t s) {
    prof::Scope ps(s, "k_real_pack");
    const dim3 grid(2 * N, pairs);
    if (dtype == 0)
        hipLaunchKernelGGL(k_real_pack<double>, grid, dim3(256), 0, s, N, nreal, (const double *)half, (double *)full);
    else
        hipLaunchKernelGGL(k_real_pack<float>, grid, dim3(256), 0, s, N, nreal, (const float *)half, (float *)full);
    return hipGetLastError();
}

hipError_t real_unpack(int dtype, int N, int pairs, int nreal, const void *full, void *half, hipStream_t s) {
    prof::Scope ps(s, "k_real_unpack");
    const dim3 grid(2 * N, pairs);
    if (dtype == 0)
        hipLaunchKernelGGL(k_real_unpack<double>, grid, dim3(256), 0, s, N, nreal, (const double *)full, (double *)half);
    else
        hipLaunchKernelGGL(k_real_unpack<float>, grid, dim3(256), 0, s, N, nreal, (const float *)full, (float *)half);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace sht
