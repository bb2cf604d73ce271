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

#include "dft_device.h"
#include "kernels.h"
#include "prof.h"

namespace sht {
namespace dev {

namespace {

using namespace dft;

template <typename C, typename T, int MAXO>
__global__ __launch_bounds__(512) void k_dft_rows(int N, int M, Passes ps, const C *__restrict__ tw2,
                                                  const int *__restrict__ src_pos, int mode, C scale, const T *in,
                                                  T *out) {
    extern __shared__ unsigned char smem_raw[];
    typename V2<C>::t *buf = reinterpret_cast<typename V2<C>::t *>(smem_raw);
    const int64_t base = 2 * ((int64_t)blockIdx.y * 2 * N * M + (int64_t)blockIdx.x * M);
    dft_row<C, T, MAXO>(N, M, ps, tw2, src_pos, mode, scale, in + base, out + base, buf);
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
        for (const void *fn : {(const void *)&k_dft_rows<C, T, 0>, (const void *)&k_dft_rows<C, T, 8>,
                               (const void *)&k_dft_rows<C, T, 32>}) {
            hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e != hipSuccess) return e;
        }
        attr_set = true;
    }
    const C *tw = sizeof(C) == 8 ? (const C *)p.tw2 : (const C *)p.tw2f;
    int maxr = 0;
    for (int i = 0; i < p.nrad; ++i) maxr = std::max(maxr, p.radix[i]);
    prof::Scope sc(s, mode == 0 ? "k_dft_synthesis" : "k_dft_analysis");
    if (maxr <= 13)
        hipLaunchKernelGGL((k_dft_rows<C, T, 0>), dim3(2 * p.N, batch), dim3(512), lds, s, p.N, p.M, ps, tw,
                           p.src_pos, mode, (C)scale, (const T *)in, (T *)out);
    else if (p.M <= 8 * 512)
        hipLaunchKernelGGL((k_dft_rows<C, T, 8>), dim3(2 * p.N, batch), dim3(512), lds, s, p.N, p.M, ps, tw,
                           p.src_pos, mode, (C)scale, (const T *)in, (T *)out);
    else
        hipLaunchKernelGGL((k_dft_rows<C, T, 32>), dim3(2 * p.N, batch), dim3(512), lds, s, p.N, p.M, ps, tw,
                           p.src_pos, mode, (C)scale, (const T *)in, (T *)out);
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
