// Device-side tables and kernel launchers (host-callable).  All launchers
// enqueue on the given stream and return the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace sht {
namespace dev {

// Legendre tables resident in HBM (see legendre.cpp for their contents).
struct DenseTables {
    int N = 0, M = 0;
    const double *xh = nullptr;     // [N]
    const double *wh = nullptr;     // [N]
    const double *dmant = nullptr;  // [2N][N]
    const int *dexp = nullptr;      // [2N][N]
    const double *coef = nullptr;   // [tri][2]
};

// Dense forward ALT for orders a_lo..a_hi (both signs): beta -> g columns.
hipError_t alt_dense_forward(const DenseTables &t, int dtype, int batch, int a_lo, int a_hi,
                             const void *beta, void *g, hipStream_t s);

// Dense transposed ALT (weights = true: inverse A^T W; false: adjoint A^T):
// g columns -> beta.  hbuf: scratch of 2N*(a_hi-a_lo+1)*4*batch doubles;
// part: scratch of dense_part_bytes(N, batch) bytes (may be null if 0).
hipError_t alt_dense_transpose(const DenseTables &t, int dtype, int batch, int a_lo, int a_hi,
                               bool weights, const void *g, void *beta, double *hbuf, double *part,
                               hipStream_t s);
size_t dense_part_bytes(int N, int batch);

// Length-M DFT of every grid row (Section 1, phi sums), LDS resident.
struct DftPlan {
    int N = 0, M = 0;
    int nrad = 0;
    int radix[24] = {0};
    const double *tw2 = nullptr;  // [2M][2]: exp(i pi r / M), r in [0, 2M)
    const float *tw2f = nullptr;  // same in float
};
bool dft_supported(int M, int dtype);
// synthesis in place on f: f[l][j] = sum_m g[l][m mod M] e^{i m phi_j}
hipError_t dft_synthesis(const DftPlan &p, int dtype, int batch, void *f, hipStream_t s);
// analysis f -> g: g[l][m mod M] = scale * sum_j f[l][j] e^{-i m phi_j}
hipError_t dft_analysis(const DftPlan &p, int dtype, int batch, double scale, const void *f, void *g,
                        hipStream_t s);

}  // namespace dev
}  // namespace sht
