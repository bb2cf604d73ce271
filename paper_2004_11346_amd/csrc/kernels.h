// Device-side tables and kernel launchers (host-callable).  All launchers
// enqueue on the given stream and return the launch status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace sht {
namespace dev {

// Legendre tables resident in HBM (see legendre.cpp for their contents).
struct DenseTables {
    int N = 0, M = 0;
    const double *xh = nullptr;     // [N]
    const double *wh = nullptr;     // [N]
    const double *dmant = nullptr;  // [2N][N]
    const int *dexp = nullptr;      // [2N][N]
    const double *coef = nullptr;   // [tri][2] one-step recurrence
    const double *coef2 = nullptr;  // [tri][3] same-parity two-step recurrence
};

// FP64 panels used by the plain path when it runs on the matrix cores, and
// the checkpoints of its transposed product: one item per (task, 64-column
// output tile), items sorted by task; the recurrence states of every item's
// rows at its first column are recomputed per call, a chunk of tasks at a
// time, into a buffer of ck_cap states.
struct DensePanels {
    void *X = nullptr;             // [N (2N + 1)][R] coefficient panels
    void *Y = nullptr;             // [4 N^2][R] half-grid panels
    const int64_t *x_off = nullptr;  // device [4N + 1]
    int64_t max_cols = 0;
    const int32_t *adj_items = nullptr;  // device [items][2]: task, first column
    std::vector<int32_t> adj_task_first; // host [4N + 1]: first item of every task
    const int32_t *adj_task_first_d = nullptr;  // its device copy
    double *ck = nullptr;                // device [2 ck_cap]: (Pbar_{k-2}, Pbar_k) per state
    int32_t *ckexp = nullptr;            // device [ck_cap]: their binary exponent
    int64_t ck_cap = 0;                  // states per chunk (multiple of the padded row count)
};
bool dense_uses_panels(int batch);

// Dense forward ALT for orders a_lo..a_hi (both signs): beta -> g columns.
hipError_t alt_dense_forward(const DenseTables &t, const DensePanels &pn, int dtype, int batch, int a_lo, int a_hi,
                             const void *beta, void *g, hipStream_t s);

// Dense transposed ALT (weights = true: inverse A^T W; false: adjoint A^T):
// g columns -> beta.
hipError_t alt_dense_transpose(const DenseTables &t, const DensePanels &pn, int dtype, int batch, int a_lo,
                               int a_hi, bool weights, const void *g, void *beta, hipStream_t s);

// Panels (see kernels_panels.hip).  x_off: device [4N + 1] row offsets of
// the X panels; the Y panel of task t starts at row t * N.
// dtype: element type of beta / g; panel64: panels in FP64 (else same type).
hipError_t panel_pack(int dtype, bool panel64, int N, int batch, int a_lo, int a_hi, const int64_t *x_off,
                      int64_t max_cols, const void *beta, void *X, hipStream_t s);
hipError_t panel_scatter(int dtype, bool panel64, int N, int batch, int a_lo, int a_hi, const int64_t *x_off,
                         int64_t max_cols, const void *X, void *beta, hipStream_t s);
hipError_t panel_combine(int dtype, bool panel64, int N, int batch, int a_lo, int a_hi, const void *Y, void *g,
                         hipStream_t s);
hipError_t panel_fold(int dtype, bool panel64, int N, int batch, int a_lo, int a_hi, const double *wh,
                      const void *g, void *Y, hipStream_t s);

// Length-M DFT of every grid row (Section 1, phi sums), LDS resident.
struct DftPlan {
    int N = 0, M = 0;
    int nrad = 0;
    int radix[24] = {0};          // prime factors of M, largest first
    int blen[24] = {0};           // block length before each pass
    const double *tw2 = nullptr;  // [2M][2]: exp(i pi r / M), r in [0, 2M)
    const float *tw2f = nullptr;  // same in float
    const int *src_pos = nullptr;  // [M]: LDS slot holding output index c
};
bool dft_supported(int M, int dtype);
// host: radices, block lengths and the output position table for length M
void dft_passes(int M, std::vector<int> &radix, std::vector<int> &blen, std::vector<int> &src_pos);
// synthesis in place on f: f[l][j] = sum_m g[l][m mod M] e^{i m phi_j}
hipError_t dft_synthesis(const DftPlan &p, int dtype, int batch, void *f, hipStream_t s);
// analysis f -> g: g[l][m mod M] = scale * sum_j f[l][j] e^{-i m phi_j}
hipError_t dft_analysis(const DftPlan &p, int dtype, int batch, double scale, const void *f, void *g,
                        hipStream_t s);

}  // namespace dev
}  // namespace sht
