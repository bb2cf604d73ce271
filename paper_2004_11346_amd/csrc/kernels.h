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

// Length-M DFT of every grid row (Section 1, the phi sums).  Schedules:
// rows in LDS, Rader's convolution for prime M, or four-step through a
// grid-sized buffer for rows larger than LDS (see kernels_dft.hip).
enum DftKind { kDftNone = -1, kDftRows = 0, kDftRader = 1, kDftFourStep = 2 };

// host tables of one length M (built once per plan or grouped transform)
struct DftHost {
    int kind = kDftNone, M = 0;
    std::vector<int> radix, blen, src_pos;     // rows: passes of M; Rader: of M - 1; four-step: of M1
    std::vector<int> radix2, blen2, src_pos2;  // four-step: passes of M2
    std::vector<double> tab;                   // phase table of base M (lo[64], hi[...]), complex
    std::vector<float> tabf;
    std::vector<double> ctab;                  // Rader: phase table of base M - 1
    std::vector<float> ctabf;
    std::vector<int> inslot, outslot;          // Rader: slot of input n / output k
    std::vector<double> bspec;                 // Rader: [2][M - 1] complex spectra (synthesis, analysis)
    std::vector<float> bspecf;
    int M1 = 0, M2 = 0, chunk1 = 0, chunk2 = 0;  // four-step split and chunks
    // last pass of prime radix rl_R[i] > 13 by Rader's convolution, for the
    // passes of list i (0: radix/blen, 1: radix2/blen2); rl_R[i] = 0: none.
    // Tables as for the Rader schedule with M replaced by rl_R[i].
    int rl_R[2] = {0, 0};
    std::vector<int> rl_radix[2], rl_blen[2], rl_src_pos[2], rl_inslot[2], rl_outslot[2];
    std::vector<double> rl_ctab[2], rl_bspec[2];
    std::vector<float> rl_ctabf[2], rl_bspecf[2];
};
// force: 0 = by length and type, 1 = rows in LDS (generic passes for large
// primes), 2 = Rader (prime M), 3 = four-step; kind = kDftNone if the schedule
// does not apply.  rader_last: a prime factor above 13 may run as a last pass
// by Rader's convolution (rows and four-step kernels of a plan; the grouped
// kernels take the generic passes).
void dft_build(int M, int dtype, DftHost &h, int force = 0, bool rader_last = true);

// device view of the tables (arrays owned by the plan or group)
struct DftPlan {
    int N = 0, M = 0, kind = kDftNone;
    int nrad = 0, radix[24] = {0}, blen[24] = {0};
    int nrad2 = 0, radix2[24] = {0}, blen2[24] = {0};
    int M1 = 0, M2 = 0, chunk1 = 0, chunk2 = 0;
    const double *tab = nullptr;
    const float *tabf = nullptr;
    const double *ctab = nullptr;
    const float *ctabf = nullptr;
    const int *src_pos = nullptr, *src_pos2 = nullptr;
    const int *inslot = nullptr, *outslot = nullptr;
    const double *bspec = nullptr;
    const float *bspecf = nullptr;
    void *scratch = nullptr;  // four-step: [batch][2N][M] complex of the plan's type
    // Rader last pass of pass list i (DftHost::rl_*)
    int rl_R[2] = {0, 0};
    int rl_nrad[2] = {0, 0}, rl_radix[2][24] = {{0}}, rl_blen[2][24] = {{0}};
    const double *rl_ctab[2] = {nullptr, nullptr};
    const float *rl_ctabf[2] = {nullptr, nullptr};
    const int *rl_inslot[2] = {nullptr, nullptr}, *rl_outslot[2] = {nullptr, nullptr};
    const double *rl_bspec[2] = {nullptr, nullptr};
    const float *rl_bspecf[2] = {nullptr, nullptr};
};
// kernel attributes of the DFT kernels (once per process, before any capture)
hipError_t dft_init();
// synthesis in place on f: f[l][j] = sum_m g[l][m mod M] e^{i m phi_j}
hipError_t dft_synthesis(const DftPlan &p, int dtype, int batch, void *f, hipStream_t s);
// analysis f -> g: g[l][m mod M] = scale * sum_j f[l][j] e^{-i m phi_j}
hipError_t dft_analysis(const DftPlan &p, int dtype, int batch, double scale, const void *f, void *g,
                        hipStream_t s);
// real fields: complex rows z (pairs fields) -> real rows of fields 2b and
// 2b + 1 (its real and imaginary part; fields >= nreal are not written)
hipError_t dft_synthesis_real(const DftPlan &p, int dtype, int pairs, int nreal, const void *z, void *f,
                              hipStream_t s);
// real fields: real rows of fields 2b, 2b + 1 (zero past nreal) as one
// complex row -> analysed complex rows z
hipError_t dft_analysis_real(const DftPlan &p, int dtype, int pairs, int nreal, double scale, const void *f,
                             void *z, hipStream_t s);

// Real fields (see kernels_real.hip): half coefficients [nreal][N (2N + 1)]
// of fields 2p, 2p + 1 <-> full complex coefficients [pairs][4N^2] of
// z = f1 + i f2 (fields past nreal read as zero / are not written).
hipError_t real_pack(int dtype, int N, int pairs, int nreal, const void *half, void *full, hipStream_t s);
hipError_t real_unpack(int dtype, int N, int pairs, int nreal, const void *full, void *half, hipStream_t s);

}  // namespace dev
}  // namespace sht
