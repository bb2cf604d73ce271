// Internal declarations of the SHT library (host side).
//
// Half-grid convention used throughout: the Gauss-Legendre nodes are symmetric
// (x_{2N-1-l} = -x_l), so the ALT is evaluated on the N nodes with x > 0 and
// mirrored (Section 3.1.2).  Half-grid row r (0 <= r < N) is node
// l = 2N-1-r, i.e. rows run from the pole (largest x, smallest theta) towards
// the equator, theta ascending -- the order in which the turning point
// t*_{k,m} of Section 3.2 splits each row into a non-oscillatory head and an
// oscillatory tail.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "sht.h"

namespace sht {

// ------------------------------------------------------------- errors
void set_error_detail(const std::string &msg);

// ------------------------------------------------------------- fixed scratch
// Bytes of the per-GPU device array used by sht_inverse_noalloc for the
// phi-analysed grid (128 MiB: one FP64 field at N = 1024).
constexpr size_t kNoallocScratchBytes = (size_t)128 << 20;
// Looks up the array's device address on `device` (which must be current);
// once per device, idempotent.  Returns the hipError_t status as an int.
int noalloc_scratch_init(int device);
// The address found by the lookup, or nullptr if it has not run.
void *noalloc_scratch(int device);

// ------------------------------------------------------------- layout
// Start (complex entries) of order m in the m-major coefficient layout.
inline int64_t coef_offset(int N, int m) {
    int64_t a = m < 0 ? -(int64_t)m : m;
    int64_t twoN = 2 * (int64_t)N;
    if (a == 0) return 0;
    int64_t off = twoN * (2 * a - 1) - a * (a - 1);
    if (m < 0) off += twoN - a;
    return off;
}

// Number of columns of the odd / even half matrix of order |m| (Section 3.1.2):
// odd N - ceil(|m|/2), even N - floor(|m|/2).
inline int half_cols(int N, int absm, int parity) {
    return parity ? N - (absm + 1) / 2 : N - absm / 2;
}

// Packed start of order |m| in the per-order recurrence tables (2N - j
// entries for order j).
inline int64_t tri_offset(int N, int a) {
    return 2 * (int64_t)N * a - (int64_t)a * (a - 1) / 2;
}

// ------------------------------------------------------------- quadrature
// 2N-point Gauss-Legendre rule, ascending, exactly symmetric.
void gauss_legendre(int n, double *x, double *w);

// Legendre tables used by the plain (dense) kernels and by the plan builder.
struct LegendreTables {
    int N = 0;
    std::vector<double> xh;       // [N] half-grid nodes, xh[r] = x_{2N-1-r}
    std::vector<double> wh;       // [N] their weights
    std::vector<double> diag_m;   // [2N][N] mantissa of Pbar_m^m(xh[r]) in [0.5, 1)
    std::vector<int32_t> diag_e;  // [2N][N] binary exponent
    std::vector<double> coef;     // [tri][2]: (a_k, b_k) of order m at k = m + j
    // [tri][3]: two steps of the recurrence composed, same parity:
    // P_k = (alpha_k x^2 + beta_k) P_{k-2} + gamma_k P_{k-4}, k = m + j, j >= 2
    std::vector<double> coef2;
};

// Orders outside [m_lo, m_hi] (m_hi < 0: up to 2N - 1) get no recurrence
// coefficients (zeros): plans restricted to an order range never read them.
void build_legendre_tables(int N, LegendreTables &t, int m_lo = 0, int m_hi = -1);

// Dense half-grid matrix of order a and parity p: out[r * cols + j] =
// Pbar_{a + p + 2j}^{a}(xh[r]).  Uses the same scaled recurrence.
void alt_half_matrix(const LegendreTables &t, int a, int parity, double *out);

}  // namespace sht
