// Host FP64 quadrature and Legendre tables (plan time).
//
// * Gauss-Legendre rule of Section 1 (2N nodes in x = cos(theta), ascending):
//   Newton's method on P_n(x) from Tricomi's asymptotic guess, carried in
//   long double and mirrored so that x_{n-1-i} = -x_i exactly.
// * Pbar_m^m(x) for every order at every half-grid node, stored as
//   (mantissa, binary exponent) so that values far below the binary64 range
//   keep their significant digits; the kernels and the plan builder resume the
//   three-term recurrence in k from these, rescaling by exact powers of two.
// * Coefficients (a_k, b_k) of the normalised three-term recurrence
//   Pbar_k^m = a_k (x Pbar_{k-1}^m - b_k Pbar_{k-2}^m), packed per order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "sht_internal.h"

namespace sht {

namespace {
typedef long double ld;

// Run body(i) for i in [0, n) on all hardware threads (static interleave).
template <typename F>
void parallel_for(int n, F body) {
    int nth = (int)std::thread::hardware_concurrency();
    nth = std::max(1, std::min({nth, 64, n}));
    if (nth == 1) {
        for (int i = 0; i < n; ++i) body(i);
        return;
    }
    std::vector<std::thread> th;
    for (int w = 0; w < nth; ++w)
        th.emplace_back([&, w]() {
            for (int i = w; i < n; i += nth) body(i);
        });
    for (auto &t : th) t.join();
}
const ld kPi = 3.141592653589793238462643383279502884L;

// P_n(t) and P_n'(t) by the Legendre three-term recurrence.
void legendre_and_derivative(int n, ld t, ld &p, ld &dp) {
    ld pm1 = 1.0L, pc = t;
    if (n == 0) {
        p = 1.0L;
        dp = 0.0L;
        return;
    }
    for (int j = 2; j <= n; ++j) {
        ld pn = ((2 * j - 1) * t * pc - (j - 1) * pm1) / j;
        pm1 = pc;
        pc = pn;
    }
    p = pc;
    dp = n * (pm1 - t * pc) / (1.0L - t * t);
}
}  // namespace

void gauss_legendre(int n, double *x, double *w) {
    const int half = n / 2;
    auto root = [&](int k) {
        // k-th largest root; Tricomi's first-order asymptotic guess
        ld th = kPi * (4 * k - 1) / (4.0L * n + 2.0L);
        ld t = (1.0L - (n - 1.0L) / (8.0L * n * n * n)) * cosl(th);
        ld p = 0, dp = 1;
        for (int it = 0; it < 60; ++it) {
            legendre_and_derivative(n, t, p, dp);
            ld step = p / dp;
            t -= step;
            if (fabsl(step) < 1e-20L) break;
        }
        legendre_and_derivative(n, t, p, dp);
        ld wt = 2.0L / ((1.0L - t * t) * dp * dp);
        int hi = n - k, lo = k - 1;
        if (hi == lo) {  // middle node of an odd rule
            x[hi] = 0.0;
            w[hi] = (double)wt;
        } else {
            x[hi] = (double)t;
            x[lo] = -(double)t;
            w[hi] = (double)wt;
            w[lo] = (double)wt;
        }
    };
    if (n >= 512)
        parallel_for((n + 1) / 2, [&](int i) { root(i + 1); });
    else
        for (int k = 1; k <= (n + 1) / 2; ++k) root(k);
    (void)half;
}

void build_legendre_tables(int N, LegendreTables &t, int m_lo, int m_hi) {
    const int n = 2 * N;
    // orders whose recurrence coefficients are computed (the others stay 0)
    m_lo = std::max(0, m_lo);
    m_hi = m_hi < 0 ? n - 1 : std::min(m_hi, n - 1);
    t.N = N;
    std::vector<double> x(n), w(n);
    gauss_legendre(n, x.data(), w.data());
    t.xh.resize(N);
    t.wh.resize(N);
    for (int r = 0; r < N; ++r) {
        t.xh[r] = x[n - 1 - r];
        t.wh[r] = w[n - 1 - r];
    }
    // diagonal values Pbar_m^m(x) = Pbar_{m-1}^{m-1}(x) sqrt((2m+1)/(2m)) s
    t.diag_m.assign((size_t)n * N, 0.0);
    t.diag_e.assign((size_t)n * N, 0);
    std::vector<ld> fac(n);
    for (int m = 1; m < n; ++m) fac[m] = sqrtl((ld)(2 * m + 1) / (ld)(2 * m));
    parallel_for(N, [&](int r) {
        ld xv = t.xh[r];
        ld s = sqrtl((1.0L - xv) * (1.0L + xv));
        ld mu = 1.0L / sqrtl(2.0L);
        int e = 0;
        for (int m = 0; m <= m_hi; ++m) {
            if (m > 0) mu *= fac[m] * s;
            int ee = 0;
            mu = frexpl(mu, &ee);
            e += ee;
            t.diag_m[(size_t)m * N + r] = (double)mu;
            t.diag_e[(size_t)m * N + r] = e;
        }
    });
    // recurrence coefficients
    t.coef.assign((size_t)2 * tri_offset(N, n), 0.0);
    parallel_for(m_hi - m_lo + 1, [&](int i) {
        const int m = m_lo + i;
        double *c = &t.coef[2 * tri_offset(N, m)];
        if (m + 1 < n) {
            c[2] = (double)sqrtl((ld)(2 * m + 3));
            c[3] = 0.0;
        }
        for (int k = m + 2; k < n; ++k) {
            ld kk = k, mm = m;
            ld a = sqrtl((4.0L * kk * kk - 1.0L) / ((kk - mm) * (kk + mm)));
            ld b = sqrtl(((kk - 1 - mm) * (kk - 1 + mm)) / (4.0L * (kk - 1) * (kk - 1) - 1.0L));
            c[2 * (k - m)] = (double)a;
            c[2 * (k - m) + 1] = (double)b;
        }
    });
    // composed two-step coefficients: from P_{k-1} = a_{k-1} (x P_{k-2} - b_{k-1} P_{k-3})
    // and x P_{k-3} = P_{k-2} / a_{k-2} + b_{k-2} P_{k-4},
    //   alpha_k = a_k a_{k-1},  beta_k = -a_k (b_k + a_{k-1} b_{k-1} / a_{k-2}),
    //   gamma_k = -a_k a_{k-1} b_{k-1} b_{k-2};
    // b_{m+1} = 0 removes the terms that would need a_m or b_m
    t.coef2.assign((size_t)3 * tri_offset(N, n), 0.0);
    parallel_for(m_hi - m_lo + 1, [&](int i) {
        const int m = m_lo + i;
        double *c2 = &t.coef2[3 * tri_offset(N, m)];
        auto A = [&](int k) -> ld {
            if (k == m + 1) return sqrtl((ld)(2 * m + 3));
            ld kk = k, mm = m;
            return sqrtl((4.0L * kk * kk - 1.0L) / ((kk - mm) * (kk + mm)));
        };
        auto B = [&](int k) -> ld {
            if (k <= m + 1) return 0.0L;
            ld kk = k, mm = m;
            return sqrtl(((kk - 1 - mm) * (kk - 1 + mm)) / (4.0L * (kk - 1) * (kk - 1) - 1.0L));
        };
        for (int k = m + 2; k < n; ++k) {
            const ld ak = A(k), ak1 = A(k - 1), bk = B(k), bk1 = B(k - 1);
            const ld mid = bk1 == 0.0L ? 0.0L : ak1 * bk1 / A(k - 2);
            const ld gam = (bk1 == 0.0L || k - 2 <= m) ? 0.0L : -ak * ak1 * bk1 * B(k - 2);
            c2[3 * (k - m)] = (double)(ak * ak1);
            c2[3 * (k - m) + 1] = (double)(-ak * (bk + mid));
            c2[3 * (k - m) + 2] = (double)gam;
        }
    });
}

void alt_half_matrix(const LegendreTables &t, int a, int parity, double *out) {
    const int N = t.N, n = 2 * N;
    const int cols = half_cols(N, a, parity);
    const double *c = &t.coef[2 * tri_offset(N, a)];
    const double kBig = 0x1p200, kShrink = 0x1p-200;
    for (int r = 0; r < N; ++r) {
        double x = t.xh[r];
        double p1 = t.diag_m[(size_t)a * N + r], p0 = 0.0;
        int e = t.diag_e[(size_t)a * N + r];
        double *row = out + (size_t)r * cols;
        auto emit = [&](int k, double v) {
            int par = (k - a) & 1;
            if (par == parity) row[(k - a - parity) / 2] = (e < -1100) ? 0.0 : std::ldexp(v, e);
        };
        emit(a, p1);
        for (int k = a + 1; k < n; ++k) {
            double p2 = c[2 * (k - a)] * (x * p1 - c[2 * (k - a) + 1] * p0);
            p0 = p1;
            p1 = p2;
            if (std::fabs(p1) > kBig) {
                p0 *= kShrink;
                p1 *= kShrink;
                e += 200;
            }
            emit(k, p1);
        }
    }
}

}  // namespace sht
