// Small dense FP64 linear algebra for plan construction (host only).
#include "linalg.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

namespace sht {
namespace la {

int pivoted_qr(int m, int n, double *a, int lda, double tol, int kmax, std::vector<int> &perm,
               std::vector<double> *tau_out) {
    perm.resize(n);
    std::iota(perm.begin(), perm.end(), 0);
    // partial column norms: vn1 is kept up to date by downdating with the new
    // row of R after each step; vn2 is the value at the last exact
    // computation.  When the downdate has cancelled most of a norm, it is
    // recomputed exactly (the safeguard of LAPACK's column-pivoted QR).
    std::vector<double> vn1(n), vn2(n);
    for (int j = 0; j < n; ++j) {
        const double *c = a + (size_t)j * lda;
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += c[i] * c[i];
        vn1[j] = vn2[j] = std::sqrt(s);
    }
    const double tol3z = std::sqrt(2.220446049250313e-16);
    std::vector<double> tau;
    const int kk = std::min(std::min(m, n), kmax);
    int rank = 0;
    for (int k = 0; k < kk; ++k) {
        int p = k;
        for (int j = k + 1; j < n; ++j)
            if (vn1[j] > vn1[p]) p = j;
        if (p != k) {
            std::swap_ranges(a + (size_t)k * lda, a + (size_t)k * lda + m, a + (size_t)p * lda);
            std::swap(perm[k], perm[p]);
            std::swap(vn1[k], vn1[p]);
            std::swap(vn2[k], vn2[p]);
        }
        // exact norm of the pivot column's remaining part
        double *c = a + (size_t)k * lda;
        double best = 0.0;
        for (int i = k; i < m; ++i) best += c[i] * c[i];
        const double xnorm = std::sqrt(best);
        if (xnorm <= tol) break;
        // Householder reflector for column k, rows k..m-1
        double alpha = c[k];
        double beta = alpha >= 0 ? -xnorm : xnorm;
        double t = (beta - alpha) / beta;
        double scale = 1.0 / (alpha - beta);
        for (int i = k + 1; i < m; ++i) c[i] *= scale;
        c[k] = beta;
        // apply H = I - t v v^T (v = [1; c[k+1:m]]) to the remaining columns
        // and downdate their norms by the new entry R(k, j)
        for (int j = k + 1; j < n; ++j) {
            double *d = a + (size_t)j * lda;
            double s = d[k];
            for (int i = k + 1; i < m; ++i) s += c[i] * d[i];
            s *= t;
            d[k] -= s;
            for (int i = k + 1; i < m; ++i) d[i] -= s * c[i];
            if (vn1[j] != 0.0) {
                double r = std::fabs(d[k]) / vn1[j];
                r = std::max(0.0, (1.0 + r) * (1.0 - r));
                const double q = vn1[j] / vn2[j];
                if (r * q * q <= tol3z) {
                    double e = 0.0;
                    for (int i = k + 1; i < m; ++i) e += d[i] * d[i];
                    vn1[j] = vn2[j] = std::sqrt(e);
                } else {
                    vn1[j] *= std::sqrt(r);
                }
            }
        }
        tau.push_back(t);
        rank = k + 1;
    }
    if (tau_out) *tau_out = tau;
    return rank;
}

void solve_upper(int k, int n, const double *r, int ldr, double *t) {
    // columns j = k..n-1 of R give right-hand sides
    for (int j = k; j < n; ++j) {
        double *x = t + (size_t)(j - k) * k;
        const double *b = r + (size_t)j * ldr;
        for (int i = k - 1; i >= 0; --i) {
            double s = b[i];
            for (int q = i + 1; q < k; ++q) s -= r[i + (size_t)q * ldr] * x[q];
            x[i] = s / r[i + (size_t)i * ldr];
        }
    }
}

void form_q(int m, int k, const double *a, int lda, const std::vector<double> &tau, double *q) {
    std::fill(q, q + (size_t)m * k, 0.0);
    for (int j = 0; j < k; ++j) q[j + (size_t)j * m] = 1.0;
    for (int h = (int)tau.size() - 1; h >= 0; --h) {
        if (h >= k) continue;
        const double *v = a + (size_t)h * lda;  // v = [1; v[h+1:m]]
        for (int j = 0; j < k; ++j) {
            double *d = q + (size_t)j * m;
            double s = d[h];
            for (int i = h + 1; i < m; ++i) s += v[i] * d[i];
            s *= tau[h];
            d[h] -= s;
            for (int i = h + 1; i < m; ++i) d[i] -= s * v[i];
        }
    }
}

void jacobi_svd(int m, int n, double *a, int lda, double *s, double *v) {
    std::fill(v, v + (size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[i + (size_t)i * n] = 1.0;
    const double eps = 1e-15;
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int i = 0; i < n - 1; ++i) {
            for (int j = i + 1; j < n; ++j) {
                double *ai = a + (size_t)i * lda, *aj = a + (size_t)j * lda;
                double al = 0, be = 0, ga = 0;
                for (int r = 0; r < m; ++r) {
                    al += ai[r] * ai[r];
                    be += aj[r] * aj[r];
                    ga += ai[r] * aj[r];
                }
                if (std::fabs(ga) <= eps * std::sqrt(al * be) || ga == 0.0) continue;
                rotated = true;
                double zeta = (be - al) / (2.0 * ga);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
                for (int r = 0; r < m; ++r) {
                    double x = ai[r], y = aj[r];
                    ai[r] = c * x - sn * y;
                    aj[r] = sn * x + c * y;
                }
                double *vi = v + (size_t)i * n, *vj = v + (size_t)j * n;
                for (int r = 0; r < n; ++r) {
                    double x = vi[r], y = vj[r];
                    vi[r] = c * x - sn * y;
                    vj[r] = sn * x + c * y;
                }
            }
        }
        if (!rotated) break;
    }
    std::vector<int> ord(n);
    std::vector<double> sv(n);
    for (int i = 0; i < n; ++i) {
        double *ai = a + (size_t)i * lda;
        double nn = 0;
        for (int r = 0; r < m; ++r) nn += ai[r] * ai[r];
        sv[i] = std::sqrt(nn);
        if (sv[i] > 0)
            for (int r = 0; r < m; ++r) ai[r] /= sv[i];
    }
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sv[x] > sv[y]; });
    std::vector<double> ua((size_t)m * n), va((size_t)n * n);
    for (int i = 0; i < n; ++i) {
        s[i] = sv[ord[i]];
        std::memcpy(&ua[(size_t)i * m], a + (size_t)ord[i] * lda, sizeof(double) * m);
        std::memcpy(&va[(size_t)i * n], v + (size_t)ord[i] * n, sizeof(double) * n);
    }
    for (int i = 0; i < n; ++i) std::memcpy(a + (size_t)i * lda, &ua[(size_t)i * m], sizeof(double) * m);
    std::memcpy(v, va.data(), sizeof(double) * n * n);
}

void pinv(int m, int n, const double *a, int lda, double rcond, double *out) {
    // work on the tall orientation
    const bool tall = m >= n;
    const int M = tall ? m : n, Nn = tall ? n : m;
    std::vector<double> u((size_t)M * Nn), s(Nn), v((size_t)Nn * Nn);
    for (int j = 0; j < Nn; ++j)
        for (int i = 0; i < M; ++i) u[i + (size_t)j * M] = tall ? a[i + (size_t)j * lda] : a[j + (size_t)i * lda];
    jacobi_svd(M, Nn, u.data(), M, s.data(), v.data());
    const double cut = s.empty() ? 0.0 : rcond * s[0];
    // pinv(B) for B = U S V^T (M x Nn) is V S^+ U^T (Nn x M)
    std::vector<double> pb((size_t)Nn * M, 0.0);
    for (int q = 0; q < Nn; ++q) {
        if (s[q] <= cut || s[q] == 0.0) continue;
        double inv = 1.0 / s[q];
        for (int j = 0; j < M; ++j) {
            double uj = u[j + (size_t)q * M] * inv;
            for (int i = 0; i < Nn; ++i) pb[i + (size_t)j * Nn] += v[i + (size_t)q * Nn] * uj;
        }
    }
    // out is n x m: tall -> pb is n x m; wide -> pinv(A) = pinv(A^T)^T, pb is m x n
    if (tall) {
        std::memcpy(out, pb.data(), sizeof(double) * pb.size());
    } else {
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < n; ++i) out[i + (size_t)j * n] = pb[j + (size_t)i * m];
    }
}

void gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double *a, int lda,
          const double *b, int ldb, double beta, double *c, int ldc) {
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int q = 0; q < k; ++q) {
                double x = ta ? a[q + (size_t)i * lda] : a[i + (size_t)q * lda];
                double y = tb ? b[j + (size_t)q * ldb] : b[q + (size_t)j * ldb];
                s += x * y;
            }
            c[i + (size_t)j * ldc] = alpha * s + (beta == 0.0 ? 0.0 : beta * c[i + (size_t)j * ldc]);
        }
    }
}

}  // namespace la
}  // namespace sht
