/*
 * Plain CPU oracle for the spherical harmonic transform (SHT) whose
 * associated-Legendre part is accelerated in Bremer, Chen & Yang,
 * "Rapid application of the spherical harmonic transform via interpolative
 * decomposition butterfly factorization" (arXiv 2004.11346).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product path: only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg load
 * this library.  It shares no code, header, table or helper with the HIP
 * library; the two meet only through the seeded synthetic inputs.
 *
 * What it computes is the plain definition, written out:
 *   - 2N-point Gauss-Legendre rule in x = cos(theta), nodes ascending
 *     (Section 1, definition of the grid);
 *   - L2-normalised associated Legendre functions Pbar_k^m on [-1,1]
 *     (Section 1, expansion of f; Section 3.1.1, orthonormal basis);
 *   - forward ALT  g(m,theta_l) = sum_{k=|m|}^{2N-1} beta_{k,m} Pbar_k^{|m|}(x_l)
 *     (Section 1, the ALT definition; Section 3.1.1), summed in ascending k
 *     with no odd/even split, every order m in [-(2N-1), 2N-1];
 *   - phi synthesis f(theta_l,phi_j) = sum_m g(m,theta_l) exp(i m phi_j),
 *     phi_j = 2 pi (j+1/2)/(4N-1) (Section 1), as a direct sum;
 *   - phi analysis g = (1/M) sum_j f exp(-i m phi_j), M = 4N-1, and the
 *     transposed ALT beta = A^T W g (Section 3.1.1, B = A^T W).
 *
 * Precision: inputs and outputs are IEEE binary64; Legendre values, phases and
 * all sums are carried in x87 long double (64-bit significand, 15-bit
 * exponent).  The long-double exponent range (down to ~1e-4951) is what keeps
 * the recurrence from underflowing: the smallest starting value Pbar_m^m(x)
 * that still grows into a value above the binary64 range before k reaches 2N
 * is about 10^(-0.32 N), i.e. 1e-1310 at N = 4096, far inside the range.  Any
 * value that does underflow to zero there is below 1e-4900 and cannot reach
 * binary64 range by k = 2N-1 for N <= 4096, so it contributes exactly zero in
 * binary64 as well.
 *
 * Conventions (readings of the paper, stated once):
 *   - normalisation: integral_{-1}^{1} Pbar_k^m(x)^2 dx = 1;
 *   - no Condon-Shortley phase: Pbar_m^m(x) >= 0;
 *   - orders m run over [-(2N-1), 2N-1], exactly M = 4N-1 residues mod M;
 *   - coefficient layout (m-major): orders in the sequence 0, 1, -1, 2, -2, ...,
 *     2N-1, -(2N-1); inside each order the degrees k = |m| .. 2N-1; values are
 *     complex, interleaved (re, im);
 *   - grid layout: [2N rows l][M columns], row l = l-th node in ascending x,
 *     column j = phi_j; the ALT output g uses the same shape with order m in
 *     column (m mod M).
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;

static const ld PI_L = 3.141592653589793238462643383279502884L;

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Start of the block of order m in the m-major coefficient layout
 * (complex entries, not reals). */
long long oracle_coef_offset(int N, int m)
{
    long long a = m < 0 ? -(long long)m : m;
    long long twoN = 2LL * N;
    if (a == 0) return 0;
    long long off = twoN * (2 * a - 1) - a * (a - 1);
    if (m < 0) off += twoN - a;
    return off;
}

/* Legendre polynomial P_n(t) and P_{n-1}(t) by the three-term recurrence
 * (j+1) P_{j+1} = (2j+1) t P_j - j P_{j-1}. */
static void legendre_pn(int n, ld t, ld *pn, ld *pnm1)
{
    ld p0 = 1.0L, p1 = t;
    if (n == 0) { *pn = 1.0L; *pnm1 = 0.0L; return; }
    for (int j = 1; j < n; ++j) {
        ld p2 = ((2 * j + 1) * t * p1 - j * p0) / (j + 1);
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *pnm1 = p0;
}

/* n-point Gauss-Legendre rule (Section 1: the 2N-point rule in x = cos(theta)).
 * Newton's method on P_n from the guess cos(pi (i + 3/4) / (n + 1/2)); the
 * derivative is P_n' = n (t P_n - P_{n-1}) / (t^2 - 1); weights
 * w = 2 / ((1 - t^2) P_n'(t)^2).  Nodes are returned ascending; the rule is
 * made exactly symmetric (x[n-1-i] = -x[i], equal weights). */
int oracle_gauss_legendre(int n, double *x_out, double *w_out)
{
    if (n < 1 || !x_out || !w_out) return -1;
    int half = (n + 1) / 2;
    for (int i = 0; i < half; ++i) {
        /* i-th largest root */
        ld t = cosl(PI_L * (i + 0.75L) / (n + 0.5L));
        ld pn, pnm1, dp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            legendre_pn(n, t, &pn, &pnm1);
            dp = n * (t * pn - pnm1) / (t * t - 1.0L);
            ld dt = pn / dp;
            t -= dt;
            if (fabsl(dt) <= 1e-19L * (fabsl(t) > 1e-3L ? fabsl(t) : 1e-3L)) break;
        }
        legendre_pn(n, t, &pn, &pnm1);
        dp = n * (t * pn - pnm1) / (t * t - 1.0L);
        ld w = 2.0L / ((1.0L - t * t) * dp * dp);
        if (2 * i + 1 == n) t = 0.0L; /* middle node of an odd rule */
        x_out[n - 1 - i] = (double)t;
        x_out[i] = (double)(-t);
        w_out[n - 1 - i] = (double)w;
        w_out[i] = (double)w;
    }
    return 0;
}

/* Pbar_k^m(t) for k = m .. kmax, L2-normalised on [-1,1], no Condon-Shortley
 * phase, by the standard stable recurrences:
 *   Pbar_0^0 = 1/sqrt(2),
 *   Pbar_m^m = sqrt((2m+1)/(2m)) s Pbar_{m-1}^{m-1},  s = sqrt(1 - t^2),
 *   Pbar_{m+1}^m = sqrt(2m+3) t Pbar_m^m,
 *   Pbar_k^m = a_k (t Pbar_{k-1}^m - b_k Pbar_{k-2}^m),
 *     a_k = sqrt((4k^2-1)/(k^2-m^2)),  b_k = sqrt(((k-1)^2-m^2)/(4(k-1)^2-1)).
 * Long double throughout (see the header for the exponent-range argument). */
static void plm_column_ld(int m, int kmax, ld t, ld *out)
{
    ld s = sqrtl((1.0L - t) * (1.0L + t));
    ld p = 1.0L / sqrtl(2.0L);
    for (int i = 1; i <= m; ++i)
        p *= sqrtl((ld)(2 * i + 1) / (ld)(2 * i)) * s;
    out[0] = p;
    if (kmax == m) return;
    ld p1 = sqrtl((ld)(2 * m + 3)) * t * p;
    out[1] = p1;
    ld p0 = p;
    for (int k = m + 2; k <= kmax; ++k) {
        ld kk = k, mm = m;
        ld a = sqrtl((4.0L * kk * kk - 1.0L) / (kk * kk - mm * mm));
        ld b = sqrtl(((kk - 1) * (kk - 1) - mm * mm) / (4.0L * (kk - 1) * (kk - 1) - 1.0L));
        ld p2 = a * (t * p1 - b * p0);
        out[k - m] = p2;
        p0 = p1;
        p1 = p2;
    }
}

int oracle_plm(int m, int kmax, double t, double *out)
{
    if (m < 0 || kmax < m || !out) return -1;
    ld *tmp = (ld *)malloc(sizeof(ld) * (size_t)(kmax - m + 1));
    if (!tmp) return -2;
    plm_column_ld(m, kmax, (ld)t, tmp);
    for (int k = m; k <= kmax; ++k) out[k - m] = (double)tmp[k - m];
    free(tmp);
    return 0;
}

/* Forward ALT for every order (Section 1, ALT definition; Section 3.1.1):
 * g[l][m mod M] = sum_{k=|m|}^{2N-1} beta_{k,m} Pbar_k^{|m|}(x_l).
 * beta: complex m-major [4N^2]; g: complex [2N][M]. */
int oracle_alt_forward_grid(int N, const double *x, const double *beta, double *g)
{
    if (N < 1) return -1;
    const int n = 2 * N, M = 4 * N - 1;
    int bad = 0;
#pragma omp parallel
    {
        ld *col = (ld *)malloc(sizeof(ld) * (size_t)n);
        if (!col) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int a = 0; a < n; ++a) {
            for (int l = 0; l < n; ++l) {
                if (!col) continue;
                plm_column_ld(a, n - 1, (ld)x[l], col);
                for (int sgn = 0; sgn < (a == 0 ? 1 : 2); ++sgn) {
                    int m = sgn ? -a : a;
                    const double *bm = beta + 2 * oracle_coef_offset(N, m);
                    ld re = 0.0L, im = 0.0L;
                    for (int k = a; k < n; ++k) {
                        re += col[k - a] * (ld)bm[2 * (k - a)];
                        im += col[k - a] * (ld)bm[2 * (k - a) + 1];
                    }
                    int c = ((m % M) + M) % M;
                    g[2 * ((size_t)l * M + c)] = (double)re;
                    g[2 * ((size_t)l * M + c) + 1] = (double)im;
                }
            }
        }
        free(col);
    }
    return bad ? -2 : 0;
}

/* Forward ALT for every order at a list of nodes (Section 1, ALT
 * definition): g_rows[i][m mod M] = sum_k beta_{k,m} Pbar_k^{|m|}(x_{rows[i]}).
 * g_rows: complex [n_rows][M]. */
int oracle_alt_forward_rows(int N, const double *x, const double *beta, int n_rows, const int *rows,
                            double *g_rows)
{
    if (N < 1 || n_rows < 0) return -1;
    const int n = 2 * N, M = 4 * N - 1;
    for (int i = 0; i < n_rows; ++i)
        if (rows[i] < 0 || rows[i] >= n) return -1;
    int bad = 0;
#pragma omp parallel
    {
        ld *col = (ld *)malloc(sizeof(ld) * (size_t)n);
        if (!col) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int i = 0; i < n_rows; ++i) {
            for (int a = 0; a < n; ++a) {
                if (!col) continue;
                plm_column_ld(a, n - 1, (ld)x[rows[i]], col);
                for (int sgn = 0; sgn < (a == 0 ? 1 : 2); ++sgn) {
                    int m = sgn ? -a : a;
                    const double *bm = beta + 2 * oracle_coef_offset(N, m);
                    ld re = 0.0L, im = 0.0L;
                    for (int k = a; k < n; ++k) {
                        re += col[k - a] * (ld)bm[2 * (k - a)];
                        im += col[k - a] * (ld)bm[2 * (k - a) + 1];
                    }
                    int c = ((m % M) + M) % M;
                    g_rows[2 * ((size_t)i * M + c)] = (double)re;
                    g_rows[2 * ((size_t)i * M + c) + 1] = (double)im;
                }
            }
        }
        free(col);
    }
    return bad ? -2 : 0;
}

/* Forward ALT for a list of orders |m|: out[i][s][l] (complex), s = 0 for +|m|
 * and 1 for -|m| (for |m| = 0 both slots hold order 0). */
int oracle_alt_forward_orders(int N, const double *x, const double *beta,
                              int n_orders, const int *absm, double *out)
{
    if (N < 1) return -1;
    const int n = 2 * N;
    for (int i = 0; i < n_orders; ++i)
        if (absm[i] < 0 || absm[i] >= n) return -1;
    int bad = 0;
#pragma omp parallel
    {
        ld *col = (ld *)malloc(sizeof(ld) * (size_t)n);
        if (!col) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int i = 0; i < n_orders; ++i) {
            for (int l = 0; l < n; ++l) {
                if (!col) continue;
                int a = absm[i];
                plm_column_ld(a, n - 1, (ld)x[l], col);
                for (int sgn = 0; sgn < 2; ++sgn) {
                    int m = sgn ? -a : a;
                    const double *bm = beta + 2 * oracle_coef_offset(N, m);
                    ld re = 0.0L, im = 0.0L;
                    for (int k = a; k < n; ++k) {
                        re += col[k - a] * (ld)bm[2 * (k - a)];
                        im += col[k - a] * (ld)bm[2 * (k - a) + 1];
                    }
                    size_t o = 2 * (((size_t)i * 2 + sgn) * n + l);
                    out[o] = (double)re;
                    out[o + 1] = (double)im;
                }
            }
        }
        free(col);
    }
    return bad ? -2 : 0;
}

/* Transposed ALT for every order (Section 3.1.1: B = A^T W):
 * beta_{k,m} = sum_l w_l Pbar_k^{|m|}(x_l) g[l][m mod M].
 * With w == NULL the weights are omitted (plain transpose A^T, used by the
 * adjoint).  g: complex [2N][M]; beta: complex m-major [4N^2]. */
int oracle_alt_transpose_grid(int N, const double *x, const double *w,
                              const double *g, double *beta)
{
    if (N < 1) return -1;
    const int n = 2 * N, M = 4 * N - 1;
    int bad = 0;
#pragma omp parallel
    {
        ld *tab = (ld *)malloc(sizeof(ld) * (size_t)n * (size_t)n);
        if (!tab) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int a = 0; a < n; ++a) {
            if (!tab) continue;
            int len = n - a;
            for (int l = 0; l < n; ++l) plm_column_ld(a, n - 1, (ld)x[l], tab + (size_t)l * len);
            for (int sgn = 0; sgn < (a == 0 ? 1 : 2); ++sgn) {
                int m = sgn ? -a : a;
                int c = ((m % M) + M) % M;
                double *bm = beta + 2 * oracle_coef_offset(N, m);
                for (int k = a; k < n; ++k) {
                    ld re = 0.0L, im = 0.0L;
                    for (int l = 0; l < n; ++l) {
                        ld p = tab[(size_t)l * len + (k - a)];
                        if (w) p *= (ld)w[l];
                        re += p * (ld)g[2 * ((size_t)l * M + c)];
                        im += p * (ld)g[2 * ((size_t)l * M + c) + 1];
                    }
                    bm[2 * (k - a)] = (double)re;
                    bm[2 * (k - a) + 1] = (double)im;
                }
            }
        }
        free(tab);
    }
    return bad ? -2 : 0;
}

/* Transposed ALT for a list of orders.  gin[i][s][l] (complex, same slots as
 * oracle_alt_forward_orders) -> bout[i][s][k - |m|] (complex, 2N - |m| each,
 * packed with stride 2N per slot). */
int oracle_alt_transpose_orders(int N, const double *x, const double *w,
                                int n_orders, const int *absm,
                                const double *gin, double *bout)
{
    if (N < 1) return -1;
    const int n = 2 * N;
    for (int i = 0; i < n_orders; ++i)
        if (absm[i] < 0 || absm[i] >= n) return -1;
    int bad = 0;
#pragma omp parallel
    {
        ld *tab = (ld *)malloc(sizeof(ld) * (size_t)n * (size_t)n);
        if (!tab) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < n_orders; ++i) {
            if (!tab) continue;
            int a = absm[i], len = n - a;
            for (int l = 0; l < n; ++l) plm_column_ld(a, n - 1, (ld)x[l], tab + (size_t)l * len);
            for (int sgn = 0; sgn < 2; ++sgn) {
                const double *gi = gin + 2 * (((size_t)i * 2 + sgn) * n);
                double *bo = bout + 2 * (((size_t)i * 2 + sgn) * n);
                for (int k = a; k < n; ++k) {
                    ld re = 0.0L, im = 0.0L;
                    for (int l = 0; l < n; ++l) {
                        ld p = tab[(size_t)l * len + (k - a)];
                        if (w) p *= (ld)w[l];
                        re += p * (ld)gi[2 * l];
                        im += p * (ld)gi[2 * l + 1];
                    }
                    bo[2 * (k - a)] = (double)re;
                    bo[2 * (k - a) + 1] = (double)im;
                }
            }
        }
        free(tab);
    }
    return bad ? -2 : 0;
}

/* Table of cos(pi r / M), sin(pi r / M) for r in [0, 2M). */
static int phase_table(int M, ld **ct, ld **st)
{
    *ct = (ld *)malloc(sizeof(ld) * 2 * (size_t)M);
    *st = (ld *)malloc(sizeof(ld) * 2 * (size_t)M);
    if (!*ct || !*st) { free(*ct); free(*st); return -2; }
    for (int r = 0; r < 2 * M; ++r) {
        (*ct)[r] = cosl(PI_L * r / M);
        (*st)[r] = sinl(PI_L * r / M);
    }
    return 0;
}

/* phi synthesis (Section 1, f = sum_m g(m, theta) e^{i m phi}):
 * f[l][j] = sum_{m=-(2N-1)}^{2N-1} g[l][m mod M] exp(i pi m (2j+1) / M),
 * for the listed rows l only (rows == NULL: all 2N rows).  The phase index
 * r = m (2j+1) mod 2M is reduced exactly in integers.
 * g: complex [2N][M]; f_rows: complex [n_rows][M]. */
int oracle_dft_synthesis(int N, const double *g, int n_rows, const int *rows, double *f_rows)
{
    if (N < 1) return -1;
    const int M = 4 * N - 1, n = 2 * N;
    if (!rows) n_rows = n;
    ld *ct, *st;
    if (phase_table(M, &ct, &st)) return -2;
#pragma omp parallel for schedule(dynamic, 4) collapse(2)
    for (int i = 0; i < n_rows; ++i) {
        for (int j = 0; j < M; ++j) {
            int l = rows ? rows[i] : i;
            const double *gl = g + 2 * (size_t)l * M;
            ld re = 0.0L, im = 0.0L;
            for (int m = -(n - 1); m <= n - 1; ++m) {
                int c = ((m % M) + M) % M;
                long long r = ((long long)m * (2 * j + 1)) % (2LL * M);
                if (r < 0) r += 2LL * M;
                ld gr = gl[2 * c], gi = gl[2 * c + 1];
                re += gr * ct[r] - gi * st[r];
                im += gr * st[r] + gi * ct[r];
            }
            f_rows[2 * ((size_t)i * M + j)] = (double)re;
            f_rows[2 * ((size_t)i * M + j) + 1] = (double)im;
        }
    }
    free(ct);
    free(st);
    return 0;
}

/* phi analysis: g[l][m mod M] = scale * sum_j f[l][j] exp(-i pi m (2j+1)/M).
 * scale = 1/M gives the inverse of the synthesis (the trapezoid rule in phi is
 * exact for the M residues); scale = 1 gives its conjugate transpose, used by
 * the adjoint.  Each row is transformed on its own, so any subset of grid rows
 * may be passed; f_rows and g_rows are complex [n_rows][M]. */
int oracle_dft_analysis(int N, const double *f_rows, int n_rows, double scale, double *g_rows)
{
    if (N < 1 || n_rows < 0) return -1;
    const int M = 4 * N - 1, n = 2 * N;
    ld *ct, *st;
    if (phase_table(M, &ct, &st)) return -2;
#pragma omp parallel for schedule(dynamic, 4) collapse(2)
    for (int i = 0; i < n_rows; ++i) {
        for (int m = -(n - 1); m <= n - 1; ++m) {
            const double *fl = f_rows + 2 * (size_t)i * M;
            ld re = 0.0L, im = 0.0L;
            for (int j = 0; j < M; ++j) {
                long long r = ((long long)m * (2 * j + 1)) % (2LL * M);
                if (r < 0) r += 2LL * M;
                ld fr = fl[2 * j], fi = fl[2 * j + 1];
                /* multiply by exp(-i pi r / M) */
                re += fr * ct[r] + fi * st[r];
                im += fi * ct[r] - fr * st[r];
            }
            int c = ((m % M) + M) % M;
            g_rows[2 * ((size_t)i * M + c)] = (double)(re * (ld)scale);
            g_rows[2 * ((size_t)i * M + c) + 1] = (double)(im * (ld)scale);
        }
    }
    free(ct);
    free(st);
    return 0;
}
