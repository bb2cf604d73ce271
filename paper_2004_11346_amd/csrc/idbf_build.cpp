// Plan construction of the fast ALT (host, FP64).
//
// For every order |m| and parity the half matrix (Section 3.1.2) is
// partitioned (Section 3.2): nearly square row blocks (eq. nb), then 2 x 2
// splits of every block crossed by the turning-point curve
// t*_{k,m} = arcsin(sqrt(m^2 - 1/4) / (k + 1/2)) (eq. new5) until it has at
// most n0 rows and columns.  Then (Section 3.3):
//   oscillatory blocks      -> interpolative decomposition butterfly (Section 2.2)
//                              built from column / row IDs on mock-Chebyshev
//                              (or random) samples (Section 2.1);
//   non-oscillatory blocks  -> trimmed to the box of non-negligible entries,
//                              then the randomized-sampling SVD of Algorithm 1
//                              (Section 2.3), or dropped when empty;
//   turning-point blocks    -> trimmed, kept dense.
// A factorization is kept only when it stores fewer entries than the dense
// block it replaces and reproduces it to the requested tolerance.
#include "idbf_build.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <sstream>
#include <thread>

#include "linalg.h"

namespace sht {
namespace idbf {

int64_t Block::stored() const {
    switch (type) {
        case kDense: return gen ? 0 : (int64_t)D.size();
        case kLowRank: return (int64_t)U.size() + (int64_t)V.size();
        default: {
            int64_t s = 0;
            for (auto &lv : bf.col)
                for (auto &id : lv) s += (int64_t)id.T.size();
            for (auto &lv : bf.row)
                for (auto &id : lv) s += (int64_t)id.T.size();
            for (auto &m : bf.S) s += (int64_t)m.size();
            return s;
        }
    }
}

void rec_step(const LegendreTables &lt, int a, double x, int k, RecState &s) {
    const double *c = &lt.coef[2 * (tri_offset(lt.N, a) + (k + 1 - a))];
    const double p2 = c[0] * (x * s.p1 - c[1] * s.p0);
    s.pm2 = s.p0;
    s.p0 = s.p1;
    s.p1 = p2;
    if (std::fabs(s.p1) > 0x1p200) {
        s.pm2 *= 0x1p-200;
        s.p0 *= 0x1p-200;
        s.p1 *= 0x1p-200;
        s.e += 200;
    }
}

RecState gen_state(const LegendreTables &lt, int a, int parity, const Block &b, int r, int col) {
    const int q = (col - b.ck_c0) >> 4;
    RecState s = b.ck[(size_t)(r - b.r0) * b.ck_n + q];
    const double x = lt.xh[r];
    for (int c = b.ck_c0 + 16 * q; c < col; ++c) {
        const int k = a + parity + 2 * c;
        rec_step(lt, a, x, k, s);
        rec_step(lt, a, x, k + 1, s);
    }
    return s;
}

double gen_value(const RecState &s) { return s.e < -1074 ? 0.0 : s.p1 * std::ldexp(1.0, s.e); }

namespace {

typedef std::mt19937_64 Rng;

// Task matrix accessor (row-major N x cols), optionally transposed.
struct View {
    const double *a;
    int ld;
    bool trans;
    double operator()(int r, int c) const { return trans ? a[(size_t)c * ld + r] : a[(size_t)r * ld + c]; }
};

// Mock-Chebyshev sample: Chebyshev-Lobatto points mapped onto [lo, hi), each
// replaced by the nearest index not taken yet (deterministic).
std::vector<int> mock_cheb(int lo, int hi, int ns) {
    const int n = hi - lo;
    std::vector<int> out;
    if (ns >= n) {
        out.resize(n);
        std::iota(out.begin(), out.end(), lo);
        return out;
    }
    std::vector<char> used(n, 0);
    for (int i = 0; i < ns; ++i) {
        double p = (n - 1) * 0.5 * (1.0 - std::cos(M_PI * i / std::max(1, ns - 1)));
        int c = (int)std::lround(p);
        int best = -1;
        for (int d = 0; d < n; ++d) {
            int u = c - d, v = c + d;
            if (u >= 0 && u < n && !used[u]) { best = u; break; }
            if (v >= 0 && v < n && !used[v]) { best = v; break; }
        }
        used[best] = 1;
        out.push_back(lo + best);
    }
    std::sort(out.begin(), out.end());
    return out;
}

std::vector<int> random_sample(int lo, int hi, int ns, Rng &rng) {
    const int n = hi - lo;
    std::vector<int> all(n);
    std::iota(all.begin(), all.end(), lo);
    if (ns >= n) return all;
    for (int i = 0; i < ns; ++i) {
        std::uniform_int_distribution<int> d(i, n - 1);
        std::swap(all[i], all[d(rng)]);
    }
    all.resize(ns);
    std::sort(all.begin(), all.end());
    return all;
}

struct Ctx {
    const sht_plan_opts *o;
    double tol;  // absolute tolerance of every factorization
    Rng rng;
};

// Column ID of K(rows [lo, hi), cand) (Section 2.1): pivoted QR of the sampled
// rows, truncated at the tolerance; T = R11^{-1} R12.  With id_check (the
// default) at least n + 8 rows are sampled, the ID is verified on a second
// sample of rows and on failure repeated with every row; without it the ID is
// taken from t min(n, r_k) sampled rows as written in Section 2.1.
ID column_id(const View &K, int lo, int hi, const std::vector<int> &cand, Ctx &cx) {
    const int n = (int)cand.size(), nrows = hi - lo;
    const bool check = cx.o->id_check != 0;
    const int want = check ? std::max(n + 8, cx.o->oversample * std::min(n, cx.o->rk))
                           : std::max(1, cx.o->oversample * std::min(n, cx.o->rk));
    for (int attempt = 0; attempt < 2; ++attempt) {
        std::vector<int> s = attempt == 0 ? (cx.o->sampling == SHT_SAMPLE_RANDOM ? random_sample(lo, hi, want, cx.rng)
                                                                                : mock_cheb(lo, hi, want))
                                          : mock_cheb(lo, hi, nrows);
        const int ns = (int)s.size();
        std::vector<double> M((size_t)ns * n);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < ns; ++i) M[i + (size_t)j * ns] = K(s[i], cand[j]);
        std::vector<int> perm;
        const int kmax = std::min(n, cx.o->rk);
        int k = la::pivoted_qr(ns, n, M.data(), ns, cx.tol, kmax, perm);
        ID id;
        id.capped = k == kmax && k < n;
        id.skel.assign(perm.begin(), perm.begin() + k);
        id.red.assign(perm.begin() + k, perm.end());
        const int nred = n - k;
        std::vector<double> Tc((size_t)k * nred);
        if (k > 0 && nred > 0) la::solve_upper(k, n, M.data(), ns, Tc.data());
        id.T.resize((size_t)k * nred);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < nred; ++j) id.T[(size_t)i * nred + j] = Tc[i + (size_t)j * k];
        if (k == 0 && nred > 0) {
            // numerically zero block: nothing to keep
        }
        for (int i = 0; i < k; ++i) id.skel_glob.push_back(cand[id.skel[i]]);
        if (!check || attempt == 1 || ns == nrows || nred == 0) return id;
        // verification on rows outside the sample
        std::vector<int> chk = random_sample(lo, hi, std::min(nrows, 48), cx.rng);
        double worst = 0.0;
        for (int r : chk) {
            for (int j = 0; j < nred; ++j) {
                double v = K(r, cand[id.red[j]]);
                for (int i = 0; i < k; ++i) v -= K(r, cand[id.skel[i]]) * id.T[(size_t)i * nred + j];
                worst = std::max(worst, std::fabs(v));
            }
        }
        if (worst <= 4.0 * cx.tol) return id;
    }
    return ID();  // unreachable
}

ID row_id(const View &K, const std::vector<int> &cand, int lo, int hi, Ctx &cx) {
    View Kt{K.a, K.ld, !K.trans};
    return column_id(Kt, lo, hi, cand, cx);
}

inline int node_lo(int lo, int n, int level, int t) { return lo + (int)(((int64_t)t * n) >> level); }

bool build_butterfly(const View &K, int r0, int r1, int c0, int c1, Ctx &cx, Butterfly &bf) {
    const int nr = r1 - r0, nc = c1 - c0;
    const int leaf = std::max(2, cx.o->leaf);
    int L = 0;
    while ((std::min(nr, nc) >> (L + 1)) >= leaf) ++L;
    if (L < 1) return false;
    const int h = L / 2;
    bf.L = L;
    bf.h = h;
    bf.r0 = r0;
    bf.r1 = r1;
    bf.c0 = c0;
    bf.c1 = c1;
    bf.col.assign(h + 1, {});
    bf.row.assign(L - h + 1, {});
    // column pass
    for (int l = 0; l <= h; ++l) {
        const int nA = 1 << l, nB = 1 << (L - l);
        bf.col[l].resize((size_t)nA * nB);
        for (int A = 0; A < nA; ++A) {
            const int alo = node_lo(r0, nr, l, A), ahi = node_lo(r0, nr, l, A + 1);
            for (int B = 0; B < nB; ++B) {
                std::vector<int> cand;
                if (l == 0) {
                    for (int c = node_lo(c0, nc, L, B); c < node_lo(c0, nc, L, B + 1); ++c) cand.push_back(c);
                } else {
                    const int Ap = A >> 1, nBp = 1 << (L - l + 1);
                    const ID &i1 = bf.col[l - 1][(size_t)Ap * nBp + 2 * B];
                    const ID &i2 = bf.col[l - 1][(size_t)Ap * nBp + 2 * B + 1];
                    cand = i1.skel_glob;
                    cand.insert(cand.end(), i2.skel_glob.begin(), i2.skel_glob.end());
                }
                bf.col[l][(size_t)A * nB + B] = column_id(K, alo, ahi, cand, cx);
            }
        }
    }
    // row pass
    for (int l = 0; l <= L - h; ++l) {
        const int nA = 1 << (L - l), nB = 1 << l;
        bf.row[l].resize((size_t)nA * nB);
        for (int A = 0; A < nA; ++A) {
            for (int B = 0; B < nB; ++B) {
                const int blo = node_lo(c0, nc, l, B), bhi = node_lo(c0, nc, l, B + 1);
                std::vector<int> cand;
                if (l == 0) {
                    for (int r = node_lo(r0, nr, L, A); r < node_lo(r0, nr, L, A + 1); ++r) cand.push_back(r);
                } else {
                    const int Bp = B >> 1, nBp = 1 << (l - 1);
                    const ID &i1 = bf.row[l - 1][(size_t)(2 * A) * nBp + Bp];
                    const ID &i2 = bf.row[l - 1][(size_t)(2 * A + 1) * nBp + Bp];
                    cand = i1.skel_glob;
                    cand.insert(cand.end(), i2.skel_glob.begin(), i2.skel_glob.end());
                }
                bf.row[l][(size_t)A * nB + B] = row_id(K, cand, blo, bhi, cx);
            }
        }
    }
    // middle couplings
    const int nA = 1 << h, nB = 1 << (L - h);
    bf.S.resize((size_t)nA * nB);
    for (int A = 0; A < nA; ++A)
        for (int B = 0; B < nB; ++B) {
            const ID &ri = bf.row[L - h][(size_t)A * nB + B];
            const ID &ci = bf.col[h][(size_t)A * nB + B];
            std::vector<double> &S = bf.S[(size_t)A * nB + B];
            S.resize((size_t)ri.k() * ci.k());
            for (int i = 0; i < ri.k(); ++i)
                for (int j = 0; j < ci.k(); ++j) S[(size_t)i * ci.k() + j] = K(ri.skel_glob[i], ci.skel_glob[j]);
        }
    // a butterfly with an ID cut at the rank cap does not compress its block
    // to the tolerance: leave the block to the dense (regenerated) path
    // (with id_check; without it the truncated butterfly is kept)
    if (cx.o->id_check == 0) return true;
    for (const auto *ids : {&bf.col, &bf.row})
        for (const auto &lv : *ids)
            for (const ID &id : lv)
                if (id.capped) return false;
    return true;
}

// Randomized-sampling low-rank factorization, Algorithm 1 (Section 2.3),
// rank r, oversampling q.  Result A ~= U V^T (Sigma folded into U).
bool rsvd(const View &K, int r0, int r1, int c0, int c1, int r, Ctx &cx, std::vector<double> &U,
          std::vector<double> &V, int &rank) {
    const int m = r1 - r0, n = c1 - c0;
    if (r > std::min(m, n)) return false;
    const int q = std::max(1, cx.o->rsvd_q);
    auto rp = [&](int total, int cnt) { return random_sample(0, total, std::min(total, cnt), cx.rng); };
    // Pi_col: first r pivots of the pivoted QR of A(R, :)
    std::vector<int> Rs = rp(m, r * q), Cs = rp(n, r * q);
    std::vector<int> pcol, prow;
    {
        std::vector<double> M((size_t)Rs.size() * n);
        for (int j = 0; j < n; ++j)
            for (size_t i = 0; i < Rs.size(); ++i) M[i + j * Rs.size()] = K(r0 + Rs[i], c0 + j);
        std::vector<int> perm;
        int k = la::pivoted_qr((int)Rs.size(), n, M.data(), (int)Rs.size(), 0.0, r, perm);
        pcol.assign(perm.begin(), perm.begin() + std::min(k, r));
    }
    {
        std::vector<double> M((size_t)Cs.size() * m);
        for (int j = 0; j < m; ++j)
            for (size_t i = 0; i < Cs.size(); ++i) M[i + j * Cs.size()] = K(r0 + j, c0 + Cs[i]);
        std::vector<int> perm;
        int k = la::pivoted_qr((int)Cs.size(), m, M.data(), (int)Cs.size(), 0.0, r, perm);
        prow.assign(perm.begin(), perm.begin() + std::min(k, r));
    }
    const int rc = (int)pcol.size(), rr = (int)prow.size();
    if (rc == 0 || rr == 0) {
        rank = 0;
        U.clear();
        V.clear();
        return true;
    }
    // Q_col = orth(A(:, Pi_col)) (m x rc); Q_row = orth(A(Pi_row, :)^T) (n x rr)
    std::vector<double> Qc((size_t)m * rc), Qr((size_t)n * rr);
    {
        std::vector<double> M((size_t)m * rc);
        for (int j = 0; j < rc; ++j)
            for (int i = 0; i < m; ++i) M[i + (size_t)j * m] = K(r0 + i, c0 + pcol[j]);
        std::vector<int> perm;
        std::vector<double> tau;
        la::pivoted_qr(m, rc, M.data(), m, 0.0, rc, perm, &tau);
        la::form_q(m, (int)tau.size(), M.data(), m, tau, Qc.data());
        if ((int)tau.size() < rc) return false;
    }
    {
        std::vector<double> M((size_t)n * rr);
        for (int j = 0; j < rr; ++j)
            for (int i = 0; i < n; ++i) M[i + (size_t)j * n] = K(r0 + prow[j], c0 + i);
        std::vector<int> perm;
        std::vector<double> tau;
        la::pivoted_qr(n, rr, M.data(), n, 0.0, rr, perm, &tau);
        la::form_q(n, (int)tau.size(), M.data(), n, tau, Qr.data());
        if ((int)tau.size() < rr) return false;
    }
    // I = [Pi_row, S_row], J = [Pi_col, S_col]
    std::vector<int> I = prow, J = pcol;
    {
        std::vector<int> sr = rp(m, r), sc = rp(n, r);
        I.insert(I.end(), sr.begin(), sr.end());
        J.insert(J.end(), sc.begin(), sc.end());
    }
    const int ni = (int)I.size(), nj = (int)J.size();
    // M = pinv(Q_col(I, :)) A(I, J) pinv(Q_row(J, :)^T)
    std::vector<double> QcI((size_t)ni * rc), QrJt((size_t)rr * nj), AIJ((size_t)ni * nj);
    for (int j = 0; j < rc; ++j)
        for (int i = 0; i < ni; ++i) QcI[i + (size_t)j * ni] = Qc[I[i] + (size_t)j * m];
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < rr; ++i) QrJt[i + (size_t)j * rr] = Qr[J[j] + (size_t)i * n];
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) AIJ[i + (size_t)j * ni] = K(r0 + I[i], c0 + J[j]);
    std::vector<double> P1((size_t)rc * ni), P2((size_t)nj * rr);
    la::pinv(ni, rc, QcI.data(), ni, 1e-14, P1.data());
    la::pinv(rr, nj, QrJt.data(), rr, 1e-14, P2.data());
    std::vector<double> T1((size_t)rc * nj), Mm((size_t)rc * rr);
    la::gemm(false, false, rc, nj, ni, 1.0, P1.data(), rc, AIJ.data(), ni, 0.0, T1.data(), rc);
    la::gemm(false, false, rc, rr, nj, 1.0, T1.data(), rc, P2.data(), nj, 0.0, Mm.data(), rc);
    // SVD of M (rc x rr), truncated at the tolerance
    const bool tall = rc >= rr;
    const int mm = tall ? rc : rr, nn = tall ? rr : rc;
    std::vector<double> W((size_t)mm * nn), sv(nn), Vv((size_t)nn * nn);
    for (int j = 0; j < nn; ++j)
        for (int i = 0; i < mm; ++i) W[i + (size_t)j * mm] = tall ? Mm[i + (size_t)j * rc] : Mm[j + (size_t)i * rc];
    la::jacobi_svd(mm, nn, W.data(), mm, sv.data(), Vv.data());
    // M = UM diag(sv) VM^T with UM (rc x nn), VM (rr x nn)
    int kk = 0;
    while (kk < nn && sv[kk] > cx.tol * 0.1) ++kk;
    rank = kk;
    U.assign((size_t)m * kk, 0.0);
    V.assign((size_t)n * kk, 0.0);
    for (int t = 0; t < kk; ++t) {
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int p = 0; p < rc; ++p) {
                double um = tall ? W[p + (size_t)t * mm] : Vv[p + (size_t)t * nn];
                s += Qc[i + (size_t)p * m] * um;
            }
            U[(size_t)i * kk + t] = s * sv[t];
        }
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int p = 0; p < rr; ++p) {
                double vm = tall ? Vv[p + (size_t)t * nn] : W[p + (size_t)t * mm];
                s += Qr[i + (size_t)p * n] * vm;
            }
            V[(size_t)i * kk + t] = s;
        }
    }
    return true;
}

double lowrank_check(const View &K, const Block &b, Ctx &cx) {
    const int m = b.r1 - b.r0, n = b.c1 - b.c0;
    std::uniform_int_distribution<int> dr(0, m - 1), dc(0, n - 1);
    double worst = 0.0;
    for (int s = 0; s < 400; ++s) {
        int i = dr(cx.rng), j = dc(cx.rng);
        double v = K(b.r0 + i, b.c0 + j);
        for (int t = 0; t < b.rank; ++t) v -= b.U[(size_t)i * b.rank + t] * b.V[(size_t)j * b.rank + t];
        worst = std::max(worst, std::fabs(v));
    }
    return worst;
}

// Apply helpers (host, R right-hand sides, rows of R contiguous).
void id_gather(const ID &id, int R, const double *in /* |cand| x R */, double *out /* k x R */) {
    const int k = id.k(), nred = (int)id.red.size();
    for (int i = 0; i < k; ++i) {
        double *o = out + (size_t)i * R;
        const double *s = in + (size_t)id.skel[i] * R;
        for (int r = 0; r < R; ++r) o[r] = s[r];
        for (int j = 0; j < nred; ++j) {
            double t = id.T[(size_t)i * nred + j];
            const double *x = in + (size_t)id.red[j] * R;
            for (int r = 0; r < R; ++r) o[r] += t * x[r];
        }
    }
}

void id_scatter_add(const ID &id, int R, const double *u /* k x R */, double *out /* |cand| x R */) {
    const int k = id.k(), nred = (int)id.red.size();
    for (int i = 0; i < k; ++i) {
        double *o = out + (size_t)id.skel[i] * R;
        for (int r = 0; r < R; ++r) o[r] += u[(size_t)i * R + r];
    }
    for (int j = 0; j < nred; ++j) {
        double *o = out + (size_t)id.red[j] * R;
        for (int i = 0; i < k; ++i) {
            double t = id.T[(size_t)i * nred + j];
            for (int r = 0; r < R; ++r) o[r] += t * u[(size_t)i * R + r];
        }
    }
}

typedef std::vector<double> Vec;

void butterfly_forward(const Butterfly &bf, int R, const double *x /* task cols */, double *y /* task rows, += */) {
    const int L = bf.L, h = bf.h;
    std::vector<std::vector<Vec>> z(h + 1);
    for (int l = 0; l <= h; ++l) {
        const int nA = 1 << l, nB = 1 << (L - l);
        z[l].resize((size_t)nA * nB);
        for (int A = 0; A < nA; ++A)
            for (int B = 0; B < nB; ++B) {
                const ID &id = bf.col[l][(size_t)A * nB + B];
                Vec in;
                if (l == 0) {
                    const int clo = node_lo(bf.c0, bf.c1 - bf.c0, L, B), chi = node_lo(bf.c0, bf.c1 - bf.c0, L, B + 1);
                    in.assign(x + (size_t)clo * R, x + (size_t)chi * R);
                } else {
                    const int Ap = A >> 1, nBp = 1 << (L - l + 1);
                    const Vec &a1 = z[l - 1][(size_t)Ap * nBp + 2 * B], &a2 = z[l - 1][(size_t)Ap * nBp + 2 * B + 1];
                    in = a1;
                    in.insert(in.end(), a2.begin(), a2.end());
                }
                Vec &o = z[l][(size_t)A * nB + B];
                o.assign((size_t)id.k() * R, 0.0);
                id_gather(id, R, in.data(), o.data());
            }
    }
    // middle: u = S z
    std::vector<std::vector<Vec>> u(L - h + 1);
    {
        const int nA = 1 << h, nB = 1 << (L - h);
        u[L - h].resize((size_t)nA * nB);
        for (int A = 0; A < nA; ++A)
            for (int B = 0; B < nB; ++B) {
                const size_t ix = (size_t)A * nB + B;
                const int kr = bf.row[L - h][ix].k(), kc = bf.col[h][ix].k();
                Vec &o = u[L - h][ix];
                o.assign((size_t)kr * R, 0.0);
                const Vec &zz = z[h][ix];
                for (int i = 0; i < kr; ++i)
                    for (int j = 0; j < kc; ++j) {
                        double s = bf.S[ix][(size_t)i * kc + j];
                        for (int r = 0; r < R; ++r) o[(size_t)i * R + r] += s * zz[(size_t)j * R + r];
                    }
            }
    }
    for (int l = L - h; l >= 1; --l) {
        const int nA = 1 << (L - l), nB = 1 << l;
        const int nBp = 1 << (l - 1);
        u[l - 1].resize((size_t)(2 * nA) * nBp);
        for (int A = 0; A < nA; ++A)
            for (int Bp = 0; Bp < nBp; ++Bp) {
                const ID &c1 = bf.row[l - 1][(size_t)(2 * A) * nBp + Bp];
                const ID &c2 = bf.row[l - 1][(size_t)(2 * A + 1) * nBp + Bp];
                const int n1 = c1.k(), n2 = c2.k();
                Vec v((size_t)(n1 + n2) * R, 0.0);
                for (int B = 2 * Bp; B <= 2 * Bp + 1; ++B)
                    id_scatter_add(bf.row[l][(size_t)A * nB + B], R, u[l][(size_t)A * nB + B].data(), v.data());
                u[l - 1][(size_t)(2 * A) * nBp + Bp].assign(v.begin(), v.begin() + (size_t)n1 * R);
                u[l - 1][(size_t)(2 * A + 1) * nBp + Bp].assign(v.begin() + (size_t)n1 * R, v.end());
            }
    }
    const int nleaf = 1 << L;
    for (int A = 0; A < nleaf; ++A) {
        const int rlo = node_lo(bf.r0, bf.r1 - bf.r0, L, A), rhi = node_lo(bf.r0, bf.r1 - bf.r0, L, A + 1);
        Vec v((size_t)(rhi - rlo) * R, 0.0);
        id_scatter_add(bf.row[0][A], R, u[0][A].data(), v.data());
        for (size_t q = 0; q < v.size(); ++q) y[(size_t)rlo * R + q] += v[q];
    }
}


double butterfly_check(const View &K, const Butterfly &bf, Ctx &cx) {
    // apply to a few random vectors and compare with the dense block
    const int nr = bf.r1 - bf.r0, nc = bf.c1 - bf.c0;
    const int R = 2;
    std::normal_distribution<double> nd;
    std::vector<double> x((size_t)(bf.c1) * R, 0.0), y((size_t)bf.r1 * R, 0.0);
    for (int c = bf.c0; c < bf.c1; ++c)
        for (int r = 0; r < R; ++r) x[(size_t)c * R + r] = nd(cx.rng);
    butterfly_forward(bf, R, x.data(), y.data());
    double err = 0.0, nx = 0.0;
    for (int c = bf.c0; c < bf.c1; ++c)
        for (int r = 0; r < R; ++r) nx += x[(size_t)c * R + r] * x[(size_t)c * R + r];
    for (int i = bf.r0; i < bf.r1; ++i)
        for (int r = 0; r < R; ++r) {
            double v = 0.0;
            for (int c = bf.c0; c < bf.c1; ++c) v += K(i, c) * x[(size_t)c * R + r];
            err = std::max(err, std::fabs(v - y[(size_t)i * R + r]));
        }
    (void)nr;
    (void)nc;
    return err / std::sqrt(nx / R);  // max row error per unit-norm input
}

struct Box {
    int r0, r1, c0, c1;
};

void trim(const View &K, Box &b, double tau, bool &empty) {
    int rlo = b.r1, rhi = b.r0 - 1, clo = b.c1, chi = b.c0 - 1;
    for (int r = b.r0; r < b.r1; ++r)
        for (int c = b.c0; c < b.c1; ++c)
            if (std::fabs(K(r, c)) >= tau) {
                rlo = std::min(rlo, r);
                rhi = std::max(rhi, r);
                clo = std::min(clo, c);
                chi = std::max(chi, c);
            }
    empty = rhi < rlo;
    if (!empty) b = Box{rlo, rhi + 1, clo, chi + 1};
}

// Recurrence states of every regenerated dense block: one walk along each
// task row from degree |m|, recording the state at the 16-aligned columns the
// blocks of that row need.
void record_checkpoints(const LegendreTables &lt, Task &t) {
    const int N = lt.N, a = t.a, par = t.parity;
    std::vector<std::vector<std::pair<int, int>>> need(N);  // row -> (col, block)
    for (int bi = 0; bi < (int)t.blocks.size(); ++bi) {
        const Block &b = t.blocks[bi];
        if (!b.gen) continue;
        for (int r = b.r0; r < b.r1; ++r)
            for (int q = 0; q < b.ck_n; ++q) need[r].push_back({b.ck_c0 + 16 * q, bi});
    }
    for (int r = 0; r < N; ++r) {
        if (need[r].empty()) continue;
        std::sort(need[r].begin(), need[r].end());
        const double x = lt.xh[r];
        RecState s;
        s.p1 = lt.diag_m[(size_t)a * N + r];
        s.e = lt.diag_e[(size_t)a * N + r];
        int k = a;  // degree of s.p1
        for (const auto &cb : need[r]) {
            const int kt = a + par + 2 * cb.first;
            while (k < kt) rec_step(lt, a, x, k++, s);
            Block &b = t.blocks[cb.second];
            b.ck[(size_t)(r - b.r0) * b.ck_n + ((cb.first - b.ck_c0) >> 4)] = s;
        }
    }
}

void build_task(int N, const LegendreTables &lt, const sht_plan_opts &o, int a, int par, Task &t,
                std::vector<double> &mat, BuildStats &st) {
    t.a = a;
    t.parity = par;
    t.rows = N;
    t.cols = half_cols(N, a, par);
    t.blocks.clear();
    if (t.cols <= 0) return;
    const int cols = t.cols;
    mat.resize((size_t)N * cols);
    alt_half_matrix(lt, a, par, mat.data());
    double scale = 0.0;
    for (double v : mat) scale = std::max(scale, std::fabs(v));
    t.scale = scale;
    View K{mat.data(), cols, false};
    Ctx cx{&o, o.eps * scale, Rng(o.seed ^ (0x9E3779B97F4A7C15ULL * (uint64_t)(2 * a + par + 1)))};
    const double tau = std::ldexp(scale, -52);
    st.dense_entries += (int64_t)N * cols;

    // partition (Section 3.2)
    std::vector<double> theta(N);
    for (int r = 0; r < N; ++r) theta[r] = std::acos(lt.xh[r]);
    auto kcol = [&](int j) { return a + par + 2 * j; };
    auto tstar = [&](int k) {
        if (a == 0) return 0.0;
        double s = std::sqrt((double)a * a - 0.25) / (k + 0.5);
        return s >= 1.0 ? M_PI / 2 : std::asin(s);
    };
    auto region = [&](const Box &b) {
        if (a == 0) return (int)kOsc;
        if (theta[b.r0] > tstar(kcol(b.c0))) return (int)kOsc;
        if (theta[b.r1 - 1] < tstar(kcol(b.c1 - 1))) return (int)kNonOsc;
        return (int)kTurning;
    };
    std::vector<Box> work, done;
    const int nb = std::max(1, (int)std::lround((double)N / cols));
    // row boundaries on multiples of 64 where that keeps every block non-empty
    // (the kernels tile outputs by 64 rows)
    auto row_cut = [&](int64_t r) {
        const int64_t a64 = (r + 32) / 64 * 64;
        return (int)(N >= 64 * nb ? a64 : r);
    };
    for (int i = 0; i < nb; ++i)
        work.push_back(Box{row_cut((int64_t)i * N / nb), i + 1 == nb ? N : row_cut((int64_t)(i + 1) * N / nb), 0, cols});
    const int n0 = std::max(8, o.n0);
    while (!work.empty()) {
        Box b = work.back();
        work.pop_back();
        if (b.r1 <= b.r0 || b.c1 <= b.c0) continue;
        if (region(b) == kTurning && std::max(b.r1 - b.r0, b.c1 - b.c0) > n0) {
            int rm = (b.r0 + b.r1) / 2, cm = (b.c0 + b.c1) / 2;
            const int rm64 = (rm + 32) / 64 * 64;
            if (rm64 > b.r0 && rm64 < b.r1) rm = rm64;
            if (b.r1 - b.r0 < 2) rm = b.r1;
            if (b.c1 - b.c0 < 2) cm = b.c1;
            work.push_back(Box{b.r0, rm, b.c0, cm});
            work.push_back(Box{b.r0, rm, cm, b.c1});
            work.push_back(Box{rm, b.r1, b.c0, cm});
            work.push_back(Box{rm, b.r1, cm, b.c1});
        } else {
            done.push_back(b);
        }
    }
    std::sort(done.begin(), done.end(), [](const Box &x, const Box &y) {
        return x.r0 != y.r0 ? x.r0 < y.r0 : x.c0 < y.c0;
    });
    const int min_bf = o.min_idbf > 0 ? o.min_idbf : 4 * std::max(2, o.leaf);
    for (Box b : done) {
        Block blk;
        blk.region = region(b);
        const Box whole = b;
        if (blk.region != kOsc) {
            bool empty = false;
            trim(K, b, tau, empty);
            if (empty) {
                st.n_dropped++;
                continue;
            }
        }
        blk.r0 = b.r0;
        blk.r1 = b.r1;
        blk.c0 = b.c0;
        blk.c1 = b.c1;
        const int m = b.r1 - b.r0, n = b.c1 - b.c0;
        const int64_t dense_sz = (int64_t)m * n;
        bool chosen = false;
        if (blk.region == kOsc && std::min(m, n) >= min_bf) {
            Butterfly bf;
            if (build_butterfly(K, b.r0, b.r1, b.c0, b.c1, cx, bf)) {
                blk.type = kButterfly;
                blk.bf = std::move(bf);
                // without id_check the truncated butterfly is kept as Section 2.1
                // builds it (the sampling and rank study measures its error)
                if (blk.stored() < dense_sz &&
                    (o.id_check == 0 || butterfly_check(K, blk.bf, cx) <= 50.0 * cx.tol)) {
                    chosen = true;
                } else {
                    blk.bf = Butterfly();
                }
            }
        }
        if (!chosen && blk.region == kNonOsc && std::min(m, n) > 2 * o.rsvd_r) {
            for (int r = o.rsvd_r; !chosen && 2 * r < std::min(m, n); r *= 2) {
                std::vector<double> U, V;
                int rank = 0;
                if (!rsvd(K, b.r0, b.r1, b.c0, b.c1, r, cx, U, V, rank)) break;
                blk.type = kLowRank;
                blk.U = std::move(U);
                blk.V = std::move(V);
                blk.rank = rank;
                if (blk.stored() < dense_sz && lowrank_check(K, blk, cx) <= 4.0 * cx.tol && rank < r) {
                    chosen = true;
                } else {
                    blk.U.clear();
                    blk.V.clear();
                    blk.rank = 0;
                }
            }
        }
        if (!chosen) {
            blk.type = kDense;
            if (o.dense_gen) {
                // rows widened to multiples of 64 inside the untrimmed box:
                // the extra entries are exact (regenerated), not stored
                blk.r0 = std::max(whole.r0, blk.r0 & ~63);
                blk.r1 = std::min(whole.r1, (blk.r1 + 63) & ~63);
                blk.gen = true;
                blk.ck_c0 = b.c0 & ~15;
                blk.ck_n = (b.c1 - 1 - blk.ck_c0) / 16 + 1;
                blk.ck.resize((size_t)(blk.r1 - blk.r0) * blk.ck_n);
            } else {
                blk.D.resize((size_t)m * n);
                for (int i = 0; i < m; ++i)
                    for (int j = 0; j < n; ++j) blk.D[(size_t)i * n + j] = K(b.r0 + i, b.c0 + j);
            }
        }
        switch (blk.type) {
            case kDense:
                st.n_dense++;
                st.dense_stored += blk.stored();
                if (blk.gen) {
                    st.n_gen++;
                    st.gen_entries += (int64_t)(blk.r1 - blk.r0) * n;
                }
                break;
            case kLowRank: st.n_lowrank++; st.lowrank_stored += blk.stored(); st.max_rank = std::max(st.max_rank, blk.rank); break;
            default: {
                st.n_butterfly++;
                st.butterfly_stored += blk.stored();
                for (auto &lv : blk.bf.col)
                    for (auto &id : lv) st.max_rank = std::max(st.max_rank, id.k());
                for (auto &lv : blk.bf.row)
                    for (auto &id : lv) st.max_rank = std::max(st.max_rank, id.k());
            }
        }
        st.stored += blk.stored();
        st.region_stored[blk.region][blk.type] += blk.stored();
        st.region_area[blk.region] += dense_sz;
        t.blocks.push_back(std::move(blk));
    }
    if (o.dense_gen) record_checkpoints(lt, t);
}

}  // namespace

// Leaf size when the options leave it to the builder.  It sets the smallest
// block given a butterfly (4 leaves); below it blocks are regenerated dense
// blocks.  The values are the measured optima on MI355X (FP64, 8-32 fields):
// at N = 1024 applying butterflies to blocks under 512 columns costs more than
// regenerating them, at N = 4096 butterflies pay from 256 columns.
int auto_leaf(int N) { return N <= 256 ? 32 : N <= 1024 ? 128 : 64; }

int build_all(int N, const sht_plan_opts &opts_in, HostPlanData &out, const LegendreTables *lt) {
    auto t0 = std::chrono::steady_clock::now();
    sht_plan_opts opts = opts_in;
    if (opts.leaf <= 0) opts.leaf = auto_leaf(N);
    out.N = N;
    out.opts = opts;
    if (lt && lt->N == N)
        out.lt = *lt;
    else
        build_legendre_tables(N, out.lt, opts.m_lo, opts.m_hi);
    const int ntask = 4 * N;  // 2N orders x 2 parities
    out.tasks.assign(ntask, Task());
    int nth = opts.threads > 0 ? opts.threads : (int)std::thread::hardware_concurrency();
    nth = std::max(1, std::min(nth, 64));
    const int m_lo = std::max(0, opts.m_lo), m_hi = opts.m_hi < 0 ? 2 * N - 1 : std::min(opts.m_hi, 2 * N - 1);
    std::atomic<int> next(2 * m_lo);
    std::vector<BuildStats> st(nth);
    std::vector<std::thread> th;
    for (int w = 0; w < nth; ++w)
        th.emplace_back([&, w]() {
            std::vector<double> mat;
            for (;;) {
                int i = next.fetch_add(1);
                if (i >= ntask || i > 2 * m_hi + 1) break;
                // heaviest (small |m|) first
                build_task(N, out.lt, opts, i / 2, i % 2, out.tasks[i], mat, st[w]);
            }
        });
    for (auto &t : th) t.join();
    BuildStats tot;
    for (auto &s : st) {
        tot.dense_entries += s.dense_entries;
        tot.stored += s.stored;
        tot.n_dense += s.n_dense;
        tot.n_lowrank += s.n_lowrank;
        tot.n_butterfly += s.n_butterfly;
        tot.n_dropped += s.n_dropped;
        tot.dense_stored += s.dense_stored;
        tot.lowrank_stored += s.lowrank_stored;
        tot.butterfly_stored += s.butterfly_stored;
        tot.n_gen += s.n_gen;
        tot.gen_entries += s.gen_entries;
        tot.max_rank = std::max(tot.max_rank, s.max_rank);
        for (int i = 0; i < 3; ++i) {
            tot.region_area[i] += s.region_area[i];
            for (int j = 0; j < 3; ++j) tot.region_stored[i][j] += s.region_stored[i][j];
        }
    }
    tot.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    out.stats = tot;
    return SHT_OK;
}

std::string HostPlanData::stats_json() const { return idbf::stats_json(stats, opts); }

std::string stats_json(const BuildStats &stats, const sht_plan_opts &opts) {
    std::ostringstream os;
    os << "{\"dense_entries\":" << stats.dense_entries << ",\"stored_entries\":" << stats.stored
       << ",\"compression\":" << (stats.stored ? (double)stats.dense_entries / stats.stored : 0.0)
       << ",\"blocks_dense\":" << stats.n_dense << ",\"blocks_lowrank\":" << stats.n_lowrank
       << ",\"blocks_butterfly\":" << stats.n_butterfly << ",\"blocks_dropped\":" << stats.n_dropped
       << ",\"dense_stored\":" << stats.dense_stored << ",\"lowrank_stored\":" << stats.lowrank_stored
       << ",\"butterfly_stored\":" << stats.butterfly_stored << ",\"blocks_generated\":" << stats.n_gen
       << ",\"generated_entries\":" << stats.gen_entries << ",\"max_rank\":" << stats.max_rank
       << ",\"build_seconds\":" << stats.seconds << ",\"eps\":" << opts.eps << ",\"n0\":" << opts.n0
       << ",\"leaf\":" << opts.leaf;
    const char *rn[3] = {"osc", "nonosc", "turning"};
    for (int i = 0; i < 3; ++i)
        os << ",\"" << rn[i] << "\":{\"area\":" << stats.region_area[i] << ",\"dense\":" << stats.region_stored[i][0]
           << ",\"lowrank\":" << stats.region_stored[i][1] << ",\"butterfly\":" << stats.region_stored[i][2] << "}";
    os << "}";
    return os.str();
}

}  // namespace idbf
}  // namespace sht
