// Packing of the factors into the op programs (forward and transposed) and
// the host executor of a packed program.
//
// Forward program:    in = coefficient panels X[task][col][R],
//                     out = half-grid panels Y[task][row][R].
// Transposed program: in = Y-shaped panels, out = X-shaped panels.
// Every block becomes a chain of non-final levels (scratch to scratch) and a
// set of final contributions (products that land in the output panel).
// Levels are right-aligned so that all final contributions read from the last
// work stage or from the input panel; intermediate levels ping-pong between
// two scratch buffers.  The final stage is one op per 64-row tile of every
// task's output panel, summing every contribution to the tile's rows, so each
// output row is written exactly once and no atomics are needed.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <climits>
#include <cmath>
#include <map>
#include <thread>

#include "idbf_build.h"
#include "idbf_pack.h"

namespace sht {
namespace idbf {

namespace {

constexpr int kTile = 64;     // output rows per final op
constexpr int kMaxIn = 64;    // gathered rows per sub-op

// A product M(:, :) x with M(i, j) = trans ? mb[j * ld + i] : mb[i * ld + j]
// restricted to the outputs out_idx, landing at positions map (level-local
// positions, or absolute output-panel rows for final contributions).
struct LSub {
    const double *mb = nullptr;
    int ld = 0;
    bool trans = false;
    std::vector<int> out_idx;
    std::vector<int64_t> map;
    int src_level = -1;  // -1: input panel
    std::vector<int64_t> in_rows;
    std::vector<std::pair<int64_t, int64_t>> dir;  // (src row, position)
    double m(int i, int j) const { return trans ? mb[(size_t)j * ld + i] : mb[(size_t)i * ld + j]; }
};

struct LOp {
    int n_out = 0;
    std::vector<LSub> subs;
};

struct Level {
    std::vector<LOp> ops;
    std::vector<int64_t> off;
    int64_t rows = 0;
    void add(LOp op) {
        off.push_back(rows);
        rows += op.n_out;
        ops.push_back(std::move(op));
    }
};

struct BlockProg {
    int task = 0;
    std::vector<Level> levels;   // non-final
    std::vector<LSub> finals;    // contributions to the output panel
    const Block *gen = nullptr;  // regenerated dense block (no levels, no finals)
};

inline int node_lo(int lo, int n, int level, int t) { return lo + (int)(((int64_t)t * n) >> level); }

std::vector<int64_t> range_rows(int64_t base, int lo, int hi) {
    std::vector<int64_t> r;
    for (int i = lo; i < hi; ++i) r.push_back(base + i);
    return r;
}

std::vector<int64_t> local_rows(int64_t off, int n) {
    std::vector<int64_t> r(n);
    for (int i = 0; i < n; ++i) r[i] = off + i;
    return r;
}

// dense product with all outputs: n_out x n_in
LSub dense_sub(const double *mb, int ld, bool trans, int n_out, int src_level, std::vector<int64_t> in_rows,
               int64_t pos0) {
    LSub s;
    s.mb = mb;
    s.ld = ld;
    s.trans = trans;
    s.src_level = src_level;
    s.in_rows = std::move(in_rows);
    for (int i = 0; i < n_out; ++i) {
        s.out_idx.push_back(i);
        s.map.push_back(pos0 + i);
    }
    return s;
}

// column-ID gather: out[i] = in[cand[skel_i]] + sum_j T[i][j] in[cand[red_j]]
LSub gather_sub(const ID &id, int src_level, const std::vector<int64_t> &cand, int64_t pos0) {
    LSub s;
    const int k = id.k(), nred = (int)id.red.size();
    s.mb = id.T.data();
    s.ld = nred;
    s.trans = false;
    s.src_level = src_level;
    if (nred > 0) {
        for (int j = 0; j < nred; ++j) s.in_rows.push_back(cand[id.red[j]]);
        for (int i = 0; i < k; ++i) {
            s.out_idx.push_back(i);
            s.map.push_back(pos0 + i);
        }
    }
    for (int i = 0; i < k; ++i) s.dir.push_back({cand[id.skel[i]], pos0 + i});
    return s;
}

// transposed application: out[skel_i] += u[i]; out[red_j] += sum_i T[i][j] u[i]
LSub scatter_sub(const ID &id, int src_level, const std::vector<int64_t> &u_rows, int64_t pos0) {
    LSub s;
    const int k = id.k(), nred = (int)id.red.size();
    s.mb = id.T.data();
    s.ld = nred;
    s.trans = true;
    s.src_level = src_level;
    if (nred > 0 && k > 0) {
        s.in_rows = u_rows;
        for (int j = 0; j < nred; ++j) {
            s.out_idx.push_back(j);
            s.map.push_back(pos0 + id.red[j]);
        }
    }
    for (int i = 0; i < k; ++i) s.dir.push_back({u_rows[i], pos0 + id.skel[i]});
    return s;
}

struct Offsets {
    std::vector<int64_t> x, y;
};

// ---- forward chains -------------------------------------------------
void forward_chain(const Block &b, const Offsets &of, int task, BlockProg &bp) {
    const int m = b.r1 - b.r0, n = b.c1 - b.c0;
    const int64_t xb = of.x[task], yb = of.y[task];
    bp.task = task;
    if (b.type == kDense && b.gen) {
        bp.gen = &b;
        return;
    }
    if (b.type == kDense) {
        bp.finals.push_back(dense_sub(b.D.data(), n, false, m, -1, range_rows(xb, b.c0, b.c1), yb + b.r0));
        return;
    }
    if (b.type == kLowRank) {
        Level l0;
        LOp op;
        op.n_out = b.rank;  // w = V^T x   (V: n x rank)
        op.subs.push_back(dense_sub(b.V.data(), b.rank, true, b.rank, -1, range_rows(xb, b.c0, b.c1), 0));
        l0.add(std::move(op));
        bp.levels.push_back(std::move(l0));
        bp.finals.push_back(dense_sub(b.U.data(), b.rank, false, m, 0, local_rows(0, b.rank), yb + b.r0));
        return;
    }
    const Butterfly &bf = b.bf;
    const int L = bf.L, h = bf.h, nc = bf.c1 - bf.c0, nr = bf.r1 - bf.r0;
    for (int l = 0; l <= h; ++l) {
        Level lv;
        const int nA = 1 << l, nB = 1 << (L - l);
        for (int A = 0; A < nA; ++A)
            for (int B = 0; B < nB; ++B) {
                const ID &id = bf.col[l][(size_t)A * nB + B];
                std::vector<int64_t> cand;
                int src;
                if (l == 0) {
                    cand = range_rows(xb, node_lo(bf.c0, nc, L, B), node_lo(bf.c0, nc, L, B + 1));
                    src = -1;
                } else {
                    const int Ap = A >> 1, nBp = 1 << (L - l + 1);
                    const size_t q1 = (size_t)Ap * nBp + 2 * B, q2 = q1 + 1;
                    const Level &pv = bp.levels[l - 1];
                    cand = local_rows(pv.off[q1], pv.ops[q1].n_out);
                    auto c2 = local_rows(pv.off[q2], pv.ops[q2].n_out);
                    cand.insert(cand.end(), c2.begin(), c2.end());
                    src = l - 1;
                }
                LOp op;
                op.n_out = id.k();
                op.subs.push_back(gather_sub(id, src, cand, 0));
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    {
        Level lv;
        const int nA = 1 << h, nB = 1 << (L - h);
        for (int A = 0; A < nA; ++A)
            for (int B = 0; B < nB; ++B) {
                const size_t ix = (size_t)A * nB + B;
                const int kr = bf.row[L - h][ix].k(), kc = bf.col[h][ix].k();
                const Level &pv = bp.levels[h];
                LOp op;
                op.n_out = kr;
                if (kc > 0) op.subs.push_back(dense_sub(bf.S[ix].data(), kc, false, kr, h, local_rows(pv.off[ix], kc), 0));
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    std::map<std::pair<int, int>, std::pair<int, int64_t>> uloc;
    {
        const int lvl = (int)bp.levels.size() - 1, nB = 1 << (L - h);
        for (int A = 0; A < (1 << h); ++A)
            for (int B = 0; B < nB; ++B) uloc[{L - h, A * nB + B}] = {lvl, bp.levels[lvl].off[(size_t)A * nB + B]};
    }
    for (int l = L - h; l >= 1; --l) {
        Level lv;
        const int nA = 1 << (L - l), nB = 1 << l, nBp = 1 << (l - 1);
        const int lvl = (int)bp.levels.size();
        for (int A = 0; A < nA; ++A)
            for (int Bp = 0; Bp < nBp; ++Bp) {
                const ID &c1 = bf.row[l - 1][(size_t)(2 * A) * nBp + Bp];
                const ID &c2 = bf.row[l - 1][(size_t)(2 * A + 1) * nBp + Bp];
                LOp op;
                op.n_out = c1.k() + c2.k();
                for (int B = 2 * Bp; B <= 2 * Bp + 1; ++B) {
                    const ID &id = bf.row[l][(size_t)A * nB + B];
                    auto loc = uloc.at({l, A * nB + B});
                    op.subs.push_back(scatter_sub(id, loc.first, local_rows(loc.second, id.k()), 0));
                }
                const int64_t base = lv.rows;
                uloc[{l - 1, (2 * A) * nBp + Bp}] = {lvl, base};
                uloc[{l - 1, (2 * A + 1) * nBp + Bp}] = {lvl, base + c1.k()};
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    for (int A = 0; A < (1 << L); ++A) {
        const ID &id = bf.row[0][A];
        const int lo = node_lo(bf.r0, nr, L, A);
        auto loc = uloc.at({0, A});
        bp.finals.push_back(scatter_sub(id, loc.first, local_rows(loc.second, id.k()), yb + lo));
    }
}

// ---- transposed chains ------------------------------------------------
void transpose_chain(const Block &b, const Offsets &of, int task, BlockProg &bp) {
    const int n = b.c1 - b.c0;
    const int64_t xb = of.x[task], yb = of.y[task];
    bp.task = task;
    if (b.type == kDense && b.gen) {
        bp.gen = &b;
        return;
    }
    if (b.type == kDense) {
        bp.finals.push_back(dense_sub(b.D.data(), n, true, n, -1, range_rows(yb, b.r0, b.r1), xb + b.c0));
        return;
    }
    if (b.type == kLowRank) {
        Level l0;
        LOp op;
        op.n_out = b.rank;  // w = U^T y   (U: m x rank)
        op.subs.push_back(dense_sub(b.U.data(), b.rank, true, b.rank, -1, range_rows(yb, b.r0, b.r1), 0));
        l0.add(std::move(op));
        bp.levels.push_back(std::move(l0));
        bp.finals.push_back(dense_sub(b.V.data(), b.rank, false, n, 0, local_rows(0, b.rank), xb + b.c0));
        return;
    }
    const Butterfly &bf = b.bf;
    const int L = bf.L, h = bf.h, nc = bf.c1 - bf.c0, nr = bf.r1 - bf.r0;
    for (int l = 0; l <= L - h; ++l) {
        Level lv;
        const int nA = 1 << (L - l), nB = 1 << l;
        for (int A = 0; A < nA; ++A)
            for (int B = 0; B < nB; ++B) {
                const ID &id = bf.row[l][(size_t)A * nB + B];
                std::vector<int64_t> cand;
                int src;
                if (l == 0) {
                    cand = range_rows(yb, node_lo(bf.r0, nr, L, A), node_lo(bf.r0, nr, L, A + 1));
                    src = -1;
                } else {
                    const int Bp = B >> 1, nBp = 1 << (l - 1);
                    const size_t q1 = (size_t)(2 * A) * nBp + Bp, q2 = (size_t)(2 * A + 1) * nBp + Bp;
                    const Level &pv = bp.levels[l - 1];
                    cand = local_rows(pv.off[q1], pv.ops[q1].n_out);
                    auto c2 = local_rows(pv.off[q2], pv.ops[q2].n_out);
                    cand.insert(cand.end(), c2.begin(), c2.end());
                    src = l - 1;
                }
                LOp op;
                op.n_out = id.k();
                op.subs.push_back(gather_sub(id, src, cand, 0));
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    {
        Level lv;
        const int nA = 1 << h, nB = 1 << (L - h);
        const int ul = L - h;
        for (int A = 0; A < nA; ++A)
            for (int B = 0; B < nB; ++B) {
                const size_t ix = (size_t)A * nB + B;
                const int kr = bf.row[L - h][ix].k(), kc = bf.col[h][ix].k();
                const Level &pv = bp.levels[ul];
                LOp op;
                op.n_out = kc;
                if (kr > 0) op.subs.push_back(dense_sub(bf.S[ix].data(), kc, true, kc, ul, local_rows(pv.off[ix], kr), 0));
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    std::map<std::pair<int, int>, std::pair<int, int64_t>> zloc;
    {
        const int lvl = (int)bp.levels.size() - 1, nB = 1 << (L - h);
        for (int A = 0; A < (1 << h); ++A)
            for (int B = 0; B < nB; ++B) zloc[{h, A * nB + B}] = {lvl, bp.levels[lvl].off[(size_t)A * nB + B]};
    }
    for (int l = h; l >= 1; --l) {
        Level lv;
        const int nAp = 1 << (l - 1), nB = 1 << (L - l), nBc = 1 << (L - l + 1);
        const int lvl = (int)bp.levels.size();
        for (int Ap = 0; Ap < nAp; ++Ap)
            for (int B = 0; B < nB; ++B) {
                const ID &ia = bf.col[l - 1][(size_t)Ap * nBc + 2 * B];
                const ID &ib = bf.col[l - 1][(size_t)Ap * nBc + 2 * B + 1];
                LOp op;
                op.n_out = ia.k() + ib.k();
                for (int A = 2 * Ap; A <= 2 * Ap + 1; ++A) {
                    const ID &id = bf.col[l][(size_t)A * nB + B];
                    auto loc = zloc.at({l, A * nB + B});
                    op.subs.push_back(scatter_sub(id, loc.first, local_rows(loc.second, id.k()), 0));
                }
                const int64_t base = lv.rows;
                zloc[{l - 1, Ap * nBc + 2 * B}] = {lvl, base};
                zloc[{l - 1, Ap * nBc + 2 * B + 1}] = {lvl, base + ia.k()};
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    for (int B = 0; B < (1 << L); ++B) {
        const ID &id = bf.col[0][B];
        const int lo = node_lo(bf.c0, nc, L, B);
        auto loc = zloc.at({0, B});
        bp.finals.push_back(scatter_sub(id, loc.first, local_rows(loc.second, id.k()), xb + lo));
    }
}

// ---- linearisation ------------------------------------------------------

struct Emitter {
    Program &p;
    explicit Emitter(Program &pp) : p(pp) {}
    int32_t push_idx(const std::vector<int32_t> &v) {
        int32_t o = (int32_t)p.idx.size();
        p.idx.insert(p.idx.end(), v.begin(), v.end());
        return o;
    }
    // Emit one LSub restricted to outputs q in `sel` (indices into s.out_idx)
    // and directs in `dsel`; positions are rebased by -pos0.  Inputs longer
    // than kMaxIn are split across several SubOps.
    void emit(const LSub &s, const std::vector<int> &sel, const std::vector<int> &dsel, int srcbuf, int64_t srcbase,
              int64_t pos0, std::vector<SubOp> &out) {
        const int nin = (int)s.in_rows.size();
        const int nmap = (int)sel.size();
        bool first = true;
        for (int j0 = 0; j0 < std::max(nin, 1); j0 += kMaxIn) {
            const int jn = nmap > 0 ? std::min(kMaxIn, nin - j0) : 0;
            SubOp so{};
            so.src = srcbuf;
            so.mat_off = (int64_t)p.vals.size();
            std::vector<int32_t> in, map;
            if (jn > 0) {
                for (int j = 0; j < jn; ++j) in.push_back((int32_t)(s.in_rows[j0 + j] + srcbase));
                for (int q : sel) map.push_back((int32_t)(s.map[q] - pos0));
                for (int j = 0; j < jn; ++j)
                    for (int q : sel) p.vals.push_back(s.m(s.out_idx[q], j0 + j));
                while (p.vals.size() & 1) p.vals.push_back(0.0);
            }
            so.n_in = jn;
            so.n_map = jn > 0 ? nmap : 0;
            so.in_off = push_idx(in);
            so.map_off = push_idx(map);
            std::vector<int32_t> dr;
            if (first)
                for (int d : dsel) {
                    dr.push_back((int32_t)(s.dir[d].first + srcbase));
                    dr.push_back((int32_t)(s.dir[d].second - pos0));
                }
            so.n_dir = (int32_t)(dr.size() / 2);
            so.dir_off = push_idx(dr);
            first = false;
            if (so.n_map > 0 || so.n_dir > 0) {
                p.max_n_in = std::max(p.max_n_in, (int)so.n_in);
                out.push_back(so);
            }
            if (jn == 0) break;
        }
    }
};

// gen_tiles[t][i]: the regenerated blocks have an item for output tile i of
// task t.  A final op with no contribution is left out for such a tile (the
// item writes it); written[t][i] records which tiles got a final op.
void schedule(std::vector<BlockProg> &bps, int ntask, const std::vector<int64_t> &out_off,
              const std::vector<int64_t> &in_off, bool fwd, int64_t value_hint, Program &p,
              const std::vector<std::vector<char>> &gen_tiles, std::vector<std::vector<char>> &written) {
    const int64_t in_rows = in_off[ntask];
    int D = 0;  // number of work stages
    for (auto &b : bps) D = std::max(D, (int)b.levels.size());
    std::vector<std::vector<Op>> st_ops(D);
    std::vector<std::vector<int32_t>> st_task(D);
    std::vector<std::vector<std::vector<SubOp>>> st_subs(D);
    std::vector<std::vector<std::vector<int>>> st_sublvl(D);  // source level of every sub-op
    std::vector<int64_t> st_rows(D, 0);
    Emitter em(p);
    p.ops.clear();
    p.op_task.clear();
    p.subs.clear();
    p.idx.clear();
    p.vals.clear();
    p.vals.reserve((size_t)value_hint);
    {
        // index stream: inputs, maps and identity pairs of every sub-op; final
        // contributions repeat their inputs once per output tile they touch
        int64_t n = 0;
        for (const BlockProg &b : bps) {
            for (const Level &lv : b.levels)
                for (const LOp &op : lv.ops)
                    for (const LSub &ls : op.subs) n += ls.in_rows.size() + ls.map.size() + 2 * ls.dir.size();
            for (const LSub &ls : b.finals) {
                int64_t lo = INT64_MAX, hi = INT64_MIN;
                for (int64_t m : ls.map) lo = std::min(lo, m), hi = std::max(hi, m);
                const int64_t tiles = ls.map.empty() ? 1 : (hi - lo) / kTile + 2;
                n += tiles * ls.in_rows.size() + ls.map.size() + 2 * ls.dir.size();
            }
        }
        p.idx.reserve((size_t)n + 1024);
    }
    p.stages.clear();
    // per block: stage and base row of every level
    std::vector<std::vector<int>> bstage(bps.size());
    std::vector<std::vector<int64_t>> bbase(bps.size());
    for (size_t bi = 0; bi < bps.size(); ++bi) {
        BlockProg &b = bps[bi];
        const int nl = (int)b.levels.size();
        bstage[bi].resize(nl);
        bbase[bi].resize(nl);
        for (int l = 0; l < nl; ++l) {
            const int s = D - nl + l;
            bstage[bi][l] = s;
            bbase[bi][l] = st_rows[s];
            st_rows[s] += b.levels[l].rows;
        }
    }
    auto srcinfo = [&](size_t bi, int lvl, int &buf, int64_t &base) {
        if (lvl < 0) {
            buf = kIn;
            base = 0;
        } else {
            buf = (bstage[bi][lvl] & 1) ? kScrB : kScrA;
            base = bbase[bi][lvl];
        }
    };
    // ops of level l of block bi: st_ops[s][lvl_ops[bi][l].first .. second)
    std::vector<std::vector<std::pair<size_t, size_t>>> lvl_ops(bps.size());
    for (size_t bi = 0; bi < bps.size(); ++bi) {
        BlockProg &b = bps[bi];
        lvl_ops[bi].resize(b.levels.size());
        for (int l = 0; l < (int)b.levels.size(); ++l) {
            const int s = bstage[bi][l];
            Level &lv = b.levels[l];
            lvl_ops[bi][l].first = st_ops[s].size();
            for (size_t q = 0; q < lv.ops.size(); ++q) {
                const LOp &lo = lv.ops[q];
                // outputs in chunks of at most kTile rows; every chunk keeps the
                // matrix outputs and identity terms that land in it
                for (int p0 = 0; p0 < std::max(lo.n_out, 1); p0 += kTile) {
                    const int p1 = std::min(lo.n_out, p0 + kTile);
                    Op op{};
                    op.n_out = std::max(0, p1 - p0);
                    op.dst = (s & 1) ? kScrB : kScrA;
                    op.dst_row = bbase[bi][l] + lv.off[q] + p0;
                    std::vector<SubOp> subs;
                    std::vector<int> sublvl;
                    for (const LSub &ls : lo.subs) {
                        int buf;
                        int64_t base;
                        srcinfo(bi, ls.src_level, buf, base);
                        std::vector<int> sel, dsel;
                        for (size_t i = 0; i < ls.map.size(); ++i)
                            if (ls.map[i] >= p0 && ls.map[i] < p1) sel.push_back((int)i);
                        for (size_t i = 0; i < ls.dir.size(); ++i)
                            if (ls.dir[i].second >= p0 && ls.dir[i].second < p1) dsel.push_back((int)i);
                        if (sel.empty() && dsel.empty()) continue;
                        em.emit(ls, sel, dsel, buf, base, p0, subs);
                        sublvl.resize(subs.size(), ls.src_level);
                    }
                    op.nsub = (int32_t)subs.size();
                    st_ops[s].push_back(op);
                    st_task[s].push_back(b.task);
                    st_subs[s].push_back(std::move(subs));
                    st_sublvl[s].push_back(std::move(sublvl));
                    if (lo.n_out == 0) break;
                }
            }
            lvl_ops[bi][l].second = st_ops[s].size();
        }
    }
    for (int s = 0; s < D; ++s) {
        Stage st{};
        st.op_begin = (int32_t)p.ops.size();
        for (size_t q = 0; q < st_ops[s].size(); ++q) {
            Op op = st_ops[s][q];
            op.sub0 = (int32_t)p.subs.size();
            p.subs.insert(p.subs.end(), st_subs[s][q].begin(), st_subs[s][q].end());
            p.ops.push_back(op);
            p.op_task.push_back(st_task[s][q]);
            st.max_out = std::max(st.max_out, op.n_out);
            for (auto &so : st_subs[s][q]) st.max_in = std::max(st.max_in, so.n_in);
        }
        st.op_end = (int32_t)p.ops.size();
        p.stages.push_back(st);
        p.scr_rows = std::max(p.scr_rows, st_rows[s]);
        p.max_n_out = std::max(p.max_n_out, st.max_out);
    }
    p.n_work_stages = D;
    // fused form of the work stages: one group per block with levels.  An LDS
    // group's levels alternate between two LDS buffers of lr rows.  A group
    // whose levels exceed them keeps its rows in HBM, but in rows of its own
    // past the staged scratch rows (buffer A): its workgroup runs all its
    // levels while other groups run, so the staged rows, which later stages
    // reuse, are not free for it; its last level goes to the staged rows the
    // final stage reads, as an LDS group's does.
    p.fgroups.clear();
    p.flevels.clear();
    p.fops.clear();
    p.fsubs.clear();
    p.f_max_lds_rows = 0;
    p.f_extra_rows = 0;
    bool fok = true;
    for (size_t bi = 0; bi < bps.size(); ++bi) {
        const BlockProg &b = bps[bi];
        const int nl = (int)b.levels.size();
        if (nl == 0) continue;
        int64_t lr = 0;
        for (const Level &lv : b.levels) lr = std::max(lr, lv.rows);
        const bool inlds = lr <= kFusedMaxRows;
        // first row of level l in its buffer, and the buffer
        std::vector<int64_t> lbase(nl);
        std::vector<int32_t> lbuf(nl);
        for (int l = 0; l < nl; ++l) {
            if (inlds) {
                lbase[l] = (int64_t)(l & 1) * lr;
                lbuf[l] = kLds;
            } else if (l < nl - 1) {
                lbase[l] = p.scr_rows + p.f_extra_rows;
                lbuf[l] = kScrA;
                p.f_extra_rows += b.levels[l].rows;
            } else {
                lbase[l] = bbase[bi][l];
                lbuf[l] = (bstage[bi][l] & 1) ? kScrB : kScrA;
            }
        }
        FusedGroup g{};
        g.lvl_begin = (int32_t)p.flevels.size();
        g.nlev = nl;
        g.lds_rows = (int32_t)std::min<int64_t>(lr, INT32_MAX);
        g.out_buf = (bstage[bi][nl - 1] & 1) ? kScrB : kScrA;
        g.out_row = bbase[bi][nl - 1];
        g.task = b.task;
        for (int l = 0; l < nl; ++l) {
            const int s = bstage[bi][l];
            FusedLevel fl{};
            fl.op_begin = (int32_t)p.fops.size();
            fl.rows = (int32_t)b.levels[l].rows;
            for (size_t q = lvl_ops[bi][l].first; q < lvl_ops[bi][l].second; ++q) {
                const Op &so = p.ops[(size_t)p.stages[s].op_begin + q];
                Op fo = so;
                fo.dst = lbuf[l];
                fo.dst_row = lbase[l] + (so.dst_row - bbase[bi][l]);
                fo.sub0 = (int32_t)p.fsubs.size();
                for (int k = 0; k < so.nsub; ++k) {
                    SubOp fs = p.subs[(size_t)so.sub0 + k];
                    if (fs.src != kIn) {
                        const int sl = st_sublvl[s][q][k];
                        if (sl != l - 1 || sl < 0) {
                            fok = false;
                        } else {
                            const int64_t off = lbase[sl] - bbase[bi][sl];
                            std::vector<int32_t> in(fs.n_in), dr(2 * (size_t)fs.n_dir);
                            for (int j = 0; j < fs.n_in; ++j) in[j] = (int32_t)(p.idx[fs.in_off + j] + off);
                            for (int d = 0; d < fs.n_dir; ++d) {
                                dr[2 * d] = (int32_t)(p.idx[fs.dir_off + 2 * d] + off);
                                dr[2 * d + 1] = p.idx[fs.dir_off + 2 * d + 1];
                            }
                            fs.src = lbuf[sl];
                            fs.in_off = em.push_idx(in);
                            fs.dir_off = em.push_idx(dr);
                        }
                    }
                    p.fsubs.push_back(fs);
                }
                p.fops.push_back(fo);
            }
            fl.op_end = (int32_t)p.fops.size();
            p.flevels.push_back(fl);
        }
        p.fgroups.push_back(g);
        p.f_max_lds_rows = std::max(p.f_max_lds_rows, g.lds_rows);
    }
    // bounds of the fused form, as its kernel assumes them: an LDS group's ops
    // write inside the rows its level clears and read inside the rows of the
    // level before; a staged-row group's ops fit the 64-row accumulator
    for (const FusedGroup &g : p.fgroups) {
        const bool inlds = g.lds_rows <= kFusedMaxRows;
        for (int l = 0; l < g.nlev && fok; ++l) {
            const FusedLevel &fl = p.flevels[(size_t)g.lvl_begin + l];
            const int64_t lo = (int64_t)(l & 1) * g.lds_rows, hi = lo + fl.rows;
            const int64_t plo = (int64_t)((l + 1) & 1) * g.lds_rows;
            const int64_t phi = l > 0 ? plo + p.flevels[(size_t)g.lvl_begin + l - 1].rows : plo;
            if (fl.rows > g.lds_rows) fok = false;
            for (int q = fl.op_begin; q < fl.op_end && fok; ++q) {
                const Op &op = p.fops[q];
                if (inlds ? (op.dst != kLds || op.dst_row < lo || op.dst_row + op.n_out > hi)
                          : (op.n_out > kTile || (op.dst != kScrA && op.dst != kScrB) || op.dst_row < 0 ||
                             op.dst_row + op.n_out > p.scr_rows + p.f_extra_rows ||
                             (l < g.nlev - 1 && (op.dst != kScrA || op.dst_row < p.scr_rows))))
                    fok = false;
                for (int k = 0; k < op.nsub && fok; ++k) {
                    const SubOp &so = p.fsubs[(size_t)op.sub0 + k];
                    for (int q2 = 0; q2 < so.n_map; ++q2) {
                        const int32_t m = p.idx[(size_t)so.map_off + q2];
                        if (m < 0 || m >= op.n_out) fok = false;
                    }
                    for (int d = 0; d < so.n_dir; ++d) {
                        const int32_t m = p.idx[(size_t)so.dir_off + 2 * d + 1];
                        if (m < 0 || m >= op.n_out) fok = false;
                    }
                    if (so.src == kScrA || so.src == kScrB) {
                        // a staged-row group reads its own rows of the level before
                        if (inlds || so.src != kScrA) fok = false;
                        for (int j = 0; j < so.n_in; ++j) {
                            const int32_t r = p.idx[(size_t)so.in_off + j];
                            if (r < p.scr_rows || r >= p.scr_rows + p.f_extra_rows) fok = false;
                        }
                        for (int d = 0; d < so.n_dir; ++d) {
                            const int32_t r = p.idx[(size_t)so.dir_off + 2 * d];
                            if (r < p.scr_rows || r >= p.scr_rows + p.f_extra_rows) fok = false;
                        }
                    }
                    if (so.src == kLds) {
                        if (!inlds) fok = false;
                        for (int j = 0; j < so.n_in; ++j) {
                            const int32_t r = p.idx[(size_t)so.in_off + j];
                            if (r < plo || r >= phi) fok = false;
                        }
                        for (int d = 0; d < so.n_dir; ++d) {
                            const int32_t r = p.idx[(size_t)so.dir_off + 2 * d];
                            if (r < plo || r >= phi) fok = false;
                        }
                    }
                }
            }
        }
    }
    p.fused_ok = fok ? 1 : 0;
    // final stage: output tiles per task
    std::vector<std::vector<size_t>> by_task(ntask);
    for (size_t bi = 0; bi < bps.size(); ++bi) by_task[bps[bi].task].push_back(bi);
    Stage fst{};
    fst.op_begin = (int32_t)p.ops.size();
    written.assign(ntask, {});
    for (int t = 0; t < ntask; ++t) {
        const int64_t r0 = out_off[t], r1 = out_off[t + 1];
        written[t].assign((size_t)((r1 - r0 + kTile - 1) / kTile), 0);
        for (int64_t T0 = r0; T0 < r1; T0 += kTile) {
            const int64_t T1 = std::min(r1, T0 + kTile);
            Op op{};
            op.n_out = (int32_t)(T1 - T0);
            op.dst = kOut;
            op.dst_row = T0;
            op.sub0 = (int32_t)p.subs.size();
            std::vector<SubOp> subs;
            for (size_t bi : by_task[t]) {
                const BlockProg &b = bps[bi];
                for (const LSub &ls : b.finals) {
                    std::vector<int> sel, dsel;
                    for (size_t q = 0; q < ls.map.size(); ++q)
                        if (ls.map[q] >= T0 && ls.map[q] < T1) sel.push_back((int)q);
                    for (size_t d = 0; d < ls.dir.size(); ++d)
                        if (ls.dir[d].second >= T0 && ls.dir[d].second < T1) dsel.push_back((int)d);
                    if (sel.empty() && dsel.empty()) continue;
                    int buf;
                    int64_t base;
                    srcinfo(bi, ls.src_level, buf, base);
                    em.emit(ls, sel, dsel, buf, base, T0, subs);
                }
            }
            op.nsub = (int32_t)subs.size();
            const size_t ti = (size_t)((T0 - r0) / kTile);
            if (subs.empty() && ti < gen_tiles[t].size() && gen_tiles[t][ti]) continue;
            written[t][ti] = 1;
            p.subs.insert(p.subs.end(), subs.begin(), subs.end());
            p.ops.push_back(op);
            p.op_task.push_back(t);
            fst.max_out = std::max(fst.max_out, op.n_out);
            for (auto &so : subs) fst.max_in = std::max(fst.max_in, so.n_in);
        }
    }
    fst.op_end = (int32_t)p.ops.size();
    p.stages.push_back(fst);
    p.max_n_out = std::max(p.max_n_out, fst.max_out);
    p.in_rows = in_rows;
    p.out_rows = out_off[ntask];
}

}  // namespace

namespace {

void build_gen_forward(const HostPlanData &hp, GenForward &gf) {
    const int N = hp.N, ntask = 4 * N;
    gf = GenForward();
    gf.task_first.assign(ntask + 1, 0);
    for (int t = 0; t < ntask; ++t) {
        gf.task_first[t] = (int32_t)gf.items.size();
        const Task &tk = hp.tasks[t];
        if (tk.cols <= 0) continue;
        std::vector<const Block *> gb;
        for (const Block &b : tk.blocks)
            if (b.type == kDense && b.gen) gb.push_back(&b);
        if (gb.empty()) continue;
        for (int r0 = 0; r0 < N; r0 += kTile) {
            GenForward::Item it{t, r0, (int32_t)gf.segs.size(), 0};
            for (const Block *b : gb) {
                if (b->r1 <= r0 || b->r0 >= r0 + kTile) continue;
                GenForward::Seg sg{b->c0, b->c1 - b->c0, (int32_t)gf.ckexp.size(), 0};
                gf.segs.push_back(sg);
                for (int q = 0; q < kTile; ++q) {
                    const int r = r0 + q;
                    RecState st;
                    if (r >= b->r0 && r < b->r1 && r < N) {
                        st = gen_state(hp.lt, tk.a, tk.parity, *b, r, b->c0);
                        gf.entries += sg.ncol;
                    } else {
                        st.pm2 = st.p1 = 0.0;
                        st.e = 0;
                    }
                    gf.ck.push_back(st.pm2);
                    gf.ck.push_back(st.p1);
                    gf.ckexp.push_back(st.e);
                }
            }
            it.seg_end = (int32_t)gf.segs.size();
            if (it.seg_end > it.seg_begin) gf.items.push_back(it);
        }
    }
    gf.task_first[ntask] = (int32_t)gf.items.size();
}

void build_gen_adjoint(const HostPlanData &hp, GenAdjoint &ga) {
    const int N = hp.N, ntask = 4 * N;
    ga = GenAdjoint();
    ga.task_first.assign(ntask + 1, 0);
    for (int t = 0; t < ntask; ++t) {
        ga.task_first[t] = (int32_t)ga.items.size();
        const Task &tk = hp.tasks[t];
        if (tk.cols <= 0) continue;
        std::vector<const Block *> gb;
        for (const Block &b : tk.blocks)
            if (b.type == kDense && b.gen) gb.push_back(&b);
        if (gb.empty()) continue;
        for (int C0 = 0; C0 < tk.cols; C0 += kTile) {
            GenAdjoint::Item it{t, C0, (int32_t)ga.segs.size(), 0};
            for (const Block *b : gb) {
                const int c0 = std::max(b->c0, C0), c1 = std::min(b->c1, C0 + kTile);
                if (c1 <= c0) continue;
                for (int R0 = b->r0 & ~63; R0 < b->r1; R0 += kTile) {
                    GenAdjoint::Seg sg{R0, c0, c1 - c0, (int32_t)ga.ckexp.size()};
                    ga.segs.push_back(sg);
                    for (int q = 0; q < kTile; ++q) {
                        const int r = R0 + q;
                        RecState st;
                        if (r >= b->r0 && r < b->r1 && r < N) {
                            st = gen_state(hp.lt, tk.a, tk.parity, *b, r, c0);
                        } else {
                            st.pm2 = st.p1 = 0.0;
                            st.e = 0;
                        }
                        ga.ck.push_back(st.pm2);
                        ga.ck.push_back(st.p1);
                        ga.ckexp.push_back(st.e);
                    }
                }
            }
            it.seg_end = (int32_t)ga.segs.size();
            if (it.seg_end > it.seg_begin) ga.items.push_back(it);
        }
    }
    ga.task_first[ntask] = (int32_t)ga.items.size();
}

}  // namespace

void pack_programs(const HostPlanData &hp, PackedPlan &pk) {
    const int N = hp.N;
    const int ntask = 4 * N;
    Offsets of;
    of.x.resize(ntask + 1, 0);
    of.y.resize(ntask + 1, 0);
    for (int t = 0; t < ntask; ++t) {
        of.x[t + 1] = of.x[t] + std::max(0, hp.tasks[t].cols);
        of.y[t + 1] = of.y[t] + N;
    }
    pk.x_off = of.x;
    pk.y_off = of.y;
    auto T = [] { return std::chrono::steady_clock::now(); };
    auto D = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
        return std::chrono::duration<double>(b - a).count();
    };
    const bool verbose = std::getenv("SHT_VERBOSE") != nullptr;
    // every stored factor entry is emitted once per program, plus the padding
    // of each sub-op to an even length
    int64_t nblocks = 0;
    for (const Task &t : hp.tasks) nblocks += (int64_t)t.blocks.size();
    const int64_t hint = hp.stats.stored + 64 * nblocks + 1024;
    // regenerated-block items first: the op programs leave the output tiles
    // that only these items contribute to
    std::thread tg([&] { build_gen_adjoint(hp, pk.gen_adj); });
    build_gen_forward(hp, pk.gen_fwd);
    tg.join();
    std::vector<std::vector<char>> cov_fwd(ntask), cov_adj(ntask), wr_fwd, wr_adj;
    for (int t = 0; t < ntask; ++t) {
        cov_fwd[t].assign((size_t)((N + kTile - 1) / kTile), 0);
        cov_adj[t].assign((size_t)((std::max(0, hp.tasks[t].cols) + kTile - 1) / kTile), 0);
    }
    for (const GenForward::Item &it : pk.gen_fwd.items) cov_fwd[it.task][it.row0 / kTile] = 1;
    for (const GenAdjoint::Item &it : pk.gen_adj.items) cov_adj[it.task][it.col0 / kTile] = 1;
    auto pack_dir = [&](bool fwd) {
        auto t0 = T();
        std::vector<BlockProg> bps;
        for (int ti = 0; ti < ntask; ++ti)
            for (const Block &b : hp.tasks[ti].blocks) {
                BlockProg bp;
                if (fwd)
                    forward_chain(b, of, ti, bp);
                else
                    transpose_chain(b, of, ti, bp);
                bps.push_back(std::move(bp));
            }
        auto t1 = T();
        if (fwd)
            schedule(bps, ntask, of.y, of.x, true, hint, pk.fwd, cov_fwd, wr_fwd);
        else
            schedule(bps, ntask, of.x, of.y, false, hint, pk.adj, cov_adj, wr_adj);
        if (verbose)
            std::fprintf(stderr, "[sht] %s chains %.2fs schedule %.2fs\n", fwd ? "fwd" : "adj", D(t0, t1), D(t1, T()));
    };
    std::thread th([&] { pack_dir(false); });
    pack_dir(true);
    th.join();
    for (GenForward::Item &it : pk.gen_fwd.items)
        if (!wr_fwd[it.task][it.row0 / kTile]) it.task |= GenForward::kOverwrite;
    for (GenAdjoint::Item &it : pk.gen_adj.items)
        if (!wr_adj[it.task][it.col0 / kTile]) it.task |= GenAdjoint::kOverwrite;
}

void host_run_gen_forward(const GenForward &gf, int N, int t_lo, int t_hi, int R, const std::vector<int64_t> &x_off,
                          const std::vector<int64_t> &y_off, const double *in, double *out, const double *xh,
                          const double *coef2) {
    for (int i = gf.task_first[t_lo]; i < gf.task_first[t_hi + 1]; ++i) {
        const GenForward::Item &it = gf.items[i];
        const int task = it.task & ~GenForward::kOverwrite;
        const int a = task / 2, par = task % 2;
        const double *cf = coef2 + 3 * (tri_offset(N, a) + par);
        for (int q = 0; q < 64 && it.row0 + q < N; ++q) {
            const int r = it.row0 + q;
            const double x = xh[r], x2 = x * x;
            double *y = out + (size_t)(y_off[task] + r) * R;
            if (it.task & GenForward::kOverwrite) std::fill(y, y + R, 0.0);
            for (int s = it.seg_begin; s < it.seg_end; ++s) {
                const GenForward::Seg &sg = gf.segs[s];
                double p0 = gf.ck[2 * ((int64_t)sg.ck + q)], p1 = gf.ck[2 * ((int64_t)sg.ck + q) + 1];
                int e = gf.ckexp[sg.ck + q];
                for (int t = 0; t < sg.ncol; ++t) {
                    const int c = sg.c0 + t;
                    if (t > 0) {
                        const double *c3 = cf + 3 * (2 * (int64_t)c);
                        const double p2 = (c3[0] * x2 + c3[1]) * p1 + c3[2] * p0;
                        p0 = p1;
                        p1 = p2;
                        if (std::fabs(p1) > 0x1p200) {
                            p0 *= 0x1p-200;
                            p1 *= 0x1p-200;
                            e += 200;
                        }
                    }
                    const double v = e < -1074 ? 0.0 : p1 * std::ldexp(1.0, e);
                    const double *xr = in + (size_t)(x_off[task] + c) * R;
                    for (int k = 0; k < R; ++k) y[k] += v * xr[k];
                }
            }
        }
    }
}

void host_run_gen_adjoint(const GenAdjoint &ga, int N, int t_lo, int t_hi, int R, const std::vector<int64_t> &x_off,
                          const std::vector<int64_t> &y_off, const double *in, double *out, const double *xh,
                          const double *coef2) {
    for (int i = ga.task_first[t_lo]; i < ga.task_first[t_hi + 1]; ++i) {
        const GenAdjoint::Item &it = ga.items[i];
        const int task = it.task & ~GenAdjoint::kOverwrite;
        const int a = task / 2, par = task % 2;
        const double *cf = coef2 + 3 * (tri_offset(N, a) + par);
        if (it.task & GenAdjoint::kOverwrite) {
            const int64_t cols = x_off[task + 1] - x_off[task];
            for (int64_t c = it.col0; c < std::min<int64_t>(cols, it.col0 + 64); ++c)
                std::fill(out + (size_t)(x_off[task] + c) * R, out + (size_t)(x_off[task] + c + 1) * R, 0.0);
        }
        for (int s = it.seg_begin; s < it.seg_end; ++s) {
            const GenAdjoint::Seg &sg = ga.segs[s];
            for (int q = 0; q < 64 && sg.row0 + q < N; ++q) {
                const int r = sg.row0 + q;
                const double x = xh[r], x2 = x * x;
                double p0 = ga.ck[2 * ((int64_t)sg.ck + q)], p1 = ga.ck[2 * ((int64_t)sg.ck + q) + 1];
                int e = ga.ckexp[sg.ck + q];
                const double *h = in + (size_t)(y_off[task] + r) * R;
                for (int t = 0; t < sg.ncol; ++t) {
                    const int c = sg.c0 + t;
                    if (t > 0) {
                        const double *c3 = cf + 3 * (2 * (int64_t)c);
                        const double p2 = (c3[0] * x2 + c3[1]) * p1 + c3[2] * p0;
                        p0 = p1;
                        p1 = p2;
                        if (std::fabs(p1) > 0x1p200) {
                            p0 *= 0x1p-200;
                            p1 *= 0x1p-200;
                            e += 200;
                        }
                    }
                    const double v = e < -1074 ? 0.0 : p1 * std::ldexp(1.0, e);
                    double *xo = out + (size_t)(x_off[task] + c) * R;
                    for (int k = 0; k < R; ++k) xo[k] += v * h[k];
                }
            }
        }
    }
}

std::string fused_stats_json(const PackedPlan &pk) {
    std::string s;
    for (int d = 0; d < 2; ++d) {
        const Program &p = d ? pk.adj : pk.fwd;
        const std::string pre = d ? ",\"adj_fused_" : ",\"fwd_fused_";
        s += pre + "ok\":" + std::to_string(p.fused_ok) + pre + "groups\":" + std::to_string(p.fgroups.size()) +
             pre + "max_lds_rows\":" + std::to_string(p.f_max_lds_rows) + pre + "ops\":" + std::to_string(p.fops.size());
        // groups and their stored values by rows per buffer (up to 128, 256,
        // 384, 512, 768, more)
        const int lim[5] = {128, 256, 384, 512, 768};
        int64_t ng[6] = {0}, nv[6] = {0};
        for (const FusedGroup &g : p.fgroups) {
            int b = 0;
            while (b < 5 && g.lds_rows > lim[b]) ++b;
            ++ng[b];
            for (int l = 0; l < g.nlev; ++l) {
                const FusedLevel &fl = p.flevels[(size_t)g.lvl_begin + l];
                for (int q = fl.op_begin; q < fl.op_end; ++q)
                    for (int k = 0; k < p.fops[q].nsub; ++k) {
                        const SubOp &so = p.fsubs[(size_t)p.fops[q].sub0 + k];
                        nv[b] += (int64_t)so.n_map * so.n_in;
                    }
            }
        }
        s += pre + "rows_hist\":[";
        for (int b = 0; b < 6; ++b) s += "[" + std::to_string(ng[b]) + "," + std::to_string(nv[b]) + "]" + (b < 5 ? "," : "");
        s += "]";
    }
    return s;
}

namespace {

// acc[0 .. n_out) += the sub-ops of op (rows of R values); src_of maps a
// buffer id to its rows
template <typename Src>
void host_op(const Program &p, const Op &op, const std::vector<SubOp> &subs, int R, Src src_of, double *acc) {
    for (int s = 0; s < op.nsub; ++s) {
        const SubOp &sb = subs[(size_t)op.sub0 + s];
        const double *src = src_of(sb.src);
        const int32_t *inr = &p.idx[sb.in_off];
        const int32_t *map = &p.idx[sb.map_off];
        for (int qq = 0; qq < sb.n_map; ++qq) {
            double *a = acc + (size_t)map[qq] * R;
            for (int j = 0; j < sb.n_in; ++j) {
                const double mv = p.vals[sb.mat_off + (int64_t)j * sb.n_map + qq];
                const double *x = src + (size_t)inr[j] * R;
                for (int r = 0; r < R; ++r) a[r] += mv * x[r];
            }
        }
        const int32_t *dir = &p.idx[sb.dir_off];
        for (int d = 0; d < sb.n_dir; ++d) {
            const double *x = src + (size_t)dir[2 * d] * R;
            double *a = acc + (size_t)dir[2 * d + 1] * R;
            for (int r = 0; r < R; ++r) a[r] += x[r];
        }
    }
}

}  // namespace

void host_run_program(const Program &p, int R, const double *in, double *out, bool fused) {
    std::vector<double> scr[2];
    scr[0].assign((size_t)std::max<int64_t>(1, p.scr_rows + (fused ? p.f_extra_rows : 0)) * R, 0.0);
    scr[1].assign((size_t)std::max<int64_t>(1, p.scr_rows) * R, 0.0);
    std::vector<double> acc, lds;
    size_t st0 = 0;
    if (fused) {
        auto gsrc = [&](int32_t b) { return b == kIn ? in : b == kScrA ? scr[0].data() : scr[1].data(); };
        for (const FusedGroup &g : p.fgroups) {
            if (g.lds_rows > kFusedMaxRows) {  // staged rows, level by level
                for (int l = 0; l < g.nlev; ++l) {
                    const FusedLevel &fl = p.flevels[(size_t)g.lvl_begin + l];
                    for (int q = fl.op_begin; q < fl.op_end; ++q) {
                        const Op &op = p.fops[q];
                        acc.assign((size_t)op.n_out * R, 0.0);
                        host_op(p, op, p.fsubs, R, gsrc, acc.data());
                        double *dst = op.dst == kScrA ? scr[0].data() : scr[1].data();
                        std::memcpy(dst + (size_t)op.dst_row * R, acc.data(), sizeof(double) * acc.size());
                    }
                }
                continue;
            }
            lds.assign(2 * (size_t)g.lds_rows * R, 0.0);
            auto src_of = [&](int32_t b) { return b == kIn ? in : lds.data(); };
            for (int l = 0; l < g.nlev; ++l) {
                const FusedLevel &fl = p.flevels[(size_t)g.lvl_begin + l];
                double *buf = lds.data() + (size_t)(l & 1) * g.lds_rows * R;
                std::fill(buf, buf + (size_t)fl.rows * R, 0.0);
                for (int q = fl.op_begin; q < fl.op_end; ++q) {
                    const Op &op = p.fops[q];
                    host_op(p, op, p.fsubs, R, src_of, lds.data() + (size_t)op.dst_row * R);
                }
            }
            const FusedLevel &last = p.flevels[(size_t)g.lvl_begin + g.nlev - 1];
            const double *buf = lds.data() + (size_t)((g.nlev - 1) & 1) * g.lds_rows * R;
            double *dst = (g.out_buf == kScrA ? scr[0].data() : scr[1].data()) + (size_t)g.out_row * R;
            std::memcpy(dst, buf, sizeof(double) * (size_t)last.rows * R);
        }
        st0 = (size_t)p.n_work_stages;
    }
    auto src_of = [&](int32_t b) { return b == kIn ? in : b == kScrA ? scr[0].data() : scr[1].data(); };
    for (size_t si = st0; si < p.stages.size(); ++si) {
        const Stage &st = p.stages[si];
        for (int q = st.op_begin; q < st.op_end; ++q) {
            const Op &op = p.ops[q];
            acc.assign((size_t)op.n_out * R, 0.0);
            host_op(p, op, p.subs, R, src_of, acc.data());
            double *dst = op.dst == kOut ? out : op.dst == kScrA ? scr[0].data() : scr[1].data();
            std::memcpy(dst + (size_t)op.dst_row * R, acc.data(), sizeof(double) * acc.size());
        }
    }
}

}  // namespace idbf
}  // namespace sht
