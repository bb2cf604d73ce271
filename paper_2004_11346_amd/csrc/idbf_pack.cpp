// Packing of the factors into the op programs (forward and transposed) and
// the host executor of a packed program.
//
// Forward program:    in = coefficient panels X[task][col][R],
//                     out = half-grid panels Y[task][row][R].
// Transposed program: in = Y-shaped panels, out = X-shaped panels.
// Every block becomes a chain of levels; the last level of every block is
// final (adds into the output panel).  Levels are right-aligned so that all
// final levels coincide, intermediate levels ping-pong between two scratch
// buffers, and final ops are coloured into slots with disjoint rows.
#include <algorithm>
#include <cstring>
#include <map>

#include "idbf_build.h"
#include "idbf_pack.h"

namespace sht {
namespace idbf {

namespace {

constexpr int kTileRows = 32;   // dense / low-rank row tiles
constexpr int kTileCols = 64;   // column tiles of wide blocks

struct LSub {
    int64_t mat_off = 0;
    int mrows = 0, mcols = 0, ld = 0, trans = 0;
    int src_level = -1;                   // -1: program input panel
    std::vector<int64_t> in_rows;         // input panel row (task-absolute) or level-local row
    std::vector<int> map;                 // output positions
    std::vector<std::pair<int64_t, int>> dir;
};

struct LOp {
    int n_out = 0;
    bool final = false;
    int64_t out_row = 0;  // final: absolute row of the output panel
    std::vector<LSub> subs;
};

struct Level {
    std::vector<LOp> ops;
    std::vector<int64_t> off;  // local row offset of each op
    int64_t rows = 0;
    void add(LOp op) {
        off.push_back(rows);
        rows += op.n_out;
        ops.push_back(std::move(op));
    }
};

struct BlockProg {
    int task = 0;
    std::vector<Level> levels;  // last level final
};

struct ValueStream {
    std::vector<double> v;
    int64_t put(const std::vector<double> &m) {
        int64_t o = (int64_t)v.size();
        v.insert(v.end(), m.begin(), m.end());
        // keep every block 16-byte aligned for vector loads
        while (v.size() & 1) v.push_back(0.0);
        return o;
    }
};

inline int node_lo(int lo, int n, int level, int t) { return lo + (int)(((int64_t)t * n) >> level); }

// dense product out (+)= M in with M (m x n, ld) at mat_off, tiled:
// trans = 0: out rows i < m, in rows j < n; trans = 1: out rows j < n, in rows i < m.
void emit_dense(Level &lv, int64_t mat_off, int m, int n, int ld, bool trans, int src_level,
                const std::vector<int64_t> &in_rows, bool final, int64_t out_row0) {
    const int n_out = trans ? n : m, n_in = trans ? m : n;
    for (int t0 = 0; t0 < n_out; t0 += kTileRows) {
        const int tr = std::min(kTileRows, n_out - t0);
        LOp op;
        op.n_out = tr;
        op.final = final;
        op.out_row = out_row0 + t0;
        for (int c0 = 0; c0 < n_in; c0 += kTileCols) {
            const int tc = std::min(kTileCols, n_in - c0);
            LSub s;
            if (!trans) {
                s.mat_off = mat_off + (int64_t)t0 * ld + c0;
                s.mrows = tr;
                s.mcols = tc;
            } else {
                s.mat_off = mat_off + (int64_t)c0 * ld + t0;
                s.mrows = tc;
                s.mcols = tr;
            }
            s.ld = ld;
            s.trans = trans ? 1 : 0;
            s.src_level = src_level;
            s.in_rows.assign(in_rows.begin() + c0, in_rows.begin() + c0 + tc);
            for (int i = 0; i < tr; ++i) s.map.push_back(i);
            op.subs.push_back(std::move(s));
        }
        lv.add(std::move(op));
    }
}

// column-ID gather: out[i] = in[cand[skel_i]] + sum_j T[i][j] in[cand[red_j]]
LSub gather_sub(const ID &id, int64_t toff, int src_level, const std::vector<int64_t> &cand_rows) {
    LSub s;
    const int k = id.k(), nred = (int)id.red.size();
    s.mat_off = toff;
    s.mrows = k;
    s.mcols = nred;
    s.ld = nred;
    s.trans = 0;
    s.src_level = src_level;
    for (int j = 0; j < nred; ++j) s.in_rows.push_back(cand_rows[id.red[j]]);
    for (int i = 0; i < k; ++i) s.map.push_back(i);
    for (int i = 0; i < k; ++i) s.dir.push_back({cand_rows[id.skel[i]], i});
    if (nred == 0) s.mrows = 0;
    return s;
}

// transpose application: out[skel_i] += u[i]; out[red_j] += sum_i T[i][j] u[i]
// (positions relative to the op's output); u rows given.
LSub scatter_sub(const ID &id, int64_t toff, int src_level, const std::vector<int64_t> &u_rows, int pos_base) {
    LSub s;
    const int k = id.k(), nred = (int)id.red.size();
    s.mat_off = toff;
    s.mrows = k;
    s.mcols = nred;
    s.ld = nred;
    s.trans = 1;
    s.src_level = src_level;
    s.in_rows = u_rows;
    for (int j = 0; j < nred; ++j) s.map.push_back(pos_base + id.red[j]);
    for (int i = 0; i < k; ++i) s.dir.push_back({u_rows[i], pos_base + id.skel[i]});
    if (nred == 0) {
        s.mrows = 0;
        s.in_rows.clear();
    }
    return s;
}

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

struct Offsets {
    std::vector<int64_t> x;  // X panel row offset per task
    std::vector<int64_t> y;  // Y panel row offset per task
};

// Matrix offsets of one butterfly in the value stream.
struct BfOffsets {
    std::vector<std::vector<int64_t>> col, row;
    std::vector<int64_t> S;
};

void pack_values(const Block &b, ValueStream &vs, int64_t &d_off, int64_t &u_off, int64_t &v_off, BfOffsets &bo) {
    if (b.type == kDense) {
        d_off = vs.put(b.D);
    } else if (b.type == kLowRank) {
        u_off = vs.put(b.U);
        v_off = vs.put(b.V);
    } else {
        const Butterfly &bf = b.bf;
        bo.col.resize(bf.col.size());
        for (size_t l = 0; l < bf.col.size(); ++l)
            for (auto &id : bf.col[l]) bo.col[l].push_back(vs.put(id.T));
        bo.row.resize(bf.row.size());
        for (size_t l = 0; l < bf.row.size(); ++l)
            for (auto &id : bf.row[l]) bo.row[l].push_back(vs.put(id.T));
        for (auto &m : bf.S) bo.S.push_back(vs.put(m));
    }
}

// ---- forward chains -------------------------------------------------
void forward_chain(const Task &t, const Block &b, const Offsets &of, int task, int64_t d_off, int64_t u_off,
                   int64_t v_off, const BfOffsets &bo, BlockProg &bp) {
    const int m = b.r1 - b.r0, n = b.c1 - b.c0;
    const int64_t xb = of.x[task], yb = of.y[task];
    bp.task = task;
    (void)t;
    if (b.type == kDense) {
        Level lv;
        emit_dense(lv, d_off, m, n, n, false, -1, range_rows(xb, b.c0, b.c1), true, yb + b.r0);
        bp.levels.push_back(std::move(lv));
        return;
    }
    if (b.type == kLowRank) {
        Level l0, l1;
        // w = V^T x  (V: n x rank, row-major)
        emit_dense(l0, v_off, n, b.rank, b.rank, true, -1, range_rows(xb, b.c0, b.c1), false, 0);
        std::vector<int64_t> w;
        for (size_t q = 0; q < l0.ops.size(); ++q)
            for (int i = 0; i < l0.ops[q].n_out; ++i) w.push_back(l0.off[q] + i);
        emit_dense(l1, u_off, m, b.rank, b.rank, false, 0, w, true, yb + b.r0);
        bp.levels.push_back(std::move(l0));
        bp.levels.push_back(std::move(l1));
        return;
    }
    const Butterfly &bf = b.bf;
    const int L = bf.L, h = bf.h, nc = bf.c1 - bf.c0, nr = bf.r1 - bf.r0;
    // column pass
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
                op.subs.push_back(gather_sub(id, bo.col[l][(size_t)A * nB + B], src, cand));
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    // middle: u = S z   (op index A * nB + B, same as col[h])
    {
        Level lv;
        const int nA = 1 << h, nB = 1 << (L - h);
        const int hl = h;
        for (int A = 0; A < nA; ++A)
            for (int B = 0; B < nB; ++B) {
                const size_t ix = (size_t)A * nB + B;
                const int kr = bf.row[L - h][ix].k(), kc = bf.col[h][ix].k();
                const Level &pv = bp.levels[hl];
                LOp op;
                op.n_out = kr;
                LSub s;
                s.mat_off = bo.S[ix];
                s.mrows = kr;
                s.mcols = kc;
                s.ld = kc;
                s.trans = 0;
                s.src_level = hl;
                s.in_rows = local_rows(pv.off[ix], kc);
                for (int i = 0; i < kr; ++i) s.map.push_back(i);
                if (kc == 0) s.mrows = 0;
                op.subs.push_back(std::move(s));
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    // where u_l[A, B] lives: (level index, local offset)
    std::map<std::pair<int, int>, std::pair<int, int64_t>> uloc;  // key (l, A * 2^l + B)
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
                    op.subs.push_back(scatter_sub(id, bo.row[l][(size_t)A * nB + B], loc.first,
                                                  local_rows(loc.second, id.k()), 0));
                }
                // outputs: u_{l-1}[2A, Bp] then u_{l-1}[2A+1, Bp]
                const int64_t base = lv.rows;
                uloc[{l - 1, (2 * A) * nBp + Bp}] = {lvl, base};
                uloc[{l - 1, (2 * A + 1) * nBp + Bp}] = {lvl, base + c1.k()};
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    // final: leaves
    {
        Level lv;
        for (int A = 0; A < (1 << L); ++A) {
            const ID &id = bf.row[0][A];
            const int lo = node_lo(bf.r0, nr, L, A), hi = node_lo(bf.r0, nr, L, A + 1);
            auto loc = uloc.at({0, A});
            LOp op;
            op.n_out = hi - lo;
            op.final = true;
            op.out_row = yb + lo;
            op.subs.push_back(scatter_sub(id, bo.row[0][A], loc.first, local_rows(loc.second, id.k()), 0));
            lv.add(std::move(op));
        }
        bp.levels.push_back(std::move(lv));
    }
}

// ---- transposed chains ------------------------------------------------
void transpose_chain(const Task &t, const Block &b, const Offsets &of, int task, int64_t d_off, int64_t u_off,
                     int64_t v_off, const BfOffsets &bo, BlockProg &bp) {
    const int m = b.r1 - b.r0, n = b.c1 - b.c0;
    const int64_t xb = of.x[task], yb = of.y[task];
    bp.task = task;
    (void)t;
    if (b.type == kDense) {
        Level lv;
        emit_dense(lv, d_off, m, n, n, true, -1, range_rows(yb, b.r0, b.r1), true, xb + b.c0);
        bp.levels.push_back(std::move(lv));
        return;
    }
    if (b.type == kLowRank) {
        Level l0, l1;
        emit_dense(l0, u_off, m, b.rank, b.rank, true, -1, range_rows(yb, b.r0, b.r1), false, 0);
        std::vector<int64_t> w;
        for (size_t q = 0; q < l0.ops.size(); ++q)
            for (int i = 0; i < l0.ops[q].n_out; ++i) w.push_back(l0.off[q] + i);
        emit_dense(l1, v_off, n, b.rank, b.rank, false, 0, w, true, xb + b.c0);
        bp.levels.push_back(std::move(l0));
        bp.levels.push_back(std::move(l1));
        return;
    }
    const Butterfly &bf = b.bf;
    const int L = bf.L, h = bf.h, nc = bf.c1 - bf.c0, nr = bf.r1 - bf.r0;
    // row pass (gathers), level 0 reads the input panel
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
                op.subs.push_back(gather_sub(id, bo.row[l][(size_t)A * nB + B], src, cand));
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    // middle: z = S^T u
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
                LSub s;
                s.mat_off = bo.S[ix];
                s.mrows = kr;
                s.mcols = kc;
                s.ld = kc;
                s.trans = 1;
                s.src_level = ul;
                s.in_rows = local_rows(pv.off[ix], kr);
                for (int i = 0; i < kc; ++i) s.map.push_back(i);
                if (kr == 0) {
                    s.mrows = 0;
                    s.in_rows.clear();
                }
                op.subs.push_back(std::move(s));
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    std::map<std::pair<int, int>, std::pair<int, int64_t>> zloc;  // key (l, A * 2^(L-l) + B)
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
                    op.subs.push_back(scatter_sub(id, bo.col[l][(size_t)A * nB + B], loc.first,
                                                  local_rows(loc.second, id.k()), 0));
                }
                const int64_t base = lv.rows;
                zloc[{l - 1, Ap * nBc + 2 * B}] = {lvl, base};
                zloc[{l - 1, Ap * nBc + 2 * B + 1}] = {lvl, base + ia.k()};
                lv.add(std::move(op));
            }
        bp.levels.push_back(std::move(lv));
    }
    {
        Level lv;
        for (int B = 0; B < (1 << L); ++B) {
            const ID &id = bf.col[0][B];
            const int lo = node_lo(bf.c0, nc, L, B), hi = node_lo(bf.c0, nc, L, B + 1);
            auto loc = zloc.at({0, B});
            LOp op;
            op.n_out = hi - lo;
            op.final = true;
            op.out_row = xb + lo;
            op.subs.push_back(scatter_sub(id, bo.col[0][B], loc.first, local_rows(loc.second, id.k()), 0));
            lv.add(std::move(op));
        }
        bp.levels.push_back(std::move(lv));
    }
}

// Linearise block chains into a program.
void schedule(std::vector<BlockProg> &bps, int64_t in_rows, int64_t out_rows, Program &p) {
    int D = 0;
    for (auto &b : bps) D = std::max(D, (int)b.levels.size());
    const int W = D - 1;  // work stages
    std::vector<std::vector<Op>> stage_ops(std::max(W, 0));
    std::vector<std::vector<int32_t>> stage_task(std::max(W, 0));
    std::vector<std::vector<std::vector<SubOp>>> stage_subs(std::max(W, 0));
    std::vector<int64_t> stage_rows(std::max(W, 0), 0);
    // finals per task with row extents, for slot colouring
    struct Fin {
        int task;
        int64_t lo, hi;
        Op op;
        std::vector<SubOp> subs;
    };
    std::vector<Fin> finals;
    p.idx.clear();
    auto push_idx = [&](const std::vector<int32_t> &v) {
        int32_t o = (int32_t)p.idx.size();
        p.idx.insert(p.idx.end(), v.begin(), v.end());
        return o;
    };
    for (auto &b : bps) {
        const int nl = (int)b.levels.size();
        std::vector<int64_t> base(nl, 0);
        std::vector<int> stage(nl);
        for (int l = 0; l < nl; ++l) stage[l] = D - nl + l;
        for (int l = 0; l < nl; ++l) {
            Level &lv = b.levels[l];
            const bool fin = l == nl - 1;
            if (!fin) {
                base[l] = stage_rows[stage[l]];
                stage_rows[stage[l]] += lv.rows;
            }
            for (size_t q = 0; q < lv.ops.size(); ++q) {
                LOp &lo = lv.ops[q];
                Op op;
                op.n_out = lo.n_out;
                op.nsub = (int)lo.subs.size();
                op.sub0 = 0;
                op.dst = fin ? kOut : ((stage[l] & 1) ? kScrB : kScrA);
                op.dst_row = fin ? lo.out_row : base[l] + lv.off[q];
                std::vector<SubOp> subs;
                for (auto &ls : lo.subs) {
                    SubOp s{};
                    s.mat_off = ls.mat_off;
                    s.mrows = ls.mrows;
                    s.mcols = ls.mcols;
                    s.ld = ls.ld;
                    s.trans = ls.trans;
                    int srcbuf;
                    int64_t srcbase = 0;
                    if (ls.src_level < 0) {
                        srcbuf = kIn;
                    } else {
                        srcbuf = (stage[ls.src_level] & 1) ? kScrB : kScrA;
                        srcbase = base[ls.src_level];
                    }
                    s.src = srcbuf;
                    std::vector<int32_t> in;
                    for (auto r : ls.in_rows) in.push_back((int32_t)(r + srcbase));
                    s.n_in = (int32_t)in.size();
                    s.in_off = push_idx(in);
                    s.n_map = (int32_t)ls.map.size();
                    s.map_off = push_idx(std::vector<int32_t>(ls.map.begin(), ls.map.end()));
                    std::vector<int32_t> dr;
                    for (auto &d : ls.dir) {
                        dr.push_back((int32_t)(d.first + srcbase));
                        dr.push_back(d.second);
                    }
                    s.n_dir = (int32_t)ls.dir.size();
                    s.dir_off = push_idx(dr);
                    if (s.mrows == 0 || s.mcols == 0) {
                        s.n_map = 0;
                        s.n_in = 0;
                    }
                    p.max_n_in = std::max(p.max_n_in, (int)s.n_in);
                    p.max_mat = std::max(p.max_mat, s.mrows * s.mcols);
                    subs.push_back(s);
                }
                p.max_n_out = std::max(p.max_n_out, op.n_out);
                if (fin) {
                    finals.push_back(Fin{b.task, lo.out_row, lo.out_row + lo.n_out, op, std::move(subs)});
                } else {
                    stage_ops[stage[l]].push_back(op);
                    stage_task[stage[l]].push_back(b.task);
                    stage_subs[stage[l]].push_back(std::move(subs));
                }
            }
        }
    }
    p.ops.clear();
    p.op_task.clear();
    p.subs.clear();
    p.stages.clear();
    for (int s = 0; s < W; ++s) {
        Stage st;
        st.op_begin = (int32_t)p.ops.size();
        for (size_t q = 0; q < stage_ops[s].size(); ++q) {
            Op op = stage_ops[s][q];
            op.sub0 = (int32_t)p.subs.size();
            p.subs.insert(p.subs.end(), stage_subs[s][q].begin(), stage_subs[s][q].end());
            p.ops.push_back(op);
            p.op_task.push_back(stage_task[s][q]);
        }
        st.op_end = (int32_t)p.ops.size();
        p.stages.push_back(st);
        p.scr_rows = std::max(p.scr_rows, stage_rows[s]);
    }
    p.n_work_stages = W;
    // slot colouring of the final ops (disjoint rows within a slot)
    std::vector<std::vector<std::pair<int64_t, int64_t>>> slot_rows;
    std::vector<std::vector<size_t>> slot_ops;
    std::vector<size_t> order(finals.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return finals[a].lo < finals[b].lo; });
    for (size_t i : order) {
        const Fin &f = finals[i];
        size_t s = 0;
        for (; s < slot_rows.size(); ++s) {
            bool clash = false;
            // rows of one slot are kept sorted by lo; only the last ones can overlap
            auto &v = slot_rows[s];
            for (auto it = v.rbegin(); it != v.rend(); ++it) {
                if (it->second <= f.lo) break;
                if (it->first < f.hi && f.lo < it->second) {
                    clash = true;
                    break;
                }
            }
            if (!clash) break;
        }
        if (s == slot_rows.size()) {
            slot_rows.emplace_back();
            slot_ops.emplace_back();
        }
        slot_rows[s].push_back({f.lo, f.hi});
        slot_ops[s].push_back(i);
    }
    for (size_t s = 0; s < slot_ops.size(); ++s) {
        Stage st;
        st.op_begin = (int32_t)p.ops.size();
        for (size_t i : slot_ops[s]) {
            Op op = finals[i].op;
            op.sub0 = (int32_t)p.subs.size();
            p.subs.insert(p.subs.end(), finals[i].subs.begin(), finals[i].subs.end());
            p.ops.push_back(op);
            p.op_task.push_back(finals[i].task);
        }
        st.op_end = (int32_t)p.ops.size();
        p.stages.push_back(st);
    }
    p.in_rows = in_rows;
    p.out_rows = out_rows;
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
    ValueStream vs;
    std::vector<BlockProg> fw, tr;
    for (int ti = 0; ti < ntask; ++ti) {
        const Task &t = hp.tasks[ti];
        for (const Block &b : t.blocks) {
            int64_t d_off = 0, u_off = 0, v_off = 0;
            BfOffsets bo;
            pack_values(b, vs, d_off, u_off, v_off, bo);
            BlockProg f, a;
            forward_chain(t, b, of, ti, d_off, u_off, v_off, bo, f);
            transpose_chain(t, b, of, ti, d_off, u_off, v_off, bo, a);
            fw.push_back(std::move(f));
            tr.push_back(std::move(a));
        }
    }
    schedule(fw, of.x[ntask], of.y[ntask], pk.fwd);
    schedule(tr, of.y[ntask], of.x[ntask], pk.adj);
    pk.vals = std::move(vs.v);
}

void host_run_program(const Program &p, const double *vals, int R, const double *in, double *out) {
    std::vector<double> scr[2];
    scr[0].assign((size_t)p.scr_rows * R, 0.0);
    scr[1].assign((size_t)p.scr_rows * R, 0.0);
    std::fill(out, out + (size_t)p.out_rows * R, 0.0);
    std::vector<double> acc;
    for (size_t si = 0; si < p.stages.size(); ++si) {
        const Stage &st = p.stages[si];
        for (int q = st.op_begin; q < st.op_end; ++q) {
            const Op &op = p.ops[q];
            acc.assign((size_t)op.n_out * R, 0.0);
            for (int s = 0; s < op.nsub; ++s) {
                const SubOp &sb = p.subs[op.sub0 + s];
                const double *src = sb.src == kIn ? in : sb.src == kScrA ? scr[0].data() : scr[1].data();
                const int32_t *inr = &p.idx[sb.in_off];
                const int32_t *map = &p.idx[sb.map_off];
                for (int i = 0; i < sb.n_map; ++i) {
                    double *a = &acc[(size_t)map[i] * R];
                    for (int j = 0; j < sb.n_in; ++j) {
                        double mv = sb.trans ? vals[sb.mat_off + (int64_t)j * sb.ld + i]
                                             : vals[sb.mat_off + (int64_t)i * sb.ld + j];
                        const double *x = src + (size_t)inr[j] * R;
                        for (int r = 0; r < R; ++r) a[r] += mv * x[r];
                    }
                }
                const int32_t *dir = &p.idx[sb.dir_off];
                for (int d = 0; d < sb.n_dir; ++d) {
                    const double *x = src + (size_t)dir[2 * d] * R;
                    double *a = &acc[(size_t)dir[2 * d + 1] * R];
                    for (int r = 0; r < R; ++r) a[r] += x[r];
                }
            }
            double *dst = op.dst == kOut ? out : op.dst == kScrA ? scr[0].data() : scr[1].data();
            for (int i = 0; i < op.n_out; ++i)
                for (int r = 0; r < R; ++r) {
                    double &d = dst[(size_t)(op.dst_row + i) * R + r];
                    d = op.dst == kOut ? d + acc[(size_t)i * R + r] : acc[(size_t)i * R + r];
                }
        }
    }
}

}  // namespace idbf
}  // namespace sht
