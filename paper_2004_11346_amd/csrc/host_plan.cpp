// Host-side plan verification entry points (include/sht.h): build the FP64
// plan without a device and apply its factors with plain loops.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "idbf_build.h"
#include "idbf_pack.h"
#include "plan_cache.h"
#include "sht.h"
#include "sht_internal.h"

using namespace sht;

struct sht_host_plan {
    int method = SHT_DENSE;
    int cache = idbf::kCacheOff;  // plan cache outcome (fast form)
    idbf::HostPlanData data;      // tasks are empty when the plan came from the cache
    idbf::PackedPlan packed;
};

extern "C" {

int sht_host_plan_create(int N, int method, const sht_plan_opts *opts, sht_host_plan_t **out) {
    if (!out) return SHT_ERR_INVALID_ARG;
    *out = nullptr;
    if (N < 1 || N > 8192) return SHT_ERR_INVALID_ARG;
    if (method != SHT_DENSE && method != SHT_IDBF) return SHT_ERR_UNSUPPORTED;
    sht_plan_opts o;
    sht_plan_opts_default(&o);
    if (opts) o = *opts;
    sht_host_plan *hp = new (std::nothrow) sht_host_plan;
    if (!hp) return SHT_ERR_OOM;
    hp->method = method;
    try {
        if (method == SHT_IDBF) {
            std::string key, path;
            bool loaded = false;
            if (o.cache_dir && o.cache_dir[0]) {
                key = idbf::cache_key(N, o);
                path = idbf::cache_path(o.cache_dir, key);
                const int lrc = idbf::cache_load(path, key, hp->packed, hp->data.stats);
                loaded = lrc == SHT_OK;
                hp->cache = loaded ? idbf::kCacheHit : lrc == SHT_ERR_PLAN_CORRUPT ? idbf::kCacheRebuilt
                                                                                   : idbf::kCacheMiss;
            }
            if (loaded) {
                hp->data.N = N;
                hp->data.opts = o;
                build_legendre_tables(N, hp->data.lt, o.m_lo, o.m_hi);
            } else {
                int rc = idbf::build_all(N, o, hp->data);
                if (rc) {
                    delete hp;
                    return rc;
                }
                auto tp = std::chrono::steady_clock::now();
                idbf::pack_programs(hp->data, hp->packed);
                if (std::getenv("SHT_VERBOSE"))
                    std::fprintf(stderr, "[sht] factors %.2fs, packing %.2fs\n", hp->data.stats.seconds,
                                 std::chrono::duration<double>(std::chrono::steady_clock::now() - tp).count());
                if (hp->cache != idbf::kCacheOff && idbf::cache_store(path, key, hp->packed, hp->data.stats) != SHT_OK)
                    hp->cache = idbf::kCacheOff;
            }
            hp->data.opts.cache_dir = nullptr;  // the caller's string is not kept
        } else {
            hp->data.N = N;
            hp->data.opts = o;
            build_legendre_tables(N, hp->data.lt);
        }
    } catch (const std::bad_alloc &) {
        delete hp;
        return SHT_ERR_OOM;
    }
    *out = hp;
    return SHT_OK;
}

void sht_host_plan_destroy(sht_host_plan_t *hp) { delete hp; }

int sht_host_plan_apply(const sht_host_plan_t *hp, int absm, int parity, int dir, int R, const double *in,
                        double *out) {
    if (!hp || !in || !out || R < 1) return SHT_ERR_INVALID_ARG;
    const int N = hp->data.N;
    if (absm < 0 || absm >= 2 * N || parity < 0 || parity > 1 || (dir != SHT_FWD && dir != SHT_ADJ))
        return SHT_ERR_INVALID_ARG;
    if (hp->method != SHT_IDBF) return SHT_ERR_UNSUPPORTED;
    const int task = 2 * absm + parity;
    const int rows = N, cols = half_cols(N, absm, parity);
    if (cols <= 0) return SHT_OK;
    // run the packed program on panels that are zero outside this task
    const idbf::PackedPlan &pk = hp->packed;
    const bool fwd = dir == SHT_FWD;
    const idbf::Program &p = fwd ? pk.fwd : pk.adj;
    std::vector<double> pin((size_t)p.in_rows * R, 0.0), pout((size_t)p.out_rows * R, 0.0);
    const int64_t ib = fwd ? pk.x_off[task] : pk.y_off[task];
    const int64_t ob = fwd ? pk.y_off[task] : pk.x_off[task];
    const int nin = fwd ? cols : rows, nout = fwd ? rows : cols;
    std::memcpy(&pin[(size_t)ib * R], in, sizeof(double) * (size_t)nin * R);
    // the fused level form where the plan would run it (same arithmetic)
    const bool fused = hp->data.opts.level_schedule == SHT_LEVELS_FUSED && p.fused_ok;
    idbf::host_run_program(p, R, pin.data(), pout.data(), fused);
    if (fwd)
        idbf::host_run_gen_forward(pk.gen_fwd, N, task, task, R, pk.x_off, pk.y_off, pin.data(), pout.data(),
                                   hp->data.lt.xh.data(), hp->data.lt.coef2.data());
    else
        idbf::host_run_gen_adjoint(pk.gen_adj, N, task, task, R, pk.x_off, pk.y_off, pin.data(), pout.data(),
                                   hp->data.lt.xh.data(), hp->data.lt.coef2.data());
    std::memcpy(out, &pout[(size_t)ob * R], sizeof(double) * (size_t)nout * R);
    return SHT_OK;
}

int sht_host_alt_matrix(const sht_host_plan_t *hp, int absm, int parity, double *out) {
    if (!hp || !out) return SHT_ERR_INVALID_ARG;
    const int N = hp->data.N;
    if (absm < 0 || absm >= 2 * N || parity < 0 || parity > 1) return SHT_ERR_INVALID_ARG;
    if (half_cols(N, absm, parity) <= 0) return SHT_OK;
    alt_half_matrix(hp->data.lt, absm, parity, out);
    return SHT_OK;
}

int sht_host_plan_stats(const sht_host_plan_t *hp, char *json, size_t cap) {
    if (!hp) return SHT_ERR_INVALID_ARG;
    std::string s = "{}";
    if (hp->method == SHT_IDBF) {
        s = hp->data.stats_json();
        s.pop_back();
        s += std::string(",\"plan_cache\":\"") + idbf::cache_status_name(hp->cache) + "\"";
        const idbf::PackedPlan &pk = hp->packed;
        s += ",\"fwd_stages\":" + std::to_string(pk.fwd.stages.size()) + ",\"fwd_work_stages\":" +
             std::to_string(pk.fwd.n_work_stages) + ",\"fwd_ops\":" + std::to_string(pk.fwd.ops.size()) +
             ",\"adj_stages\":" + std::to_string(pk.adj.stages.size()) + ",\"scratch_rows\":" +
             std::to_string(std::max(pk.fwd.scr_rows, pk.adj.scr_rows)) + ",\"max_n_out\":" +
             std::to_string(pk.fwd.max_n_out) + ",\"max_n_in\":" + std::to_string(pk.fwd.max_n_in) +
             ",\"fwd_values\":" + std::to_string(pk.fwd.vals.size()) + ",\"adj_values\":" + std::to_string(pk.adj.vals.size()) +
             idbf::fused_stats_json(pk);
        // stored values by sub-op output count (1-8, 9-16, 17-32, 33-64),
        // work stages vs final stage, per program
        for (int d = 0; d < 2; ++d) {
            const idbf::Program &pr = d ? pk.adj : pk.fwd;
            int64_t h[2][4] = {{0}}, nsub[2][4] = {{0}};
            for (size_t si = 0; si < pr.stages.size(); ++si) {
                const int fin = si + 1 == pr.stages.size();
                for (int q = pr.stages[si].op_begin; q < pr.stages[si].op_end; ++q)
                    for (int k = 0; k < pr.ops[q].nsub; ++k) {
                        const idbf::SubOp &so = pr.subs[pr.ops[q].sub0 + k];
                        if (so.n_map == 0) continue;
                        const int b = so.n_map <= 8 ? 0 : so.n_map <= 16 ? 1 : so.n_map <= 32 ? 2 : 3;
                        h[fin][b] += (int64_t)so.n_map * so.n_in;
                        nsub[fin][b] += 1;
                    }
            }
            s += std::string(",\"") + (d ? "adj" : "fwd") + "_nmap_hist\":[";
            for (int f = 0; f < 2; ++f)
                for (int b = 0; b < 4; ++b)
                    s += "[" + std::to_string(h[f][b]) + "," + std::to_string(nsub[f][b]) + "]" + (f == 1 && b == 3 ? "" : ",");
            s += "]";
        }
        {
            // forward program per stage: ops, sub-ops, stored values, outputs,
            // gathered inputs, identity terms
            std::string st = ",\"fwd_stage_detail\":[";
            for (size_t si = 0; si < pk.fwd.stages.size(); ++si) {
                int64_t nops = 0, nsub = 0, nval = 0, nout = 0, nin = 0, ndir = 0;
                for (int q = pk.fwd.stages[si].op_begin; q < pk.fwd.stages[si].op_end; ++q) {
                    const idbf::Op &op = pk.fwd.ops[q];
                    ++nops;
                    nout += op.n_out;
                    for (int k = 0; k < op.nsub; ++k) {
                        const idbf::SubOp &so = pk.fwd.subs[op.sub0 + k];
                        ++nsub;
                        nval += (int64_t)so.n_map * so.n_in;
                        nin += so.n_in;
                        ndir += so.n_dir;
                    }
                }
                st += std::string(si ? "," : "") + "[" + std::to_string(nops) + "," + std::to_string(nsub) + "," +
                      std::to_string(nval) + "," + std::to_string(nout) + "," + std::to_string(nin) + "," +
                      std::to_string(ndir) + "]";
            }
            s += st + "]";
        }
        s += ",\"gen_fwd_items\":" + std::to_string(pk.gen_fwd.items.size()) + ",\"gen_fwd_segs\":" +
             std::to_string(pk.gen_fwd.segs.size()) + ",\"gen_adj_items\":" + std::to_string(pk.gen_adj.items.size()) +
             ",\"gen_adj_segs\":" + std::to_string(pk.gen_adj.segs.size());
        {
            int64_t cols = 0;
            for (auto &sg : pk.gen_adj.segs) cols += sg.ncol;
            s += ",\"gen_adj_seg_cols\":" + std::to_string(cols);
            cols = 0;
            for (auto &sg : pk.gen_fwd.segs) cols += sg.ncol;
            s += ",\"gen_fwd_seg_cols\":" + std::to_string(cols);
            // entries the matrix-core kernels multiply: 16-column groups of the
            // transposed items' 64-column tiles times 64 rows; 8-column steps of
            // the forward segments times 64 rows
            int64_t ea = 0, ef = 0;
            for (auto &it : pk.gen_adj.items)
                for (int q = it.seg_begin; q < it.seg_end; ++q) {
                    const auto &sg = pk.gen_adj.segs[q];
                    for (int g = 0; g < 4; ++g) {
                        const int g0 = it.col0 + 16 * g;
                        if (g0 + 16 > sg.c0 && g0 < sg.c0 + sg.ncol) ea += 16 * 64;
                    }
                }
            for (auto &sg : pk.gen_fwd.segs) ef += (int64_t)((sg.ncol + 7) / 8) * 8 * 64;
            s += ",\"gen_adj_mfma_entries\":" + std::to_string(ea) + ",\"gen_fwd_mfma_entries\":" + std::to_string(ef);
        }
        s += "}";
    }
    if (json && cap) {
        size_t n = std::min(cap - 1, s.size());
        std::memcpy(json, s.data(), n);
        json[n] = 0;
    }
    return (int)s.size() + 1;
}

}  // extern "C"
