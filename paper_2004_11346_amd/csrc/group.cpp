// Grouped transforms (include/sht.h, sht_group_*): tables per distinct
// degree, descriptors and work queues on the device, persistent launches,
// a small autotuner for the persistent grid sizes and hipGraph capture of the
// steady-state call sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "group.h"
#include "kernels.h"
#include "prof.h"
#include "sht.h"
#include "sht_internal.h"

using namespace sht;
using namespace sht::group;

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

struct Table {
    int N = 0, M = 0;
    DevBuf xh, wh, dmant, dexp, coef, tw2, tw2f, src_pos;
    std::vector<int> radix, blen;
};

template <typename V>
hipError_t put(const std::vector<V> &h, DevBuf &d) {
    hipError_t e = hipMalloc(&d.p, std::max<size_t>(1, h.size() * sizeof(V)));
    if (e != hipSuccess) return e;
    if (h.empty()) return hipSuccess;
    return hipMemcpy(d.p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice);
}

int hip_err(hipError_t e, const char *what) {
    std::string s = std::string(what) + ": " + hipGetErrorString(e);
    set_error_detail(s);
    return e == hipErrorOutOfMemory ? SHT_ERR_OOM : SHT_ERR_HIP;
}

}  // namespace

struct sht_group {
    int n = 0, dtype = 0, device = 0, cus = 0;
    std::vector<int> Ns, fields;
    std::vector<Table *> tabs;
    std::vector<int> tab_of;
    std::vector<GTrans> h_tr;
    DevBuf d_tr, d_items[4], d_counters, d_g;
    int nitems[4] = {0, 0, 0, 0};
    int grid[4] = {0, 0, 0, 0};
    int max_M = 0;
    bool bound = false, tuned = false;
    std::string tune_log;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipGraph_t graph_def[2] = {nullptr, nullptr};
    ~sht_group() {
        for (int i = 0; i < 2; ++i) {
            if (graph[i]) (void)hipGraphExecDestroy(graph[i]);
            if (graph_def[i]) (void)hipGraphDestroy(graph_def[i]);
        }
        for (Table *t : tabs) delete t;
    }
    void drop_graphs() {
        for (int i = 0; i < 2; ++i) {
            if (graph[i]) (void)hipGraphExecDestroy(graph[i]);
            if (graph_def[i]) (void)hipGraphDestroy(graph_def[i]);
            graph[i] = nullptr;
            graph_def[i] = nullptr;
        }
    }
};

namespace {

// the phases of one direction: forward = ALT then synthesis; inverse =
// analysis then transposed ALT
const int kPhases[2][2] = {{kFwdAlt, kDftSyn}, {kDftAna, kAdjAlt}};

int run_dir(const sht_group_t *g, int dir, hipStream_t s) {
    hipError_t e = launch_reset((int *)g->d_counters.p, 4, s);
    if (e != hipSuccess) return hip_err(e, "group counter reset");
    for (int k = 0; k < 2; ++k) {
        const int ph = kPhases[dir][k];
        e = launch_phase(ph, g->dtype, g->grid[ph], (const GTrans *)g->d_tr.p, (const GItem *)g->d_items[ph].p,
                         g->nitems[ph], (int *)g->d_counters.p + ph, g->max_M, s);
        if (e != hipSuccess) return hip_err(e, "group launch");
    }
    return SHT_OK;
}

}  // namespace

extern "C" {

int sht_group_create(int n, const int *Ns, const int *fields, int dtype, sht_group_t **out) {
    if (!out || n < 1 || !Ns || !fields) return SHT_ERR_INVALID_ARG;
    *out = nullptr;
    if (dtype != SHT_F64 && dtype != SHT_F32) return SHT_ERR_INVALID_ARG;
    for (int i = 0; i < n; ++i) {
        if (Ns[i] < 1 || Ns[i] > 1024 || fields[i] < 1 || fields[i] > 4) {
            set_error_detail("group transforms need 1 <= N <= 1024 and 1 <= fields <= 4");
            return SHT_ERR_INVALID_ARG;
        }
    }
    sht_group *g = new (std::nothrow) sht_group;
    if (!g) return SHT_ERR_OOM;
    std::unique_ptr<sht_group> guard(g);
    g->n = n;
    g->dtype = dtype;
    g->Ns.assign(Ns, Ns + n);
    g->fields.assign(fields, fields + n);
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) return hip_err(e, "hipGetDevice");
    e = hipDeviceGetAttribute(&g->cus, hipDeviceAttributeMultiprocessorCount, g->device);
    if (e != hipSuccess) return hip_err(e, "device attributes");
    if ((e = init_attributes()) != hipSuccess) return hip_err(e, "kernel attributes");
    try {
        std::map<int, int> idx;
        for (int i = 0; i < n; ++i) {
            auto it = idx.find(Ns[i]);
            if (it == idx.end()) {
                const int N = Ns[i];
                Table *t = new Table;
                g->tabs.push_back(t);
                idx[N] = (int)g->tabs.size() - 1;
                t->N = N;
                t->M = 4 * N - 1;
                LegendreTables lt;
                build_legendre_tables(N, lt);
                if ((e = put(lt.xh, t->xh)) != hipSuccess || (e = put(lt.wh, t->wh)) != hipSuccess ||
                    (e = put(lt.diag_m, t->dmant)) != hipSuccess || (e = put(lt.diag_e, t->dexp)) != hipSuccess ||
                    (e = put(lt.coef, t->coef)) != hipSuccess)
                    return hip_err(e, "group tables");
                std::vector<int> sp;
                dev::dft_passes(t->M, t->radix, t->blen, sp);
                if ((int)t->radix.size() > kMaxPass) return SHT_ERR_UNSUPPORTED;
                std::vector<double> tw(4 * (size_t)t->M);
                std::vector<float> twf(4 * (size_t)t->M);
                const long double pi = 3.141592653589793238462643383279502884L;
                for (int r = 0; r < 2 * t->M; ++r) {
                    const long double ph = pi * r / t->M;
                    tw[2 * r] = (double)cosl(ph);
                    tw[2 * r + 1] = (double)sinl(ph);
                    twf[2 * r] = (float)cosl(ph);
                    twf[2 * r + 1] = (float)sinl(ph);
                }
                if ((e = put(tw, t->tw2)) != hipSuccess || (e = put(twf, t->tw2f)) != hipSuccess ||
                    (e = put(sp, t->src_pos)) != hipSuccess)
                    return hip_err(e, "group DFT tables");
            }
            g->tab_of.push_back(idx[Ns[i]]);
        }
        // descriptors (buffers bound later) and workspace for the inverse
        size_t goff = 0;
        std::vector<size_t> gofs;
        const size_t es = dtype == SHT_F64 ? 16 : 8;
        for (int i = 0; i < n; ++i) {
            gofs.push_back(goff);
            goff += es * (size_t)fields[i] * 2 * Ns[i] * (4 * Ns[i] - 1);
            g->max_M = std::max(g->max_M, 4 * Ns[i] - 1);
        }
        if (es * (size_t)g->max_M > 150 * 1024) return SHT_ERR_UNSUPPORTED;
        if ((e = hipMalloc(&g->d_g.p, std::max<size_t>(goff, 16))) != hipSuccess) return hip_err(e, "group workspace");
        g->h_tr.resize(n);
        for (int i = 0; i < n; ++i) {
            const Table *t = g->tabs[g->tab_of[i]];
            GTrans &d = g->h_tr[i];
            std::memset(&d, 0, sizeof d);
            d.N = t->N;
            d.M = t->M;
            d.fields = fields[i];
            d.xh = (const double *)t->xh.p;
            d.wh = (const double *)t->wh.p;
            d.dmant = (const double *)t->dmant.p;
            d.coef = (const double *)t->coef.p;
            d.dexp = (const int *)t->dexp.p;
            d.tw2 = (const double *)t->tw2.p;
            d.tw2f = (const float *)t->tw2f.p;
            d.src_pos = (const int *)t->src_pos.p;
            d.npass = (int)t->radix.size();
            for (int q = 0; q < d.npass; ++q) {
                d.R[q] = t->radix[q];
                d.L[q] = t->blen[q];
            }
            d.g = (char *)g->d_g.p + gofs[i];
        }
        if ((e = put(g->h_tr, *(DevBuf *)&g->d_tr)) != hipSuccess) return hip_err(e, "group descriptors");
        // work queues, longest first
        struct W {
            double cost;
            GItem it;
        };
        std::vector<W> q[4];
        const int tile = fwd_rows_per_tile();
        for (int i = 0; i < n; ++i) {
            const int N = Ns[i], f = fields[i], M = 4 * N - 1;
            for (int a = 0; a < 2 * N; ++a) {
                for (int b = 0; b * tile < N; ++b)
                    q[kFwdAlt].push_back({(double)(2 * N - a) * f * std::min(tile, N - b * tile), {i, a, b, 0}});
                q[kAdjAlt].push_back({(double)(2 * N - a) * N * f, {i, a, 0, 0}});
            }
            const double dc = M * std::log2((double)M + 1.0);
            for (int fb = 0; fb < f; ++fb)
                for (int r = 0; r < 2 * N; ++r) {
                    q[kDftSyn].push_back({dc, {i, fb, r, 0}});
                    q[kDftAna].push_back({dc, {i, fb, r, 0}});
                }
        }
        for (int ph = 0; ph < 4; ++ph) {
            std::stable_sort(q[ph].begin(), q[ph].end(), [](const W &x, const W &y) { return x.cost > y.cost; });
            std::vector<GItem> items;
            for (const W &w : q[ph]) items.push_back(w.it);
            g->nitems[ph] = (int)items.size();
            if ((e = put(items, g->d_items[ph])) != hipSuccess) return hip_err(e, "group work queue");
        }
        if ((e = hipMalloc(&g->d_counters.p, 4 * sizeof(int))) != hipSuccess) return hip_err(e, "group counters");
    } catch (const std::bad_alloc &) {
        return SHT_ERR_OOM;
    }
    // untuned defaults: enough persistent workgroups to fill every CU
    g->grid[kFwdAlt] = 16 * g->cus;
    g->grid[kAdjAlt] = 4 * g->cus;
    g->grid[kDftSyn] = 2 * g->cus;
    g->grid[kDftAna] = 2 * g->cus;
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_err(e, "group setup");
    *out = guard.release();
    return SHT_OK;
}

void sht_group_destroy(sht_group_t *g) { delete g; }

int sht_group_bind(sht_group_t *g, void *const *beta, void *const *f) {
    if (!g || !beta || !f) return SHT_ERR_INVALID_ARG;
    const size_t al = g->dtype == SHT_F64 ? 8 : 4;
    for (int i = 0; i < g->n; ++i) {
        if (!beta[i] || !f[i] || ((uintptr_t)beta[i] % al) || ((uintptr_t)f[i] % al)) return SHT_ERR_MISALIGNED;
        g->h_tr[i].beta = beta[i];
        g->h_tr[i].f = f[i];
    }
    hipError_t e = hipMemcpy(g->d_tr.p, g->h_tr.data(), sizeof(GTrans) * g->n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_err(e, "group bind");
    g->drop_graphs();
    g->bound = true;
    return SHT_OK;
}

int sht_group_forward(sht_group_t *g, void *stream) {
    if (!g || !g->bound) return SHT_ERR_INVALID_ARG;
    return run_dir(g, 0, (hipStream_t)stream);
}

int sht_group_inverse(sht_group_t *g, void *stream) {
    if (!g || !g->bound) return SHT_ERR_INVALID_ARG;
    return run_dir(g, 1, (hipStream_t)stream);
}

int sht_group_tune(sht_group_t *g, void *stream) {
    if (!g || !g->bound) return SHT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SHT_ERR_HIP;
    std::ostringstream log;
    log << "{";
    const char *names[4] = {"fwd_alt", "adj_alt", "dft_synthesis", "dft_analysis"};
    const int mult[4][4] = {{4, 8, 16, 32}, {2, 4, 6, 8}, {1, 2, 3, 4}, {1, 2, 3, 4}};
    // analysis reads f and writes the workspace; synthesis runs in place on f
    // and the ALT phases overwrite their outputs, so every candidate computes
    // the same thing
    const int order[4] = {kDftAna, kAdjAlt, kFwdAlt, kDftSyn};
    int rc = SHT_OK;
    for (int oi = 0; oi < 4 && rc == SHT_OK; ++oi) {
        const int ph = order[oi];
        float best = 1e30f;
        int best_grid = g->grid[ph];
        log << (oi ? ", " : "") << "\"" << names[ph] << "\": {";
        for (int c = 0; c < 4; ++c) {
            const int grid = mult[ph][c] * g->cus;
            float ms = 0.f;
            for (int rep = 0; rep < 3 && rc == SHT_OK; ++rep) {
                hipError_t e = launch_reset((int *)g->d_counters.p, 4, s);
                if (e == hipSuccess) e = hipEventRecord(e0, s);
                if (e == hipSuccess)
                    e = launch_phase(ph, g->dtype, grid, (const GTrans *)g->d_tr.p, (const GItem *)g->d_items[ph].p,
                                     g->nitems[ph], (int *)g->d_counters.p + ph, g->max_M, s);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float t = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
                if (e != hipSuccess) rc = hip_err(e, "group tuning");
                if (rep > 0) ms += t;  // first run warms up
            }
            ms /= 2;
            log << (c ? ", " : "") << "\"" << grid << "\": " << ms;
            if (ms < best) {
                best = ms;
                best_grid = grid;
            }
        }
        log << ", \"chosen\": " << best_grid << "}";
        g->grid[ph] = best_grid;
    }
    log << "}";
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    g->tune_log = log.str();
    g->tuned = true;
    g->drop_graphs();
    return SHT_OK;
}

int sht_group_capture(sht_group_t *g, int dir, void *stream) {
    if (!g || !g->bound || (dir != SHT_FWD && dir != SHT_INV)) return SHT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (!s) {
        set_error_detail("graph capture needs a non-default stream");
        return SHT_ERR_INVALID_ARG;
    }
    const int k = dir == SHT_FWD ? 0 : 1;
    if (g->graph[k]) (void)hipGraphExecDestroy(g->graph[k]);
    if (g->graph_def[k]) (void)hipGraphDestroy(g->graph_def[k]);
    g->graph[k] = nullptr;
    g->graph_def[k] = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_err(e, "begin capture");
    int rc = run_dir(g, k, s);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_err(e, "end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_err(e, "graph instantiate");
    }
    g->graph_def[k] = graph;
    g->graph[k] = exec;
    return SHT_OK;
}

int sht_group_replay(sht_group_t *g, int dir, void *stream) {
    if (!g || (dir != SHT_FWD && dir != SHT_INV)) return SHT_ERR_INVALID_ARG;
    const int k = dir == SHT_FWD ? 0 : 1;
    if (!g->graph[k]) {
        set_error_detail("no graph captured for this direction (or the group was re-bound or re-tuned)");
        return SHT_ERR_INVALID_ARG;
    }
    hipError_t e = hipGraphLaunch(g->graph[k], (hipStream_t)stream);
    if (e != hipSuccess) return hip_err(e, "graph launch");
    return SHT_OK;
}

int sht_group_stats(const sht_group_t *g, char *json, size_t cap) {
    if (!g) return SHT_ERR_INVALID_ARG;
    std::ostringstream os;
    os << "{\"transforms\": " << g->n << ", \"distinct_N\": " << g->tabs.size() << ", \"cus\": " << g->cus
       << ", \"items\": {\"fwd_alt\": " << g->nitems[kFwdAlt] << ", \"adj_alt\": " << g->nitems[kAdjAlt]
       << ", \"dft\": " << g->nitems[kDftSyn] << "}, \"grid\": {\"fwd_alt\": " << g->grid[kFwdAlt]
       << ", \"adj_alt\": " << g->grid[kAdjAlt] << ", \"dft_synthesis\": " << g->grid[kDftSyn]
       << ", \"dft_analysis\": " << g->grid[kDftAna] << "}, \"tuned\": " << (g->tuned ? "true" : "false");
    if (g->tuned) os << ", \"tuning_ms\": " << g->tune_log;
    os << "}";
    const std::string s = os.str();
    if (json && cap) {
        const size_t k = std::min(cap - 1, s.size());
        std::memcpy(json, s.data(), k);
        json[k] = 0;
    }
    return (int)s.size() + 1;
}

}  // extern "C"
