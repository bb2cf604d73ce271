// Grouped transforms (include/sht.h, sht_group_*): tables per distinct
// degree, descriptors and work queues on the device, persistent launches,
// a small autotuner for the persistent grid sizes and hipGraph capture of the
// steady-state call sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "dft_device.h"
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
    DevBuf xh, wh, dmant, dexp, coef, tab, tabf, src_pos;
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

// Batched mode: the transforms of one degree N form one batch of sum(fields)
// fields, run by one plan (plain or fast form, chosen by the tuner) on
// staging buffers; segment copies move each transform's fields in and out.
struct BatchClass {
    int N = 0, fields = 0;
    std::vector<int> members;  // transform indices, in order
    sht_plan_t *plan = nullptr;
    std::string choice = "dense";  // "dense" or "idbf" (+ leaf)
    int leaf = 0;
    double fwd_ms = -1.0, inv_ms = -1.0;
    DevBuf beta_stage, f_stage;
    DevBuf segs_beta, segs_f;  // CopySeg per member
    int64_t max_units_beta = 0, max_units_f = 0;
    ~BatchClass() {
        if (plan) sht_plan_destroy(plan);
    }
};

struct sht_group {
    int n = 0, dtype = 0, device = 0, cus = 0;
    int mode = SHT_GROUP_PERSISTENT;
    std::vector<BatchClass *> classes;
    std::string tune_file, plan_cache_dir, arch;
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
        for (BatchClass *c : classes) delete c;
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

// ---------------------------------------------------------------- batched mode

int plan_for(const sht_group_t *g, BatchClass *c, const std::string &method, int leaf, sht_plan_t **out) {
    sht_plan_opts o;
    sht_plan_opts_default(&o);
    o.leaf = leaf;
    if (!g->plan_cache_dir.empty()) o.cache_dir = g->plan_cache_dir.c_str();
    return sht_plan_create(c->N, c->fields, g->dtype, method == "idbf" ? SHT_IDBF : SHT_DENSE, &o, out);
}

int run_class(const sht_group_t *g, const BatchClass *c, int dir, hipStream_t s) {
    const bool direct = c->members.size() == 1;
    void *beta = direct ? g->h_tr[c->members[0]].beta : c->beta_stage.p;
    void *f = direct ? g->h_tr[c->members[0]].f : c->f_stage.p;
    const int nm = (int)c->members.size();
    hipError_t e;
    int rc;
    if (dir == 0) {
        if (!direct && (e = launch_copy_segs((const CopySeg *)c->segs_beta.p, nm, c->max_units_beta, 1, s)))
            return hip_err(e, "group gather");
        if ((rc = sht_forward(c->plan, beta, f, s))) return rc;
        if (!direct && (e = launch_copy_segs((const CopySeg *)c->segs_f.p, nm, c->max_units_f, 0, s)))
            return hip_err(e, "group scatter");
    } else {
        if (!direct && (e = launch_copy_segs((const CopySeg *)c->segs_f.p, nm, c->max_units_f, 1, s)))
            return hip_err(e, "group gather");
        if ((rc = sht_inverse(c->plan, f, beta, s))) return rc;
        if (!direct && (e = launch_copy_segs((const CopySeg *)c->segs_beta.p, nm, c->max_units_beta, 0, s)))
            return hip_err(e, "group scatter");
    }
    return SHT_OK;
}

int run_batched(const sht_group_t *g, int dir, hipStream_t s) {
    for (const BatchClass *c : g->classes) {
        const int rc = run_class(g, c, dir, s);
        if (rc) return rc;
    }
    return SHT_OK;
}

int run_any(const sht_group_t *g, int dir, hipStream_t s) {
    return g->mode == SHT_GROUP_BATCHED ? run_batched(g, dir, s) : run_dir(g, dir, s);
}

const char *dtype_name(int dtype) { return dtype == SHT_F64 ? "f64" : "f32"; }

// tuned choices, one JSON object per line:
// {"arch": "...", "N": n, "R": r, "dtype": "f64", "method": "idbf", "leaf": l, "fwd_ms": t, "inv_ms": t}
struct TuneEntry {
    std::string arch, dtype, method;
    int N = 0, R = 0, leaf = 0;
    double fwd_ms = 0, inv_ms = 0;
};

std::string json_str(const std::string &line, const char *key) {
    const std::string k = std::string("\"") + key + "\": \"";
    const size_t a = line.find(k);
    if (a == std::string::npos) return "";
    const size_t b = line.find('"', a + k.size());
    return b == std::string::npos ? "" : line.substr(a + k.size(), b - a - k.size());
}

double json_num(const std::string &line, const char *key, double dflt) {
    const std::string k = std::string("\"") + key + "\": ";
    const size_t a = line.find(k);
    if (a == std::string::npos) return dflt;
    return std::atof(line.c_str() + a + k.size());
}

std::vector<TuneEntry> read_tune_file(const std::string &path) {
    std::vector<TuneEntry> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        TuneEntry t;
        t.arch = json_str(line, "arch");
        t.dtype = json_str(line, "dtype");
        t.method = json_str(line, "method");
        t.N = (int)json_num(line, "N", 0);
        t.R = (int)json_num(line, "R", 0);
        t.leaf = (int)json_num(line, "leaf", 0);
        t.fwd_ms = json_num(line, "fwd_ms", 0);
        t.inv_ms = json_num(line, "inv_ms", 0);
        if (!t.arch.empty() && t.N > 0 && (t.method == "dense" || t.method == "idbf")) out.push_back(t);
    }
    return out;
}

void write_tune_file(const std::string &path, const std::vector<TuneEntry> &es) {
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return;
        f << "{\"entries\": [\n";
        for (size_t i = 0; i < es.size(); ++i) {
            const TuneEntry &t = es[i];
            f << "{\"arch\": \"" << t.arch << "\", \"N\": " << t.N << ", \"R\": " << t.R << ", \"dtype\": \""
              << t.dtype << "\", \"method\": \"" << t.method << "\", \"leaf\": " << t.leaf
              << ", \"fwd_ms\": " << t.fwd_ms << ", \"inv_ms\": " << t.inv_ms << "}"
              << (i + 1 < es.size() ? "," : "") << "\n";
        }
        f << "]}\n";
    }
    std::rename(tmp.c_str(), path.c_str());
}

int setup_batched(sht_group_t *g) {
    std::map<int, BatchClass *> byN;
    for (int i = 0; i < g->n; ++i) {
        BatchClass *&c = byN[g->Ns[i]];
        if (!c) {
            c = new BatchClass;
            c->N = g->Ns[i];
            g->classes.push_back(c);
        }
        c->members.push_back(i);
        c->fields += g->fields[i];
    }
    std::vector<TuneEntry> tuned;
    if (!g->tune_file.empty()) tuned = read_tune_file(g->tune_file);
    const size_t es = g->dtype == SHT_F64 ? 16 : 8;
    for (BatchClass *c : g->classes) {
        for (const TuneEntry &t : tuned)
            if (t.arch == g->arch && t.N == c->N && t.R == 4 * c->fields && t.dtype == dtype_name(g->dtype)) {
                c->choice = t.method;
                c->leaf = t.leaf;
                c->fwd_ms = t.fwd_ms;
                c->inv_ms = t.inv_ms;
            }
        int rc = plan_for(g, c, c->choice, c->leaf, &c->plan);
        if (rc) return rc;
        if (c->members.size() > 1) {
            const int64_t M = 4 * (int64_t)c->N - 1;
            hipError_t e;
            if ((e = hipMalloc(&c->beta_stage.p, es * c->fields * 4 * (int64_t)c->N * c->N)) != hipSuccess ||
                (e = hipMalloc(&c->f_stage.p, es * c->fields * 2 * (int64_t)c->N * M)) != hipSuccess ||
                (e = hipMalloc(&c->segs_beta.p, sizeof(CopySeg) * c->members.size())) != hipSuccess ||
                (e = hipMalloc(&c->segs_f.p, sizeof(CopySeg) * c->members.size())) != hipSuccess)
                return hip_err(e, "group staging buffers");
        }
    }
    return SHT_OK;
}

int bind_batched(sht_group_t *g) {
    const size_t es = g->dtype == SHT_F64 ? 16 : 8;
    for (BatchClass *c : g->classes) {
        if (c->members.size() <= 1) continue;
        const int64_t N = c->N, M = 4 * N - 1;
        std::vector<CopySeg> sb, sf;
        int64_t off = 0;
        c->max_units_beta = c->max_units_f = 0;
        for (int i : c->members) {
            const int64_t nf = g->fields[i];
            const int64_t ub = nf * 4 * N * N * (int64_t)es / 8, uf = nf * 2 * N * M * (int64_t)es / 8;
            sb.push_back({g->h_tr[i].beta, (char *)c->beta_stage.p + off * 4 * N * N * es, ub});
            sf.push_back({g->h_tr[i].f, (char *)c->f_stage.p + off * 2 * N * M * es, uf});
            c->max_units_beta = std::max(c->max_units_beta, ub);
            c->max_units_f = std::max(c->max_units_f, uf);
            off += nf;
        }
        hipError_t e;
        if ((e = hipMemcpy(c->segs_beta.p, sb.data(), sizeof(CopySeg) * sb.size(), hipMemcpyHostToDevice)) !=
                hipSuccess ||
            (e = hipMemcpy(c->segs_f.p, sf.data(), sizeof(CopySeg) * sf.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_err(e, "group bind");
    }
    return SHT_OK;
}

// time one class's forward and inverse (ms per call, after one warm-up)
int time_class(const sht_group_t *g, const BatchClass *c, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
               double &fwd, double &inv) {
    for (int dir = 0; dir < 2; ++dir) {
        int rc = run_class(g, c, dir, s);
        if (rc) return rc;
        hipError_t e = hipEventRecord(e0, s);
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
            if ((rc = run_class(g, c, dir, s))) return rc;
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) return hip_err(e, "group tuning");
        (dir == 0 ? fwd : inv) = ms / 3.0;
    }
    return SHT_OK;
}

int tune_batched(sht_group_t *g, hipStream_t s) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SHT_ERR_HIP;
    std::ostringstream log;
    log << "{";
    int rc = SHT_OK;
    std::vector<TuneEntry> file;
    if (!g->tune_file.empty()) file = read_tune_file(g->tune_file);
    for (size_t ci = 0; ci < g->classes.size() && rc == SHT_OK; ++ci) {
        BatchClass *c = g->classes[ci];
        std::vector<std::pair<std::string, int>> cand = {{"dense", 0}, {"idbf", 0}};
        if (c->N >= 256) {
            cand.push_back({"idbf", 32});
            cand.push_back({"idbf", 64});
        }
        log << (ci ? ", " : "") << "\"N=" << c->N << " R=" << 4 * c->fields << "\": {";
        double best = 1e300;
        sht_plan_t *best_plan = nullptr;
        std::string best_m;
        int best_leaf = 0;
        double bf = 0, bi = 0;
        for (size_t k = 0; k < cand.size() && rc == SHT_OK; ++k) {
            sht_plan_t *p = nullptr;
            if ((rc = plan_for(g, c, cand[k].first, cand[k].second, &p))) break;
            sht_plan_t *keep = c->plan;
            c->plan = p;
            double fw = 0, iv = 0;
            rc = time_class(g, c, s, e0, e1, fw, iv);
            c->plan = keep;
            log << (k ? ", " : "") << "\"" << cand[k].first << ":" << cand[k].second << "\": [" << fw << ", " << iv
                << "]";
            if (rc == SHT_OK && fw + iv < best) {
                best = fw + iv;
                if (best_plan) sht_plan_destroy(best_plan);
                best_plan = p;
                best_m = cand[k].first;
                best_leaf = cand[k].second;
                bf = fw;
                bi = iv;
            } else {
                sht_plan_destroy(p);
            }
        }
        log << "}";
        if (rc == SHT_OK && best_plan) {
            sht_plan_destroy(c->plan);
            c->plan = best_plan;
            c->choice = best_m;
            c->leaf = best_leaf;
            c->fwd_ms = bf;
            c->inv_ms = bi;
            TuneEntry t;
            t.arch = g->arch;
            t.dtype = dtype_name(g->dtype);
            t.method = best_m;
            t.N = c->N;
            t.R = 4 * c->fields;
            t.leaf = best_leaf;
            t.fwd_ms = bf;
            t.inv_ms = bi;
            bool found = false;
            for (TuneEntry &x : file)
                if (x.arch == t.arch && x.N == t.N && x.R == t.R && x.dtype == t.dtype) {
                    x = t;
                    found = true;
                }
            if (!found) file.push_back(t);
        } else if (best_plan) {
            sht_plan_destroy(best_plan);
        }
    }
    log << "}";
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (!g->tune_file.empty()) write_tune_file(g->tune_file, file);
    g->tune_log = log.str();
    return SHT_OK;
}

}  // namespace

extern "C" {

void sht_group_opts_default(sht_group_opts *o) {
    if (!o) return;
    o->mode = SHT_GROUP_PERSISTENT;
    o->tune_file = nullptr;
    o->plan_cache_dir = nullptr;
}

int sht_group_create(int n, const int *Ns, const int *fields, int dtype, sht_group_t **out) {
    return sht_group_create_ex(n, Ns, fields, dtype, nullptr, out);
}

int sht_group_create_ex(int n, const int *Ns, const int *fields, int dtype, const sht_group_opts *opts,
                        sht_group_t **out) {
    if (!out || n < 1 || !Ns || !fields) return SHT_ERR_INVALID_ARG;
    *out = nullptr;
    if (dtype != SHT_F64 && dtype != SHT_F32) return SHT_ERR_INVALID_ARG;
    sht_group_opts o;
    sht_group_opts_default(&o);
    if (opts) o = *opts;
    if (o.mode != SHT_GROUP_PERSISTENT && o.mode != SHT_GROUP_BATCHED) return SHT_ERR_INVALID_ARG;
    const bool batched = o.mode == SHT_GROUP_BATCHED;
    for (int i = 0; i < n; ++i) {
        if (Ns[i] < 1 || Ns[i] > (batched ? 8192 : 1024) || fields[i] < 1 || (!batched && fields[i] > 4)) {
            set_error_detail(batched ? "batched groups need 1 <= N <= 8192 and fields >= 1"
                                     : "group transforms need 1 <= N <= 1024 and 1 <= fields <= 4");
            return SHT_ERR_INVALID_ARG;
        }
    }
    sht_group *g = new (std::nothrow) sht_group;
    if (!g) return SHT_ERR_OOM;
    std::unique_ptr<sht_group> guard(g);
    g->n = n;
    g->dtype = dtype;
    g->mode = o.mode;
    if (o.tune_file) g->tune_file = o.tune_file;
    if (o.plan_cache_dir) g->plan_cache_dir = o.plan_cache_dir;
    g->Ns.assign(Ns, Ns + n);
    g->fields.assign(fields, fields + n);
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) return hip_err(e, "hipGetDevice");
    e = hipDeviceGetAttribute(&g->cus, hipDeviceAttributeMultiprocessorCount, g->device);
    if (e != hipSuccess) return hip_err(e, "device attributes");
    {
        hipDeviceProp_t prop;
        if ((e = hipGetDeviceProperties(&prop, g->device)) != hipSuccess) return hip_err(e, "device properties");
        g->arch = prop.gcnArchName;
    }
    if (batched) {
        g->h_tr.assign(n, GTrans{});
        int rc;
        try {
            rc = setup_batched(g);
        } catch (const std::bad_alloc &) {
            return SHT_ERR_OOM;
        }
        if (rc) return rc;
        *out = guard.release();
        return SHT_OK;
    }
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
                dev::DftHost dh;
                dev::dft_build(t->M, dtype, dh, 1, false);
                if (dh.kind != dev::kDftRows || (int)dh.radix.size() > kMaxPass) return SHT_ERR_UNSUPPORTED;
                t->radix = dh.radix;
                t->blen = dh.blen;
                if ((e = put(dh.tab, t->tab)) != hipSuccess || (e = put(dh.tabf, t->tabf)) != hipSuccess ||
                    (e = put(dh.src_pos, t->src_pos)) != hipSuccess)
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
        if (es * ((size_t)g->max_M + 1) + 16 * (size_t)dev::dft::tab_entries(g->max_M) > kGroupDftLds)
            return SHT_ERR_UNSUPPORTED;
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
            d.tab = (const double *)t->tab.p;
            d.tabf = (const float *)t->tabf.p;
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
    const size_t al = g->dtype == SHT_F64 ? 16 : 8;  // complex elements
    for (int i = 0; i < g->n; ++i) {
        if (!beta[i] || !f[i] || ((uintptr_t)beta[i] % al) || ((uintptr_t)f[i] % al)) return SHT_ERR_MISALIGNED;
        g->h_tr[i].beta = beta[i];
        g->h_tr[i].f = f[i];
    }
    g->drop_graphs();
    if (g->mode == SHT_GROUP_BATCHED) {
        const int rc = bind_batched(g);
        if (rc) return rc;
        g->bound = true;
        return SHT_OK;
    }
    hipError_t e = hipMemcpy(g->d_tr.p, g->h_tr.data(), sizeof(GTrans) * g->n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_err(e, "group bind");
    g->bound = true;
    return SHT_OK;
}

int sht_group_forward(sht_group_t *g, void *stream) {
    if (!g || !g->bound) return SHT_ERR_INVALID_ARG;
    return run_any(g, 0, (hipStream_t)stream);
}

int sht_group_inverse(sht_group_t *g, void *stream) {
    if (!g || !g->bound) return SHT_ERR_INVALID_ARG;
    return run_any(g, 1, (hipStream_t)stream);
}

int sht_group_tune(sht_group_t *g, void *stream) {
    if (!g || !g->bound) return SHT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (g->mode == SHT_GROUP_BATCHED) {
        const int rc = tune_batched(g, s);
        if (rc) return rc;
        g->tuned = true;
        g->drop_graphs();
        return SHT_OK;
    }
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
    int rc = run_any(g, k, s);
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
    if (g->mode == SHT_GROUP_BATCHED) {
        os << "{\"transforms\": " << g->n << ", \"mode\": \"batched\", \"arch\": \"" << g->arch
           << "\", \"classes\": [";
        for (size_t i = 0; i < g->classes.size(); ++i) {
            const BatchClass *c = g->classes[i];
            os << (i ? ", " : "") << "{\"N\": " << c->N << ", \"fields\": " << c->fields << ", \"transforms\": "
               << c->members.size() << ", \"method\": \"" << c->choice << "\", \"leaf\": " << c->leaf
               << ", \"fwd_ms\": " << c->fwd_ms << ", \"inv_ms\": " << c->inv_ms << "}";
        }
        os << "], \"tuned\": " << (g->tuned ? "true" : "false");
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
