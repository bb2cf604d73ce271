// C-ABI entry points (include/sht.h): plan construction, upload and the
// forward / inverse / adjoint / ALT-only calls.  Every transform call only
// enqueues HIP kernels on the caller's stream; nothing here computes a
// transform on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "idbf.h"
#include "kernels.h"
#include "plan_cache.h"
#include "prof.h"
#include "sht_internal.h"

namespace sht {

static thread_local std::string g_detail;
void set_error_detail(const std::string &msg) { g_detail = msg; }

}  // namespace sht

using namespace sht;

struct sht_plan {
    int N = 0, M = 0, batch = 0, dtype = 0, method = 0, device = 0;
    bool dft_ok = true;
    sht_plan_opts opts{};
    std::vector<double> x, w;  // full rule, ascending
    // device tables
    double *d_xh = nullptr, *d_wh = nullptr, *d_dmant = nullptr, *d_coef = nullptr, *d_coef2 = nullptr;
    int *d_dexp = nullptr;
    // phi DFT tables and the four-step intermediate rows
    double *d_tab = nullptr, *d_ctab = nullptr, *d_bspec = nullptr;
    float *d_tabf = nullptr, *d_ctabf = nullptr, *d_bspecf = nullptr;
    int *d_src_pos = nullptr, *d_src_pos2 = nullptr, *d_inslot = nullptr, *d_outslot = nullptr;
    // Rader last passes of the two pass lists
    double *d_rl_ctab[2] = {nullptr, nullptr}, *d_rl_bspec[2] = {nullptr, nullptr};
    float *d_rl_bspecf[2] = {nullptr, nullptr};
    int *d_rl_inslot[2] = {nullptr, nullptr}, *d_rl_outslot[2] = {nullptr, nullptr};
    void *d_dft_scr = nullptr;
    dev::DenseTables dense;
    dev::DftPlan dft;
    // workspace
    void *d_g = nullptr;         // [batch][2N][M] complex (dtype)
    void *d_bz = nullptr;        // [batch][4N^2] complex: coefficients of real-field pairs
    void *d_X = nullptr;         // dense path FP64 panels
    void *d_Y = nullptr;
    int64_t *d_x_off = nullptr;
    int32_t *d_adj_items = nullptr, *d_adj_task_first = nullptr;  // dense transposed product
    double *d_ck = nullptr;
    int32_t *d_ckexp = nullptr;
    dev::DensePanels panels;
    // IDBF program (device)
    idbf::DeviceProgram prog;
    std::string stats;
    double build_seconds = 0.0;
    // per-kernel timing (off unless sht_profile enables it)
    bool profiling = false;
    mutable prof::Recorder recorder;
    prof::Recorder *rec() const { return profiling ? &recorder : nullptr; }
    // calls on one plan are ordered: the mutex serialises host threads, the
    // event makes a call on another stream wait for the previous call's work
    mutable std::mutex mu;
    mutable hipEvent_t last_done = nullptr;
    mutable hipStream_t last_stream = nullptr;
    mutable bool has_last = false;
    // graph mode: instantiated graphs per (direction, input, output)
    struct GraphEntry {
        int dir;
        const void *in;
        void *out;
        hipGraphExec_t exec;
        uint64_t used;
    };
    bool graph_mode = false;
    hipStream_t cap_stream = nullptr;
    mutable std::vector<GraphEntry> graphs;
    mutable uint64_t tick = 0;
    void drop_graphs() const;
    ~sht_plan();
};

void sht_plan::drop_graphs() const {
    for (GraphEntry &g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
}

static void dfree(void *p) {
    if (p) (void)hipFree(p);
}

sht_plan::~sht_plan() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (last_done) (void)hipEventDestroy(last_done);
    dfree(d_xh);
    dfree(d_wh);
    dfree(d_dmant);
    dfree(d_coef);
    dfree(d_coef2);
    dfree(d_dexp);
    for (void *q : {(void *)d_tab, (void *)d_ctab, (void *)d_bspec, (void *)d_tabf, (void *)d_ctabf,
                    (void *)d_bspecf, (void *)d_src_pos, (void *)d_src_pos2, (void *)d_inslot,
                    (void *)d_outslot, d_dft_scr})
        dfree(q);
    for (int i = 0; i < 2; ++i)
        for (void *q : {(void *)d_rl_ctab[i], (void *)d_rl_bspec[i], (void *)d_rl_bspecf[i], (void *)d_rl_inslot[i],
                        (void *)d_rl_outslot[i]})
            dfree(q);
    dfree(d_g);
    dfree(d_bz);
    dfree(d_X);
    dfree(d_Y);
    dfree(d_x_off);
    dfree(d_adj_items);
    dfree(d_adj_task_first);
    dfree(d_ck);
    dfree(d_ckexp);
    prog.release();
}

namespace {

int hip_fail(hipError_t e, const char *what) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    set_error_detail(buf);
    return e == hipErrorOutOfMemory ? SHT_ERR_OOM : SHT_ERR_HIP;
}

#define HIP_TRY(expr, what)                       \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

template <typename V>
int upload(const std::vector<V> &h, V **d, const char *what) {
    HIP_TRY(hipMalloc((void **)d, std::max<size_t>(1, h.size() * sizeof(V))), what);
    if (!h.empty()) HIP_TRY(hipMemcpy(*d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice), what);
    return SHT_OK;
}

int check_ptr(const void *p, size_t align) {
    if (!p) {
        set_error_detail("null buffer");
        return SHT_ERR_INVALID_ARG;
    }
    if (reinterpret_cast<uintptr_t>(p) % align) {
        set_error_detail("buffer not aligned to its complex element (16 bytes FP64, 8 bytes FP32)");
        return SHT_ERR_MISALIGNED;
    }
    return SHT_OK;
}

size_t elt_size(int dtype) { return dtype == SHT_F64 ? 8 : 4; }

}  // namespace

extern "C" {

void sht_plan_opts_default(sht_plan_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->eps = 1e-12;
    o->n0 = 256;
    o->leaf = 0;  // by size (see the builder)
    o->rk = 150;
    o->oversample = 2;
    o->rsvd_r = 30;
    o->rsvd_q = 2;
    o->sampling = SHT_SAMPLE_MOCK_CHEB;
    o->seed = 20200423ULL;
    o->threads = 0;
    o->f32_mode = SHT_F32_VALU;
    o->min_idbf = 0;
    o->dense_gen = 1;
    o->m_lo = 0;
    o->m_hi = -1;
    o->dft_schedule = SHT_DFT_AUTO;
    o->id_check = 1;
    o->cache_dir = nullptr;
    o->level_schedule = SHT_LEVELS_AUTO;
}

const char *sht_strerror(int code) {
    switch (code) {
        case SHT_OK: return "ok";
        case SHT_ERR_INVALID_ARG: return "invalid argument";
        case SHT_ERR_UNSUPPORTED: return "unsupported configuration";
        case SHT_ERR_OOM: return "out of memory";
        case SHT_ERR_HIP: return "HIP runtime error";
        case SHT_ERR_PLAN: return "plan construction failed";
        case SHT_ERR_MISALIGNED: return "misaligned buffer";
        case SHT_ERR_PLAN_CORRUPT: return "corrupt plan file";
        default: return "unknown error";
    }
}

const char *sht_last_error_detail(void) { return g_detail.c_str(); }

int sht_host_gauss_legendre(int n, double *x, double *w) {
    if (n < 1 || !x || !w) return SHT_ERR_INVALID_ARG;
    gauss_legendre(n, x, w);
    return SHT_OK;
}

static int copy_json(const std::string &s, char *json, size_t cap);

int sht_host_dft_tables(int N, int dtype, int schedule, char *json, size_t cap) {
    if (N < 1 || N > 8192 || (dtype != SHT_F64 && dtype != SHT_F32) || schedule < SHT_DFT_AUTO ||
        schedule > SHT_DFT_FOUR_STEP)
        return SHT_ERR_INVALID_ARG;
    dev::DftHost h;
    dev::dft_build(4 * N - 1, dtype, h, schedule);
    std::ostringstream os;
    os.precision(17);
    auto ints = [&](const char *name, const std::vector<int> &v) {
        os << ",\"" << name << "\":[";
        for (size_t i = 0; i < v.size(); ++i) os << (i ? "," : "") << v[i];
        os << "]";
    };
    auto dbls = [&](const char *name, const std::vector<double> &v) {
        os << ",\"" << name << "\":[";
        for (size_t i = 0; i < v.size(); ++i) os << (i ? "," : "") << v[i];
        os << "]";
    };
    static const char *kinds[] = {"none", "rows", "rader", "four_step"};
    os << "{\"kind\":\"" << kinds[h.kind + 1] << "\",\"M\":" << h.M << ",\"M1\":" << h.M1 << ",\"M2\":" << h.M2
       << ",\"chunk1\":" << h.chunk1 << ",\"chunk2\":" << h.chunk2;
    ints("radix", h.radix);
    ints("blen", h.blen);
    ints("src_pos", h.src_pos);
    ints("radix2", h.radix2);
    ints("blen2", h.blen2);
    ints("src_pos2", h.src_pos2);
    ints("inslot", h.inslot);
    ints("outslot", h.outslot);
    dbls("bspec", h.bspec);
    os << ",\"rader_last\":[";
    for (int i = 0; i < 2; ++i) {
        os << (i ? "," : "") << "{\"R\":" << h.rl_R[i];
        ints("radix", h.rl_radix[i]);
        ints("blen", h.rl_blen[i]);
        ints("src_pos", h.rl_src_pos[i]);
        ints("inslot", h.rl_inslot[i]);
        ints("outslot", h.rl_outslot[i]);
        dbls("bspec", h.rl_bspec[i]);
        os << "}";
    }
    os << "]}";
    return copy_json(os.str(), json, cap);
}

int sht_plan_create(int N, int batch, int dtype, int method, const sht_plan_opts *opts,
                    sht_plan_t **out) {
    if (!out) return SHT_ERR_INVALID_ARG;
    *out = nullptr;
    if (N < 1 || N > 8192 || batch < 1 || batch > 4096) {
        set_error_detail("N must be in [1, 8192] and batch in [1, 4096]");
        return SHT_ERR_INVALID_ARG;
    }
    if (dtype != SHT_F64 && dtype != SHT_F32) return SHT_ERR_UNSUPPORTED;
    if (method != SHT_DENSE && method != SHT_IDBF) return SHT_ERR_UNSUPPORTED;
    auto t0 = std::chrono::steady_clock::now();
    std::unique_ptr<sht_plan> p(new (std::nothrow) sht_plan);
    if (!p) return SHT_ERR_OOM;
    p->N = N;
    p->M = 4 * N - 1;
    p->batch = batch;
    p->dtype = dtype;
    p->method = method;
    sht_plan_opts_default(&p->opts);
    if (opts) p->opts = *opts;
    HIP_TRY(hipGetDevice(&p->device), "hipGetDevice");
    HIP_TRY((hipError_t)noalloc_scratch_init(p->device), "fixed scratch address");
    HIP_TRY(dev::dft_init(), "DFT kernel attributes");
    HIP_TRY(hipEventCreateWithFlags(&p->last_done, hipEventDisableTiming), "plan event");
    if (p->opts.f32_mode != SHT_F32_VALU && p->opts.f32_mode != SHT_F32_SPLIT_BF16 &&
        p->opts.f32_mode != SHT_F32_SPLIT_BF16_6)
        return SHT_ERR_INVALID_ARG;
    if (p->opts.f32_mode != SHT_F32_VALU && (dtype != SHT_F32 || method != SHT_IDBF)) {
        set_error_detail("split-BF16 products apply to FP32 plans of the fast form");
        return SHT_ERR_UNSUPPORTED;
    }
    if (p->opts.m_hi < 0) p->opts.m_hi = 2 * N - 1;
    if (p->opts.m_lo < 0 || p->opts.m_lo > p->opts.m_hi || p->opts.m_hi > 2 * N - 1) {
        set_error_detail("order range of the plan out of bounds");
        return SHT_ERR_INVALID_ARG;
    }
    if (method == SHT_DENSE && (p->opts.m_lo != 0 || p->opts.m_hi != 2 * N - 1)) {
        set_error_detail("order ranges apply to the fast form (the plain form stores no per-order data)");
        return SHT_ERR_UNSUPPORTED;
    }

    LegendreTables lt;
    try {
        build_legendre_tables(N, lt, p->opts.m_lo, p->opts.m_hi);
    } catch (const std::bad_alloc &) {
        return SHT_ERR_OOM;
    }
    p->x.resize(2 * N);
    p->w.resize(2 * N);
    gauss_legendre(2 * N, p->x.data(), p->w.data());

    int rc;
    if ((rc = upload(lt.xh, &p->d_xh, "upload nodes"))) return rc;
    if ((rc = upload(lt.wh, &p->d_wh, "upload weights"))) return rc;
    if ((rc = upload(lt.diag_m, &p->d_dmant, "upload diag"))) return rc;
    if ((rc = upload(lt.diag_e, &p->d_dexp, "upload diag exponents"))) return rc;
    if ((rc = upload(lt.coef, &p->d_coef, "upload recurrence coefficients"))) return rc;
    if ((rc = upload(lt.coef2, &p->d_coef2, "upload recurrence coefficients"))) return rc;
    p->dense.N = N;
    p->dense.M = p->M;
    p->dense.xh = p->d_xh;
    p->dense.wh = p->d_wh;
    p->dense.dmant = p->d_dmant;
    p->dense.dexp = p->d_dexp;
    p->dense.coef = p->d_coef;
    p->dense.coef2 = p->d_coef2;

    // phi DFT: schedule and tables for this length and type
    {
        dev::DftHost dh;
        if (p->opts.dft_schedule < SHT_DFT_AUTO || p->opts.dft_schedule > SHT_DFT_FOUR_STEP) {
            set_error_detail("unknown phi DFT schedule");
            return SHT_ERR_INVALID_ARG;
        }
        if (p->opts.level_schedule < SHT_LEVELS_AUTO || p->opts.level_schedule > SHT_LEVELS_FUSED) {
            set_error_detail("unknown level schedule");
            return SHT_ERR_INVALID_ARG;
        }
        dev::dft_build(p->M, dtype, dh, p->opts.dft_schedule);
        if (p->opts.dft_schedule != SHT_DFT_AUTO && dh.kind == dev::kDftNone) {
            set_error_detail("the requested phi DFT schedule does not apply to this length and type");
            return SHT_ERR_UNSUPPORTED;
        }
        dev::DftPlan &d = p->dft;
        d.N = N;
        d.M = p->M;
        d.kind = dh.kind;
        p->dft_ok = dh.kind != dev::kDftNone;
        if (dh.radix.size() > 24 || dh.radix2.size() > 24) return SHT_ERR_UNSUPPORTED;
        d.nrad = (int)dh.radix.size();
        for (int i = 0; i < d.nrad; ++i) {
            d.radix[i] = dh.radix[i];
            d.blen[i] = dh.blen[i];
        }
        d.nrad2 = (int)dh.radix2.size();
        for (int i = 0; i < d.nrad2; ++i) {
            d.radix2[i] = dh.radix2[i];
            d.blen2[i] = dh.blen2[i];
        }
        d.M1 = dh.M1;
        d.M2 = dh.M2;
        d.chunk1 = dh.chunk1;
        d.chunk2 = dh.chunk2;
        if ((rc = upload(dh.tab, &p->d_tab, "upload DFT table"))) return rc;
        if ((rc = upload(dh.tabf, &p->d_tabf, "upload DFT table"))) return rc;
        if ((rc = upload(dh.ctab, &p->d_ctab, "upload DFT table"))) return rc;
        if ((rc = upload(dh.ctabf, &p->d_ctabf, "upload DFT table"))) return rc;
        if ((rc = upload(dh.src_pos, &p->d_src_pos, "upload DFT positions"))) return rc;
        if ((rc = upload(dh.src_pos2, &p->d_src_pos2, "upload DFT positions"))) return rc;
        if ((rc = upload(dh.inslot, &p->d_inslot, "upload DFT slots"))) return rc;
        if ((rc = upload(dh.outslot, &p->d_outslot, "upload DFT slots"))) return rc;
        if ((rc = upload(dh.bspec, &p->d_bspec, "upload DFT spectrum"))) return rc;
        if ((rc = upload(dh.bspecf, &p->d_bspecf, "upload DFT spectrum"))) return rc;
        d.tab = p->d_tab;
        d.tabf = p->d_tabf;
        d.ctab = p->d_ctab;
        d.ctabf = p->d_ctabf;
        d.src_pos = p->d_src_pos;
        d.src_pos2 = p->d_src_pos2;
        d.inslot = p->d_inslot;
        d.outslot = p->d_outslot;
        d.bspec = p->d_bspec;
        d.bspecf = p->d_bspecf;
        for (int i = 0; i < 2; ++i) {
            if (!dh.rl_R[i]) continue;
            if (dh.rl_radix[i].size() > 24) return SHT_ERR_UNSUPPORTED;
            d.rl_R[i] = dh.rl_R[i];
            d.rl_nrad[i] = (int)dh.rl_radix[i].size();
            for (int q = 0; q < d.rl_nrad[i]; ++q) {
                d.rl_radix[i][q] = dh.rl_radix[i][q];
                d.rl_blen[i][q] = dh.rl_blen[i][q];
            }
            if ((rc = upload(dh.rl_ctab[i], &p->d_rl_ctab[i], "upload DFT table"))) return rc;
            if ((rc = upload(dh.rl_bspec[i], &p->d_rl_bspec[i], "upload DFT spectrum"))) return rc;
            if ((rc = upload(dh.rl_bspecf[i], &p->d_rl_bspecf[i], "upload DFT spectrum"))) return rc;
            if ((rc = upload(dh.rl_inslot[i], &p->d_rl_inslot[i], "upload DFT slots"))) return rc;
            if ((rc = upload(dh.rl_outslot[i], &p->d_rl_outslot[i], "upload DFT slots"))) return rc;
            d.rl_ctab[i] = p->d_rl_ctab[i];
            d.rl_bspec[i] = p->d_rl_bspec[i];
            d.rl_bspecf[i] = p->d_rl_bspecf[i];
            d.rl_inslot[i] = p->d_rl_inslot[i];
            d.rl_outslot[i] = p->d_rl_outslot[i];
        }
        if (dh.kind == dev::kDftFourStep) {
            HIP_TRY(hipMalloc(&p->d_dft_scr, 2 * elt_size(dtype) * (size_t)batch * 2 * N * p->M),
                    "DFT intermediate rows");
            d.scratch = p->d_dft_scr;
        }
    }

    // workspace
    const size_t gbytes = 2 * elt_size(dtype) * (size_t)batch * 2 * N * p->M;
    HIP_TRY(hipMalloc(&p->d_g, gbytes), "workspace g");
    HIP_TRY(hipMalloc(&p->d_bz, 2 * elt_size(dtype) * (size_t)batch * 4 * N * N), "workspace real-field coefficients");
    if (method == SHT_DENSE) {
        // FP64 panels: X [sum of half-matrix columns][R], Y [4N^2][R]
        std::vector<int64_t> xo(4 * (size_t)N + 1, 0);
        int64_t maxc = 0;
        for (int t = 0; t < 4 * N; ++t) {
            const int c = half_cols(N, t / 2, t % 2);
            xo[t + 1] = xo[t] + std::max(0, c);
            maxc = std::max<int64_t>(maxc, c);
        }
        const size_t R = 4 * (size_t)batch;
        HIP_TRY(hipMalloc(&p->d_X, sizeof(double) * std::max<int64_t>(1, xo[4 * N]) * R), "dense X panels");
        HIP_TRY(hipMalloc(&p->d_Y, sizeof(double) * (size_t)4 * N * N * R), "dense Y panels");
        if ((rc = upload(xo, &p->d_x_off, "upload panel offsets"))) return rc;
        p->panels.X = p->d_X;
        p->panels.Y = p->d_Y;
        p->panels.x_off = p->d_x_off;
        p->panels.max_cols = maxc;
        // transposed product: items (task, first column) of 64-column output
        // tiles; recurrence states of one chunk of tasks at a time (64-node
        // padded rows per item), by default at most 64M states (1.3 GB)
        std::vector<int32_t> items, tfirst(4 * (size_t)N + 1, 0);
        int64_t max_task_items = 0;
        for (int t = 0; t < 4 * N; ++t) {
            const int c = std::max(0, half_cols(N, t / 2, t % 2));
            for (int c0 = 0; c0 < c; c0 += 64) {
                items.push_back(t);
                items.push_back(c0);
            }
            tfirst[t + 1] = (int32_t)(items.size() / 2);
            max_task_items = std::max<int64_t>(max_task_items, tfirst[t + 1] - tfirst[t]);
        }
        const int64_t NP = 64 * (int64_t)((N + 63) / 64);
        int64_t cap = 64ll << 20;
        if (const char *ev = std::getenv("SHT_DENSE_CKPT_STATES")) cap = std::atoll(ev);
        cap = std::max(cap, max_task_items * NP);
        cap = std::min(cap, std::max<int64_t>(1, (int64_t)tfirst[4 * N]) * NP);
        cap = (cap / NP) * NP;
        if ((rc = upload(items, &p->d_adj_items, "upload transposed items"))) return rc;
        if ((rc = upload(tfirst, &p->d_adj_task_first, "upload transposed items"))) return rc;
        HIP_TRY(hipMalloc(&p->d_ck, sizeof(double) * 2 * (size_t)cap), "transposed checkpoints");
        HIP_TRY(hipMalloc(&p->d_ckexp, sizeof(int32_t) * (size_t)cap), "transposed checkpoints");
        p->panels.adj_items = p->d_adj_items;
        p->panels.adj_task_first = tfirst;
        p->panels.adj_task_first_d = p->d_adj_task_first;
        p->panels.ck = p->d_ck;
        p->panels.ckexp = p->d_ckexp;
        p->panels.ck_cap = cap;
    } else {
        idbf::HostProgram hp;
        int brc;
        try {
            brc = idbf::build_program(N, batch, lt, p->opts, hp);
        } catch (const std::bad_alloc &) {
            return SHT_ERR_OOM;
        }
        if (brc) return brc;
        brc = idbf::upload_program(hp, dtype, batch, p->d_wh, p->d_xh, p->d_coef2, p->prog);
        if (brc) return brc;
        p->stats = hp.stats_json;
    }
    p->opts.cache_dir = nullptr;  // the caller's string is not kept
    p->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    HIP_TRY(hipDeviceSynchronize(), "plan upload");
    *out = p.release();
    return SHT_OK;
}

void sht_plan_destroy(sht_plan_t *plan) { delete plan; }

int sht_plan_info(const sht_plan_t *p, int *N, int *batch, int *dtype, int *method) {
    if (!p) return SHT_ERR_INVALID_ARG;
    if (N) *N = p->N;
    if (batch) *batch = p->batch;
    if (dtype) *dtype = p->dtype;
    if (method) *method = p->method;
    return SHT_OK;
}

int sht_plan_nodes(const sht_plan_t *p, double *x, double *w) {
    if (!p || !x || !w) return SHT_ERR_INVALID_ARG;
    std::copy(p->x.begin(), p->x.end(), x);
    std::copy(p->w.begin(), p->w.end(), w);
    return SHT_OK;
}

int sht_plan_stats(const sht_plan_t *p, char *json, size_t cap) {
    if (!p) return SHT_ERR_INVALID_ARG;
    std::ostringstream os;
    static const char *kinds[] = {"none", "rows", "rader", "four_step"};
    const int kind = p->dft.kind + 1;  // kDftNone = -1
    os << "{\"N\":" << p->N << ",\"batch\":" << p->batch << ",\"dtype\":\""
       << (p->dtype == SHT_F64 ? "f64" : "f32") << "\",\"method\":\""
       << (p->method == SHT_DENSE ? "dense" : "idbf") << "\",\"build_seconds\":" << p->build_seconds
       << ",\"dft\":\"" << (kind >= 0 && kind <= 3 ? kinds[kind] : "?") << "\",\"dft_rader_last\":["
       << p->dft.rl_R[0] << "," << p->dft.rl_R[1] << "]";
    if (p->method == SHT_IDBF && !p->stats.empty()) os << ",\"program\":" << p->stats;
    os << "}";
    std::string s = os.str();
    if (json && cap) {
        size_t n = std::min(cap - 1, s.size());
        std::memcpy(json, s.data(), n);
        json[n] = 0;
    }
    return (int)s.size() + 1;
}

static int full_transform_ok(const sht_plan_t *p) {
    if (!p->dft_ok) {
        set_error_detail("no phi DFT schedule for this N and dtype (a prime 4N-1 whose row exceeds LDS, or a "
                         "length without a four-step split); use sht_alt_apply");
        return SHT_ERR_UNSUPPORTED;
    }
    if (p->opts.m_lo != 0 || p->opts.m_hi != 2 * p->N - 1) {
        set_error_detail("the plan covers a range of orders only; use sht_alt_apply");
        return SHT_ERR_UNSUPPORTED;
    }
    return SHT_OK;
}

static int copy_json(const std::string &s, char *json, size_t cap) {
    if (json && cap) {
        size_t n = std::min(cap - 1, s.size());
        std::memcpy(json, s.data(), n);
        json[n] = 0;
    }
    return (int)s.size() + 1;
}

int sht_profile(sht_plan_t *p, int enable) {
    if (!p) return SHT_ERR_INVALID_ARG;
    p->recorder.clear();
    p->profiling = enable != 0;
    return SHT_OK;
}

int sht_profile_report(const sht_plan_t *p, char *json, size_t cap) {
    if (!p) return SHT_ERR_INVALID_ARG;
    return copy_json(p->recorder.report(), json, cap);
}

static int run_alt(const sht_plan_t *p, int a_lo, int a_hi, int dir, const void *in, void *out,
                   hipStream_t s) {
    prof::Install inst(p->rec());
    hipError_t e;
    if (p->method == SHT_DENSE) {
        if (dir == SHT_FWD)
            e = dev::alt_dense_forward(p->dense, p->panels, p->dtype, p->batch, a_lo, a_hi, in, out, s);
        else
            e = dev::alt_dense_transpose(p->dense, p->panels, p->dtype, p->batch, a_lo, a_hi, dir == SHT_INV, in,
                                         out, s);
    } else {
        e = idbf::run(p->prog, p->dense, p->dtype, p->batch, a_lo, a_hi, dir, in, out, s);
    }
    if (e != hipSuccess) return hip_fail(e, "ALT launch");
    return SHT_OK;
}

}  // extern "C"

// Enqueue one call's work on stream s in the plan's order (see sht.h,
// Ownership): under the plan's lock, wait for the previous call's work if it
// ran on another stream, enqueue, record.  A stream that the caller is
// capturing into a graph is left alone (the caller orders its captures).
template <typename F>
static int ordered(const sht_plan_t *p, hipStream_t s, F &&enqueue) {
    std::lock_guard<std::mutex> lk(p->mu);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs), "stream capture status");
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (!capturing && p->has_last && p->last_stream != s)
        HIP_TRY(hipStreamWaitEvent(s, p->last_done, 0), "order after the previous call");
    const int rc = enqueue(s);
    if (!capturing) {
        HIP_TRY(hipEventRecord(p->last_done, s), "record call end");
        p->last_stream = s;
        p->has_last = true;
    }
    return rc;
}

// Graph mode: run `enqueue` from an instantiated graph keyed by (dir, in,
// out), capturing it on the plan's own stream the first time.  Called under
// the plan's lock (inside ordered()).
template <typename F>
static int via_graph(const sht_plan_t *p, int dir, const void *in, void *out, hipStream_t s, F &&enqueue) {
    sht_plan::GraphEntry *hit = nullptr;
    for (sht_plan::GraphEntry &g : p->graphs)
        if (g.dir == dir && g.in == in && g.out == out) hit = &g;
    if (!hit) {
        if (p->graphs.size() >= 16) {
            auto lru = std::min_element(p->graphs.begin(), p->graphs.end(),
                                        [](const sht_plan::GraphEntry &a, const sht_plan::GraphEntry &b) {
                                            return a.used < b.used;
                                        });
            (void)hipGraphExecDestroy(lru->exec);
            p->graphs.erase(lru);
        }
        prof::Install none(nullptr);  // no timing events inside a graph
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        const int rc = enqueue(p->cap_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return hip_fail(ei, "instantiate graph");
        p->graphs.push_back({dir, in, out, exec, 0});
        hit = &p->graphs.back();
    }
    hit->used = ++p->tick;
    HIP_TRY(hipGraphLaunch(hit->exec, s), "launch graph");
    return SHT_OK;
}

extern "C" {

int sht_set_graph_capture(sht_plan_t *p, int enable) {
    if (!p) return SHT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(p->mu);
    p->drop_graphs();
    p->graph_mode = enable != 0;
    if (p->graph_mode && !p->cap_stream)
        HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "capture stream");
    return SHT_OK;
}

int sht_plan_cache_verify(const char *path) {
    if (!path) return SHT_ERR_INVALID_ARG;
    return idbf::cache_verify(path);
}

int sht_plan_cache_path(int N, const sht_plan_opts *opts, char *path, size_t cap) {
    if (!opts || !opts->cache_dir || N < 1) return SHT_ERR_INVALID_ARG;
    return copy_json(idbf::cache_path(opts->cache_dir, idbf::cache_key(N, *opts)), path, cap);
}

int sht_alt_apply(const sht_plan_t *p, int m_lo, int m_hi, int dir, const void *in, void *out,
                  void *stream) {
    if (!p) return SHT_ERR_INVALID_ARG;
    if (m_lo < 0 || m_hi < m_lo || m_hi > 2 * p->N - 1 || (dir != SHT_FWD && dir != SHT_INV && dir != SHT_ADJ)) {
        set_error_detail("order range or direction out of bounds");
        return SHT_ERR_INVALID_ARG;
    }
    if (m_lo < p->opts.m_lo || m_hi > p->opts.m_hi) {
        set_error_detail("orders outside the range the plan was built for");
        return SHT_ERR_INVALID_ARG;
    }
    int rc;
    if ((rc = check_ptr(in, 2 * elt_size(p->dtype)))) return rc;
    if ((rc = check_ptr(out, 2 * elt_size(p->dtype)))) return rc;
    return ordered(p, (hipStream_t)stream,
                   [&](hipStream_t s) { return run_alt(p, m_lo, m_hi, dir, in, out, s); });
}

static int forward_work(const sht_plan_t *p, const void *beta, void *f, hipStream_t s) {
    int rc;
    if ((rc = run_alt(p, 0, 2 * p->N - 1, SHT_FWD, beta, f, s))) return rc;
    prof::Install inst(p->rec());
    hipError_t e = dev::dft_synthesis(p->dft, p->dtype, p->batch, f, s);
    if (e != hipSuccess) return hip_fail(e, "DFT synthesis");
    return SHT_OK;
}

static int transposed_work(const sht_plan_t *p, const void *f, void *beta, void *g, bool inverse, hipStream_t s) {
    prof::Install inst(p->rec());
    hipError_t e = dev::dft_analysis(p->dft, p->dtype, p->batch, inverse ? 1.0 / p->M : 1.0, f, g, s);
    if (e != hipSuccess) return hip_fail(e, "DFT analysis");
    return run_alt(p, 0, 2 * p->N - 1, inverse ? SHT_INV : SHT_ADJ, g, beta, s);
}

int sht_forward(const sht_plan_t *p, const void *beta, void *f, void *stream) {
    if (!p) return SHT_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_ptr(beta, 2 * elt_size(p->dtype)))) return rc;
    if ((rc = check_ptr(f, 2 * elt_size(p->dtype)))) return rc;
    if (beta == f) {
        set_error_detail("f may not alias beta");
        return SHT_ERR_INVALID_ARG;
    }
    if ((rc = full_transform_ok(p))) return rc;
    return ordered(p, (hipStream_t)stream, [&](hipStream_t s) {
        auto work = [&](hipStream_t w) { return forward_work(p, beta, f, w); };
        return p->graph_mode ? via_graph(p, SHT_FWD, beta, f, s, work) : work(s);
    });
}

static int transposed(const sht_plan_t *p, const void *f, void *beta, void *stream, bool inverse) {
    if (!p) return SHT_ERR_INVALID_ARG;
    int rc;
    if ((rc = full_transform_ok(p))) return rc;
    if ((rc = check_ptr(beta, 2 * elt_size(p->dtype)))) return rc;
    if ((rc = check_ptr(f, 2 * elt_size(p->dtype)))) return rc;
    return ordered(p, (hipStream_t)stream, [&](hipStream_t s) {
        auto work = [&](hipStream_t w) { return transposed_work(p, f, beta, p->d_g, inverse, w); };
        return p->graph_mode ? via_graph(p, inverse ? SHT_INV : SHT_ADJ, f, beta, s, work) : work(s);
    });
}

int sht_inverse(const sht_plan_t *p, const void *f, void *beta, void *stream) {
    return transposed(p, f, beta, stream, true);
}

int sht_backward(const sht_plan_t *p, const void *grad_f, void *grad_beta, void *stream) {
    return transposed(p, grad_f, grad_beta, stream, false);
}

static int real_args(const sht_plan_t *p, int nreal, const void *a, const void *b) {
    if (!p) return SHT_ERR_INVALID_ARG;
    int rc;
    if ((rc = full_transform_ok(p))) return rc;
    if (nreal < 1 || nreal > 2 * p->batch) {
        set_error_detail("nreal must be in [1, 2 batch]");
        return SHT_ERR_INVALID_ARG;
    }
    if ((rc = check_ptr(a, elt_size(p->dtype)))) return rc;
    return check_ptr(b, elt_size(p->dtype));
}

int sht_forward_real(const sht_plan_t *p, int nreal, const void *beta_half, void *f, void *stream) {
    int rc;
    if ((rc = real_args(p, nreal, beta_half, f))) return rc;
    return ordered(p, (hipStream_t)stream, [&](hipStream_t s) {
        prof::Install inst(p->rec());
        hipError_t e = dev::real_pack(p->dtype, p->N, p->batch, nreal, beta_half, p->d_bz, s);
        if (e != hipSuccess) return hip_fail(e, "real-field coefficients");
        int r = run_alt(p, 0, 2 * p->N - 1, SHT_FWD, p->d_bz, p->d_g, s);
        if (r) return r;
        prof::Install inst2(p->rec());
        e = dev::dft_synthesis_real(p->dft, p->dtype, p->batch, nreal, p->d_g, f, s);
        if (e != hipSuccess) return hip_fail(e, "DFT synthesis");
        return SHT_OK;
    });
}

int sht_inverse_real(const sht_plan_t *p, int nreal, const void *f, void *beta_half, void *stream) {
    int rc;
    if ((rc = real_args(p, nreal, f, beta_half))) return rc;
    return ordered(p, (hipStream_t)stream, [&](hipStream_t s) {
        prof::Install inst(p->rec());
        hipError_t e = dev::dft_analysis_real(p->dft, p->dtype, p->batch, nreal, 1.0 / p->M, f, p->d_g, s);
        if (e != hipSuccess) return hip_fail(e, "DFT analysis");
        int r = run_alt(p, 0, 2 * p->N - 1, SHT_INV, p->d_g, p->d_bz, s);
        if (r) return r;
        prof::Install inst2(p->rec());
        e = dev::real_unpack(p->dtype, p->N, p->batch, nreal, p->d_bz, beta_half, s);
        if (e != hipSuccess) return hip_fail(e, "real-field coefficients");
        return SHT_OK;
    });
}

int sht_inverse_noalloc(const sht_plan_t *p, const void *f, void *beta, void *stream) {
    if (!p) return SHT_ERR_INVALID_ARG;
    int rc;
    if ((rc = full_transform_ok(p))) return rc;
    if ((rc = check_ptr(beta, 2 * elt_size(p->dtype)))) return rc;
    if ((rc = check_ptr(f, 2 * elt_size(p->dtype)))) return rc;
    const size_t need = 2 * elt_size(p->dtype) * (size_t)p->batch * 2 * p->N * p->M;
    if (need > kNoallocScratchBytes) {
        set_error_detail("sht_inverse_noalloc: the grid of this plan needs " + std::to_string(need) +
                         " bytes of fixed scratch, more than its " + std::to_string(kNoallocScratchBytes) +
                         "; use sht_inverse");
        return SHT_ERR_UNSUPPORTED;
    }
    void *g = noalloc_scratch(p->device);
    if (!g) {
        set_error_detail("sht_inverse_noalloc: fixed scratch of this device was not looked up");
        return SHT_ERR_HIP;
    }
    return ordered(p, (hipStream_t)stream,
                   [&](hipStream_t s) { return transposed_work(p, f, beta, g, true, s); });
}

}  // extern "C"
