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
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "idbf.h"
#include "kernels.h"
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
    double *d_tw2 = nullptr;
    float *d_tw2f = nullptr;
    int *d_src_pos = nullptr;
    dev::DenseTables dense;
    dev::DftPlan dft;
    // workspace
    void *d_g = nullptr;         // [batch][2N][M] complex (dtype)
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
    ~sht_plan();
};

static void dfree(void *p) {
    if (p) (void)hipFree(p);
}

sht_plan::~sht_plan() {
    dfree(d_xh);
    dfree(d_wh);
    dfree(d_dmant);
    dfree(d_coef);
    dfree(d_coef2);
    dfree(d_dexp);
    dfree(d_tw2);
    dfree(d_tw2f);
    dfree(d_src_pos);
    dfree(d_g);
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
        set_error_detail("buffer not aligned to its element size");
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
        default: return "unknown error";
    }
}

const char *sht_last_error_detail(void) { return g_detail.c_str(); }

int sht_host_gauss_legendre(int n, double *x, double *w) {
    if (n < 1 || !x || !w) return SHT_ERR_INVALID_ARG;
    gauss_legendre(n, x, w);
    return SHT_OK;
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
    // the phi DFT holds a row in LDS; without it the plan serves sht_alt_apply only
    p->dft_ok = dev::dft_supported(p->M, dtype);

    LegendreTables lt;
    try {
        build_legendre_tables(N, lt);
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

    // phi DFT: radices and the e^{i pi r / M} table (long double, rounded)
    {
        std::vector<int> f, bl, sp;
        dev::dft_passes(p->M, f, bl, sp);
        p->dft.N = N;
        p->dft.M = p->M;
        p->dft.nrad = (int)f.size();
        for (size_t i = 0; i < f.size(); ++i) {
            p->dft.radix[i] = f[i];
            p->dft.blen[i] = bl[i];
        }
        if ((rc = upload(sp, &p->d_src_pos, "upload DFT positions"))) return rc;
        p->dft.src_pos = p->d_src_pos;
        std::vector<double> tw(4 * (size_t)p->M);
        std::vector<float> twf(4 * (size_t)p->M);
        const long double pi = 3.141592653589793238462643383279502884L;
        for (int r = 0; r < 2 * p->M; ++r) {
            long double ph = pi * r / p->M;
            tw[2 * r] = (double)cosl(ph);
            tw[2 * r + 1] = (double)sinl(ph);
            twf[2 * r] = (float)cosl(ph);
            twf[2 * r + 1] = (float)sinl(ph);
        }
        if ((rc = upload(tw, &p->d_tw2, "upload twiddles"))) return rc;
        if ((rc = upload(twf, &p->d_tw2f, "upload twiddles"))) return rc;
        p->dft.tw2 = p->d_tw2;
        p->dft.tw2f = p->d_tw2f;
    }

    // workspace
    const size_t gbytes = 2 * elt_size(dtype) * (size_t)batch * 2 * N * p->M;
    HIP_TRY(hipMalloc(&p->d_g, gbytes), "workspace g");
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
    os << "{\"N\":" << p->N << ",\"batch\":" << p->batch << ",\"dtype\":\""
       << (p->dtype == SHT_F64 ? "f64" : "f32") << "\",\"method\":\""
       << (p->method == SHT_DENSE ? "dense" : "idbf") << "\",\"build_seconds\":" << p->build_seconds;
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
        set_error_detail("the phi DFT row does not fit in LDS for this N and dtype; use sht_alt_apply");
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
    if ((rc = check_ptr(in, elt_size(p->dtype)))) return rc;
    if ((rc = check_ptr(out, elt_size(p->dtype)))) return rc;
    return run_alt(p, m_lo, m_hi, dir, in, out, (hipStream_t)stream);
}

int sht_forward(const sht_plan_t *p, const void *beta, void *f, void *stream) {
    if (!p) return SHT_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_ptr(beta, elt_size(p->dtype)))) return rc;
    if ((rc = check_ptr(f, elt_size(p->dtype)))) return rc;
    if (beta == f) {
        set_error_detail("f may not alias beta");
        return SHT_ERR_INVALID_ARG;
    }
    if ((rc = full_transform_ok(p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = run_alt(p, 0, 2 * p->N - 1, SHT_FWD, beta, f, s))) return rc;
    prof::Install inst(p->rec());
    hipError_t e = dev::dft_synthesis(p->dft, p->dtype, p->batch, f, s);
    if (e != hipSuccess) return hip_fail(e, "DFT synthesis");
    return SHT_OK;
}

static int transposed(const sht_plan_t *p, const void *f, void *beta, void *stream, bool inverse) {
    if (!p) return SHT_ERR_INVALID_ARG;
    int rc;
    if ((rc = full_transform_ok(p))) return rc;
    if ((rc = check_ptr(beta, elt_size(p->dtype)))) return rc;
    if ((rc = check_ptr(f, elt_size(p->dtype)))) return rc;
    hipStream_t s = (hipStream_t)stream;
    prof::Install inst(p->rec());
    hipError_t e = dev::dft_analysis(p->dft, p->dtype, p->batch, inverse ? 1.0 / p->M : 1.0, f, p->d_g, s);
    if (e != hipSuccess) return hip_fail(e, "DFT analysis");
    return run_alt(p, 0, 2 * p->N - 1, inverse ? SHT_INV : SHT_ADJ, p->d_g, beta, s);
}

int sht_inverse(const sht_plan_t *p, const void *f, void *beta, void *stream) {
    return transposed(p, f, beta, stream, true);
}

int sht_backward(const sht_plan_t *p, const void *grad_f, void *grad_beta, void *stream) {
    return transposed(p, grad_f, grad_beta, stream, false);
}

int sht_inverse_noalloc(const sht_plan_t *p, const void *f, void *beta, void *stream) {
    if (!p) return SHT_ERR_INVALID_ARG;
    int rc;
    if ((rc = full_transform_ok(p))) return rc;
    if ((rc = check_ptr(beta, elt_size(p->dtype)))) return rc;
    if ((rc = check_ptr(f, elt_size(p->dtype)))) return rc;
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
    hipStream_t s = (hipStream_t)stream;
    prof::Install inst(p->rec());
    hipError_t e = dev::dft_analysis(p->dft, p->dtype, p->batch, 1.0 / p->M, f, g, s);
    if (e != hipSuccess) return hip_fail(e, "DFT analysis");
    return run_alt(p, 0, 2 * p->N - 1, SHT_INV, g, beta, s);
}

}  // extern "C"
