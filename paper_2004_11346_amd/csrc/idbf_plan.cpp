// Fast-ALT plan: build the factors on the host, pack them, upload once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <sstream>

#include "idbf.h"
#include "plan_cache.h"

namespace sht {
namespace idbf {

namespace {

template <typename V>
hipError_t up(const std::vector<V> &h, V **d) {
    hipError_t e = hipMalloc((void **)d, std::max<size_t>(1, h.size() * sizeof(V)));
    if (e != hipSuccess) return e;
    if (h.empty()) return hipSuccess;
    return hipMemcpy(*d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice);
}

hipError_t upload_dir(Program &p, int ntask, int dtype, DeviceProgramDir &d) {
    hipError_t e;
    d.n_vals = (int64_t)p.vals.size();
    if (dtype == SHT_F64) {
        if ((e = up(p.vals, (double **)&d.d_vals)) != hipSuccess) return e;
    } else {
        std::vector<float> vf(p.vals.begin(), p.vals.end());
        if ((e = up(vf, (float **)&d.d_vals)) != hipSuccess) return e;
    }
    p.vals.clear();
    p.vals.shrink_to_fit();
    if ((e = up(p.ops, &d.d_ops)) != hipSuccess) return e;
    if ((e = up(p.subs, &d.d_subs)) != hipSuccess) return e;
    if ((e = up(p.idx, &d.d_idx)) != hipSuccess) return e;
    d.stages = p.stages;
    d.stage_task_first.clear();
    for (const Stage &st : p.stages) {
        std::vector<int32_t> tf(ntask + 1);
        int q = st.op_begin;
        for (int t = 0; t <= ntask; ++t) {
            while (q < st.op_end && p.op_task[q] < t) ++q;
            tf[t] = q;
        }
        tf[ntask] = st.op_end;
        d.stage_task_first.push_back(std::move(tf));
    }
    d.fused_ok = p.fused_ok != 0;
    if (d.fused_ok) {
        if ((e = up(p.fgroups, &d.d_fgroups)) != hipSuccess || (e = up(p.flevels, &d.d_flevels)) != hipSuccess ||
            (e = up(p.fops, &d.d_fops)) != hipSuccess || (e = up(p.fsubs, &d.d_fsubs)) != hipSuccess)
            return e;
        std::vector<int32_t> glist;
        d.cls_first.assign(3, 0);
        d.cls_task_first.assign(3, std::vector<int32_t>(ntask + 1, 0));
        for (int c = 0; c < 3; ++c) {
            d.cls_first[c] = (int32_t)glist.size();
            std::vector<int32_t> &tf = d.cls_task_first[c];
            for (size_t gi = 0; gi < p.fgroups.size(); ++gi) {
                const int r = p.fgroups[gi].lds_rows;
                const int gc = r <= kFusedRowsSmall ? 0 : r <= kFusedMaxRows ? 1 : 2;
                if (gc != c) continue;
                tf[p.fgroups[gi].task + 1]++;
                glist.push_back((int32_t)gi);
            }
            for (int t = 0; t < ntask; ++t) tf[t + 1] += tf[t];
        }
        if ((e = up(glist, &d.d_glist)) != hipSuccess) return e;
    }
    return hipSuccess;
}

int fail(hipError_t e, const char *what) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    set_error_detail(buf);
    return e == hipErrorOutOfMemory ? SHT_ERR_OOM : SHT_ERR_HIP;
}

}  // namespace

void DeviceProgram::release() {
    for (void *p : {d_X, d_Y, d_scrA, d_scrB, (void *)d_x_off, fwd.d_vals, (void *)fwd.d_ops, (void *)fwd.d_subs,
                    (void *)fwd.d_idx, adj.d_vals, (void *)adj.d_ops, (void *)adj.d_subs, (void *)adj.d_idx})
        if (p) (void)hipFree(p);
    for (DeviceProgramDir *dd : {&fwd, &adj})
        for (void *p : {(void *)dd->d_fgroups, (void *)dd->d_flevels, (void *)dd->d_fops, (void *)dd->d_fsubs,
                        (void *)dd->d_glist})
            if (p) (void)hipFree(p);
    for (Gen *g : {&gen, &gena}) {
        for (void *q : {g->d_items, g->d_segs, (void *)g->d_ck, (void *)g->d_ckexp})
            if (q) (void)hipFree(q);
        *g = Gen();
    }
    d_X = d_Y = d_scrA = d_scrB = nullptr;
    d_x_off = nullptr;
    fwd = DeviceProgramDir();
    adj = DeviceProgramDir();
    valid = false;
}

int build_program(int N, int batch, const LegendreTables &lt, const sht_plan_opts &opts, HostProgram &out) {
    (void)batch;
    int cache = kCacheOff;
    std::string key, path;
    bool loaded = false;
    if (opts.cache_dir && opts.cache_dir[0]) {
        key = cache_key(N, opts);
        path = cache_path(opts.cache_dir, key);
        const int lrc = cache_load(path, key, out.packed, out.stats);
        loaded = lrc == SHT_OK;
        cache = loaded ? kCacheHit : lrc == SHT_ERR_PLAN_CORRUPT ? kCacheRebuilt : kCacheMiss;
    }
    if (!loaded) {
        HostPlanData hp;
        int rc = build_all(N, opts, hp, &lt);
        if (rc) return rc;
        pack_programs(hp, out.packed);
        out.stats = hp.stats;
        if (cache != kCacheOff && cache_store(path, key, out.packed, out.stats) != SHT_OK)
            cache = kCacheOff;  // not writable: the plan is still built
    }
    out.N = N;
    out.f32_mode = opts.f32_mode;
    out.level_schedule = opts.level_schedule;
    std::ostringstream os;
    std::string base = idbf::stats_json(out.stats, opts);
    base.pop_back();  // strip '}'
    base += std::string(",\"plan_cache\":\"") + cache_status_name(cache) + "\"";
    int64_t idx_bytes = 4 * (int64_t)(out.packed.fwd.idx.size() + out.packed.adj.idx.size()) +
                        (int64_t)(out.packed.fwd.ops.size() + out.packed.adj.ops.size()) * sizeof(Op) +
                        (int64_t)(out.packed.fwd.subs.size() + out.packed.adj.subs.size()) * sizeof(SubOp);
    os << base << ",\"fwd_values\":" << out.packed.fwd.vals.size() << ",\"adj_values\":" << out.packed.adj.vals.size()
       << ",\"index_bytes\":" << idx_bytes << ",\"ckpt_states\":"
       << (out.packed.gen_fwd.ckexp.size() + out.packed.gen_adj.ckexp.size()) << ",\"ckpt_bytes\":"
       << 20 * (int64_t)(out.packed.gen_fwd.ckexp.size() + out.packed.gen_adj.ckexp.size())
       << ",\"fwd_stages\":" << out.packed.fwd.stages.size() << ",\"fwd_work_stages\":"
       << out.packed.fwd.n_work_stages << ",\"adj_stages\":" << out.packed.adj.stages.size()
       << ",\"fwd_ops\":" << out.packed.fwd.ops.size() << ",\"scratch_rows\":"
       << std::max(out.packed.fwd.scr_rows, out.packed.adj.scr_rows) << fused_stats_json(out.packed);
    // per direction: index stream and recurrence states read by one call
    const PackedPlan &pk = out.packed;
    const int64_t fwd_idx = 4 * (int64_t)pk.fwd.idx.size() + (int64_t)pk.fwd.ops.size() * sizeof(Op) +
                            (int64_t)pk.fwd.subs.size() * sizeof(SubOp) +
                            (int64_t)pk.gen_fwd.items.size() * sizeof(GenForward::Item) +
                            (int64_t)pk.gen_fwd.segs.size() * sizeof(GenForward::Seg);
    const int64_t fwd_states = (int64_t)pk.gen_fwd.ckexp.size();
    const int64_t adj_states = (int64_t)pk.gen_adj.ckexp.size();
    // rows moved by the op kernels per right-hand side: gathered inputs (matrix
    // and identity parts) and written outputs, per direction
    auto rows_moved = [](const Program &pr, int64_t &in_rows, int64_t &out_rows) {
        in_rows = 0;
        out_rows = 0;
        for (const Op &op : pr.ops) {
            out_rows += op.n_out;
            for (int k = 0; k < op.nsub; ++k) {
                const SubOp &so = pr.subs[op.sub0 + k];
                in_rows += (so.n_map > 0 ? so.n_in : 0) + so.n_dir;
            }
        }
    };
    int64_t fin = 0, fout = 0, ain = 0, aout = 0;
    rows_moved(pk.fwd, fin, fout);
    rows_moved(pk.adj, ain, aout);
    // distinct input-panel rows the program reads and output-panel rows its
    // final stage writes: the vector rows one call must move at least once
    auto vector_rows = [](const Program &pr, int64_t &in_rows, int64_t &out_rows) {
        std::vector<unsigned char> seen((size_t)std::max<int64_t>(1, pr.in_rows), 0);
        in_rows = 0;
        out_rows = 0;
        for (const Op &op : pr.ops) {
            if (op.dst == kOut) out_rows += op.n_out;
            for (int k = 0; k < op.nsub; ++k) {
                const SubOp &so = pr.subs[op.sub0 + k];
                if (so.src != kIn) continue;
                auto mark = [&](int64_t r) {
                    if (r >= 0 && r < pr.in_rows && !seen[(size_t)r]) {
                        seen[(size_t)r] = 1;
                        ++in_rows;
                    }
                };
                if (so.n_map > 0)
                    for (int j = 0; j < so.n_in; ++j) mark(pr.idx[(size_t)so.in_off + j]);
                for (int j = 0; j < so.n_dir; ++j) mark(pr.idx[(size_t)so.dir_off + 2 * j]);
            }
        }
    };
    int64_t fvi = 0, fvo = 0, avi = 0, avo = 0;
    vector_rows(pk.fwd, fvi, fvo);
    vector_rows(pk.adj, avi, avo);
    const int64_t adj_idx = 4 * (int64_t)pk.adj.idx.size() + (int64_t)pk.adj.ops.size() * sizeof(Op) +
                            (int64_t)pk.adj.subs.size() * sizeof(SubOp) +
                            (int64_t)pk.gen_adj.items.size() * sizeof(GenAdjoint::Item) +
                            (int64_t)pk.gen_adj.segs.size() * sizeof(GenAdjoint::Seg);
    os << ",\"fwd_gather_rows\":" << fin << ",\"fwd_out_rows\":" << fout << ",\"adj_gather_rows\":" << ain
       << ",\"adj_out_rows\":" << aout << ",\"fwd_vector_in_rows\":" << fvi << ",\"fwd_vector_out_rows\":" << fvo
       << ",\"adj_vector_in_rows\":" << avi << ",\"adj_vector_out_rows\":" << avo
       << ",\"adj_index_bytes\":" << adj_idx;
    os << ",\"fwd_index_bytes\":" << fwd_idx << ",\"fwd_state_bytes\":" << 20 * fwd_states
       << ",\"adj_state_bytes\":" << 20 * adj_states << ",\"gen_fwd_items\":" << pk.gen_fwd.items.size()
       << ",\"gen_adj_items\":" << pk.gen_adj.items.size() << "}";
    out.stats_json = os.str();
    return SHT_OK;
}

int upload_program(HostProgram &hp, int dtype, int batch, const double *d_wh, const double *d_xh,
                   const double *d_coef2, DeviceProgram &d) {
    hipError_t e;
    PackedPlan &pk = hp.packed;
    const int N = hp.N, ntask = 4 * N;
    d.N = N;
    d.batch = batch;
    d.dtype = dtype;
    const int R = 4 * batch;
    d.RC = R <= 4 ? 4 : R <= 8 ? 8 : 16;
    // Many right-hand sides: FP64 matrix-core executor (FP32 plans keep FP32
    // storage), all columns (at most 256, a multiple of 16) per pass
    // (SHT_IDBF_RCW overrides the pass width: a multiple of 16 up to 256; 0
    // disables)
    d.RCW = 0;
    if (R >= 16) d.RCW = std::min(256, (R + 15) & ~15);
    if (const char *e = std::getenv("SHT_IDBF_RCW")) {
        int v = std::atoi(e);
        d.RCW = (v >= 16 && v <= 256 && v % 16 == 0) ? v : 0;
    }
    if (dtype == SHT_F32 && (hp.f32_mode == SHT_F32_SPLIT_BF16 || hp.f32_mode == SHT_F32_SPLIT_BF16_6)) {
        d.bf16 = true;
        d.bf16_terms = hp.f32_mode == SHT_F32_SPLIT_BF16 ? 3 : 6;
        d.RCW = R <= 16 ? 16 : R <= 32 ? 32 : 64;
    }
    d.d_wh = d_wh;
    d.d_xh = d_xh;
    d.d_coef2 = d_coef2;
    if ((e = upload_dir(hp.packed.fwd, ntask, dtype, d.fwd)) != hipSuccess) return fail(e, "upload program");
    if ((e = upload_dir(hp.packed.adj, ntask, dtype, d.adj)) != hipSuccess) return fail(e, "upload program");
    // fused levels on request, on the matrix-core executor (every block's
    // levels in one workgroup); the staged schedule otherwise
    d.fused = d.RCW > 0 && !d.bf16 && hp.level_schedule == SHT_LEVELS_FUSED && d.fwd.fused_ok && d.adj.fused_ok;
    if (hp.level_schedule == SHT_LEVELS_FUSED && !d.fused) {
        set_error_detail("fused levels need the FP64 matrix-core executor (16 or more right-hand sides, "
                         "not split-BF16)");
        return SHT_ERR_UNSUPPORTED;
    }
    {
        GenForward &gf = pk.gen_fwd;
        d.gen.n_items = (int)gf.items.size();
        d.gen.task_first_h = gf.task_first;
        if ((e = up(gf.items, (GenForward::Item **)&d.gen.d_items)) != hipSuccess ||
            (e = up(gf.segs, (GenForward::Seg **)&d.gen.d_segs)) != hipSuccess ||
            (e = up(gf.ck, &d.gen.d_ck)) != hipSuccess || (e = up(gf.ckexp, &d.gen.d_ckexp)) != hipSuccess)
            return fail(e, "upload regenerated blocks");
        gf = GenForward();
        GenAdjoint &ga = pk.gen_adj;
        d.gena.n_items = (int)ga.items.size();
        d.gena.task_first_h = ga.task_first;
        if ((e = up(ga.items, (GenAdjoint::Item **)&d.gena.d_items)) != hipSuccess ||
            (e = up(ga.segs, (GenAdjoint::Seg **)&d.gena.d_segs)) != hipSuccess ||
            (e = up(ga.ck, &d.gena.d_ck)) != hipSuccess || (e = up(ga.ckexp, &d.gena.d_ckexp)) != hipSuccess)
            return fail(e, "upload regenerated blocks");
        ga = GenAdjoint();
    }
    d.x_off_h = pk.x_off;
    d.y_off_h = pk.y_off;
    if ((e = up(pk.x_off, &d.d_x_off)) != hipSuccess) return fail(e, "upload offsets");
    d.max_task_cols = 0;
    for (int t = 0; t < ntask; ++t) d.max_task_cols = std::max(d.max_task_cols, pk.x_off[t + 1] - pk.x_off[t]);
    const size_t es = dtype == SHT_F64 ? 8 : 4;
    if ((e = hipMalloc(&d.d_X, es * std::max<int64_t>(1, pk.x_off[ntask]) * R)) != hipSuccess)
        return fail(e, "X panels");
    if ((e = hipMalloc(&d.d_Y, es * std::max<int64_t>(1, pk.y_off[ntask]) * R)) != hipSuccess)
        return fail(e, "Y panels");
    // the fused form's rows of its own follow the staged rows in buffer A
    const int64_t sr = std::max<int64_t>(1, std::max(pk.fwd.scr_rows, pk.adj.scr_rows));
    const int64_t sra = std::max<int64_t>(sr, std::max(pk.fwd.scr_rows + pk.fwd.f_extra_rows,
                                                       pk.adj.scr_rows + pk.adj.f_extra_rows));
    const int64_t sw = std::max(d.RC, d.RCW);
    if ((e = hipMalloc(&d.d_scrA, es * sra * sw)) != hipSuccess) return fail(e, "scratch");
    if ((e = hipMalloc(&d.d_scrB, es * sr * sw)) != hipSuccess) return fail(e, "scratch");
    if ((e = set_kernel_attributes()) != hipSuccess) return fail(e, "kernel attributes");
    d.valid = true;
    return SHT_OK;
}

hipError_t run(const DeviceProgram &prog, const dev::DenseTables &t, int dtype, int batch, int a_lo, int a_hi,
               int dir, const void *in, void *out, hipStream_t s) {
    (void)t;
    if (!prog.valid) return hipErrorInvalidValue;
    return run_device(prog, dtype, batch, a_lo, a_hi, dir, in, out, s);
}

}  // namespace idbf
}  // namespace sht
