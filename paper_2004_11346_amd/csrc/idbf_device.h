// Device-resident fast-ALT plan.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "idbf_program.h"

namespace sht {
namespace idbf {

struct DeviceProgramDir {
    void *d_vals = nullptr;  // output-major value stream (FP64 or FP32)
    int64_t n_vals = 0;
    Op *d_ops = nullptr;
    SubOp *d_subs = nullptr;
    int32_t *d_idx = nullptr;
    // stage_task_first[s][t]: first op (global index) of task t in stage s;
    // entry ntask is the stage end
    std::vector<std::vector<int32_t>> stage_task_first;
    std::vector<Stage> stages;  // host copy (LDS sizing per stage)
    // fused levels: groups split into size classes (LDS buffers of up to
    // kFusedRowsSmall rows, up to kFusedMaxRows rows, staged rows in HBM);
    // class c's group ids are glist[cls_first[c] ..], task ranges by
    // cls_task_first[c][t]
    bool fused_ok = false;
    FusedGroup *d_fgroups = nullptr;
    FusedLevel *d_flevels = nullptr;
    Op *d_fops = nullptr;
    SubOp *d_fsubs = nullptr;
    int32_t *d_glist = nullptr;
    std::vector<int32_t> cls_first;                    // [3]
    std::vector<std::vector<int32_t>> cls_task_first;  // [3][ntask + 1], relative to cls_first
};

// groups with at most this many rows per LDS buffer run in 64 KB of LDS
constexpr int kFusedRowsSmall = 256;

struct DeviceProgram {
    bool valid = false;
    int N = 0, batch = 0, dtype = 0, RC = 16;
    int RCW = 0;  // > 0: matrix-core executor with RCW columns per pass
    bool fused = false;  // the matrix-core executor runs the fused level form
    bool bf16 = false;  // FP32 plan on the BF16 matrix cores (split-BF16)
    int bf16_terms = 3;  // 3 or 6 products per value pair
    void *d_X = nullptr, *d_Y = nullptr, *d_scrA = nullptr, *d_scrB = nullptr;
    int64_t *d_x_off = nullptr;    // [4N + 1]
    const double *d_wh = nullptr;  // half-grid weights (owned by the plan)
    const double *d_xh = nullptr;    // half-grid nodes (owned by the plan)
    const double *d_coef2 = nullptr;  // composed two-step recurrence coefficients (owned by the plan)
    std::vector<int64_t> x_off_h, y_off_h;
    int64_t max_task_cols = 0;
    int64_t index_bytes = 0;
    DeviceProgramDir fwd, adj;
    // regenerated forward blocks applied by their own kernel
    struct Gen {
        int n_items = 0;
        void *d_items = nullptr, *d_segs = nullptr;
        double *d_ck = nullptr;
        int32_t *d_ckexp = nullptr;
        std::vector<int32_t> task_first_h;
    } gen, gena;  // forward, transposed
    void release();
};

hipError_t set_kernel_attributes();
hipError_t run_device(const DeviceProgram &p, int dtype, int batch, int a_lo, int a_hi, int dir, const void *in,
                      void *out, hipStream_t s);

}  // namespace idbf
}  // namespace sht
