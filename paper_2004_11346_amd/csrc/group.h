// Grouped transforms: many independent transforms of different degrees and
// field counts applied by persistent kernels that pull (transform, order,
// node tile) or (transform, field, row) work items from a queue ordered
// longest first.  Plain (dense) ALT with the VALU kernels and the phi DFT.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sht {
namespace group {

constexpr int kMaxPass = 24;
// dynamic LDS of the grouped DFT kernel (160 KB less room for its static LDS)
constexpr int kGroupDftLds = 159 * 1024;

// one transform, as the kernels see it
struct GTrans {
    int N, M, fields, pad;
    const double *xh, *wh, *dmant, *coef;
    const int *dexp;
    const double *tab;  // phi DFT phase table (two-level, base M)
    const float *tabf;
    const int *src_pos;
    int npass;
    int R[kMaxPass], L[kMaxPass];
    void *beta;  // [fields][4N^2] complex
    void *f;     // [fields][2N][M] complex
    void *g;     // workspace [fields][2N][M] complex (inverse)
};

// work item: transform t, order a (or field), node tile (or row)
struct GItem {
    int t, a, b, pad;
};

enum Phase { kFwdAlt = 0, kAdjAlt = 1, kDftSyn = 2, kDftAna = 3 };

// batched mode: a copy between a transform's buffer (ext) and its place in
// a per-degree staging buffer, in 8-byte words
struct CopySeg {
    void *ext;
    void *stage;
    int64_t units;
};
hipError_t launch_copy_segs(const CopySeg *segs, int nseg, int64_t max_units, int to_stage, hipStream_t s);

hipError_t launch_reset(int *counters, int n, hipStream_t s);
// grid: number of persistent workgroups
hipError_t launch_phase(int phase, int dtype, int grid, const GTrans *tr, const GItem *items, int nitems,
                        int *counter, int max_M, hipStream_t s);
int fwd_rows_per_tile();
hipError_t init_attributes();  // once per process, before the first launch

}  // namespace group
}  // namespace sht
