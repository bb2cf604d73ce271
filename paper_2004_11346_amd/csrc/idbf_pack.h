// Packed fast-ALT plan: value stream + forward and transposed op programs.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "idbf_build.h"
#include "idbf_program.h"

namespace sht {
namespace idbf {

// Regenerated dense blocks of the forward product, applied after the op
// program by their own kernel: one item per (task, 64-row output tile) with
// the blocks crossing that tile as segments.  A segment holds, for each of the
// tile's 64 rows, the same-parity recurrence pair (degrees k - 2, k) at the
// block's first column (zeros for rows outside the block).
// Items whose output tile gets no contribution from the op program carry
// kOverwrite in `task`: their kernel writes the tile instead of adding to it,
// and the op program has no final op for that tile.
struct GenForward {
    static constexpr int32_t kOverwrite = 1 << 30;
    struct Item {
        int32_t task, row0, seg_begin, seg_end;
    };
    struct Seg {
        int32_t c0, ncol, ck, pad;  // first task column, columns, first state
    };
    std::vector<Item> items;        // sorted by task
    std::vector<int32_t> task_first;  // [ntask + 1]
    std::vector<Seg> segs;
    std::vector<double> ck;         // (p_{k-2}, p_k) per state
    std::vector<int32_t> ckexp;
    int64_t entries = 0;            // block entries covered
};

// Regenerated blocks of the transposed product: one item per (task, 64-column
// output tile); a segment is a block's rows [row0, row0 + 64) (a 64-row chunk)
// and columns [c0, c0 + ncol) inside the tile, with the recurrence pair of
// each of the 64 rows at column c0 (zeros for rows outside the block).
struct GenAdjoint {
    static constexpr int32_t kOverwrite = 1 << 30;  // as GenForward::kOverwrite
    struct Item {
        int32_t task, col0, seg_begin, seg_end;
    };
    struct Seg {
        int32_t row0, c0, ncol, ck;
    };
    std::vector<Item> items;          // sorted by task
    std::vector<int32_t> task_first;  // [ntask + 1]
    std::vector<Seg> segs;
    std::vector<double> ck;
    std::vector<int32_t> ckexp;
};

struct PackedPlan {
    Program fwd, adj;  // each with its own output-major value stream
    std::vector<int64_t> x_off, y_off;  // panel row offsets per task (+ total)
    // regenerated blocks, applied by their own kernels after the op programs
    // (the programs leave them out)
    GenForward gen_fwd;
    GenAdjoint gen_adj;
};

void pack_programs(const HostPlanData &hp, PackedPlan &pk);

// ",\"fused_ok\":..." statistics of the fused level form of both programs
std::string fused_stats_json(const PackedPlan &pk);

// Host application of the regenerated transposed blocks of tasks t_lo..t_hi
// (verification): out (X panels) += blocks^T x in (Y panels).
void host_run_gen_adjoint(const GenAdjoint &ga, int N, int t_lo, int t_hi, int R, const std::vector<int64_t> &x_off,
                          const std::vector<int64_t> &y_off, const double *in, double *out, const double *xh,
                          const double *coef2);

// Host application of the regenerated forward blocks of tasks t_lo..t_hi
// (verification): out (Y panels) += blocks x in (X panels).
void host_run_gen_forward(const GenForward &gf, int N, int t_lo, int t_hi, int R, const std::vector<int64_t> &x_off,
                          const std::vector<int64_t> &y_off, const double *in, double *out, const double *xh,
                          const double *coef2);

}  // namespace idbf
}  // namespace sht
