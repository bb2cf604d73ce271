// Packed op program of the fast ALT, shared by the HIP executor and the host
// executor used for verification.
//
// A program is a sequence of stages; every stage is a list of ops that are
// independent of each other and depend only on earlier stages.  An op writes
// n_out rows (each row = the RC right-hand sides of one vector entry) as the
// sum of its sub-ops:
//   acc[out_map[i]] += sum_j M(i, j) * src[in_rows[j]]       (matrix part)
//   acc[dir_pos[d]] += src[dir_rows[d]]                       (identity part)
// M is a stored row-major block (mrows x mcols, leading dimension ld), used as
// is (trans = 0: i < mrows, j < mcols) or transposed (trans = 1: i < mcols,
// j < mrows).
// Column and row interpolative decompositions, their transposes, the middle
// butterfly couplings, trimmed dense blocks and low-rank factors are all of
// this form.  Non-final ops write their rows to a scratch buffer; final ops
// add their rows into the output panel (a task's half-grid rows in the forward
// direction, its coefficient rows in the transposed one).  Final ops are
// split into "slots" so that two ops of one launch never touch the same row.
#pragma once

#include <cstdint>
#include <vector>

namespace sht {
namespace idbf {

// source / destination buffers
enum Buf : int32_t { kIn = 0, kScrA = 1, kScrB = 2, kOut = 3 };

struct SubOp {
    int64_t mat_off;   // value offset of the stored matrix
    int32_t mrows, mcols, trans;
    int32_t src;       // Buf
    int32_t n_in;      // gathered rows (= mcols if !trans else mrows)
    int32_t in_off;    // idx offset: n_in source rows
    int32_t n_map;     // matrix output rows (= mrows if !trans else mcols)
    int32_t map_off;   // idx offset: n_map output positions (< n_out)
    int32_t n_dir;     // identity part
    int32_t dir_off;   // idx offset: n_dir (src row, out pos) pairs
    int32_t ld;        // leading dimension of the stored block (>= mcols)
};

struct Op {
    int32_t n_out;
    int32_t nsub;
    int32_t sub0;     // first SubOp
    int32_t dst;      // Buf: kScrA / kScrB (write) or kOut (add)
    int64_t dst_row;  // first destination row
};

struct Stage {
    int32_t op_begin, op_end;  // range in Program::ops
};

struct Program {
    std::vector<Op> ops;
    std::vector<int32_t> op_task;  // task of every op (ops of a stage are sorted by task)
    std::vector<SubOp> subs;
    std::vector<int32_t> idx;
    std::vector<Stage> stages;  // non-final stages, then one stage per final slot
    int n_work_stages = 0;      // stages[0 .. n_work_stages) are non-final
    int64_t scr_rows = 0;       // rows of each scratch buffer
    int64_t in_rows = 0, out_rows = 0;
    int max_n_out = 0, max_n_in = 0, max_mat = 0;
};

// Host execution of a program (verification): in [in_rows][R], out
// [out_rows][R] (overwritten), vals = the value stream.
void host_run_program(const Program &p, const double *vals, int R, const double *in, double *out);

}  // namespace idbf
}  // namespace sht
