// Packed op program of the fast ALT, shared by the HIP executor and the host
// executor used for verification.
//
// A program is a sequence of stages; every stage is a list of ops that are
// independent of each other and depend only on earlier stages.  An op produces
// n_out rows (each row = the RC right-hand sides of one vector entry) as the
// sum of its sub-ops:
//   acc[map[q]]   += sum_j V[j * n_map + q] * src[in_rows[j]]     (matrix part)
//   acc[dir_pos]  += src[dir_row]                                 (identity part)
// The matrix of every sub-op is stored output-major in the program's own value
// stream (element (output q, input j) at j * n_map + q), so that consecutive
// lanes read consecutive words.  Column and row interpolative decompositions,
// their transposes, the middle butterfly couplings, trimmed dense blocks and
// low-rank factors all take this form.
//
// Non-final ops write their rows to a scratch buffer (two buffers alternate
// between stages).  Final ops are output tiles: every row of every task's
// output panel belongs to exactly one final op, which gathers all block
// contributions to its rows and writes the tile once.
#pragma once

#include <cstdint>
#include <vector>

namespace sht {
namespace idbf {

// source / destination buffers (kLds: the fused form's workgroup-local rows)
enum Buf : int32_t { kIn = 0, kScrA = 1, kScrB = 2, kOut = 3, kLds = 4 };

struct SubOp {
    int64_t mat_off;  // value offset of the output-major matrix (n_in x n_map)
    int32_t src;      // Buf
    int32_t n_in;     // gathered rows
    int32_t in_off;   // idx offset: n_in source rows
    int32_t n_map;    // matrix outputs
    int32_t map_off;  // idx offset: n_map output positions (< n_out)
    int32_t n_dir;    // identity part
    int32_t dir_off;  // idx offset: n_dir (src row, out pos) pairs
    int32_t pad;
};

struct Op {
    int32_t n_out;
    int32_t nsub;
    int32_t sub0;     // first SubOp
    int32_t dst;      // Buf: kScrA / kScrB / kOut
    int64_t dst_row;  // first destination row
};

struct Stage {
    int32_t op_begin, op_end;  // range in Program::ops
    int32_t max_out, max_in;   // largest n_out / n_in of the stage (LDS sizing)
};

// Fused form of the work stages: all non-final levels of one block (a
// butterfly's column pass, middle couplings and row pass, or a low-rank
// block's V^T) run in one workgroup, level after level, with the intermediate
// rows in two LDS buffers that alternate between levels (level l writes
// buffer l & 1).  Ops and sub-ops are those of the staged program with rows
// renumbered into the buffers (src / dst kLds); the matrices are the staged
// program's (same value offsets).  The block's last level is then written to
// the scratch rows the final stage reads.  A block whose levels exceed
// kFusedMaxRows rows keeps its intermediate rows in HBM (rows of its own past
// the staged scratch rows) and runs its levels in its workgroup.
struct FusedLevel {
    int32_t op_begin, op_end;  // range in Program::fops
    int32_t rows;              // rows the level writes (from row 0 of its buffer)
    int32_t pad;
};

struct FusedGroup {
    int32_t lvl_begin, nlev;  // range in Program::flevels
    int32_t lds_rows;         // rows of each LDS buffer (> kFusedMaxRows: rows in HBM)
    int32_t out_buf;          // kScrA / kScrB: destination of the last level
    int64_t out_row;          // its first scratch row
    int32_t task;
    int32_t pad;
};

struct Program {
    std::vector<Op> ops;
    std::vector<int32_t> op_task;  // task of every op (ops of a stage are sorted by task)
    std::vector<SubOp> subs;
    std::vector<int32_t> idx;
    std::vector<double> vals;      // value stream of this program
    std::vector<Stage> stages;
    int n_work_stages = 0;         // stages[0 .. n_work_stages) write scratch
    int64_t scr_rows = 0;          // rows of each scratch buffer
    int64_t in_rows = 0, out_rows = 0;
    int max_n_out = 0, max_n_in = 0;
    // fused form of stages [0, n_work_stages) (groups sorted by task);
    // fused_ok: every sub-op reads the input panel or the level before its
    // own
    std::vector<FusedGroup> fgroups;
    std::vector<FusedLevel> flevels;
    std::vector<Op> fops;
    std::vector<SubOp> fsubs;
    int32_t f_max_lds_rows = 0;
    int32_t fused_ok = 0;
    int64_t f_extra_rows = 0;  // rows of scratch buffer A past scr_rows used by the fused form
};

// LDS rows per buffer of a fused group (two buffers of 16 FP64 columns: 128 KB)
constexpr int kFusedMaxRows = 512;

// Host execution of a program (verification): in [in_rows][R], out
// [out_rows][R] (overwritten).  Regenerated dense blocks are not part of a
// program; they run separately (see the regenerated-block executors).
// fused: the work stages run in their fused form (requires fused_ok).
void host_run_program(const Program &p, int R, const double *in, double *out, bool fused = false);

}  // namespace idbf
}  // namespace sht
