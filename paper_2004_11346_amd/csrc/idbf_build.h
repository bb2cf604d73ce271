// Host-side factor structures of the fast ALT (plan time, FP64).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "sht.h"
#include "sht_internal.h"

namespace sht {
namespace idbf {

// Interpolative decomposition over a candidate index list `cand` (global
// row or column indices of the task matrix).
//   column ID:  K(:, cand[red]) ~= K(:, cand[skel]) T        (T: k x nred)
//   row ID:     K(cand[red], :) ~= T^T K(cand[skel], :)
// Applying a column ID to a vector aligned with cand: z = x[skel] + T x[red];
// the transpose (row ID in the forward direction): y[skel] += u, y[red] += T^T u.
struct ID {
    std::vector<int> skel, red;   // positions in cand
    std::vector<double> T;        // k x nred, row-major
    std::vector<int> skel_glob;   // cand[skel]
    bool capped = false;          // stopped at the rank cap with columns left (tolerance not shown)
    int k() const { return (int)skel.size(); }
};

// Interpolative decomposition butterfly factorization of one block
// (Section 2.2):  K ~= U^L ... U^h S^h V^h ... V^L.
struct Butterfly {
    int L = 0, h = 0;
    int r0 = 0, r1 = 0, c0 = 0, c1 = 0;  // block extent in the task matrix
    // column pass, level l = 0..h: row node A at row level l, column node B at
    // column level L-l; index A * 2^(L-l) + B
    std::vector<std::vector<ID>> col;
    // row pass, level l = 0..L-h: row node A at row level L-l, column node B at
    // column level l; index A * 2^l + B
    std::vector<std::vector<ID>> row;
    // middle couplings S(A, B) = K(r(A,B), c(A,B)), A at row level h, B at
    // column level L-h; row-major |r| x |c|
    std::vector<std::vector<double>> S;
};

enum BlockType { kDense = 0, kLowRank = 1, kButterfly = 2 };

// Three-term recurrence state of one matrix row (node x_r) at a degree k:
// the entries of degrees k-1 and k are p0 * 2^e and p1 * 2^e.
struct RecState {
    double p0 = 0.0, p1 = 0.0;
    double pm2 = 0.0;  // entry of degree k-2 (same parity as k), same scale
    int32_t e = 0;
};

// Advance a state of order a at node x from degree k to k + 1 (same
// arithmetic and rescaling as the table builder and the device kernels).
void rec_step(const LegendreTables &lt, int a, double x, int k, RecState &s);
enum Region { kOsc = 0, kNonOsc = 1, kTurning = 2 };

struct Block {
    int type = kDense;
    int region = kOsc;
    int r0 = 0, r1 = 0, c0 = 0, c1 = 0;  // extent after trimming
    std::vector<double> D;               // dense: (r1-r0) x (c1-c0) row-major
    int rank = 0;                        // low rank: A ~= U V^T
    std::vector<double> U, V;            // U: rows x rank, V: cols x rank (row-major)
    Butterfly bf;
    // dense blocks regenerated on the device: no values, but the recurrence
    // state of every row at columns ck_c0 + 16 q (q < ck_n, ck_c0 = c0 & ~15)
    bool gen = false;
    int ck_c0 = 0, ck_n = 0;
    std::vector<RecState> ck;  // [row - r0][q]
    int64_t stored() const;    // stored factor entries
};

// State of block row r (task row) at task column col (c0 <= col < c1) of a
// regenerated dense block: nearest checkpoint, then the recurrence.
RecState gen_state(const LegendreTables &lt, int a, int parity, const Block &b, int r, int col);
// Entry (r, col) of a regenerated dense block as the device forms it.
double gen_value(const RecState &s);

struct Task {
    int a = 0, parity = 0, rows = 0, cols = 0;
    double scale = 0.0;  // largest |entry| of the task matrix
    std::vector<Block> blocks;
};

struct BuildStats {
    int64_t dense_entries = 0;   // entries of all task matrices
    int64_t stored = 0;          // stored factor entries
    int64_t n_dense = 0, n_lowrank = 0, n_butterfly = 0, n_dropped = 0;
    int64_t dense_stored = 0, lowrank_stored = 0, butterfly_stored = 0;
    int64_t n_gen = 0, gen_entries = 0;   // regenerated dense blocks and their area
    int max_rank = 0;
    double seconds = 0.0;
    int64_t region_stored[3][3] = {{0}};  // [region][type]
    int64_t region_area[3] = {0};         // dense entries per region (after trimming)
};

struct HostPlanData {
    int N = 0;
    sht_plan_opts opts{};
    LegendreTables lt;
    std::vector<Task> tasks;  // index 2 * a + parity
    BuildStats stats;
    std::string stats_json() const;
};

// Statistics of a plan as a JSON object.
std::string stats_json(const BuildStats &stats, const sht_plan_opts &opts);

// Build every task (all orders, both parities).  `lt`, when given, holds the
// Legendre tables of degree N already built by the caller (copied into out).
int build_all(int N, const sht_plan_opts &opts, HostPlanData &out, const LegendreTables *lt = nullptr);


}  // namespace idbf
}  // namespace sht
