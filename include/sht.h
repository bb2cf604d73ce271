/*
 * sht.h -- C-ABI of the MI355X (gfx950) spherical harmonic transform library.
 *
 * The library applies the spherical harmonic transform (SHT) of degree N
 * described in Bremer, Chen & Yang, "Rapid application of the spherical
 * harmonic transform via interpolative decomposition butterfly
 * factorization" (arXiv 2004.11346):
 *
 *   f(theta, phi) = sum_{k=0}^{2N-1} sum_{m=-k}^{k} beta_{k,m} Pbar_k^{|m|}(cos theta) e^{i m phi}
 *
 * (Section 1, the expansion of f), evaluated on the tensor grid of the 2N
 * Gauss-Legendre nodes in x = cos(theta) and the M = 4N-1 equispaced
 * phi_j = 2 pi (j + 1/2) / M (Section 1, grid definition).  The associated
 * Legendre transform (ALT) g(m, theta_l) = sum_k beta_{k,m} Pbar_k^{|m|}(x_l)
 * (Section 1; Section 3.1.1) is applied either densely (the plain O(N^3)
 * form, Legendre values regenerated on the fly) or through the hierarchically
 * partitioned interpolative decomposition butterfly factorization (IDBF) of
 * Section 3.2-3.3; the phi sums are length-M DFTs.
 *
 * Conventions
 *   Pbar_k^m   L2-normalised on [-1, 1], no Condon-Shortley phase.
 *   beta       device buffer, complex, interleaved (re, im), element type
 *              double (SHT_F64) or float (SHT_F32); shape [batch][4 N^2];
 *              m-major: orders in the sequence 0, 1, -1, 2, -2, ...,
 *              2N-1, -(2N-1); inside an order the degrees k = |m| .. 2N-1.
 *   f          device buffer, complex interleaved, shape [batch][2N][M];
 *              row l = l-th Gauss-Legendre node in ascending x (Section 1),
 *              column j = phi_j.
 *   g          (ALT-only calls) same shape as f, order m stored in column
 *              (m mod M).
 *   stream     a hipStream_t passed as void*; NULL is the default stream.
 *              Every call only enqueues work on that stream (asynchronous);
 *              the caller owns all buffers and must keep them alive until
 *              the work has completed.
 *
 * Ownership: a plan owns every device array it allocates (factor streams,
 * tables, workspace).  Its factors are immutable after creation.  A plan may
 * be used from several host threads and streams: calls on one plan are
 * ordered by the plan (a call enqueued on stream B after a call on stream A
 * first makes B wait for A's work on the plan), because they share the plan's
 * workspace.  Independent plans run concurrently.
 *
 * Errors: every int-returning call returns SHT_OK (0) or a negative SHT_ERR_*
 * code; no exception crosses the ABI.  Kernels never abort: NaN and Inf in the
 * inputs propagate to the outputs.  sht_strerror() gives a message, and
 * sht_last_error_detail() the last detailed message of the calling thread.
 */
#ifndef SHT_H_
#define SHT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- codes ------------------------------------------------------------- */
#define SHT_OK 0
#define SHT_ERR_INVALID_ARG (-1)  /* bad N, batch, range, NULL pointer, ... */
#define SHT_ERR_UNSUPPORTED (-2)  /* dtype/method/size combination not built */
#define SHT_ERR_OOM (-3)          /* host or device allocation failed */
#define SHT_ERR_HIP (-4)          /* a HIP runtime call failed (detail kept) */
#define SHT_ERR_PLAN (-5)         /* plan construction failed numerically */
#define SHT_ERR_PLAN_CORRUPT (-7) /* a cached plan file failed its header or
                                     checksum test (see cache_dir) */
#define SHT_ERR_MISALIGNED (-6)   /* buffer not aligned to its complex element
                                     (16 bytes FP64, 8 bytes FP32) */

/* element types of beta / f / g */
#define SHT_F64 0
#define SHT_F32 1

/* ALT methods */
#define SHT_DENSE 0 /* plain form: dense per-order product, Pbar regenerated */
#define SHT_IDBF 1  /* fast form: partitioned IDBF / low-rank / dense blocks */

/* directions for sht_alt_apply */
#define SHT_FWD 0 /* beta -> g:  g(m, theta_l) = sum_k beta_{k,m} Pbar_k^{|m|}(x_l) */
#define SHT_INV 1 /* g -> beta:  beta = A_m^T W g  (Section 3.1.1, B = A^T W) */
#define SHT_ADJ 2 /* g -> beta:  beta = A_m^T g    (transpose, no weights) */

/* F32 arithmetic for the IDBF block products */
#define SHT_F32_VALU 0       /* FP32 factors and vectors; products on the vector
                                ALUs below 16 right-hand sides (4 batch), on
                                the FP64 matrix cores (FP64 products and sums)
                                from 16 */
#define SHT_F32_SPLIT_BF16 1 /* split-BF16 three-product MFMA, FP32 accumulate
                                (two BF16 parts per value: a few 1e-6 to 1e-5
                                relative) */
#define SHT_F32_SPLIT_BF16_6 2 /* six products of three BF16 parts per value
                                  (FP32 accuracy on the BF16 matrix cores) */

/* phi DFT schedule (sht_plan_opts.dft_schedule) */
#define SHT_DFT_AUTO 0      /* by length and type (below) */
#define SHT_DFT_ROWS 1      /* one row per workgroup in LDS, mixed-radix passes */
#define SHT_DFT_RADER 2     /* prime M: Rader's length-(M-1) convolution in LDS */
#define SHT_DFT_FOUR_STEP 3 /* M = M1 M2: two kernels through a grid-sized buffer */

/* fast-form level schedules (sht_plan_opts.level_schedule) */
#define SHT_LEVELS_AUTO 0
#define SHT_LEVELS_STAGED 1
#define SHT_LEVELS_FUSED 2

/* ID row sampling (Section 2.1) */
#define SHT_SAMPLE_MOCK_CHEB 0
#define SHT_SAMPLE_RANDOM 1

typedef struct sht_plan sht_plan_t;

/* Plan-construction parameters (Section 2.1, 2.3, 3.2 and Section 5).  Call
 * sht_plan_opts_default() and change fields; a NULL opts means defaults. */
typedef struct sht_plan_opts {
    double eps;        /* ID / low-rank tolerance, relative to the block's
                          largest entry (paper: 1e-10; default 1e-12) */
    int n0;            /* partition: split turning-point blocks while
                          max(rows, cols) > n0 (paper: 512; default 256) */
    int leaf;          /* IDBF leaf size; 0 (default): by size, 32 up to
                          N = 256, 128 up to N = 1024, 64 above (the measured
                          crossover between applying butterflies and
                          regenerating dense blocks on MI355X) */
    int rk;            /* adaptive rank cap r_k of each ID (paper: 150) */
    int oversample;    /* ID row oversampling t (default 2) */
    int rsvd_r;        /* randomized-SVD rank r (paper: 30) */
    int rsvd_q;        /* randomized-SVD oversampling q (paper: 2) */
    int sampling;      /* SHT_SAMPLE_MOCK_CHEB or SHT_SAMPLE_RANDOM */
    uint64_t seed;     /* seed of every random choice of the plan */
    int threads;       /* host threads for plan construction (0 = all) */
    int f32_mode;      /* SHT_F32_VALU, SHT_F32_SPLIT_BF16 or SHT_F32_SPLIT_BF16_6
                          (FP32 plans of the fast form) */
    int min_idbf;      /* smallest block side given an IDBF (default 4*leaf) */
    int dense_gen;     /* 1 (default): dense blocks of the fast form are not
                          stored; their own kernels regenerate the entries with
                          the three-term recurrence from per-row checkpoints
                          (at the block's first column per 64-row tile, and
                          per 64-column output tile for the transpose).
                          0: store their values. */
    int m_lo, m_hi;    /* orders |m| in [m_lo, m_hi] covered by the fast form's
                          factors (default 0 and -1 = all).  A plan restricted
                          to a range serves sht_alt_apply inside it (one GPU's
                          share of the orders); the full transforms need all. */
    int dft_schedule;  /* SHT_DFT_AUTO (default): rows in LDS when the row fits
                          and M is not a prime above 13; Rader when M is prime
                          and M - 1 fits; else four-step.  The others force a
                          schedule (plan creation fails with UNSUPPORTED where
                          it does not apply); the results agree to rounding. */
    int id_check;      /* 1 (default): every ID samples at least n + 8 rows, is
                          verified on other rows (recomputed from all rows if
                          the check fails), and a butterfly with an ID cut at
                          r_k becomes a regenerated dense block.  0: the IDs
                          of Section 2.1 as written (t min(n, r_k) sampled
                          rows, no check, truncated butterflies kept), for
                          the sampling and rank study of Section 5. */
    const char *cache_dir; /* NULL (default): no plan cache.  Else a directory
                          where fast-form plans are stored after their first
                          build and reloaded by later plans with the same N and
                          factor options (eps, n0, leaf, rk, oversample,
                          rsvd_r, rsvd_q, sampling, seed, f32_mode, min_idbf,
                          dense_gen, m_lo, m_hi, id_check; batch, dtype and the DFT
                          schedule do not enter).  A file that fails its
                          header or checksum test (SHT_ERR_PLAN_CORRUPT from
                          sht_plan_cache_verify) is rebuilt and rewritten; the
                          plan statistics report "plan_cache": "hit", "miss",
                          "corrupt_rebuilt" or "off". */
    int level_schedule; /* fast form, non-final levels of the butterflies
                          (Section 2.2: column IDs level by level, middle
                          couplings, row IDs) and of the low-rank blocks
                          (Section 2.3).  SHT_LEVELS_AUTO (default) and
                          SHT_LEVELS_STAGED: one launch per level, the
                          intermediate rows of every level through the
                          scratch buffers (the faster schedule on MI355X).
                          SHT_LEVELS_FUSED: one workgroup per block and 16
                          right-hand sides runs all the block's levels, the
                          intermediate rows in LDS (in HBM rows of its own
                          for blocks whose levels exceed 512 rows); it needs
                          the matrix-core executor (16 or more real
                          right-hand sides, not split-BF16), else plan
                          creation fails with UNSUPPORTED.  The products and
                          their order are the same in every schedule. */
} sht_plan_opts;

void sht_plan_opts_default(sht_plan_opts *opts);

/* Build a plan for degree N (2N latitudes, 4N-1 longitudes) and `batch`
 * fields on the current HIP device.  dtype: SHT_F64 or SHT_F32; method:
 * SHT_DENSE or SHT_IDBF.  Nodes, weights, Legendre tables and every
 * factorisation are computed on the host in FP64 (Section 3), then uploaded
 * once.  N >= 1, batch >= 1.  On success *out owns the plan; release it with
 * sht_plan_destroy().  Errors: INVALID_ARG, UNSUPPORTED, OOM, HIP, PLAN. */
int sht_plan_create(int N, int batch, int dtype, int method,
                    const sht_plan_opts *opts, sht_plan_t **out);

void sht_plan_destroy(sht_plan_t *plan);

/* Check a cached plan file (see sht_plan_opts.cache_dir): SHT_OK,
 * SHT_ERR_PLAN_CORRUPT (bad magic or format version, truncated, checksum
 * mismatch) or SHT_ERR_INVALID_ARG (cannot be read). */
int sht_plan_cache_verify(const char *path);

/* File name of the cached plan of degree N with these options under
 * opts->cache_dir (NUL-terminated, at most `cap` bytes); returns the length
 * needed including the NUL, or a negative error. */
int sht_plan_cache_path(int N, const sht_plan_opts *opts, char *path, size_t cap);

/* Graph mode (Section 1: the steady-state forward, inverse and adjoint calls
 * of a plan).  With enable = 1, each sht_forward / sht_inverse /
 * sht_backward call is served from a hipGraph: the first call with a given
 * (direction, input, output) triple records the call's kernels into a graph
 * (captured on a stream of the plan, so any caller stream, including the
 * default one, works) and every call launches the instantiated graph on the
 * caller's stream.  Results equal the eager calls bit for bit.  Graphs are
 * kept per buffer triple (at most 16 per plan, least recently used dropped
 * first); enable = 0 drops them.  Kernel timing (sht_profile) does not see
 * kernels inside graphs. */
int sht_set_graph_capture(sht_plan_t *plan, int enable);

/* Forward SHT (Section 1): beta [batch][4N^2] -> f [batch][2N][M].
 * ALT for every order, parity split (Section 3.1.2), then the phi synthesis
 * f(theta_l, phi_j) = sum_m g(m, theta_l) e^{i m phi_j}.  `f` may not alias
 * `beta`. */
int sht_forward(const sht_plan_t *plan, const void *beta, void *f, void *stream);

/* Inverse SHT (Section 1; Section 3.1.1): f -> beta with
 * g = (1/M) sum_j f e^{-i m phi_j} and beta = A_m^T W g.  Exact left inverse
 * of sht_forward.  `f` is not modified. */
int sht_inverse(const sht_plan_t *plan, const void *f, void *beta, void *stream);

/* Adjoint of sht_forward (conjugate transpose; the transposed butterfly and
 * DFT of Section 3.1.1): grad_beta = S^H grad_f, i.e. the inverse without the
 * 1/M and without the weights.  This is the vector-Jacobian product in
 * PyTorch's complex convention. */
int sht_backward(const sht_plan_t *plan, const void *grad_f, void *grad_beta, void *stream);

/* Allocation-free inverse, for callers that cannot allocate device memory
 * during the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same result as sht_inverse, bit for bit:
 * the same kernels run, but the phi-analysed grid g (2 x elt x batch x 2N x M
 * bytes) is staged in a fixed device array of 128 MiB that the library holds
 * once per GPU until the process ends (its address is looked up when the
 * first plan is created on that GPU), instead of in the plan's workspace.
 * Nothing is allocated or freed.  Plans whose grid exceeds 128 MiB (e.g. more
 * than one FP64 field at N = 1024) are rejected with SHT_ERR_UNSUPPORTED.
 * Every call on one GPU shares the array: calls that overlap in time on that
 * GPU (several streams, several host threads) race and must be serialised by
 * the caller.  Every byte read from the array is written earlier in the same
 * call, so nothing needs clearing between calls. */
int sht_inverse_noalloc(const sht_plan_t *plan, const void *f, void *beta, void *stream);

/* Real fields (Section 1, the expansion of f with real values).  A real f
 * has beta_{k,-m} = conj(beta_{k,m}) (the same Pbar_k^{|m|} serves both signs
 * of m), so only the orders m >= 0 are stored:
 *   beta_half  [nreal][N (2N + 1)] complex: orders m = 0 .. 2N-1, inside an
 *              order the degrees k = m .. 2N-1 (order m starts at
 *              2N m - m (m - 1) / 2); the imaginary parts at m = 0 are
 *              ignored by the forward transform and returned as 0;
 *   f          [nreal][2N][M] real (double or float as the plan's dtype).
 * Fields 2p and 2p + 1 are carried as one complex field z = f1 + i f2, so a
 * plan of `batch` complex fields transforms up to 2 batch real fields at the
 * cost of `batch` complex ones: the ALT has 2 real right-hand sides per real
 * field instead of 4, and one complex phi DFT serves two real rows.
 * 1 <= nreal <= 2 batch (the ALT always runs over all `batch` pairs).
 * Buffers aligned to the element type.  sht_inverse_real is the exact left
 * inverse of sht_forward_real on real band-limited grids. */
int sht_forward_real(const sht_plan_t *plan, int nreal, const void *beta_half, void *f, void *stream);
int sht_inverse_real(const sht_plan_t *plan, int nreal, const void *f, void *beta_half, void *stream);

/* ALT only, for the orders with m_lo <= |m| <= m_hi (both signs), no DFT
 * (Section 1, ALT; Section 3.1.1).
 *   dir = SHT_FWD: in = beta [batch][4N^2], out = g [batch][2N][M]; only the
 *                  columns of the selected orders are written.
 *   dir = SHT_INV / SHT_ADJ: in = g [batch][2N][M], out = beta; only the
 *                  slots of the selected orders are written.
 * 0 <= m_lo <= m_hi <= 2N-1.  This is the per-GPU share when the orders are
 * distributed over several GPUs. */
int sht_alt_apply(const sht_plan_t *plan, int m_lo, int m_hi, int dir,
                  const void *in, void *out, void *stream);

/* Plan statistics as JSON (block counts by type, ranks, stored entries,
 * bytes, build time; the phi DFT schedule "dft" (rows, rader, four_step or
 * none) and "dft_rader_last", the prime of each pass list (rows or first
 * four-step kernel, second four-step kernel; 0: none) whose last pass runs
 * by Rader's convolution).  Writes at most `cap` bytes including the NUL;
 * returns the full length needed (>= 0) or a negative error. */
int sht_plan_stats(const sht_plan_t *plan, char *json, size_t cap);

/* Per-kernel timing.  sht_profile(plan, 1) clears earlier records and makes
 * every later call on this plan bracket each kernel launch with HIP events
 * recorded on the call's stream; sht_profile(plan, 0) stops recording.
 * sht_profile_report waits for the recorded events and writes JSON
 * {"<kernel>": {"launches": n, "total_ms": t, "avg_ms": t / n}, ...}
 * (same size convention as sht_plan_stats).  Not for use while the stream
 * is being captured into a graph; the recorder is not thread-safe, so a
 * profiled plan is used from one host thread at a time. */
int sht_profile(sht_plan_t *plan, int enable);
int sht_profile_report(const sht_plan_t *plan, char *json, size_t cap);

/* Sizes of the plan. */
int sht_plan_info(const sht_plan_t *plan, int *N, int *batch, int *dtype, int *method);

/* Gauss-Legendre nodes (ascending) and weights of the plan, copied to host
 * arrays of 2N doubles. */
int sht_plan_nodes(const sht_plan_t *plan, double *x, double *w);

const char *sht_strerror(int code);
const char *sht_last_error_detail(void);

/* ---- grouped transforms ------------------------------------------------
 * Many independent transforms of different degrees applied together (the
 * uneven workload: e.g. 64 transforms with N in {128, 256, 512, 1024} and 1-4
 * fields each).  Transform i has degree Ns[i] (1 <= Ns[i] <= 1024) and
 * fields[i] (1..4) fields; all share the dtype.  Each phase (forward ALT, phi
 * synthesis; phi analysis, transposed ALT) is one persistent launch whose
 * workgroups pull (transform, order, node tile) or (transform, field, row)
 * items from a device queue ordered longest first.  The plain (dense) ALT is
 * used.  The group owns its tables, queues and an inverse workspace; the
 * caller owns the coefficient and grid buffers and binds them once. */
typedef struct sht_group sht_group_t;

int sht_group_create(int n, const int *Ns, const int *fields, int dtype, sht_group_t **out);

/* Group execution modes.
 *   SHT_GROUP_PERSISTENT: the persistent kernels above (plain ALT).
 *   SHT_GROUP_BATCHED: the transforms of each distinct degree N form one
 *     batch of sum(fields) fields applied by one plan (plain or fast form),
 *     so many fields share the matrix-core paths of the per-plan kernels;
 *     each transform's fields are copied into and out of per-degree staging
 *     buffers (a degree with a single transform uses its buffers directly).
 *     sht_group_tune times, per degree, the plain form and fast-form plans
 *     with several leaf sizes (Section 2.2; the smallest block given a
 *     butterfly) on the bound buffers and keeps the fastest; choices are
 *     cached in tune_file (one JSON entry per (arch, N, R = 4 fields, dtype))
 *     and read back when a group is created.  1 <= N <= 8192, fields >= 1. */
#define SHT_GROUP_PERSISTENT 0
#define SHT_GROUP_BATCHED 1
typedef struct sht_group_opts {
    int mode;                   /* SHT_GROUP_PERSISTENT (default) or SHT_GROUP_BATCHED */
    const char *tune_file;      /* batched: JSON file of tuned choices (read at create, written by tune); NULL: none */
    const char *plan_cache_dir; /* batched: plan cache directory (sht_plan_opts.cache_dir) of its plans */
} sht_group_opts;
void sht_group_opts_default(sht_group_opts *opts);
int sht_group_create_ex(int n, const int *Ns, const int *fields, int dtype, const sht_group_opts *opts,
                        sht_group_t **out);
void sht_group_destroy(sht_group_t *grp);

/* Bind device buffers: beta[i] [fields_i][4 N_i^2] and f[i] [fields_i][2 N_i][4 N_i - 1]
 * complex, laid out as for a plan.  Forward reads beta and writes f; inverse
 * reads f and writes beta.  Re-binding drops captured graphs. */
int sht_group_bind(sht_group_t *grp, void *const *beta, void *const *f);
int sht_group_forward(sht_group_t *grp, void *stream);
int sht_group_inverse(sht_group_t *grp, void *stream);

/* Autotuner: times a few persistent grid sizes per phase on the bound
 * buffers (overwriting f, beta and the workspace) and keeps the fastest;
 * the timings are reported by sht_group_stats.  Drops captured graphs. */
int sht_group_tune(sht_group_t *grp, void *stream);

/* Capture one direction (SHT_FWD or SHT_INV) on a non-default stream into a
 * hipGraph for the bound buffers, and replay it.  The graph holds kernel
 * nodes only (counters are cleared by a kernel, not a memset). */
int sht_group_capture(sht_group_t *grp, int dir, void *stream);
int sht_group_replay(sht_group_t *grp, int dir, void *stream);

/* Work items, grid sizes and tuning timings as JSON (size convention as
 * sht_plan_stats). */
int sht_group_stats(const sht_group_t *grp, char *json, size_t cap);

/* ---- plan verification on the host (no GPU needed) --------------------
 * These calls build the same FP64 plan as sht_plan_create without touching
 * a device, and apply it with a plain host loop over the packed factor
 * stream in the order the kernels use.  They exist so that the plan builder
 * can be checked on a machine without a GPU; the transform entry points
 * above never call them. */
typedef struct sht_host_plan sht_host_plan_t;

int sht_host_plan_create(int N, int method, const sht_plan_opts *opts, sht_host_plan_t **out);
void sht_host_plan_destroy(sht_host_plan_t *hp);

/* Apply the packed ALT program of order |m| and parity (0 even: k-|m| even,
 * 1 odd) to R real right-hand sides.  dir = SHT_FWD: in [cols][R] ->
 * out [N][R] (half-grid rows, row r = node 2N-1-r, i.e. theta ascending);
 * dir = SHT_ADJ: in [N][R] -> out [cols][R].  cols = N - ceil(|m|/2) (odd)
 * or N - floor(|m|/2) (even), Section 3.1.2. */
int sht_host_plan_apply(const sht_host_plan_t *hp, int absm, int parity, int dir,
                        int R, const double *in, double *out);

/* Dense half-grid matrix of (|m|, parity) from the plan builder's own
 * Legendre recurrence: out [N][cols] row-major. */
int sht_host_alt_matrix(const sht_host_plan_t *hp, int absm, int parity, double *out);

int sht_host_plan_stats(const sht_host_plan_t *hp, char *json, size_t cap);

/* The library's own 2N-point Gauss-Legendre rule (ascending). */
int sht_host_gauss_legendre(int n, double *x, double *w);

/* The phi DFT tables a plan of degree N, element type dtype (SHT_F64 or
 * SHT_F32) and schedule (SHT_DFT_*) hands to its kernels, as JSON (same size
 * convention as sht_plan_stats): "kind" (rows, rader, four_step, none), "M",
 * the pass lists ("radix", "blen", "src_pos": radices in pass order, block
 * length before each pass, and the slot of every output frequency after the
 * passes; "radix2", ... for the second four-step kernel, of length M2), "M1",
 * "M2", "chunk1", "chunk2"; for the Rader schedule "inslot", "outslot" and
 * "bspec" ([2][M - 1] complex, sign +1 then -1, in the slots of the passes of
 * M - 1); and "rader_last": for each pass list, {"R": prime or 0, "radix",
 * "blen", "src_pos" of R - 1, "inslot", "outslot", "bspec"}.  Host only, no
 * GPU; for checking the DFT schedules (Section 1, the phi sums). */
int sht_host_dft_tables(int N, int dtype, int schedule, char *json, size_t cap);

#ifdef __cplusplus
}
#endif

#endif /* SHT_H_ */
