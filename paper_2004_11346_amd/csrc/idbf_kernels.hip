// HIP executor of the packed fast-ALT program and the panel kernels around it.
//
// Panels: X[task][col][R] holds the coefficients of one (|m|, parity) task as
// R = 4 * batch real right-hand sides per column (field f, sign of m, re/im:
// column 4f + 2s + c); Y[task][row][R] holds half-grid values (row r = node
// 2N-1-r).  k_pack / k_scatter move between beta and X, k_combine / k_fold
// between Y and the (l, m mod M) grid with the parity split of Section 3.1.2.
//
// k_ops executes one stage of the program: one wave per op (see below); the
// input rows of each sub-op are gathered into LDS, the stored matrix streams
// from HBM output-major (consecutive lanes, consecutive words), and the
// products, identity (skeleton) terms and the final write (scratch) or
// accumulation (output panel) follow.  Ops of one stage never write the same
// rows, so there are no atomics and the result is bitwise reproducible.
//
// Regenerated dense blocks (near the turning point, Section 3.2) are not part
// of the program: k_gen_fwd* and k_gen_adj apply them after it, walking the
// same-parity recurrence from stored per-row states.
#include <hip/hip_runtime.h>

#include "idbf_device.h"
#include "prof.h"
#include "kernels.h"

namespace sht {
namespace idbf {

namespace {

__device__ __forceinline__ int64_t d_coef_offset(int N, int m) {
    int64_t a = m < 0 ? -(int64_t)m : m;
    int64_t twoN = 2 * (int64_t)N;
    if (a == 0) return 0;
    int64_t off = twoN * (2 * a - 1) - a * (a - 1);
    if (m < 0) off += twoN - a;
    return off;
}


__device__ __forceinline__ double scale_of(int e) { return e < -1074 ? 0.0 : ldexp(1.0, e); }

// next column of the same parity: the composed two-step recurrence
// p_k = (alpha_k x^2 + beta_k) p_{k-2} + gamma_k p_{k-4}; c3 = (alpha, beta, gamma)
__device__ __forceinline__ void gen_2step(const double *__restrict__ c3, double x2, double &p0, double &p1, int &e,
                                          double &sc) {
    const double p2 = fma(c3[0], x2, c3[1]) * p1 + c3[2] * p0;
    p0 = p1;
    p1 = p2;
    if (fabs(p1) > 0x1p200) {
        p0 *= 0x1p-200;
        p1 *= 0x1p-200;
        e += 200;
        sc = scale_of(e);
    }
}

// n consecutive columns of the same parity with no column guard (tiles that
// lie inside their segment, past its first column): values p_k * 2^e go to
// out[j * stride], and the rescale test runs once at the end.  Scaling by
// 2^-200 is exact, so the values equal those of n gen_2step calls; n steps
// grow |p| far less than from 2^200 to the top of the FP64 range.
template <int n>
__device__ __forceinline__ void gen_run(const double *__restrict__ c3, double x2, double &p0, double &p1, int &e,
                                        double &sc, double *out, int stride) {
    static_assert(n % 2 == 0, "steps come in pairs");
    double q0 = p0, q1 = p1;
#pragma unroll
    for (int j = 0; j < n; j += 2) {
        const double *c = c3 + 3 * j;
        const double r2 = fma(c[0], x2, c[1]) * q1 + c[2] * q0;
        out[j * stride] = r2 * sc;
        const double r3 = fma(c[3], x2, c[4]) * r2 + c[5] * q1;
        out[(j + 1) * stride] = r3 * sc;
        q0 = r2;
        q1 = r3;
    }
    p0 = q0;
    p1 = q1;
    if (fabs(p1) > 0x1p200 || fabs(p0) > 0x1p200) {
        p0 *= 0x1p-200;
        p1 *= 0x1p-200;
        e += 200;
        sc = scale_of(e);
    }
}

__device__ __forceinline__ int64_t d_tri_offset2(int N, int a) {
    return 2 * (int64_t)N * a - (int64_t)a * (a - 1) / 2;
}

// Workgroups go to the eight XCDs in turn (workgroup i to XCD i mod 8).  The
// op and gen kernels hand out items (ops, items) in chunks of kXc consecutive ones: chunk c runs
// on XCD c mod 8, so neighbouring items of a task, which read the same input
// rows, share that XCD's L2, while the chunks (and the uneven work of the
// tasks) still spread over all XCDs.  Grid: 8 kXc ceil(chunks / 8).
constexpr int kXc = 16;
__device__ __forceinline__ int xcd_item(int n, int xc) {
    if (xc <= 0) return blockIdx.x;
    const int x = blockIdx.x & 7, l = blockIdx.x >> 3;
    return ((l / xc) * 8 + x) * xc + l % xc;
}
inline unsigned xcd_grid(int n) {
    if (kXc <= 0) return (unsigned)n;
    const int chunks = (n + kXc - 1) / kXc;
    return 8u * kXc * (unsigned)((chunks + 7) / 8);
}

// One wave per op.  Lanes own matrix outputs: lane q of a sub-op streams
// column q of its output-major matrix (consecutive lanes, consecutive words)
// and keeps the RC right-hand-side sums in registers; the gathered input rows
// sit in LDS and are read as wave-wide broadcasts.
template <typename T, int RC>
__global__ __launch_bounds__(64) void k_ops(const Op *__restrict__ ops, const SubOp *__restrict__ subs,
                                            const int32_t *__restrict__ idx, const T *__restrict__ vals,
                                            int op_begin, int n_ops, const T *__restrict__ in, int64_t in_stride,
                                            T *__restrict__ out, int64_t out_stride, T *__restrict__ scrA,
                                            T *__restrict__ scrB, int rc, int max_out, int max_in) {
    extern __shared__ unsigned char smem_raw[];
    T *acc = reinterpret_cast<T *>(smem_raw);
    T *xin = acc + (size_t)max_out * RC;
    const int oi = xcd_item(n_ops, kXc);
    if (oi >= n_ops) return;
    const Op op = ops[op_begin + oi];
    const int lane = threadIdx.x;
    const int n_out = op.n_out;
    for (int e = lane; e < n_out * RC; e += 64) acc[e] = (T)0;
    for (int s = 0; s < op.nsub; ++s) {
        const SubOp sb = subs[op.sub0 + s];
        const T *src;
        int64_t sstride;
        if (sb.src == kIn) {
            src = in;
            sstride = in_stride;
        } else {
            src = sb.src == kScrA ? scrA : scrB;
            sstride = RC;
        }
        __syncthreads();
        const int nin = sb.n_in, nmap = sb.n_map;
        if (nmap > 0) {
            const int32_t *inr = idx + sb.in_off;
            for (int e = lane; e < nin * RC; e += 64) {
                const int j = e / RC, r = e - j * RC;
                xin[e] = r < rc ? src[(int64_t)inr[j] * sstride + r] : (T)0;
            }
            __syncthreads();
            const int32_t *map = idx + sb.map_off;
            for (int q0 = 0; q0 < nmap; q0 += 64) {
                const int q = q0 + lane;
                if (q < nmap) {
                    T a[RC];
#pragma unroll
                    for (int r = 0; r < RC; ++r) a[r] = (T)0;
                    const T *mp = vals + sb.mat_off + q;
                    int j = 0;
                    for (; j + 4 <= nin; j += 4) {
                        const T m0 = mp[(int64_t)(j + 0) * nmap];
                        const T m1 = mp[(int64_t)(j + 1) * nmap];
                        const T m2 = mp[(int64_t)(j + 2) * nmap];
                        const T m3 = mp[(int64_t)(j + 3) * nmap];
#pragma unroll
                        for (int r = 0; r < RC; ++r) {
                            a[r] += m0 * xin[(j + 0) * RC + r];
                            a[r] += m1 * xin[(j + 1) * RC + r];
                            a[r] += m2 * xin[(j + 2) * RC + r];
                            a[r] += m3 * xin[(j + 3) * RC + r];
                        }
                    }
                    for (; j < nin; ++j) {
                        const T m0 = mp[(int64_t)j * nmap];
#pragma unroll
                        for (int r = 0; r < RC; ++r) a[r] += m0 * xin[j * RC + r];
                    }
                    const int pos = map[q];
#pragma unroll
                    for (int r = 0; r < RC; ++r) acc[pos * RC + r] += a[r];
                }
            }
        }
        __syncthreads();
        if (sb.n_dir > 0) {
            const int32_t *dir = idx + sb.dir_off;
            for (int e = lane; e < sb.n_dir * RC; e += 64) {
                const int d = e / RC, r = e - d * RC;
                if (r < rc) acc[dir[2 * d + 1] * RC + r] += src[(int64_t)dir[2 * d] * sstride + r];
            }
        }
    }
    __syncthreads();
    if (op.dst == kOut) {
        for (int e = lane; e < n_out * RC; e += 64) {
            const int i = e / RC, r = e - i * RC;
            if (r < rc) out[(op.dst_row + i) * out_stride + r] = acc[e];
        }
    } else {
        T *dst = op.dst == kScrA ? scrA : scrB;
        for (int e = lane; e < n_out * RC; e += 64) dst[op.dst_row * RC + e] = acc[e];
    }
}

typedef double d4v __attribute__((ext_vector_type(4)));

// FP64 matrix-core op kernel, one wave per (op, block of 16 right-hand-side
// columns).  For each sub-op the wave gathers its input fragments into
// registers (B = inputs[4 st + l/16][column l % 16], st < 16) and streams the
// output-major values from memory as A = values[16 outputs][4 inputs];
// v_mfma_f64_16x16x4f64 leaves output 16 t + l/16 + 4 i, column l % 16 in
// element i of lane l, which is added into the op's outputs held in LDS
// (n_out x 16) through the sub-op's output map; the identity part is added
// there too and the outputs are stored once.  The column blocks of an op are
// neighbouring work items (same XCD, about the same time), so its values come
// from HBM about once per pass and from L2 for the other blocks.  T is the
// storage type of values and vectors (FP32 plans keep FP32 factors and
// panels); products and sums are FP64.
template <typename T>
__global__ __launch_bounds__(64) void k_ops_mfma(const Op *__restrict__ ops, const SubOp *__restrict__ subs,
                                                   const int32_t *__restrict__ idx, const T *__restrict__ vals,
                                                   int op_begin, int n_items, int ncb, const T *__restrict__ in,
                                                   int64_t in_stride, T *__restrict__ out, int64_t out_stride,
                                                   T *__restrict__ scrA, T *__restrict__ scrB,
                                                   int64_t scr_stride, int rc) {
    extern __shared__ unsigned char smem_raw[];
    double *acc = reinterpret_cast<double *>(smem_raw);
    const int wi = xcd_item(n_items, kXc);
    if (wi >= n_items) return;
    const int oi = wi / ncb, cb = wi - oi * ncb;
    const Op op = ops[op_begin + oi];
    const int lane = threadIdx.x, jl = lane >> 4, cl = lane & 15;
    const int col = 16 * cb + cl;
    const bool cok = col < rc;
    const int n_out = op.n_out;
    for (int e = lane; e < n_out * 16; e += 64) acc[e] = 0.0;
    __syncthreads();
    for (int s = 0; s < op.nsub; ++s) {
        const SubOp sb = subs[op.sub0 + s];
        const T *src;
        int64_t sstride;
        if (sb.src == kIn) {
            src = in;
            sstride = in_stride;
        } else {
            src = sb.src == kScrA ? scrA : scrB;
            sstride = scr_stride;
        }
        const int nin = sb.n_in, nmap = sb.n_map;
        if (nmap > 0) {
            const int32_t *inr = idx + sb.in_off;
            int rows[16];
#pragma unroll
            for (int st = 0; st < 16; ++st) {
                const int j = 4 * st + jl;
                rows[st] = j < nin ? inr[j] : -1;
            }
            double B[16];
#pragma unroll
            for (int st = 0; st < 16; ++st)
                B[st] = (rows[st] >= 0 && cok) ? (double)src[(int64_t)rows[st] * sstride + col] : 0.0;
            const int32_t *map = idx + sb.map_off;
            const T *mv = vals + sb.mat_off;
            const int ntile = (nmap + 15) >> 4;
            for (int t = 0; t < ntile; ++t) {
                const int q = 16 * t + cl;
                // value (4 st + jl, q): wave-uniform row-group base + 32-bit lane offset
                const int aoff = jl * nmap + q;
                double A[16];
#pragma unroll
                for (int st = 0; st < 16; ++st) {
                    const T *mg = mv + (int64_t)(4 * st) * nmap;
                    A[st] = (q < nmap && 4 * st + jl < nin) ? (double)mg[aoff] : 0.0;
                }
                int dst[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int qq = 16 * t + jl + 4 * i;
                    dst[i] = qq < nmap ? map[qq] : -1;
                }
                d4v D = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int st = 0; st < 16; ++st) {
                    if (4 * st >= nin) break;
                    D = __builtin_amdgcn_mfma_f64_16x16x4f64(A[st], B[st], D, 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (dst[i] >= 0) acc[dst[i] * 16 + cl] += D[i];
            }
        }
        if (sb.n_dir > 0) {
            __syncthreads();
            const int32_t *dir = idx + sb.dir_off;
            // identity part: four rows per step, lanes = 16 columns; eight steps batched
            for (int d0 = 0; d0 < sb.n_dir; d0 += 32) {
                int sr[8], dr[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int d = d0 + 4 * k + jl;
                    sr[k] = d < sb.n_dir ? dir[2 * d] : -1;
                    dr[k] = d < sb.n_dir ? dir[2 * d + 1] : -1;
                }
                double v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) v[k] = (sr[k] >= 0 && cok) ? (double)src[(int64_t)sr[k] * sstride + col] : 0.0;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (dr[k] >= 0) acc[dr[k] * 16 + cl] += v[k];
            }
        }
        __syncthreads();
    }
    if (!cok) return;
    if (op.dst == kOut) {
        for (int i = jl; i < n_out; i += 4) out[(op.dst_row + i) * out_stride + col] = (T)acc[i * 16 + cl];
    } else {
        T *dst = op.dst == kScrA ? scrA : scrB;
        for (int i = jl; i < n_out; i += 4) dst[(op.dst_row + i) * scr_stride + col] = (T)acc[i * 16 + cl];
    }
}

// FP32 plans on the BF16 matrix cores (split-BF16): every FP32 factor value
// a and input x is split into BF16 parts by repeated round-to-nearest-even,
// a_h = bf16(a), a_m = bf16(a - a_h), a_l = bf16(a - a_h - a_m), and a x is
// accumulated in FP32 by v_mfma_f32_16x16x16_bf16 products of the parts:
//   TERMS = 3:  a_h x_h + a_h x_m + a_m x_h   (two parts each; the residuals
//               and the dropped a_m x_m are about 2^-17 of the product)
//   TERMS = 6:  the above + a_m x_m + a_h x_l + a_l x_h   (three parts each;
//               dropped terms below 2^-24, i.e. FP32 accuracy)
// Inputs are split once when staged into LDS as [j / 4][column][j % 4] so
// that a lane's four k values of the B operand are one 8-byte read; A values
// are split as they stream from HBM.  Operand layouts of the 16x16x16 shape:
// A lane l: row l % 16, k = 4 (l / 16) + i; B lane l: column l % 16,
// k = 4 (l / 16) + i; D lane l: rows 4 (l / 16) + i, column l % 16.
typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float v) {
    unsigned u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

template <int NP>
__device__ __forceinline__ void split_bf16(float v, short *parts) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const unsigned short b = bf16_rne(v);
        parts[i] = (short)b;
        v -= bf16_val(b);
    }
}

template <int RCW, int TERMS>
__global__ __launch_bounds__(256) void k_ops_bf16(const Op *__restrict__ ops, const SubOp *__restrict__ subs,
                                                  const int32_t *__restrict__ idx, const float *__restrict__ vals,
                                                  int op_begin, int n_ops, const float *__restrict__ in, int64_t in_stride,
                                                  float *__restrict__ out, int64_t out_stride,
                                                  float *__restrict__ scrA, float *__restrict__ scrB, int rc,
                                                  int max_out, int max_in) {
    constexpr int NCB = RCW / 16;
    constexpr int NP = TERMS == 3 ? 2 : 3;  // BF16 parts per value
    extern __shared__ unsigned char smem_raw[];
    float *acc = reinterpret_cast<float *>(smem_raw);
    const int mi16 = (max_in + 15) & ~15;
    short *xp16 = reinterpret_cast<short *>(acc + (size_t)max_out * RCW);  // NP x [mi16 / 4][RCW][4]
    const size_t pstride = (size_t)mi16 * RCW;
    const int oi = xcd_item(n_ops, kXc);
    if (oi >= n_ops) return;
    const Op op = ops[op_begin + oi];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n_out = op.n_out;
    for (int e = tid; e < n_out * RCW; e += 256) acc[e] = 0.f;
    for (int s = 0; s < op.nsub; ++s) {
        const SubOp sb = subs[op.sub0 + s];
        const float *src;
        int64_t sstride;
        if (sb.src == kIn) {
            src = in;
            sstride = in_stride;
        } else {
            src = sb.src == kScrA ? scrA : scrB;
            sstride = RCW;
        }
        __syncthreads();
        const int nin = sb.n_in, nmap = sb.n_map;
        if (nmap > 0) {
            const int32_t *inr = idx + sb.in_off;
            const int nin16 = (nin + 15) & ~15;
            for (int e = tid; e < nin16 * RCW; e += 256) {
                const int j = e / RCW, c = e - j * RCW;
                const int64_t row = inr[j < nin ? j : 0];
                const float v = (j < nin && c < rc) ? src[row * sstride + c] : 0.f;
                short pt[NP];
                split_bf16<NP>(v, pt);
                const int o = ((j >> 2) * RCW + c) * 4 + (j & 3);
#pragma unroll
                for (int k = 0; k < NP; ++k) xp16[k * pstride + o] = pt[k];
            }
            __syncthreads();
            const int32_t *map = idx + sb.map_off;
            const int ntile = (nmap + 15) >> 4;
            const int jl = lane >> 4, cl = lane & 15;
            const int nks = (nin + 15) >> 4;  // k-steps of 16 inputs
            for (int t = wave; t < ntile; t += 4) {
                const int q = t * 16 + cl;
                float av[16];  // A values: k-step st, slot i -> input 16 st + 4 jl + i
                {
#pragma unroll
                    for (int st = 0; st < 4; ++st)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int j = 16 * st + 4 * jl + i;
                            av[4 * st + i] = (q < nmap && j < nin) ? vals[sb.mat_off + (int64_t)j * nmap + q] : 0.f;
                        }
                }
                f4v D[NCB];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) D[cb] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    if (st >= nks) break;
                    s4v ap[NP];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        short pt[NP];
                        split_bf16<NP>(av[4 * st + i], pt);
#pragma unroll
                        for (int k = 0; k < NP; ++k) ap[k][i] = pt[k];
                    }
                    const int kq = 4 * st + jl;  // group of four inputs
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        const int o = (kq * RCW + cb * 16 + cl) * 4;
                        s4v bp[NP];
#pragma unroll
                        for (int k = 0; k < NP; ++k) bp[k] = *reinterpret_cast<const s4v *>(xp16 + k * pstride + o);
                        // smallest terms first
                        if (TERMS == 6) {
                            D[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[2], bp[0], D[cb], 0, 0, 0);
                            D[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[0], bp[2], D[cb], 0, 0, 0);
                            D[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[1], bp[1], D[cb], 0, 0, 0);
                        }
                        D[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[1], bp[0], D[cb], 0, 0, 0);
                        D[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[0], bp[1], D[cb], 0, 0, 0);
                        D[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ap[0], bp[0], D[cb], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int qq = t * 16 + 4 * jl + i;
                    if (qq < nmap) {
                        float *ar = acc + map[qq] * RCW + cl;
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb) ar[cb * 16] += D[cb][i];
                    }
                }
            }
        }
        __syncthreads();
        if (sb.n_dir > 0) {
            const int32_t *dir = idx + sb.dir_off;
            for (int e = tid; e < sb.n_dir * RCW; e += 256) {
                const int d = e / RCW, c = e - d * RCW;
                if (c < rc) acc[dir[2 * d + 1] * RCW + c] += src[(int64_t)dir[2 * d] * sstride + c];
            }
        }
    }
    __syncthreads();
    if (op.dst == kOut) {
        for (int e = tid; e < n_out * RCW; e += 256) {
            const int i = e / RCW, c = e - i * RCW;
            if (c < rc) out[(op.dst_row + i) * out_stride + c] = acc[e];
        }
    } else {
        float *dst = op.dst == kScrA ? scrA : scrB;
        for (int e = tid; e < n_out * RCW; e += 256) dst[op.dst_row * RCW + e] = acc[e];
    }
}

// ---------------------------------------------------------------------------
// Regenerated forward blocks (after the op program).  One wave per (task,
// 64-row tile): lane = row, the block's columns walked from the row's stored
// state with the two-step recurrence; coefficients and input rows staged in
// LDS by 64-column chunks.  The tile's sums are added to Y once at the end
// (items of one tile are one workgroup, so no two workgroups add to a row).
// task carries kGenOverwrite when the item is the first writer of its output
// tile (no stored factor contributes to it, so the op program leaves it alone)
constexpr int32_t kGenOverwrite = 1 << 30;
struct GenItem {
    int32_t task, row0, seg_begin, seg_end;
};
struct GenSeg {
    int32_t c0, ncol, ck, pad;
};

template <typename T, int RC>
__global__ __launch_bounds__(64) void k_gen_fwd(const GenItem *__restrict__ items, int n_items, int item0,
                                                const GenSeg *__restrict__ segs, const double *__restrict__ ck,
                                                const int32_t *__restrict__ ckexp, const double *__restrict__ xh,
                                                const double *__restrict__ coef2, int N,
                                                const int64_t *__restrict__ x_off, const T *__restrict__ X,
                                                int64_t R, int rc, T *__restrict__ Y) {
    __shared__ double s_c[64 * 3];
    __shared__ T s_x[64 * RC];
    const int ii = xcd_item(n_items, kXc);
    if (ii >= n_items) return;
    const GenItem it = items[item0 + ii];
    const int task = it.task & ~kGenOverwrite;
    const bool ow = (it.task & kGenOverwrite) != 0;  // first writer of its output tile
    const int lane = threadIdx.x;
    const int r = it.row0 + lane;
    const int a = task >> 1, par = task & 1;
    const double x = xh[r < N ? r : N - 1], x2 = x * x;
    const double *cfo = coef2 + 3 * (d_tri_offset2(N, a) + par);
    const T *Xt = X + x_off[task] * R;
    T acc[RC];
#pragma unroll
    for (int q = 0; q < RC; ++q) acc[q] = (T)0;
    for (int s = it.seg_begin; s < it.seg_end; ++s) {
        const GenSeg sg = segs[s];
        double p0 = ck[2 * ((int64_t)sg.ck + lane)], p1 = ck[2 * ((int64_t)sg.ck + lane) + 1];
        int ex = ckexp[sg.ck + lane];
        double sc = scale_of(ex);
        for (int t0 = 0; t0 < sg.ncol; t0 += 64) {
            const int n = min(64, sg.ncol - t0);
            __syncthreads();
            if (lane < n) {
                const int c = sg.c0 + t0 + lane;
#pragma unroll
                for (int k = 0; k < 3; ++k) s_c[3 * lane + k] = cfo[3 * (2 * (int64_t)c) + k];
#pragma unroll
                for (int q = 0; q < RC; ++q) s_x[lane * RC + q] = q < rc ? Xt[(int64_t)c * R + q] : (T)0;
            }
            __syncthreads();
            for (int t = 0; t < n; ++t) {
                if (t0 + t > 0) gen_2step(s_c + 3 * t, x2, p0, p1, ex, sc);
                const T v = (T)(p1 * sc);
#pragma unroll
                for (int q = 0; q < RC; ++q) acc[q] += v * s_x[t * RC + q];
            }
        }
    }
    if (r < N) {
        T *y = Y + ((int64_t)task * N + r) * R;
#pragma unroll
        for (int q = 0; q < RC; ++q)
            if (q < rc) y[q] = ow ? acc[q] : y[q] + acc[q];
    }
}


// FP64 matrix cores: 64 rows x 16 CBP columns per wave; per 8-column tile the
// lanes write their rows' values to LDS and v_mfma_f64_16x16x4f64 takes
// A = values[16 rows][4 columns], B = X[4 columns][16 columns].  The B
// fragments of the next tile are loaded while the current one is generated
// and multiplied; the recurrence coefficients are wave-uniform loads.
// Three waves per SIMD (at most 170 registers, no spills) run faster than the
// compiler's own choice of two.
template <typename T, int CBP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8)))
void k_gen_fwd_mfma(const GenItem *__restrict__ items, int n_items, int xc, int item0,
                                                     const GenSeg *__restrict__ segs, const double *__restrict__ ck,
                                                     const int32_t *__restrict__ ckexp,
                                                     const double *__restrict__ xh, const double *__restrict__ coef2,
                                                     int N, const int64_t *__restrict__ x_off,
                                                     const T *__restrict__ X, int64_t R, int col0,
                                                     T *__restrict__ Y) {
    constexpr int PAD = 9;
    __shared__ double tile[64 * PAD];
    __shared__ double s_c[8 * 3];
    const int ii = xcd_item(n_items, xc);
    if (ii >= n_items) return;
    const GenItem it = items[item0 + ii];
    const int task = it.task & ~kGenOverwrite;
    const bool ow = (it.task & kGenOverwrite) != 0;  // first writer of its output tile
    const int lane = threadIdx.x, jl = lane >> 4, cl = lane & 15;
    const int r = it.row0 + lane;
    const int a = task >> 1, par = task & 1;
    const double x = xh[r < N ? r : N - 1], x2 = x * x;
    const double *cfo = coef2 + 3 * (d_tri_offset2(N, a) + par);
    const T *Xt = X + x_off[task] * R;
    d4v D[4][CBP];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int cb = 0; cb < CBP; ++cb) D[t][cb] = d4v{0.0, 0.0, 0.0, 0.0};
    for (int s = it.seg_begin; s < it.seg_end; ++s) {
        const GenSeg sg = segs[s];
        const double *cs = cfo + 6 * (int64_t)sg.c0;  // (alpha, beta, gamma) of segment column t at cs + 6 t
        const T *Xs = Xt + (int64_t)sg.c0 * R;
        // B fragments of the tile at t0: columns t0 + 4 h + jl, RHS col0 + 16 cb + cl
        auto load_b = [&](double (&B)[2][CBP], int t0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const T *xg = Xs + (int64_t)(t0 + 4 * h) * R;  // wave-uniform base
#pragma unroll
                for (int cb = 0; cb < CBP; ++cb) {
                    const int t = t0 + 4 * h + jl, col = col0 + 16 * cb + cl;
                    B[h][cb] = (t < sg.ncol && col < R) ? (double)xg[jl * (int)R + col] : 0.0;
                }
            }
        };
        // lanes 0..23 carry the (alpha, beta, gamma) triples of a tile's 8 columns
        auto load_c = [&](int t0) {
            const int t = t0 + lane / 3;
            return (lane < 24 && t < sg.ncol) ? cs[6 * t + lane % 3] : 0.0;
        };
        double p0 = ck[2 * ((int64_t)sg.ck + lane)], p1 = ck[2 * ((int64_t)sg.ck + lane) + 1];
        int ex = ckexp[sg.ck + lane];
        double cv = load_c(0), cn = 0.0;
        double B[2][CBP], Bn[2][CBP];
        load_b(B, 0);
        double sc = scale_of(ex);
        for (int t0 = 0; t0 < sg.ncol; t0 += 8) {
            const bool more = t0 + 8 < sg.ncol;
            if (lane < 24) s_c[lane] = cv;
            __syncthreads();
            if (more) {
                cn = load_c(t0 + 8);
                load_b(Bn, t0 + 8);
            }
            if (t0 > 0 && t0 + 8 <= sg.ncol) {
                gen_run<8>(s_c, x2, p0, p1, ex, sc, tile + lane * PAD, 1);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int t = t0 + j;
                    double v = 0.0;
                    if (t < sg.ncol) {
                        if (t > 0) gen_2step(s_c + 3 * j, x2, p0, p1, ex, sc);
                        v = p1 * sc;
                    }
                    tile[lane * PAD + j] = v;
                }
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double A = tile[(16 * t + cl) * PAD + 4 * h + jl];
#pragma unroll
                    for (int cb = 0; cb < CBP; ++cb)
                        D[t][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(A, B[h][cb], D[t][cb], 0, 0, 0);
                }
            __syncthreads();
            if (more) {
                cv = cn;
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int cb = 0; cb < CBP; ++cb) B[h][cb] = Bn[h][cb];
            }
        }
    }
    // element i of lane l: row l/16 + 4 i of row block t, column l % 16
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int cb = 0; cb < CBP; ++cb) {
            const int col = col0 + 16 * cb + cl;
            if (col >= R) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = it.row0 + 16 * t + jl + 4 * i;
                if (row < N) {
                    T *y = Y + ((int64_t)task * N + row) * R + col;
                    *y = ow ? (T)D[t][cb][i] : (T)((double)*y + D[t][cb][i]);
                }
            }
        }
}

// Regenerated transposed blocks (after the op program): one wave per (task,
// 64-column output tile) and block of 16 CBP right-hand sides.  For each
// segment (a block's 64-row chunk) the wave keeps the chunk's H fragments in
// registers (B = H[4 rows][16 right-hand sides], rows 4 ks + l/16), and for
// each 16-column group of the tile the lanes (rows) step the recurrence into
// an LDS tile that is read back transposed as A = values[16 columns][4 rows];
// v_mfma_f64_16x16x4f64 sums over the 64 rows.  With two blocks of right-hand
// sides, three waves per SIMD (168 registers, four of them spilled) run faster
// than the compiler's own choice of two; with one, its own choice (four) is
// kept.
struct GenItemA {
    int32_t task, col0, seg_begin, seg_end;
};
struct GenSegA {
    int32_t row0, c0, ncol, ck;
};

template <typename T, int CBP>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(CBP == 1 ? 1 : 3, 8))) void k_gen_adj(const GenItemA *__restrict__ items, int n_items, int xc, int item0,
                                                const GenSegA *__restrict__ segs, const double *__restrict__ ck,
                                                const int32_t *__restrict__ ckexp, const double *__restrict__ xh,
                                                const double *__restrict__ coef2, int N,
                                                const int64_t *__restrict__ x_off, const T *__restrict__ H,
                                                int64_t R, int rhs0, T *__restrict__ X) {
    constexpr int PAD = 65;
    __shared__ double tile[16 * PAD];
    __shared__ double s_c[64 * 3];
    const int ii = xcd_item(n_items, xc);
    if (ii >= n_items) return;
    const GenItemA it = items[item0 + ii];
    const int task = it.task & ~kGenOverwrite;
    const bool ow = (it.task & kGenOverwrite) != 0;  // first writer of its output tile
    const int lane = threadIdx.x, jl = lane >> 4, cl = lane & 15;
    const int a = task >> 1, par = task & 1;
    const double *cfo = coef2 + 3 * (d_tri_offset2(N, a) + par);
    const int cols_task = (int)(x_off[task + 1] - x_off[task]);
    const T *Ht = H + (int64_t)task * N * R;
    d4v D[4][CBP];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int cb = 0; cb < CBP; ++cb) D[g][cb] = d4v{0.0, 0.0, 0.0, 0.0};
    for (int s = it.seg_begin; s < it.seg_end; ++s) {
        const GenSegA sg = segs[s];
        // recurrence state first: the first steps need it before the H fragments
        const int r = sg.row0 + lane;
        const double x = xh[r < N ? r : N - 1], x2 = x * x;
        double p0 = ck[2 * ((int64_t)sg.ck + lane)], p1 = ck[2 * ((int64_t)sg.ck + lane) + 1];
        int ex = ckexp[sg.ck + lane];
        const double *cs = cfo + 6 * (int64_t)sg.c0;
        // Loads without branches or selects, so that the compiler waits for the
        // early ones alone and the H fragments stay in flight while the first
        // column group is generated: coefficients past the segment's columns
        // are never read (the index is clamped to a valid one), rows past N
        // read row N - 1 and right-hand sides past R read R - 1.  Rows outside
        // the block have zero recurrence states, so their values are 0 and
        // their (finite) fragments add nothing; right-hand sides past R are
        // not stored.
        double cv[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int e = lane + 64 * i;
            const int ee = e < 3 * sg.ncol ? e : 0;
            cv[i] = cs[6 * (ee / 3) + ee % 3];
        }
        __builtin_amdgcn_sched_barrier(0);
        const bool full = sg.row0 + 64 <= N;  // wave-uniform
        double B[16][CBP];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int rr = sg.row0 + 4 * ks + jl;
            const T *hg = Ht + (int64_t)(full ? rr : min(rr, N - 1)) * R;
#pragma unroll
            for (int cb = 0; cb < CBP; ++cb) {
                const int col = rhs0 + 16 * cb + cl;
                B[ks][cb] = (double)hg[col < R ? col : (int)R - 1];
            }
        }
        double sc = scale_of(ex);
        __syncthreads();  // the previous segment no longer reads s_c
#pragma unroll
        for (int i = 0; i < 3; ++i) s_c[lane + 64 * i] = cv[i];
        __syncthreads();
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int gc0 = it.col0 + 16 * g;  // first output column of the group
            if (gc0 + 16 <= sg.c0 || gc0 >= sg.c0 + sg.ncol) continue;
            if (gc0 > sg.c0 && gc0 + 16 <= sg.c0 + sg.ncol) {
                gen_run<16>(s_c + 3 * (gc0 - sg.c0), x2, p0, p1, ex, sc, tile + lane, PAD);
            } else if (CBP > 1 && gc0 == sg.c0 && 16 <= sg.ncol) {
                // the segment's first column is the stored state itself (two
                // 16-column blocks only: with one the extra code costs a wave
                // per SIMD)
                tile[lane] = p1 * sc;
                gen_run<14>(s_c + 3, x2, p0, p1, ex, sc, tile + PAD + lane, PAD);
                gen_2step(s_c + 3 * 15, x2, p0, p1, ex, sc);
                tile[15 * PAD + lane] = p1 * sc;
            } else {
                // a group the segment covers in part: the column test is the
                // same for every lane, and, as in gen_run, the rescale test
                // runs once after the group's steps
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int t = gc0 + j - sg.c0;  // column index in the segment
                    double v = 0.0;
                    if (t >= 0 && t < sg.ncol) {
                        if (t > 0) {
                            const double *c = s_c + 3 * t;
                            const double p2 = fma(c[0], x2, c[1]) * p1 + c[2] * p0;
                            p0 = p1;
                            p1 = p2;
                        }
                        v = p1 * sc;
                    }
                    tile[j * PAD + lane] = v;
                }
                if (fabs(p1) > 0x1p200 || fabs(p0) > 0x1p200) {
                    p0 *= 0x1p-200;
                    p1 *= 0x1p-200;
                    ex += 200;
                    sc = scale_of(ex);
                }
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) {
                const double A = tile[cl * PAD + 4 * ks + jl];
#pragma unroll
                for (int cb = 0; cb < CBP; ++cb)
                    D[g][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(A, B[ks][cb], D[g][cb], 0, 0, 0);
            }
            __syncthreads();
        }
    }
    // element i of lane l: output column l/16 + 4 i of group g, right-hand side l % 16
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int cb = 0; cb < CBP; ++cb) {
            const int col = rhs0 + 16 * cb + cl;
            if (col >= R) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int oc = it.col0 + 16 * g + jl + 4 * i;
                if (oc < cols_task) {
                    T *xo = X + (x_off[task] + oc) * R + col;
                    *xo = ow ? (T)D[g][cb][i] : (T)((double)*xo + D[g][cb][i]);
                }
            }
        }
}

// Fused levels (the work stages in one launch): one workgroup of NW waves per
// (block, 16 right-hand sides).  The block's levels run in order; the ops of a
// level are spread over the waves (one wave per op, lanes as in k_ops_mfma)
// and accumulate straight into their rows of the level's LDS buffer, which
// the workgroup clears first (ops of a level write disjoint rows, so no two
// waves touch one row).  The next level reads those rows from LDS; the last
// level goes to the scratch rows the final stage reads.  GLOBAL: blocks whose
// levels exceed the LDS buffers keep their scratch rows in HBM; each wave then
// sums an op in its own 64-row LDS accumulator and writes the rows out.
template <typename T>
__device__ __forceinline__ void fused_op(const Op &op, const SubOp *__restrict__ subs, const int32_t *__restrict__ idx,
                                         const T *__restrict__ vals, const T *in, int64_t in_stride, const T *scrA,
                                         const T *scrB, int64_t scr_stride, const double *lds, int col, bool cok,
                                         double *acc) {
    const int lane = threadIdx.x & 63, jl = lane >> 4, cl = lane & 15;
    for (int s = 0; s < op.nsub; ++s) {
        const SubOp sb = subs[op.sub0 + s];
        const bool local = sb.src == kLds;
        const T *src = sb.src == kIn ? in : sb.src == kScrA ? scrA : scrB;
        const int64_t sstride = sb.src == kIn ? in_stride : scr_stride;
        const int nin = sb.n_in, nmap = sb.n_map;
        if (nmap > 0) {
            const int32_t *inr = idx + sb.in_off;
            int rows[16];
#pragma unroll
            for (int st = 0; st < 16; ++st) {
                const int j = 4 * st + jl;
                rows[st] = j < nin ? inr[j] : -1;
            }
            double B[16];
            if (local) {
#pragma unroll
                for (int st = 0; st < 16; ++st) B[st] = rows[st] >= 0 ? lds[rows[st] * 16 + cl] : 0.0;
            } else {
#pragma unroll
                for (int st = 0; st < 16; ++st)
                    B[st] = (rows[st] >= 0 && cok) ? (double)src[(int64_t)rows[st] * sstride + col] : 0.0;
            }
            const int32_t *map = idx + sb.map_off;
            const T *mv = vals + sb.mat_off;
            const int ntile = (nmap + 15) >> 4;
            for (int t = 0; t < ntile; ++t) {
                const int q = 16 * t + cl;
                const int aoff = jl * nmap + q;
                double A[16];
#pragma unroll
                for (int st = 0; st < 16; ++st) {
                    const T *mg = mv + (int64_t)(4 * st) * nmap;
                    A[st] = (q < nmap && 4 * st + jl < nin) ? (double)mg[aoff] : 0.0;
                }
                int dst[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int qq = 16 * t + jl + 4 * i;
                    dst[i] = qq < nmap ? map[qq] : -1;
                }
                d4v D = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int st = 0; st < 16; ++st) {
                    if (4 * st >= nin) break;
                    D = __builtin_amdgcn_mfma_f64_16x16x4f64(A[st], B[st], D, 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (dst[i] >= 0) acc[dst[i] * 16 + cl] += D[i];
            }
        }
        if (sb.n_dir > 0) {
            // the identity terms may land on rows the products just wrote
            // (other lanes of this wave): LDS accesses of one wave stay in order
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int32_t *dir = idx + sb.dir_off;
            for (int d0 = 0; d0 < sb.n_dir; d0 += 32) {
                int sr[8], dr[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int d = d0 + 4 * k + jl;
                    sr[k] = d < sb.n_dir ? dir[2 * d] : -1;
                    dr[k] = d < sb.n_dir ? dir[2 * d + 1] : -1;
                }
                double v[8];
                if (local) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) v[k] = sr[k] >= 0 ? lds[sr[k] * 16 + cl] : 0.0;
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        v[k] = (sr[k] >= 0 && cok) ? (double)src[(int64_t)sr[k] * sstride + col] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (dr[k] >= 0) acc[dr[k] * 16 + cl] += v[k];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <typename T, int NW, bool GLOBAL>
__global__ __launch_bounds__(64 * NW) void k_ops_fused(const FusedGroup *__restrict__ groups,
                                                        const int32_t *__restrict__ glist, int g0, int n_items, int ncb,
                                                        const FusedLevel *__restrict__ levels,
                                                        const Op *__restrict__ fops, const SubOp *__restrict__ fsubs,
                                                        const int32_t *__restrict__ idx, const T *__restrict__ vals,
                                                        const T *__restrict__ in, int64_t in_stride, T *scrA, T *scrB,
                                                        int64_t scr_stride, int rc) {
    extern __shared__ double fsm[];
    const int wi = xcd_item(n_items, kXc);
    if (wi >= n_items) return;
    const int gi = glist[g0 + wi / ncb], cb = wi % ncb;
    const FusedGroup g = groups[gi];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, cl = lane & 15, jl = lane >> 4;
    const int col = 16 * cb + cl;
    const bool cok = col < rc;
    const int lr = g.lds_rows;
    for (int l = 0; l < g.nlev; ++l) {
        const FusedLevel fl = levels[g.lvl_begin + l];
        if (!GLOBAL) {
            double *ob = fsm + (size_t)(l & 1) * lr * 16;
            for (int e = threadIdx.x; e < fl.rows * 16; e += 64 * NW) ob[e] = 0.0;
            __syncthreads();
        }
        for (int o = fl.op_begin + wave; o < fl.op_end; o += NW) {
            const Op op = fops[o];
            if (GLOBAL) {
                double *acc = fsm + (size_t)wave * 64 * 16;
                for (int e = lane; e < op.n_out * 16; e += 64) acc[e] = 0.0;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                fused_op<T>(op, fsubs, idx, vals, in, in_stride, scrA, scrB, scr_stride, fsm, col, cok, acc);
                T *dst = op.dst == kScrA ? scrA : scrB;
                if (cok)
                    for (int i = jl; i < op.n_out; i += 4) dst[(op.dst_row + i) * scr_stride + col] = (T)acc[i * 16 + cl];
            } else {
                fused_op<T>(op, fsubs, idx, vals, in, in_stride, scrA, scrB, scr_stride, fsm, col, cok,
                            fsm + (size_t)op.dst_row * 16);
            }
        }
        __syncthreads();
    }
    if (!GLOBAL) {
        const FusedLevel last = levels[g.lvl_begin + g.nlev - 1];
        const double *lb = fsm + (size_t)((g.nlev - 1) & 1) * lr * 16;
        T *dst = g.out_buf == kScrA ? scrA : scrB;
        for (int e = threadIdx.x; e < last.rows * 16; e += 64 * NW) {
            const int r = e >> 4, c = e & 15;
            if (16 * cb + c < rc) dst[(g.out_row + r) * scr_stride + 16 * cb + c] = (T)lb[e];
        }
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }


template <typename T>
hipError_t run_t(const DeviceProgram &p, int batch, int a_lo, int a_hi, int dir, const void *inp, void *outp,
                 hipStream_t s) {
    const int N = p.N, M = 4 * N - 1, R = 4 * batch;
    const int t_lo = 2 * a_lo, t_hi = 2 * a_hi + 1, nt = t_hi - t_lo + 1;
    const bool fwd = dir == 0;
    const DeviceProgramDir &pd = fwd ? p.fwd : p.adj;
    T *X = (T *)p.d_X, *Y = (T *)p.d_Y;
    T *scrA = (T *)p.d_scrA, *scrB = (T *)p.d_scrB;
    const int dt = sizeof(T) == 8 ? 0 : 1;
    hipError_t pe;
    if (fwd)
        pe = dev::panel_pack(dt, false, N, batch, a_lo, a_hi, p.d_x_off, p.max_task_cols, inp, X, s);
    else
        pe = dev::panel_fold(dt, false, N, batch, a_lo, a_hi, dir == 1 ? p.d_wh : nullptr, inp, Y, s);
    if (pe != hipSuccess) return pe;
    T *in = fwd ? X : Y;
    T *out = fwd ? Y : X;
    const T *vals = (const T *)pd.d_vals;
    const bool mfma = p.RCW > 0 && !p.bf16;
    const bool bf16 = sizeof(T) == 4 && p.bf16;
    const int RC = (mfma || bf16) ? p.RCW : p.RC;
    const bool fused = mfma && p.fused;
    for (int c0 = 0; c0 < R; c0 += RC) {
        const int rc = std::min(RC, R - c0);
        if (fused) {
            // every block's levels in one launch per size class
            prof::Scope ps(s, "k_ops_fused");
            const int ncb = (rc + 15) / 16;
            for (int c = 0; c < 3; ++c) {
                const std::vector<int32_t> &tf = pd.cls_task_first[c];
                const int gb = tf[t_lo], ge = tf[t_hi + 1];
                if (ge <= gb) continue;
                const int n_items = (ge - gb) * ncb;
                const int g0 = pd.cls_first[c] + gb;
#define SHT_FUSED_LAUNCH(NW, GL, LDSB)                                                                             \
    hipLaunchKernelGGL((k_ops_fused<T, NW, GL>), dim3(xcd_grid(n_items)), dim3(64 * NW), LDSB, s, pd.d_fgroups,      \
                       pd.d_glist, g0, n_items, ncb, pd.d_flevels, pd.d_fops, pd.d_fsubs, pd.d_idx, vals,            \
                       (const T *)(in + c0), (int64_t)R, scrA, scrB, (int64_t)RC, rc)
                if (c == 0)
                    SHT_FUSED_LAUNCH(4, false, 2 * kFusedRowsSmall * 16 * sizeof(double));
                else if (c == 1)
                    SHT_FUSED_LAUNCH(8, false, 2 * kFusedMaxRows * 16 * sizeof(double));
                else
                    SHT_FUSED_LAUNCH(4, true, 4 * 64 * 16 * sizeof(double));
#undef SHT_FUSED_LAUNCH
            }
        }
        for (size_t st = fused ? (size_t)pd.stages.size() - 1 : 0; st < pd.stage_task_first.size(); ++st) {
            const std::vector<int32_t> &tf = pd.stage_task_first[st];
            const int ob = tf[t_lo], oe = tf[t_hi + 1];
            if (oe <= ob) continue;
            const Stage &sg = pd.stages[st];
            const int mo = std::max(1, (int)sg.max_out), mi = std::max(4, ((int)sg.max_in + 3) & ~3);
            size_t lds = sizeof(T) * (size_t)(mo + mi) * RC;  // outputs + gathered inputs
            if (bf16)  // FP32 accumulators and the split BF16 inputs
                lds = 4 * (size_t)mo * RC + (p.bf16_terms == 3 ? 2 : 3) * 2 * (size_t)((mi + 15) & ~15) * RC;
            if (mfma) lds = (size_t)mo * 16 * 8;  // outputs x 16 columns
            if (lds > 160 * 1024) return hipErrorInvalidValue;
            const bool last = st + 1 == pd.stage_task_first.size();
            static const char *const kLab[3][9] = {
                {"k_ops[L0]", "k_ops[L1]", "k_ops[L2]", "k_ops[L3]", "k_ops[L4]", "k_ops[L5]", "k_ops[L6]",
                 "k_ops[L7+]", "k_ops[final]"},
                {"k_ops_mfma[L0]", "k_ops_mfma[L1]", "k_ops_mfma[L2]", "k_ops_mfma[L3]", "k_ops_mfma[L4]",
                 "k_ops_mfma[L5]", "k_ops_mfma[L6]", "k_ops_mfma[L7+]", "k_ops_mfma[final]"},
                {"k_ops_bf16[L0]", "k_ops_bf16[L1]", "k_ops_bf16[L2]", "k_ops_bf16[L3]", "k_ops_bf16[L4]",
                 "k_ops_bf16[L5]", "k_ops_bf16[L6]", "k_ops_bf16[L7+]", "k_ops_bf16[final]"}};
            prof::Scope ps(s, kLab[mfma ? 1 : bf16 ? 2 : 0][last ? 8 : std::min<size_t>(st, 7)]);
            if (bf16) {
                const float *vf = (const float *)vals;
                const float *inf = (const float *)(in + c0);
                float *outf = (float *)(out + c0);
#define SHT_BF16_LAUNCH(W, TM)                                                                                    \
    hipLaunchKernelGGL((k_ops_bf16<W, TM>), dim3(xcd_grid(oe - ob)), dim3(256), lds, s, pd.d_ops, pd.d_subs, pd.d_idx, vf, \
                       ob, oe - ob,                                                                                   \
                       inf, (int64_t)R, outf, (int64_t)R, (float *)scrA, (float *)scrB, rc, mo, mi)
                if (p.bf16_terms == 3) {
                    if (RC == 64)
                        SHT_BF16_LAUNCH(64, 3);
                    else if (RC == 32)
                        SHT_BF16_LAUNCH(32, 3);
                    else
                        SHT_BF16_LAUNCH(16, 3);
                } else {
                    if (RC == 64)
                        SHT_BF16_LAUNCH(64, 6);
                    else if (RC == 32)
                        SHT_BF16_LAUNCH(32, 6);
                    else
                        SHT_BF16_LAUNCH(16, 6);
                }
#undef SHT_BF16_LAUNCH
                continue;
            }
            if (mfma) {
                const int ncb = (rc + 15) / 16;
                const int n_items = (oe - ob) * ncb;
                hipLaunchKernelGGL(k_ops_mfma<T>, dim3(xcd_grid(n_items)), dim3(64), lds, s, pd.d_ops, pd.d_subs,
                                   pd.d_idx, vals, ob, n_items, ncb, (const T *)(in + c0), (int64_t)R, out + c0,
                                   (int64_t)R, scrA, scrB, (int64_t)RC, rc);
                continue;
            }
#define SHT_OPS_LAUNCH(RCV)                                                                                      \
    hipLaunchKernelGGL((k_ops<T, RCV>), dim3(xcd_grid(oe - ob)), dim3(64), lds, s, pd.d_ops, pd.d_subs, pd.d_idx, vals, \
                       ob, oe - ob,                                                                                  \
                       (const T *)(in + c0), (int64_t)R, out + c0, (int64_t)R, scrA, scrB, rc, mo, mi)
            if (RC == 4)
                SHT_OPS_LAUNCH(4);
            else if (RC == 8)
                SHT_OPS_LAUNCH(8);
            else
                SHT_OPS_LAUNCH(16);
#undef SHT_OPS_LAUNCH
        }
    }
    // regenerated blocks: on the FP64 matrix cores from 16 right-hand sides,
    // also in split-BF16 plans (their entries come from the FP64 recurrence,
    // so their products keep FP64 accuracy); on the VALU below
    const bool gen_mfma = p.RCW > 0 && R >= 16;
    if (fwd && p.gen.n_items > 0) {
        const int i0 = p.gen.task_first_h[t_lo], i1 = p.gen.task_first_h[t_hi + 1];
        if (i1 > i0) {
            prof::Scope ps(s, gen_mfma ? "k_gen_fwd_mfma" : "k_gen_fwd");
            const GenItem *gi = (const GenItem *)p.gen.d_items;
            const GenSeg *gs = (const GenSeg *)p.gen.d_segs;
            if (gen_mfma) {
                for (int c0 = 0; c0 < R; c0 += 32)
                    hipLaunchKernelGGL((k_gen_fwd_mfma<T, 2>), dim3(xcd_grid(i1 - i0)), dim3(64), 0, s, gi, i1 - i0,
                                       kXc, i0, gs, p.gen.d_ck, p.gen.d_ckexp, p.d_xh, p.d_coef2, N, p.d_x_off,
                                       (const T *)X, (int64_t)R, c0, Y);
            } else {
#define SHT_GEN_LAUNCH(RCV)                                                                                      \
    for (int c0 = 0; c0 < R; c0 += RCV)                                                                          \
        hipLaunchKernelGGL((k_gen_fwd<T, RCV>), dim3(xcd_grid(i1 - i0)), dim3(64), 0, s, gi, i1 - i0, i0, gs, p.gen.d_ck, \
                           p.gen.d_ckexp, \
                           p.d_xh, p.d_coef2, N, p.d_x_off, (const T *)X + c0, (int64_t)R, std::min(RCV, R - c0), \
                           Y + c0)
                if (p.RC == 4)
                    SHT_GEN_LAUNCH(4);
                else if (p.RC == 8)
                    SHT_GEN_LAUNCH(8);
                else
                    SHT_GEN_LAUNCH(16);
#undef SHT_GEN_LAUNCH
            }
            hipError_t ge = hipGetLastError();
            if (ge != hipSuccess) return ge;
        }
    }
    if (!fwd && p.gena.n_items > 0) {
        const int i0 = p.gena.task_first_h[t_lo], i1 = p.gena.task_first_h[t_hi + 1];
        if (i1 > i0) {
            prof::Scope ps(s, "k_gen_adj");
            const GenItemA *gi = (const GenItemA *)p.gena.d_items;
            const GenSegA *gs = (const GenSegA *)p.gena.d_segs;
            if (R <= 16)
                hipLaunchKernelGGL((k_gen_adj<T, 1>), dim3(xcd_grid(i1 - i0)), dim3(64), 0, s, gi, i1 - i0, kXc, i0, gs,
                                   p.gena.d_ck,
                                   p.gena.d_ckexp, p.d_xh, p.d_coef2, N, p.d_x_off, (const T *)Y, (int64_t)R, 0, X);
            else
                for (int c0 = 0; c0 < R; c0 += 32)
                    hipLaunchKernelGGL((k_gen_adj<T, 2>), dim3(xcd_grid(i1 - i0)), dim3(64), 0, s, gi, i1 - i0, kXc, i0, gs,
                                       p.gena.d_ck,
                                       p.gena.d_ckexp, p.d_xh, p.d_coef2, N, p.d_x_off, (const T *)Y, (int64_t)R,
                                       c0, X);
            hipError_t ge = hipGetLastError();
            if (ge != hipSuccess) return ge;
        }
    }
    if (fwd) return dev::panel_combine(dt, false, N, batch, a_lo, a_hi, Y, outp, s);
    return dev::panel_scatter(dt, false, N, batch, a_lo, a_hi, p.d_x_off, p.max_task_cols, X, outp, s);
}

}  // namespace

hipError_t set_kernel_attributes() {
    const void *fns[] = {(const void *)&k_ops<double, 4>,   (const void *)&k_ops<double, 8>,
                         (const void *)&k_ops<double, 16>,  (const void *)&k_ops<float, 4>,
                         (const void *)&k_ops<float, 8>,    (const void *)&k_ops<float, 16>,
                         (const void *)&k_ops_bf16<16, 3>,
                         (const void *)&k_ops_bf16<32, 3>,  (const void *)&k_ops_bf16<64, 3>,
                         (const void *)&k_ops_bf16<16, 6>,  (const void *)&k_ops_bf16<32, 6>,
                         (const void *)&k_ops_bf16<64, 6>,
                         (const void *)&k_ops_fused<double, 4, false>, (const void *)&k_ops_fused<double, 8, false>,
                         (const void *)&k_ops_fused<double, 4, true>,  (const void *)&k_ops_fused<float, 4, false>,
                         (const void *)&k_ops_fused<float, 8, false>,  (const void *)&k_ops_fused<float, 4, true>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t run_device(const DeviceProgram &p, int dtype, int batch, int a_lo, int a_hi, int dir, const void *in,
                      void *out, hipStream_t s) {
    if (dtype == 0) return run_t<double>(p, batch, a_lo, a_hi, dir, in, out, s);
    return run_t<float>(p, batch, a_lo, a_hi, dir, in, out, s);
}

}  // namespace idbf
}  // namespace sht
