// Persistent kernels of grouped transforms (see group.h).  Every workgroup
// loops: one lane takes the next item index from the phase's counter (a
// vector atomic in global memory), the index is shared through LDS, and the
// workgroup runs the same device bodies as the per-plan kernels for that
// item.  Items are ordered by decreasing cost, so the queue drains longest
// first and the tail is short.  Each item is computed by one workgroup from
// start to end, so results do not depend on the schedule.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dense_device.h"
#include "dft_device.h"
#include "group.h"
#include "prof.h"

namespace sht {
namespace group {

namespace {

using namespace dev::dense;

constexpr int kNpl = 2;  // nodes per lane in the forward ALT items

__global__ void k_group_reset(int *counters, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) counters[i] = 0;
}

__device__ __forceinline__ int next_item(int *counter, int *slot) {
    if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
    __syncthreads();
    const int it = *slot;
    __syncthreads();
    return it;
}

template <typename T>
__global__ __launch_bounds__(64) void k_group_fwd(const GTrans *__restrict__ tr, const GItem *__restrict__ items,
                                                  int nitems, int *counter) {
    __shared__ double lds[fwd_tile_lds(4)];
    __shared__ int slot;
    for (;;) {
        const int it = next_item(counter, &slot);
        if (it >= nitems) break;
        const GItem w = items[it];
        const GTrans &d = tr[w.t];
        const T *beta = (const T *)d.beta;
        T *f = (T *)d.f;
        switch (d.fields) {
            case 1: dense_fwd_tile<T, 1, kNpl>(d.N, d.M, 1, w.a, w.b, d.xh, d.dmant, d.dexp, d.coef, beta, f, lds); break;
            case 2: dense_fwd_tile<T, 2, kNpl>(d.N, d.M, 2, w.a, w.b, d.xh, d.dmant, d.dexp, d.coef, beta, f, lds); break;
            case 3: dense_fwd_tile<T, 3, kNpl>(d.N, d.M, 3, w.a, w.b, d.xh, d.dmant, d.dexp, d.coef, beta, f, lds); break;
            default: dense_fwd_tile<T, 4, kNpl>(d.N, d.M, d.fields, w.a, w.b, d.xh, d.dmant, d.dexp, d.coef, beta, f, lds); break;
        }
    }
}

// One field pair (or a last odd field) of one order: the recurrence is walked
// once for both fields of a pair.
template <typename T, int NR>
__device__ __forceinline__ void group_adj_order(const GTrans &d, int a, const T *g, T *beta, double *red) {
    int b0 = 0;
    for (; b0 + 2 <= d.fields; b0 += 2)
        dense_adj_order<T, 2, NR>(d.N, d.M, d.fields, b0, a, 4, d.xh, d.wh, d.dmant, d.dexp, d.coef, g, beta, red);
    if (b0 < d.fields)
        dense_adj_order<T, 1, NR>(d.N, d.M, d.fields, b0, a, 4, d.xh, d.wh, d.dmant, d.dexp, d.coef, g, beta, red);
}

// 4 waves; NR = 1, 2 or 4 nodes per lane, the fewest that cover N <= 1024
// nodes, so that every wave owns nodes from N = 256 up (below that, lanes past
// the last node form zero products).
template <typename T>
__global__ __launch_bounds__(256) void k_group_adj(const GTrans *__restrict__ tr, const GItem *__restrict__ items,
                                                   int nitems, int *counter) {
    __shared__ double red[4 * 64];
    __shared__ int slot;
    for (;;) {
        const int it = next_item(counter, &slot);
        if (it >= nitems) break;
        const GItem w = items[it];
        const GTrans &d = tr[w.t];
        const T *g = (const T *)d.g;
        T *beta = (T *)d.beta;
        if (d.N <= 256)
            group_adj_order<T, 1>(d, w.a, g, beta, red);
        else if (d.N <= 512)
            group_adj_order<T, 2>(d, w.a, g, beta, red);
        else
            group_adj_order<T, 4>(d, w.a, g, beta, red);
    }
}

// mode 0: synthesis in place on f; mode 1: analysis f -> g (scale 1/M)
template <typename C, typename T>
__global__ __launch_bounds__(512) void k_group_dft(const GTrans *__restrict__ tr, const GItem *__restrict__ items,
                                                   int nitems, int *counter, int mode) {
    extern __shared__ unsigned char smem_raw[];
    typename dev::dft::V2<C>::t *buf = reinterpret_cast<typename dev::dft::V2<C>::t *>(smem_raw);
    __shared__ int slot;
    __shared__ dev::dft::Passes ps;
    for (;;) {
        const int it = next_item(counter, &slot);
        if (it >= nitems) break;
        const GItem w = items[it];
        const GTrans &d = tr[w.t];
        if (threadIdx.x == 0) {
            ps.n = d.npass;
            for (int i = 0; i < kMaxPass; ++i) {
                ps.R[i] = d.R[i];
                ps.L[i] = d.L[i];
            }
        }
        __syncthreads();
        const int64_t base = 2 * ((int64_t)w.a * 2 * d.N * d.M + (int64_t)w.b * d.M);
        const double *tw = d.tab;
        if (mode == 0) {
            T *row = (T *)d.f + base;
            dev::dft::dft_row<C, T, 8>(d.N, d.M, ps, tw, d.src_pos, 0, (C)1, row, nullptr, row, nullptr, buf);
        } else {
            dev::dft::dft_row<C, T, 8>(d.N, d.M, ps, tw, d.src_pos, 1, (C)(1.0 / d.M), (const T *)d.f + base,
                                       nullptr, (T *)d.g + base, nullptr, buf);
        }
        __syncthreads();
    }
}

// segment copies of the batched mode: segment y copies segs[y].units 8-byte
// words from (to_stage ? ext : stage) to the other side
__global__ __launch_bounds__(256) void k_copy_segs(const CopySeg *__restrict__ segs, int to_stage) {
    const CopySeg sg = segs[blockIdx.y];
    const uint2 *src = (const uint2 *)(to_stage ? sg.ext : sg.stage);
    uint2 *dst = (uint2 *)(to_stage ? sg.stage : sg.ext);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < sg.units; i += 4 * stride) {
        const uint2 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < sg.units; i += stride) dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy_segs(const CopySeg *segs, int nseg, int64_t max_units, int to_stage, hipStream_t s) {
    if (nseg <= 0) return hipSuccess;
    prof::Scope ps(s, to_stage ? "k_copy_segs[gather]" : "k_copy_segs[scatter]");
    const int64_t blocks = std::min<int64_t>(1024, std::max<int64_t>(1, (max_units + 1023) / 1024));
    hipLaunchKernelGGL(k_copy_segs, dim3((unsigned)blocks, nseg), dim3(256), 0, s, segs, to_stage);
    return hipGetLastError();
}

int fwd_rows_per_tile() { return 64 * kNpl; }

hipError_t init_attributes() {
    for (const void *fn : {(const void *)&k_group_dft<double, double>, (const void *)&k_group_dft<float, float>}) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kGroupDftLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_reset(int *counters, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_group_reset, dim3((n + 63) / 64), dim3(64), 0, s, counters, n);
    return hipGetLastError();
}

hipError_t launch_phase(int phase, int dtype, int grid, const GTrans *tr, const GItem *items, int nitems,
                        int *counter, int max_M, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    switch (phase) {
        case kFwdAlt: {
            prof::Scope ps(s, "k_group_fwd");
            if (dtype == 0)
                hipLaunchKernelGGL(k_group_fwd<double>, dim3(grid), dim3(64), 0, s, tr, items, nitems, counter);
            else
                hipLaunchKernelGGL(k_group_fwd<float>, dim3(grid), dim3(64), 0, s, tr, items, nitems, counter);
            break;
        }
        case kAdjAlt: {
            prof::Scope ps(s, "k_group_adj");
            if (dtype == 0)
                hipLaunchKernelGGL(k_group_adj<double>, dim3(grid), dim3(256), 0, s, tr, items, nitems, counter);
            else
                hipLaunchKernelGGL(k_group_adj<float>, dim3(grid), dim3(256), 0, s, tr, items, nitems, counter);
            break;
        }
        default: {
            const int mode = phase == kDftSyn ? 0 : 1;
            prof::Scope ps(s, mode == 0 ? "k_group_dft_synthesis" : "k_group_dft_analysis");
            const size_t lds = (dtype == 0 ? 16 : 8) * ((size_t)max_M + 1) + 16 * (size_t)dev::dft::tab_entries(max_M);
            if (dtype == 0)
                hipLaunchKernelGGL((k_group_dft<double, double>), dim3(grid), dim3(512), lds, s, tr, items, nitems,
                                   counter, mode);
            else
                hipLaunchKernelGGL((k_group_dft<float, float>), dim3(grid), dim3(512), lds, s, tr, items, nitems,
                                   counter, mode);
        }
    }
    return hipGetLastError();
}

}  // namespace group
}  // namespace sht
