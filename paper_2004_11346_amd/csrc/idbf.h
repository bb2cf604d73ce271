// Fast form of the ALT: hierarchical block partitioning (Section 3.2) with an
// interpolative decomposition butterfly factorization (IDBF, Section 2.2) of
// every oscillatory block, a randomized-sampling low-rank factorization
// (Section 2.3, Algorithm 1) of every non-oscillatory block and a trimmed
// dense product for every block that contains turning points (Section 3.3).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "idbf_build.h"
#include "idbf_device.h"
#include "idbf_pack.h"
#include "kernels.h"
#include "sht.h"
#include "sht_internal.h"

namespace sht {
namespace idbf {

struct HostProgram {
    int N = 0;
    int f32_mode = 0;  // SHT_F32_VALU or SHT_F32_SPLIT_BF16
    int level_schedule = 0;  // SHT_LEVELS_*
    PackedPlan packed;
    BuildStats stats;
    std::string stats_json;
};

int build_program(int N, int batch, const LegendreTables &lt, const sht_plan_opts &opts, HostProgram &out);
int upload_program(HostProgram &hp, int dtype, int batch, const double *d_wh, const double *d_xh,
                   const double *d_coef2, DeviceProgram &out);
hipError_t run(const DeviceProgram &prog, const dev::DenseTables &t, int dtype, int batch, int a_lo, int a_hi,
               int dir, const void *in, void *out, hipStream_t s);

}  // namespace idbf
}  // namespace sht
