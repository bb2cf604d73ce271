// Packed fast-ALT plan: value stream + forward and transposed op programs.
#pragma once

#include <cstdint>
#include <vector>

#include "idbf_build.h"
#include "idbf_program.h"

namespace sht {
namespace idbf {

struct PackedPlan {
    Program fwd, adj;  // each with its own output-major value stream
    std::vector<int64_t> x_off, y_off;  // panel row offsets per task (+ total)
};

void pack_programs(const HostPlanData &hp, PackedPlan &pk);

}  // namespace idbf
}  // namespace sht
