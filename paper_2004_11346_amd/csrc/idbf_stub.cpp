#include "idbf.h"

namespace sht {
namespace idbf {

int build_program(int, const LegendreTables &, const sht_plan_opts &, HostProgram &) {
    set_error_detail("IDBF method not built yet");
    return SHT_ERR_UNSUPPORTED;
}
int upload_program(const HostProgram &, int, int, const sht_plan_opts &, DeviceProgram &) {
    return SHT_ERR_UNSUPPORTED;
}
hipError_t run(const DeviceProgram &, const dev::DenseTables &, int, int, int, int, int, const void *,
               void *, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace idbf
}  // namespace sht
