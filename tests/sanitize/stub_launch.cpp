// Host-only stand-ins for the device launchers of the solver library, so that
// the host side of the C-ABI (argument and mesh validation, parameters,
// interpolation tables, reduction coefficients) can be built and run under
// AddressSanitizer / UndefinedBehaviorSanitizer without a GPU.  Every
// launcher reports that it cannot run; the block counts follow the same
// shapes as the library's (only their magnitude matters to the caller).
#include "../../paper_2509_01099_amd/csrc/islbm_launch.hpp"

namespace islbm {

int step_blocks(const DevState& s) { return (s.n[0] / 32 + 1) * (s.n[1] / 4 + 1) * (s.n[2] / 4 + 1); }
int reduce_state_blocks(const DevState&) { return 1024; }
hipError_t launch_step(const DevState&, const void*, const void*, void*, void*, bool, double*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_fill_zero(void*, size_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_copy16(void*, const void*, size_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_convert_in(const DevState&, const double*, void*, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_convert_out(const DevState&, const void*, double*, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_collide_only(const DevState&, const void*, const void*, void*, void*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_init_eq(const DevState&, const double*, const double*, const double*, const double*, void*, void*,
                          hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_fields(const DevState&, const void*, const void*, double*, double*, double*, double*, double*,
                         hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_reduce_state(const DevState&, const void*, const void*, double*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_finish(const double*, int, double*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_steady_change(const DevState&, const void*, const void*, double*, int, double*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace islbm
