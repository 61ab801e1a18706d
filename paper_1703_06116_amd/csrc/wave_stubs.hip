// Entry points of the one-wave-per-beam kernels for phase space m = 2d > 2.
#include "device.h"

namespace shgb {

bool step_wave_supported(int) { return false; }
hipError_t launch_step_wave(const DevModel &, const shgb_state &, int, double, uint64_t, uint64_t *, hipStream_t) {
  return hipErrorInvalidValue;
}
bool recon_wave_supported(int) { return false; }
int64_t recon_wave_workspace_bytes(int64_t, int, int64_t) { return 0; }
hipError_t launch_recon_wave(const DevModel &, const shgb_state &, const double *, int64_t, double *, void *,
                             hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace shgb
