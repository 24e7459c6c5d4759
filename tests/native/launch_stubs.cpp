// Host-only stand-ins for the kernel launchers, so that the planner
// (aln_api.cpp) links without device code for the sanitizer build of its
// host logic.  Contexts without a device never launch; every stub reports
// an error if called.
#include "internal.h"
#include "runtime.h"

namespace alnk {
hipError_t launch_validate(const ValidateArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_strip(int, int, bool, bool, const StripArgs &, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_band_strip(int, int, bool, bool, const StripArgs &, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_walk(int, const WalkArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_sw16(int, const Sw16Args &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_diag(int, int, int, bool, const DiagArgs &, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_xdrop_group(int, const DiagArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_walk_diag(const WalkArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_xdrop_lanes(bool, const XdlArgs &, int, hipStream_t) {
  return hipErrorNotSupported;
}
int xdrop_lanes_waves_per_cu(bool) { return 12; }
size_t xdrop_lanes_lds_bytes() { return 0; }
hipError_t launch_search(const SearchArgs &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fold(int, int, int, const FoldArgs &, hipStream_t) {
  return hipErrorNotSupported;
}
} // namespace alnk

aln_status alnrt::scratch_init(aln_ctx *) { return ALN_E_DEVICE; }
