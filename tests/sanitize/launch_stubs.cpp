// Stand-ins for the per-precision kernel launchers (test infrastructure): the
// host-sanitizer build of the library's host code links these instead of the
// step kernels, which it never launches (there is no device).
#include "tpf3_launch.h"
#include "tpf_launch.h"

namespace tpf {
hipError_t launch_tiles_f32(int, bool, int, const TileLaunch&) { return hipErrorInvalidValue; }
hipError_t launch_tiles_f64(int, bool, int, const TileLaunch&) { return hipErrorInvalidValue; }
hipError_t launch_persistent_f32(int, bool, const PersistentLaunch&) { return hipErrorInvalidValue; }
hipError_t launch_persistent_f64(int, bool, const PersistentLaunch&) { return hipErrorInvalidValue; }
bool persistent_code(int) { return false; }
}  // namespace tpf

namespace tpf3 {
hipError_t launch3_f32(int, bool, int, const Tile3Launch&) { return hipErrorInvalidValue; }
hipError_t launch3_f64(int, bool, int, const Tile3Launch&) { return hipErrorInvalidValue; }
}  // namespace tpf3
