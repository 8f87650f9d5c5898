// FP64 instances of the 3D step-kernel launchers (see tpf3_launch.h).
#include "tpf3_launch_impl.h"

namespace tpf3 {
hipError_t launch3_f64(int ty, bool with_s, int mode, const Tile3Launch& a) { return launch3<double>(ty, with_s, mode, a); }
}  // namespace tpf3
