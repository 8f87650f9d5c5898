// FP32 instances of the 3D step-kernel launchers (see tpf3_launch.h).
#include "tpf3_launch_impl.h"

namespace tpf3 {
hipError_t launch3_f32(int ty, bool with_s, int mode, const Tile3Launch& a) { return launch3<float>(ty, with_s, mode, a); }
}  // namespace tpf3
