// FP32 instances of the step-kernel launchers (see tpf_launch.h).
#include "tpf_launch_impl.h"

namespace tpf {
hipError_t launch_tiles_f32(int code, bool with_s, int mode, const TileLaunch& a) {
    return launch_tiles<float>(code, with_s, mode, a);
}
hipError_t launch_persistent_f32(int code, bool with_s, const PersistentLaunch& a) {
    return launch_persistent<float>(code, with_s, a);
}
bool persistent_code(int code) {
    return code == 8 || code == 9 || code == 10 || code == 17 || (code >= 20 && code <= 24);
}
}  // namespace tpf
