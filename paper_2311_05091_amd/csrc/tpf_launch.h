// Launchers of the step kernels, instantiated per storage precision in their
// own translation units (tpf_launch_f32.hip, tpf_launch_f64.hip) so that the
// library builds in parallel.  Host-side only; called by tpf_api.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "tpf_device.h"

namespace tpf {

// One launch of the step (mode 0) or moments (mode 1) kernel over tiles
// [0, ntiles) of a tile table.
struct TileLaunch {
    hipStream_t stream;
    const DomDev* doms;
    const int4* tiles;
    int ntiles;
    int offset;    // step offset added to each domain's buffer parity
    double* mom;   // moments output (mode 1), else null
};

// One persistent launch: a.nsteps steps of every domain in the tile table,
// with residual checks when a.check_every > 0.
struct PersistentLaunch {
    hipStream_t stream;
    const DomDev* doms;
    PersistArgs a;
    int n_cu;
};

// hipErrorInvalidValue for an unknown tile code.
hipError_t launch_tiles_f32(int code, bool with_s, int mode, const TileLaunch& a);
hipError_t launch_tiles_f64(int code, bool with_s, int mode, const TileLaunch& a);
// Strip codes 8-10 and group codes 17, 20-24.
bool persistent_code(int code);
hipError_t launch_persistent_f32(int code, bool with_s, const PersistentLaunch& a);
hipError_t launch_persistent_f64(int code, bool with_s, const PersistentLaunch& a);

}  // namespace tpf
