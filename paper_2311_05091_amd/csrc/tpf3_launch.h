// Launchers of the 3D step kernel, instantiated per storage precision in
// their own translation units (tpf3_launch_f32.hip, tpf3_launch_f64.hip).
// Host-side only; called by tpf3_api.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "tpf3_device.h"

namespace tpf3 {

struct Tile3Launch {
    hipStream_t stream;
    const DomDev3* doms;
    const int4* tiles;   // (domain, x0, y0, z0)
    int ntiles;
    int offset;          // step offset added to each domain's buffer parity
    double* mom;         // moments output (mode 1), else null
};

constexpr int kTileZ3 = 32;   // planes per tile

// hipErrorInvalidValue for a (ty, with_s) pair without an instance.
hipError_t launch3_f32(int ty, bool with_s, int mode, const Tile3Launch& a);
hipError_t launch3_f64(int ty, bool with_s, int mode, const Tile3Launch& a);

}  // namespace tpf3
