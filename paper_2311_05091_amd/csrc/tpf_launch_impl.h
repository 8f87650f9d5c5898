// Template bodies of the launchers declared in tpf_launch.h (included by the
// per-precision translation units only).
#pragma once
#include <algorithm>

#include "tpf_kernels.h"
#include "tpf_launch.h"

namespace tpf {

template <typename T, int TX, int TY, bool S, int MODE>
hipError_t launch_step_t(const TileLaunch& a) {
    hipLaunchKernelGGL((step_kernel<T, TX, TY, 256, S, MODE>), dim3(a.ntiles), dim3(256), 0, a.stream, a.doms,
                       a.tiles, a.ntiles, a.offset, a.mom);
    return hipGetLastError();
}

template <typename T, int CH, bool S, int MODE>
hipError_t launch_strip_t(const TileLaunch& a) {
    hipLaunchKernelGGL((strip_kernel<T, CH, S, MODE>), dim3(a.ntiles), dim3(64), 0, a.stream, a.doms, a.tiles,
                       a.ntiles, a.offset, a.mom);
    return hipGetLastError();
}

template <typename T, int CH, bool S, int MODE, int NW, bool SHARE>
hipError_t launch_strip_group_t(const TileLaunch& a) {
    hipLaunchKernelGGL((strip_group_kernel<T, CH, S, MODE, NW, SHARE>), dim3(a.ntiles), dim3(64 * NW), 0, a.stream,
                       a.doms, a.tiles, a.ntiles, a.offset, a.mom);
    return hipGetLastError();
}

template <typename T, int CH, bool S, int MODE, int NW, int NT, bool SHARE>
hipError_t launch_strip_group_wide_t(const TileLaunch& a) {
    hipLaunchKernelGGL((strip_group_kernel_wide<T, CH, S, MODE, NW, NT, SHARE>), dim3(a.ntiles), dim3(64 * NW), 0, a.stream,
                       a.doms, a.tiles, a.ntiles, a.offset, a.mom);
    return hipGetLastError();
}

template <typename T, bool S, int MODE>
hipError_t launch_shape(int code, const TileLaunch& a) {
    switch (code) {
        case 17: return launch_strip_group_t<T, 32, S, MODE, 4, true>(a);
        case 18: return launch_strip_group_t<T, 32, S, MODE, 2, true>(a);
        case 20: return launch_strip_group_t<T, 16, S, MODE, 4, true>(a);
        case 21: return launch_strip_group_wide_t<T, 32, S, MODE, 4, 0, true>(a);
        case 22: return launch_strip_group_wide_t<T, 64, S, MODE, 4, 0, true>(a);
        case 23: return launch_strip_group_wide_t<T, 64, S, MODE, 4, 3, false>(a);
        case 24: return launch_strip_group_wide_t<T, 64, S, MODE, 4, 1, true>(a);
        case 8: return launch_strip_t<T, 16, S, MODE>(a);
        case 9: return launch_strip_t<T, 32, S, MODE>(a);
        case 10: return launch_strip_t<T, 64, S, MODE>(a);
        case 1: return launch_step_t<T, 64, 4, S, MODE>(a);
        case 2: return launch_step_t<T, 64, 8, S, MODE>(a);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_tiles(int code, bool with_s, int mode, const TileLaunch& a) {
    if (a.ntiles <= 0) return hipSuccess;
    if (mode == kModeStep)
        return with_s ? launch_shape<T, true, kModeStep>(code, a) : launch_shape<T, false, kModeStep>(code, a);
    return with_s ? launch_shape<T, true, kModeMoments>(code, a) : launch_shape<T, false, kModeMoments>(code, a);
}

// Persistent launch: a grid of the device's resident capacity (occupancy x
// compute units), capped at the number of work items.
template <typename T, int CH, bool S>
hipError_t launch_persistent_t(const PersistentLaunch& a) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_strip_kernel<T, CH, S>, 64, 0);
    if (e != hipSuccess) return e;
    if (per_cu <= 0) per_cu = 1;
    const int64_t total = (int64_t)a.nsteps * a.ntiles;
    const int grid = (int)std::min<int64_t>((int64_t)per_cu * a.n_cu, total);
    hipLaunchKernelGGL((persistent_strip_kernel<T, CH, S>), dim3(grid), dim3(64), 0, a.stream, a.doms, a.tiles,
                       a.ntiles, a.nsteps, a.dom_tiles, a.ctl, a.done, a.spin_limit);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_persistent(int code, bool with_s, const PersistentLaunch& a) {
    switch (code) {
        case 8: return with_s ? launch_persistent_t<T, 16, true>(a) : launch_persistent_t<T, 16, false>(a);
        case 9: return with_s ? launch_persistent_t<T, 32, true>(a) : launch_persistent_t<T, 32, false>(a);
        case 10: return with_s ? launch_persistent_t<T, 64, true>(a) : launch_persistent_t<T, 64, false>(a);
    }
    return hipErrorInvalidValue;
}

}  // namespace tpf
