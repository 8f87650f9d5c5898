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
// compute units), capped at twice the items of one step (more workgroups
// would only wait on later steps) and at the number of work items.
template <typename T, int CH, bool S, int NW, int NT, bool SHARE>
hipError_t launch_persistent_t(const PersistentLaunch& p) {
    auto k = persistent_kernel<T, CH, S, NW, NT, SHARE>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64 * NW, 0);
    if (e != hipSuccess) return e;
    if (per_cu <= 0) per_cu = 1;
    const int64_t per_step = p.a.ntiles + (p.a.check_every > 0 ? p.a.nlive : 0);
    const int64_t total = (int64_t)p.a.nsteps * per_step;
    const int64_t cap = std::min<int64_t>((int64_t)per_cu * p.n_cu, 2 * per_step);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cap, total));
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * NW), 0, p.stream, p.doms, p.a);
    return hipGetLastError();
}

template <typename T, bool S>
hipError_t launch_persistent_s(int code, const PersistentLaunch& p) {
    switch (code) {
        case 8: return launch_persistent_t<T, 16, S, 1, 0, false>(p);
        case 9: return launch_persistent_t<T, 32, S, 1, 0, false>(p);
        case 10: return launch_persistent_t<T, 64, S, 1, 0, false>(p);
        case 17:
        case 21: return launch_persistent_t<T, 32, S, 4, 0, true>(p);
        case 20: return launch_persistent_t<T, 16, S, 4, 0, true>(p);
        case 22: return launch_persistent_t<T, 64, S, 4, 0, true>(p);
        case 23: return launch_persistent_t<T, 64, S, 4, 3, false>(p);
        case 24: return launch_persistent_t<T, 64, S, 4, 1, true>(p);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_persistent(int code, bool with_s, const PersistentLaunch& p) {
    return with_s ? launch_persistent_s<T, true>(code, p) : launch_persistent_s<T, false>(code, p);
}

}  // namespace tpf
