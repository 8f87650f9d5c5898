// Template body of the 3D launchers (included by the per-precision units).
#pragma once
#include "tpf3_kernels.h"
#include "tpf3_launch.h"

namespace tpf3 {

template <typename T, int TY, bool S, int MODE>
hipError_t launch3_t(const Tile3Launch& a) {
    hipLaunchKernelGGL((step3_kernel<T, TY, kTileZ3, S, MODE>), dim3(a.ntiles), dim3(64 * TY), 0, a.stream, a.doms,
                       a.tiles, a.ntiles, a.offset, a.mom);
    return hipGetLastError();
}

// LDS of a workgroup is limited to 64 KB: FP32 holds 64 x 8 tiles without the
// flux S and 64 x 4 with it; FP64 64 x 4 without and 64 x 2 with.
template <typename T, int MODE>
hipError_t launch3_mode(int ty, bool with_s, const Tile3Launch& a) {
    if (a.ntiles <= 0) return hipSuccess;
    if constexpr (sizeof(T) == 4) {
        if (ty == 8 && !with_s) return launch3_t<T, 8, false, MODE>(a);
        if (ty == 4) return with_s ? launch3_t<T, 4, true, MODE>(a) : launch3_t<T, 4, false, MODE>(a);
    } else {
        if (ty == 4 && !with_s) return launch3_t<T, 4, false, MODE>(a);
        if (ty == 2) return with_s ? launch3_t<T, 2, true, MODE>(a) : launch3_t<T, 2, false, MODE>(a);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch3(int ty, bool with_s, int mode, const Tile3Launch& a) {
    return mode == 0 ? launch3_mode<T, 0>(ty, with_s, a) : launch3_mode<T, 1>(ty, with_s, a);
}

}  // namespace tpf3
