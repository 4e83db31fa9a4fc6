// device_common.h -- small device helpers shared by the kernel files.
#pragma once

#include "mpx_internal.h"

namespace mpx {

// index along an axis of extent n: wrapped once on a periodic axis; -1 when
// outside the domain (or still outside after one wrap)
__device__ __forceinline__ int fold(int i, int n, int per) {
    if (per) {
        if (i < 0)
            i += n;
        else if (i >= n)
            i -= n;
    }
    return (i < 0 || i >= n) ? -1 : i;
}

// central difference over a spacing: a true division in float64 (the plain
// definition), a multiply by the reciprocal in float32
template <typename T>
__device__ __forceinline__ T dif(T hi, T lo, T d, T invd) {
    if constexpr (sizeof(T) == 8) {
        (void)invd;
        return (hi - lo) / d;
    } else {
        (void)d;
        return (hi - lo) * invd;
    }
}

} // namespace mpx
