// Work-group order for the 8 XCDs of gfx950. The dispatcher hands work-group i to XCD
// i mod 8; each XCD has its own L2. Remapping the linear index so that every XCD gets one
// contiguous range of logical work items keeps neighbouring items (which share input
// rows or halo columns) in the same L2.
#pragma once

#include <hip/hip_runtime.h>

namespace aa {

// logical item of work-group `bid` out of `n`: XCD x gets items [x q + min(x, r), ...)
__device__ __forceinline__ int xcd_remap(int bid, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = bid & 7, k = bid >> 3;
    return x * q + min(x, r) + k;
}

}  // namespace aa
