// Device helpers shared by the kernels of libstencil.so.
#pragma once

#include <hip/hip_runtime.h>

namespace stn {

// MI355X dispatches workgroup `lin` of a launch to XCD lin % 8 (round robin
// over the 8 XCDs, each with its own L2).  This maps the hardware order to a
// logical tile index such that every XCD receives one contiguous range of
// logical tiles, so tiles that share halo rows also share an L2.
__device__ __forceinline__ int xcd_remap(int lin, int n) {
    const int xcd = lin & 7, slot = lin >> 3;
    const int per = n >> 3, rem = n & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + slot;
}

}  // namespace stn
