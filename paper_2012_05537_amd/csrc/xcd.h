// Block order for the XCDs of MI355X.  The hardware deals the workgroups of
// a launch round-robin to its 8 XCDs, each with its own L2; xcd_linear maps
// the hardware block index b (of nb) to a logical index so that every XCD
// receives one contiguous range of logical blocks, and blocks that share
// source lines (neighbouring tiles, the planes of one velocity) meet in one
// L2.
#pragma once

#include <hip/hip_runtime.h>

namespace sllbm {

__device__ __forceinline__ int xcd_linear(int b, int nb)
{
    const int xcd = b & 7, slot = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

}  // namespace sllbm
