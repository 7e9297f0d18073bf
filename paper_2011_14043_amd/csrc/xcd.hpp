// xcd.hpp -- XCD-aware block order.
#pragma once
#include <hip/hip_runtime.h>

namespace fdtd {

// Blocks are dispatched round-robin over the 8 XCDs (block L -> XCD L % 8),
// each with its own L2.  With remap, XCD c receives a contiguous range of
// work items, so spatially adjacent tiles (which share 128-byte lines and
// neighbour rows) run on the same XCD at about the same time.
__device__ __forceinline__ int xcd_remap(int L, int G) {
    const int c = L & 7, q = L >> 3;
    const int per = G >> 3, rem = G & 7;
    return c * per + (c < rem ? c : rem) + q;
}

}  // namespace fdtd
