// XCD-aware work-group numbering for kernels whose neighbouring work-groups read each other's
// data.  gfx950 dispatches the work-groups of a grid to its 8 XCDs in turn (linear work-group id
// b to XCD b mod 8) and each XCD has its own L2; renumbering the grid so that every XCD takes one
// contiguous range of ids lets such neighbours share an L2.  Device code only.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace sfm {

// The work-group's id in XCD-contiguous order: a bijection of [0, total) for linear ids
// b in [0, total) (x fastest in a multi-dimensional grid).
__device__ __forceinline__ int64_t xcd_contiguous_id(int64_t b, int64_t total) {
  constexpr int kXcds = 8;
  const int64_t q = total / kXcds, r = total % kXcds, x = b % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}

}  // namespace sfm
