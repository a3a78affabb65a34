// Leaf keys of the forest: tree id in the high bits, then the Morton code of
// the anchor scaled to level kKeyLevel with x in the lowest bit, so that key
// order is "tree by tree, Morton order inside a tree" (block n = leaf n).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace f4 {

__host__ __device__ inline uint64_t leaf_key(int ndim, const int32_t nt[3], int32_t level,
                                             const int32_t g[3]) {
  constexpr int KL = 16;
  int32_t t[3] = {0, 0, 0};
  uint32_t a[3] = {0, 0, 0};
  for (int d = 0; d < ndim; d++) {
    t[d] = g[d] >> level;
    a[d] = (uint32_t)(g[d] - (t[d] << level)) << (KL - level);
  }
  const uint64_t tid = (uint64_t)t[0] + (uint64_t)nt[0] * ((uint64_t)t[1] + (uint64_t)nt[1] * (uint64_t)t[2]);
  uint64_t m = 0;
  for (int bit = 0; bit < KL; bit++)
    for (int d = 0; d < ndim; d++) m |= (uint64_t)((a[d] >> bit) & 1u) << (bit * ndim + d);
  return (tid << (ndim * KL)) | m;
}

}  // namespace f4
