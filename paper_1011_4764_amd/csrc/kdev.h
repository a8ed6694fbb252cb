// Device-side definitions shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>

namespace ofm {
namespace k {

constexpr int WG = 256;

// 4th-order central second-difference weights (times 1/h^2)
constexpr double W0 = -2.5, W1 = 4.0 / 3.0, W2 = -1.0 / 12.0;

typedef double d4 __attribute__((ext_vector_type(4)));

// Workgroup i is dispatched to XCD i % 8; remap so that each XCD receives a
// contiguous range of logical tiles (tiles of one fragment share V_j and
// their neighbours' planes in that XCD's L2).
__device__ __forceinline__ int xcd_tile(int bid, int nblk_pad) {
  const int per = nblk_pad >> 3;
  return (bid & 7) * per + (bid >> 3);
}
static inline int pad8(int n) { return (n + 7) / 8 * 8; }

}  // namespace k
}  // namespace ofm
