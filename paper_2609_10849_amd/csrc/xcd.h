// Device helper shared by the kernel sources.
#pragma once
#include <hip/hip_runtime.h>

// Workgroups are handed to the 8 XCDs of the chip round-robin (workgroup b on XCD b % 8), and each
// XCD has its own L2.  xcd_block() renumbers the grid so that XCD x works through one contiguous
// range of blocks: element tiles that are neighbours in y (one mesh row apart) are then processed
// by the same XCD shortly after each other, and the face data they share hit in that XCD's L2.
// It is a bijection of [0, gridDim.x), so results never depend on the dispatch order.
__device__ __forceinline__ long xcd_block() {
  const long nb = gridDim.x, b = blockIdx.x;
  const long q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}
