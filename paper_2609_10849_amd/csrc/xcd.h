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

// Run-table launches: one launch covers several independent runs, whose blocks are consecutive
// ranges; boff[r] is the first block of run r and boff[nr] the grid size.  Returns the run of the
// calling block (the same for all its threads) by bisection.
__device__ __forceinline__ int rt_run(const int* __restrict__ boff, int nr) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = nr;  // boff[lo] <= b < boff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (boff[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}
