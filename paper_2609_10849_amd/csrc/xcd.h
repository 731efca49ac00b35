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
// calling block (the same for all its threads) by bisection.  The result is declared wave-uniform
// (readfirstlane), so that the run's argument struct is fetched with scalar loads into scalar
// registers; otherwise its pointers and constants occupy vector registers in every lane (the OE/PP
// map went from 95 to 177 VGPRs, 5 to 2 waves per SIMD).
__device__ __forceinline__ int rt_run(const int* __restrict__ boff, int nr) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = nr;  // boff[lo] <= b < boff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (boff[mid] <= b) lo = mid;
    else hi = mid;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// Run-table argument structs hold their array pointers as plain (generic) pointers.  Read through
// gl() they are loaded as global-memory pointers, so that a kernel body inlined into a run-table
// kernel addresses its arrays with global rather than flat memory instructions, as it does with
// kernel arguments (with flat ones the OE/PP map needed 192 VGPRs instead of 107: 2 waves per
// SIMD instead of 4).  Fields that are not pointers pass through unchanged.
#ifndef MHD_GLOBAL_AS
#define MHD_GLOBAL_AS __attribute__((address_space(1)))
#endif
template <class T>
__device__ __forceinline__ T* gl(T* const& field) {
  typedef MHD_GLOBAL_AS T* gptr;
  return (T*)(*reinterpret_cast<const gptr*>(&field));
}
template <class T>
__device__ __forceinline__ const T& gl(const T& field) {
  return field;
}
