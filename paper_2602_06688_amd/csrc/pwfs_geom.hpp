// pwfs_geom.hpp -- pupil-image window coordinates shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace pwfs {

// compact index of plane coordinate X in window mode, -1 if outside the two
// windows [lo, lo + D) and [hi, hi + D)
__device__ __forceinline__ int window_index(int X, int D, int lo, int hi) {
  if (X >= lo && X < lo + D) return X - lo;
  if (X >= hi && X < hi + D) return X - hi + D;
  return -1;
}
// plane coordinate of compact window index xc
__device__ __forceinline__ int window_coord(int xc, int D, int lo, int hi) {
  return xc < D ? lo + xc : hi + xc - D;
}

}  // namespace pwfs
