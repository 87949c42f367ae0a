// Device helpers shared by the batched kernels: the owner lookup of a flat
// element in a batch of instances, and compensated (Neumaier) summation for the
// FP64 reductions (a running sum and its correction term, combined across a
// wavefront by butterfly shuffles and across the waves of a workgroup in a fixed
// order, so a reduction gives the same bits on every run).
#pragma once

#include <hip/hip_runtime.h>

namespace etdm {

// Instance that owns flat element idx of a batch laid out back to back:
// begin[] holds the ascending first element of each of the n instances.
__device__ __forceinline__ int instance_of(const int* __restrict__ begin, int n, int idx) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= idx) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
  double t = s + x;
  c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
  s = t;
}

__device__ inline double block_sum_neumaier(double s, double c, double* red) {
  for (int o = 32; o > 0; o >>= 1) {
    double s2 = __shfl_xor(s, o), c2 = __shfl_xor(c, o);
    double t = s + s2;
    c += c2 + ((fabs(s) >= fabs(s2)) ? (s - t) + s2 : (s2 - t) + s);
    s = t;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    red[2 * wave] = s;
    red[2 * wave + 1] = c;
  }
  __syncthreads();
  double S = 0.0, Cc = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    double x = red[2 * w], t = S + x;
    Cc += ((fabs(S) >= fabs(x)) ? (S - t) + x : (x - t) + S) + red[2 * w + 1];
    S = t;
  }
  return S + Cc;
}

// Workgroups are handed to the 8 XCDs in turn (workgroup b runs on XCD b mod 8). This
// maps them to tiles so that each XCD takes one contiguous range of the tile list: the
// tiles of one problem, which share its A rows and B columns, then meet in one L2.
__device__ __forceinline__ int xcd_tile(int b, int total) {
  constexpr int XCDS = 8;
  const int x = b % XCDS, q = b / XCDS, base = total / XCDS, rem = total % XCDS;
  return x * base + min(x, rem) + q;
}

}  // namespace etdm
