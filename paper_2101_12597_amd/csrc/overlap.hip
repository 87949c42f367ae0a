// Lowdin factors S^1/2, S^-1/2 of the overlap of a non-orthogonal basis by the
// coupled Newton-Schulz iteration (the products are launched by the caller).
#include <algorithm>

#include "overlap.h"
#include "reduce.h"

namespace etdm {
namespace {

constexpr int TPB = 256;

inline int blocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

__device__ double block_max(double v) {
  __shared__ double red[TPB];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  return red[0];
}

// one workgroup per instance: c = max_i sum_j |S_ij|
__global__ __launch_bounds__(TPB) void scale_kernel(const OvlInst* __restrict__ oi, int cplx) {
  const OvlInst& z = oi[blockIdx.x];
  const int M = z.M;
  double mx = 0.0;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    double r = 0.0;
    for (int j = 0; j < M; ++j) {
      if (cplx) {
        const double2 v = reinterpret_cast<const double2*>(z.S)[(size_t)i * M + j];
        r += sqrt(v.x * v.x + v.y * v.y);
      } else {
        r += fabs(z.S[(size_t)i * M + j]);
      }
    }
    mx = fmax(mx, r);
  }
  const double c = block_max(mx);
  if (threadIdx.x == 0) *z.c = c;
}

__global__ void start_kernel(const OvlInst* __restrict__ oi, const int* __restrict__ begin, int n, int total,
                             int cplx) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const OvlInst& z = oi[ii];
  const int e = idx - begin[ii], i = e / z.M, j = e - i * z.M;
  const double inv = 1.0 / *z.c;
  if (cplx) {
    const double2 v = reinterpret_cast<const double2*>(z.S)[e];
    reinterpret_cast<double2*>(z.Y)[e] = make_double2(v.x * inv, v.y * inv);
    reinterpret_cast<double2*>(z.Z)[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  } else {
    z.Y[e] = z.S[e] * inv;
    z.Z[e] = i == j ? 1.0 : 0.0;
  }
}

// one workgroup per instance: T = (3 I - P) / 2 and max |I - P|
__global__ __launch_bounds__(TPB) void step_kernel(const OvlInst* __restrict__ oi, int cplx, double* resid) {
  const OvlInst& z = oi[blockIdx.x];
  const int M = z.M;
  const int64_t MM = (int64_t)M * M;
  double mx = 0.0;
  for (int64_t e = threadIdx.x; e < MM; e += blockDim.x) {
    const int i = (int)(e / M), j = (int)(e - (int64_t)i * M);
    const double d = i == j ? 1.0 : 0.0;
    if (cplx) {
      const double2 p = reinterpret_cast<const double2*>(z.P)[e];
      reinterpret_cast<double2*>(z.T)[e] = make_double2(0.5 * (3.0 * d - p.x), -0.5 * p.y);
      mx = fmax(mx, fmax(fabs(d - p.x), fabs(p.y)));
    } else {
      const double p = z.P[e];
      z.T[e] = 0.5 * (3.0 * d - p);
      mx = fmax(mx, fabs(d - p));
    }
  }
  const double r = block_max(mx);
  if (threadIdx.x == 0) resid[blockIdx.x] = r;
}

__global__ void finish_kernel(const OvlInst* __restrict__ oi, const int* __restrict__ begin, int n, int total,
                              int cplx) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const OvlInst& z = oi[ii];
  const int e = idx - begin[ii];
  const double sc = sqrt(*z.c);
  if (cplx) {
    double2& y = reinterpret_cast<double2*>(z.Y)[e];
    double2& w = reinterpret_cast<double2*>(z.Z)[e];
    y = make_double2(y.x * sc, y.y * sc);
    w = make_double2(w.x / sc, w.y / sc);
  } else {
    z.Y[e] *= sc;
    z.Z[e] /= sc;
  }
}

}  // namespace

void launch_ovl_start(const OvlInst* d, const int* d_begin, int n_inst, int total, int cplx, hipStream_t s) {
  if (n_inst <= 0) return;
  scale_kernel<<<n_inst, TPB, 0, s>>>(d, cplx);
  if (total > 0) start_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total, cplx);
}

void launch_ovl_step(const OvlInst* d, int n_inst, int cplx, double* resid, hipStream_t s) {
  if (n_inst > 0) step_kernel<<<n_inst, TPB, 0, s>>>(d, cplx, resid);
}

void launch_ovl_finish(const OvlInst* d, const int* d_begin, int n_inst, int total, int cplx, hipStream_t s) {
  if (total > 0) finish_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total, cplx);
}

}  // namespace etdm
