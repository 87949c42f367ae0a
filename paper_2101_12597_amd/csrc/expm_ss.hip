// Scaling and squaring with the [9/9] Pade approximant for the complex generators
// (Sec. 3.4, Eq. ss).  The products (powers of X, U = X T, the squarings) are grouped
// complex GEMMs launched by the caller; this file holds the norm and scaling
// choice, the elementwise combinations of the powers and the denominator solve.
#include <algorithm>

#include "expm_ss.h"
#include "reduce.h"

namespace etdm {
namespace {

constexpr int TPB = 256;
constexpr int SOLVE_TPB = 1024;
constexpr int SOLVE_NB_MAX = 16;
constexpr int SOLVE_GROUPS = 8;  // workgroups per instance in the row updates (16 measured slower)

inline int blocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

// element (i, j) of the skew-Hermitian generator from the upper triangle of the
// parameters: a_ij (i < j), i Im a_jj on the diagonal, -conj(a_ji) below
__device__ __forceinline__ double2 generator_at(const double* __restrict__ A, int M, int i, int j) {
  if (i < j) return reinterpret_cast<const double2*>(A)[(size_t)i * M + j];
  const double2 a = reinterpret_cast<const double2*>(A)[(size_t)j * M + i];
  return i == j ? make_double2(0.0, a.y) : make_double2(-a.x, a.y);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// one workgroup per instance: the largest column sum of |A_ij|
__global__ __launch_bounds__(TPB) void norm1_kernel(const SsInst* __restrict__ si, double* norms) {
  const SsInst& z = si[blockIdx.x];
  const int M = z.M;
  double mx = 0.0;
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    double c = 0.0;
    for (int i = 0; i < M; ++i) {
      const double2 a = generator_at(z.A, M, i, j);
      c += sqrt(a.x * a.x + a.y * a.y);
    }
    mx = fmax(mx, c);
  }
  __shared__ double red[TPB];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) norms[blockIdx.x] = red[0];
}

// the fewest halvings that bring every instance's 1-norm under theta_9
__global__ void scaling_kernel(const double* norms, int n_inst, int* s_dev) {
  int s = 0;
  for (int i = 0; i < n_inst; ++i) {
    const double v = norms[i];
    if (!isfinite(v)) continue;  // non-finite input: caught by the energy and gradient scans
    while (s < SS_MAX_HALVINGS && ldexp(v, -s) > SS_THETA9) ++s;
  }
  *s_dev = s;
}

__global__ void build_kernel(const SsInst* __restrict__ si, const int* __restrict__ begin, int n, int total,
                             const int* s_dev) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsInst& z = si[ii];
  const int e = idx - begin[ii], i = e / z.M, j = e - i * z.M;
  const double sc = ldexp(1.0, -*s_dev);
  const double2 a = generator_at(z.A, z.M, i, j);
  reinterpret_cast<double2*>(z.X)[e] = make_double2(sc * a.x, sc * a.y);
}

__global__ void combine_odd_kernel(const SsInst* __restrict__ si, const int* __restrict__ begin, int n, int total,
                                   PadeB9 b) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsInst& z = si[ii];
  const int e = idx - begin[ii], i = e / z.M, j = e - i * z.M;
  const double2 x2 = reinterpret_cast<const double2*>(z.X2)[e];
  const double2 x4 = reinterpret_cast<const double2*>(z.X4)[e];
  const double2 x6 = reinterpret_cast<const double2*>(z.X6)[e];
  const double2 x8 = reinterpret_cast<const double2*>(z.X8)[e];
  reinterpret_cast<double2*>(z.T)[e] =
      make_double2(b.b[9] * x8.x + b.b[7] * x6.x + b.b[5] * x4.x + b.b[3] * x2.x + (i == j ? b.b[1] : 0.0),
                   b.b[9] * x8.y + b.b[7] * x6.y + b.b[5] * x4.y + b.b[3] * x2.y);
}

__global__ void combine_even_kernel(const SsInst* __restrict__ si, const int* __restrict__ begin, int n, int total,
                                    PadeB9 b) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsInst& z = si[ii];
  const int e = idx - begin[ii], i = e / z.M, j = e - i * z.M;
  const double2 x2 = reinterpret_cast<const double2*>(z.X2)[e];
  const double2 x4 = reinterpret_cast<const double2*>(z.X4)[e];
  const double2 x6 = reinterpret_cast<const double2*>(z.X6)[e];
  const double2 x8 = reinterpret_cast<const double2*>(z.X8)[e];
  const double2 u = reinterpret_cast<const double2*>(z.U)[e];
  const double vx = b.b[8] * x8.x + b.b[6] * x6.x + b.b[4] * x4.x + b.b[2] * x2.x + (i == j ? b.b[0] : 0.0);
  const double vy = b.b[8] * x8.y + b.b[6] * x6.y + b.b[4] * x4.y + b.b[2] * x2.y;
  reinterpret_cast<double2*>(z.Z)[e] = make_double2(vx - u.x, vy - u.y);
  reinterpret_cast<double2*>(z.R)[e] = make_double2(vx + u.x, vy + u.y);
}

__device__ __forceinline__ double2 cinv(double2 d) {
  const double dd = d.x * d.x + d.y * d.y;
  return make_double2(d.x / dd, -d.y / dd);
}

// Block Gauss-Jordan elimination on [Z | R] without pivoting (Z has a positive
// definite Hermitian part), one panel of nb rows k0..k0+nb at a time in two launches:
//   panel_kernel   (one workgroup per instance) the panel rows (columns k0.. of Z and
//                  all of R) are reduced to D^-1 (panel rows) in LDS and written back;
//   update_kernel  (SOLVE_GROUPS workgroups per instance, whole rows each) every other
//                  row i takes row_i -= Z[i, k0:k0+nb] (D^-1 panel rows), its multipliers
//                  read before the row is rewritten.
// [Z | R] is streamed once per panel, by the whole chip.
__global__ __launch_bounds__(SOLVE_TPB) void panel_kernel(const SsInst* __restrict__ si, int k0, int NB) {
  const SsInst& z = si[blockIdx.x];
  const int M = z.M;
  if (k0 >= M) return;
  double2* __restrict__ Q = reinterpret_cast<double2*>(z.Z);
  double2* __restrict__ R = reinterpret_cast<double2*>(z.R);
  extern __shared__ double2 sh[];
  const int nb = min(NB, M - k0);
  const int wq = M - k0, W = wq + M;
  double2* P = sh;              // panel rows, nb x W
  double2* fc = sh + nb * W;    // one column of the panel
  for (int t = threadIdx.x; t < nb * W; t += blockDim.x) {
    const int r = t / W, c = t - r * W;
    P[t] = c < wq ? Q[(size_t)(k0 + r) * M + k0 + c] : R[(size_t)(k0 + r) * M + (c - wq)];
  }
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    if ((int)threadIdx.x < nb) fc[threadIdx.x] = P[threadIdx.x * W + c];
    __syncthreads();
    const double2 inv = cinv(fc[c]);
    for (int t = threadIdx.x; t < W; t += blockDim.x) P[c * W + t] = cmul(P[c * W + t], inv);
    __syncthreads();
    for (int t = threadIdx.x; t < (nb - 1) * W; t += blockDim.x) {
      int r = t / W;
      const int col = t - r * W;
      r += r >= c;
      const double2 f = fc[r], q = P[c * W + col];
      P[r * W + col].x -= f.x * q.x - f.y * q.y;
      P[r * W + col].y -= f.x * q.y + f.y * q.x;
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < nb * W; t += blockDim.x) {
    const int r = t / W, c = t - r * W;
    if (c < wq) Q[(size_t)(k0 + r) * M + k0 + c] = P[t];
    else R[(size_t)(k0 + r) * M + (c - wq)] = P[t];
  }
}

__global__ __launch_bounds__(TPB) void update_kernel(const SsInst* __restrict__ si, int k0, int NB) {
  const int g = blockIdx.x % SOLVE_GROUPS;
  const SsInst& z = si[blockIdx.x / SOLVE_GROUPS];
  const int M = z.M;
  if (k0 >= M) return;
  double2* __restrict__ Q = reinterpret_cast<double2*>(z.Z);
  double2* __restrict__ R = reinterpret_cast<double2*>(z.R);
  extern __shared__ double2 sh[];
  const int nb = min(NB, M - k0);
  const int wq = M - k0, W = wq + M;
  // this workgroup's block of the M - nb rows outside the panel
  const int rows = M - nb, r0 = g * rows / SOLVE_GROUPS, r1 = (g + 1) * rows / SOLVE_GROUPS, nr = r1 - r0;
  if (nr <= 0) return;
  double2* P = sh;               // reduced panel rows, nb x W
  double2* F = sh + nb * W;      // multipliers of the block's rows, nr x nb
  for (int t = threadIdx.x; t < nb * W; t += blockDim.x) {
    const int r = t / W, c = t - r * W;
    P[t] = c < wq ? Q[(size_t)(k0 + r) * M + k0 + c] : R[(size_t)(k0 + r) * M + (c - wq)];
  }
  for (int t = threadIdx.x; t < nr * nb; t += blockDim.x) {
    const int r = t / nb, c = t - r * nb;
    const int i = r0 + r < k0 ? r0 + r : r0 + r + nb;
    F[t] = Q[(size_t)i * M + k0 + c];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nr * W; t += blockDim.x) {
    const int r = t / W, col = t - r * W;
    const int i = r0 + r < k0 ? r0 + r : r0 + r + nb;
    double2* dst = col < wq ? &Q[(size_t)i * M + k0 + col] : &R[(size_t)i * M + (col - wq)];
    if (col < nb) {
      *dst = make_double2(0.0, 0.0);
      continue;
    }
    double2 acc = *dst;
    const double2* f = F + r * nb;
    for (int u = 0; u < nb; ++u) {
      const double2 q = P[u * W + col];
      acc.x -= f[u].x * q.x - f[u].y * q.y;
      acc.y -= f[u].x * q.y + f[u].y * q.x;
    }
    *dst = acc;
  }
}

__global__ void deriv_scale_kernel(const SsDeriv* __restrict__ di, const int* __restrict__ begin, int n, int total,
                                   const int* s_dev) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsDeriv& z = di[ii];
  const int e = idx - begin[ii];
  const double sc = ldexp(1.0, -*s_dev);
  const double2 l = reinterpret_cast<const double2*>(z.L)[e];
  reinterpret_cast<double2*>(z.Es)[e] = make_double2(sc * l.x, sc * l.y);
}

__global__ void deriv_combine_kernel(const SsDeriv* __restrict__ di, const int* __restrict__ begin, int n,
                                     int total, PadeB9 b) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsDeriv& z = di[ii];
  const int e = idx - begin[ii];
  const double2 m2 = reinterpret_cast<const double2*>(z.M2)[e];
  const double2 m4 = reinterpret_cast<const double2*>(z.M4)[e];
  const double2 m6 = reinterpret_cast<const double2*>(z.M6)[e];
  const double2 m8 = reinterpret_cast<const double2*>(z.M8)[e];
  reinterpret_cast<double2*>(z.LT)[e] = make_double2(b.b[9] * m8.x + b.b[7] * m6.x + b.b[5] * m4.x + b.b[3] * m2.x,
                                                     b.b[9] * m8.y + b.b[7] * m6.y + b.b[5] * m4.y + b.b[3] * m2.y);
  reinterpret_cast<double2*>(z.LV)[e] = make_double2(b.b[8] * m8.x + b.b[6] * m6.x + b.b[4] * m4.x + b.b[2] * m2.x,
                                                     b.b[8] * m8.y + b.b[6] * m6.y + b.b[4] * m4.y + b.b[2] * m2.y);
}

__global__ void deriv_rhs_kernel(const SsDeriv* __restrict__ di, const double* const* __restrict__ lu,
                                 const int* __restrict__ begin, int n, int total) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsDeriv& z = di[ii];
  const int e = idx - begin[ii];
  const double2 u = reinterpret_cast<const double2*>(lu[ii])[e];
  const double2 v = reinterpret_cast<const double2*>(z.LV)[e];
  reinterpret_cast<double2*>(z.LT)[e] = make_double2(v.x - u.x, v.y - u.y);
  reinterpret_cast<double2*>(z.LV)[e] = make_double2(v.x + u.x, v.y + u.y);
}

__global__ void copy_kernel(const double* const* __restrict__ src, double* const* __restrict__ dst,
                            const int* __restrict__ begin, int n, int total) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const int e = idx - begin[ii];
  reinterpret_cast<double2*>(dst[ii])[e] = reinterpret_cast<const double2*>(src[ii])[e];
}

__global__ void copy_back_kernel(const SsInst* __restrict__ si, const int* __restrict__ begin, int n, int total) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsInst& z = si[ii];
  const int e = idx - begin[ii];
  reinterpret_cast<double2*>(z.R)[e] = reinterpret_cast<const double2*>(z.Sq)[e];
}

}  // namespace

void launch_ss_scaling(const SsInst* d, int n_inst, double* norms, int* s_dev, hipStream_t s) {
  if (n_inst <= 0) return;
  norm1_kernel<<<n_inst, TPB, 0, s>>>(d, norms);
  scaling_kernel<<<1, 1, 0, s>>>(norms, n_inst, s_dev);
}

void launch_ss_build(const SsInst* d, const int* d_begin, int n_inst, int total, const int* s_dev, hipStream_t s) {
  if (total > 0) build_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total, s_dev);
}

void launch_ss_combine_odd(const SsInst* d, const int* d_begin, int n_inst, int total, const PadeB9& b,
                           hipStream_t s) {
  if (total > 0) combine_odd_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total, b);
}

void launch_ss_combine_even(const SsInst* d, const int* d_begin, int n_inst, int total, const PadeB9& b,
                            hipStream_t s) {
  if (total > 0) combine_even_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total, b);
}

// LDS one workgroup may use: the device's limit, read once (64 KiB if it cannot be read)
static size_t solve_lds_limit() {
  static const size_t limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      return (size_t)65536;
    return (size_t)v;
  }();
  return limit;
}

int ss_solve_panel(int max_m) {
  // LDS: nb panel rows of up to 2M complex, and per panel row one multiplier of each of
  // the block's rows (at most M / SOLVE_GROUPS + 1) or one column value
  const size_t per_row = sizeof(double2) * (2 * (size_t)max_m + (size_t)max_m / SOLVE_GROUPS + 2);
  const int nb = (int)(solve_lds_limit() / per_row);
  return std::max(1, std::min(SOLVE_NB_MAX, nb));
}

void launch_ss_solve(const SsInst* d, int n_inst, int max_m, hipStream_t s) {
  if (n_inst <= 0 || max_m <= 0) return;
  const int nb = ss_solve_panel(max_m);
  const size_t lds = sizeof(double2) * ((size_t)nb * (2 * (size_t)max_m + (size_t)max_m / SOLVE_GROUPS + 2));
  if (lds > 65536) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(panel_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(update_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  for (int k0 = 0; k0 < max_m; k0 += nb) {
    panel_kernel<<<n_inst, SOLVE_TPB, lds, s>>>(d, k0, nb);
    update_kernel<<<n_inst * SOLVE_GROUPS, TPB, lds, s>>>(d, k0, nb);
  }
}

void launch_ss_deriv_scale(const SsDeriv* d, const int* d_begin, int n_inst, int total, const int* s_dev,
                           hipStream_t s) {
  if (total > 0) deriv_scale_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total, s_dev);
}

void launch_ss_deriv_combine(const SsDeriv* d, const int* d_begin, int n_inst, int total, const PadeB9& b,
                             hipStream_t s) {
  if (total > 0) deriv_combine_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total, b);
}

void launch_ss_deriv_rhs(const SsDeriv* d, const double* const* lu, const int* d_begin, int n_inst, int total,
                         hipStream_t s) {
  if (total > 0) deriv_rhs_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, lu, d_begin, n_inst, total);
}

void launch_ss_copy(const double* const* src, double* const* dst, const int* d_begin, int n_inst, int total,
                    hipStream_t s) {
  if (total > 0) copy_kernel<<<blocks(total, TPB), TPB, 0, s>>>(src, dst, d_begin, n_inst, total);
}

void launch_ss_copy_back(const SsInst* d, const int* d_begin, int n_inst, int total, hipStream_t s) {
  if (total > 0) copy_back_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total);
}

}  // namespace etdm
