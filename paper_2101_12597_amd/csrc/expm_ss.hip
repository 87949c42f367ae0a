// Scaling and squaring with the [13/13] Pade approximant for the complex generators
// (Sec. 3.4, Eq. ss).  The products (powers of X, the three products of the
// numerator's evaluation, the squarings) are grouped complex GEMMs launched by the
// caller; this file holds the norm and scaling choice, the elementwise
// combinations of the powers and the denominator solve.
#include <algorithm>

#include "expm_ss.h"

namespace etdm {
namespace {

constexpr int TPB = 256;
constexpr int SOLVE_TPB = 1024;

inline int blocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

__device__ __forceinline__ int instance_of(const int* __restrict__ begin, int n, int idx) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= idx) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

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

// the fewest halvings that bring every instance's 1-norm under theta_13
__global__ void scaling_kernel(const double* norms, int n_inst, int* s_dev) {
  int s = 0;
  for (int i = 0; i < n_inst; ++i) {
    const double v = norms[i];
    if (!isfinite(v)) continue;  // non-finite input: caught by the energy and gradient scans
    while (s < SS_MAX_HALVINGS && ldexp(v, -s) > SS_THETA13) ++s;
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

__global__ void combine_high_kernel(const SsInst* __restrict__ si, const int* __restrict__ begin, int n, int total,
                                    PadeB13 b) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsInst& z = si[ii];
  const int e = idx - begin[ii];
  const double2 x2 = reinterpret_cast<const double2*>(z.X2)[e];
  const double2 x4 = reinterpret_cast<const double2*>(z.X4)[e];
  const double2 x6 = reinterpret_cast<const double2*>(z.X6)[e];
  reinterpret_cast<double2*>(z.W)[e] = make_double2(b.b[13] * x6.x + b.b[11] * x4.x + b.b[9] * x2.x,
                                                    b.b[13] * x6.y + b.b[11] * x4.y + b.b[9] * x2.y);
  reinterpret_cast<double2*>(z.Z)[e] = make_double2(b.b[12] * x6.x + b.b[10] * x4.x + b.b[8] * x2.x,
                                                    b.b[12] * x6.y + b.b[10] * x4.y + b.b[8] * x2.y);
}

__global__ void combine_odd_kernel(const SsInst* __restrict__ si, const int* __restrict__ begin, int n, int total,
                                   PadeB13 b) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsInst& z = si[ii];
  const int e = idx - begin[ii], i = e / z.M, j = e - i * z.M;
  const double2 x2 = reinterpret_cast<const double2*>(z.X2)[e];
  const double2 x4 = reinterpret_cast<const double2*>(z.X4)[e];
  const double2 x6 = reinterpret_cast<const double2*>(z.X6)[e];
  double2& t = reinterpret_cast<double2*>(z.T)[e];
  t.x += b.b[7] * x6.x + b.b[5] * x4.x + b.b[3] * x2.x + (i == j ? b.b[1] : 0.0);
  t.y += b.b[7] * x6.y + b.b[5] * x4.y + b.b[3] * x2.y;
}

__global__ void combine_even_kernel(const SsInst* __restrict__ si, const int* __restrict__ begin, int n, int total,
                                    PadeB13 b) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsInst& z = si[ii];
  const int e = idx - begin[ii], i = e / z.M, j = e - i * z.M;
  const double2 x2 = reinterpret_cast<const double2*>(z.X2)[e];
  const double2 x4 = reinterpret_cast<const double2*>(z.X4)[e];
  const double2 x6 = reinterpret_cast<const double2*>(z.X6)[e];
  const double2 v = reinterpret_cast<const double2*>(z.V)[e];
  const double2 u = reinterpret_cast<const double2*>(z.W)[e];
  const double vx = v.x + b.b[6] * x6.x + b.b[4] * x4.x + b.b[2] * x2.x + (i == j ? b.b[0] : 0.0);
  const double vy = v.y + b.b[6] * x6.y + b.b[4] * x4.y + b.b[2] * x2.y;
  reinterpret_cast<double2*>(z.Z)[e] = make_double2(vx - u.x, vy - u.y);
  reinterpret_cast<double2*>(z.R)[e] = make_double2(vx + u.x, vy + u.y);
}

// Gauss-Jordan elimination on [Z | R] with row pivoting on the largest |Z_ik|
// (ties: the lowest row).  Rows stay in global memory (L2-resident for the sizes
// of one workgroup's matrix); the pivot rows and the multipliers of a step are
// staged in LDS.
__global__ __launch_bounds__(SOLVE_TPB) void solve_kernel(const SsInst* __restrict__ si) {
  const SsInst& z = si[blockIdx.x];
  const int M = z.M;
  double2* __restrict__ Q = reinterpret_cast<double2*>(z.Z);
  double2* __restrict__ R = reinterpret_cast<double2*>(z.R);
  extern __shared__ double2 sh[];
  double2* prQ = sh;          // scaled pivot row of Q
  double2* prR = sh + M;      // scaled pivot row of R
  double2* mult = sh + 2 * M; // column k of Q (the multipliers)
  __shared__ double red_v[SOLVE_TPB / 64];
  __shared__ int red_i[SOLVE_TPB / 64];
  __shared__ int piv_sh;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k < M; ++k) {
    double best = -1.0;
    int bi = M;
    for (int i = k + threadIdx.x; i < M; i += blockDim.x) {
      const double2 v = Q[(size_t)i * M + k];
      const double a = v.x * v.x + v.y * v.y;
      if (a > best) {
        best = a;
        bi = i;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[wave] = best;
      red_i[wave] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double bb = red_v[0];
      int ib = red_i[0];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
        if (red_v[w] > bb || (red_v[w] == bb && red_i[w] < ib)) {
          bb = red_v[w];
          ib = red_i[w];
        }
      piv_sh = ib < M ? ib : k;
    }
    __syncthreads();
    const int piv = piv_sh;
    if (piv != k) {
      for (int j = k + threadIdx.x; j < M; j += blockDim.x) {
        const double2 t = Q[(size_t)k * M + j];
        Q[(size_t)k * M + j] = Q[(size_t)piv * M + j];
        Q[(size_t)piv * M + j] = t;
      }
      for (int j = threadIdx.x; j < M; j += blockDim.x) {
        const double2 t = R[(size_t)k * M + j];
        R[(size_t)k * M + j] = R[(size_t)piv * M + j];
        R[(size_t)piv * M + j] = t;
      }
    }
    __syncthreads();
    const double2 d = Q[(size_t)k * M + k];
    const double dd = d.x * d.x + d.y * d.y;
    const double2 inv = make_double2(d.x / dd, -d.y / dd);
    for (int j = k + 1 + threadIdx.x; j < M; j += blockDim.x) prQ[j] = cmul(Q[(size_t)k * M + j], inv);
    for (int j = threadIdx.x; j < M; j += blockDim.x) prR[j] = cmul(R[(size_t)k * M + j], inv);
    for (int i = threadIdx.x; i < M; i += blockDim.x) mult[i] = Q[(size_t)i * M + k];
    __syncthreads();
    for (int j = k + 1 + threadIdx.x; j < M; j += blockDim.x) Q[(size_t)k * M + j] = prQ[j];
    for (int j = threadIdx.x; j < M; j += blockDim.x) R[(size_t)k * M + j] = prR[j];
    if (threadIdx.x == 0) Q[(size_t)k * M + k] = make_double2(1.0, 0.0);
    // rows i != k: row_i -= Q_ik * (pivot row), over Q's columns k+1.. and all of R's
    const int wq = M - k - 1, width = wq + M;
    const int64_t work = (int64_t)M * width;
    for (int64_t t = threadIdx.x; t < work; t += blockDim.x) {
      const int i = (int)(t / width), c = (int)(t - (int64_t)i * width);
      if (i == k) continue;
      const double2 f = mult[i];
      if (c < wq) {
        const int j = k + 1 + c;
        const double2 p = prQ[j];
        double2& q = Q[(size_t)i * M + j];
        q.x -= f.x * p.x - f.y * p.y;
        q.y -= f.x * p.y + f.y * p.x;
      } else {
        const int j = c - wq;
        const double2 p = prR[j];
        double2& r = R[(size_t)i * M + j];
        r.x -= f.x * p.x - f.y * p.y;
        r.y -= f.x * p.y + f.y * p.x;
      }
    }
    for (int i = threadIdx.x; i < M; i += blockDim.x)
      if (i != k) Q[(size_t)i * M + k] = make_double2(0.0, 0.0);
    __syncthreads();
  }
}

__global__ void copy_back_kernel(const SsInst* __restrict__ si, const int* __restrict__ begin, int n, int total) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n, idx);
  const SsInst& z = si[ii];
  const int e = idx - begin[ii];
  reinterpret_cast<double2*>(z.R)[e] = reinterpret_cast<const double2*>(z.X)[e];
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

void launch_ss_combine_high(const SsInst* d, const int* d_begin, int n_inst, int total, const PadeB13& b,
                            hipStream_t s) {
  if (total > 0) combine_high_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total, b);
}

void launch_ss_combine_odd(const SsInst* d, const int* d_begin, int n_inst, int total, const PadeB13& b,
                           hipStream_t s) {
  if (total > 0) combine_odd_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total, b);
}

void launch_ss_combine_even(const SsInst* d, const int* d_begin, int n_inst, int total, const PadeB13& b,
                            hipStream_t s) {
  if (total > 0) combine_even_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total, b);
}

void launch_ss_solve(const SsInst* d, int n_inst, int max_m, hipStream_t s) {
  if (n_inst > 0) solve_kernel<<<n_inst, SOLVE_TPB, 3 * (size_t)max_m * sizeof(double2), s>>>(d);
}

void launch_ss_copy_back(const SsInst* d, const int* d_begin, int n_inst, int total, hipStream_t s) {
  if (total > 0) copy_back_kernel<<<blocks(total, TPB), TPB, 0, s>>>(d, d_begin, n_inst, total);
}

}  // namespace etdm
