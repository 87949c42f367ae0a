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
constexpr int SOLVE_NB = 32;     // panel rows: two k-tiles of the complex GEMM that updates the rest
constexpr int SOLVE_COLS = 32;   // columns right of the diagonal block per panel workgroup (one wavefront)
constexpr int SOLVE_TPB = SOLVE_NB + SOLVE_COLS;  // one column of the panel per thread

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
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
}

// Largest column 1-norm over one tile of 64 columns of a generator, read from the
// stored upper triangle: column j of the generator has |a_ij| (i < j) above the
// diagonal, |Im a_jj| on it and |a_ji| (i > j) below, which is row j of the upper
// triangle.  Four wavefronts: the column parts row by row (lanes over columns) and the
// row parts of the tile's 64 rows (lanes over the row); every read is coalesced.
__global__ __launch_bounds__(TPB) void norm1_kernel(const SsInst* __restrict__ si, double* norms) {
  static_assert(TPB == 256, "four wavefronts");
  const SsInst& z = si[blockIdx.x / SS_NORM_TILES];
  const int M = z.M, j0 = (blockIdx.x % SS_NORM_TILES) * 64;
  if (j0 >= M) {
    if (threadIdx.x == 0) norms[blockIdx.x] = 0.0;
    return;
  }
  const double2* __restrict__ A = reinterpret_cast<const double2*>(z.A);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = j0 + lane;
  __shared__ double cs[4][64];
  __shared__ double rs[64];
  double col = 0.0;
  if (j < M) {
    for (int i = wave; i < j; i += 4) {
      const double2 a = A[(size_t)i * M + j];
      col += sqrt(a.x * a.x + a.y * a.y);
    }
    if (wave == 0) col += fabs(A[(size_t)j * M + j].y);
  }
  cs[wave][lane] = col;
  for (int rr = wave; rr < 64; rr += 4) {
    const int r = j0 + rr;
    double p = 0.0;
    if (r < M)
      for (int i = r + 1 + lane; i < M; i += 64) {
        const double2 a = A[(size_t)r * M + i];
        p += sqrt(a.x * a.x + a.y * a.y);
      }
    p = wave_sum(p);
    if (lane == 0) rs[rr] = p;
  }
  __syncthreads();
  if (wave == 0) {
    const double t = j < M ? ((cs[0][lane] + cs[1][lane]) + (cs[2][lane] + cs[3][lane])) + rs[lane] : 0.0;
    const double m = wave_max(t);
    if (lane == 0) norms[blockIdx.x] = m;
  }
}

// the fewest halvings s that bring every finite norm under theta_9: from the largest one
__global__ __launch_bounds__(TPB) void scaling_kernel(const double* __restrict__ norms, int n, int* s_dev) {
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += TPB) {
    const double v = norms[i];
    if (isfinite(v)) mx = fmax(mx, v);  // non-finite input: caught by the energy and gradient scans
  }
  mx = wave_max(mx);
  __shared__ double wm[TPB / 64];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < TPB / 64; ++w) mx = fmax(mx, wm[w]);
    mx = fmax(mx, wm[0]);
    int s = 0;
    while (s < SS_MAX_HALVINGS && ldexp(mx, -s) > SS_THETA9) ++s;
    *s_dev = s;
  }
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
// definite Hermitian part), one panel of nb <= SOLVE_NB rows k0..k0+nb at a time:
//   panel_kernel  the panel rows (columns k0.. of Z, all of R) are reduced by the
//                 inverse of their diagonal block D.  Workgroup g of an instance holds
//                 D's columns and its own SOLVE_COLS columns right of D, one column of
//                 nb rows per thread in registers; step c scales row c by 1 / D_cc and
//                 subtracts it from the other rows, the pivot column shared through LDS
//                 (two buffers: the next one is written while the current one is read).
//                 Only the columns right of D are written back.
//   then every other row i takes row_i -= Z[i, k0:k0+nb] (reduced panel rows) over the
//   columns right of the panel, a rank-nb update that the caller launches as grouped
//   complex GEMMs.  Columns of Z left of the panel (D included) are never read again
//   and are not written.
__global__ __launch_bounds__(SOLVE_TPB) void panel_kernel(const SsInst* __restrict__ si, int k0, int NB,
                                                          int groups) {
  const SsInst& z = si[blockIdx.x / groups];
  const int g = blockIdx.x % groups;
  const int M = z.M;
  if (k0 >= M) return;
  const int nb = min(min(NB, SOLVE_NB), M - k0), wq = M - k0, W = wq + M;
  const int c0 = nb + g * SOLVE_COLS;  // first column of this workgroup right of D
  if (c0 >= W) return;                 // whole workgroup
  double2* __restrict__ Q = reinterpret_cast<double2*>(z.Z);
  double2* __restrict__ R = reinterpret_cast<double2*>(z.R);
  __shared__ double2 piv[2][SOLVE_NB];
  const int t = threadIdx.x;
  // panel column (counted from k0 across [Z | R]) of this thread
  const int col = t < SOLVE_NB ? t : c0 + (t - SOLVE_NB);
  const bool act = t < SOLVE_NB ? t < nb : col < W;
  double2 x[SOLVE_NB];
#pragma unroll
  for (int r = 0; r < SOLVE_NB; ++r) {
    x[r] = make_double2(0.0, 0.0);
    if (act && r < nb)
      x[r] = col < wq ? Q[(size_t)(k0 + r) * M + k0 + col] : R[(size_t)(k0 + r) * M + (col - wq)];
  }
  if (t == 0)
#pragma unroll
    for (int r = 0; r < SOLVE_NB; ++r) piv[0][r] = x[r];
  __syncthreads();
  // steps in blocks of 8, unrolled; after each block the register array turns by 8
  // rows, so step c always finds its pivot row in x[c % 8] and the code stays small.
  // The turn precedes the block's last pivot-column write, so every published column
  // is in the order its readers hold; after the SOLVE_NB / 8 blocks x[r] is row r again.
  static_assert(SOLVE_NB % 8 == 0, "whole blocks of 8 steps");
  for (int o = 0; o < SOLVE_NB / 8; ++o) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int c = 8 * o + i;
      // the update runs for every c (no merges of the register array); a step past
      // nb has multiplier 0 and leaves x alone (its pivot row holds zeros)
      const double2* f = piv[c & 1];
      const double2 d = f[i];
      const double rd = c < nb ? 1.0 / (d.x * d.x + d.y * d.y) : 0.0;
      const double2 xi = x[i];
      const double2 q = make_double2((xi.x * d.x + xi.y * d.y) * rd, (xi.y * d.x - xi.x * d.y) * rd);
#pragma unroll
      for (int rb = 0; rb < SOLVE_NB; rb += 8) {  // pivot column read 8 entries at a time
        double2 fb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) fb[u] = f[rb + u];  // rows past nb hold zeros
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = rb + u;
          if (r == i) continue;
          x[r].x = fma(-fb[u].x, q.x, fma(fb[u].y, q.y, x[r].x));
          x[r].y = fma(-fb[u].x, q.y, fma(-fb[u].y, q.x, x[r].y));
        }
      }
      x[i] = q;
      if (i == 7) {
        double2 head[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) head[r] = x[r];
#pragma unroll
        for (int r = 0; r < SOLVE_NB - 8; ++r) x[r] = x[r + 8];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[SOLVE_NB - 8 + r] = head[r];
      }
      if (c < nb) {
        if (t == c + 1 && c + 1 < nb)
#pragma unroll
          for (int r = 0; r < SOLVE_NB; ++r) piv[(c + 1) & 1][r] = x[r];
        __syncthreads();
      }
    }
  }
  if (t >= SOLVE_NB && act)
#pragma unroll
    for (int r = 0; r < SOLVE_NB; ++r)
      if (r < nb) {
        if (col < wq) Q[(size_t)(k0 + r) * M + k0 + col] = x[r];
        else R[(size_t)(k0 + r) * M + (col - wq)] = x[r];
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
  norm1_kernel<<<n_inst * SS_NORM_TILES, TPB, 0, s>>>(d, norms);
  scaling_kernel<<<1, TPB, 0, s>>>(norms, n_inst * SS_NORM_TILES, s_dev);
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

int ss_solve_panel(int) { return SOLVE_NB; }

void launch_ss_panel(const SsInst* d, int n_inst, int max_m, int k0, int nb, hipStream_t s) {
  if (n_inst <= 0 || max_m <= 0 || nb <= 0 || nb > SOLVE_NB) return;
  // columns right of the diagonal block: at most 2 max_m - 1
  const int groups = blocks(2 * (int64_t)max_m - 1, SOLVE_COLS);
  panel_kernel<<<n_inst * groups, SOLVE_TPB, 0, s>>>(d, k0, nb, groups);
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
