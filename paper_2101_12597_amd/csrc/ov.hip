// Kernels of the real occupied-virtual path (Hutter's parametrization
// A = [[0, B], [-B^T, 0]], equal occupations f_occ on the first N orbitals).
//
// With P = B B^T = X diag(s) X^T and sigma = sqrt(s) (the rotation angles):
//   exp(A) = [[cos sqrt(P), sinc sqrt(P) B], [-B^T sinc sqrt(P), I + B^T W B]],
//   W = (cos sqrt(P) - I) P^{-1} = X diag(-1/2 sinc^2(sigma/2)) X^T      (Eq. uinv)
// and the exact gradient (Eq. gradients) in the singular-value basis of B is
//   dE/dB = -2 (sinc sqrt(P) L_ov + X Nm X^T B),  Gam = X^T (L_ov B^T) X,
//   Nm[k][l] = Gam[k][l] mu1[k][l] + Gam[l][k] mu2[k][l],
//   mu1[k][l] = -int_0^1 (t^2/2) cos(t sigma_k) sinc^2(t sigma_l / 2) dt,
//   mu2[k][l] =  int_0^1 t^2 sinc(t sigma_k) sinc(t sigma_l) dt.
//
// Every product is taken in the eigenbasis of P, through V = X^T B (row k is
// sigma_k times a unit vector):
//   C_occ  = (C0_o X cos - C0_v V^T sinc) X^T,
//   C_virt = C0_v + (C0_o X sinc + C0_v V^T W) V,
//   Gam    = X^T (L_ov V^T),   dE/dB = -2 (sinc sqrt(P) L_ov + (X Nm) V),
// where the diagonal factors act on column k.  Each term of these sums is then
// bounded independently of the angles (sinc(s) s = sin s, W(s) s^2 = cos s - 1), so a
// split-precision product, whose error is relative to the sum of the absolute values of
// its terms, keeps its accuracy at any rotation angle.  Products with B itself in
// another basis (B^T W B, L_ov B^T) would sum terms of size sigma_max that cancel.
//
// The two pair integrals are evaluated by Gauss-Legendre quadrature written as
// two rank-NQ matrix products (tables built here, products on the GEMM kernel) while
// both angles are at most OV_SIGQ; a pair with a larger angle takes closed forms
// (ov_pair_large), so rotations of any size are covered.
#include "ov.h"

namespace etdm {

__device__ __forceinline__ double sincd(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

__device__ __forceinline__ int find_range(const int* __restrict__ begin, int n, int idx) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= idx) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Pair integrals of a pair with max(a, b) > OV_SIGQ (a = sigma_k, b = sigma_l).
// With Kc = int_0^1 cos(ta) cos(tb) dt and Ks = int_0^1 sin(ta) sin(tb) dt,
//   mu1 = -(sinc a - Kc) / b^2,   mu2 = Ks / (a b),
// exact identities that lose accuracy only when the angle they divide by is small.
// There the small angle is expanded instead: sinc^2(x) = sum_n c_n x^(2n) with
// c_n = (-1)^n 2^(2n+1) / (2n+2)! and sinc(x) = sum_n (-1)^n x^(2n) / (2n+1)!, which
// leaves the moments C_m = int_0^1 t^m cos(tL) dt and S_m = int_0^1 t^m sin(tL) dt of
// the large angle L > OV_SIGQ.  Integration by parts gives them upward,
//   S_m = (m C_{m-1} - cos L) / L,   C_m = (sin L - m S_{m-1}) / L,
// which is stable for m < L.  OV_NSER terms reach rounding for a small angle below
// OV_TAU (the largest term left out is below 1e-19 relative).
constexpr double OV_TAU = 0.5;
constexpr int OV_NSER = 9;

__device__ void ov_pair_large(double a, double b, double& m1, double& m2) {
  const double lo = fmin(a, b), L = fmax(a, b);
  const bool ser1 = b < OV_TAU;   // then L = a
  const bool ser2 = lo < OV_TAU;  // (ser1 implies ser2)
  if (!ser1) m1 = -(sincd(a) - 0.5 * (sincd(a - b) + sincd(a + b))) / (b * b);
  if (!ser2) m2 = (sincd(a - b) - sincd(a + b)) / (2.0 * a * b);
  if (!ser2) return;
  double sL, cL;
  sincos(L, &sL, &cL);
  const double rL = 1.0 / L;
  double Cm = sL * rL, Sm = (1.0 - cL) * rL;  // m = 0
  double acc1 = 0.0, acc2 = 0.0;
  double p1 = 1.0, c1 = 1.0;        // (b/2)^(2n), c_n
  double p2 = 1.0, c2 = 1.0;        // lo^(2n), (-1)^n / (2n+1)!
  const double x1 = 0.25 * b * b, x2 = lo * lo;
  for (int m = 1; m <= 2 * OV_NSER + 2; ++m) {
    const double Sn = (m * Cm - cL) * rL;
    const double Cn = (sL - m * Sm) * rL;
    Sm = Sn;
    Cm = Cn;
    if (m & 1) {  // m = 2n + 1: a term of mu2
      acc2 += c2 * p2 * Sm;
      p2 *= x2;
      c2 *= -1.0 / ((m + 1.0) * (m + 2.0));
    } else {      // m = 2n + 2: a term of mu1
      acc1 += c1 * p1 * Cm;
      p1 *= x1;
      c1 *= -4.0 / ((m + 1.0) * (m + 2.0));
    }
  }
  if (ser1) m1 = -0.5 * acc1;
  m2 = acc2 * rL;
}

// mu1, mu2 of pair (k, l): the quadrature tables below OV_SIGQ, closed forms above
__device__ __forceinline__ void ov_pair_values(const double* __restrict__ s, const double* __restrict__ mu1,
                                               const double* __restrict__ mu2, int k, int l, int e, double& m1,
                                               double& m2) {
  const double a = sqrt(fmax(s[k], 0.0)), b = sqrt(fmax(s[l], 0.0));
  if (fmax(a, b) > OV_SIGQ) {
    ov_pair_large(a, b, m1, m2);
  } else {
    m1 = mu1[e];
    m2 = mu2[e];
  }
}

// Spectral pass of one instance, three kinds of 256-thread blocks:
//  * 32 x 32 tiles of X: X^T and (X diag(sinc))^T through an LDS transpose, and for
//    exp(A) the row-major copies [X diag(cos); X diag(sinc); X diag(W)];
//  * the quadrature tables, node-major ([q][j][k], k fastest):
//      T1s = cos(t_j s_k)(-w_j t_j^2 / 2), T2 = sinc^2(t_j s_k / 2),
//      T3s = sinc(t_j s_k) w_j t_j^2,       T3 = sinc(t_j s_k);
//  * the per-angle factors [cos | sinc | W].
constexpr int SP_TILE = 32;

int ov_spectral_blocks(int N) {
  const int nt = (N + SP_TILE - 1) / SP_TILE;
  return nt * nt + (OV_NQ * N + 255) / 256 + (N + 255) / 256;
}

__device__ __forceinline__ void spectral_factors(double sk, double& c, double& sn, double& w) {
  const double sig = sqrt(fmax(sk, 0.0));
  const double h = sincd(0.5 * sig);
  c = cos(sig);
  sn = sincd(sig);
  w = -0.5 * h * h;
}

__global__ __launch_bounds__(256) void ov_spectral_kernel(const OvSpec* __restrict__ specs,
                                                          const int* __restrict__ begin, int n_inst,
                                                          const double* __restrict__ gl_t,
                                                          const double* __restrict__ gl_w, int want_exp) {
  __shared__ double tile[SP_TILE][SP_TILE + 1];
  __shared__ double fsn[SP_TILE];
  const int ii = find_range(begin, n_inst, blockIdx.x);
  const OvSpec& sp = specs[ii];
  const int N = sp.N, t = threadIdx.x;
  if (N <= 0) return;
  const int nt = (N + SP_TILE - 1) / SP_TILE;
  int b = blockIdx.x - begin[ii];
  if (b < nt * nt) {
    const int i0 = (b / nt) * SP_TILE, k0 = (b % nt) * SP_TILE;
    const int lc = t & (SP_TILE - 1), lr = t >> 5;  // 8 rows per pass
    const int k = k0 + lc;
    double c = 0.0, sn = 0.0, w = 0.0;
    if (k < N) spectral_factors(sp.s[k], c, sn, w);
    if (lr == 0) fsn[lc] = sn;
    for (int r = lr; r < SP_TILE; r += 8) {
      const int i = i0 + r;
      double x = 0.0;
      if (i < N && k < N) {
        x = sp.X[(size_t)i * N + k];
        if (want_exp) {
          sp.Xcsw[(size_t)i * N + k] = x * c;
          sp.Xcsw[(size_t)(N + i) * N + k] = x * sn;
          sp.Xcsw[(size_t)(2 * N + i) * N + k] = x * w;
        }
      }
      tile[r][lc] = x;
    }
    __syncthreads();
    // transposed: output row k0 + r, column i0 + lc
    for (int r = lr; r < SP_TILE; r += 8) {
      const int ko = k0 + r, io = i0 + lc;
      if (ko < N && io < N) {
        const double x = tile[lc][r];
        sp.XT[(size_t)ko * N + io] = x;
        sp.XsnT[(size_t)ko * N + io] = x * fsn[r];
      }
    }
    return;
  }
  b -= nt * nt;
  const int ntab = (OV_NQ * N + 255) / 256;
  if (b < ntab) {
    const int idx = b * 256 + t;
    if (idx >= OV_NQ * N) return;
    const int j = idx / N, k = idx - j * N;
    const double sig = sqrt(fmax(sp.s[k], 0.0));
    const double tj = gl_t[j], wj = gl_w[j];
    const double ts = tj * sig;
    const double h = sincd(0.5 * ts);
    const double sc = sincd(ts);
    const size_t q = (size_t)OV_NQ * N;
    sp.tab[idx] = cos(ts) * (-0.5 * wj * tj * tj);
    sp.tab[q + idx] = h * h;
    sp.tab[2 * q + idx] = sc * (wj * tj * tj);
    sp.tab[3 * q + idx] = sc;
    return;
  }
  b -= ntab;
  const int k = b * 256 + t;
  if (k >= N) return;
  double c, sn, w;
  spectral_factors(sp.s[k], c, sn, w);
  sp.fac[k] = c;
  sp.fac[N + k] = sn;
  sp.fac[2 * N + k] = w;
}

// In-place eigenbasis combination (see OvRot), one thread per element of M x N.
__global__ void ov_rot_kernel(const OvRot* __restrict__ rots, const int* __restrict__ begin, int n_inst,
                              int total) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = find_range(begin, n_inst, idx);
  const OvRot& q = rots[ii];
  const int N = q.N;
  const int e = idx - begin[ii];
  const int k = e % N;
  const double c = q.fac[k], sn = q.fac[N + k], w = q.fac[2 * N + k];
  const double cx = q.CX[e], cv = q.CV[e];
  q.CX[e] = cx * c - cv * sn;
  q.CV[e] = cx * sn + cv * w;
  if (q.HX) q.HX[e] = q.HX[e] * c - q.HV[e] * sn;
}

template <typename T>
__device__ __forceinline__ T sf_conj(T v) { return v; }
template <>
__device__ __forceinline__ double2 sf_conj<double2>(double2 v) { return make_double2(v.x, -v.y); }
template <typename T>
__device__ __forceinline__ T sf_real(T v) { return v; }
template <>
__device__ __forceinline__ double2 sf_real<double2>(double2 v) { return make_double2(v.x, 0.0); }

template <typename T>
__global__ __launch_bounds__(256) void sym_fill_kernel(const SymFill* __restrict__ fills,
                                                       const int* __restrict__ begin, int n_inst,
                                                       double* __restrict__ dst) {
  __shared__ T tile[SP_TILE][SP_TILE + 1];
  const int ii = find_range(begin, n_inst, blockIdx.x);
  const SymFill& q = fills[ii];
  const int M = q.M, nt = (M + SP_TILE - 1) / SP_TILE;
  const int b = blockIdx.x - begin[ii];
  const int bi = b / nt, bj = b - bi * nt;
  const int lo = min(bi, bj), hi = max(bi, bj);
  const int lc = threadIdx.x & (SP_TILE - 1), lr = threadIdx.x >> 5;
  const T* src = reinterpret_cast<const T*>(q.src);
  for (int r = lr; r < SP_TILE; r += 8) {  // the upper tile (lo, hi)
    const int i = lo * SP_TILE + r, j = hi * SP_TILE + lc;
    T v{};
    if (i < M && j < M) v = src[(size_t)i * M + j];
    tile[r][lc] = v;
  }
  __syncthreads();
  T* out = reinterpret_cast<T*>(dst + q.dst_off);
  for (int r = lr; r < SP_TILE; r += 8) {
    const int i = bi * SP_TILE + r, j = bj * SP_TILE + lc;
    if (i >= M || j >= M) continue;
    const bool upper = bi < bj || (bi == bj && r <= lc);
    const T v = upper ? tile[r][lc] : sf_conj(tile[lc][r]);
    out[(size_t)i * M + j] = i == j ? sf_real(v) : v;
  }
}

__global__ void scale_cols_kernel(const ScaleCols* __restrict__ sc, const int* __restrict__ begin, int n_inst,
                                  int total) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = find_range(begin, n_inst, idx);
  const ScaleCols& q = sc[ii];
  const int e = idx - begin[ii];
  const double fk = q.f[e % q.M];
  const double2 c = reinterpret_cast<const double2*>(q.C)[e];
  reinterpret_cast<double2*>(q.out)[e] = make_double2(c.x * fk, c.y * fk);
}

// Row pass over the occupied orbitals: d_mu = f sum_i C_mu_i^2 (diagonal of rho),
// e_mu = sum_i C_mu_i (H0 C)_mu_i, then T = H0 C + U diag(d) C in place.
// One wavefront per row; lanes stride over columns, reduced in a fixed order.
__global__ __launch_bounds__(256) void ov_rows_kernel(const OvRows* __restrict__ rows,
                                                      const int* __restrict__ begin, int n_inst,
                                                      int total_rows, double U) {
  const int lane = threadIdx.x & 63;
  const int row_g = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row_g >= total_rows) return;
  const int ii = find_range(begin, n_inst, row_g);
  const OvRows& r = rows[ii];
  const int mu = row_g - begin[ii];
  const int N = r.N;
  const double* c = r.Cocc + (size_t)mu * N;
  double* t = r.T + (size_t)mu * N;
  double sd = 0.0, se = 0.0;
  for (int i = lane; i < N; i += 64) {
    const double ci = c[i];
    sd += ci * ci;
    se += ci * t[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    sd += __shfl_xor(sd, o);
    se += __shfl_xor(se, o);
  }
  const double d = r.f_occ * sd;
  if (lane == 0) {
    r.d[mu] = d;
    r.e[mu] = se;
  }
  const double ud = U * d;
  for (int i = lane; i < N; i += 64) t[i] += ud * c[i];
}

// Neumaier-compensated FP64 sum over a block, fixed order (deterministic).
__device__ double block_sum_comp(double s, double c, double* red) {
  // combine (s, c) pairs: first within the wavefront, then across wavefronts
  for (int o = 32; o > 0; o >>= 1) {
    double s2 = __shfl_xor(s, o), c2 = __shfl_xor(c, o);
    double t = s + s2;
    double err = (fabs(s) >= fabs(s2)) ? (s - t) + s2 : (s2 - t) + s;
    s = t;
    c += c2 + err;
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

__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
  double t = s + x;
  c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
  s = t;
}

// E_i = w_i (f sum_mu e_mu) + (U/2) sum_mu d_mu^2, one block per instance.
__global__ __launch_bounds__(256) void ov_energy_kernel(const OvEnergy* __restrict__ en, double U,
                                                        double* __restrict__ E) {
  __shared__ double red[16];
  const OvEnergy& q = en[blockIdx.x];
  double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
  for (int mu = threadIdx.x; mu < q.M; mu += blockDim.x) {
    neumaier_add(s1, c1, q.e[mu]);
    neumaier_add(s2, c2, q.d[mu] * q.d[mu]);
  }
  const double band = block_sum_comp(s1, c1, red);
  const double hub = block_sum_comp(s2, c2, red);
  if (threadIdx.x == 0) E[blockIdx.x] = q.weight * q.f_occ * band + 0.5 * U * hub;
}

// E_total = sum_i E_i (fixed order), and the non-finite check.
__global__ void total_energy_kernel(double* E, int n_inst, double extra_hub, const double* hub_vec,
                                    int hub_n, double U, int* status) {
  __shared__ double red[16];
  double s = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) neumaier_add(s, c, E[i]);
  const double tot = block_sum_comp(s, c, red);
  double hs = 0.0, hc = 0.0;
  for (int i = threadIdx.x; i < hub_n; i += blockDim.x) neumaier_add(hs, hc, hub_vec[i] * hub_vec[i]);
  const double hub = hub_n > 0 ? block_sum_comp(hs, hc, red) : 0.0;
  if (threadIdx.x == 0) {
    const double v = tot + 0.5 * U * hub + extra_hub;
    E[n_inst] = v;
    if (!isfinite(v)) atomicOr(status, ST_NONFINITE);
  }
}

// Nm[k][l] = Gam[k][l] mu1[k][l] + Gam[l][k] mu2[k][l]
__global__ void ov_pair_kernel(const OvPair* __restrict__ pr, const int* __restrict__ begin, int n_inst,
                               int total) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = find_range(begin, n_inst, idx);
  const OvPair& q = pr[ii];
  const int N = q.N;
  const int e = idx - begin[ii];
  const int k = e / N, l = e - k * N;
  double m1, m2;
  ov_pair_values(q.s, q.mu1, q.mu2, k, l, e, m1, m2);
  q.Nm[e] = q.Gam[e] * m1 + q.Gam[(size_t)l * N + k] * m2;
}

// Gradient chain of a small instance (N <= EIGH_LDS_MAX), one workgroup of CG_NT
// threads: X and the working matrix W in LDS with leading dimension N + 1 (an odd
// stride spreads the row-strided operand reads over the banks); each product is a grid
// of 16 x 16 tiles, wavefront w owning tiles w, w + 16, w + 32, on mfma_f64_16x16x4.
constexpr int CG_NT = 1024;
constexpr int CG_MAXT = 3;                                     // ceil(88 / 16)^2 = 36 tiles <= 16 x 3
constexpr int CG_PER = (EIGH_LDS_MAX * EIGH_LDS_MAX + CG_NT - 1) / CG_NT;  // elements per thread
typedef double cg_d4 __attribute__((ext_vector_type(4)));

// acc = op(A) op(B), n x n LDS matrices with leading dimension ld
template <bool AT, bool BT>
__device__ void cg_mm(const double* A, const double* B, int n, int ld, cg_d4 (&acc)[CG_MAXT]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = (n + 15) >> 4, lr = lane & 15, lk = lane >> 4;
  for (int s = 0; s < CG_MAXT; ++s) {
    acc[s] = cg_d4{0.0, 0.0, 0.0, 0.0};
    const int t = wave + 16 * s;
    if (t >= nt * nt) continue;  // uniform in the wavefront
    const int row = (t / nt) * 16 + lr, col = (t % nt) * 16 + lr;
    for (int k0 = 0; k0 < n; k0 += 4) {
      const int k = k0 + lk;
      double a = 0.0, b = 0.0;
      if (k < n) {
        if (row < n) a = AT ? A[k * ld + row] : A[row * ld + k];
        if (col < n) b = BT ? B[col * ld + k] : B[k * ld + col];
      }
      acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
    }
  }
}

// (i, j) of accumulator element r of tile slot s of this lane; false outside n x n
__device__ __forceinline__ bool cg_elem(int n, int s, int r, int& i, int& j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = (n + 15) >> 4, t = wave + 16 * s;
  if (t >= nt * nt) return false;
  i = (t / nt) * 16 + (lane >> 4) + 4 * r;
  j = (t % nt) * 16 + (lane & 15);
  return i < n && j < n;
}

__device__ __forceinline__ void cg_store(double* C, int n, int ld, const cg_d4 (&acc)[CG_MAXT]) {
  for (int s = 0; s < CG_MAXT; ++s)
    for (int r = 0; r < 4; ++r) {
      int i, j;
      if (cg_elem(n, s, r, i, j)) C[i * ld + j] = acc[s][r];
    }
}

__global__ __launch_bounds__(CG_NT) void ov_congruence_kernel(const OvCong* __restrict__ cg) {
  extern __shared__ double sm[];
  const OvCong& q = cg[blockIdx.x];
  const int n = q.N, ld = n + 1, tid = threadIdx.x;
  if (n <= 0) return;
  double* sX = sm;
  double* sW = sm + n * ld;
  for (int e = tid; e < n * n; e += CG_NT) {
    const int i = e / n, j = e - i * n;
    sX[i * ld + j] = q.X[e];
    sW[i * ld + j] = q.LV[e];
  }
  __syncthreads();
  cg_d4 acc[CG_MAXT];
  cg_mm<true, false>(sX, sW, n, ld, acc);  // Gam = X^T LV
  __syncthreads();
  cg_store(sW, n, ld, acc);
  __syncthreads();
  double nm[CG_PER];  // Nm = Gam o mu1 + Gam^T o mu2, this thread's elements
#pragma unroll
  for (int u = 0; u < CG_PER; ++u) {
    const int e = tid + u * CG_NT;
    nm[u] = 0.0;
    if (e < n * n) {
      const int k = e / n, l = e - k * n;
      double m1, m2;
      ov_pair_values(q.s, q.mu1, q.mu2, k, l, e, m1, m2);
      nm[u] = sW[k * ld + l] * m1 + sW[l * ld + k] * m2;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < CG_PER; ++u) {
    const int e = tid + u * CG_NT;
    if (e < n * n) {
      const int k = e / n, l = e - k * n;
      sW[k * ld + l] = nm[u];
    }
  }
  __syncthreads();
  cg_mm<false, false>(sX, sW, n, ld, acc);  // XNm = X Nm
  for (int s = 0; s < CG_MAXT; ++s)
    for (int r = 0; r < 4; ++r) {
      int i, j;
      if (cg_elem(n, s, r, i, j)) q.XNm[(size_t)i * n + j] = acc[s][r];
    }
}

// Non-finite scan of a gradient range (sets ST_NONFINITE).
__global__ void nonfinite_scan_kernel(const double* __restrict__ g, int64_t n, int* status) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) bad |= !isfinite(g[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(status, ST_NONFINITE);
}

// Y[i][j] = alpha * I (diagonal) for a strided square block
__global__ void set_identity_kernel(double* Y, int64_t ld, int n, double alpha) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  int i = idx / n, j = idx - i * n;
  Y[(size_t)i * ld + j] = (i == j) ? alpha : 0.0;
}

// copy an m x n block between strided row-major matrices, optionally scaled
__global__ void copy_block_kernel(double* dst, int64_t ldd, const double* src, int64_t lds, int m, int n,
                                  double alpha) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  int i = (int)(idx / n), j = (int)(idx - (int64_t)i * n);
  dst[(size_t)i * ldd + j] = alpha * src[(size_t)i * lds + j];
}

// T = H C for a block-sparse H (square bs x bs blocks, bs <= BSR_MAX_BS = 32) and a
// dense row-major C (ncols columns), on the FP64 matrix cores.  Grid: (column
// tiles of BSR_TC, block rows).  A workgroup computes one block row x BSR_TC
// columns: every block of the row is staged in LDS zero-padded to 32 x kp (kp =
// bs rounded up to 4) together with its bs x BSR_TC slab of C, and wavefront w
// accumulates the 32 x 16 columns [16 w, 16 w + 16) as two v_mfma_f64_16x16x4f64
// blocks.  The next block and slab are fetched into registers while the current
// ones are multiplied.
typedef double bsr_d4 __attribute__((ext_vector_type(4)));
constexpr int BSR_TC = 64;                                         // columns per workgroup
constexpr int BSR_HPER = (BSR_MAX_BS * BSR_MAX_BS + 255) / 256;    // block values per thread
constexpr int BSR_CPER = (BSR_MAX_BS * BSR_TC + 255) / 256;        // slab values per thread
__global__ __launch_bounds__(256) void bsr_spmm_kernel(BsrMat H, const double* __restrict__ C, int64_t ldc,
                                                       int ncols, double* __restrict__ T, int64_t ldt) {
  __shared__ double hs[BSR_MAX_BS][BSR_MAX_BS + 1];
  __shared__ double cs[BSR_MAX_BS][BSR_TC + 1];
  const int I = blockIdx.y, bs = H.bs, kp = (bs + 3) & ~3;
  const int j0 = blockIdx.x * BSR_TC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  // the padding (rows and columns >= bs) is zeroed once and never written
  for (int e = tid; e < BSR_MAX_BS * (BSR_MAX_BS + 1); e += 256) (&hs[0][0])[e] = 0.0;
  for (int e = tid; e < BSR_MAX_BS * (BSR_TC + 1); e += 256) (&cs[0][0])[e] = 0.0;
  const int p0 = H.row_ptr[I], p1 = H.row_ptr[I + 1];
  double rh[BSR_HPER], rc[BSR_CPER];
  auto fetch = [&](int p) {
    const double* hb = H.blocks + (size_t)p * bs * bs;
    const double* cb = C + (size_t)H.col_idx[p] * bs * ldc + j0;
#pragma unroll
    for (int u = 0; u < BSR_HPER; ++u) {
      const int e = tid + 256 * u;
      rh[u] = e < bs * bs ? hb[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < BSR_CPER; ++u) {
      const int e = tid + 256 * u, k = e / BSR_TC, jj = e - k * BSR_TC;
      rc[u] = (k < bs && j0 + jj < ncols) ? cb[(size_t)k * ldc + jj] : 0.0;
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int u = 0; u < BSR_HPER; ++u) {
      const int e = tid + 256 * u;
      if (e < bs * bs) hs[e / bs][e % bs] = rh[u];
    }
#pragma unroll
    for (int u = 0; u < BSR_CPER; ++u) {
      const int e = tid + 256 * u, k = e / BSR_TC, jj = e - k * BSR_TC;
      if (k < bs) cs[k][jj] = rc[u];
    }
  };
  bsr_d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  if (p0 < p1) fetch(p0);
  __syncthreads();
  for (int p = p0; p < p1; ++p) {
    commit();
    __syncthreads();
    if (p + 1 < p1) fetch(p + 1);
    for (int ks = 0; ks < kp; ks += 4) {
      const double a0 = hs[lr][ks + lk], a1 = hs[16 + lr][ks + lk];
      const double b = cs[ks + lk][wave * 16 + lr];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc1, 0, 0, 0);
    }
    __syncthreads();
  }
  // element r of lane l: row l / 16 + 4 r of the 16-row block, column l % 16
  const int col = j0 + wave * 16 + lr;
  if (col >= ncols) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int r0 = lk + 4 * r, r1 = 16 + lk + 4 * r;
    if (r0 < bs) T[(size_t)(I * bs + r0) * ldt + col] = acc0[r];
    if (r1 < bs) T[(size_t)(I * bs + r1) * ldt + col] = acc1[r];
  }
}

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

void launch_ov_spectral(const OvSpec* d, const int* d_begin, int n_inst, int total_blocks, const double* gl_t,
                        const double* gl_w, int want_exp, hipStream_t s) {
  if (total_blocks > 0) ov_spectral_kernel<<<total_blocks, 256, 0, s>>>(d, d_begin, n_inst, gl_t, gl_w, want_exp);
}
void launch_ov_rot(const OvRot* d, const int* d_begin, int n_inst, int total, hipStream_t s) {
  if (total > 0) ov_rot_kernel<<<nblk(total, 256), 256, 0, s>>>(d, d_begin, n_inst, total);
}
void launch_sym_fill(const SymFill* d, const int* d_begin, int n_inst, int total_tiles, double* dst, int cplx,
                     hipStream_t s) {
  if (total_tiles <= 0) return;
  if (cplx) sym_fill_kernel<double2><<<total_tiles, 256, 0, s>>>(d, d_begin, n_inst, dst);
  else sym_fill_kernel<double><<<total_tiles, 256, 0, s>>>(d, d_begin, n_inst, dst);
}
void launch_scale_cols(const ScaleCols* d, const int* d_begin, int n_inst, int total, hipStream_t s) {
  if (total > 0) scale_cols_kernel<<<nblk(total, 256), 256, 0, s>>>(d, d_begin, n_inst, total);
}
void launch_ov_rows(const OvRows* d, const int* d_begin, int n_inst, int total_rows, double U, hipStream_t s) {
  if (total_rows > 0) ov_rows_kernel<<<nblk(total_rows, 4), 256, 0, s>>>(d, d_begin, n_inst, total_rows, U);
}
void launch_ov_energy(const OvEnergy* d, int n_inst, double U, double* E, hipStream_t s) {
  if (n_inst > 0) ov_energy_kernel<<<n_inst, 256, 0, s>>>(d, U, E);
}
void launch_total_energy(double* E, int n_inst, double extra_hub, const double* hub_vec, int hub_n, double U,
                         int* status, hipStream_t s) {
  total_energy_kernel<<<1, 256, 0, s>>>(E, n_inst, extra_hub, hub_vec, hub_n, U, status);
}
void launch_ov_pair(const OvPair* d, const int* d_begin, int n_inst, int total, hipStream_t s) {
  if (total > 0) ov_pair_kernel<<<nblk(total, 256), 256, 0, s>>>(d, d_begin, n_inst, total);
}
void launch_ov_congruence(const OvCong* d, int n_inst, hipStream_t s) {
  if (n_inst <= 0) return;
  const size_t bytes = 2 * sizeof(double) * EIGH_LDS_MAX * (EIGH_LDS_MAX + 1);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&ov_congruence_kernel),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    attr = true;
  }
  ov_congruence_kernel<<<n_inst, CG_NT, bytes, s>>>(d);
}
void launch_nonfinite_scan(const double* g, int64_t n, int* status, hipStream_t s) {
  if (n > 0) nonfinite_scan_kernel<<<(int)std::min<int64_t>(1024, (n + 255) / 256), 256, 0, s>>>(g, n, status);
}
void launch_set_identity(double* Y, int64_t ld, int n, double alpha, hipStream_t s) {
  if (n > 0) set_identity_kernel<<<nblk((int64_t)n * n, 256), 256, 0, s>>>(Y, ld, n, alpha);
}
void launch_copy_block(double* dst, int64_t ldd, const double* src, int64_t lds, int m, int n, double alpha,
                       hipStream_t s) {
  if (m > 0 && n > 0) copy_block_kernel<<<nblk((int64_t)m * n, 256), 256, 0, s>>>(dst, ldd, src, lds, m, n, alpha);
}

void launch_bsr_spmm(const BsrMat& H, const double* C, int64_t ldc, int ncols, double* T, int64_t ldt,
                     hipStream_t s) {
  if (ncols <= 0 || H.nbr <= 0) return;
  dim3 grid((unsigned)nblk(ncols, BSR_TC), (unsigned)H.nbr);
  bsr_spmm_kernel<<<grid, 256, 0, s>>>(H, C, ldc, ncols, T, ldt);
}

}  // namespace etdm
