// Kernels of the complex full path: one skew-Hermitian A per k-point.
//
//   iA = V diag(w) V^H                      (FP64 Jacobi)          Sec. 3.4, Eq. ed
//   exp(A) = V diag(exp(-i w)) V^H,  C = C0 exp(A)
//   d_mu = sum_m f_m |C_mu_m|^2 = (rho)_mu_mu,  n = sum_k w_k d_k (coupled k-points)
//   H = H0 + U diag(n),  H_MO = C^H H C,  L = w [F, H_MO]            Sec. 2
//   Y = V ((V^H L V) o D) V^H,  D_pq = int_0^1 exp(-i t (w_p - w_q)) dt
//   G_ij = dE/dRe a_ij + i dE/dIm a_ij = -(2 - delta_ij) Y_ij  (i <= j)   Eq. gradients
#include "ov.h"
#include "reduce.h"

namespace etdm {

__device__ __forceinline__ double sincz(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

// H = iA from the upper triangle (incl. the diagonal) of A; Re of the diagonal is ignored.
__global__ void z_build_iA_kernel(const ZInst* __restrict__ zi, const int* __restrict__ begin, int n_inst,
                                  int total) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n_inst, idx);
  const ZInst& z = zi[ii];
  const int M = z.M, e = idx - begin[ii];
  const int i = e / M, j = e - i * M;
  const double2* A = reinterpret_cast<const double2*>(z.A);
  double2* H = reinterpret_cast<double2*>(z.Hk);
  double2 v;
  if (i < j) {
    double2 a = A[(size_t)i * M + j];
    v = make_double2(-a.y, a.x);  // i * a
  } else if (i > j) {
    double2 a = A[(size_t)j * M + i];
    v = make_double2(-a.y, -a.x);  // conj(i * a_ji)
  } else {
    v = make_double2(-A[(size_t)i * M + i].y, 0.0);
  }
  H[e] = v;
}

// Vp[i][p] = V[i][p] exp(-i w_p)
__global__ void z_phase_kernel(const ZInst* __restrict__ zi, const int* __restrict__ begin, int n_inst,
                               int total) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n_inst, idx);
  const ZInst& z = zi[ii];
  const int M = z.M, e = idx - begin[ii];
  const int p = e % M;
  double sn, cs;
  sincos(z.w[p], &sn, &cs);
  const double2 v = reinterpret_cast<const double2*>(z.V)[e];
  reinterpret_cast<double2*>(z.Vp)[e] = make_double2(v.x * cs + v.y * sn, v.y * cs - v.x * sn);
}

// d_mu = sum_m f_m |C_mu_m|^2 and e_mu = sum_m f_m Re(conj(C_mu_m) (H0 C)_mu_m); one wavefront per row
__global__ __launch_bounds__(256) void z_rows_kernel(const ZInst* __restrict__ zi, const int* __restrict__ begin,
                                                     int n_inst, int total_rows) {
  const int lane = threadIdx.x & 63;
  const int row_g = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row_g >= total_rows) return;
  const int ii = instance_of(begin, n_inst, row_g);
  const ZInst& z = zi[ii];
  const int M = z.M, mu = row_g - begin[ii];
  const double2* C = reinterpret_cast<const double2*>(z.C) + (size_t)mu * M;
  const double2* T = reinterpret_cast<const double2*>(z.T) + (size_t)mu * M;
  double sd = 0.0, se = 0.0;
  for (int m = lane; m < M; m += 64) {
    const double2 c = C[m], t = T[m];
    const double fm = z.f[m];
    sd += fm * (c.x * c.x + c.y * c.y);
    se += fm * (c.x * t.x + c.y * t.y);
  }
  for (int o = 32; o > 0; o >>= 1) {
    sd += __shfl_xor(sd, o);
    se += __shfl_xor(se, o);
  }
  if (lane == 0) {
    z.d[mu] = sd;
    z.e[mu] = se;
  }
}

// n_mu = sum_k w_k d_k,mu in a fixed order over k
__global__ void z_hubbard_density_kernel(const ZInst* __restrict__ zi, int n_inst, double* n_out, int M) {
  int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu >= M) return;
  double s = 0.0;
  for (int k = 0; k < n_inst; ++k) s += zi[k].weight * zi[k].d[mu];
  n_out[mu] = s;
}

// T = H0 C + U diag(n) C, one wavefront per row
__global__ __launch_bounds__(256) void z_apply_hubbard_kernel(const ZInst* __restrict__ zi,
                                                              const int* __restrict__ begin, int n_inst,
                                                              int total_rows, double U) {
  const int lane = threadIdx.x & 63;
  const int row_g = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row_g >= total_rows) return;
  const int ii = instance_of(begin, n_inst, row_g);
  const ZInst& z = zi[ii];
  const int M = z.M, mu = row_g - begin[ii];
  const double un = U * z.n[mu];
  const double2* C = reinterpret_cast<const double2*>(z.C) + (size_t)mu * M;
  double2* T = reinterpret_cast<double2*>(z.T) + (size_t)mu * M;
  for (int m = lane; m < M; m += 64) {
    double2 t = T[m], c = C[m];
    T[m] = make_double2(t.x + un * c.x, t.y + un * c.y);
  }
}

// E_k = w_k sum_mu e_mu (+ (U/2) sum d^2 for independent instances)
__global__ __launch_bounds__(256) void z_energy_kernel(const ZInst* __restrict__ zi, int couple, double U,
                                                       double* E) {
  __shared__ double red[16];
  const ZInst& z = zi[blockIdx.x];
  double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0, s3 = 0.0, c3 = 0.0;
  for (int mu = threadIdx.x; mu < z.M; mu += blockDim.x) {
    neumaier_add(s1, c1, z.e[mu]);
    if (!couple) neumaier_add(s2, c2, z.d[mu] * z.d[mu]);
    if (z.eodd) neumaier_add(s3, c3, z.eodd[mu]);
  }
  const double band = block_sum_neumaier(s1, c1, red);
  const double hub = block_sum_neumaier(s2, c2, red);
  const double odd = block_sum_neumaier(s3, c3, red);
  if (threadIdx.x == 0)
    E[blockIdx.x] = z.weight * band + (couple ? 0.0 : 0.5 * U * hub) - 0.5 * z.lam * z.weight * odd;
}

// orbital-dependent model term, one wave per row mu: VC[mu][k] = -lam |C_mu_k|^2 C_mu_k and
// eodd[mu] = sum_k f_k |C_mu_k|^4
__global__ __launch_bounds__(256) void z_odd_rows_kernel(const ZInst* __restrict__ zi, const int* __restrict__ begin,
                                                         int n_inst, int total_rows) {
  const int lane = threadIdx.x & 63;
  const int row_g = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row_g >= total_rows) return;
  const int ii = instance_of(begin, n_inst, row_g);
  const ZInst& z = zi[ii];
  const int M = z.M, mu = row_g - begin[ii];
  const double2* C = reinterpret_cast<const double2*>(z.C) + (size_t)mu * M;
  double2* VC = reinterpret_cast<double2*>(z.VC) + (size_t)mu * M;
  double e = 0.0;
  for (int k = lane; k < M; k += 64) {
    const double2 c = C[k];
    const double a = c.x * c.x + c.y * c.y;
    VC[k] = make_double2(-z.lam * a * c.x, -z.lam * a * c.y);
    e += z.f[k] * a * a;
  }
  for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
  if (lane == 0) z.eodd[mu] = e;
}

// L[m][k] += w (f_m W[m][k] - f_k conj(W[k][m])), W[m][k] = <m|V^m|k>
__global__ void z_odd_L_kernel(const ZInst* __restrict__ zi, const int* __restrict__ begin, int n_inst, int total) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n_inst, idx);
  const ZInst& z = zi[ii];
  const int M = z.M, e = idx - begin[ii];
  const int m = e / M, k = e - m * M;
  const double2 wmk = reinterpret_cast<const double2*>(z.W)[e];
  const double2 wkm = reinterpret_cast<const double2*>(z.W)[(size_t)k * M + m];
  double2& l = reinterpret_cast<double2*>(z.L)[e];
  l.x += z.weight * (z.f[m] * wmk.x - z.f[k] * wkm.x);
  l.y += z.weight * (z.f[m] * wmk.y + z.f[k] * wkm.y);
}

// L[m][k] = w (f_m - f_k) H_MO[m][k], in place
__global__ void z_commutator_kernel(const ZInst* __restrict__ zi, const int* __restrict__ begin, int n_inst,
                                    int total) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n_inst, idx);
  const ZInst& z = zi[ii];
  const int M = z.M, e = idx - begin[ii];
  const int m = e / M, k = e - m * M;
  const double fac = z.weight * (z.f[m] - z.f[k]);
  double2* L = reinterpret_cast<double2*>(z.L);
  const double2 h = L[e];
  L[e] = make_double2(fac * h.x, fac * h.y);
}

// Lt[p][q] *= exp(-i x/2) sinc(x/2), x = w_p - w_q (stored in z.L)
__global__ void z_divdiff_kernel(const ZInst* __restrict__ zi, const int* __restrict__ begin, int n_inst,
                                 int total) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n_inst, idx);
  const ZInst& z = zi[ii];
  const int M = z.M, e = idx - begin[ii];
  const int p = e / M, q = e - p * M;
  const double x = 0.5 * (z.w[p] - z.w[q]);
  double sn, cs;
  sincos(x, &sn, &cs);
  const double sc = sincz(x);
  const double dr = cs * sc, di = -sn * sc;
  double2* L = reinterpret_cast<double2*>(z.L);
  const double2 v = L[e];
  L[e] = make_double2(v.x * dr - v.y * di, v.x * di + v.y * dr);
}

// G_ij = -(2 - delta_ij) Y_ij for i <= j (Re of the diagonal is not a variable), 0 below
__global__ void z_grad_kernel(const ZInst* __restrict__ zi, const int* __restrict__ begin, int n_inst,
                              int total, int* status) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n_inst, idx);
  const ZInst& z = zi[ii];
  const int M = z.M, e = idx - begin[ii];
  const int i = e / M, j = e - i * M;
  const double2 y = reinterpret_cast<const double2*>(z.Y)[e];
  double2 g;
  if (i < j) g = make_double2(-2.0 * y.x, -2.0 * y.y);
  else if (i == j) g = make_double2(0.0, -y.y);
  else g = make_double2(0.0, 0.0);
  reinterpret_cast<double2*>(z.G)[e] = g;
  if (!(isfinite(g.x) && isfinite(g.y))) atomicOr(status, ST_NONFINITE);
}

static inline int zb(int64_t n, int b) { return (int)((n + b - 1) / b); }

void launch_z_build_iA(const ZInst* d, const int* b, int n, int total, hipStream_t s) {
  if (total > 0) z_build_iA_kernel<<<zb(total, 256), 256, 0, s>>>(d, b, n, total);
}
void launch_z_phase(const ZInst* d, const int* b, int n, int total, hipStream_t s) {
  if (total > 0) z_phase_kernel<<<zb(total, 256), 256, 0, s>>>(d, b, n, total);
}
void launch_z_rows(const ZInst* d, const int* b, int n, int rows, hipStream_t s) {
  if (rows > 0) z_rows_kernel<<<zb(rows, 4), 256, 0, s>>>(d, b, n, rows);
}
void launch_z_hubbard_density(const ZInst* d, int n, int couple, double* n_out, int M, hipStream_t s) {
  (void)couple;
  if (M > 0) z_hubbard_density_kernel<<<zb(M, 256), 256, 0, s>>>(d, n, n_out, M);
}
void launch_z_apply_hubbard(const ZInst* d, const int* b, int n, int rows, double U, hipStream_t s) {
  if (rows > 0) z_apply_hubbard_kernel<<<zb(rows, 4), 256, 0, s>>>(d, b, n, rows, U);
}
void launch_z_energy(const ZInst* d, int n, int couple, double U, double* E, hipStream_t s) {
  if (n > 0) z_energy_kernel<<<n, 256, 0, s>>>(d, couple, U, E);
}
void launch_z_commutator(const ZInst* d, const int* b, int n, int total, hipStream_t s) {
  if (total > 0) z_commutator_kernel<<<zb(total, 256), 256, 0, s>>>(d, b, n, total);
}
void launch_z_odd_rows(const ZInst* d, const int* b, int n, int rows, hipStream_t s) {
  if (rows > 0) z_odd_rows_kernel<<<zb(rows, 4), 256, 0, s>>>(d, b, n, rows);
}
void launch_z_odd_L(const ZInst* d, const int* b, int n, int total, hipStream_t s) {
  if (total > 0) z_odd_L_kernel<<<zb(total, 256), 256, 0, s>>>(d, b, n, total);
}
void launch_z_divdiff(const ZInst* d, const int* b, int n, int total, hipStream_t s) {
  if (total > 0) z_divdiff_kernel<<<zb(total, 256), 256, 0, s>>>(d, b, n, total);
}
void launch_z_grad(const ZInst* d, const int* b, int n, int total, int* status, hipStream_t s) {
  if (total > 0) z_grad_kernel<<<zb(total, 256), 256, 0, s>>>(d, b, n, total, status);
}

// ---------------------------------------------------------------------------
// Preconditioner set-up of the L-BFGS driver (FP64), whole batch per launch
// ---------------------------------------------------------------------------
// n0_mu = sum_i f_i |C0_mu_i|^2, one wave per row of the batch
__global__ __launch_bounds__(256) void prec_density_kernel(const PrecInst* __restrict__ pi,
                                                           const int* __restrict__ begin, int n_inst,
                                                           int total_rows, int cplx) {
  const int lane = threadIdx.x & 63;
  const int row_g = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row_g >= total_rows) return;
  const int ii = instance_of(begin, n_inst, row_g);
  const PrecInst& q = pi[ii];
  const int M = q.M, mu = row_g - begin[ii];
  double s = 0.0;
  for (int i = lane; i < M; i += 64) {
    if (cplx) {
      const double2 c = reinterpret_cast<const double2*>(q.C0)[(size_t)mu * M + i];
      s += q.f[i] * (c.x * c.x + c.y * c.y);
    } else {
      const double c = q.C0[(size_t)mu * M + i];
      s += q.f[i] * c * c;
    }
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) q.n0[mu] = s;
}

// eps_i = Re sum_mu conj(C0_mu_i) ((H0 C0)_mu_i + U n_mu C0_mu_i), one thread per column
__global__ void prec_eps_kernel(const PrecInst* __restrict__ pi, const int* __restrict__ begin, int n_inst,
                                int total_cols, double U, int cplx) {
  const int col_g = blockIdx.x * blockDim.x + threadIdx.x;
  if (col_g >= total_cols) return;
  const int ii = instance_of(begin, n_inst, col_g);
  const PrecInst& q = pi[ii];
  const int M = q.M, i = col_g - begin[ii];
  double s = 0.0;
  for (int mu = 0; mu < M; ++mu) {
    if (cplx) {
      const double2 c = reinterpret_cast<const double2*>(q.C0)[(size_t)mu * M + i];
      const double2 h = reinterpret_cast<const double2*>(q.HC0)[(size_t)mu * M + i];
      s += c.x * h.x + c.y * h.y + U * q.nH[mu] * (c.x * c.x + c.y * c.y);
    } else {
      const double c = q.C0[(size_t)mu * M + i];
      s += c * (q.HC0[(size_t)mu * M + i] + U * q.nH[mu] * c);
    }
  }
  q.eps[i] = s;
}

// h = w max(0, -2 (eps_i - eps_j)(f_i - f_j)) and the weight w over the free variables:
// REAL_OV rows i < N, columns j >= N; complex: Re part for i < j, Im part for i <= j,
// 0 (and weight 1) elsewhere
__global__ void prec_hdiag_kernel(const PrecInst* __restrict__ pi, const int* __restrict__ begin, int n_inst,
                                  int total, int cplx) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n_inst, idx);
  const PrecInst& q = pi[ii];
  const int e = idx - begin[ii];
  if (!cplx) {
    const int Nv = q.M - q.N;
    const int i = e / Nv, j = q.N + (e - i * Nv);
    q.hd[e] = q.w * fmax(0.0, -2.0 * (q.eps[i] - q.eps[j]) * (q.f[i] - q.f[j]));
    q.wv[e] = q.w;
    return;
  }
  const int i = e / q.M, j = e - i * q.M;
  const double v = q.w * fmax(0.0, -2.0 * (q.eps[i] - q.eps[j]) * (q.f[i] - q.f[j]));
  q.hd[2 * e] = (i < j) ? v : 0.0;
  q.hd[2 * e + 1] = (i <= j) ? v : 0.0;
  q.wv[2 * e] = (i < j) ? q.w : 1.0;
  q.wv[2 * e + 1] = (i <= j) ? q.w : 1.0;
}

// C0 <- [C_occ | C_virt] for every instance (the reference update of the ov form)
__global__ void c0_update_kernel(const C0Inst* __restrict__ ci, const int* __restrict__ begin, int n_inst,
                                 int total) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int ii = instance_of(begin, n_inst, idx);
  const C0Inst& q = ci[ii];
  const int e = idx - begin[ii], mu = e / q.M, j = e - mu * q.M;
  q.C0[e] = j < q.N ? q.Cocc[(size_t)mu * q.N + j] : q.Cvirt[(size_t)mu * (q.M - q.N) + (j - q.N)];
}

__global__ void fill_kernel(double* x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

// out[mu] = sum_k w_k x_k[mu], fixed order over k
__global__ void weighted_vsum_kernel(const double* const* xs, const double* ws, int n, int M, double* out) {
  int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu >= M) return;
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += ws[k] * xs[k][mu];
  out[mu] = s;
}

static inline int vgrid(int64_t n) { return (int)std::min<int64_t>(2048, std::max<int64_t>(1, (n + 255) / 256)); }

void launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n > 0) fill_kernel<<<vgrid(n), 256, 0, s>>>(x, n, v);
}


void launch_prec_setup(const PrecInst* d, const int* d_rows, int total_rows, const int* d_elems, int total_elems,
                       int n_inst, int cplx, double U, const double* const* coupled_n0, const double* coupled_w,
                       double* coupled_n, int couple_M, hipStream_t s) {
  if (n_inst <= 0) return;
  if (total_rows > 0) prec_density_kernel<<<zb(total_rows, 4), 256, 0, s>>>(d, d_rows, n_inst, total_rows, cplx);
  if (coupled_n0 && couple_M > 0)
    weighted_vsum_kernel<<<zb(couple_M, 256), 256, 0, s>>>(coupled_n0, coupled_w, n_inst, couple_M, coupled_n);
  if (total_rows > 0) prec_eps_kernel<<<zb(total_rows, 256), 256, 0, s>>>(d, d_rows, n_inst, total_rows, U, cplx);
  if (total_elems > 0)
    prec_hdiag_kernel<<<zb(total_elems, 256), 256, 0, s>>>(d, d_elems, n_inst, total_elems, cplx);
}
void launch_c0_update(const C0Inst* d, const int* d_begin, int n_inst, int total, hipStream_t s) {
  if (total > 0) c0_update_kernel<<<zb(total, 256), 256, 0, s>>>(d, d_begin, n_inst, total);
}
void launch_weighted_vsum(const double* const* xs, const double* ws, int n, int M, double* out, hipStream_t s) {
  if (M > 0) weighted_vsum_kernel<<<zb(M, 256), 256, 0, s>>>(xs, ws, n, M, out);
}

}  // namespace etdm
