// exp(A) of the complex skew-Hermitian generators by scaling and squaring with a
// diagonal Pade approximant (Sec. 3.4, Eq. ss).
//
//   s      halvings that bring the largest 1-norm of the batch under theta_9
//   X      = A / 2^s; the [9/9] approximant is accurate to the unit roundoff there
//   p(X)   = U + V, U = X (b9 X^8 + b7 X^6 + b5 X^4 + b3 X^2 + b1 I) the odd part,
//            V = b8 X^8 + ... + b0 I the even part (powers X^2, X^4, X^6, X^8 and one
//            more product)
//   R      = q(X)^-1 p(X), q(X) = p(-X) = V - U
//   exp(A) = R^(2^s)  (s squarings, grouped GEMMs launched by the caller)
//
// X is skew-Hermitian, so V is Hermitian, U skew-Hermitian, and q(X) has Hermitian
// part V with eigenvalues Re p(i w) for the eigenvalues i w of X.  With |w| <=
// theta_9 < pi these are positive (Re p(i w) > 0 up to |w| = pi for this degree), so
// elimination without pivoting is stable and the solve is blocked by panels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace etdm {

constexpr double SS_THETA9 = 2.097847961257068;  // 1-norm bound of the degree-9 approximant
constexpr int SS_MAX_HALVINGS = 64;
constexpr int SS_MAX_M = 1024;  // largest M of the scaling-and-squaring path
constexpr int SS_NORM_TILES = (SS_MAX_M + 63) / 64;  // column tiles of the 1-norm per instance

// Per instance: M x M complex matrices (interleaved re, im), row-major.
struct SsInst {
  const double* A;  // parameters (upper triangle read; the generator is skew-Hermitian)
  double *X, *X2, *X4, *X6, *X8;
  double *T, *U, *Z;  // T = odd polynomial in X^2, U = X T, Z = q(X)
  double* R;          // p(X) in, q(X)^-1 p(X) out (the exp(A) buffer)
  double* Sq;         // partner of R in the squarings (the result sits there after an odd count)
  int32_t M;
};

// Frechet derivative L(A, E) of exp at the same A (Eq. ss differentiated), for the
// exact gradient Y = L(A, L) exp(A)^H: with Es = E / 2^s the derivatives of the
// powers are M2 = X Es + Es X, M4 = X2 M2 + M2 X2, M6 = X4 M2 + M4 X2,
// M8 = X4 M4 + M4 X4 (grouped GEMMs); LT, LV are the odd / even combinations,
// LU = X LT + Es T, L_r = q^-1 (L_p - L_q r) with L_p - L_q r = (LU + LV) - (LV - LU) r,
// and each squaring carries L <- R L + L R.
struct SsDeriv {
  const double* L;  // direction E (the commutator L of the energy)
  double *Es, *M2, *M4, *M6, *M8;
  double *LT, *LV;  // odd / even combinations; LT then holds LV - LU, LV the right-hand side
  int32_t M;
};

// numerator coefficients b_0..b_9 of the [9/9] approximant
struct PadeB9 {
  double b[10];
};

// 1-norm of every generator (largest column sum per tile of 64 columns; norms holds
// n_inst * SS_NORM_TILES doubles), then the batch's halvings s (device int).
void launch_ss_scaling(const SsInst* d, int n_inst, double* norms, int* s_dev, hipStream_t s);
// X = A / 2^s as a full matrix
void launch_ss_build(const SsInst* d, const int* d_begin, int n_inst, int total, const int* s_dev, hipStream_t s);
// T = b9 X8 + b7 X6 + b5 X4 + b3 X2 + b1 I
void launch_ss_combine_odd(const SsInst* d, const int* d_begin, int n_inst, int total, const PadeB9& b,
                           hipStream_t s);
// V = b8 X8 + b6 X6 + b4 X4 + b2 X2 + b0 I and U:  Z = V - U,  R = V + U
void launch_ss_combine_even(const SsInst* d, const int* d_begin, int n_inst, int total, const PadeB9& b,
                            hipStream_t s);
// Panel width nb of the solve (32, two k-tiles of the complex GEMM; the same for every M).
int ss_solve_panel(int max_m);
// One panel of R <- Z^-1 R by block Gauss-Jordan elimination without pivoting: the
// rows k0..k0+nb of [Z | R] (columns k0.. of Z, all of R) are reduced by the inverse
// of their diagonal block, several workgroups per instance over the columns
// (instances with M <= k0 are left alone).  The caller then updates every other row i with
// row_i -= Z[i, k0:k0+nb] (reduced panel rows), over the columns of Z right of the
// panel and all of R (grouped complex GEMMs, C = -A B + C), before the next panel.
// After the last panel R holds the solution; Z is overwritten.
void launch_ss_panel(const SsInst* d, int n_inst, int max_m, int k0, int nb, hipStream_t s);
// Es = E / 2^s
void launch_ss_deriv_scale(const SsDeriv* d, const int* d_begin, int n_inst, int total, const int* s_dev,
                           hipStream_t s);
// LT = b9 M8 + b7 M6 + b5 M4 + b3 M2,  LV = b8 M8 + b6 M6 + b4 M4 + b2 M2
void launch_ss_deriv_combine(const SsDeriv* d, const int* d_begin, int n_inst, int total, const PadeB9& b,
                             hipStream_t s);
// with LU (in `lu` of instance i at the same offsets): LT <- LV - LU, LV <- LU + LV
void launch_ss_deriv_rhs(const SsDeriv* d, const double* const* lu, const int* d_begin, int n_inst, int total,
                         hipStream_t s);
// dst <- src elementwise over every instance's M x M complex matrix
void launch_ss_copy(const double* const* src, double* const* dst, const int* d_begin, int n_inst, int total,
                    hipStream_t s);
// R <- Sq (after an odd number of squarings the result sits in Sq)
void launch_ss_copy_back(const SsInst* d, const int* d_begin, int n_inst, int total, hipStream_t s);

}  // namespace etdm
