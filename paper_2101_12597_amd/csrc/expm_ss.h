// exp(A) of the complex skew-Hermitian generators by scaling and squaring with the
// [13/13] Pade approximant (Sec. 3.4, Eq. ss).
//
//   s      halvings that bring the largest 1-norm of the batch under theta_13
//   X      = A / 2^s
//   p(X)   = U + V with U the odd and V the even part (powers X^2, X^4, X^6 and
//            three more products, the usual evaluation of the degree-13 numerator)
//   R      = q(X)^-1 p(X), q(X) = p(-X) = V - U  (Gauss-Jordan, partial pivoting)
//   exp(A) = R^(2^s)  (s squarings, grouped GEMMs launched by the caller)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace etdm {

constexpr double SS_THETA13 = 5.371920351148152;  // 1-norm bound of the degree-13 approximant
constexpr int SS_MAX_HALVINGS = 64;
constexpr int SS_MAX_M = 1024;  // LDS of the solve: 3 rows of M complex

// Per instance: M x M complex matrices (interleaved re, im), row-major.
struct SsInst {
  const double* A;  // parameters (upper triangle read; the generator is skew-Hermitian)
  double *X, *X2, *X4, *X6;
  double *W, *Z, *T, *V;  // W becomes U = X T, Z becomes the denominator q(X)
  double* R;              // p(X) in, q(X)^-1 p(X) out (the exp(A) buffer)
  int32_t M;
};

// numerator coefficients b_0..b_13 of the [13/13] approximant
struct PadeB13 {
  double b[14];
};

// 1-norm of every generator, then the batch's halvings s (device int) and a copy for the host.
void launch_ss_scaling(const SsInst* d, int n_inst, double* norms, int* s_dev, hipStream_t s);
// X = A / 2^s as a full matrix
void launch_ss_build(const SsInst* d, const int* d_begin, int n_inst, int total, const int* s_dev, hipStream_t s);
// W = b13 X6 + b11 X4 + b9 X2,  Z = b12 X6 + b10 X4 + b8 X2
void launch_ss_combine_high(const SsInst* d, const int* d_begin, int n_inst, int total, const PadeB13& b,
                            hipStream_t s);
// T += b7 X6 + b5 X4 + b3 X2 + b1 I
void launch_ss_combine_odd(const SsInst* d, const int* d_begin, int n_inst, int total, const PadeB13& b,
                           hipStream_t s);
// with V_full = V + b6 X6 + b4 X4 + b2 X2 + b0 I and U (in W):  Z = V_full - U,  R = V_full + U
void launch_ss_combine_even(const SsInst* d, const int* d_begin, int n_inst, int total, const PadeB13& b,
                            hipStream_t s);
// R <- Z^-1 R by Gauss-Jordan elimination with partial pivoting (one workgroup per
// instance, 3 max_m complex of LDS); Z is overwritten.
void launch_ss_solve(const SsInst* d, int n_inst, int max_m, hipStream_t s);
// R <- X (after an odd number of squarings the result sits in X)
void launch_ss_copy_back(const SsInst* d, const int* d_begin, int n_inst, int total, hipStream_t s);

}  // namespace etdm
