// Descriptors and launchers of the elementwise / reduction kernels.
#pragma once

#include <algorithm>

#include "common.h"

namespace etdm {

constexpr int OV_NQ = 48;
// The 48-node rule of the pair integrals is exact to rounding while both angles are at
// most OV_SIGQ (it still is at 60 rad); pairs with a larger angle take closed forms.
constexpr double OV_SIGQ = 40.0;
constexpr int BSR_MAX_BS = 32;  // largest block size of a block-sparse H0

// block-sparse rows, square blocks (device arrays)
struct BsrMat {
  const double* blocks;  // [nnzb][bs][bs]
  const int* row_ptr;    // [nbr + 1]
  const int* col_idx;    // [nnzb]
  int nbr, bs;
};
// T = H C (C: M x ncols row-major, ld ldc; T: ld ldt)
void launch_bsr_spmm(const BsrMat& H, const double* C, int64_t ldc, int ncols, double* T, int64_t ldt,
                     hipStream_t s);

// Spectral factors and eigenbasis copies of one instance (the spectral kernel):
// per angle sigma_k = sqrt(max(s_k, 0)) the factors cos, sinc and W = -1/2 sinc^2(sigma/2),
// the transposes X^T and (X diag(sinc))^T the eigenbasis products take, the quadrature
// tables of the pair integrals stored node-major, and for exp(A) the scaled copies
// [X diag(cos); X diag(sinc); X diag(W)].
struct OvSpec {
  const double* s;  // eigenvalues of P [N]
  const double* X;  // eigenvectors [N x N] (column k belongs to s_k)
  double* fac;      // [3 x N]: cos, sinc, W of each angle
  double* XT;       // [N x N] X^T
  double* XsnT;     // [N x N] (X diag(sinc))^T
  double* tab;      // [4 x OV_NQ x N]: T1s, T2, T3s, T3 (node-major)
  double* Xcsw;     // [3N x N], written only when the exponential itself is wanted
  int32_t N;
};
// per instance: ceil(N/32)^2 transpose tiles, then the table and factor blocks
int ov_spectral_blocks(int N);

// The eigenbasis combination of the rotated orbitals (Eq. uinv in the basis of the
// eigenvectors of P), per column k with the factors of sigma_k, in place:
//   CX <- CX cos - CV sinc      (then C_occ = CX X^T)
//   CV <- CX sinc + CV W        (then C_virt = C0_v + CV V)
//   HX <- HX cos - HV sinc      (dense H0: then T = H0 C_occ = HX X^T)
struct OvRot {
  double* CX;  // [M x N] C0_o X
  double* CV;  // [M x N] C0_v V^T, V = X^T B
  double* HX;  // [M x N] (H0 C0)_o X, or null
  const double* HV;  // [M x N] (H0 C0)_v V^T
  const double* fac;
  int32_t M, N;
};
void launch_ov_rot(const OvRot* d, const int* d_begin, int n_inst, int total, hipStream_t s);

// Symmetric (Hermitian) fill of the density output: dst + dst_off (M x M) from the
// upper triangle of src, dst[i][j] = src[i][j] for i <= j and conj(src[j][i]) below,
// with a real diagonal (complex: interleaved pairs, offsets count doubles), in 32 x 32
// tiles; begin = prefix sum of the ceil(M/32)^2 tiles of each instance.
struct SymFill {
  const double* src;
  int64_t dst_off;
  int32_t M;
};
void launch_sym_fill(const SymFill* d, const int* d_begin, int n_inst, int total_tiles, double* dst, int cplx,
                     hipStream_t s);
// out = C diag(f) (complex M x M, f real), one thread per element.
struct ScaleCols {
  const double* C;
  const double* f;
  double* out;
  int32_t M;
};
void launch_scale_cols(const ScaleCols* d, const int* d_begin, int n_inst, int total, hipStream_t s);

struct OvRows {
  const double* Cocc;  // [M x N]
  double* T;           // [M x N]: H0 Cocc in, H Cocc out
  double* d;           // [M]
  double* e;           // [M]
  int32_t M, N;
  double f_occ;
};

struct OvEnergy {
  const double* d;
  const double* e;
  int32_t M;
  double f_occ;
  double weight;
};

struct OvPair {
  const double* s;  // eigenvalues of P [N] (squared rotation angles)
  const double* Gam;
  const double* mu1;
  const double* mu2;
  double* Nm;
  int32_t N;
};

// The middle of the gradient chain of one instance with N <= EIGH_LDS_MAX in one
// workgroup (Eq. gradients): Gam = X^T LV, Nm = Gam o mu1 + Gam^T o mu2, XNm = X Nm.
// X and one working matrix sit in LDS; the two N x N x N products run on the FP64
// matrix cores.
struct OvCong {
  const double* s;    // [N] eigenvalues of P (squared rotation angles)
  const double* X;    // [N x N] eigenvectors of P
  const double* LV;   // [N x N] L_ov V^T
  const double* mu1;  // [N x N] pair integrals
  const double* mu2;
  double* XNm;        // [N x N] out
  int32_t N;
};
void launch_ov_congruence(const OvCong* d, int n_inst, hipStream_t s);

void launch_ov_spectral(const OvSpec* d, const int* d_begin, int n_inst, int total_blocks, const double* gl_t,
                        const double* gl_w, int want_exp, hipStream_t s);
void launch_ov_rows(const OvRows* d, const int* d_begin, int n_inst, int total_rows, double U, hipStream_t s);
void launch_ov_energy(const OvEnergy* d, int n_inst, double U, double* E, hipStream_t s);
void launch_total_energy(double* E, int n_inst, double extra_hub, const double* hub_vec, int hub_n, double U,
                         int* status, hipStream_t s);
void launch_ov_pair(const OvPair* d, const int* d_begin, int n_inst, int total, hipStream_t s);
void launch_nonfinite_scan(const double* g, int64_t n, int* status, hipStream_t s);
void launch_set_identity(double* Y, int64_t ld, int n, double alpha, hipStream_t s);
void launch_copy_block(double* dst, int64_t ldd, const double* src, int64_t lds, int m, int n, double alpha,
                       hipStream_t s);

// ---------------------------------------------------------------------------
// complex full path (interleaved complex float64; pointers address doubles)
// ---------------------------------------------------------------------------
struct ZInst {
  const double* A;   // parameters [M x M] complex (upper triangle read)
  double* Hk;        // iA workspace [M x M]
  double* V;         // eigenvectors [M x M]
  const double* w;   // eigenvalues [M]
  double* Vp;        // V diag(exp(-i w)) [M x M]
  const double* C;   // orbitals [M x M]
  double* T;         // H0 C in, H C out [M x M]
  double* d;         // diag(rho) [M] (real)
  double* e;         // row energies [M] (real)
  const double* n;   // Hubbard density used for this instance [M]
  double* L;         // H_MO in, L out [M x M]
  double* G;         // gradient out [M x M]
  const double* Y;   // Y [M x M]
  const double* f;   // occupations [M]
  int32_t M;
  double weight;
  // orbital-dependent model term (null eodd: off): VC = -lam |C|^2 o C, W = VC^H C,
  // eodd[mu] = sum_k f_k |C_mu_k|^4
  double* VC;
  const double* W;
  double* eodd;
  double lam;
};

void launch_z_build_iA(const ZInst* d, const int* d_begin, int n_inst, int total, hipStream_t s);
void launch_z_phase(const ZInst* d, const int* d_begin, int n_inst, int total, hipStream_t s);
void launch_z_rows(const ZInst* d, const int* d_begin, int n_inst, int total_rows, hipStream_t s);
void launch_z_hubbard_density(const ZInst* d, int n_inst, int couple, double* n_out, int M, hipStream_t s);
void launch_z_apply_hubbard(const ZInst* d, const int* d_begin, int n_inst, int total_rows, double U,
                            hipStream_t s);
void launch_z_energy(const ZInst* d, int n_inst, int couple, double U, double* E, hipStream_t s);
void launch_z_commutator(const ZInst* d, const int* d_begin, int n_inst, int total, hipStream_t s);
// orbital-dependent model term: VC and eodd per row (one wave per row)
void launch_z_odd_rows(const ZInst* d, const int* d_begin_rows, int n_inst, int total_rows, hipStream_t s);
// L[m][k] += w (f_m W[m][k] - f_k conj(W[k][m]))
void launch_z_odd_L(const ZInst* d, const int* d_begin, int n_inst, int total, hipStream_t s);
void launch_z_divdiff(const ZInst* d, const int* d_begin, int n_inst, int total, hipStream_t s);
void launch_z_grad(const ZInst* d, const int* d_begin, int n_inst, int total, int* status, hipStream_t s);

// ---------------------------------------------------------------------------
// Preconditioner set-up of the L-BFGS driver (FP64)
// ---------------------------------------------------------------------------
// Per instance of the preconditioner set-up: n0 = diag(C0 F C0^H), eps_i =
// Re (C0^H H(n) C0)_ii with H(n) = H0 + U diag(nH) (nH: own n0 or the coupled sum),
// h and w over the instance's slice of the free variables.
struct PrecInst {
  const double* C0;
  const double* HC0;  // H0 C0
  const double* f;
  double* n0;
  const double* nH;
  double* eps;
  double* hd;
  double* wv;
  int32_t M, N;
  double w;
};
// One instance of the ov reference update C0 <- [C_occ | C_virt].
struct C0Inst {
  double* C0;
  const double* Cocc;
  const double* Cvirt;
  int32_t M, N;
};
// The whole batch: densities (rows offsets d_rows), optionally the coupled sum
// coupled_n = sum_k w_k n0_k (couple_M > 0), orbital energies, then h and w over the
// free variables (element offsets d_elems: N (M - N) real, M^2 complex per instance).
void launch_prec_setup(const PrecInst* d, const int* d_rows, int total_rows, const int* d_elems, int total_elems,
                       int n_inst, int cplx, double U, const double* const* coupled_n0, const double* coupled_w,
                       double* coupled_n, int couple_M, hipStream_t s);
void launch_c0_update(const C0Inst* d, const int* d_begin, int n_inst, int total, hipStream_t s);
void launch_fill(double* x, int64_t n, double v, hipStream_t s);

void launch_weighted_vsum(const double* const* xs, const double* ws, int n, int M, double* out, hipStream_t s);

}  // namespace etdm
