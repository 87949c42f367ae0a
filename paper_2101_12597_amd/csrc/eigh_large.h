// Large symmetric eigensolver (block-cyclic Jacobi with matrix-core updates).
#pragma once

#include <algorithm>

#include "common.h"

namespace etdm {

struct EighLargeState {
  double scale;                  // ||A||_F
  unsigned long long sweep_off;  // bit pattern of the largest off-diagonal |a_ik| after the sweep
  int sweeps;
  int done;
  int finite;
};

struct EighLarge {
  const double* P;  // n x n input (its symmetric part is used)
  double* X;        // n x n eigenvectors (columns)
  double* w;        // n eigenvalues (unsorted)
  double* Aw;       // npad x npad work matrix
  double* Vw;       // npad x npad accumulated rotations
  double* Qb;       // (nb / 2) x 64 x 64 rotations of one round
  double* partial;  // reduction scratch (256 doubles)
  EighLargeState* st;
  int n, npad, nb;
  // reduction to tridiagonal form, tried first (the Jacobi sweeps are its fallback);
  // it reuses Aw (work matrix, ld n; later Z^T Z) and Vw (reflectors, ld n: v_k in
  // column k below row k, tau_k at [k][n-1])
  double* Zw;       // n x n eigenvectors of T
  double* Ps;       // n x n symmetric part of P (for the final residual check)
  double* d;        // n: diagonal of T
  double* e;        // n: off-diagonal of T
  double* pv;       // 3 x n: tau A v of a step (buffers by step mod 3; tb_reduce uses two)
  double* rowbuf;   // 3 x n: look-ahead rows (buffers by row index mod 3; tb_reduce uses two)
  double* W1;       // nkc x TB_NBW x n compact-WY scratch: the partial products Y_b^T X of
                    // the TB_KC-row chunks of a block, stacked (chunk c at row c m_b)
  double* W2;       // TB_NBW x n
  double* Tw;       // ceil((n-1)/TB_NBW) blocks of TB_NBW x (nkc TB_NBW) compact-WY factors:
                    // T_b (m_b x m_b) repeated nkc times side by side (at columns c m_b)
  double* Gw;       // the same number of Gram matrices Y_b^T Y_b (m_b x m_b, ld m_b)
  unsigned* bar;    // grid synchronization words: [2] abort, [64 ..) arrival flags of the workgroups
  int* ok;          // 1 when the tridiagonal result passed its checks
  double* scan;     // 4: maxima / sums of the grid-wide checks
  double* blo;      // n: eigenvalue brackets of T
  double* bhi;      // n
  int* bb;          // 2 n: unreduced block [b0, b1) of each eigenvalue
  int grid;         // workgroups of the reduction (one per CU, all resident)
  int nkc;          // ceil((n - 1) / TB_KC): most K chunks of a block's Y_b^T X
};

constexpr int TB_NBW = 64;   // reflectors per compact-WY block of the back-transform
constexpr int TB_KC = 256;   // K chunk of Y_b^T X (split K, so that the product fills the GPU)

// float64 elements of workspace for size n; npad returned.
size_t eigh_large_workspace(int n, size_t* npad_out);
// Point the members of e at the workspace ws (n set; grid from the CU count).
void eigh_large_layout(EighLarge& e, double* ws, EighLargeState* st, int cu_count);
// Tridiagonal path, part 1: the reduction (cooperative: every workgroup must be
// resident, so nothing else should be queued beside it), then the eigenpairs of T
// (Zw, w) and their residual check.  Part 2 (orthogonality check, one Newton-Schulz
// step into X, compact-WY back-transform of X) is launched by the caller with
// grouped GEMMs; launch_tb_wy_t forms the T factors from the Gram matrices in Gw.
void launch_tb_reduce(const EighLarge& e, hipStream_t s);
void launch_tb_eigenpairs(const EighLarge& e, hipStream_t s);
void launch_tb_wy_t(const EighLarge& e, hipStream_t s);
// X <- Q X in one launch (the panel of 16 columns of X per workgroup in registers),
// after launch_tb_wy_t; for n up to tb_apply_wy_fits (else the grouped GEMM blocks).
bool tb_apply_wy_fits(int n);
void launch_tb_apply_wy(const EighLarge& e, hipStream_t s);
// After G = Z^T Z has been formed in Aw: *ok = 0 unless max|G - I| <= 1e-6; Aw <- (I - G) / 2
// (the Newton-Schulz step is then X = Z + Z Aw).
void launch_tb_orth_check(const EighLarge& e, hipStream_t s);
// After R = sym(P) X has been formed in Aw: *ok = 0 unless max|R - X diag(w)| <= 1e-11 ||sym(P)||_F.
void launch_tb_final_check(const EighLarge& e, hipStream_t s);
// Launch the whole solve on stream s.  With check_host the host reads the
// convergence flag after every sweep and stops launching early (not usable
// under graph capture); otherwise all max_sweeps sweeps are launched and the
// ones after convergence return immediately.
void launch_eigh_large(const EighLarge& e, int max_sweeps, int* status, hipStream_t s, bool check_host);

}  // namespace etdm
