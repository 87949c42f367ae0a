// Internal declarations shared by the HIP kernels and the host orchestration.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace etdm {

// ---------------------------------------------------------------------------
// grouped GEMM problems (row-major operands)
//   C = alpha * op(A) op(B) + alpha2 * op(A2) op(B2) + beta * D
// op(A) is m x k, op(B) is k x n (second segment: k2).  All problems of one
// launch share the transposition flags.  Every workgroup computes one 64 x 64
// tile; tile_begin is the prefix sum of tiles over the problem list, and the
// launch's tile table maps each workgroup to its problem.
// ---------------------------------------------------------------------------
struct GemmProb {
  const double* A;
  const double* B;
  const double* A2;
  const double* B2;
  const double* D;
  double* C;
  int64_t lda, ldb, lda2, ldb2, ldd, ldc;
  int32_t m, n, k, k2;
  double alpha, alpha2, beta;
  int32_t tiles_n, tile_begin;
};

enum GemmPrec : int32_t { GP_FP64 = 0, GP_FP32 = 1, GP_BF16X3 = 2, GP_BF16X6 = 3 };
enum GemmOp : int32_t { OP_N = 0, OP_T = 1, OP_C = 2 };  // C = conjugate transpose

constexpr int GEMM_BM = 64;
constexpr int GEMM_BN = 64;

// Real grouped GEMM; opA/opB in {OP_N, OP_T}.
void launch_gemm(const GemmProb* d_probs, const int* d_tile_prob, int total_tiles, int opA, int opB, int prec,
                 hipStream_t s);
// Complex (interleaved re,im float64) grouped GEMM; the double pointers in the
// problems address complex elements, leading dimensions count complex elements,
// alpha/alpha2/beta are real.  opA/opB in {OP_N, OP_T, OP_C}.
void launch_zgemm(const GemmProb* d_probs, const int* d_tile_prob, int total_tiles, int opA, int opB,
                  hipStream_t s);

// ---------------------------------------------------------------------------
// split-precision GEMM on pre-split operands (large problems, gemm_split.hip)
// ---------------------------------------------------------------------------
constexpr int PK_R = 64;  // rows per panel of a packed operand
constexpr int PK_K = 32;  // k per k-tile
constexpr int PK_S = 3;   // BF16 slices per value
// Pack op(X) = alpha * (trans ? X^T : X) (rows x K, FP64 row-major X with leading
// dimension ld) into k-tiles [kt0, kt0 + ceil(K / 32)) of a packed operand with
// ktiles k-tiles per panel.  The job covers whole tiles of panels (zero rows past
// the end); begin is the prefix sum of chunks (panels x kt_n) over the jobs, and
// the launch's chunk table maps each workgroup to its job.
// dst: BF16 slices (split_pack) or FP64 values (copy_pack64).
struct PackJob {
  const double* src;
  void* dst;
  int64_t ld;
  double alpha;
  int32_t trans, rows, K, kt0, ktiles, kt_n, begin;
  // complex operands (interleaved, ld in complex elements) packed as their real view:
  // cplx 1: op(A) (m x k) as the m x 2k matrix [Re a_il, Im a_il]; cplx 2: op(B) (k x n)
  // as the rows of the 2k x 2n matrix [[Re, Im], [-Im, Re]] transposed, so that the real
  // product of the two is the interleaved complex product; op is OP_N, OP_T or OP_C
  int32_t cplx, op;
};
// C (m x n, FP64) = sum over k of A[i][k] B[j][k] + beta D for packed A (m rows) and
// B (n rows) with ktiles k-tiles, in tiles of tpm x tpn panels (64 tpm rows, 64 tpn
// columns); begin = prefix sum of tiles.  The tile table of a launch of `total` tiles
// holds 2 total entries: [0, total) tile -> problem, [total, 2 total) workgroup ->
// tile (the order in which the plan deals the tiles out to the XCDs).
struct SplitProb {
  const void* A;
  const void* B;
  const double* D;
  double* C;
  int64_t ldc, ldd;
  double beta;
  int32_t m, n, ktiles, tiles_m, tiles_n, begin;
};
constexpr int PK_CHUNK_X6 = PK_S * PK_R * PK_K;  // BF16 values of a split chunk
constexpr int PK_CHUNK_64 = PK_R * PK_K;         // FP64 values of an FP64 chunk
void launch_split_pack(const PackJob* d_jobs, const int* d_chunk_job, int chunks, hipStream_t s);
void launch_copy_pack64(const PackJob* d_jobs, const int* d_chunk_job, int chunks, hipStream_t s);
// tiles of tpm x tpn panels of 64 (tpm, tpn in {1, 2})
void launch_gemm_f64_packed(int tpm, int tpn, const SplitProb* d_probs, const int* d_tile_prob, int tiles,
                            hipStream_t s);
void launch_gemm_x6_packed(int tpm, int tpn, const SplitProb* d_probs, const int* d_tile_prob, int tiles,
                           hipStream_t s);

// ---------------------------------------------------------------------------
// Jacobi eigensolver (FP64), one workgroup per matrix
// ---------------------------------------------------------------------------
struct EighProb {
  double* A;    // n x n (real) or complex n x n; destroyed (diagonalized in place)
  double* V;    // n x n eigenvectors (columns), same element type as A
  double* w;    // n eigenvalues (unsorted)
  int32_t n;
  int32_t lds;  // 1: small real problem solved in LDS (n <= EIGH_LDS_MAX)
  double* ws;   // complex tridiagonal path: Q^H (complex n x n)
  int* ok;      // complex tridiagonal path: 1 when its result passed the checks (the
                // Jacobi solver skips such problems), else 0
};
constexpr int EIGH_LDS_MAX = 88;
// dynamic LDS bytes of the staged real solver for size n
size_t eigh_lds_bytes(int n);
void launch_eigh_real_lds(const EighProb* d_probs, int nprob, int* d_status, hipStream_t s);
void launch_eigh_complex(const EighProb* d_probs, int nprob, int nmax, int* d_status, hipStream_t s);

// Complex Hermitian eigensolver by reduction to real tridiagonal form (n <= HT_MAX),
// one workgroup per matrix: writes the eigenvalues, the real eigenvectors Z of T
// into the first n*n doubles of V, the reflectors into ws (n x n complex: v_k in
// column k, tau_k at [k][n-1]) and the acceptance flag *ok.
constexpr int HT_MAX = 512;
constexpr int HT_NB = 32;  // reflectors per compact-WY block of the back-transform
struct HermWY {
  const double* Y;  // reflectors (as written by the solver)
  double* T;        // ceil((n-1)/HT_NB) blocks of HT_NB x HT_NB complex
  int n;
};
// T factors of all blocks (grid: instances x blocks).
void launch_herm_wy_t(const HermWY* d, int nprob, int nblk, hipStream_t s);
void launch_eigh_herm_tridiag(const EighProb* d_probs, int nprob, int nmax, int* d_status, hipStream_t s);
// After G = Z^T Z: *ok &= max|G - I| <= 1e-6, and G <- (3 I - G) / 2 in place.
struct HermCheck {
  double* G;
  int* ok;
  int n;
};
void launch_herm_check(const HermCheck* d, int nprob, hipStream_t s);
// Complex copy (imaginary part 0) of real n x n matrices.
struct RealToComplex {
  const double* src;
  double* dst;
  int n;
};
void launch_real_to_complex(const RealToComplex* d, int nprob, hipStream_t s);

// device status bits
enum : int { ST_EIGH = 1, ST_NONFINITE = 2 };

}  // namespace etdm
