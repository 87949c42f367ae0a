// Grouped GEMM kernels on CDNA4 matrix cores (gfx950).
//
// One workgroup (4 wavefronts of 64 lanes) computes one 64 x 64 tile of one
// problem of a grouped launch; each wavefront owns a 32 x 32 quarter made of
// 2 x 2 MFMA 16x16 blocks.  Operands are staged through LDS in k-major order so
// that the 16 lanes that share an MFMA k-slice read consecutive addresses.
//
// Precision modes of the real kernel (operands always arrive as float64):
//   FP64    v_mfma_f64_16x16x4_f64, FP64 accumulation
//   FP32    operands rounded to FP32 on the way into LDS, v_mfma_f32_16x16x4_f32,
//           the FP32 accumulators are added into FP64 registers every 128 k
//   BF16X3  x = hi + lo (BF16, round-to-nearest-even splits), products
//   BF16X6  hi*hi + hi*lo + lo*hi (+ hi*md, md*hi, md*md for the 3-way split
//           x = hi + md + lo), v_mfma_f32_16x16x32_bf16, FP64 flush every 128 k
//
// MFMA operand layout used below (16x16xK blocks, lane l of the wavefront):
//   A operand: row l % 16, k slice l / 16;  B operand: column l % 16, same slice;
//   accumulator element r of lane l, FP32 results (f32 and bf16 inputs):
//     row 4 * (l / 16) + r, column l % 16;
//   accumulator element r of lane l, FP64 16x16x4:
//     row l / 16 + 4 * r, column l % 16.
#include <type_traits>

#include "common.h"
#include "reduce.h"

namespace etdm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int BM = GEMM_BM, BN = GEMM_BN;
constexpr int NTHREADS = 256;
constexpr int FLUSH_K = 128;

// ---------------------------------------------------------------------------
// operand staging: element (r, c) of op(X) for a row-major X
// ---------------------------------------------------------------------------
template <bool T>
__device__ __forceinline__ double ld_op(const double* __restrict__ X, int64_t ld, int r, int c,
                                        int rows, int cols) {
  if (r >= rows || c >= cols) return 0.0;
  return T ? X[(int64_t)c * ld + r] : X[(int64_t)r * ld + c];
}

// Fill an LDS tile S[kk][mm] (kk < BK, mm < BM) with op(A)[row0 + mm][k0 + kk].
// The thread -> element map follows the contiguous direction in memory.
template <bool TA, int BK, typename F>
__device__ __forceinline__ void stage_a(const double* __restrict__ A, int64_t lda, int row0, int k0,
                                        int m, int K, F&& put) {
  for (int e = threadIdx.x; e < BM * BK; e += NTHREADS) {
    int mm, kk;
    if (TA) { kk = e / BM; mm = e % BM; }
    else { mm = e / BK; kk = e % BK; }
    put(kk, mm, ld_op<TA>(A, lda, row0 + mm, k0 + kk, m, K));
  }
}

// Fill S[kk][nn] with op(B)[k0 + kk][col0 + nn].
template <bool TB, int BK, typename F>
__device__ __forceinline__ void stage_b(const double* __restrict__ B, int64_t ldb, int k0, int col0,
                                        int K, int n, F&& put) {
  for (int e = threadIdx.x; e < BN * BK; e += NTHREADS) {
    int nn, kk;
    if (TB) { nn = e / BK; kk = e % BK; }
    else { kk = e / BN; nn = e % BN; }
    put(kk, nn, ld_op<TB>(B, ldb, k0 + kk, col0 + nn, K, n));
  }
}

// row of accumulator element r of this lane inside a 16 x 16 block
template <bool F64>
__device__ __forceinline__ int acc_row(int lane, int r) {
  return F64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
}

template <bool F64>
__device__ __forceinline__ void store_tile(const GemmProb& p, int row0, int col0, int wm, int wn,
                                           const double (&acc)[2][2][4]) {
  const int lane = threadIdx.x & 63;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        int row = row0 + wm + i * 16 + acc_row<F64>(lane, r);
        int col = col0 + wn + j * 16 + (lane & 15);
        if (row < p.m && col < p.n) {
          double v = acc[i][j][r];
          if (p.beta != 0.0) v += p.beta * p.D[(int64_t)row * p.ldd + col];
          p.C[(int64_t)row * p.ldc + col] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// FP64 / FP32 kernel (16x16x4 MFMA, BK = 32)
//
// The next k-tile is fetched into registers while the MFMAs consume the current
// one from LDS.  LDS layouts follow the contiguous direction of each operand in
// memory so that the staging stores are conflict free:
//   op(A) = A   : A_s[m][k], row length BK + 1     op(A) = A^T : A_s[k][m], row length BM + 16
//   op(B) = B   : B_s[k][n], row length BN + 16    op(B) = B^T : B_s[n][k], row length BK + 1
// ---------------------------------------------------------------------------
constexpr int K4_BK = 32;
constexpr int K4_PER = GEMM_BM * K4_BK / NTHREADS;  // staged elements per thread and operand
constexpr int K4_LDS = (K4_BK * (GEMM_BM + 16) > GEMM_BM * (K4_BK + 1)) ? K4_BK * (GEMM_BM + 16)
                                                                          : GEMM_BM * (K4_BK + 1);

template <bool TA>
__device__ __forceinline__ int a_lds(int kk, int mm) {
  return TA ? kk * (GEMM_BM + 16) + mm : mm * (K4_BK + 1) + kk;
}
template <bool TB>
__device__ __forceinline__ int b_lds(int kk, int nn) {
  return TB ? nn * (K4_BK + 1) + kk : kk * (GEMM_BN + 16) + nn;
}
// element e of a 64 x 32 staging pass -> (kk, mm), following the memory-contiguous direction
template <bool T>
__device__ __forceinline__ void stage_coord(int e, int& kk, int& mm) {
  if (T) { kk = e / GEMM_BM; mm = e % GEMM_BM; }
  else { mm = e / K4_BK; kk = e % K4_BK; }
}

template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(NTHREADS) void gemm_k4(const GemmProb* __restrict__ probs, const int* __restrict__ tile_prob) {
  constexpr int BK = K4_BK;
  __shared__ T As[K4_LDS];
  __shared__ T Bs[K4_LDS];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const GemmProb& p = probs[tile_prob[tile]];
  const int t = tile - p.tile_begin;
  const int row0 = (t / p.tiles_n) * BM, col0 = (t % p.tiles_n) * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;

  double acc[2][2][4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
  const bool live_m[2] = {row0 + wm < p.m, row0 + wm + 16 < p.m};
  const bool live_n[2] = {col0 + wn < p.n, col0 + wn + 16 < p.n};
  const bool interior = live_m[1] && live_n[1];

  for (int seg = 0; seg < 2; ++seg) {
    const double* A = seg ? p.A2 : p.A;
    const double* B = seg ? p.B2 : p.B;
    const int64_t lda = seg ? p.lda2 : p.lda, ldb = seg ? p.ldb2 : p.ldb;
    const int K = seg ? p.k2 : p.k;
    const double alpha = seg ? p.alpha2 : p.alpha;
    if (K <= 0) continue;
    double ra[K4_PER], rb[K4_PER];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int i = 0; i < K4_PER; ++i) {
        int kk, mm;
        stage_coord<TA>(threadIdx.x + i * NTHREADS, kk, mm);
        ra[i] = ld_op<TA>(A, lda, row0 + mm, k0 + kk, p.m, K);
        int kb, nn;
        stage_coord<TB>(threadIdx.x + i * NTHREADS, kb, nn);
        rb[i] = ld_op<TB>(B, ldb, k0 + kb, col0 + nn, K, p.n);
      }
    };
    auto commit = [&]() {
#pragma unroll
      for (int i = 0; i < K4_PER; ++i) {
        int kk, mm;
        stage_coord<TA>(threadIdx.x + i * NTHREADS, kk, mm);
        As[a_lds<TA>(kk, mm)] = (T)(alpha * ra[i]);
        int kb, nn;
        stage_coord<TB>(threadIdx.x + i * NTHREADS, kb, nn);
        Bs[b_lds<TB>(kb, nn)] = (T)rb[i];
      }
    };
    using V4 = typename std::conditional<sizeof(T) == 8, d4, f4>::type;
    V4 c[2][2];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) c[i][j] = V4{0, 0, 0, 0};
    int since_flush = 0;
    auto flush = [&]() {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)c[i][j][r];
          c[i][j] = V4{0, 0, 0, 0};
        }
      since_flush = 0;
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
      commit();
      __syncthreads();
      if (k0 + BK < K) fetch(k0 + BK);
      // 16 x 16 sub-tiles wholly outside C take no MFMAs (wavefront-uniform test;
      // interior tiles run the unguarded loop)
      auto step = [&](auto guarded) {
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
          const T a[2] = {As[a_lds<TA>(ks + lk, wm + lr)], As[a_lds<TA>(ks + lk, wm + 16 + lr)]};
          const T b[2] = {Bs[b_lds<TB>(ks + lk, wn + lr)], Bs[b_lds<TB>(ks + lk, wn + 16 + lr)]};
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              if (decltype(guarded)::value && !(live_m[i] && live_n[j])) continue;
              if constexpr (sizeof(T) == 8)
                c[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], c[i][j], 0, 0, 0);
              else
                c[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], c[i][j], 0, 0, 0);
            }
        }
      };
      if (interior) step(std::false_type{});
      else step(std::true_type{});
      __syncthreads();
      if constexpr (sizeof(T) == 4) {
        since_flush += BK;
        if (since_flush >= FLUSH_K) flush();
      }
    }
    flush();
  }
  store_tile<sizeof(T) == 8>(p, row0, col0, wm, wn, acc);
}

// ---------------------------------------------------------------------------
// BF16 split kernel (16x16x32 MFMA, BK = 32).  NS = number of BF16 slices
// (2 or 3); the products kept are those with slice indices i + j < NS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ __bf16 to_bf16_rne(float x) { return (__bf16)x; }

template <int NS>
__device__ __forceinline__ void split_bf16(double v, __bf16 (&out)[NS]) {
  // x = s0 + s1 (+ s2), every slice rounded to nearest even; the remainder of
  // each step is formed exactly in FP64.
  double r = v;
  for (int i = 0; i < NS; ++i) {
    __bf16 h = to_bf16_rne((float)r);
    out[i] = h;
    r -= (double)(float)h;
  }
}

// Staging task of one thread for a 64 x 32 tile: one row (or column) and one
// octet of 8 consecutive k.  The map follows the contiguous direction in memory:
// consecutive threads take consecutive octets of one row when k is contiguous,
// and consecutive rows of one octet when the row index is contiguous.
template <bool KCONTIG>
__device__ __forceinline__ void octet_task(int t, int& row, int& oct) {
  if (KCONTIG) { row = t >> 2; oct = t & 3; }
  else { row = t & 63; oct = t >> 6; }
}

template <int NS, bool TA, bool TB>
__global__ __launch_bounds__(NTHREADS) void gemm_bf16split(const GemmProb* __restrict__ probs, const int* __restrict__ tile_prob) {
  constexpr int BK = 32;
  // slice-major k-blocked layout: S[slice][kk / 8][row][kk % 8] so that one lane
  // reads its 8 consecutive k values of one row as a single 16-byte vector
  __shared__ __attribute__((aligned(16))) __bf16 As[NS][BK / 8][BM][8];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[NS][BK / 8][BN][8];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const GemmProb& p = probs[tile_prob[tile]];
  const int t = tile - p.tile_begin;
  const int row0 = (t / p.tiles_n) * BM, col0 = (t % p.tiles_n) * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  int arow, aoct, bcol, boct;
  octet_task<!TA>(threadIdx.x, arow, aoct);
  octet_task<TB>(threadIdx.x, bcol, boct);

  double acc[2][2][4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;

  for (int seg = 0; seg < 2; ++seg) {
    const double* A = seg ? p.A2 : p.A;
    const double* B = seg ? p.B2 : p.B;
    const int64_t lda = seg ? p.lda2 : p.lda, ldb = seg ? p.ldb2 : p.ldb;
    const int K = seg ? p.k2 : p.k;
    const double alpha = seg ? p.alpha2 : p.alpha;
    if (K <= 0) continue;
    double ra[8], rb[8];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        ra[u] = ld_op<TA>(A, lda, row0 + arow, k0 + aoct * 8 + u, p.m, K);
        rb[u] = ld_op<TB>(B, ldb, k0 + boct * 8 + u, col0 + bcol, K, p.n);
      }
    };
    auto commit = [&]() {
      bf8 sa[NS], sb[NS];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        __bf16 x[NS], y[NS];
        split_bf16<NS>(alpha * ra[u], x);
        split_bf16<NS>(rb[u], y);
        for (int q = 0; q < NS; ++q) {
          sa[q][u] = x[q];
          sb[q][u] = y[q];
        }
      }
      for (int q = 0; q < NS; ++q) {
        *reinterpret_cast<bf8*>(&As[q][aoct][arow][0]) = sa[q];
        *reinterpret_cast<bf8*>(&Bs[q][boct][bcol][0]) = sb[q];
      }
    };
    f4 c[2][2];
    int since_flush = 0;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) c[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    auto flush = [&]() {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)c[i][j][r];
          c[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
      since_flush = 0;
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
      commit();
      __syncthreads();
      if (k0 + BK < K) fetch(k0 + BK);
      bf8 a[NS][2], b[NS][2];
      for (int q = 0; q < NS; ++q) {
        a[q][0] = *reinterpret_cast<const bf8*>(&As[q][lk][wm + lr][0]);
        a[q][1] = *reinterpret_cast<const bf8*>(&As[q][lk][wm + 16 + lr][0]);
        b[q][0] = *reinterpret_cast<const bf8*>(&Bs[q][lk][wn + lr][0]);
        b[q][1] = *reinterpret_cast<const bf8*>(&Bs[q][lk][wn + 16 + lr][0]);
      }
      // smallest products first so they are not absorbed by the large ones
#pragma unroll
      for (int sum = NS - 1; sum >= 0; --sum)
#pragma unroll
        for (int qa = 0; qa < NS; ++qa) {
          const int qb = sum - qa;
          if (qb < 0 || qb >= NS) continue;
          for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
              c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[qa][i], b[qb][j], c[i][j], 0, 0, 0);
        }
      __syncthreads();
      since_flush += BK;
      if (since_flush >= FLUSH_K) flush();
    }
    flush();
  }
  store_tile<false>(p, row0, col0, wm, wn, acc);
}

// ---------------------------------------------------------------------------
// complex FP64 kernel: 4 real MFMAs per block and k-step
// ---------------------------------------------------------------------------
template <int OP>
__device__ __forceinline__ double2 ld_zop(const double2* __restrict__ X, int64_t ld, int r, int c,
                                          int rows, int cols) {
  if (r >= rows || c >= cols) return make_double2(0.0, 0.0);
  if (OP == OP_N) return X[(int64_t)r * ld + c];
  double2 v = X[(int64_t)c * ld + r];
  if (OP == OP_C) v.y = -v.y;
  return v;
}

template <int OPA, int OPB>
__global__ __launch_bounds__(NTHREADS) void zgemm_k4(const GemmProb* __restrict__ probs, const int* __restrict__ tile_prob) {
  constexpr int BK = 16;
  static_assert(BM * BK % NTHREADS == 0 && BN * BK % NTHREADS == 0, "whole k-tiles per thread");
  __shared__ double Ar[BK][BM + 1], Ai[BK][BM + 1];
  __shared__ double Br[BK][BN + 1], Bi[BK][BN + 1];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const GemmProb& p = probs[tile_prob[tile]];
  const int t = tile - p.tile_begin;
  const int row0 = (t / p.tiles_n) * BM, col0 = (t % p.tiles_n) * BN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;

  d4 cr[2][2], ci[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      ci[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  const bool live_m[2] = {row0 + wm < p.m, row0 + wm + 16 < p.m};
  const bool live_n[2] = {col0 + wn < p.n, col0 + wn + 16 < p.n};
  const bool interior = live_m[1] && live_n[1];
  for (int seg = 0; seg < 2; ++seg) {
    const double2* A = reinterpret_cast<const double2*>(seg ? p.A2 : p.A);
    const double2* B = reinterpret_cast<const double2*>(seg ? p.B2 : p.B);
    const int64_t lda = seg ? p.lda2 : p.lda, ldb = seg ? p.ldb2 : p.ldb;
    const int K = seg ? p.k2 : p.k;
    const double alpha = seg ? p.alpha2 : p.alpha;
    if (K <= 0) continue;
    // software pipeline: the next k-tile's global loads are issued into registers
    // before the MFMAs of the current one
    constexpr int EA = BM * BK / NTHREADS, EB = BN * BK / NTHREADS;
    double2 ra[EA], rb[EB];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int e = threadIdx.x + u * NTHREADS;
        int mm, kk;
        if (OPA != OP_N) { kk = e / BM; mm = e % BM; }
        else { mm = e / BK; kk = e % BK; }
        ra[u] = ld_zop<OPA>(A, lda, row0 + mm, k0 + kk, p.m, K);
      }
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        const int e = threadIdx.x + u * NTHREADS;
        int nn, kk;
        if (OPB != OP_N) { nn = e / BK; kk = e % BK; }
        else { kk = e / BN; nn = e % BN; }
        rb[u] = ld_zop<OPB>(B, ldb, k0 + kk, col0 + nn, K, p.n);
      }
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int e = threadIdx.x + u * NTHREADS;
        int mm, kk;
        if (OPA != OP_N) { kk = e / BM; mm = e % BM; }
        else { mm = e / BK; kk = e % BK; }
        Ar[kk][mm] = alpha * ra[u].x;
        Ai[kk][mm] = alpha * ra[u].y;
      }
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        const int e = threadIdx.x + u * NTHREADS;
        int nn, kk;
        if (OPB != OP_N) { nn = e / BK; kk = e % BK; }
        else { kk = e / BN; nn = e % BN; }
        Br[kk][nn] = rb[u].x;
        Bi[kk][nn] = rb[u].y;
      }
      __syncthreads();
      if (k0 + BK < K) fetch(k0 + BK);
      // 16 x 16 sub-tiles wholly outside C (the ragged edge) take no MFMAs; the test is
      // uniform per wavefront, and interior tiles run the unguarded loop
      auto step = [&](auto guarded) {
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
          double ar[2], ai[2], nai[2], br[2], bi[2];
          for (int i = 0; i < 2; ++i) {
            ar[i] = Ar[ks + lk][wm + i * 16 + lr];
            ai[i] = Ai[ks + lk][wm + i * 16 + lr];
            nai[i] = -ai[i];
            br[i] = Br[ks + lk][wn + i * 16 + lr];
            bi[i] = Bi[ks + lk][wn + i * 16 + lr];
          }
          for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
              if (decltype(guarded)::value && !(live_m[i] && live_n[j])) continue;
              cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cr[i][j], 0, 0, 0);
              cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[i], bi[j], cr[i][j], 0, 0, 0);
              ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], ci[i][j], 0, 0, 0);
              ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], ci[i][j], 0, 0, 0);
            }
        }
      };
      if (interior) step(std::false_type{});
      else step(std::true_type{});
      __syncthreads();
    }
  }
  double2* C = reinterpret_cast<double2*>(p.C);
  const double2* D = reinterpret_cast<const double2*>(p.D);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        int row = row0 + wm + i * 16 + acc_row<true>(lane, r);
        int col = col0 + wn + j * 16 + (lane & 15);
        if (row < p.m && col < p.n) {
          double2 v = make_double2(cr[i][j][r], ci[i][j][r]);
          if (p.beta != 0.0) {
            double2 d = D[(int64_t)row * p.ldd + col];
            v.x += p.beta * d.x;
            v.y += p.beta * d.y;
          }
          C[(int64_t)row * p.ldc + col] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <bool TA, bool TB>
static void launch_real(const GemmProb* d, const int* tp, int tiles, int prec, hipStream_t s) {
  switch (prec) {
    case GP_FP64: gemm_k4<double, TA, TB><<<tiles, NTHREADS, 0, s>>>(d, tp); break;
    case GP_FP32: gemm_k4<float, TA, TB><<<tiles, NTHREADS, 0, s>>>(d, tp); break;
    case GP_BF16X3: gemm_bf16split<2, TA, TB><<<tiles, NTHREADS, 0, s>>>(d, tp); break;
    default: gemm_bf16split<3, TA, TB><<<tiles, NTHREADS, 0, s>>>(d, tp); break;
  }
}

void launch_gemm(const GemmProb* d_probs, const int* d_tile_prob, int total_tiles, int opA, int opB, int prec,
                 hipStream_t s) {
  if (total_tiles <= 0) return;
  if (opA == OP_N && opB == OP_N) launch_real<false, false>(d_probs, d_tile_prob, total_tiles, prec, s);
  else if (opA == OP_N) launch_real<false, true>(d_probs, d_tile_prob, total_tiles, prec, s);
  else if (opB == OP_N) launch_real<true, false>(d_probs, d_tile_prob, total_tiles, prec, s);
  else launch_real<true, true>(d_probs, d_tile_prob, total_tiles, prec, s);
}

template <int OPA>
static void launch_z_b(const GemmProb* d, const int* tp, int tiles, int opB, hipStream_t s) {
  switch (opB) {
    case OP_N: zgemm_k4<OPA, OP_N><<<tiles, NTHREADS, 0, s>>>(d, tp); break;
    case OP_T: zgemm_k4<OPA, OP_T><<<tiles, NTHREADS, 0, s>>>(d, tp); break;
    default: zgemm_k4<OPA, OP_C><<<tiles, NTHREADS, 0, s>>>(d, tp); break;
  }
}

void launch_zgemm(const GemmProb* d_probs, const int* d_tile_prob, int total_tiles, int opA, int opB,
                  hipStream_t s) {
  if (total_tiles <= 0) return;
  switch (opA) {
    case OP_N: launch_z_b<OP_N>(d_probs, d_tile_prob, total_tiles, opB, s); break;
    case OP_T: launch_z_b<OP_T>(d_probs, d_tile_prob, total_tiles, opB, s); break;
    default: launch_z_b<OP_C>(d_probs, d_tile_prob, total_tiles, opB, s); break;
  }
}

}  // namespace etdm
