// Split-precision GEMM for large problems on pre-split operands (gfx950).
//
// The BF16x6 product of the grouped GEMM in gemm.hip splits every FP64 operand
// element into three BF16 slices x = hi + md + lo inside each workgroup, so an
// element is split once per tile that reads it.  For large problems the split
// is done once instead, by split_pack, into a packed layout that the GEMM reads
// with plain 16-byte loads:
//
//   op(X) (rows x K) -> panels of PK_R = 64 rows, each a run of k-tiles of
//   PK_K = 32; one (panel, k-tile) chunk holds [slice][row][k] BF16 values,
//   3 x 64 x 32 x 2 bytes = 12 KB, contiguous.  Inside a row the four 8-value
//   octets are permuted by an XOR of the row index (pk_phys), so the MFMA
//   fragment reads of 16 consecutive rows hit distinct LDS banks.
//
// Rows are padded to a multiple of 128 and k to a multiple of 32 with zeros.  A
// problem with two K segments (C = a1 A1 B1 + a2 A2 B2) packs [a1 A1 | a2 A2] and
// [B1; B2] along k, so the GEMM sees one K.
//
// gemm_x6_packed: C = op(A) op(B) + beta D for packed op(A) and op(B)^T (both
// rows x K).  One workgroup of 4 wavefronts computes a 128 x 128 tile; each
// wavefront owns 64 x 64 as 4 x 4 blocks of v_mfma_f32_16x16x32_bf16 and
// accumulates the six slice products with i + j <= 2 in FP32, added into FP64
// registers every FLUSH k.  k-tiles of 32 are double-buffered in LDS (96 KB)
// with the next one fetched into registers during the MFMAs.
//
// The FP64 pair (copy_pack64, gemm_f64_packed) uses the same panels and tile
// order without the split: a chunk is [k][row] FP64 (64 x 32 x 8 bytes = 16 KB),
// so the 16 lanes that share a k of a v_mfma_f64_16x16x4f64 fragment read 128
// consecutive bytes; 128 KB of LDS double-buffer the k-tiles.
#include "common.h"

namespace etdm {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int PK_CHUNK = PK_CHUNK_X6;
constexpr int XT = 128;                        // workgroup tile (rows and columns)
constexpr int XNT = 256;
constexpr int X_FLUSH = 4;                     // k-tiles between FP64 flushes (128 k)
constexpr int X_GROUP = 4;                     // tile rows per group of the tile order

// octet position inside a 64-byte row: conflict free for 8 and for 16
// consecutive rows read at the same octet
__device__ __forceinline__ int pk_phys(int oct, int row) {
  return oct ^ (((row >> 1) ^ (row >> 3)) & 3);
}

template <typename J>
__device__ __forceinline__ int find_item(const J* __restrict__ v, int n, int bid) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (v[mid].begin <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace

// ---------------------------------------------------------------------------
// split_pack: one workgroup per (panel, k-tile) chunk of one job
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void split_pack(const PackJob* __restrict__ jobs, int njobs) {
  __shared__ double t[PK_R][PK_K + 1];
  const PackJob& j = jobs[find_item(jobs, njobs, blockIdx.x)];
  const int c = blockIdx.x - j.begin;
  const int panel = c / j.kt_n, q = c % j.kt_n;
  const int r0 = panel * PK_R, k0 = q * PK_K;
  if (!j.trans) {
    for (int e = threadIdx.x; e < PK_R * PK_K; e += 256) {
      const int r = e / PK_K, k = e % PK_K;
      const int gr = r0 + r, gk = k0 + k;
      t[r][k] = (gr < j.rows && gk < j.K) ? j.src[(int64_t)gr * j.ld + gk] : 0.0;
    }
  } else {
    for (int e = threadIdx.x; e < PK_R * PK_K; e += 256) {
      const int k = e / PK_R, r = e % PK_R;
      const int gr = r0 + r, gk = k0 + k;
      t[r][k] = (gr < j.rows && gk < j.K) ? j.src[(int64_t)gk * j.ld + gr] : 0.0;
    }
  }
  __syncthreads();
  const int r = threadIdx.x >> 2, oct = threadIdx.x & 3;
  bf8 out[PK_S];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    // x = s0 + s1 + s2 + O(2^-24 |x|), each slice rounded to nearest even; the
    // remainders are exact in FP64
    double x = j.alpha * t[r][oct * 8 + u];
#pragma unroll
    for (int s = 0; s < PK_S; ++s) {
      const __bf16 h = (__bf16)(float)x;
      out[s][u] = h;
      x -= (double)(float)h;
    }
  }
  __bf16* base = static_cast<__bf16*>(j.dst) + ((int64_t)panel * j.ktiles + j.kt0 + q) * PK_CHUNK;
#pragma unroll
  for (int s = 0; s < PK_S; ++s)
    *reinterpret_cast<bf8*>(base + (s * PK_R + r) * PK_K + pk_phys(oct, r) * 8) = out[s];
}

// ---------------------------------------------------------------------------
// gemm_x6_packed
// ---------------------------------------------------------------------------
// tile index inside one problem, grouped X_GROUP tile rows at a time so that the
// workgroups resident together share A and B panels
__device__ __forceinline__ void x6_tile(const SplitProb& p, int lt, int& tm, int& tn) {
  const int per_group = X_GROUP * p.tiles_n;
  const int g = lt / per_group;
  const int gr = min(X_GROUP, p.tiles_m - g * X_GROUP);
  const int idx = lt - g * per_group;
  tm = g * X_GROUP + idx % gr;
  tn = idx / gr;
}

__global__ __launch_bounds__(XNT) void gemm_x6_packed(const SplitProb* __restrict__ probs, int nprob,
                                                      int total) {
  extern __shared__ __attribute__((aligned(16))) __bf16 x6_lds[];
  // logical tile: workgroups are dealt to the 8 XCDs in turn, so consecutive
  // logical tiles are given to the workgroups of one XCD (shared L2)
  const int b = blockIdx.x, t8 = total & ~7;
  const int tile = b < t8 ? (b & 7) * (t8 >> 3) + (b >> 3) : b;
  const SplitProb& p = probs[find_item(probs, nprob, tile)];
  int tm, tn;
  x6_tile(p, tile - p.begin, tm, tn);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int pa = wave >> 1, pb = wave & 1;  // this wavefront's A and B panel inside the tile
  const int lr = lane & 15, lo = lane >> 4;

  // LDS: [buffer][operand][panel][slice][row][k]
  constexpr int OPER = 2 * PK_CHUNK;
  constexpr int BUF = 2 * OPER;
  const __bf16* Ag = static_cast<const __bf16*>(p.A) + (int64_t)(2 * tm) * p.ktiles * PK_CHUNK;
  const __bf16* Bg = static_cast<const __bf16*>(p.B) + (int64_t)(2 * tn) * p.ktiles * PK_CHUNK;
  const int64_t pstride = (int64_t)p.ktiles * PK_CHUNK;  // panel stride in the packed operand

  // staging: 2 operands x 2 panels x 768 pieces of 16 bytes; thread t takes
  // pieces t + 256 u (u < 6) of each operand
  i4 ra[6], rb[6];
  auto fetch = [&](int kt) {
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int e = threadIdx.x + u * XNT;
      const int pan = e / 768, w = e % 768;
      ra[u] = *reinterpret_cast<const i4*>(Ag + pan * pstride + (int64_t)kt * PK_CHUNK + w * 8);
      rb[u] = *reinterpret_cast<const i4*>(Bg + pan * pstride + (int64_t)kt * PK_CHUNK + w * 8);
    }
  };
  auto commit = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int e = threadIdx.x + u * XNT;
      const int pan = e / 768, w = e % 768;
      *reinterpret_cast<i4*>(x6_lds + buf * BUF + pan * PK_CHUNK + w * 8) = ra[u];
      *reinterpret_cast<i4*>(x6_lds + buf * BUF + OPER + pan * PK_CHUNK + w * 8) = rb[u];
    }
  };

  double acc[4][4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
  f4 c[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) c[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // fragment offset (BF16 elements) of 16-row block blk, slice s, inside a panel
  auto frag = [&](int s, int blk) {
    const int row = blk * 16 + lr;
    return (s * PK_R + row) * PK_K + pk_phys(lo, row) * 8;
  };

  if (p.ktiles > 0) {
    fetch(0);
    commit(0);
  }
  __syncthreads();
  for (int kt = 0; kt < p.ktiles; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < p.ktiles) fetch(kt + 1);
    const __bf16* As = x6_lds + buf * BUF + pa * PK_CHUNK;
    const __bf16* Bs = x6_lds + buf * BUF + OPER + pb * PK_CHUNK;
    bf8 bv[PK_S][4];
#pragma unroll
    for (int s = 0; s < PK_S; ++s)
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[s][j] = *reinterpret_cast<const bf8*>(Bs + frag(s, j));
    // A slice sa meets the B slices sb <= 2 - sa; lowest-order products first
#pragma unroll
    for (int sa = PK_S - 1; sa >= 0; --sa) {
      bf8 av[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = *reinterpret_cast<const bf8*>(As + frag(sa, i));
#pragma unroll
      for (int sb = PK_S - 1 - sa; sb >= 0; --sb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[sb][j], c[i][j], 0, 0, 0);
    }
    if (kt + 1 < p.ktiles) commit(buf ^ 1);
    if ((kt + 1) % X_FLUSH == 0 || kt + 1 == p.ktiles) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)c[i][j][r];
          c[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    __syncthreads();
  }

  // epilogue: element r of lane l of block (i, j) is row 4 (l / 16) + r, column l % 16
  const int row0 = tm * XT + pa * 64, col0 = tn * XT + pb * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + i * 16 + 4 * lo + r, col = col0 + j * 16 + lr;
        if (row < p.m && col < p.n) {
          double v = acc[i][j][r];
          if (p.beta != 0.0) v += p.beta * p.D[(int64_t)row * p.ldd + col];
          p.C[(int64_t)row * p.ldc + col] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// copy_pack64 / gemm_f64_packed
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void copy_pack64(const PackJob* __restrict__ jobs, int njobs) {
  __shared__ double t[PK_R][PK_K + 1];
  const PackJob& j = jobs[find_item(jobs, njobs, blockIdx.x)];
  const int c = blockIdx.x - j.begin;
  const int panel = c / j.kt_n, q = c % j.kt_n;
  const int r0 = panel * PK_R, k0 = q * PK_K;
  if (!j.trans) {
    for (int e = threadIdx.x; e < PK_R * PK_K; e += 256) {
      const int r = e / PK_K, k = e % PK_K;
      const int gr = r0 + r, gk = k0 + k;
      t[r][k] = (gr < j.rows && gk < j.K) ? j.alpha * j.src[(int64_t)gr * j.ld + gk] : 0.0;
    }
  } else {
    for (int e = threadIdx.x; e < PK_R * PK_K; e += 256) {
      const int k = e / PK_R, r = e % PK_R;
      const int gr = r0 + r, gk = k0 + k;
      t[r][k] = (gr < j.rows && gk < j.K) ? j.alpha * j.src[(int64_t)gk * j.ld + gr] : 0.0;
    }
  }
  __syncthreads();
  double* base = static_cast<double*>(j.dst) + ((int64_t)panel * j.ktiles + j.kt0 + q) * PK_CHUNK_64;
  for (int e = threadIdx.x; e < PK_R * PK_K; e += 256) base[e] = t[e % PK_R][e / PK_R];
}

__global__ __launch_bounds__(XNT) void gemm_f64_packed(const SplitProb* __restrict__ probs, int nprob,
                                                       int total) {
  extern __shared__ __attribute__((aligned(16))) double f64_lds[];
  const int b = blockIdx.x, t8 = total & ~7;
  const int tile = b < t8 ? (b & 7) * (t8 >> 3) + (b >> 3) : b;
  const SplitProb& p = probs[find_item(probs, nprob, tile)];
  int tm, tn;
  x6_tile(p, tile - p.begin, tm, tn);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int pa = wave >> 1, pb = wave & 1;
  const int lr = lane & 15, lk = lane >> 4;

  // LDS: [buffer][operand][panel][k][row]
  constexpr int OPER = 2 * PK_CHUNK_64;
  constexpr int BUF = 2 * OPER;
  const double* Ag = static_cast<const double*>(p.A) + (int64_t)(2 * tm) * p.ktiles * PK_CHUNK_64;
  const double* Bg = static_cast<const double*>(p.B) + (int64_t)(2 * tn) * p.ktiles * PK_CHUNK_64;
  const int64_t pstride = (int64_t)p.ktiles * PK_CHUNK_64;

  // staging: per operand 2 panels x 1024 pieces of 16 bytes; thread t takes
  // pieces t + 256 u (u < 8)
  i4 ra[8], rb[8];
  auto fetch = [&](int kt) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + u * XNT;
      const int pan = e >> 10, w = e & 1023;
      ra[u] = *reinterpret_cast<const i4*>(Ag + pan * pstride + (int64_t)kt * PK_CHUNK_64 + w * 2);
      rb[u] = *reinterpret_cast<const i4*>(Bg + pan * pstride + (int64_t)kt * PK_CHUNK_64 + w * 2);
    }
  };
  auto commit = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + u * XNT;
      const int pan = e >> 10, w = e & 1023;
      *reinterpret_cast<i4*>(f64_lds + buf * BUF + pan * PK_CHUNK_64 + w * 2) = ra[u];
      *reinterpret_cast<i4*>(f64_lds + buf * BUF + OPER + pan * PK_CHUNK_64 + w * 2) = rb[u];
    }
  };

  d4 c[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) c[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  if (p.ktiles > 0) {
    fetch(0);
    commit(0);
  }
  __syncthreads();
  for (int kt = 0; kt < p.ktiles; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < p.ktiles) fetch(kt + 1);
    const double* As = f64_lds + buf * BUF + pa * PK_CHUNK_64;
    const double* Bs = f64_lds + buf * BUF + OPER + pb * PK_CHUNK_64;
#pragma unroll
    for (int ks = 0; ks < PK_K; ks += 4) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        av[i] = As[(ks + lk) * PK_R + i * 16 + lr];
        bv[i] = Bs[(ks + lk) * PK_R + i * 16 + lr];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) c[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], c[i][j], 0, 0, 0);
    }
    if (kt + 1 < p.ktiles) commit(buf ^ 1);
    __syncthreads();
  }

  // epilogue: element r of lane l of block (i, j) is row l / 16 + 4 r, column l % 16
  const int row0 = tm * XT + pa * 64, col0 = tn * XT + pb * 64;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + i * 16 + lk + 4 * r, col = col0 + j * 16 + lr;
        if (row < p.m && col < p.n) {
          double v = c[i][j][r];
          if (p.beta != 0.0) v += p.beta * p.D[(int64_t)row * p.ldd + col];
          p.C[(int64_t)row * p.ldc + col] = v;
        }
      }
}

size_t split_gemm_lds_bytes() { return (size_t)2 * 2 * 2 * PK_CHUNK * sizeof(__bf16); }

void launch_split_pack(const PackJob* d_jobs, int njobs, int chunks, hipStream_t s) {
  if (njobs <= 0 || chunks <= 0) return;
  split_pack<<<chunks, 256, 0, s>>>(d_jobs, njobs);
}

void launch_copy_pack64(const PackJob* d_jobs, int njobs, int chunks, hipStream_t s) {
  if (njobs <= 0 || chunks <= 0) return;
  copy_pack64<<<chunks, 256, 0, s>>>(d_jobs, njobs);
}

void launch_gemm_f64_packed(const SplitProb* d_probs, int nprob, int tiles, hipStream_t s) {
  if (nprob <= 0 || tiles <= 0) return;
  const size_t lds = (size_t)2 * 2 * 2 * PK_CHUNK_64 * sizeof(double);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(gemm_f64_packed),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  gemm_f64_packed<<<tiles, XNT, lds, s>>>(d_probs, nprob, tiles);
}

void launch_gemm_x6_packed(const SplitProb* d_probs, int nprob, int tiles, hipStream_t s) {
  if (nprob <= 0 || tiles <= 0) return;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(gemm_x6_packed),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)split_gemm_lds_bytes());
    attr = true;
  }
  gemm_x6_packed<<<tiles, XNT, split_gemm_lds_bytes(), s>>>(d_probs, nprob, tiles);
}

}  // namespace etdm
