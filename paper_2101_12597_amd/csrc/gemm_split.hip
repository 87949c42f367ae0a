// GEMMs on packed operands (gfx950): FP64, and the split-precision BF16x6
// product for large problems.
//
// The BF16x6 product of the grouped GEMM in gemm.hip splits every FP64 operand
// element into three BF16 slices x = hi + md + lo inside each workgroup, so an
// element is split once per tile that reads it, and every tile computes its own
// bounds-checked addresses.  Here the operands are packed once per launch
// (split_pack, copy_pack64) into a layout that the GEMMs read with plain
// contiguous 16-byte loads:
//
//   op(X) (rows x K) -> panels of PK_R = 64 rows, each a run of k-tiles of
//   PK_K = 32.  A BF16x6 chunk (one panel, one k-tile) holds [slice][row][k]
//   values, 3 x 64 x 32 x 2 bytes = 12 KB, contiguous; inside a row the four
//   8-value octets are permuted by an XOR of the row index (pk_phys), so that the
//   MFMA fragment reads of 16 consecutive rows do not conflict in the LDS.  An FP64
//   chunk is [k][row], 64 x 32 x 8 bytes = 16 KB, so the 16 lanes that share a
//   k of a v_mfma_f64_16x16x4f64 fragment read 128 consecutive bytes.
//
// Rows are padded with zeros to whole tiles and k to a multiple of 32.  A problem
// with two K segments (C = a1 A1 B1 + a2 A2 B2) packs [a1 A1 | a2 A2] and
// [B1; B2] along k, so the GEMM sees one K.
//
// gemm_x6_packed<TPM, TPN>: C = op(A) op(B) + beta D
// for packed op(A) and op(B)^T (both rows x K).  A workgroup of 4 wavefronts
// computes a tile of TPM x TPN panels (64 TPM x 64 TPN, TPM and TPN in {1, 2});
// each wavefront owns a 32 TPM x 32 TPN quarter as 2 TPM x 2 TPN blocks of
// 16 x 16.  Larger wavefront tiles read fewer LDS fragments per MFMA; smaller
// ones leave room for more wavefronts per SIMD.  BF16x6 sums the
// six slice products with i + j <= 2 (v_mfma_f32_16x16x32_bf16) in FP32 and adds
// them into FP64 registers every X_FLUSH k-tiles.  The k-tiles are
// double-buffered in LDS with the next one fetched into registers during the
// MFMAs; tiles are ordered in groups of X_GROUP tile rows and dealt out so that
// each XCD works on a contiguous range.  gemm_x6_ring (BF16x6 128 x 128 with eight
// wavefronts, and 64 x 64 also with eight) and gemm_f64_ring (FP64, every tile shape) fill
// their LDS buffers straight from global memory instead (global_load_lds_dwordx4);
// the 128 x 64 and 64 x 128 BF16x6 tiles keep the register-staged kernel, whose two
// workgroups per CU the ring's three buffers (108 KB) would not leave room for.
#include "common.h"
#include "reduce.h"

namespace etdm {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int PK_CHUNK = PK_CHUNK_X6;
constexpr int XNT = 256;
constexpr int X_FLUSH = 4;                     // k-tiles between FP64 flushes (128 k)
constexpr int X_GROUP = 4;                     // tile rows per group of the tile order

// octet position inside a 64-byte row.  The MFMA fragment read of a wavefront takes
// octet lane / 16 of rows r0 + lane % 16 (r0 a multiple of 16); with this permutation
// (period 8 in the row) the LDS counters show no bank conflict for it on gfx950, while
// XOR-ing in row bit 3 as well, or no permutation, conflicts.
__device__ __forceinline__ int pk_phys(int oct, int row) { return oct ^ ((row >> 1) & 3); }

}  // namespace

// ---------------------------------------------------------------------------
// split_pack: one workgroup per (panel, k-tile) chunk of one job
// ---------------------------------------------------------------------------
// element (r, q) of the real view of a complex operand (PackJob::cplx 1 or 2)
__device__ __forceinline__ double pack_zview(const PackJob& j, int r, int q) {
  if (j.cplx == 1) {  // op(A)[r][l], component d
    const int l = q >> 1, d = q & 1;
    const int64_t idx = j.op == OP_N ? (int64_t)r * j.ld + l : (int64_t)l * j.ld + r;
    const double x = j.src[2 * idx + d];
    return (j.op == OP_C && d) ? -x : x;
  }
  // op(B)[l][c] = re + i im: rows 2c (re, -im) and 2c + 1 (im, re) along k = 2l + d
  const int cc = r >> 1, e = r & 1, l = q >> 1, d = q & 1;
  const int64_t idx = j.op == OP_N ? (int64_t)l * j.ld + cc : (int64_t)cc * j.ld + l;
  const double re = j.src[2 * idx], im = j.op == OP_C ? -j.src[2 * idx + 1] : j.src[2 * idx + 1];
  return e == d ? re : (e ? im : -im);
}

__global__ __launch_bounds__(256) void split_pack(const PackJob* __restrict__ jobs,
                                                  const int* __restrict__ chunk_job) {
  __shared__ double t[PK_R][PK_K + 1];
  const PackJob& j = jobs[chunk_job[blockIdx.x]];
  const int c = blockIdx.x - j.begin;
  const int panel = c / j.kt_n, q = c % j.kt_n;
  const int r0 = panel * PK_R, k0 = q * PK_K;
  if (j.cplx) {
    for (int e = threadIdx.x; e < PK_R * PK_K; e += 256) {
      const int r = e / PK_K, k = e % PK_K;
      const int gr = r0 + r, gk = k0 + k;
      t[r][k] = (gr < j.rows && gk < j.K) ? pack_zview(j, gr, gk) : 0.0;
    }
  } else if (!j.trans) {
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
// gemm_x6_packed<TPM, TPN>: tiles of TPM x TPN panels (64 TPM rows, 64 TPN
// columns); the four wavefronts form a 2 x 2 grid of 32 TPM x 32 TPN sub-tiles,
// NBM = 2 TPM by NBN = 2 TPN blocks of 16 x 16
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

// NT threads: 256 (four wavefronts in 2 x 2, each 32 TPM x 32 TPN) or 512 (eight in
// 2 x 4, each 32 TPM x 16 TPN: fewer registers per wavefront, so that two of them
// share a SIMD and hide each other's latencies)
template <int TPM, int TPN, int NT>
__global__ __launch_bounds__(NT) void gemm_x6_packed(const SplitProb* __restrict__ probs,
                                                     const int* __restrict__ tile_prob, int total) {
  constexpr int WC = NT / 128;  // wavefront columns (two wavefront rows)
  constexpr int NBM = 2 * TPM, NBN = 4 * TPN / WC;
  static_assert((TPM * 768) % NT == 0 && (TPN * 768) % NT == 0, "staging pieces per thread");
  extern __shared__ __attribute__((aligned(16))) __bf16 x6_lds[];
  const int tile = tile_prob[total + blockIdx.x];  // the plan's workgroup -> tile order
  const SplitProb& p = probs[tile_prob[tile]];
  int tm, tn;
  x6_tile(p, tile - p.begin, tm, tn);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wrow = (wave / WC) * 32 * TPM, wcol = (wave % WC) * 16 * NBN;  // sub-tile offsets
  const int lr = lane & 15, lo = lane >> 4;

  // LDS: [buffer][A panels | B panels][slice][row][k]
  constexpr int OPERA = TPM * PK_CHUNK, OPERB = TPN * PK_CHUNK;
  constexpr int BUF = OPERA + OPERB;
  const int64_t pstride = (int64_t)p.ktiles * PK_CHUNK;  // panel stride in the packed operand
  const __bf16* Ag = static_cast<const __bf16*>(p.A) + (int64_t)(TPM * tm) * pstride;
  const __bf16* Bg = static_cast<const __bf16*>(p.B) + (int64_t)(TPN * tn) * pstride;

  // staging: TPM (TPN) panels x 768 pieces of 16 bytes of A (B); thread t takes
  // pieces t + 256 u
  constexpr int UA = TPM * 768 / NT, UB = TPN * 768 / NT;
  i4 ra[UA], rb[UB];
  auto fetch = [&](int kt) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const int e = threadIdx.x + u * NT;
      const int pan = e / 768, w = e % 768;
      ra[u] = *reinterpret_cast<const i4*>(Ag + pan * pstride + (int64_t)kt * PK_CHUNK + w * 8);
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int e = threadIdx.x + u * NT;
      const int pan = e / 768, w = e % 768;
      rb[u] = *reinterpret_cast<const i4*>(Bg + pan * pstride + (int64_t)kt * PK_CHUNK + w * 8);
    }
  };
  auto commit = [&](int buf) {
#pragma unroll
    for (int u = 0; u < UA; ++u)
      *reinterpret_cast<i4*>(x6_lds + buf * BUF + (threadIdx.x + u * NT) * 8) = ra[u];
#pragma unroll
    for (int u = 0; u < UB; ++u)
      *reinterpret_cast<i4*>(x6_lds + buf * BUF + OPERA + (threadIdx.x + u * NT) * 8) = rb[u];
  };

  double acc[NBM][NBN][4];
#pragma unroll
  for (int i = 0; i < NBM; ++i)
#pragma unroll
    for (int j = 0; j < NBN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
  f4 c[NBM][NBN];
#pragma unroll
  for (int i = 0; i < NBM; ++i)
#pragma unroll
    for (int j = 0; j < NBN; ++j) c[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // fragment offset (BF16 elements) of the 16-row block starting at tile row
  // off + 16 blk, slice s
  auto frag = [&](int off, int s, int blk) {
    const int trow = off + blk * 16;
    const int row = (trow & 63) + lr;
    return (trow >> 6) * PK_CHUNK + (s * PK_R + row) * PK_K + pk_phys(lo, row) * 8;
  };

  if (p.ktiles > 0) {
    fetch(0);
    commit(0);
  }
  __syncthreads();
  for (int kt = 0; kt < p.ktiles; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < p.ktiles) fetch(kt + 1);
    const __bf16* As = x6_lds + buf * BUF;
    const __bf16* Bs = x6_lds + buf * BUF + OPERA;
    bf8 bv[PK_S][NBN];
#pragma unroll
    for (int s = 0; s < PK_S; ++s)
#pragma unroll
      for (int j = 0; j < NBN; ++j) bv[s][j] = *reinterpret_cast<const bf8*>(Bs + frag(wcol, s, j));
    // A slice sa meets the B slices sb <= 2 - sa; lowest-order products first
#pragma unroll
    for (int sa = PK_S - 1; sa >= 0; --sa) {
      bf8 av[NBM];
#pragma unroll
      for (int i = 0; i < NBM; ++i) av[i] = *reinterpret_cast<const bf8*>(As + frag(wrow, sa, i));
#pragma unroll
      for (int sb = PK_S - 1 - sa; sb >= 0; --sb)
#pragma unroll
        for (int i = 0; i < NBM; ++i)
#pragma unroll
          for (int j = 0; j < NBN; ++j)
            c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[sb][j], c[i][j], 0, 0, 0);
    }
    if (kt + 1 < p.ktiles) commit(buf ^ 1);
    if ((kt + 1) % X_FLUSH == 0 || kt + 1 == p.ktiles) {
#pragma unroll
      for (int i = 0; i < NBM; ++i)
#pragma unroll
        for (int j = 0; j < NBN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)c[i][j][r];
          c[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    __syncthreads();
  }

  // epilogue: element r of lane l of block (i, j) is row 4 (l / 16) + r, column l % 16
  const int row0 = tm * 64 * TPM + wrow, col0 = tn * 64 * TPN + wcol;
#pragma unroll
  for (int i = 0; i < NBM; ++i)
#pragma unroll
    for (int j = 0; j < NBN; ++j)
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
// gemm_x6_ring<TPM, TPN, NT>: the same product for tiles of TPM x TPN panels with
// NT / 64 wavefronts (2 x NT / 128, each 32 TPM x 128 TPN / (NT / 128)) and a ring of
// three LDS buffers filled straight from global memory (global_load_lds_dwordx4: no
// staging registers).  While k-tile kt is multiplied from registers, k-tile kt + 1 is
// read from LDS into the registers its products free and k-tiles kt + 2 and kt + 3
// are in flight.  One barrier per k-tile: after it, buffer kt + 1 is complete and
// every wavefront is done with buffer kt, which then takes k-tile kt + 3.
// ---------------------------------------------------------------------------
constexpr int RING_NT = 512;
constexpr int RING_NBUF = 3;

// s_waitcnt immediate: vmcnt(vm) (6 bits, split over [3:0] and [15:14]), expcnt not
// waited on, lgkmcnt(0) when lgkm0 else not waited on
constexpr int ring_wait(int vm, bool lgkm0) {
  return (vm & 15) | ((vm >> 4) << 14) | 0x0070 | (lgkm0 ? 0 : 0x0f00);
}

template <int TPM, int TPN, int NT>
__global__ __launch_bounds__(NT) void gemm_x6_ring(const SplitProb* __restrict__ probs,
                                                   const int* __restrict__ tile_prob, int total) {
  constexpr int WC = NT / 128;  // wavefront columns (two wavefront rows)
  constexpr int NBM = 2 * TPM, NBN = 4 * TPN / WC;
  constexpr int OPERA = TPM * PK_CHUNK, BUF = (TPM + TPN) * PK_CHUNK;  // BF16 values
  constexpr int GROUPS = (TPM + TPN) * PK_CHUNK / 512;  // 1 KB groups of a k-tile (64 lanes x 16 bytes)
  constexpr int GPW = GROUPS / (NT / 64);               // groups per wavefront
  static_assert(GROUPS % (NT / 64) == 0 && PK_CHUNK % 512 == 0, "k-tile groups per wavefront");
  static_assert(2 * GPW < 64, "vmcnt immediates of the ring waits");
  extern __shared__ __attribute__((aligned(16))) __bf16 ring_lds[];
  const int tile = tile_prob[total + blockIdx.x];  // the plan's workgroup -> tile order
  const SplitProb& p = probs[tile_prob[tile]];
  int tm, tn;
  x6_tile(p, tile - p.begin, tm, tn);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wrow = (wave / WC) * 32 * TPM, wcol = (wave % WC) * 16 * NBN;
  const int lr = lane & 15, lo = lane >> 4;
  const int64_t pstride = (int64_t)p.ktiles * PK_CHUNK;
  const __bf16* Ag = static_cast<const __bf16*>(p.A) + (int64_t)(TPM * tm) * pstride;
  const __bf16* Bg = static_cast<const __bf16*>(p.B) + (int64_t)(TPN * tn) * pstride;

  // k-tile kt into ring buffer buf: group g (1 KB) of the tile's operands is copied by
  // wavefront g % 8, lane l taking its 16 bytes l
  auto issue = [&](int kt, int buf) {
#pragma unroll
    for (int u = 0; u < GPW; ++u) {
      const int g = wave + (NT / 64) * u;
      const int e = g * 64;  // first 16-byte piece of the group
      const __bf16* src = e < TPM * (PK_CHUNK / 8)
                              ? Ag + (e / (PK_CHUNK / 8)) * pstride + (int64_t)kt * PK_CHUNK + (e % (PK_CHUNK / 8)) * 8
                              : Bg + ((e - TPM * (PK_CHUNK / 8)) / (PK_CHUNK / 8)) * pstride + (int64_t)kt * PK_CHUNK +
                                    ((e - TPM * (PK_CHUNK / 8)) % (PK_CHUNK / 8)) * 8;
      __builtin_amdgcn_global_load_lds(src + lane * 8, ring_lds + buf * BUF + e * 8, 16, 0, 0);
    }
  };

  double acc[NBM][NBN][4];
#pragma unroll
  for (int i = 0; i < NBM; ++i)
#pragma unroll
    for (int j = 0; j < NBN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;
  f4 c[NBM][NBN];
#pragma unroll
  for (int i = 0; i < NBM; ++i)
#pragma unroll
    for (int j = 0; j < NBN; ++j) c[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  auto frag = [&](int off, int s, int blk) {
    const int trow = off + blk * 16;
    const int row = (trow & 63) + lr;
    return (trow >> 6) * PK_CHUNK + (s * PK_R + row) * PK_K + pk_phys(lo, row) * 8;
  };

  // the fragments of one k-tile for this wavefront's MFMAs
  struct Frag {
    bf8 b[PK_S][NBN];
    bf8 a[PK_S][NBM];
  };
  auto load_b = [&](Frag& f, int buf, int s) {
    const __bf16* Bs = ring_lds + buf * BUF + OPERA;
#pragma unroll
    for (int j = 0; j < NBN; ++j) f.b[s][j] = *reinterpret_cast<const bf8*>(Bs + frag(wcol, s, j));
  };
  auto load_a = [&](Frag& f, int buf, int s) {
    const __bf16* As = ring_lds + buf * BUF;
#pragma unroll
    for (int i = 0; i < NBM; ++i) f.a[s][i] = *reinterpret_cast<const bf8*>(As + frag(wrow, s, i));
  };
  // the product of A slice sa with B slice sb
  auto mma = [&](const Frag& f, int sa, int sb) {
#pragma unroll
    for (int i = 0; i < NBM; ++i)
#pragma unroll
      for (int j = 0; j < NBN; ++j)
        c[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.a[sa][i], f.b[sb][j], c[i][j], 0, 0, 0);
  };
  const int nk = p.ktiles;
  auto flush = [&](int kt) {
    if ((kt + 1) % X_FLUSH == 0 || kt + 1 == nk) {
#pragma unroll
      for (int i = 0; i < NBM; ++i)
#pragma unroll
        for (int j = 0; j < NBN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)c[i][j][r];
          c[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
  };
  // The six slice products of a k-tile, smallest terms first: (2,0) (1,1) (1,0) (0,2)
  // (0,1) (0,0).  Step kt < nk - 1 runs them on k-tile kt's fragments (in registers,
  // the last A slice possibly still arriving) and reads k-tile kt + 1's in between:
  // B slice 0 right after the barrier, every other fragment once the one it replaces
  // has had its last product, so that the next k-tile's reads overlap this one's
  // MFMAs in the registers of about one k-tile.
  // After the first product: wait until this wavefront's reads of k-tile kt are in
  // and its loads of kt + 1 have landed, then a bare barrier (__syncthreads would also
  // wait for the loads of kt + 2).  After it every wavefront is done with buffer kt,
  // which takes k-tile kt + 3, and k-tile kt + 1 is complete.  sched_barrier keeps
  // the compiler from moving reads ahead of the products that free their registers.
  auto step = [&](int kt, const Frag& cur, Frag& nxt) {
    mma(cur, 2, 0);
    __builtin_amdgcn_sched_barrier(0);
    if (kt + 2 < nk)
      __builtin_amdgcn_s_waitcnt(ring_wait(GPW, true));
    else
      __builtin_amdgcn_s_waitcnt(ring_wait(0, true));
    __builtin_amdgcn_s_barrier();
    if (kt + 3 < nk) issue(kt + 3, kt % RING_NBUF);
    const int nb = (kt + 1) % RING_NBUF;
    load_b(nxt, nb, 0);
    load_a(nxt, nb, 2);
    __builtin_amdgcn_sched_barrier(0);
    mma(cur, 1, 1);
    mma(cur, 1, 0);
    __builtin_amdgcn_sched_barrier(0);
    load_a(nxt, nb, 1);
    __builtin_amdgcn_sched_barrier(0);
    mma(cur, 0, 2);
    __builtin_amdgcn_sched_barrier(0);
    load_b(nxt, nb, 2);
    __builtin_amdgcn_sched_barrier(0);
    mma(cur, 0, 1);
    __builtin_amdgcn_sched_barrier(0);
    load_b(nxt, nb, 1);
    __builtin_amdgcn_sched_barrier(0);
    mma(cur, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    load_a(nxt, nb, 0);
    flush(kt);
  };
  auto last = [&](int kt, const Frag& cur) {
    mma(cur, 2, 0);
    mma(cur, 1, 1);
    mma(cur, 1, 0);
    mma(cur, 0, 2);
    mma(cur, 0, 1);
    mma(cur, 0, 0);
    flush(kt);
  };
  Frag f0, f1;
  if (nk > 0) {
    issue(0, 0);
    if (nk > 1) issue(1, 1);
    if (nk > 2) issue(2, 2);
    // this wavefront's loads of k-tile 0 landed (those of 1 and 2 may be in flight)
    if (nk > 2)
      __builtin_amdgcn_s_waitcnt(ring_wait(2 * GPW, false));
    else if (nk > 1)
      __builtin_amdgcn_s_waitcnt(ring_wait(GPW, false));
    else
      __builtin_amdgcn_s_waitcnt(ring_wait(0, false));
    __builtin_amdgcn_s_barrier();
#pragma unroll
    for (int s = 0; s < PK_S; ++s) {
      load_b(f0, 0, s);
      load_a(f0, 0, PK_S - 1 - s);
    }
    int kt = 0;
    for (; kt + 2 < nk; kt += 2) {
      step(kt, f0, f1);
      step(kt + 1, f1, f0);
    }
    // one or two k-tiles left, the last without a successor
    if (kt + 1 < nk) {
      step(kt, f0, f1);
      last(kt + 1, f1);
    } else {
      last(kt, f0);
    }
  }

  const int row0 = tm * 64 * TPM + wrow, col0 = tn * 64 * TPN + wcol;
#pragma unroll
  for (int i = 0; i < NBM; ++i)
#pragma unroll
    for (int j = 0; j < NBN; ++j)
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
// copy_pack64 / gemm_f64_ring
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void copy_pack64(const PackJob* __restrict__ jobs,
                                                   const int* __restrict__ chunk_job) {
  __shared__ double t[PK_R][PK_K + 1];
  const PackJob& j = jobs[chunk_job[blockIdx.x]];
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

// gemm_f64_ring<TPM, TPN, NT>: the FP64 product on packed operands with NT / 64
// wavefronts (2 x NT / 128, each 32 TPM x 128 TPN / (NT / 128)) and two LDS buffers
// filled straight from global memory (global_load_lds_dwordx4): k-tile kt + 1 loads
// while kt is multiplied (an FP64 k-tile keeps the matrix cores busy for thousands of
// cycles, so one tile ahead hides the load latency), one bare barrier per k-tile.
template <int TPM, int TPN, int NT>
__global__ __launch_bounds__(NT) void gemm_f64_ring(const SplitProb* __restrict__ probs,
                                                    const int* __restrict__ tile_prob, int total) {
  constexpr int WC = NT / 128;
  constexpr int NBM = 2 * TPM, NBN = 4 * TPN / WC;
  constexpr int OPERA = TPM * PK_CHUNK_64, BUF = (TPM + TPN) * PK_CHUNK_64;  // doubles
  constexpr int GROUPS = (TPM + TPN) * PK_CHUNK_64 / 128;  // 1 KB groups (64 lanes x 16 bytes)
  constexpr int GPW = GROUPS / (NT / 64);
  static_assert(GROUPS % (NT / 64) == 0 && PK_CHUNK_64 % 128 == 0, "k-tile groups per wavefront");
  static_assert(NBN >= 1 && 4 * TPN % WC == 0, "wavefront columns");
  extern __shared__ __attribute__((aligned(16))) double r64_lds[];
  const int tile = tile_prob[total + blockIdx.x];  // the plan's workgroup -> tile order
  const SplitProb& p = probs[tile_prob[tile]];
  int tm, tn;
  x6_tile(p, tile - p.begin, tm, tn);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wrow = (wave / WC) * 32 * TPM, wcol = (wave % WC) * 16 * NBN;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t pstride = (int64_t)p.ktiles * PK_CHUNK_64;
  const double* Ag = static_cast<const double*>(p.A) + (int64_t)(TPM * tm) * pstride;
  const double* Bg = static_cast<const double*>(p.B) + (int64_t)(TPN * tn) * pstride;

  // k-tile kt into buffer buf: group g (128 doubles) copied by wavefront g % 8, lane l
  // taking its two doubles l
  auto issue = [&](int kt, int buf) {
#pragma unroll
    for (int u = 0; u < GPW; ++u) {
      const int g = wave + (NT / 64) * u;
      const int e = g * 128;  // first double of the group
      const double* src = e < TPM * PK_CHUNK_64
                              ? Ag + (e / PK_CHUNK_64) * pstride + (int64_t)kt * PK_CHUNK_64 + (e % PK_CHUNK_64)
                              : Bg + ((e - TPM * PK_CHUNK_64) / PK_CHUNK_64) * pstride + (int64_t)kt * PK_CHUNK_64 +
                                    ((e - TPM * PK_CHUNK_64) % PK_CHUNK_64);
      __builtin_amdgcn_global_load_lds(src + lane * 2, r64_lds + buf * BUF + e, 16, 0, 0);
    }
  };
  auto at = [&](int k, int off, int blk) {
    const int trow = off + blk * 16;
    return (trow >> 6) * PK_CHUNK_64 + k * PK_R + (trow & 63) + lr;
  };

  d4 c[NBM][NBN];
#pragma unroll
  for (int i = 0; i < NBM; ++i)
#pragma unroll
    for (int j = 0; j < NBN; ++j) c[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int nk = p.ktiles;
  if (nk > 0) issue(0, 0);
  for (int kt = 0; kt < nk; ++kt) {
    // this wavefront's pieces of k-tile kt are in (nothing else is loading), then a bare
    // barrier: every piece of kt is in and every wavefront is done with buffer kt - 1
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0); expcnt, lgkmcnt not waited on
    __builtin_amdgcn_s_barrier();
    if (kt + 1 < nk) issue(kt + 1, (kt + 1) & 1);
    const double* As = r64_lds + (kt & 1) * BUF;
    const double* Bs = As + OPERA;
#pragma unroll
    for (int ks = 0; ks < PK_K; ks += 4) {
      double av[NBM], bv[NBN];
#pragma unroll
      for (int i = 0; i < NBM; ++i) av[i] = As[at(ks + lk, wrow, i)];
#pragma unroll
      for (int j = 0; j < NBN; ++j) bv[j] = Bs[at(ks + lk, wcol, j)];
#pragma unroll
      for (int i = 0; i < NBM; ++i)
#pragma unroll
        for (int j = 0; j < NBN; ++j) c[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], c[i][j], 0, 0, 0);
    }
  }

  // epilogue: element r of lane l of block (i, j) is row l / 16 + 4 r, column l % 16
  const int row0 = tm * 64 * TPM + wrow, col0 = tn * 64 * TPN + wcol;
#pragma unroll
  for (int i = 0; i < NBM; ++i)
#pragma unroll
    for (int j = 0; j < NBN; ++j)
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

void launch_split_pack(const PackJob* d_jobs, const int* d_chunk_job, int chunks, hipStream_t s) {
  if (chunks <= 0) return;
  split_pack<<<chunks, 256, 0, s>>>(d_jobs, d_chunk_job);
}

void launch_copy_pack64(const PackJob* d_jobs, const int* d_chunk_job, int chunks, hipStream_t s) {
  if (chunks <= 0) return;
  copy_pack64<<<chunks, 256, 0, s>>>(d_jobs, d_chunk_job);
}

template <typename K>
static void set_lds_limit(K kernel, size_t bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)bytes);
}

// tile shapes (tpm, tpn) in {(1,1), (2,1), (1,2), (2,2)}
template <int TPM, int TPN, int NT = RING_NT>
static void x6_ring(const SplitProb* d_probs, const int* d_tile_prob, int tiles, hipStream_t s) {
  const size_t lds = (size_t)RING_NBUF * (TPM + TPN) * PK_CHUNK * sizeof(__bf16);
  static bool attr = false;
  if (!attr) {
    set_lds_limit(gemm_x6_ring<TPM, TPN, NT>, lds);
    attr = true;
  }
  gemm_x6_ring<TPM, TPN, NT><<<tiles, NT, lds, s>>>(d_probs, d_tile_prob, tiles);
}
template <int TPM, int TPN, int NT = XNT>
static void x6_packed(const SplitProb* d_probs, const int* d_tile_prob, int tiles, hipStream_t s) {
  const size_t lds = (size_t)2 * (TPM + TPN) * PK_CHUNK * sizeof(__bf16);
  static bool attr = false;
  if (!attr) {
    set_lds_limit(gemm_x6_packed<TPM, TPN, NT>, lds);
    attr = true;
  }
  gemm_x6_packed<TPM, TPN, NT><<<tiles, NT, lds, s>>>(d_probs, d_tile_prob, tiles);
}

template <int TPM, int TPN, int NT>
static void f64_ring(const SplitProb* d_probs, const int* d_tile_prob, int tiles, hipStream_t s) {
  const size_t lds = (size_t)2 * (TPM + TPN) * PK_CHUNK_64 * sizeof(double);
  static bool attr = false;
  if (!attr) {
    set_lds_limit(gemm_f64_ring<TPM, TPN, NT>, lds);
    attr = true;
  }
  gemm_f64_ring<TPM, TPN, NT><<<tiles, NT, lds, s>>>(d_probs, d_tile_prob, tiles);
}

void launch_gemm_f64_packed(int tpm, int tpn, const SplitProb* d_probs, const int* d_tile_prob, int tiles,
                            hipStream_t s) {
  if (tiles <= 0) return;
  if (tpm == 2 && tpn == 2) f64_ring<2, 2, 512>(d_probs, d_tile_prob, tiles, s);
  else if (tpm == 2) f64_ring<2, 1, 512>(d_probs, d_tile_prob, tiles, s);
  else if (tpn == 2) f64_ring<1, 2, 512>(d_probs, d_tile_prob, tiles, s);
  else f64_ring<1, 1, 512>(d_probs, d_tile_prob, tiles, s);
}

void launch_gemm_x6_packed(int tpm, int tpn, const SplitProb* d_probs, const int* d_tile_prob, int tiles,
                           hipStream_t s) {
  if (tiles <= 0) return;
  if (tpm == 2 && tpn == 2) x6_ring<2, 2>(d_probs, d_tile_prob, tiles, s);
  else if (tpm == 2) x6_packed<2, 1>(d_probs, d_tile_prob, tiles, s);
  else if (tpn == 2) x6_packed<1, 2>(d_probs, d_tile_prob, tiles, s);
  else x6_ring<1, 1, 512>(d_probs, d_tile_prob, tiles, s);
}

}  // namespace etdm
