// FP64 symmetric eigensolver for large n (the ov matrix P = B B^T, n > 88).
//
// Main path (Sec. 3.4 asks only for the eigenpairs of iA; the method here is the
// classical one for dense symmetric matrices):
//   1. tb_reduce: Householder reduction A = Q T Q^T by all CUs together, one grid
//      barrier per step (below);
//   2. tb_bisect: eigenvalue brackets of T by multisection on Sturm counts;
//   3. tb_vectors: eigenvectors of T by twisted factorizations, one lane each;
//   4. on the host stream: Z^T Z and one Newton-Schulz step (GEMMs), the
//      back-transform X = Q Z in compact-WY blocks of TB_NBW reflectors, and a
//      final residual check of sym(P) X = X diag(w).
// Every check that fails leaves *ok = 0.
//
// Fallback: block-cyclic Jacobi with matrix-core updates.  It returns at once
// when *ok is set.  The matrix (padded with zero rows/columns to
// npad = 64 * ceil(n / 64), which never rotate) is split into nb = npad / 32
// blocks of 32 indices, and a sweep runs nb - 1 rounds of the round-robin
// pairing of the blocks.  In a round:
//   1. bjl_inner: every block pair (I, J) is one workgroup: it loads the 64 x 64
//      subproblem S = A[{I,J},{I,J}] into LDS and applies ONE sweep of the
//      parallel cyclic Jacobi of eigh.hip to it, accumulating the orthogonal
//      Q_IJ (S <- Q^T S Q).  Q goes to global memory; S is not written back.
//   2. bjl_update: every 64 x 64 block of the two-sided update
//        A[{Ia,Ja},{Ib,Jb}] <- Q_a^T A[{Ia,Ja},{Ib,Jb}] Q_b
//      and every 64-row block of V[:, {I,J}] <- V[:, {I,J}] Q is one workgroup
//      computing 64x64x64 FP64 MFMA products (4 wavefronts x 2 x 2 16x16x4 tiles).
// Every index pair is rotated at least once per sweep (pairs inside a block once
// per round), so the sweep converges at least as fast as a scalar cyclic sweep.
// Convergence is decided on the device: after every sweep the largest
// off-diagonal |a_ik| of the work matrix is compared with 1e-14 ||A||_F (a large
// multiple eigenvalue, such as the null space of B B^T when B has more rows than
// columns, converges only linearly in this ordering; well separated spectra
// converge quadratically and do not pay for the tight threshold); later
// launches see the flag and return at once, so the whole sequence can be
// captured in a graph.
#include <hip/hip_runtime.h>

#include "eigh_large.h"
#include "tridiag.h"

namespace etdm {

constexpr int L_NT = 512;     // threads of the inner kernel
constexpr int U_NT = 256;     // threads of the update kernel
constexpr int SUB = 64;       // subproblem size
constexpr int BLK = 32;       // block size
constexpr int LD = SUB + 1;   // padded LDS row length of the update tiles
constexpr double L_TOL = 1e-14;

typedef double d4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void rrp(int r, int j, int nn, int& p, int& q) {
  const int m = nn - 1;
  if (j == 0) {
    p = r;
    q = nn - 1;
  } else {
    p = r + j;
    if (p >= m) p -= m;
    q = r - j;
    if (q < 0) q += m;
  }
}

__device__ __forceinline__ void rot_cs(double app, double aqq, double apq, double& c, double& s) {
  const double mag = fabs(apq);
  const double tau = (aqq - app) / (2.0 * mag);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
  if (apq < 0.0) s = -s;
}

__device__ __forceinline__ int gmap(int x, int I, int J) { return x < BLK ? BLK * I + x : BLK * J + x - BLK; }

// A_work = sym(P) padded, V_work = I, and per-block partial sums of A^2.
__global__ void bjl_prepare(EighLarge e, double* partial) {
  const int npad = e.npad, n = e.n;
  double s = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)npad * npad;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / npad), k = (int)(idx - (int64_t)i * npad);
    double v = 0.0;
    if (i < n && k < n) v = 0.5 * (e.P[(size_t)i * n + k] + e.P[(size_t)k * n + i]);
    e.Aw[idx] = v;
    e.Vw[idx] = (i == k) ? 1.0 : 0.0;
    s += v * v;
  }
  __shared__ double red[U_NT / 64];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < U_NT / 64; ++w) t += red[w];
    partial[blockIdx.x] = t;
  }
}

constexpr int PREP_BLOCKS = 256;

__global__ void bjl_start(EighLarge e, const double* partial) {
  if (threadIdx.x != 0) return;
  if (e.ok && *e.ok) {  // the tridiagonal path already produced X and w
    e.st->done = 1;
    e.st->finite = 1;
    return;
  }
  double t = 0.0;
  for (int b = 0; b < PREP_BLOCKS; ++b) t += partial[b];
  const double scale = sqrt(t);
  e.st->scale = scale;
  e.st->sweep_off = 0ull;
  e.st->sweeps = 0;
  e.st->done = (!isfinite(scale) || scale == 0.0 || e.n <= 1) ? 1 : 0;
  e.st->finite = isfinite(scale) ? 1 : 0;
}

// One Jacobi sweep on every 64 x 64 block-pair subproblem of round r.
__global__ __launch_bounds__(L_NT) void bjl_inner(EighLarge e, int r) {
  if (e.st->done) return;
  extern __shared__ double sm[];
  double* S = sm;               // 64 x 64
  double* Q = S + SUB * SUB;    // 64 x 64
  double* pc = Q + SUB * SUB;   // 32
  double* ps = pc + SUB / 2;    // 32
  const int j = blockIdx.x, npad = e.npad;
  int I, J;
  rrp(r, j, e.nb, I, J);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < SUB * SUB; idx += L_NT) {
    const int a = idx >> 6, b = idx & 63;
    S[idx] = e.Aw[(size_t)gmap(a, I, J) * npad + gmap(b, I, J)];
    Q[idx] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int half = SUB / 2;
  const int jb = tid & (half - 1), ja0 = tid >> 5;  // 16 row-pair starts, stride 16
  for (int rr = 0; rr < SUB - 1; ++rr) {
    if (tid < half) {
      int p, q;
      rrp(rr, tid, SUB, p, q);
      const double apq = S[p * SUB + q];
      double c = 1.0, s = 0.0;
      if (apq != 0.0) rot_cs(S[p * SUB + p], S[q * SUB + q], apq, c, s);
      pc[tid] = c;
      ps[tid] = s;
    }
    __syncthreads();
    int pb, qb;
    rrp(rr, jb, SUB, pb, qb);
    const double cb = pc[jb], sb = ps[jb];
    for (int ja = ja0; ja < half; ja += L_NT / half) {
      int pa, qa;
      rrp(rr, ja, SUB, pa, qa);
      const double ca = pc[ja], sa = ps[ja];
      const double x00 = S[pa * SUB + pb], x01 = S[pa * SUB + qb];
      const double x10 = S[qa * SUB + pb], x11 = S[qa * SUB + qb];
      const double y00 = x00 * cb - x01 * sb, y01 = x00 * sb + x01 * cb;
      const double y10 = x10 * cb - x11 * sb, y11 = x10 * sb + x11 * cb;
      double z00 = ca * y00 - sa * y10, z01 = ca * y01 - sa * y11;
      double z10 = sa * y00 + ca * y10, z11 = sa * y01 + ca * y11;
      if (ja == jb) z01 = z10 = 0.0;
      S[pa * SUB + pb] = z00;
      S[pa * SUB + qb] = z01;
      S[qa * SUB + pb] = z10;
      S[qa * SUB + qb] = z11;
    }
    for (int i = ja0; i < SUB; i += L_NT / half) {
      const double vp = Q[i * SUB + pb], vq = Q[i * SUB + qb];
      Q[i * SUB + pb] = vp * cb - vq * sb;
      Q[i * SUB + qb] = vp * sb + vq * cb;
    }
    __syncthreads();
  }
  double* Qg = e.Qb + (size_t)j * SUB * SUB;
  for (int idx = tid; idx < SUB * SUB; idx += L_NT) Qg[idx] = Q[idx];
}

// Largest |a_ik| (i != k) of the work matrix after a sweep: atomic max on the
// bit pattern (which orders like the value for non-negative doubles).
constexpr int OFF_BLOCKS = 512;
__global__ __launch_bounds__(U_NT) void bjl_offmax(EighLarge e) {
  if (e.st->done) return;
  const int npad = e.npad, n = e.n;
  double m = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)npad * npad;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / npad), k = (int)(idx - (int64_t)i * npad);
    if (i != k && i < n && k < n) m = fmax(m, fabs(e.Aw[idx]));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  __shared__ double red[U_NT / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < U_NT / 64; ++w) t = fmax(t, red[w]);
    atomicMax(&e.st->sweep_off, (unsigned long long)__double_as_longlong(t));
  }
}

// 64 x 64 x 64 product of two LDS tiles (row length LD): C = op(X) Y with
// op(X) = X or X^T; each wavefront computes its 32 x 32 quadrant.
template <bool XT>
__device__ __forceinline__ void tile_mm(const double* X, const double* Y, d4v (&c)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  for (int i = 0; i < 2; ++i)
    for (int jj = 0; jj < 2; ++jj) c[i][jj] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int s4 = 0; s4 < SUB / 4; ++s4) {
    const int k = 4 * s4 + lk;
    double a[2], b[2];
    for (int i = 0; i < 2; ++i) {
      const int row = wm + 16 * i + li;
      a[i] = XT ? X[k * LD + row] : X[row * LD + k];
      b[i] = Y[k * LD + wn + 16 * i + li];
    }
    for (int i = 0; i < 2; ++i)
      for (int jj = 0; jj < 2; ++jj) c[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[jj], c[i][jj], 0, 0, 0);
  }
}

// Two-sided block update of A and column update of V for round r.
__global__ __launch_bounds__(U_NT) void bjl_update(EighLarge e, int r) {
  if (e.st->done) return;
  extern __shared__ double sm[];
  double* X = sm;              // 64 x LD
  double* Y = X + SUB * LD;    // 64 x LD
  const int half = e.nb / 2, npad = e.npad, t = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  d4v c[2][2];
  if (t < half * half) {
    const int ja = t / half, jb = t - ja * half;
    int Ia, Ja, Ib, Jb;
    rrp(r, ja, e.nb, Ia, Ja);
    rrp(r, jb, e.nb, Ib, Jb);
    const double* Qa = e.Qb + (size_t)ja * SUB * SUB;
    const double* Qbb = e.Qb + (size_t)jb * SUB * SUB;
    for (int idx = threadIdx.x; idx < SUB * SUB; idx += U_NT) {
      const int a = idx >> 6, b = idx & 63;
      X[a * LD + b] = e.Aw[(size_t)gmap(a, Ia, Ja) * npad + gmap(b, Ib, Jb)];
      Y[a * LD + b] = Qbb[idx];
    }
    __syncthreads();
    tile_mm<false>(X, Y, c);  // T = A_blk Q_b
    __syncthreads();
    for (int i = 0; i < 2; ++i)
      for (int jj = 0; jj < 2; ++jj)
        for (int q = 0; q < 4; ++q) X[(wm + 16 * i + lk + 4 * q) * LD + wn + 16 * jj + li] = c[i][jj][q];
    for (int idx = threadIdx.x; idx < SUB * SUB; idx += U_NT) Y[(idx >> 6) * LD + (idx & 63)] = Qa[idx];
    __syncthreads();
    tile_mm<true>(Y, X, c);  // Q_a^T T
    for (int i = 0; i < 2; ++i)
      for (int jj = 0; jj < 2; ++jj)
        for (int q = 0; q < 4; ++q) {
          const int row = wm + 16 * i + lk + 4 * q, col = wn + 16 * jj + li;
          e.Aw[(size_t)gmap(row, Ia, Ja) * npad + gmap(col, Ib, Jb)] = c[i][jj][q];
        }
  } else {
    const int t2 = t - half * half;
    const int rb = t2 / half, j = t2 - rb * half;
    int I, J;
    rrp(r, j, e.nb, I, J);
    const double* Qj = e.Qb + (size_t)j * SUB * SUB;
    for (int idx = threadIdx.x; idx < SUB * SUB; idx += U_NT) {
      const int a = idx >> 6, b = idx & 63;
      X[a * LD + b] = e.Vw[(size_t)(rb * SUB + a) * npad + gmap(b, I, J)];
      Y[a * LD + b] = Qj[idx];
    }
    __syncthreads();
    tile_mm<false>(X, Y, c);  // V_blk Q
    for (int i = 0; i < 2; ++i)
      for (int jj = 0; jj < 2; ++jj)
        for (int q = 0; q < 4; ++q) {
          const int row = wm + 16 * i + lk + 4 * q, col = wn + 16 * jj + li;
          e.Vw[(size_t)(rb * SUB + row) * npad + gmap(col, I, J)] = c[i][jj][q];
        }
  }
}

__global__ void bjl_sweep_end(EighLarge e, int max_sweeps, int* status) {
  if (threadIdx.x != 0 || e.st->done) return;
  const double off = __longlong_as_double((long long)e.st->sweep_off);
  e.st->sweep_off = 0ull;
  e.st->sweeps += 1;
  if (off <= L_TOL * e.st->scale) {
    e.st->done = 1;
  } else if (e.st->sweeps >= max_sweeps) {
    e.st->done = 1;
    atomicOr(status, ST_EIGH);
  }
}

__global__ void bjl_finish(EighLarge e, int* status) {
  if (e.ok && *e.ok) return;
  const int n = e.n, npad = e.npad;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), k = (int)(idx - (int64_t)i * n);
    e.X[idx] = e.Vw[(size_t)i * npad + k];
    if (k == 0) e.w[i] = e.Aw[(size_t)i * npad + i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && !e.st->finite) atomicOr(status, ST_NONFINITE);
}

// ---------------------------------------------------------------------------
// Reduction to tridiagonal form by all CUs together (tried before the Jacobi
// sweeps).  Workgroup g owns rows g, g + G, ... of the work matrix A (G
// workgroups, one per CU, all resident).  Step k applies reflector k
// (H = I - tau v v^T, v_{k+1} = 1) as A_t <- A_t - v w^T - w v^T with p = tau A_t v
// and w = p - (tau/2)(p.v) v, and at the same time forms p for step k + 1:
//   after the grid barrier every workgroup has p_k (global), forms w_k, and
//   updates its copy of row k + 1 (kept by the row's owner in a look-ahead buffer
//   before the owner changes it) -> reflector k + 1, computed identically by every
//   workgroup; then each owner updates its rows i >= k + 2 (columns >= k + 2) and
//   in the same pass accumulates p_{k+1,i} = tau_{k+1} sum_j a_ij v_{k+1,j}.
// One grid barrier per step (tb_reduce; the register-resident tb_reduce_reg polls
// the exchanged slots instead); A is read and written once per step.  The waits are
// bounded: a wait longer than TB_SPIN sets the abort word, every workgroup leaves,
// *ok stays 0 and the Jacobi sweeps take over.
// ---------------------------------------------------------------------------
constexpr int TB_NT = 256;      // threads of the reduction
constexpr int TB_RMAX = 2;      // own rows per pass (all their loads issued before any store)
constexpr int TB_CMAX = 10;     // columns per thread and row and chunk (TB_NT * TB_CMAX columns per chunk)
constexpr int TB_GRP = 16;      // the grid has at most 64 TB_GRP workgroups
constexpr int TB_BAR_WORDS = 64 + 32 * 64;  // synchronization words: [2] abort, [64 ..) arrival flags
constexpr unsigned long long TB_SPIN = 20000000ull;  // 0.2 s of the 100 MHz wall clock
// Slots of p and of the look-ahead rows (register-resident reduction) that hold no
// value of the current step carry this signalling-NaN pattern; arithmetic never
// produces a signalling NaN.
constexpr unsigned long long TR_EMPTY = 0x7ff4a5a5a5a5a5a5ull;
// Multisection: TE_CH eigenvalues per workgroup of TE_NT threads, TE_C chains per lane:
// TE_C floor(TE_NT / TE_CH) = 25 points per eigenvalue and round (4.7 bits).  A Sturm
// count is a chain of n dependent pivots (a reciprocal and a few FP64 operations each)
// that occupies its SIMD's issue slots: one chain per lane (two measured 1.5x slower)
// and about one wavefront per SIMD (n = 2304: 461 workgroups of two wavefronts, d and
// e^2 in 37 KB of LDS) keep the round short.
constexpr int TE_CH = 5;
constexpr int TE_NT = 128;
constexpr int TE_C = 1;
static size_t tb_bisect_lds(int n) { return sizeof(double) * 2 * (size_t)n; }

size_t eigh_large_workspace(int n, size_t* npad_out) {
  const size_t npad = (size_t)((n + SUB - 1) / SUB) * SUB;
  if (npad_out) *npad_out = npad;
  const size_t half = npad / BLK / 2;
  const size_t nblk = (size_t)(n - 1 + TB_NBW - 1) / TB_NBW;
  const size_t nkc = (size_t)std::max(1, (n - 1 + TB_KC - 1) / TB_KC);
  return 2 * npad * npad + half * SUB * SUB + PREP_BLOCKS + 2 * (size_t)n * n + 8 * (size_t)n +
         (nkc + 1) * TB_NBW * n + nblk * TB_NBW * TB_NBW * (nkc + 1) + TB_BAR_WORDS / 2 + 2 + 4 +
         3 * (size_t)n;
}

// dynamic LDS of the reduction kernels: more than half of a CU's LDS, so that no two
// workgroups share a CU
static size_t tb_reduce_lds(int n) { return std::max<size_t>(sizeof(double) * 4 * (size_t)n, 96 * 1024); }
static void tb_cap_grid(EighLarge& e, int cu_count);

void eigh_large_layout(EighLarge& e, double* ws, EighLargeState* st, int cu_count) {
  size_t npad = 0;
  eigh_large_workspace(e.n, &npad);
  const int n = e.n;
  e.npad = (int)npad;
  e.nb = (int)npad / BLK;
  e.Aw = ws;
  e.Vw = e.Aw + npad * npad;
  e.Qb = e.Vw + npad * npad;
  e.partial = e.Qb + (size_t)(e.nb / 2) * SUB * SUB;
  e.Zw = e.partial + PREP_BLOCKS;
  e.Ps = e.Zw + (size_t)n * n;
  e.d = e.Ps + (size_t)n * n;
  e.e = e.d + n;
  e.pv = e.e + n;
  e.rowbuf = e.pv + 3 * n;
  e.nkc = std::max(1, (n - 1 + TB_KC - 1) / TB_KC);
  e.W1 = e.rowbuf + 3 * n;
  e.W2 = e.W1 + (size_t)e.nkc * TB_NBW * n;
  e.Tw = e.W2 + (size_t)TB_NBW * n;
  const size_t nblk = (size_t)(n - 1 + TB_NBW - 1) / TB_NBW;
  e.Gw = e.Tw + nblk * TB_NBW * TB_NBW * e.nkc;
  e.bar = reinterpret_cast<unsigned*>(e.Gw + nblk * TB_NBW * TB_NBW);
  e.ok = reinterpret_cast<int*>(e.bar + TB_BAR_WORDS);
  e.scan = reinterpret_cast<double*>(e.bar + TB_BAR_WORDS + 4);
  e.blo = e.scan + 4;
  e.bhi = e.blo + n;
  e.bb = reinterpret_cast<int*>(e.bhi + n);
  e.st = st;
  e.grid = std::max(1, std::min(std::min(cu_count, n / 8), 64 * TB_GRP));
  tb_cap_grid(e, cu_count);
}

// workgroup sum of TB_NT threads, returned to every thread
__device__ __forceinline__ double tb_sum(double v, double* red) {
  v = tl_wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < TB_NT / 64; ++q) t += red[q];
  return t;
}

// Grid synchronization by arrival flags.  Every thread waits for its own stores to
// complete (only p and the look-ahead rows cross workgroups, stored and loaded with
// device-scope atomics, so no cache writeback or invalidation is needed); then the
// workgroup publishes the number of steps it has finished in its own word
// bar[TB_FLAG0 + g], and its wave 0 polls all the flags (a few loads per lane) until
// each has reached that number.  One store and one polled read per step, with no
// read-modify-write on a shared word.  Every wait is bounded: past TB_SPIN the abort
// word bar[2] is set and every workgroup leaves (false).
constexpr int TB_FLAG0 = 64;  // flags bar[64 .. 64 + grid), grid <= 64 TB_GRP
static_assert(TB_FLAG0 + 64 * TB_GRP <= TB_BAR_WORDS, "barrier words too few for the flags");
__device__ bool tb_grid_sync(unsigned* bar, unsigned& gen) {
  __shared__ int s_go;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  const unsigned want = gen + 1;
  if (threadIdx.x < 64) {
    const int G = gridDim.x, lane = threadIdx.x;
    int go = __hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    if (lane == 0) __hip_atomic_store(&bar[TB_FLAG0 + blockIdx.x], want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long t0 = wall_clock64();
    while (go) {
      unsigned mn = 0xffffffffu;
      for (int w = lane; w < G; w += 64)
        mn = min(mn, __hip_atomic_load(&bar[TB_FLAG0 + w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      for (int o = 32; o > 0; o >>= 1) mn = min(mn, (unsigned)__shfl_xor((int)mn, o));
      if (mn >= want) break;
      if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        go = 0;
        break;
      }
      if (wall_clock64() - t0 > TB_SPIN) {
        if (lane == 0) atomicExch(&bar[2], 1u);
        go = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) s_go = go;
  }
  __syncthreads();
  gen = want;
  return s_go != 0;
}

__device__ __forceinline__ void tb_put(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double tb_get(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reflector from row r (= column k below the diagonal): alpha = r[k+1],
// sigma^2 = sum_{j>=k+2} r_j^2; v[k+1] = 1, v[j] = r_j / (alpha - beta).
__device__ double tb_reflector(const double* r, int k, int n, double* v, double* red, double& beta) {
  double s2 = 0.0;
  for (int j = k + 2 + (int)threadIdx.x; j < n; j += TB_NT) s2 += r[j] * r[j];
  s2 = tb_sum(s2, red);
  const double alpha = r[k + 1];
  double tau = 0.0, inv = 0.0;
  beta = alpha;
  if (s2 != 0.0) {
    beta = -copysign(sqrt(alpha * alpha + s2), alpha);
    tau = (beta - alpha) / beta;
    inv = 1.0 / (alpha - beta);
  }
  for (int j = k + 1 + (int)threadIdx.x; j < n; j += TB_NT) v[j] = (j == k + 1) ? 1.0 : r[j] * inv;
  __syncthreads();
  return tau;
}

// Own rows i >= ilo over columns j >= jlo: with upd, a_ij -= v_i w_j + w_i v_j;
// then p[i] = tau1 sum_j a_ij v1_j.  Row rowcopy (if owned) is also written to rb.
// TB_RMAX rows at a time, all their loads issued before any store.
__device__ void tb_rows(double* A, int n, int ilo, int jlo, bool upd, const double* v, const double* w,
                        double tau1, const double* v1, double* p, int rowcopy, double* rb, double (*red2)[TB_RMAX]) {
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int first = ilo + ((g - ilo) % G + G) % G;
  for (int base = first; base < n; base += G * TB_RMAX) {
    double acc[TB_RMAX];
#pragma unroll
    for (int q = 0; q < TB_RMAX; ++q) acc[q] = 0.0;
    for (int c0 = jlo; c0 < n; c0 += TB_NT * TB_CMAX) {
      double x[TB_RMAX][TB_CMAX];
#pragma unroll
      for (int q = 0; q < TB_RMAX; ++q) {
        const int i = min(base + q * G, n - 1);
        const double* row = A + (size_t)i * n;
#pragma unroll
        for (int c = 0; c < TB_CMAX; ++c) {
          const int j = c0 + tid + c * TB_NT;
          x[q][c] = row[min(j, n - 1)];
        }
      }
#pragma unroll
      for (int q = 0; q < TB_RMAX; ++q) {
        const int i = base + q * G;
        if (i < n) {
          double* row = A + (size_t)i * n;
          const double vi = upd ? v[i] : 0.0, wi = upd ? w[i] : 0.0;
#pragma unroll
          for (int c = 0; c < TB_CMAX; ++c) {
            const int j = c0 + tid + c * TB_NT;
            if (j < n) {
              if (upd) {
                x[q][c] -= vi * w[j] + wi * v[j];
                row[j] = x[q][c];
              }
              if (i == rowcopy) tb_put(&rb[j], x[q][c]);
              acc[q] += x[q][c] * v1[j];
            }
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < TB_RMAX; ++q) acc[q] = tl_wave_sum(acc[q]);
    if (lane == 0)
      for (int q = 0; q < TB_RMAX; ++q) red2[wave][q] = acc[q];
    __syncthreads();
    if (tid < TB_RMAX) {
      const int i = base + tid * G;
      if (i < n) {
        double t = 0.0;
        for (int q = 0; q < TB_NT / 64; ++q) t += red2[q][tid];
        tb_put(&p[i], tau1 * t);
      }
    }
    __syncthreads();
  }
}

// polled: the slots of p and of the look-ahead rows of the register-resident reduction
// start empty
__global__ void tb_init(EighLarge e, int polled) {
  for (int q = threadIdx.x; q < TB_BAR_WORDS; q += blockDim.x) e.bar[q] = 0u;
  // The compact-WY blocks count n - 1 reflector columns, one more than the reduction
  // forms: column n - 2 is an identity reflector, tau = 0 and a zero column, written
  // here because the reflector matrix may hold anything from an earlier use.
  const int n = e.n;
  if (n >= 3) {
    for (int j = threadIdx.x; j < n; j += blockDim.x) e.Vw[(size_t)j * n + (n - 2)] = 0.0;
    if (threadIdx.x == 0) e.Vw[(size_t)(n - 2) * n + (n - 1)] = 0.0;
  }
  if (polled)
    for (int q = threadIdx.x; q < 6 * e.n; q += blockDim.x)
      reinterpret_cast<unsigned long long*>(e.pv)[q] = TR_EMPTY;
  if (threadIdx.x < 4) e.scan[threadIdx.x] = 0.0;
  if (threadIdx.x == 0) *e.ok = 0;
}

__global__ __launch_bounds__(TB_NT) void tb_reduce(EighLarge e) {
  extern __shared__ double sm[];
  __shared__ double red[TB_NT / 64];
  __shared__ double red2[TB_NT / 64][TB_RMAX];
  const int n = e.n, G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  double* A = e.Aw;  // ld n
  double* Y = e.Vw;  // ld n
  double* vc = sm;   // reflector of the current step
  double* vn = vc + n;
  double* w = vn + n;
  double* r = w + n;
  unsigned gen = 0;
  // own rows of A = sym(P).  Y is written by workgroup 0 only: each reflector
  // column with the zeros above it that its compact-WY block reads (rows k0+1..c of
  // column c, k0 the first column of the block), so no other workgroup's stores to
  // Y can race with them.
  for (int i = g; i < n; i += G)
    for (int j = tid; j < n; j += TB_NT) {
      const double a = 0.5 * (e.P[(size_t)i * n + j] + e.P[(size_t)j * n + i]);
      A[(size_t)i * n + j] = a;
      e.Ps[(size_t)i * n + j] = a;
    }
  // reflector 0 from row 0 (formed from P by every workgroup); p_0 and the look-ahead copy of row 1
  for (int j = tid; j < n; j += TB_NT) r[j] = 0.5 * (e.P[j] + e.P[(size_t)j * n]);
  __syncthreads();
  double beta;
  double tau = tb_reflector(r, 0, n, vc, red, beta);
  if (g == 0) {
    for (int j = 1 + tid; j < n; j += TB_NT) Y[(size_t)j * n] = vc[j];
    if (tid == 0) {
      Y[n - 1] = tau;
      e.d[0] = r[0];
      e.e[0] = beta;
    }
  }
  tb_rows(A, n, 1, 1, false, vc, w, tau, vc, e.pv, 1, e.rowbuf + n, red2);
  if (!tb_grid_sync(e.bar, gen)) return;
  for (int k = 0; k < n - 2; ++k) {
    const double* p = e.pv + (size_t)(k & 1) * n;
    double part = 0.0;
    for (int i = k + 1 + tid; i < n; i += TB_NT) {
      const double pi = tb_get(&p[i]);
      w[i] = pi;
      part += pi * vc[i];
    }
    const double K = -0.5 * tau * tb_sum(part, red);
    for (int i = k + 1 + tid; i < n; i += TB_NT) w[i] += K * vc[i];
    __syncthreads();
    const double* rb = e.rowbuf + (size_t)((k + 1) & 1) * n;
    const double vk1 = vc[k + 1], wk1 = w[k + 1];
    for (int j = k + 1 + tid; j < n; j += TB_NT) r[j] = tb_get(&rb[j]) - (vk1 * w[j] + wk1 * vc[j]);
    __syncthreads();
    double taun = 0.0;
    if (k + 1 <= n - 3) {
      taun = tb_reflector(r, k + 1, n, vn, red, beta);
      if (g == 0) {
        const int c = k + 1, k0 = (c / TB_NBW) * TB_NBW;
        for (int j = k0 + 1 + tid; j < n; j += TB_NT) Y[(size_t)j * n + c] = j >= c + 1 ? vn[j] : 0.0;
        if (tid == 0) {
          Y[(size_t)(k + 1) * n + (n - 1)] = taun;
          e.d[k + 1] = r[k + 1];
          e.e[k + 1] = beta;
        }
      }
    } else if (g == 0 && tid == 0) {  // the last 2 x 2 block
      e.d[n - 2] = r[n - 2];
      e.e[n - 2] = r[n - 1];
    }
    tb_rows(A, n, k + 2, k + 2, true, vc, w, taun, vn, e.pv + (size_t)((k + 1) & 1) * n, k + 2,
            e.rowbuf + (size_t)((k + 2) & 1) * n, red2);
    if (k == n - 3 && g == (n - 1) % G && tid == 0) e.d[n - 1] = A[(size_t)(n - 1) * n + (n - 1)];
    double* t = vc;
    vc = vn;
    vn = t;
    tau = taun;
    if (!tb_grid_sync(e.bar, gen)) return;
  }
  if (g == 0 && tid == 0) *e.ok = 1;  // reached only when no barrier aborted
}

// ---------------------------------------------------------------------------
// The same reduction with the owned rows held in registers (n <= TR_NT TR_Q and
// at most TR_R rows per workgroup): thread t of workgroup g keeps a_ij for the
// rows i = g + G r and the columns j = t + TR_NT q.  The rank-2 update and the
// fused product for p then never touch memory; per step only p, the look-ahead
// row and the reflector column of Y cross the chip.  One grid barrier per step,
// three workgroup barriers (the dot p.v, the reflector norm, the row dots).
// ---------------------------------------------------------------------------
constexpr int TR_NT = 512;
constexpr int TR_Q = 5;    // columns per thread
constexpr int TR_R = 9;    // own rows per workgroup
constexpr int TR_W = TR_NT / 64;

// Reflector c from register row c (entries j >= c + 1 valid): alpha = row[c+1],
// sigma^2 = sum_{j >= c+2} row_j^2; v_{c+1} = 1, v_j = row_j / (alpha - beta).
__device__ __forceinline__ double tr_reflector(const double (&row)[TR_Q], int c, int n, double (&v)[TR_Q],
                                               double* red, double* s_alpha, double& beta) {
  const int tid = threadIdx.x;
  double s2 = 0.0;
#pragma unroll
  for (int q = 0; q < TR_Q; ++q) {
    const int j = tid + TR_NT * q;
    if (j == c + 1) *s_alpha = row[q];
    if (j >= c + 2 && j < n) s2 += row[q] * row[q];
  }
  s2 = tl_wave_sum(s2);
  if ((tid & 63) == 0) red[tid >> 6] = s2;
  __syncthreads();
  s2 = 0.0;
#pragma unroll
  for (int w = 0; w < TR_W; ++w) s2 += red[w];
  const double alpha = *s_alpha;
  double tau = 0.0, inv = 0.0;
  beta = alpha;
  if (s2 != 0.0) {
    beta = -copysign(sqrt(alpha * alpha + s2), alpha);
    tau = (beta - alpha) / beta;
    inv = 1.0 / (alpha - beta);
  }
#pragma unroll
  for (int q = 0; q < TR_Q; ++q) {
    const int j = tid + TR_NT * q;
    v[q] = j == c + 1 ? 1.0 : (j >= c + 2 && j < n ? row[q] * inv : 0.0);
  }
  return tau;
}

// Reflector column c of Y (workgroup 0): v_c below row c, zeros above it within
// its compact-WY block, tau_c in the last column; d_c and e_c of T.
__device__ __forceinline__ void tr_store_reflector(EighLarge& e, const double (&v)[TR_Q], double tau, double beta,
                                                   int c, const double (&row)[TR_Q]) {
  const int n = e.n, k0 = (c / TB_NBW) * TB_NBW;
#pragma unroll
  for (int q = 0; q < TR_Q; ++q) {
    const int j = threadIdx.x + TR_NT * q;
    if (j >= k0 + 1 && j < n) e.Vw[(size_t)j * n + c] = j >= c + 1 ? v[q] : 0.0;
    if (j == c) e.d[c] = row[q];
  }
  if (threadIdx.x == 0) {
    e.Vw[(size_t)c * n + (n - 1)] = tau;
    e.e[c] = beta;
  }
}

__device__ __forceinline__ void tr_clear(double* p) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), TR_EMPTY, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Entries j = tid + TR_NT q, lo <= j < n, of p and rb (zero elsewhere), each polled
// until it is no longer empty.  False for the whole workgroup when the grid aborts or
// a wait exceeds TB_SPIN (which sets the abort word).
// Also forms this wavefront's part of p . v_k into red1[wave] (and p_{k+1} into *pk1)
// before the workgroup barrier that ends the wait, so that one barrier serves both.
__device__ bool tr_take(const double* p, const double* rb, int lo, int n, double (&pj)[TR_Q], double (&rj)[TR_Q],
                        unsigned* bar, const double (&vc)[TR_Q], double* red1, double* pk1) {
  unsigned pend = 0u;
#pragma unroll
  for (int q = 0; q < TR_Q; ++q) {
    const int j = threadIdx.x + TR_NT * q;
    pj[q] = 0.0;
    rj[q] = 0.0;
    if (j >= lo && j < n) pend |= 3u << (2 * q);
  }
  int fail = 0;
  const unsigned long long t0 = wall_clock64();
  while (pend) {
#pragma unroll
    for (int q = 0; q < TR_Q; ++q) {
      const int j = threadIdx.x + TR_NT * q;
      if (pend & (1u << (2 * q))) {
        const double x = tb_get(&p[j]);
        if ((unsigned long long)__double_as_longlong(x) != TR_EMPTY) {
          pj[q] = x;
          pend &= ~(1u << (2 * q));
        }
      }
      if (pend & (2u << (2 * q))) {
        const double x = tb_get(&rb[j]);
        if ((unsigned long long)__double_as_longlong(x) != TR_EMPTY) {
          rj[q] = x;
          pend &= ~(2u << (2 * q));
        }
      }
    }
    if (!pend) break;
    if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
      fail = 1;
      break;
    }
    if (wall_clock64() - t0 > TB_SPIN) {
      atomicExch(&bar[2], 1u);
      fail = 1;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  double part = 0.0;
#pragma unroll
  for (int q = 0; q < TR_Q; ++q) {
    part += pj[q] * vc[q];
    if ((int)threadIdx.x + TR_NT * q == lo) *pk1 = pj[q];
  }
  part = tl_wave_sum(part);
  if ((threadIdx.x & 63) == 0) red1[threadIdx.x >> 6] = part;
  return !__syncthreads_or(fail);
}

// The reduction with the rows of A in registers (n <= TR_NT TR_Q, at most TR_R rows
// per workgroup).  No grid barrier: the only data that cross workgroups are p and
// the look-ahead rows, and readers poll those slots directly.  p_k sits in buffer
// k mod 3, row k in row buffer k mod 3; the slots are emptied again by their writers
// once every reader is known to be done with them:
//   * step k begins when all of p_k (rows >= k + 1) is in, so every workgroup that
//     read p_{k-1} (all own a row >= k + 1) has finished doing so: each owner then
//     empties its slots of buffer (k + 2) mod 3, and the owner of row k + 3 empties
//     row buffer k mod 3 (row k, read in step k - 1);
//   * those stores complete before the owner stores p_{k+1}, and a reader of
//     p_{k+2} or of row k + 3 (step k + 2, k + 1... later) has read that owner's
//     p_{k+1} entry first, so it sees the empty slot or the new value, never the old.
// A workgroup leaves after the last step that updates one of its rows; the owner of
// row n - 1 takes every step and stores the reflectors and T.
// The parts of reflector column c of Y that are not owned rows below row c + 1: the
// zeros in rows (k0, c] of its compact-WY block, tau_c in the last column, d_c and e_c
// of T (stored by the keeper after its p entries, off the critical path).  Every owner
// of a row i > c stores v_i itself.
__device__ __forceinline__ void tr_store_reflector_head(EighLarge& e, double tau, double beta, double dc, int c) {
  // n as an opaque value here, so that the row offsets are not held across steps
  int n = e.n;
  asm volatile("" : "+s"(n));
  const int k0 = (c / TB_NBW) * TB_NBW;
#pragma unroll
  for (int q = 0; q < TR_Q; ++q) {
    const int j = threadIdx.x + TR_NT * q;
    if (j >= k0 + 1 && j <= c) e.Vw[(size_t)j * n + c] = 0.0;
  }
  if (threadIdx.x == 0) {
    e.Vw[(size_t)c * n + (n - 1)] = tau;
    e.e[c] = beta;
    e.d[c] = dc;
  }
}

__global__ __launch_bounds__(TR_NT) void tb_reduce_reg(EighLarge e) {
  extern __shared__ double sm[];
  __shared__ double red1[TR_W], red2[TR_W], red3[TR_W][TR_R];
  __shared__ double s_pk1, s_alpha, s_dk;
  __shared__ double pown[TR_R], vow[TR_R];  // p and v at the own rows updated in the next step
  const int n = e.n, G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // scalar: LDS slots addressed without VGPRs
  const bool keeper = g == (n - 1) % G;  // owns row n - 1
  const int last_row = g + G * ((n - 1 - g) / G);
  double* vfull = sm;  // the reflector of the step (n), read for the own rows
  double a[TR_R][TR_Q];
  // own rows of A = sym(P), also kept in Ps for the final residual check
#pragma unroll
  for (int r = 0; r < TR_R; ++r) {
    const int i = g + G * r;
#pragma unroll
    for (int q = 0; q < TR_Q; ++q) {
      const int j = tid + TR_NT * q;
      double x = 0.0;
      if (i < n && j < n) {
        x = 0.5 * (e.P[(size_t)i * n + j] + e.P[(size_t)j * n + i]);
        e.Ps[(size_t)i * n + j] = x;
      }
      a[r][q] = x;
    }
  }
  // reflector 0 from row 0 of sym(P), formed by every workgroup
  double row[TR_Q], vc[TR_Q], vn[TR_Q];
#pragma unroll
  for (int q = 0; q < TR_Q; ++q) {
    const int j = tid + TR_NT * q;
    row[q] = j < n ? 0.5 * (e.P[j] + e.P[(size_t)j * n]) : 0.0;
  }
  double beta;
  double tau = tr_reflector(row, 0, n, vc, red2, &s_alpha, beta);
  if (keeper) tr_store_reflector(e, vc, tau, beta, 0, row);
#pragma unroll
  for (int q = 0; q < TR_Q; ++q) {
    const int j = tid + TR_NT * q;
    if (j < n) vfull[j] = vc[q];
  }
  // p_0 = tau_0 A v_0 for the own rows i >= 1 (buffer 0), and row 1 (row buffer 1)
  {
    double acc[TR_R];
#pragma unroll
    for (int r = 0; r < TR_R; ++r) {
      const int i = g + G * r;
      acc[r] = 0.0;
      if (i >= 1 && i < n) {
#pragma unroll
        for (int q = 0; q < TR_Q; ++q) {
          const int j = tid + TR_NT * q;
          if (j >= 1 && j < n) {
            acc[r] += a[r][q] * vc[q];
            if (i == 1) tb_put(&e.rowbuf[n + j], a[r][q]);
          }
        }
      }
      acc[r] = tl_wave_sum(acc[r]);
    }
    if (lane == 0)
#pragma unroll
      for (int r = 0; r < TR_R; ++r) red3[wave][r] = acc[r];
    __syncthreads();
    if (tid < TR_R) {
      int i = g + G * tid;
      asm volatile("" : "+v"(i));
      double t = 0.0;
      for (int w = 0; w < TR_W; ++w) t += red3[w][tid];
      pown[tid] = (i >= 2 && i < n) ? tau * t : 0.0;  // rows updated in step 0
      if (i >= 1 && i < n) tb_put(&e.pv[i], tau * t);
    }
  }
  if (tid < TR_R) {
    const int i = g + G * tid;
    vow[tid] = (i >= 2 && i < n) ? vfull[i] : 0.0;  // rows updated in step 0
  }
  __syncthreads();

  const int k_end = min(n - 2, last_row - 1);  // steps k < k_end update an own row
  for (int k = 0; k < k_end; ++k) {
    // p_k and the look-ahead row k + 1 (as after step k - 1)
    double pj[TR_Q], rj[TR_Q];
    if (!tr_take(e.pv + (size_t)(k % 3) * n, e.rowbuf + (size_t)((k + 1) % 3) * n, k + 1, n, pj, rj, e.bar, vc,
                 red1, &s_pk1))
      return;
    // slots no reader needs any more: own entries of p_{k-1}, and row k
    {
      double* pold = e.pv + (size_t)((k + 2) % 3) * n;
      int own = g + G * tid;  // opaque: formed here, not held in registers across the steps
      asm volatile("" : "+v"(own));
      if (tid < TR_R && own < n) tr_clear(&pold[own]);
      if (k + 3 < n && (k + 3) % G == g) {
        double* rold = e.rowbuf + (size_t)(k % 3) * n;
#pragma unroll
        for (int q = 0; q < TR_Q; ++q) {
          const int j = tid + TR_NT * q;
          if (j < n) tr_clear(&rold[j]);
        }
      }
    }
    // w = p - (tau / 2) (p . v) v, with p . v summed over the wavefronts' parts
    double dot = 0.0;
#pragma unroll
    for (int w = 0; w < TR_W; ++w) dot += red1[w];
    const double K = -0.5 * tau * dot;
    const double wk1 = s_pk1 + K;  // w_{k+1} (v_{k+1} = 1)
    double wv[TR_Q];
#pragma unroll
    for (int q = 0; q < TR_Q; ++q) {
      wv[q] = pj[q] + K * vc[q];
      row[q] = rj[q] - (wv[q] + wk1 * vc[q]);  // row k + 1 after this step
    }
    // reflector k + 1 from row k + 1
    double taun = 0.0;
    if (k + 1 <= n - 3) {
      taun = tr_reflector(row, k + 1, n, vn, red2, &s_alpha, beta);
      if (keeper)
#pragma unroll
        for (int q = 0; q < TR_Q; ++q)
          if (tid + TR_NT * q == k + 1) s_dk = row[q];  // d_{k+1}
#pragma unroll
      for (int q = 0; q < TR_Q; ++q) {
        const int j = tid + TR_NT * q;
        if (j >= k + 2 && j < n) vfull[j] = vn[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < TR_Q; ++q) {
        vn[q] = 0.0;
        const int j = tid + TR_NT * q;
        if (keeper && j == n - 2) e.d[n - 2] = row[q];  // the last 2 x 2 block
        if (keeper && j == n - 1) e.e[n - 2] = row[q];
      }
    }
    // own rows i >= k + 2, columns j >= k + 2: a_ij -= v_i w_j + w_i v_j, and the
    // partial sums of p_{k+1} = tau_{k+1} A v_{k+1}
    // Branch-free: vow and pown are zero for rows below k + 2 (and past n), v_k and
    // w_k are zero in columns below k + 1 (and past n), and v_{k+1} below k + 2, so
    // only the trailing block changes, except column k + 1 of the own rows, which no
    // later step reads.
    const int rnext = k + 2;
    double acc[TR_R];
#pragma unroll
    for (int r = 0; r < TR_R; ++r) {
      const double vo = vow[r], wo = pown[r] + K * vo;
      acc[r] = 0.0;
#pragma unroll
      for (int q = 0; q < TR_Q; ++q) {
        a[r][q] -= vo * wv[q] + wo * vc[q];
        acc[r] += a[r][q] * vn[q];
      }
    }
#pragma unroll
    for (int r = 0; r < TR_R; ++r) acc[r] = tl_wave_sum(acc[r]);
    if (lane == 0)
#pragma unroll
      for (int r = 0; r < TR_R; ++r) red3[wave][r] = acc[r];
    // the emptied slots are written before any p_{k+1} entry of this workgroup
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (tid < TR_R) {
      int i = g + G * tid;
      asm volatile("" : "+v"(i));
      double t = 0.0;
      for (int w = 0; w < TR_W; ++w) t += red3[w][tid];
      pown[tid] = (i >= rnext + 1 && i < n) ? taun * t : 0.0;  // rows updated in step k + 1
      if (i >= rnext && i < n) tb_put(&e.pv[(size_t)((k + 1) % 3) * n + i], taun * t);
    }
    // the look-ahead row k + 2, stored by its owner
    if (rnext < n && rnext % G == g) {
      double* rbn = e.rowbuf + (size_t)(rnext % 3) * n;
      const int r = (rnext - g) / G;
#pragma unroll
      for (int rr = 0; rr < TR_R; ++rr)
        if (rr == r)
#pragma unroll
          for (int q = 0; q < TR_Q; ++q) {
            const int j = tid + TR_NT * q;
            if (j >= rnext && j < n) tb_put(&rbn[j], a[rr][q]);
          }
    }
#pragma unroll
    for (int q = 0; q < TR_Q; ++q) vc[q] = vn[q];
    tau = taun;
    // v_{k+1} at the own rows: kept for step k + 1, and stored as reflector column
    // k + 1 (rows i >= k + 2); the rest of the column and T by the keeper
    if (tid < TR_R) {
      int i = g + G * tid;
      asm volatile("" : "+v"(i));
      vow[tid] = (i >= rnext + 1 && i < n) ? vfull[i] : 0.0;  // rows updated in step k + 1
      if (k + 1 <= n - 3 && i >= k + 2 && i < n) e.Vw[(size_t)i * n + (k + 1)] = vfull[i];
    }
    if (keeper && k + 1 <= n - 3) tr_store_reflector_head(e, taun, beta, s_dk, k + 1);
  }
  // the last diagonal entry of T: row n - 1, column n - 1 after the last step
  if (keeper && tid == (n - 1) % TR_NT) {
#pragma unroll
    for (int r = 0; r < TR_R; ++r)
#pragma unroll
      for (int q = 0; q < TR_Q; ++q)
        if (g + G * r == n - 1 && q == (n - 1) / TR_NT) e.d[n - 1] = a[r][q];
  }
  // reached only when no wait aborted
  if (keeper && tid == 0 && __hip_atomic_load(&e.bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
    *e.ok = 1;
}

// Eigenvalue brackets of T: workgroup b takes eigenvalues [b m, (b+1) m) (m = TE_CH):
// brackets on the unreduced blocks and multisection down to TB_BISECT_TOL ||T||,
// written to lo / hi (and the block bounds) for the vector kernel.  The brackets are
// narrowed to a few ulps of ||T||, so that the vector kernel's first twisted
// factorization is taken within TB_RQI_TOL eps ||T|| of the eigenvalue and needs no
// second one (a multisection round over all eigenvalues costs less than a factorization
// pass, whose pivots go through global memory).
constexpr double TB_BISECT_TOL = 2e-15;
constexpr double TB_RQI_TOL = 8.0;

__global__ __launch_bounds__(TE_NT) void tb_bisect(EighLarge e) {
  extern __shared__ double sm[];
  __shared__ double red[TE_NT / 64];
  __shared__ double lo_s[TE_CH], hi_s[TE_CH];
  __shared__ int b0_s[TE_CH], b1_s[TE_CH];
  __shared__ double xs[TE_C * TE_NT];
  __shared__ int cnt[TE_C * TE_NT];
  if (!*e.ok) return;  // the reduction aborted
  const int n = e.n, tid = threadIdx.x;
  double* d = sm;
  double* e2 = d + n;
  double tn_loc = 0.0, e2_loc = 0.0;
  for (int i = tid; i < n; i += TE_NT) {
    const double di = e.d[i], el = i > 0 ? fabs(e.e[i - 1]) : 0.0, er = i < n - 1 ? fabs(e.e[i]) : 0.0;
    d[i] = di;
    e2[i] = er * er;
    tn_loc = fmax(tn_loc, fabs(di) + el + er);
    e2_loc = fmax(e2_loc, er * er);
  }
  const double tn = block_max<TE_NT>(tn_loc, red);
  const double pivmin = DBL_MIN * fmax(1.0, block_max<TE_NT>(e2_loc, red));
  const double eps = DBL_EPSILON, split = eps * tn;
  const int j0 = blockIdx.x * TE_CH, m = min(TE_CH, n - j0);
  // per eigenvalue j: its unreduced block [b0, b1) (b0 the last split index <= j, b1 the
  // first one > j; index i is a split where |e_{i-1}| <= eps ||T||) and the Gershgorin
  // bounds of that block, by the whole workgroup
  for (int jj = 0; jj < m; ++jj) {
    const int j = j0 + jj;
    double lo_i = 0.0, hi_i = n;
    for (int i = tid + 1; i < n; i += TE_NT)
      if (fabs(e.e[i - 1]) <= split) {
        if (i <= j) lo_i = fmax(lo_i, (double)i);
        else hi_i = fmin(hi_i, (double)i);
      }
    const int b0 = (int)block_max<TE_NT>(lo_i, red), b1 = (int)-block_max<TE_NT>(-hi_i, red);
    double gl = INFINITY, gu = -INFINITY;
    for (int i = b0 + tid; i < b1; i += TE_NT) {
      const double rr = (i > b0 ? fabs(e.e[i - 1]) : 0.0) + (i < b1 - 1 ? fabs(e.e[i]) : 0.0);
      gl = fmin(gl, d[i] - rr);
      gu = fmax(gu, d[i] + rr);
    }
    gl = -block_max<TE_NT>(-gl, red);
    gu = block_max<TE_NT>(gu, red);
    if (tid == 0) {
      const double margin = 8.0 * n * eps * tn + 4.0 * pivmin;
      lo_s[jj] = gl - margin;
      hi_s[jj] = gu + margin;
      b0_s[jj] = b0;
      b1_s[jj] = b1;
    }
  }
  __syncthreads();
  const int T = max(1, TE_NT / max(m, 1)), K = TE_C * T;
  for (int it = 0; it < TL_MAXIT; ++it) {
    if (tid < m * T) {
      const int jj = tid / T, q = tid - jj * T;
      const double lo = lo_s[jj], hi = hi_s[jj], wd = hi - lo;
      double x[TE_C];
      int c[TE_C];
#pragma unroll
      for (int u = 0; u < TE_C; ++u) x[u] = lo + wd * ((double)(TE_C * q + u + 1) / (double)(K + 1));
      tl_sturm_n<TE_C>(d, e2, b0_s[jj], b1_s[jj], x, pivmin, c);
#pragma unroll
      for (int u = 0; u < TE_C; ++u) {
        xs[TE_C * tid + u] = x[u];
        cnt[TE_C * tid + u] = c[u];
      }
    }
    __syncthreads();
    int more = 0;
    if (tid < m) {
      const int jl = j0 + tid - b0_s[tid];
      double lo = lo_s[tid], hi = hi_s[tid];
      for (int q = 0; q < K; ++q) {
        const double x = xs[tid * K + q];
        if (cnt[tid * K + q] <= jl)
          lo = fmax(lo, x);
        else
          hi = fmin(hi, x);
      }
      lo_s[tid] = lo;
      hi_s[tid] = hi;
      more = (hi - lo) > TB_BISECT_TOL * tn;
    }
    if (!__syncthreads_or(more)) break;
  }
  if (tid < m) {
    e.blo[j0 + tid] = lo_s[tid];
    e.bhi[j0 + tid] = hi_s[tid];
    e.bb[2 * (j0 + tid)] = b0_s[tid];
    e.bb[2 * (j0 + tid) + 1] = b1_s[tid];
  }
}

// Eigenvectors of T: two lanes per eigenvalue (32 eigenvalues per workgroup of 64).
// The twisted factorization of T - lam I splits into independent halves, so the even
// lane of a pair takes the forward pivots D+ (into column j of Zw) and the vector
// above the twist, the odd lane the backward pivots D- (into column j of Aw, free at
// this point) and the vector below it; the twist index (the smallest
// |gamma_i| = |D+_i + D-_i - (d_i - lam)|) and the norm are combined across the pair.
// Both lanes take the same Rayleigh-quotient corrections while they exceed
// TB_RQI_TOL eps ||T|| (the bracket bounds every step), so the pair stays in step.
// Lanes read and write consecutive addresses of the row i of Zw / Aw; the loads are
// issued TV_PF indices ahead.  The residual max|T z - lambda z| is checked.
constexpr int TV_NT = 64;
constexpr int TV_PF = 16;

// The twisted factorization at lam for the pair's eigenvalue (this lane: odd or even);
// writes z / ||z|| into Z (column pointer, ld n) and returns gamma_r / ||z||^2.
__device__ __forceinline__ double tv_twisted(const double* d, const double* ee, const double* e2, int b0, int b1, double lam,
                             double pivmin, double* Z, double* W, int n, bool odd) {
  // 1. pivots: D+ forward from b0 (even lane, into Z), D- backward from b1 - 1 (odd, into W)
  {
    double* P = odd ? W : Z;
    int i = odd ? b1 - 1 : b0;
    double D = tl_piv(d[i] - lam, pivmin);
    P[(size_t)i * n] = D;
    for (int t = 1; t < b1 - b0; ++t) {
      i = odd ? b1 - 1 - t : b0 + t;
      D = tl_piv((d[i] - lam) - (odd ? e2[i] : e2[i - 1]) * tl_rcp(D), pivmin);
      P[(size_t)i * n] = D;
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the partner lane reads these pivots
  // 2. twist index: each lane scans half of the block, the pair keeps the smaller
  //    |gamma| (the larger index on a tie)
  const int mid = (b0 + b1) >> 1, ia = odd ? mid : b0, ib = odd ? b1 : mid;
  int r = ib - 1;
  double best = INFINITY, gr = 0.0;
  {
    double cz[TV_PF], cw[TV_PF];
#pragma unroll
    for (int u = 0; u < TV_PF; ++u) {
      const int i = ia + u;
      cz[u] = i < ib ? Z[(size_t)i * n] : 0.0;
      cw[u] = i < ib ? W[(size_t)i * n] : 0.0;
    }
    for (int i0 = ia; i0 < ib; i0 += TV_PF) {
      double nz[TV_PF], nw[TV_PF];
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) {
        const int i = i0 + TV_PF + u;
        nz[u] = i < ib ? Z[(size_t)i * n] : 0.0;
        nw[u] = i < ib ? W[(size_t)i * n] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) {
        const int i = i0 + u;
        if (i < ib) {
          const double g = cz[u] + cw[u] - (d[i] - lam);
          if (fabs(g) <= best) {
            best = fabs(g);
            gr = g;
            r = i;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) {
        cz[u] = nz[u];
        cw[u] = nw[u];
      }
    }
  }
  {
    const double ob = __shfl_xor(best, 1), og = __shfl_xor(gr, 1);
    const int orr = __shfl_xor(r, 1);
    if (ob < best || (ob == best && orr > r)) {
      best = ob;
      gr = og;
      r = orr;
    }
  }
  // 3. z_r = 1 and the one-sided recurrences: above the twist (even lane)
  //    z_i = -(e_i / D+_i) z_{i+1}, below it (odd lane) z_i = -(e_{i-1} / D-_i) z_{i-1}
  const int len = odd ? b1 - 1 - r : r - b0, step = odd ? 1 : -1;
  const double* src = odd ? W : Z;
  double part = 0.0;
  {
    double z = 1.0, cur[TV_PF];
#pragma unroll
    for (int u = 0; u < TV_PF; ++u) cur[u] = u < len ? src[(size_t)(r + step * (1 + u)) * n] : 1.0;
    for (int t0 = 0; t0 < len; t0 += TV_PF) {
      double nxt[TV_PF];
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) {
        const int t = t0 + TV_PF + u;
        nxt[u] = t < len ? src[(size_t)(r + step * (1 + t)) * n] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) {
        const int t = t0 + u;
        if (t < len) {
          const int i = r + step * (1 + t);
          z = -((odd ? ee[i - 1] : ee[i]) * tl_rcp(cur[u])) * z;
          Z[(size_t)i * n] = z;
          part += z * z;
        }
      }
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) cur[u] = nxt[u];
    }
  }
  if (!odd) Z[(size_t)r * n] = 1.0;
  const double po = __shfl_xor(part, 1);
  const double nrm = 1.0 + (odd ? po + part : part + po);  // the same order on both lanes
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the partner lane scales these entries
  // 4. normalization, each lane one half of the block
  const double sc = 1.0 / sqrt(nrm);
  {
    double cur[TV_PF];
#pragma unroll
    for (int u = 0; u < TV_PF; ++u) cur[u] = ia + u < ib ? Z[(size_t)(ia + u) * n] : 0.0;
    for (int i0 = ia; i0 < ib; i0 += TV_PF) {
      double nxt[TV_PF];
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) {
        const int i = i0 + TV_PF + u;
        nxt[u] = i < ib ? Z[(size_t)i * n] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) {
        const int i = i0 + u;
        if (i < ib) Z[(size_t)i * n] = cur[u] * sc;
      }
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) cur[u] = nxt[u];
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // before the partner reads z or pivots again
  return gr / nrm;
}

__global__ __launch_bounds__(TV_NT) void tb_vectors(EighLarge e) {
  extern __shared__ double sm[];
  if (!*e.ok) return;
  const int n = e.n, tid = threadIdx.x;
  double* d = sm;
  double* ee = d + n;
  double* e2 = ee + n;
  double tn_loc = 0.0, e2_loc = 0.0, fro = 0.0;
  for (int i = tid; i < n; i += TV_NT) {
    d[i] = e.d[i];
    ee[i] = i < n - 1 ? e.e[i] : 0.0;
    e2[i] = ee[i] * ee[i];
    const double el = i > 0 ? fabs(e.e[i - 1]) : 0.0;
    tn_loc = fmax(tn_loc, fabs(d[i]) + el + fabs(ee[i]));
    e2_loc = fmax(e2_loc, e2[i]);
    fro += d[i] * d[i] + 2.0 * e2[i];
  }
  const double tn = tl_wave_max(tn_loc);
  const double pivmin = DBL_MIN * fmax(1.0, tl_wave_max(e2_loc));
  const double scale = sqrt(tl_wave_sum(fro));
  __syncthreads();
  const bool odd = tid & 1;
  const int j = blockIdx.x * (TV_NT / 2) + (tid >> 1);
  double res = 0.0;
  if (j < n) {  // uniform within the pair
    const int b0 = e.bb[2 * j], b1 = e.bb[2 * j + 1];
    double* Z = e.Zw + j;
    double* W = e.Aw + j;
    const int mid = (b0 + b1) >> 1;
    // zeros outside the block, each lane one side
    for (int i = odd ? b1 : 0; i < (odd ? n : b0); ++i) Z[(size_t)i * n] = 0.0;
    const double lo = e.blo[j], hi = e.bhi[j];
    double lam = 0.5 * (lo + hi);
    if (b1 - b0 == 1) {
      if (!odd) Z[(size_t)b0 * n] = 1.0;
      lam = d[b0];
    } else {
      double dl = tv_twisted(d, ee, e2, b0, b1, lam, pivmin, Z, W, n, odd);
      for (int it = 0; it < TL_RQI_MAX && fabs(dl) > TB_RQI_TOL * DBL_EPSILON * tn; ++it) {
        const double nl = lam + dl;
        if (!(nl >= lo && nl <= hi)) break;
        lam = nl;
        dl = tv_twisted(d, ee, e2, b0, b1, lam, pivmin, Z, W, n, odd);
      }
      const double nl = lam + dl;
      lam = (nl >= lo && nl <= hi) ? nl : lam;
    }
    if (!odd) e.w[j] = lam;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    // residual |T z - lam z| over this lane's half of the block, z read once with the
    // loads of the next TV_PF entries in flight
    const int ia = odd ? mid : b0, ib = odd ? b1 : mid;
    double cur[TV_PF], nxt[TV_PF];
#pragma unroll
    for (int u = 0; u < TV_PF; ++u) cur[u] = ia + u < ib ? Z[(size_t)(ia + u) * n] : 0.0;
    double zprev = ia > b0 ? Z[(size_t)(ia - 1) * n] : 0.0;
    const double zend = ib < b1 ? Z[(size_t)ib * n] : 0.0;
    for (int i0 = ia; i0 < ib; i0 += TV_PF) {
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) {
        const int i = i0 + TV_PF + u;
        nxt[u] = i < ib ? Z[(size_t)i * n] : zend;
      }
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) {
        const int i = i0 + u;
        if (i < ib) {
          const double zi = cur[u], znext = u + 1 < TV_PF ? (i + 1 < ib ? cur[u + 1] : zend) : nxt[0];
          double t = (d[i] - lam) * zi;
          if (i > b0) t += ee[i - 1] * zprev;
          if (i < b1 - 1) t += ee[i] * znext;
          res = fmax(res, tl_err(fabs(t)));
          zprev = zi;
        }
      }
#pragma unroll
      for (int u = 0; u < TV_PF; ++u) cur[u] = nxt[u];
    }
  }
  res = tl_wave_max(res);
  if (tid == 0 && !(res <= 1e-12 * scale)) atomicExch(e.ok, 0);
}

// Orthogonality of Z over many workgroups: max |G - I| (G = Z^T Z in Aw) into
// scan[0] (atomic max on the bit pattern), and G <- (I - G) / 2, the factor of the
// Newton-Schulz correction X = Z (3 I - G) / 2 = Z + Z (I - G) / 2.
__global__ __launch_bounds__(256) void tb_orth_scan(EighLarge e) {
  __shared__ double red[4];
  if (!*e.ok) return;
  const int n = e.n;
  double m = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < (int64_t)n * n; idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx / n), j = (int)(idx - (int64_t)i * n);
    const double g = e.Aw[idx], dlt = i == j ? 1.0 : 0.0;
    m = fmax(m, tl_err(fabs(g - dlt)));
    e.Aw[idx] = 0.5 * (dlt - g);
  }
  m = block_max<256>(m, red);
  if (threadIdx.x == 0) atomicMax(reinterpret_cast<unsigned long long*>(e.scan), (unsigned long long)__double_as_longlong(m));
}

// Residual of the accepted result against sym(P): max |R - X diag(w)| (R = sym(P) X
// in Aw) into scan[1] (a max: exact in any order); the partial sums of ||sym(P)||_F^2
// into partial[block], summed in a fixed order by tb_decide, so that the accept-or-
// fall-back decision does not depend on the order the workgroups finish in.
constexpr int TB_RES_BLOCKS = 256;  // <= PREP_BLOCKS: the partials share the Jacobi scratch
static_assert(TB_RES_BLOCKS <= PREP_BLOCKS, "residual partials exceed the scratch");
__global__ __launch_bounds__(256) void tb_res_scan(EighLarge e) {
  __shared__ double red[4];
  if (!*e.ok) return;
  const int n = e.n;
  double r = 0.0, f = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < (int64_t)n * n; idx += (int64_t)gridDim.x * 256) {
    const int j = (int)(idx % n);
    r = fmax(r, tl_err(fabs(e.Aw[idx] - e.X[idx] * e.w[j])));
    f += e.Ps[idx] * e.Ps[idx];
  }
  r = block_max<256>(r, red);
  f = block_sum<256>(f, red);
  if (threadIdx.x == 0) {
    atomicMax(reinterpret_cast<unsigned long long*>(e.scan) + 1, (unsigned long long)__double_as_longlong(r));
    e.partial[blockIdx.x] = f;
  }
}

// which = 0: *ok = 0 unless max|G - I| <= 1e-6;  which = 1: unless the residual
// max <= 1e-11 ||sym(P)||_F.
__global__ void tb_decide(EighLarge e, int which) {
  if (threadIdx.x != 0 || !*e.ok) return;
  const unsigned long long* b = reinterpret_cast<const unsigned long long*>(e.scan);
  if (which == 0) {
    if (!(__longlong_as_double((long long)b[0]) <= 1e-6)) *e.ok = 0;
  } else {
    double f = 0.0;
    for (int q = 0; q < TB_RES_BLOCKS; ++q) f += e.partial[q];
    if (!(__longlong_as_double((long long)b[1]) <= 1e-11 * sqrt(f))) *e.ok = 0;
  }
}

// T factors of the compact WY form of blocks of TB_NBW reflectors (one workgroup
// per block): T[:c, c] = T[:c, :c] (-tau_c g[:c, c]), T[c][c] = tau_c, with the Gram
// matrix g = Y_b^T Y_b of the block already in Gw.  T_b is written nkc times side by
// side, so that T_b (sum over chunks of the partial Y_b^T X) is one product.
__global__ __launch_bounds__(256) void tb_wy_t(EighLarge e) {
  if (!*e.ok) return;
  const int n = e.n, k0 = blockIdx.x * TB_NBW;
  const int m = min(TB_NBW, n - 1 - k0);
  const double* Y = e.Vw;
  const double* Gb = e.Gw + (size_t)blockIdx.x * TB_NBW * TB_NBW;
  const int ldT = e.nkc * TB_NBW;
  double* Tb = e.Tw + (size_t)blockIdx.x * TB_NBW * ldT;
  __shared__ double g[TB_NBW][TB_NBW + 1];
  __shared__ double T[TB_NBW][TB_NBW + 1];
  __shared__ double col[TB_NBW];
  __shared__ double taus[TB_NBW];
  for (int q = threadIdx.x; q < TB_NBW * TB_NBW; q += 256) {
    const int r = q / TB_NBW, c = q - r * TB_NBW;
    g[r][c] = (r < m && c < m) ? Gb[r * m + c] : 0.0;
    T[r][c] = 0.0;
  }
  if (threadIdx.x < m) taus[threadIdx.x] = Y[(size_t)(k0 + threadIdx.x) * n + (n - 1)];
  __syncthreads();
  for (int c = 0; c < m; ++c) {
    const double tau = taus[c];
    const int r = threadIdx.x;
    if (r < c) col[r] = -tau * g[r][c];
    __syncthreads();
    if (r < c) {
      // four partial sums, so that the LDS loads of a group are in flight together
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int q = r;
      for (; q + 4 <= c; q += 4) {
        a0 += T[r][q] * col[q];
        a1 += T[r][q + 1] * col[q + 1];
        a2 += T[r][q + 2] * col[q + 2];
        a3 += T[r][q + 3] * col[q + 3];
      }
      for (; q < c; ++q) a0 += T[r][q] * col[q];
      T[r][c] = (a0 + a1) + (a2 + a3);
    }
    if (r == c) T[c][c] = tau;
    __syncthreads();
  }
  for (int q = threadIdx.x; q < e.nkc * m * m; q += 256) {
    const int c = q / (m * m), rem = q - c * m * m, r = rem / m, j = rem - r * m;
    Tb[(size_t)r * ldT + c * m + j] = T[r][j];
  }
}

// X <- Q X, Q = H_0 H_1 ... H_{n-3} = prod_b (I - Y_b T_b Y_b^T) over the compact-WY
// blocks of TB_NBW reflectors, last block first, in one launch.  The columns of X are
// independent, so workgroup c keeps the 16-column panel c of X in registers for the
// whole product and per block forms
//   W = Y_b^T X_p  (partial sums of the wavefronts over their rows, then summed in a
//                   fixed order, so that the result does not depend on timing),
//   W2 = T_b W,    X_p -= Y_b W2,
// the two large products on the FP64 matrix cores.  Wavefront w holds the 16-row
// blocks w, w + WY_W, ... of the panel in the accumulator layout of
// v_mfma_f64_16x16x4f64 (element r of lane l: row l / 16 + 4 r, column l % 16), which
// is also the operand layout of the four k-steps of those 16 rows in W = Y_b^T X_p.
// Only rows below k0 (the block's first reflector index) take part in block b, and the
// row blocks are dealt out cyclically, so every wavefront has a share of them; the
// steps of the others issue no loads (each step waits for its loads, so an unused load
// would cost a full L2 round trip).
//
// The blocks Y_b are first copied (tb_wy_pack) into the free work matrix as
// Yc[b][row][0 .. TB_NBW) with rows padded to a multiple of 16 and zeros outside
// rows (k0, n) and reflectors [0, mb): the product kernel then loads without masks,
// at offsets that are compile-time constants from one base per row block.  The update
// X_p -= Y_b W2 reads a second, negated copy in the order of its fragments
// (tb_wy_pack_u), so that each of its loads is 512 contiguous bytes.
constexpr int WY_NT = 512;
constexpr int WY_W = WY_NT / 64;  // wavefronts
constexpr int WY_RB = 18;         // row blocks per wavefront
constexpr int WY_NMAX = 16 * WY_W * WY_RB;

__global__ void tb_wy_pack(EighLarge e) {
  if (!*e.ok) return;
  const int n = e.n, np16 = (n + 15) & ~15, nblk = (n - 1 + TB_NBW - 1) / TB_NBW;
  const int64_t total = (int64_t)nblk * np16 * TB_NBW;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(q % TB_NBW);
    const int64_t rq = q / TB_NBW;
    const int row = (int)(rq % np16), b = (int)(rq / np16);
    const int k0 = b * TB_NBW, mb = min(TB_NBW, n - 1 - k0);
    e.Aw[q] = (row > k0 && row < n && c < mb) ? e.Vw[(size_t)row * n + k0 + c] : 0.0;
  }
}

// The blocks again, negated and in the order of the update's fragments, into Vw (free
// once the T factors are formed; npad^2 >= nblk np16 TB_NBW): for block b, row block rb,
// half h, step u and lane l the value -Y_b[16 rb + l % 16][32 h + 4 u + l / 16], so
// that every load of the update reads 512 consecutive bytes.
__global__ void tb_wy_pack_u(EighLarge e) {
  if (!*e.ok) return;
  const int n = e.n, np16 = (n + 15) & ~15, nblk = (n - 1 + TB_NBW - 1) / TB_NBW;
  const int64_t total = (int64_t)nblk * np16 * TB_NBW;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(q & 63), u = (int)((q >> 6) & 7), h = (int)((q >> 9) & 1);
    const int64_t rbb = q >> 10;  // b np16 / 16 + rb
    const int64_t row = 16 * rbb + (l & 15);  // row of block b's Yc, counted from block 0
    e.Vw[q] = -e.Aw[row * TB_NBW + 32 * h + 4 * u + (l >> 4)];
  }
}

__global__ __launch_bounds__(WY_NT) void tb_apply_wy(EighLarge e) {
  if (!*e.ok) return;
  __shared__ double part[WY_W][4][4][64];
  __shared__ double Wl[TB_NBW][17];
  __shared__ double W2l[TB_NBW][17];
  __shared__ double Tl[TB_NBW][TB_NBW + 1];
  const int n = e.n, lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: row-block values are scalar
  const int lr = lane & 15, lk = lane >> 4;
  const int col = blockIdx.x * 16 + lr;
  const int nrb = (n + 15) >> 4, np16 = nrb * 16;
  d4v x[WY_RB];
#pragma unroll
  for (int t = 0; t < WY_RB; ++t) {
    const int rb = wave + WY_W * t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * rb + lk + 4 * r;
      x[t][r] = (rb < nrb && row < n && col < n) ? e.X[(size_t)row * n + col] : 0.0;
    }
  }
  const int nblk = (n - 1 + TB_NBW - 1) / TB_NBW;
  const int ldT = e.nkc * TB_NBW;
  // lane offsets (in doubles) of the two fragment patterns inside a row block of Yc
  const int off_w = lk * TB_NBW + lr;  // W = Y_b^T X: row 4 ks + lk, reflector 16 it + lr
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = b * TB_NBW, mb = min(TB_NBW, n - 1 - k0), rlo = k0 + 1;
    const double* Yc = e.Aw + (size_t)b * np16 * TB_NBW;
    // half row block st of this wavefront takes part in block b (uniform in the
    // wavefront): its loads are issued only then, so the steps above row k0 cost nothing
    auto active = [&](int st) {
      const int rb = wave + WY_W * (st >> 1);
      return rb < nrb && 16 * rb + 15 >= rlo;
    };
    // W = Y_b^T X_p over this wavefront's rows; the loads of each step (half a row
    // block) are issued before the products of the step before, and no instruction
    // moves across steps (which bounds the registers held by loads in flight)
    d4v acc[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) acc[it] = d4v{0.0, 0.0, 0.0, 0.0};
    {
      // steps of half a row block (k-steps 2 h, 2 h + 1)
      double cur[8], nxt[8];
      auto load_w = [&](int st, double (&buf)[8]) {
        const int rb = min(wave + WY_W * (st >> 1), nrb - 1);
        const double* y = Yc + (size_t)rb * 16 * TB_NBW + off_w + 8 * (st & 1) * TB_NBW;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
          for (int it = 0; it < 4; ++it) buf[4 * ks + it] = y[4 * ks * TB_NBW + 16 * it];
      };
      if (active(0)) load_w(0, cur);
#pragma unroll
      for (int st = 0; st < 2 * WY_RB; ++st) {
        if (st + 1 < 2 * WY_RB && active(st + 1)) load_w(st + 1, nxt);
        const int t = st >> 1;
        if (active(st)) {
#pragma unroll
          for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int it = 0; it < 4; ++it)
              acc[it] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[4 * ks + it], x[t][2 * (st & 1) + ks], acc[it], 0,
                                                             0, 0);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) cur[q] = nxt[q];
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r) part[wave][it][r][lane] = acc[it][r];
    __syncthreads();
    // the wavefronts' partial sums, in order; W (64 x 16) element q: row q / 16, column q % 16
    for (int q = threadIdx.x; q < TB_NBW * 16; q += WY_NT) {
      const int i = q >> 4, j = q & 15, it = i >> 4, ii = i & 15;
      const int r = ii >> 2, ln = (ii & 3) * 16 + j;
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < WY_W; ++w) sum += part[w][it][r][ln];
      Wl[i][j] = sum;
    }
    __syncthreads();
    // W2 = T_b W (T_b upper triangular, row i at Tw + i ldT), with T_b staged in LDS
    // (all its loads in flight together)
    {
      const double* Tb = e.Tw + (size_t)b * TB_NBW * ldT;
      for (int q = threadIdx.x; q < TB_NBW * TB_NBW; q += WY_NT) {
        const int i = q / TB_NBW, c = q % TB_NBW;
        Tl[i][c] = (i < mb && c < mb && c >= i) ? Tb[(size_t)i * ldT + c] : 0.0;
      }
      __syncthreads();
      // on the matrix cores: wavefront w < 4 forms rows [16 w, 16 w + 16) of W2
      if (wave < 4) {
        d4v c4 = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < TB_NBW / 4; ++ks)
          c4 = __builtin_amdgcn_mfma_f64_16x16x4f64(Tl[16 * wave + lr][4 * ks + lk], Wl[4 * ks + lk][lr], c4, 0, 0,
                                                    0);
#pragma unroll
        for (int r = 0; r < 4; ++r) W2l[16 * wave + lk + 4 * r][lr] = c4[r];
      }
    }
    __syncthreads();
    // X_p -= Y_b W2 in steps of half a row block (32 reflectors), the loads of the
    // next step issued before the products of this one
    {
      double cur[8], nxt[8];
      const double* Yu = e.Vw + (size_t)b * np16 * TB_NBW;  // the negated blocks, fragment order
      auto load_u = [&](int st, double (&buf)[8]) {
        const int rb = min(wave + WY_W * (st >> 1), nrb - 1);
        const double* y = Yu + ((size_t)rb * 2 + (st & 1)) * 512 + lane;
#pragma unroll
        for (int u = 0; u < 8; ++u) buf[u] = y[64 * u];
      };
      if (active(0)) load_u(0, cur);
#pragma unroll
      for (int st = 0; st < 2 * WY_RB; ++st) {
        if (st + 1 < 2 * WY_RB && active(st + 1)) load_u(st + 1, nxt);
        const int t = st >> 1;
        if (active(st)) {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            x[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[u], W2l[32 * (st & 1) + 4 * u + lk][lr], x[t], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) cur[q] = nxt[q];
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  {
    // bounds and addresses formed anew (opaque copies), not held from the loads above
    int nn = n, cb = col, lkb = lk;
    asm volatile("" : "+s"(nn), "+v"(cb), "+v"(lkb));
    double* Xc = e.X + cb;
#pragma unroll
    for (int t = 0; t < WY_RB; ++t) {
      const int rb = wave + WY_W * t;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * rb + lkb + 4 * r;
        if (row < nn && cb < nn) Xc[(size_t)row * nn] = x[t][r];
      }
    }
  }
}

// rows in registers when they fit: n <= TR_NT TR_Q columns, <= TR_R rows per workgroup
static bool tb_use_reg(const EighLarge& e) {
  return e.n <= TR_NT * TR_Q && e.grid > 0 && (e.n + e.grid - 1) / e.grid <= TR_R;
}

// The reduction's grid barrier needs every workgroup resident at once: cap the grid at
// what the occupancy of the kernel to be launched allows on cu_count CUs (0 when it
// cannot run at all: then only the block Jacobi solver runs).
static void tb_cap_grid(EighLarge& e, int cu_count) {
  const bool reg = tb_use_reg(e);
  const size_t lds = tb_reduce_lds(e.n);
  // the dynamic LDS above the default limit must be allowed before the query
  (void)hipFuncSetAttribute(reg ? reinterpret_cast<const void*>(&tb_reduce_reg) : reinterpret_cast<const void*>(&tb_reduce),
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                   reg ? reinterpret_cast<const void*>(&tb_reduce_reg)
                                                       : reinterpret_cast<const void*>(&tb_reduce),
                                                   reg ? TR_NT : TB_NT, lds) != hipSuccess)
    per_cu = 0;
  const int cap = std::max(per_cu, 0) * cu_count;
  if (e.grid > cap) {
    e.grid = cap;
    // fewer workgroups can move the register path past its rows-per-workgroup limit
    if (e.grid > 0 && reg && !tb_use_reg(e)) tb_cap_grid(e, cu_count);
  }
}

void launch_tb_orth_check(const EighLarge& e, hipStream_t s) {
  tb_orth_scan<<<256, 256, 0, s>>>(e);
  tb_decide<<<1, 64, 0, s>>>(e, 0);
}

void launch_tb_final_check(const EighLarge& e, hipStream_t s) {
  tb_res_scan<<<TB_RES_BLOCKS, 256, 0, s>>>(e);
  tb_decide<<<1, 64, 0, s>>>(e, 1);
}

void launch_tb_reduce(const EighLarge& e, hipStream_t s) {
  const int n = e.n;
  const size_t lds = tb_reduce_lds(n);
  const size_t eig_lds = sizeof(double) * 3 * (size_t)n;
  static size_t attr_r = 0, attr_e = 0;
  if (lds > attr_r) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&tb_reduce), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    attr_r = lds;
  }
  if (eig_lds > attr_e) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&tb_bisect), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)eig_lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&tb_vectors), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)eig_lds);
    attr_e = eig_lds;
  }
  static size_t attr_g = 0;
  if (lds > attr_g) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&tb_reduce_reg), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    attr_g = lds;
  }
  tb_init<<<1, 256, 0, s>>>(e, tb_use_reg(e) ? 1 : 0);
  if (e.grid < 1) return;  // no resident grid possible: *ok stays 0, the Jacobi solver runs
  if (tb_use_reg(e))
    tb_reduce_reg<<<e.grid, TR_NT, lds, s>>>(e);
  else
    tb_reduce<<<e.grid, TB_NT, lds, s>>>(e);
}

void launch_tb_eigenpairs(const EighLarge& e, hipStream_t s) {
  const int n = e.n;
  const size_t eig_lds = sizeof(double) * 3 * (size_t)n;
  tb_bisect<<<(n + TE_CH - 1) / TE_CH, TE_NT, tb_bisect_lds(n), s>>>(e);
  tb_vectors<<<(n + TV_NT / 2 - 1) / (TV_NT / 2), TV_NT, eig_lds, s>>>(e);
}

void launch_tb_wy_t(const EighLarge& e, hipStream_t s) {
  const int nblk = (e.n - 1 + TB_NBW - 1) / TB_NBW;
  if (nblk > 0) tb_wy_t<<<nblk, 256, 0, s>>>(e);
}

bool tb_apply_wy_fits(int n) { return n >= 2 && n <= WY_NMAX; }

void launch_tb_apply_wy(const EighLarge& e, hipStream_t s) {
  if (!tb_apply_wy_fits(e.n)) return;
  tb_wy_pack<<<1024, 256, 0, s>>>(e);
  tb_wy_pack_u<<<1024, 256, 0, s>>>(e);
  tb_apply_wy<<<(e.n + 15) / 16, WY_NT, 0, s>>>(e);
}

static bool g_attr = false;

void launch_eigh_large(const EighLarge& e, int max_sweeps, int* status, hipStream_t s, bool check_host) {
  if (e.n <= 0) return;
  const size_t inner_lds = sizeof(double) * (2 * SUB * SUB + SUB);
  const size_t upd_lds = sizeof(double) * 2 * SUB * LD;
  if (!g_attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&bjl_inner), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)inner_lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&bjl_update), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)upd_lds);
    g_attr = true;
  }
  const int half = e.nb / 2;
  const int tasks = half * half + (e.npad / SUB) * half;
  bjl_prepare<<<PREP_BLOCKS, U_NT, 0, s>>>(e, e.partial);
  bjl_start<<<1, 64, 0, s>>>(e, e.partial);
  if (check_host) {  // accepted tridiagonal result (or a zero matrix): no sweep at all
    int done = 0;
    if (hipMemcpyAsync(&done, &e.st->done, sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess &&
        hipStreamSynchronize(s) == hipSuccess && done)
      max_sweeps = 0;
  }
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int r = 0; r < e.nb - 1; ++r) {
      bjl_inner<<<half, L_NT, inner_lds, s>>>(e, r);
      bjl_update<<<tasks, U_NT, upd_lds, s>>>(e, r);
    }
    bjl_offmax<<<OFF_BLOCKS, U_NT, 0, s>>>(e);
    bjl_sweep_end<<<1, 64, 0, s>>>(e, max_sweeps, status);
    if (check_host) {
      int done = 0;
      if (hipMemcpyAsync(&done, &e.st->done, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) break;
      if (hipStreamSynchronize(s) != hipSuccess || done) break;
    }
  }
  const int64_t nn = (int64_t)e.n * e.n;
  bjl_finish<<<(int)std::min<int64_t>(1024, (nn + 255) / 256), 256, 0, s>>>(e, status);
}

}  // namespace etdm
