// FP64 symmetric eigensolver for large n: block-cyclic Jacobi with matrix-core updates.
//
// The matrix (padded with zero rows/columns to npad = 64 * ceil(n / 64), which
// never rotate) is split into nb = npad / 32 blocks of 32 indices.  A sweep runs
// nb - 1 rounds of the round-robin pairing of the blocks.  In a round:
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
  const int n = e.n, npad = e.npad;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (int64_t)n * n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / n), k = (int)(idx - (int64_t)i * n);
    e.X[idx] = e.Vw[(size_t)i * npad + k];
    if (k == 0) e.w[i] = e.Aw[(size_t)i * npad + i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && !e.st->finite) atomicOr(status, ST_NONFINITE);
}

size_t eigh_large_workspace(int n, size_t* npad_out) {
  const size_t npad = (size_t)((n + SUB - 1) / SUB) * SUB;
  if (npad_out) *npad_out = npad;
  const size_t half = npad / BLK / 2;
  return 2 * npad * npad + half * SUB * SUB + PREP_BLOCKS;
}

static bool g_attr = false;

void launch_eigh_large(const EighLarge& e, int max_sweeps, int* status, hipStream_t s, bool check_host) {
  if (e.n <= 0) return;
  const size_t inner_lds = sizeof(double) * (2 * SUB * SUB + SUB);
  const size_t upd_lds = sizeof(double) * 2 * SUB * LD;
  if (!g_attr) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&bjl_inner), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)inner_lds);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&bjl_update), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)upd_lds);
    g_attr = true;
  }
  const int half = e.nb / 2;
  const int tasks = half * half + (e.npad / SUB) * half;
  bjl_prepare<<<PREP_BLOCKS, U_NT, 0, s>>>(e, e.partial);
  bjl_start<<<1, 64, 0, s>>>(e, e.partial);
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
