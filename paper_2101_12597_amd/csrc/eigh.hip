// FP64 Hermitian eigensolvers, one workgroup per matrix: parallel cyclic Jacobi
// (complex matrices, and the fallback of the small real solver) and, for small
// real symmetric matrices, a tridiagonal solver in LDS (further below).
//
// Each sweep runs n' - 1 rounds (n' = n rounded up to even) of the round-robin
// ("circle") pairing, so every index pair is rotated exactly once per sweep and
// the n'/2 rotations of a round act on disjoint index pairs.  Because the pairs
// are disjoint, the two-sided update A <- J^H A J splits into independent 2 x 2
// blocks A[{p_a,q_a},{p_b,q_b}] <- J_a^H A_blk J_b, and V <- V J into
// independent row pairs: a round is one barrier for the rotation parameters and
// one pass over the matrix, with no dependence between threads.
//
// Rotation of pair (p, q): with a_pq = |a_pq| e^{i phi} and
//   tau = (a_qq - a_pp) / (2 |a_pq|),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1 / sqrt(1 + t^2), s = t c,
// J = [[c, s e^{i phi}], [-s e^{-i phi}, c]] makes (J^H A J)_pq = 0 (the smaller
// of the two rotation angles, |theta| <= pi/4).
//
// Convergence: the solver stops after a sweep whose largest |a_pq| (seen when
// its rotation was formed) is below 1e-12 ||A||_F.  For well separated
// eigenvalues convergence is quadratic and the entries left after that sweep are
// far smaller; a large multiple eigenvalue (the null space of B B^T when B has
// more rows than columns) converges only about tenfold per sweep below 1e-8,
// which is what sets the threshold.  More than MAX_SWEEPS sweeps sets ST_EIGH.
#include <cfloat>

#include "common.h"
#include "tridiag.h"

namespace etdm {

constexpr int MAX_SWEEPS = 40;
constexpr double CONV_TOL = 1e-12;

__device__ __forceinline__ void rr_pair(int r, int j, int nn, int& p, int& q) {
  if (j == 0) {
    p = r;
    q = nn - 1;
  } else {
    p = (r + j) % (nn - 1);
    q = (r - j + (nn - 1)) % (nn - 1);
  }
}

__device__ __forceinline__ void jacobi_cs(double app, double aqq, double mag, double& c, double& s) {
  double tau = (aqq - app) / (2.0 * mag);
  double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

// ---------------------------------------------------------------------------
// real symmetric Jacobi sweeps on a matrix and vectors in LDS (n <= EIGH_LDS_MAX),
// 1024 threads.  Same rounds as above; the per-round index maps are advanced
// incrementally (no integer division) and the pairing wraps without modulo.
// Returns whether the sweeps converged.
// ---------------------------------------------------------------------------
constexpr int JL_NT = 1024;

__device__ __forceinline__ void rr_pair_fast(int r, int j, int m, int nn, int& p, int& q) {
  // m = nn - 1 players on the circle, player nn - 1 fixed
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

__device__ bool jacobi_lds_sweeps(double* A, double* V, double* pc, double* ps, int n, double scale,
                                  double* red) {
  const int nn = n + (n & 1), half = nn / 2, m = nn - 1;
  const int tid = threadIdx.x;
  bool converged = n == 1 || scale == 0.0;
  // Thread t < nact keeps one column pair jb = t % half for the whole round (its
  // rotation is read once) and walks the row pairs ja = t / half + k * stride;
  // the same thread walks rows i of V for pair jb.  One division, done once.
  const int stride = JL_NT / half, nact = stride * half;
  const int jb = tid % half, ja0 = tid / half;
  for (int sweep = 0; sweep < MAX_SWEEPS && !converged; ++sweep) {
    double maxoff = 0.0;
    for (int r = 0; r < m; ++r) {
      if (tid < half) {
        int p, q;
        rr_pair_fast(r, tid, m, nn, p, q);
        double c = 1.0, sn = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          maxoff = fmax(maxoff, fabs(apq));
          if (apq != 0.0) {
            jacobi_cs(A[p * n + p], A[q * n + q], fabs(apq), c, sn);
            if (apq < 0.0) sn = -sn;
          }
        }
        pc[tid] = c;
        ps[tid] = sn;
      }
      __syncthreads();
      if (tid < nact) {
        int pb, qb;
        rr_pair_fast(r, jb, m, nn, pb, qb);
        const double cb = pc[jb], sb = ps[jb];
        const bool vb = qb < n;
        // A <- J^T A J, one 2 x 2 block per (ja, jb)
        for (int ja = ja0; ja < half; ja += stride) {
          int pa, qa;
          rr_pair_fast(r, ja, m, nn, pa, qa);
          const double ca = pc[ja], sa = ps[ja];
          const bool va = qa < n;
          const double x00 = A[pa * n + pb];
          const double x01 = vb ? A[pa * n + qb] : 0.0;
          const double x10 = va ? A[qa * n + pb] : 0.0;
          const double x11 = (va && vb) ? A[qa * n + qb] : 0.0;
          const double y00 = x00 * cb - x01 * sb, y01 = x00 * sb + x01 * cb;
          const double y10 = x10 * cb - x11 * sb, y11 = x10 * sb + x11 * cb;
          double z00 = ca * y00 - sa * y10, z01 = ca * y01 - sa * y11;
          double z10 = sa * y00 + ca * y10, z11 = sa * y01 + ca * y11;
          if (ja == jb) z01 = z10 = 0.0;
          A[pa * n + pb] = z00;
          if (vb) A[pa * n + qb] = z01;
          if (va) A[qa * n + pb] = z10;
          if (va && vb) A[qa * n + qb] = z11;
        }
        // V <- V J for rows i of this thread and pair jb
        if (vb)
          for (int i = ja0; i < n; i += stride) {
            const double vp = V[i * n + pb], vq = V[i * n + qb];
            V[i * n + pb] = vp * cb - vq * sb;
            V[i * n + qb] = vp * sb + vq * cb;
          }
      }
      __syncthreads();
    }
    converged = block_max<JL_NT>(maxoff, red) <= CONV_TOL * scale;
  }
  return converged;
}

// ---------------------------------------------------------------------------
// real symmetric, n <= EIGH_LDS_MAX, one workgroup of 1024 threads per matrix,
// everything in LDS:
//   1. Householder reduction A = Q T Q^T to tridiagonal T (d, e), Q^T accumulated;
//   2. T is split where |e_k| <= eps ||T||; the eigenvalues of every unreduced
//      block are bracketed by multisection (2 T points per eigenvalue and round)
//      on Sturm counts of the LDL^T pivots, down to 1e-8 ||T||;
//   3. per eigenvalue, twisted factorizations of T - lambda I (forward pivots D+,
//      backward pivots D-, twist index r minimising |D+_r + D-_r - (d_r - lambda)|)
//      give the eigenvector (z_r = 1 and the two one-sided recurrences outward) and
//      the Rayleigh-quotient correction gamma_r / ||z||^2 of lambda, iterated while
//      the correction is above rounding level (the bracket bounds every step);
//   4. X = Q Z on the matrix cores;
//   5. check: G = X^T X; one Newton-Schulz step X <- X (3 I - G) / 2 when
//      max|G - I| > 1e-13, and the residual max|A X - X diag(lambda)|.
// A matrix whose vectors are not orthogonal to 1e-6 (repeated or tightly
// clustered eigenvalues, for which independent twisted vectors coincide) or
// whose residual exceeds 1e-12 ||A||_F is solved again by the Jacobi sweeps.
// ---------------------------------------------------------------------------
constexpr int TL_NT = 1024;
constexpr int TL_MAXT = 3;             // 16 x 16 tiles per wavefront: ceil(36 / 16)
constexpr double TL_ORTH_NS = 1e-13;
constexpr double TL_ORTH_MAX = 1e-6;
constexpr double TL_RES_MAX = 1e-12;

typedef double tl_d4 __attribute__((ext_vector_type(4)));

// acc = op(X) Y for n x n row-major LDS matrices (ld n), op(X) = X or X^T.
// Wavefront w owns tiles w, w + 16, w + 32 of the ceil(n/16)^2 grid.
template <bool XT>
__device__ void tl_mm(const double* X, const double* Y, int n, tl_d4 (&acc)[TL_MAXT]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = (n + 15) >> 4, lr = lane & 15, lk = lane >> 4;
  for (int s = 0; s < TL_MAXT; ++s) {
    acc[s] = tl_d4{0.0, 0.0, 0.0, 0.0};
    const int t = wave + 16 * s;
    if (t >= nt * nt) continue;  // uniform in the wavefront
    const int row = (t / nt) * 16 + lr, col = (t % nt) * 16 + lr;
    for (int k0 = 0; k0 < n; k0 += 4) {
      const int k = k0 + lk;
      double a = 0.0, b = 0.0;
      if (k < n) {
        if (row < n) a = XT ? X[k * n + row] : X[row * n + k];
        if (col < n) b = Y[k * n + col];
      }
      acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
    }
  }
}

// (i, j) of accumulator element r of tile slot s of this lane; false outside n x n
__device__ __forceinline__ bool tl_elem(int n, int s, int r, int& i, int& j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nt = (n + 15) >> 4, t = wave + 16 * s;
  if (t >= nt * nt) return false;
  i = (t / nt) * 16 + (lane >> 4) + 4 * r;
  j = (t % nt) * 16 + (lane & 15);
  return i < n && j < n;
}

__device__ __forceinline__ void tl_store(double* C, int n, const tl_d4 (&acc)[TL_MAXT]) {
  for (int s = 0; s < TL_MAXT; ++s)
    for (int r = 0; r < 4; ++r) {
      int i, j;
      if (tl_elem(n, s, r, i, j)) C[i * n + j] = acc[s][r];
    }
}

constexpr int TL_NCH = 5;                     // row chunks of the matrix-vector products
constexpr int TL_PMLD = 2 * EIGH_LDS_MAX;     // stride of their partial sums
// LDS bytes of eigh_tridiag_lds for size n
static size_t tl_lds_bytes(int n) {
  return sizeof(double) * (2 * (size_t)n * n + 6 * (size_t)n + TL_NCH * TL_PMLD + TL_XS) +
         sizeof(int) * (2 * (size_t)n + TL_XS);
}

// Householder reduction A = Q T Q^T of the symmetric n x n matrix A (LDS,
// row-major, both triangles kept), with QT = Q^T accumulated (QT = I on entry).
// Step k takes the reflector from row k right of the diagonal (row k equals
// column k and is final); every wavefront computes the same reflector scalars
// with a DPP sum.  Then, between two barriers:
//   B: p = A_t v over the trailing columns and u = Q v over all rows, as column
//      sums (coalesced row reads), by 3 x TL_NCH wavefronts over row chunks, partial
//      sums to LDS;
//   C: K = -tau p.v / 2, w = tau p + K v; A_t -= v w^T + w v^T (8 wavefronts),
//      QT[k+1:, :] -= tau v u^T (8 wavefronts), rows in groups of 8 loads.
// The entries of v and w that a row needs come from LDS copies (vw: 256 doubles), read
// by all lanes at one address (a broadcast); every wavefront writes the same values
// there, so its own reads never wait for another wavefront.
// On return vd[0..n-1], ve[0..n-2] hold T.
__device__ void tl_tridiag(double* A, double* QT, double* vd, double* ve, double* Pm, double* vw, int n) {
  double* vsh = vw;        // v_{k+1+i}, i < L
  double* wsh = vw + 128;  // w_{k+1+i}
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int k = 0; k < n - 2; ++k) {
    const int L = n - k - 1;
    const int i0 = k + 1 + lane, i1 = i0 + 64;
    const double x0 = i0 < n ? A[k * n + i0] : 0.0;
    const double x1 = i1 < n ? A[k * n + i1] : 0.0;
    const double alpha = tl_readlane(x0, 0);
    const double s2 = tl_wave_sum((lane > 0 ? x0 * x0 : 0.0) + x1 * x1);
    double tau = 0.0, beta = alpha, inv = 0.0;
    if (s2 != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + s2), alpha);
      tau = (beta - alpha) / beta;
      inv = 1.0 / (alpha - beta);
    }
    if (threadIdx.x == 0) {
      ve[k] = beta;
      vd[k] = A[k * n + k];
    }
    if (tau == 0.0) continue;  // the column is already reduced; nothing changes
    const double v0 = lane == 0 ? 1.0 : x0 * inv;  // v_{k+1+lane}
    const double v1 = x1 * inv;                    // v_{k+65+lane}
    vsh[lane] = v0;
    vsh[lane + 64] = v1;
    if (wave < 3 * TL_NCH) {
      const int ow = wave % 3, ch = wave / 3;
      const int o = 64 * ow + lane;  // output: o < L -> p_{k+1+o}, else u_{o-L}
      const int jb = ch * L / TL_NCH, je = (ch + 1) * L / TL_NCH;
      const double* base = o < L ? A + (k + 1) * n + (k + 1 + o)
                                 : (o < L + n ? QT + (k + 1) * n + (o - L) : A + (k + 1) * n + (k + 1));
      double acc0 = 0.0, acc1 = 0.0;
      // groups of eight rows, their loads in flight together
      int jj = jb;
      for (; jj + 8 <= je; jj += 8) {
        double a[8], vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a[u] = base[(jj + u) * n];
          vv[u] = vsh[jj + u];
        }
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          acc0 += a[u] * vv[u];
          acc1 += a[u + 1] * vv[u + 1];
        }
      }
      for (; jj < je; ++jj) acc0 += base[jj * n] * vsh[jj];
      if (o < L + n) Pm[ch * TL_PMLD + o] = acc0 + acc1;
    }
    __syncthreads();
    double p0 = 0.0, p1 = 0.0;
    {  // all partial sums loaded before the first add; entries past L are not p
      double pa[TL_NCH], pb[TL_NCH];
#pragma unroll
      for (int ch = 0; ch < TL_NCH; ++ch) {
        pa[ch] = Pm[ch * TL_PMLD + lane];
        pb[ch] = Pm[ch * TL_PMLD + lane + 64];
      }
#pragma unroll
      for (int ch = 0; ch < TL_NCH; ++ch) {
        p0 += pa[ch];
        p1 += pb[ch];
      }
      if (lane >= L) p0 = 0.0;
      if (lane + 64 >= L) p1 = 0.0;
    }
    p0 *= tau;
    p1 *= tau;
    const double K = -0.5 * tau * tl_wave_sum(p0 * v0 + p1 * v1);
    const double w0 = p0 + K * v0, w1 = p1 + K * v1;
    wsh[lane] = w0;
    wsh[lane + 64] = w1;
    const int grp = wave >> 3, cb = wave & 1, rc = (wave >> 1) & 3;
    const int col = 64 * cb + lane;
    const int rb = rc * L / 4, re = (rc + 1) * L / 4;
    // groups of 8 rows whose loads are issued before any of their stores
    if (grp == 0) {
      const int j = k + 1 + min(col, L - 1);
      const double vj = cb ? v1 : v0, wj = cb ? w1 : w0;
      int ii = rb;
      for (; ii + 8 <= re; ii += 8) {
        double x[8], vv[8], ww[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          x[u] = A[(k + 1 + ii + u) * n + j];
          vv[u] = vsh[ii + u];
          ww[u] = wsh[ii + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] -= vv[u] * wj + ww[u] * vj;
        if (col < L)
#pragma unroll
          for (int u = 0; u < 8; ++u) A[(k + 1 + ii + u) * n + j] = x[u];
      }
      for (; ii < re; ++ii) {
        double* a = A + (k + 1 + ii) * n + j;
        const double x = *a - (vsh[ii] * wj + wsh[ii] * vj);
        if (col < L) *a = x;
      }
    } else {
      const int r = min(col, n - 1);
      double ur = 0.0;
      {
        double pu[TL_NCH];
#pragma unroll
        for (int ch = 0; ch < TL_NCH; ++ch) pu[ch] = Pm[ch * TL_PMLD + L + r];
#pragma unroll
        for (int ch = 0; ch < TL_NCH; ++ch) ur += pu[ch];
      }
      const double tu = tau * ur;
      int jj = rb;
      for (; jj + 8 <= re; jj += 8) {
        double x[8], vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          x[u] = QT[(k + 1 + jj + u) * n + r];
          vv[u] = vsh[jj + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] -= vv[u] * tu;
        if (col < n)
#pragma unroll
          for (int u = 0; u < 8; ++u) QT[(k + 1 + jj + u) * n + r] = x[u];
      }
      for (; jj < re; ++jj) {
        double* q = QT + (k + 1 + jj) * n + r;
        const double x = *q - vsh[jj] * tu;
        if (col < n) *q = x;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (n >= 2) {
      vd[n - 2] = A[(n - 2) * n + n - 2];
      ve[n - 2] = A[(n - 1) * n + n - 2];
    }
    vd[n - 1] = A[(n - 1) * n + n - 1];
  }
}

// Splitting of T (d, e) where |e_k| <= eps ||T||, Gershgorin brackets per
// unreduced block, and multisection on Sturm counts down to TL_BISECT_TOL ||T||.
// On return lo/hi bracket eigenvalue j (ascending within its block [b0[j], b1[j])),
// e2 holds e^2, tn = ||T||_inf-like bound, pivmin the pivot floor.  Called by all
// threads of a workgroup of TL_NT threads; xs/cnt hold TL_XS entries.
__device__ void tl_eigen_brackets(const double* vd, const double* ve, double* ve2, double* vlo, double* vhi,
                                  double* xs, int* cnt, int* ib0, int* ib1, int n, double* red, double& tn,
                                  double& pivmin) {
  const int tid = threadIdx.x;
  double tn_loc = 0.0, e2_loc = 0.0;
  for (int i = tid; i < n; i += TL_NT) {
    const double el = i > 0 ? fabs(ve[i - 1]) : 0.0, er = i < n - 1 ? fabs(ve[i]) : 0.0;
    tn_loc = fmax(tn_loc, fabs(vd[i]) + el + er);
    if (i < n - 1) {
      ve2[i] = ve[i] * ve[i];
      e2_loc = fmax(e2_loc, ve2[i]);
    }
  }
  tn = block_max<TL_NT>(tn_loc, red);
  pivmin = DBL_MIN * fmax(1.0, block_max<TL_NT>(e2_loc, red));
  const double eps = DBL_EPSILON, split = eps * tn;
  // split points of T (|e_i| <= split) as a bit mask (one ballot per wavefront,
  // n <= 64 TL_SPLIT_WORDS), so that every eigenvalue finds the unreduced block of
  // its index with bit scans
  constexpr int TL_SPLIT_WORDS = (HT_MAX + 63) / 64;
  static_assert(TL_SPLIT_WORDS * 64 <= TL_NT && EIGH_LDS_MAX <= HT_MAX, "one wavefront per mask word");
  __shared__ unsigned long long s_split[TL_SPLIT_WORDS];
  if ((tid >> 6) < TL_SPLIT_WORDS) {
    const int i = tid;
    const unsigned long long m = __ballot(i < n - 1 && fabs(ve[i]) <= split);
    if ((tid & 63) == 0) s_split[tid >> 6] = m;
  }
  // one Gershgorin interval for all blocks (the off-diagonals at the split points
  // left out); it contains the spectrum of every block
  double gl = INFINITY, gu = -INFINITY;
  for (int i = tid; i < n; i += TL_NT) {
    const double r = (i > 0 && fabs(ve[i - 1]) > split ? fabs(ve[i - 1]) : 0.0) +
                     (i < n - 1 && fabs(ve[i]) > split ? fabs(ve[i]) : 0.0);
    gl = fmin(gl, vd[i] - r);
    gu = fmax(gu, vd[i] + r);
  }
  gl = -block_max<TL_NT>(-gl, red);
  gu = block_max<TL_NT>(gu, red);
  const double margin = 8.0 * n * eps * tn + 4.0 * pivmin;
  for (int j = tid; j < n; j += TL_NT) {
    // b0 = 1 + (last split point below j), b1 = 1 + (first split point at or above j)
    int lo_split = -1, hi_split = n - 1;
    for (int w = (j - 1) >> 6; j > 0 && w >= 0; --w) {
      const int top = j - 1 - 64 * w;  // highest bit of word w to consider
      const unsigned long long m = s_split[w] & (top >= 63 ? ~0ull : ((2ull << top) - 1));
      if (m) {
        lo_split = 64 * w + 63 - __clzll(m);
        break;
      }
    }
    for (int w = j >> 6; w < TL_SPLIT_WORDS; ++w) {
      const int bot = j - 64 * w;  // lowest bit of word w to consider
      const unsigned long long m = s_split[w] & (bot <= 0 ? ~0ull : (~0ull << bot));
      if (m) {
        hi_split = min(64 * w + __ffsll(m) - 1, n - 1);
        break;
      }
    }
    vlo[j] = gl - margin;
    vhi[j] = gu + margin;
    ib0[j] = lo_split + 1;
    ib1[j] = hi_split + 1;
  }
  __syncthreads();
  // T threads per eigenvalue, two points each
  const int T = max(1, min(8, (TL_XS / 2) / n)), K = 2 * T;
  for (int it = 0; it < TL_MAXIT; ++it) {
    if (tid < n * T) {
      const int j = tid / T, m = tid - j * T;
      const double lo = vlo[j], hi = vhi[j], w = hi - lo;
      const double x0 = lo + w * ((double)(2 * m + 1) / (double)(K + 1));
      const double x1 = lo + w * ((double)(2 * m + 2) / (double)(K + 1));
      int c0, c1;
      tl_sturm2(vd, ve2, ib0[j], ib1[j], x0, x1, pivmin, c0, c1);
      xs[2 * tid] = x0;
      xs[2 * tid + 1] = x1;
      cnt[2 * tid] = c0;
      cnt[2 * tid + 1] = c1;
    }
    __syncthreads();
    int more = 0;
    if (tid < n) {
      const int jl = tid - ib0[tid];
      double lo = vlo[tid], hi = vhi[tid];
      for (int m = 0; m < K; ++m) {
        const double x = xs[tid * K + m];
        if (cnt[tid * K + m] <= jl)
          lo = fmax(lo, x);
        else
          hi = fmin(hi, x);
      }
      vlo[tid] = lo;
      vhi[tid] = hi;
      more = (hi - lo) > TL_BISECT_TOL * tn;
    }
    if (!__syncthreads_or(more)) break;
  }
}

__global__ __launch_bounds__(TL_NT) void eigh_tridiag_lds(const EighProb* __restrict__ probs, int* status) {
  extern __shared__ double smem[];
  __shared__ double red[TL_NT / 64];
  const EighProb pr = probs[blockIdx.x];
  const int n = pr.n;
  if (n <= 0) return;
  const int tid = threadIdx.x;
  double* R1 = smem;         // A, then Z, then the Newton-Schulz factor, then A again
  double* R2 = R1 + n * n;   // Q^T, then X
  double* vd = R2 + n * n;   // diagonal of T
  double* ve = vd + n;       // off-diagonal of T (n - 1)
  double* ve2 = ve + n;      // its squares
  double* vlo = ve2 + n;     // eigenvalue brackets
  double* vhi = vlo + n;
  double* vlam = vhi + n;    // eigenvalues
  double* Pm = vlam + n;     // partial matrix-vector sums (TL_NCH x TL_PMLD)
  double* xs = Pm + TL_NCH * TL_PMLD;  // multisection points (TL_XS)
  int* ib0 = reinterpret_cast<int*>(xs + TL_XS);  // unreduced block of each eigenvalue
  int* ib1 = ib0 + n;
  int* cnt = ib1 + n;        // Sturm counts (TL_XS)

  auto load_sym = [&]() {
    for (int e = tid; e < n * n; e += TL_NT) {
      const int i = e / n, k = e - i * n;
      // symmetric part: products formed in reduced precision need not be exactly symmetric
      R1[e] = 0.5 * (pr.A[e] + pr.A[k * n + i]);
    }
  };
  auto set_identity = [&](double* M) {
    for (int e = tid; e < n * n; e += TL_NT) {
      const int i = e / n;
      M[e] = (e == i * n + i) ? 1.0 : 0.0;
    }
  };
  load_sym();
  set_identity(R2);
  __syncthreads();
  double fro = 0.0;
  for (int e = tid; e < n * n; e += TL_NT) fro += R1[e] * R1[e];
  const double scale = sqrt(block_sum<TL_NT>(fro, red));
  if (!isfinite(scale) || scale == 0.0 || n == 1) {
    for (int i = tid; i < n; i += TL_NT) pr.w[i] = R1[i * n + i];
    for (int e = tid; e < n * n; e += TL_NT) pr.V[e] = R2[e];
    if (!isfinite(scale) && tid == 0) atomicOr(status, ST_NONFINITE);
    return;
  }

  // 1. tridiagonal T and Q^T
  tl_tridiag(R1, R2, vd, ve, Pm, xs, n);  // xs: free until the multisection
  __syncthreads();

  // 2. splitting, brackets, multisection down to TL_BISECT_TOL ||T||
  double tn, pivmin;
  tl_eigen_brackets(vd, ve, ve2, vlo, vhi, xs, cnt, ib0, ib1, n, red, tn, pivmin);
  const double eps = DBL_EPSILON;

  // 3. eigenvectors of T (column j of Z in R1, by thread j), with Rayleigh-quotient
  //    corrections of the eigenvalue from each twisted factorization; a correction
  //    that leaves the bracket is not taken
  if (tid < n) vlam[tid] = tl_vector<0>(vd, ve, ve2, ib0[tid], ib1[tid], vlo[tid], vhi[tid], tn, pivmin, R1, n, tid, n);
  __syncthreads();

  // 4. X = Q Z = (Q^T)^T Z
  tl_d4 acc[TL_MAXT];
  tl_mm<true>(R2, R1, n, acc);
  __syncthreads();
  tl_store(R2, n, acc);
  __syncthreads();

  // 5. orthogonality, one Newton-Schulz step if needed, residual
  tl_mm<true>(R2, R2, n, acc);
  double orth_loc = 0.0;
  for (int s = 0; s < TL_MAXT; ++s)
    for (int r = 0; r < 4; ++r) {
      int i, j;
      if (tl_elem(n, s, r, i, j)) orth_loc = fmax(orth_loc, tl_err(fabs(acc[s][r] - (i == j ? 1.0 : 0.0))));
    }
  const double orth = block_max<TL_NT>(orth_loc, red);
  bool accept = orth <= TL_ORTH_MAX;
  if (accept && orth > TL_ORTH_NS) {
    for (int s = 0; s < TL_MAXT; ++s)
      for (int r = 0; r < 4; ++r) {
        int i, j;
        if (tl_elem(n, s, r, i, j)) R1[i * n + j] = (i == j ? 1.5 : 0.0) - 0.5 * acc[s][r];
      }
    __syncthreads();
    tl_mm<false>(R2, R1, n, acc);
    __syncthreads();
    tl_store(R2, n, acc);
  }
  __syncthreads();
  load_sym();
  __syncthreads();
  if (accept) {
    tl_mm<false>(R1, R2, n, acc);
    double res_loc = 0.0;
    for (int s = 0; s < TL_MAXT; ++s)
      for (int r = 0; r < 4; ++r) {
        int i, j;
        if (tl_elem(n, s, r, i, j)) res_loc = fmax(res_loc, tl_err(fabs(acc[s][r] - R2[i * n + j] * vlam[j])));
      }
    accept = block_max<TL_NT>(res_loc, red) <= TL_RES_MAX * scale;
  }
  if (accept) {
    for (int i = tid; i < n; i += TL_NT) pr.w[i] = vlam[i];
    for (int e = tid; e < n * n; e += TL_NT) pr.V[e] = R2[e];
    return;
  }
  // fallback: Jacobi sweeps from the start (R1 holds A)
  set_identity(R2);
  __syncthreads();
  const bool converged = jacobi_lds_sweeps(R1, R2, vlo, vhi, n, scale, red);
  for (int i = tid; i < n; i += TL_NT) pr.w[i] = R1[i * n + i];
  for (int e = tid; e < n * n; e += TL_NT) pr.V[e] = R2[e];
  if (!converged && tid == 0) atomicOr(status, ST_EIGH);
}

// ---------------------------------------------------------------------------
// complex Hermitian (interleaved re, im), matrix in global memory
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

template <int NT>
__global__ __launch_bounds__(NT) void jacobi_complex(const EighProb* __restrict__ probs, int* status) {
  extern __shared__ double smem[];
  __shared__ double red[NT / 64];
  const EighProb pr = probs[blockIdx.x];
  const int n = pr.n;
  if (n <= 0 || (pr.ok && *pr.ok)) return;
  const int nn = n + (n & 1), half = nn / 2;
  double* pc = smem;                              // [half]
  double2* pz = reinterpret_cast<double2*>(pc + half + (half & 1));  // [half]
  int* pp = reinterpret_cast<int*>(pz + half);    // [half]
  int* pq = pp + half;
  double2* A = reinterpret_cast<double2*>(pr.A);
  double2* V = reinterpret_cast<double2*>(pr.V);
  for (int e = threadIdx.x; e < n * n; e += NT)
    V[e] = make_double2((e / n == e % n) ? 1.0 : 0.0, 0.0);
  double fro = 0.0;
  for (int e = threadIdx.x; e < n * n; e += NT) fro += A[e].x * A[e].x + A[e].y * A[e].y;
  const double scale = sqrt(block_sum<NT>(fro, red));

  const bool finite = isfinite(scale);
  bool converged = !finite || (n == 1) || scale == 0.0;
  for (int sweep = 0; sweep < MAX_SWEEPS && !converged; ++sweep) {
    double maxoff = 0.0;
    for (int r = 0; r < nn - 1; ++r) {
      for (int j = threadIdx.x; j < half; j += NT) {
        int p, q;
        rr_pair(r, j, nn, p, q);
        double c = 1.0;
        double2 z = make_double2(0.0, 0.0);
        if (p < n && q < n) {
          double2 apq = A[(size_t)p * n + q];
          double mag = hypot(apq.x, apq.y);
          maxoff = fmax(maxoff, mag);
          if (mag != 0.0) {
            double s;
            jacobi_cs(A[(size_t)p * n + p].x, A[(size_t)q * n + q].x, mag, c, s);
            z = cscale(s / mag, apq);
          }
        }
        pp[j] = p;
        pq[j] = q;
        pc[j] = c;
        pz[j] = z;
      }
      __syncthreads();
      for (int b = threadIdx.x; b < half * half; b += NT) {
        const int ja = b / half, jb = b - ja * half;
        const int pa = pp[ja], qa = pq[ja], pb = pp[jb], qb = pq[jb];
        const double ca = pc[ja], cb = pc[jb];
        const double2 za = pz[ja], zb = pz[jb];
        const bool va = qa < n, vb = qb < n;
        const double2 zero = make_double2(0.0, 0.0);
        double2 x00 = A[(size_t)pa * n + pb];
        double2 x01 = vb ? A[(size_t)pa * n + qb] : zero;
        double2 x10 = va ? A[(size_t)qa * n + pb] : zero;
        double2 x11 = (va && vb) ? A[(size_t)qa * n + qb] : zero;
        // A_blk J_b, J_b = [[cb, zb], [-conj(zb), cb]]
        double2 y00 = csub(cscale(cb, x00), cmulc(x01, zb));
        double2 y01 = cadd(cmul(x00, zb), cscale(cb, x01));
        double2 y10 = csub(cscale(cb, x10), cmulc(x11, zb));
        double2 y11 = cadd(cmul(x10, zb), cscale(cb, x11));
        // J_a^H (.) with J_a^H = [[ca, -za], [conj(za), ca]]
        double2 z00 = csub(cscale(ca, y00), cmul(za, y10));
        double2 z01 = csub(cscale(ca, y01), cmul(za, y11));
        double2 z10 = cadd(cconjmul(za, y00), cscale(ca, y10));
        double2 z11 = cadd(cconjmul(za, y01), cscale(ca, y11));
        if (ja == jb) {
          z01 = z10 = zero;
          z00.y = 0.0;
          z11.y = 0.0;
        }
        A[(size_t)pa * n + pb] = z00;
        if (vb) A[(size_t)pa * n + qb] = z01;
        if (va) A[(size_t)qa * n + pb] = z10;
        if (va && vb) A[(size_t)qa * n + qb] = z11;
      }
      for (int e = threadIdx.x; e < n * half; e += NT) {
        const int i = e / half, j = e - i * half;
        const int p = pp[j], q = pq[j];
        if (q >= n) continue;
        const double c = pc[j];
        const double2 z = pz[j];
        double2 vp = V[(size_t)i * n + p], vq = V[(size_t)i * n + q];
        V[(size_t)i * n + p] = csub(cscale(c, vp), cmulc(vq, z));
        V[(size_t)i * n + q] = cadd(cmul(vp, z), cscale(c, vq));
      }
      __syncthreads();
    }
    converged = block_max<NT>(maxoff, red) <= CONV_TOL * scale;
  }
  for (int i = threadIdx.x; i < n; i += NT) pr.w[i] = A[(size_t)i * n + i].x;
  if ((!converged || !finite) && threadIdx.x == 0) atomicOr(status, finite ? ST_EIGH : ST_NONFINITE);
}


// ---------------------------------------------------------------------------
// complex Hermitian, n <= HT_MAX, one workgroup of 1024 threads per matrix, the
// matrix in global memory (it stays in the L2 / last-level caches):
//   1. Householder reduction A = Q T Q^H to a REAL symmetric tridiagonal T:
//      the reflector H_k = I - tau v v^H (v_{k+1} = 1, tau complex) satisfies
//      H_k^H [alpha; x] = [beta; 0] with beta real, so every off-diagonal element
//      of T is real (the last step, on a single element, only makes it real) and
//      the diagonal of a Hermitian matrix is real; A <- H^H A H as
//      A - v w^H - w v^H with p = tau A v, w = p - (tau/2)(p^H v) v.  The
//      reflectors are kept: v_k in column k of Y (rows k+1..n-1, zero above), tau_k
//      in Y[k][n-1] (column n-1 holds no reflector);
//   2./3. eigenvalues and eigenvectors Z (real) of T as in the real solver, with
//      the residual max|T z - lambda z| checked per vector (-> *ok).
// Outside this kernel: the orthogonality check of Z and one Newton-Schulz step,
// then V = Q Z with Q applied in blocks of HT_NB reflectors in compact WY form
// (Q_b = I - Y_b T_b Y_b^H; herm_wy_t_kernel forms T_b) on the matrix cores.
// ---------------------------------------------------------------------------
constexpr int HT_NCH = 5;  // row chunks of the matrix-vector product
constexpr int HT_YC = 32;  // rows per LDS chunk of the WY Gram matrix
constexpr int HC_GROUPS = 8;  // workgroups per instance of the orthogonality check

static size_t ht_lds_bytes(int n) {
  return sizeof(double) * (6 * (size_t)n + 4 * (size_t)n + 2 * HT_NCH * (size_t)n + TL_XS) +
         sizeof(int) * (2 * (size_t)n + TL_XS);
}

__global__ __launch_bounds__(TL_NT) void eigh_herm_tridiag(const EighProb* __restrict__ probs, int* status) {
  extern __shared__ double smem[];
  __shared__ double red[TL_NT / 64];
  __shared__ double s_tau[2][2];
  const EighProb pr = probs[blockIdx.x];
  const int n = pr.n;
  if (n <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double2* A = reinterpret_cast<double2*>(pr.A);
  double2* Y = reinterpret_cast<double2*>(pr.ws);  // n x n reflectors
  double* Z = pr.V;                                 // n x n real, in the first half of V
  double* vd = smem;
  double* ve = vd + n;
  double* ve2 = ve + n;
  double* vlo = ve2 + n;
  double* vhi = vlo + n;
  double* vlam = vhi + n;
  double2* vv = reinterpret_cast<double2*>(vlam + n);  // reflector
  double2* vw = vv + n;                                 // w
  double2* Pm = vw + n;                                 // HT_NCH x n partial sums
  double* xs = reinterpret_cast<double*>(Pm + HT_NCH * n);
  int* ib0 = reinterpret_cast<int*>(xs + TL_XS);
  int* ib1 = ib0 + n;
  int* cnt = ib1 + n;

  for (int e = tid; e < n * n; e += TL_NT) Y[e] = make_double2(0.0, 0.0);
  double fro = 0.0;
  for (int e = tid; e < n * n; e += TL_NT) fro += A[e].x * A[e].x + A[e].y * A[e].y;
  const double scale = sqrt(block_sum<TL_NT>(fro, red));
  if (!isfinite(scale) || scale == 0.0 || n == 1) {  // T = diag(A), Q = I (all tau = 0)
    for (int i = tid; i < n; i += TL_NT) pr.w[i] = A[(size_t)i * n + i].x;
    for (int e = tid; e < n * n; e += TL_NT) {
      const int i = e / n;
      Z[e] = e == i * n + i ? 1.0 : 0.0;
    }
    if (tid == 0) {
      *pr.ok = 1;
      if (!isfinite(scale)) atomicOr(status, ST_NONFINITE);
    }
    return;
  }

  for (int k = 0; k < n - 1; ++k) {
    const int L = n - k - 1;
    double* tau2 = s_tau[k & 1];  // two buffers: a step without update has one barrier only
    if (wave == 0) {
      // x_i = A[i][k] = conj(A[k][i]) for i in [k+1, n)
      double ar = 0.0, ai = 0.0, s2 = 0.0;
      for (int i = k + 1 + lane; i < n; i += 64) {
        const double2 a = A[(size_t)k * n + i];
        if (i == k + 1) {
          ar = a.x;
          ai = -a.y;
        } else {
          s2 += a.x * a.x + a.y * a.y;
        }
      }
      s2 = tl_wave_sum(s2);
      ar = tl_readlane(ar, 0);
      ai = tl_readlane(ai, 0);
      double taur = 0.0, taui = 0.0, beta = ar;
      double2 inv = make_double2(0.0, 0.0);
      if (s2 != 0.0 || ai != 0.0) {
        beta = -copysign(sqrt(ar * ar + ai * ai + s2), ar);
        taur = (beta - ar) / beta;
        taui = -ai / beta;
        const double dr = ar - beta, den = dr * dr + ai * ai;
        inv = make_double2(dr / den, -ai / den);  // 1 / (alpha - beta)
      }
      for (int i = k + 1 + lane; i < n; i += 64) {
        const double2 a = A[(size_t)k * n + i];
        const double2 v = i == k + 1 ? make_double2(1.0, 0.0) : cmul(make_double2(a.x, -a.y), inv);
        vv[i] = v;
        Y[(size_t)i * n + k] = v;
      }
      if (lane == 0) {
        tau2[0] = taur;
        tau2[1] = taui;
        Y[(size_t)k * n + (n - 1)] = make_double2(taur, taui);
        ve[k] = beta;
        vd[k] = A[(size_t)k * n + k].x;
      }
    }
    __syncthreads();
    const double2 tau = make_double2(tau2[0], tau2[1]);
    if (tau.x == 0.0 && tau.y == 0.0) continue;
    // p = A_t v as sums over the rows j of A_t of conj(A[j][o]) v_j: lanes over the
    // columns o, wavefronts over segments of 64 columns and row chunks
    const int nseg = (L + 63) >> 6;
    const int nch = max(1, min(HT_NCH, (TL_NT / 64) / nseg));
    if (wave < nseg * nch) {
      const int seg = wave % nseg, ch = wave / nseg;
      const int o = 64 * seg + lane;
      const int jb = ch * L / nch, je = (ch + 1) * L / nch;
      if (o < L) {
        const double2* base = A + (size_t)(k + 1) * n + (k + 1 + o);
        double2 acc0 = make_double2(0.0, 0.0), acc1 = acc0;
        int jj = jb;
        for (; jj + 1 < je; jj += 2) {
          const double2 m0 = base[(size_t)jj * n], m1 = base[(size_t)(jj + 1) * n];
          acc0 = cadd(acc0, cconjmul(m0, vv[k + 1 + jj]));
          acc1 = cadd(acc1, cconjmul(m1, vv[k + 2 + jj]));
        }
        if (jj < je) acc0 = cadd(acc0, cconjmul(base[(size_t)jj * n], vv[k + 1 + jj]));
        Pm[ch * n + o] = cadd(acc0, acc1);
      }
    }
    __syncthreads();
    if (wave == 0) {  // p = tau * sum, K = -(tau/2) p^H v, w = p + K v
      double dr = 0.0, di = 0.0;
      for (int i = lane; i < L; i += 64) {
        double2 p = make_double2(0.0, 0.0);
        for (int ch = 0; ch < nch; ++ch) p = cadd(p, Pm[ch * n + i]);
        p = cmul(tau, p);
        vw[k + 1 + i] = p;
        const double2 t = cconjmul(p, vv[k + 1 + i]);
        dr += t.x;
        di += t.y;
      }
      dr = tl_wave_sum(dr);
      di = tl_wave_sum(di);
      const double2 K = cmul(make_double2(-0.5 * tau.x, -0.5 * tau.y), make_double2(dr, di));
      for (int i = lane; i < L; i += 64) vw[k + 1 + i] = cadd(vw[k + 1 + i], cmul(K, vv[k + 1 + i]));
    }
    __syncthreads();
    // A_t -= v w^H + w v^H (diagonal kept real); one row segment of 64 columns per item
    {
      const int sa = (L + 63) >> 6, na = L * sa;
      for (int t = wave; t < na; t += TL_NT / 64) {
        const int ii = t / sa, sg = t - ii * sa;
        const int i = k + 1 + ii, c = 64 * sg + lane, j = k + 1 + c;
        if (c < L) {
          const double2 vi = vv[i], wi = vw[i], vj = vv[j], wj = vw[j];
          double2 a = A[(size_t)i * n + j];
          a = csub(a, cadd(cmulc(vi, wj), cmulc(wi, vj)));
          if (i == j) a.y = 0.0;
          A[(size_t)i * n + j] = a;
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) vd[n - 1] = A[(size_t)(n - 1) * n + n - 1].x;
  __syncthreads();

  double tn, pivmin;
  tl_eigen_brackets(vd, ve, ve2, vlo, vhi, xs, cnt, ib0, ib1, n, red, tn, pivmin);
  double res = 0.0;
  for (int j = tid; j < n; j += TL_NT) {
    const int b0 = ib0[j], b1 = ib1[j];
    const double lam = tl_vector<0>(vd, ve, ve2, b0, b1, vlo[j], vhi[j], tn, pivmin, Z, n, j, n);
    pr.w[j] = lam;
    for (int i = b0; i < b1; ++i) {
      double t = (vd[i] - lam) * Z[(size_t)i * n + j];
      if (i > b0) t += ve[i - 1] * Z[(size_t)(i - 1) * n + j];
      if (i < b1 - 1) t += ve[i] * Z[(size_t)(i + 1) * n + j];
      res = fmax(res, tl_err(fabs(t)));
    }
  }
  res = block_max<TL_NT>(res, red);
  if (tid == 0) *pr.ok = res <= TL_RES_MAX * scale ? 1 : 0;
}

// T_b of the compact WY form Q_b = H_k0 ... H_(k0+m-1) = I - Y_b T_b Y_b^H (upper
// triangular, columnwise forward recurrence T[:c, c] = T[:c, :c] (-tau_c Y_b^H y_c))
// for block blockIdx.y of instance blockIdx.x; workgroup of 256 threads.
__global__ __launch_bounds__(256) void herm_wy_t_kernel(const HermWY* __restrict__ wy) {
  const HermWY w = wy[blockIdx.x];
  const int n = w.n, k0 = blockIdx.y * HT_NB;
  if (k0 >= n - 1) return;
  const int m = min(HT_NB, n - 1 - k0);
  const double2* Y = reinterpret_cast<const double2*>(w.Y);
  double2* Tb = reinterpret_cast<double2*>(w.T) + (size_t)blockIdx.y * HT_NB * HT_NB;
  __shared__ double2 g[HT_NB][HT_NB + 1];
  __shared__ double2 T[HT_NB][HT_NB + 1];
  __shared__ double2 col[HT_NB];
  __shared__ double2 ys[HT_YC][HT_NB + 1];  // a chunk of rows of the block's columns
  // Gram g = Y_b^H Y_b (strictly upper part): the block's columns are staged through LDS
  // HT_YC rows at a time (coalesced loads, all in flight), each thread summing its
  // (HT_NB x HT_NB) / 256 entries; rows above k0 + r + 1 of column k0 + r are zero
  constexpr int PER = HT_NB * HT_NB / 256;
  static_assert(HT_NB * HT_NB % 256 == 0, "whole entries per thread");
  double2 acc[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) acc[u] = make_double2(0.0, 0.0);
  for (int i0 = k0 + 1; i0 < n; i0 += HT_YC) {
    for (int q = threadIdx.x; q < HT_YC * HT_NB; q += 256) {
      const int rr = q / HT_NB, cc = q - rr * HT_NB, i = i0 + rr;
      ys[rr][cc] = i < n && cc < m ? Y[(size_t)i * n + k0 + cc] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = threadIdx.x + 256 * u, r = q / HT_NB, c = q - r * HT_NB;
      if (r < c && c < m)
        for (int rr = 0; rr < HT_YC; ++rr)
          if (i0 + rr >= k0 + 1 + r) acc[u] = cadd(acc[u], cconjmul(ys[rr][r], ys[rr][c]));
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = threadIdx.x + 256 * u, r = q / HT_NB, c = q - r * HT_NB;
    g[r][c] = acc[u];
    T[r][c] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int c = 0; c < m; ++c) {
    const double2 tau = Y[(size_t)(k0 + c) * n + (n - 1)];
    const int r = threadIdx.x;
    if (r < c) col[r] = cmul(make_double2(-tau.x, -tau.y), g[r][c]);
    __syncthreads();
    if (r < c) {
      double2 acc = make_double2(0.0, 0.0);
      for (int q = r; q < c; ++q) acc = cadd(acc, cmul(T[r][q], col[q]));
      T[r][c] = acc;
    }
    if (r == c) T[c][c] = tau;
    __syncthreads();
  }
  for (int q = threadIdx.x; q < HT_NB * HT_NB; q += 256) Tb[q] = T[q / HT_NB][q % HT_NB];
}

// HC_GROUPS workgroups per instance, each over one slice of G; a slice that fails
// clears the flag (every writer writes 0)
__global__ __launch_bounds__(256) void herm_check_kernel(const HermCheck* __restrict__ chk) {
  const HermCheck c = chk[blockIdx.x / HC_GROUPS];
  const int n = c.n, grp = blockIdx.x % HC_GROUPS;
  const int chunk = (n * n + HC_GROUPS - 1) / HC_GROUPS, e0 = grp * chunk, e1 = min(n * n, e0 + chunk);
  double m = 0.0;
  for (int e = e0 + threadIdx.x; e < e1; e += 256) {
    const int i = e / n;
    const double g = c.G[e], dlt = (e == i * n + i) ? 1.0 : 0.0;
    m = fmax(m, tl_err(fabs(g - dlt)));
    c.G[e] = 1.5 * dlt - 0.5 * g;
  }
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (!(t <= TL_ORTH_MAX)) *c.ok = 0;
  }
}

__global__ void real_to_complex_kernel(const RealToComplex* __restrict__ rc) {
  const RealToComplex r = rc[blockIdx.y];
  double2* dst = reinterpret_cast<double2*>(r.dst);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)r.n * r.n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = make_double2(r.src[e], 0.0);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t eigh_lds_bytes(int n) { return tl_lds_bytes(n); }

void launch_eigh_real_lds(const EighProb* d_probs, int nprob, int* d_status, hipStream_t s) {
  if (nprob <= 0) return;
  const size_t bytes = tl_lds_bytes(EIGH_LDS_MAX);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&eigh_tridiag_lds), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)bytes);
    attr = true;
  }
  eigh_tridiag_lds<<<nprob, TL_NT, bytes, s>>>(d_probs, d_status);
}

void launch_eigh_complex(const EighProb* d_probs, int nprob, int nmax, int* d_status, hipStream_t s) {
  if (nprob <= 0) return;
  const int half = (nmax + 1) / 2;  // n <= 4000 keeps this below 64 KB
  size_t bytes = (size_t)(half + 1) * sizeof(double) + (size_t)half * sizeof(double2) +
                 (size_t)half * 2 * sizeof(int);
  jacobi_complex<1024><<<nprob, 1024, bytes, s>>>(d_probs, d_status);
}

void launch_eigh_herm_tridiag(const EighProb* d_probs, int nprob, int nmax, int* d_status, hipStream_t s) {
  if (nprob <= 0) return;
  const size_t bytes = ht_lds_bytes(nmax);
  static size_t attr = 0;
  if (bytes > attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&eigh_herm_tridiag), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)bytes);
    attr = bytes;
  }
  eigh_herm_tridiag<<<nprob, TL_NT, bytes, s>>>(d_probs, d_status);
}

void launch_herm_check(const HermCheck* d, int nprob, hipStream_t s) {
  if (nprob > 0) herm_check_kernel<<<nprob * HC_GROUPS, 256, 0, s>>>(d);
}

void launch_herm_wy_t(const HermWY* d, int nprob, int nblk, hipStream_t s) {
  if (nprob > 0 && nblk > 0) herm_wy_t_kernel<<<dim3(nprob, nblk), 256, 0, s>>>(d);
}

void launch_real_to_complex(const RealToComplex* d, int nprob, hipStream_t s) {
  if (nprob > 0) real_to_complex_kernel<<<dim3(64, nprob), 256, 0, s>>>(d);
}

}  // namespace etdm
