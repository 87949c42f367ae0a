// FP64 Hermitian eigensolver: parallel cyclic Jacobi, one workgroup per matrix.
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
#include "common.h"

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

template <int NT>
__device__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

template <int NT>
__device__ double block_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / 64; ++w) s = fmax(s, red[w]);
  return s;
}

// ---------------------------------------------------------------------------
// real symmetric, matrix and vectors in LDS (n <= EIGH_LDS_MAX), 1024 threads.
// Same rounds as jacobi_real; the per-round index maps are advanced
// incrementally (no integer division) and the pairing wraps without modulo.
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

__global__ __launch_bounds__(JL_NT) void jacobi_real_lds(const EighProb* __restrict__ probs, int* status) {
  extern __shared__ double smem[];
  __shared__ double red[JL_NT / 64];
  const EighProb pr = probs[blockIdx.x];
  const int n = pr.n;
  if (n <= 0) return;
  const int nn = n + (n & 1), half = nn / 2, m = nn - 1;
  double* pc = smem;
  double* ps = pc + half;
  int* pp = reinterpret_cast<int*>(ps + half);
  int* pq = pp + half;
  double* A = reinterpret_cast<double*>(pq + half);
  double* V = A + n * n;
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += JL_NT) {
    const int i = e / n, k = e - i * n;
    // symmetric part: products formed in reduced precision need not be exactly symmetric
    A[e] = 0.5 * (pr.A[e] + pr.A[k * n + i]);
    V[e] = (i == k) ? 1.0 : 0.0;
  }
  __syncthreads();
  double fro = 0.0;
  for (int e = tid; e < n * n; e += JL_NT) fro += A[e] * A[e];
  const double scale = sqrt(block_sum<JL_NT>(fro, red));
  const bool finite = isfinite(scale);
  bool converged = !finite || n == 1 || scale == 0.0;
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
  for (int i = tid; i < n; i += JL_NT) pr.w[i] = A[i * n + i];
  for (int e = tid; e < n * n; e += JL_NT) pr.V[e] = V[e];
  if ((!converged || !finite) && tid == 0) atomicOr(status, finite ? ST_EIGH : ST_NONFINITE);
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
  if (n <= 0) return;
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
// launchers
// ---------------------------------------------------------------------------
static size_t real_params_bytes(int n) {
  int half = (n + (n & 1)) / 2;
  return (size_t)half * 2 * sizeof(double) + (size_t)half * 2 * sizeof(int);
}

size_t eigh_lds_bytes(int n) { return real_params_bytes(n) + 2 * (size_t)n * n * sizeof(double); }

void launch_eigh_real_lds(const EighProb* d_probs, int nprob, int* d_status, hipStream_t s) {
  if (nprob <= 0) return;
  size_t bytes = eigh_lds_bytes(EIGH_LDS_MAX);
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_real_lds), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)bytes);
    attr = true;
  }
  jacobi_real_lds<<<nprob, JL_NT, bytes, s>>>(d_probs, d_status);
}

void launch_eigh_complex(const EighProb* d_probs, int nprob, int nmax, int* d_status, hipStream_t s) {
  if (nprob <= 0) return;
  const int half = (nmax + 1) / 2;  // n <= 4000 keeps this below 64 KB
  size_t bytes = (size_t)(half + 1) * sizeof(double) + (size_t)half * sizeof(double2) +
                 (size_t)half * 2 * sizeof(int);
  jacobi_complex<1024><<<nprob, 1024, bytes, s>>>(d_probs, d_status);
}

}  // namespace etdm
