// Device helpers of the FP64 eigensolvers: workgroup reductions, DPP wave sums,
// the symmetric-tridiagonal pivot recurrences (Sturm counts, twisted
// factorizations) and the per-eigenvalue vector refinement.
#pragma once

#include <cfloat>

#include "common.h"

namespace etdm {

constexpr int TL_MAXIT = 64;  // multisection rounds (a few tens are ever needed)

template <int NT>
__device__ inline double block_sum(double v, double* red) {
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
__device__ inline double block_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = red[0];  // any sign
  for (int w = 1; w < NT / 64; ++w) s = fmax(s, red[w]);
  return s;
}

// NaN and overflow map to +inf so that a max-reduction cannot hide them
__device__ __forceinline__ double tl_err(double x) { return (x <= 1e300) ? x : INFINITY; }

// Cross-lane sums through DPP (no LDS round trip).  Every lane of a quad (and
// of the wavefront, for tl_wave_sum) ends with bit-identical results.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double tl_dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double tl_quad_sum(double v) {
  v += tl_dpp<0xB1>(v);  // quad_perm [1,0,3,2]
  v += tl_dpp<0x4E>(v);  // quad_perm [2,3,0,1]
  return v;
}
// N independent wavefront sums, each DPP stage applied to all N values before the
// next (so that their latencies overlap); same lane order as tl_wave_sum
template <int N>
__device__ __forceinline__ void tl_wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] += tl_dpp<0xB1>(v[r]);
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] += tl_dpp<0x4E>(v[r]);
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] += tl_dpp<0x141>(v[r]);
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] += tl_dpp<0x140>(v[r]);
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] += tl_dpp<0x142, 0xa>(v[r]);
#pragma unroll
  for (int r = 0; r < N; ++r) v[r] += tl_dpp<0x143, 0xc>(v[r]);
#pragma unroll
  for (int r = 0; r < N; ++r) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v[r]), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v[r]), 63);
    v[r] = __hiloint2double(hi, lo);
  }
}
__device__ __forceinline__ double tl_wave_sum(double v) {
  v = tl_quad_sum(v);
  v += tl_dpp<0x141>(v);       // row_half_mirror: sums of 8 lanes
  v += tl_dpp<0x140>(v);       // row_mirror: sums of 16 lanes
  v += tl_dpp<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += tl_dpp<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3: lane 63 holds the total
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double tl_wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// 1 / q from the hardware reciprocal (about 28 correct bits) refined by one
// Newton step (about 10 ulp): the pivot recurrences below are backward stable
// with any relative error of a few ulps per operation.
__device__ __forceinline__ double tl_rcp(double q) {
  const double r = __builtin_amdgcn_rcp(q);
  return fma(r, fma(-q, r, 1.0), r);
}

__device__ __forceinline__ double tl_readlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// numbers of eigenvalues below x0 and below x1 of the unreduced block [b0, b1)
// of T (two independent pivot chains; d and e^2 are read from LDS eight rows at
// a time so that the loads overlap)
__device__ inline void tl_sturm2(const double* d, const double* e2, int b0, int b1, double x0, double x1,
                          double pivmin, int& c0, int& c1) {
  double q0 = d[b0] - x0, q1 = d[b0] - x1;
  if (fabs(q0) < pivmin) q0 = -pivmin;
  if (fabs(q1) < pivmin) q1 = -pivmin;
  c0 = q0 < 0.0;
  c1 = q1 < 0.0;
  int i = b0 + 1;
  for (; i + 8 <= b1; i += 8) {
    double dd[8], ee[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      dd[u] = d[i + u];
      ee[u] = e2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      q0 = (dd[u] - x0) - ee[u] * tl_rcp(q0);
      q1 = (dd[u] - x1) - ee[u] * tl_rcp(q1);
      if (fabs(q0) < pivmin) q0 = -pivmin;
      if (fabs(q1) < pivmin) q1 = -pivmin;
      c0 += q0 < 0.0;
      c1 += q1 < 0.0;
    }
  }
  for (; i < b1; ++i) {
    const double dd = d[i], ee = e2[i - 1];
    q0 = (dd - x0) - ee * tl_rcp(q0);
    q1 = (dd - x1) - ee * tl_rcp(q1);
    if (fabs(q0) < pivmin) q0 = -pivmin;
    if (fabs(q1) < pivmin) q1 = -pivmin;
    c0 += q0 < 0.0;
    c1 += q1 < 0.0;
  }
}

// numbers of eigenvalues below x[c] (c < C) of the unreduced block [b0, b1): C
// independent pivot chains in lockstep, so that their latencies overlap
template <int C>
__device__ inline void tl_sturm_n(const double* d, const double* e2, int b0, int b1, const double (&x)[C],
                                  double pivmin, int (&cnt)[C]) {
  double q[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    q[c] = d[b0] - x[c];
    if (fabs(q[c]) < pivmin) q[c] = -pivmin;
    cnt[c] = q[c] < 0.0;
  }
  int i = b0 + 1;
  for (; i + 8 <= b1; i += 8) {
    double dd[8], ee[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      dd[u] = d[i + u];
      ee[u] = e2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        q[c] = (dd[u] - x[c]) - ee[u] * tl_rcp(q[c]);
        if (fabs(q[c]) < pivmin) q[c] = -pivmin;
        cnt[c] += q[c] < 0.0;
      }
  }
  for (; i < b1; ++i) {
    const double dd = d[i], ee = e2[i - 1];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      q[c] = (dd - x[c]) - ee * tl_rcp(q[c]);
      if (fabs(q[c]) < pivmin) q[c] = -pivmin;
      cnt[c] += q[c] < 0.0;
    }
  }
}

__device__ __forceinline__ double tl_piv(double x, double pivmin) { return fabs(x) < pivmin ? -pivmin : x; }

constexpr int TL_XS = 1024;                   // multisection points per round
constexpr double TL_BISECT_TOL = 1e-8;        // bracket width / ||T|| handed to the RQI
constexpr int TL_RQI_MAX = 4;                 // Rayleigh-quotient corrections per eigenvalue

// Twisted factorization of T - lam I on the unreduced block [b0, b1) (size >= 2):
// forward pivots D+, backward pivots D-, twist r minimising
// |gamma_i| = |D+_i + D-_i - (d_i - lam)|, then z_r = 1 and
// z_i = -(e_i / D+_i) z_{i+1} (i < r), z_i = -(e_{i-1} / D-_i) z_{i-1} (i > r).
// Writes z / ||z|| into column j of Z (ld n; D+ and D- are kept there meanwhile)
// and returns the Rayleigh-quotient correction gamma_r / ||z||^2.
// Twisted factorization at lam (pivots in Z), the twist index r minimising
// |gamma_r|, the vector z (z_r = 1) normalized into column j of Z; returns the
// Rayleigh-quotient correction gamma_r / ||z||^2.  Plain loops, for Z in LDS.
__device__ inline double tl_twisted(const double* d, const double* e, const double* e2, int b0, int b1, double lam,
                             double pivmin, double* Z, int ld, int j) {
  double D = tl_piv(d[b0] - lam, pivmin);
  Z[b0 * ld + j] = D;
  for (int i = b0 + 1; i < b1; ++i) {
    D = tl_piv((d[i] - lam) - e2[i - 1] * tl_rcp(D), pivmin);
    Z[i * ld + j] = D;
  }
  D = tl_piv(d[b1 - 1] - lam, pivmin);
  int r = b1 - 1;
  double gr = Z[(b1 - 1) * ld + j] + D - (d[b1 - 1] - lam);
  double best = fabs(gr);
  for (int i = b1 - 2; i >= b0; --i) {
    D = tl_piv((d[i] - lam) - e2[i] * tl_rcp(D), pivmin);
    const double g = Z[i * ld + j] + D - (d[i] - lam);
    if (fabs(g) < best) {
      best = fabs(g);
      gr = g;
      r = i;
    }
  }
  if (r < b1 - 1) {  // backward pivots below the twist
    D = tl_piv(d[b1 - 1] - lam, pivmin);
    Z[(b1 - 1) * ld + j] = D;
    for (int i = b1 - 2; i > r; --i) {
      D = tl_piv((d[i] - lam) - e2[i] * tl_rcp(D), pivmin);
      Z[i * ld + j] = D;
    }
  }
  double nrm = 1.0, z = 1.0;
  Z[r * ld + j] = 1.0;
  for (int i = r - 1; i >= b0; --i) {
    z = -(e[i] * tl_rcp(Z[i * ld + j])) * z;
    Z[i * ld + j] = z;
    nrm += z * z;
  }
  z = 1.0;
  for (int i = r + 1; i < b1; ++i) {
    z = -(e[i - 1] * tl_rcp(Z[i * ld + j])) * z;
    Z[i * ld + j] = z;
    nrm += z * z;
  }
  const double sc = 1.0 / sqrt(nrm);
  for (int i = b0; i < b1; ++i) Z[i * ld + j] *= sc;
  return gr / nrm;
}

// The same with the loads issued TL_PF indices ahead (the next chunk while the
// current one is used), for Z in global memory: their addresses do not depend on
// the recurrences, but without this each step would wait for its own load, since
// the compiler keeps the loads behind the stores to the same array.
template <int TL_PF>
__device__ inline double tl_twisted_pf(const double* d, const double* e, const double* e2, int b0, int b1, double lam,
                             double pivmin, double* Z, int ld, int j) {
  // forward pivots D+ (stored in Z)
  double D = tl_piv(d[b0] - lam, pivmin);
  Z[b0 * ld + j] = D;
  for (int i = b0 + 1; i < b1; ++i) {
    D = tl_piv((d[i] - lam) - e2[i - 1] * tl_rcp(D), pivmin);
    Z[i * ld + j] = D;
  }
  // backward pivots D- and the twist index r minimising |gamma_r| = |D+_r + D-_r - (d_r - lam)|
  D = tl_piv(d[b1 - 1] - lam, pivmin);
  int r = b1 - 1;
  double gr = Z[(b1 - 1) * ld + j] + D - (d[b1 - 1] - lam);
  double best = fabs(gr);
  {
    double cur[TL_PF];
#pragma unroll
    for (int u = 0; u < TL_PF; ++u) {
      const int i = b1 - 2 - u;
      cur[u] = i >= b0 ? Z[i * ld + j] : 0.0;
    }
    for (int i0 = b1 - 2; i0 >= b0; i0 -= TL_PF) {
      double nxt[TL_PF];
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) {
        const int i = i0 - TL_PF - u;
        nxt[u] = i >= b0 ? Z[i * ld + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) {
        const int i = i0 - u;
        if (i >= b0) {
          D = tl_piv((d[i] - lam) - e2[i] * tl_rcp(D), pivmin);
          const double g = cur[u] + D - (d[i] - lam);
          if (fabs(g) < best) {
            best = fabs(g);
            gr = g;
            r = i;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) cur[u] = nxt[u];
    }
  }
  if (r < b1 - 1) {  // backward pivots below the twist
    D = tl_piv(d[b1 - 1] - lam, pivmin);
    Z[(b1 - 1) * ld + j] = D;
    for (int i = b1 - 2; i > r; --i) {
      D = tl_piv((d[i] - lam) - e2[i] * tl_rcp(D), pivmin);
      Z[i * ld + j] = D;
    }
  }
  // z_r = 1 and the two one-sided recurrences: z_i = -(e_i / D+_i) z_{i+1} above the
  // twist, z_i = -(e_{i-1} / D-_i) z_{i-1} below it
  double nrm = 1.0, z = 1.0;
  Z[r * ld + j] = 1.0;
  {
    double cur[TL_PF];
#pragma unroll
    for (int u = 0; u < TL_PF; ++u) {
      const int i = r - 1 - u;
      cur[u] = i >= b0 ? Z[i * ld + j] : 1.0;
    }
    for (int i0 = r - 1; i0 >= b0; i0 -= TL_PF) {
      double nxt[TL_PF];
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) {
        const int i = i0 - TL_PF - u;
        nxt[u] = i >= b0 ? Z[i * ld + j] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) {
        const int i = i0 - u;
        if (i >= b0) {
          z = -(e[i] * tl_rcp(cur[u])) * z;
          Z[i * ld + j] = z;
          nrm += z * z;
        }
      }
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) cur[u] = nxt[u];
    }
  }
  z = 1.0;
  {
    double cur[TL_PF];
#pragma unroll
    for (int u = 0; u < TL_PF; ++u) {
      const int i = r + 1 + u;
      cur[u] = i < b1 ? Z[i * ld + j] : 1.0;
    }
    for (int i0 = r + 1; i0 < b1; i0 += TL_PF) {
      double nxt[TL_PF];
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) {
        const int i = i0 + TL_PF + u;
        nxt[u] = i < b1 ? Z[i * ld + j] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) {
        const int i = i0 + u;
        if (i < b1) {
          z = -(e[i - 1] * tl_rcp(cur[u])) * z;
          Z[i * ld + j] = z;
          nrm += z * z;
        }
      }
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) cur[u] = nxt[u];
    }
  }
  // normalization
  const double sc = 1.0 / sqrt(nrm);
  {
    double cur[TL_PF];
#pragma unroll
    for (int u = 0; u < TL_PF; ++u) {
      const int i = b0 + u;
      cur[u] = i < b1 ? Z[i * ld + j] : 0.0;
    }
    for (int i0 = b0; i0 < b1; i0 += TL_PF) {
      double nxt[TL_PF];
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) {
        const int i = i0 + TL_PF + u;
        nxt[u] = i < b1 ? Z[i * ld + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) {
        const int i = i0 + u;
        if (i < b1) Z[i * ld + j] = cur[u] * sc;
      }
#pragma unroll
      for (int u = 0; u < TL_PF; ++u) cur[u] = nxt[u];
    }
  }
  return gr / nrm;
}

// Eigenvector of T (size n) for eigenvalue j (bracket lo..hi) into column j of Z
// (leading dimension ld), with Rayleigh-quotient corrections while the correction
// exceeds rqi_tol eps ||T||; returns the eigenvalue (the last correction applied).
// PF = 0: plain loops (Z in LDS), else loads PF indices ahead (Z in global memory).
template <int PF>
__device__ inline double tl_vector(const double* vd, const double* ve, const double* ve2, int b0, int b1, double lo,
                            double hi, double tn, double pivmin, double* Z, int n, int j, int ld,
                            double rqi_tol = 2.0) {
  const double eps = DBL_EPSILON;
  for (int i = 0; i < b0; ++i) Z[i * ld + j] = 0.0;
  for (int i = b1; i < n; ++i) Z[i * ld + j] = 0.0;
  double lam = 0.5 * (lo + hi);
  if (b1 - b0 == 1) {
    Z[b0 * ld + j] = 1.0;
    return vd[b0];
  }
  auto twisted = [&](double at) {
    if constexpr (PF > 0) return tl_twisted_pf<PF>(vd, ve, ve2, b0, b1, at, pivmin, Z, ld, j);
    else return tl_twisted(vd, ve, ve2, b0, b1, at, pivmin, Z, ld, j);
  };
  double dl = twisted(lam);
  for (int it = 0; it < TL_RQI_MAX && fabs(dl) > rqi_tol * eps * tn; ++it) {
    const double nl = lam + dl;
    if (!(nl >= lo && nl <= hi)) break;
    lam = nl;
    dl = twisted(lam);
  }
  const double nl = lam + dl;
  return (nl >= lo && nl <= hi) ? nl : lam;
}


}  // namespace etdm
