// Device-resident L-BFGS iteration (Sec. 3.1-3.3).
//
//   direction  p = -H g, two-loop recursion over the stored pairs (s_i, y_i) with
//              the diagonal preconditioner of Eq. prec_3 as the initial inverse
//              Hessian; preconditioned steepest descent when p.g >= 0
//   step       trial a = 1; strong Wolfe (Eq. strw1, strw2) accepts it at once;
//              otherwise expand while the energy decreases and the slope stays
//              negative, then zoom, with safeguarded cubic steps; a probe passing
//              strong Wolfe or approximate Wolfe with the energy condition
//              (Eq. aprw, aprw2) is accepted; after max_ls probes the lowest
//              energy seen is taken
//   update     s = a p, y = g(a) - g stored when s.y > 0, beta = y.y / s.y
//
// Scalars never leave the device: every decision is taken by a one-workgroup
// kernel that reads the reduction partials and the state, so the launch
// sequences are fixed and can be captured in HIP graphs.
#include <algorithm>

#include "lbfgs.h"
#include "reduce.h"

namespace etdm {
namespace {

constexpr int TPB = 256;

inline int vgrid(int64_t n) { return (int)std::min<int64_t>(2048, std::max<int64_t>(1, (n + TPB - 1) / TPB)); }

// Reduction over the LB_DOT_BLOCKS partials by one workgroup of TPB threads.
__device__ double sum_partials(const double* partial) {
  __shared__ double red[16];
  double s = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < LB_DOT_BLOCKS; i += blockDim.x) neumaier_add(s, c, partial[i]);
  return block_sum_neumaier(s, c, red);
}

// Slot of the k-th step of a two-loop pass: pass 0 runs newest to oldest, pass 1
// oldest to newest; steps beyond the stored count are inactive.
__device__ __forceinline__ int two_loop_slot(const LbState& st, int k, int pass) {
  if (k >= st.count) return -1;
  const int m = st.m;
  return pass == 0 ? (st.head - 1 - k + m) % m : (st.head - st.count + k + m) % m;
}

// partial sums of x.y; skipped when `only_if` points at a zero flag
__global__ __launch_bounds__(TPB) void dot_partial(const double* __restrict__ x, const double* __restrict__ y,
                                                   int64_t n, const int32_t* only_if, double* partial) {
  if (only_if && *only_if == 0) return;
  __shared__ double red[16];
  double s = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    neumaier_add(s, c, x[i] * y[i]);
  const double t = block_sum_neumaier(s, c, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Stage t of the two-loop recursion with c = st.count stored pairs, each step's
// update fused with the next step's dot product (one pass over the vectors each):
//   t < c         first loop, step t (newest to oldest): v = g at t = 0, else
//                 v = q + coef y (q = g at t = 1) of step t - 1, kept in q; partials
//                 of s.v for step t
//   t == c        end of the first loop: v as above, r = H0 v with the diagonal
//                 preconditioner of Eq. prec_3; partials of y.r for the first step of
//                 the second loop (or, with c = 0, r is the direction)
//   c < t <= 2c   second loop, step t - c - 1 (oldest to newest): p += coef s; partials
//                 of y.p for the next step, or after the last step the direction
// The direction is written as p = -H g with the partials of g.p (its slope) and the
// unit-step trial point xt = x + p.  Stages beyond 2c return at once.
__global__ __launch_bounds__(TPB) void two_loop_stage(const LbState* __restrict__ st, int t,
                                                      const double* __restrict__ g, double* __restrict__ q,
                                                      double* __restrict__ p, const double* __restrict__ S,
                                                      const double* __restrict__ Y, const double* __restrict__ h,
                                                      const double* __restrict__ w, double gamma,
                                                      const double* __restrict__ x, double* __restrict__ xt,
                                                      int64_t n, double* partial) {
  const int c = st->count;
  if (t > 2 * c) return;
  __shared__ double red[16];
  double s = 0.0, e = 0.0;
  const int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, dj = (int64_t)gridDim.x * blockDim.x;
  if (t <= c) {
    // v of the first loop: g, or the previous step's update
    const double* __restrict__ src = t <= 1 ? g : q;
    const double* __restrict__ yv = t >= 1 ? Y + (int64_t)two_loop_slot(*st, t - 1, 0) * n : nullptr;
    const double cf = st->coef;
    if (t < c) {
      const double* __restrict__ sv = S + (int64_t)two_loop_slot(*st, t, 0) * n;
      for (int64_t j = j0; j < n; j += dj) {
        double v = src[j];
        if (yv) {
          v = v + cf * yv[j];
          q[j] = v;
        }
        neumaier_add(s, e, sv[j] * v);
      }
    } else {
      const double beta = st->beta;
      const double* __restrict__ y1 = c > 0 ? Y + (int64_t)two_loop_slot(*st, 0, 1) * n : nullptr;
      for (int64_t j = j0; j < n; j += dj) {
        double v = src[j];
        if (yv) v = v + cf * yv[j];
        const double r = v / ((1.0 - gamma) * h[j] + gamma * beta * w[j]);
        if (y1) {
          p[j] = r;
          neumaier_add(s, e, y1[j] * r);
        } else {
          p[j] = -r;
          neumaier_add(s, e, g[j] * -r);
          xt[j] = x[j] - r;
        }
      }
    }
  } else {
    const int k = t - c - 1;
    const double cf = st->coef;
    const double* __restrict__ sv = S + (int64_t)two_loop_slot(*st, k, 1) * n;
    if (k < c - 1) {
      const double* __restrict__ yn = Y + (int64_t)two_loop_slot(*st, k + 1, 1) * n;
      for (int64_t j = j0; j < n; j += dj) {
        const double v = p[j] + cf * sv[j];
        p[j] = v;
        neumaier_add(s, e, yn[j] * v);
      }
    } else {
      for (int64_t j = j0; j < n; j += dj) {
        const double v = -(p[j] + cf * sv[j]);
        p[j] = v;
        neumaier_add(s, e, g[j] * v);
        xt[j] = x[j] + v;
      }
    }
  }
  const double tot = block_sum_neumaier(s, e, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// The scalar after stage t: first loop alpha_i = s_i.q / s_i.y_i and coef = -alpha_i;
// second loop coef = alpha_i - y_i.r / s_i.y_i for the next step; after the last stage
// the slope of the direction, which is replaced by preconditioned steepest descent
// (and the memory erased) when it does not descend.
__global__ __launch_bounds__(TPB) void two_loop_scalar(LbState* st, int t, const double* partial) {
  const int c = st->count;
  if (t > 2 * c) return;
  const double d = sum_partials(partial);
  if (threadIdx.x != 0) return;
  int i = -1;  // slot whose scalar follows, or -1 after the last stage
  if (t < c) {
    i = two_loop_slot(*st, t, 0);
    st->al[i] = d / st->ys[i];
    st->coef = -st->al[i];
    return;
  }
  if (t < 2 * c) i = two_loop_slot(*st, t - c, 1);
  if (i >= 0) {
    st->coef = st->al[i] - d / st->ys[i];
    return;
  }
  st->dphi0 = d;
  st->steepest = (d < 0.0) ? 0 : 1;
  if (st->steepest) st->count = 0;
}

// r = sign * q / ((1 - gamma) h + gamma beta w); skipped when `only_if` points at a zero flag
__global__ void precond(double* __restrict__ r, const double* __restrict__ q, const double* __restrict__ h,
                        const double* __restrict__ w, int64_t n, double gamma, double sign, const LbState* st,
                        const int32_t* only_if) {
  if (only_if && *only_if == 0) return;
  const double beta = st->beta;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    r[j] = sign * (q[j] / ((1.0 - gamma) * h[j] + gamma * beta * w[j]));
}

__global__ __launch_bounds__(TPB) void start_state(LbState* st, const double* E_total, double beta0, int set_beta,
                                                   int m, const double* partial) {
  const double gg = sum_partials(partial);
  if (threadIdx.x != 0) return;
  st->E = *E_total;
  st->gg = gg;
  st->count = 0;
  st->head = 0;
  st->m = m;
  if (set_beta) st->beta = beta0;
  for (int i = 0; i < LB_MMAX; ++i) st->ys[i] = st->al[i] = 0.0;
  st->result = LR_ACCEPT;
  st->status = 0;
  st->steepest = 0;
  st->evals = 0;
  st->xmax2 = 0.0;
}

__global__ void force_steepest(LbState* st) {
  st->steepest = 1;
  st->count = 0;
}

// start of the line search at a = 0; the slope is recomputed after a switch to steepest descent
__global__ __launch_bounds__(TPB) void search_begin(LbState* st, const double* partial) {
  const bool fresh = st->steepest != 0;
  const double d = fresh ? sum_partials(partial) : 0.0;
  if (threadIdx.x != 0) return;
  if (fresh) st->dphi0 = d;
  st->f0 = st->E;
  st->alpha = 1.0;
  st->phase = LS_TRIAL;
  st->first = 1;
  st->evals = 0;
  st->result = LR_CONT;
  st->prev_a = 0.0;
  st->prev_f = st->f0;
  st->prev_d = st->dphi0;
  st->best_a = 0.0;
  st->best_f = st->f0;
  st->last_a = -1.0;
  st->status = 0;
}

// xtrial = x + alpha p while the search continues; skipped when `only_if` points at
// a zero flag
__global__ void trial_point(double* __restrict__ xt, const double* __restrict__ x, const double* __restrict__ p,
                            int64_t n, const LbState* st, const int32_t* only_if) {
  if (st->result != LR_CONT || (only_if && *only_if == 0)) return;
  const double a = st->alpha;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    xt[j] = x[j] + a * p[j];
}

// ---- line-search decisions (one thread) ----

// Minimizer of the cubic through (a, fa, ga) and (b, fb, gb); ok = false when it
// has none (Sec. 3.2, cubic interpolation).
__device__ double cubic_step(double a, double fa, double ga, double b, double fb, double gb, bool& ok) {
  ok = false;
  if (a == b) return 0.0;
  const double d1 = ga + gb - 3.0 * (fa - fb) / (a - b);
  const double disc = d1 * d1 - ga * gb;
  if (disc < 0.0) return 0.0;
  const double d2 = copysign(sqrt(disc), b - a);
  const double den = gb - ga + 2.0 * d2;
  if (den == 0.0) return 0.0;
  ok = true;
  return b - (b - a) * (gb + d2 - d1) / den;
}

__device__ bool strong_wolfe(const LbState& s, const LbParams& P, double a, double f, double d) {
  return f <= s.f0 + P.c1 * a * s.dphi0 && fabs(d) <= P.c2 * fabs(s.dphi0);
}

__device__ bool approx_wolfe(const LbState& s, const LbParams& P, double f, double d) {
  return (2.0 * P.delta - 1.0) * s.dphi0 >= d && d >= P.sigma * s.dphi0 && f <= s.f0 + P.eps * fabs(s.f0);
}

__device__ void accept(LbState& s, double a, double f) {
  s.acc_a = a;
  s.acc_f = f;
  s.result = LR_ACCEPT;
}

// out of probes: the lowest energy seen, evaluated once more unless it was the last probe
__device__ void finish(LbState& s) {
  if (s.best_a > 0.0) {
    if (s.best_a != s.last_a) {
      s.alpha = s.best_a;
      s.phase = LS_BEST;
      s.result = LR_CONT;
    } else {
      accept(s, s.best_a, s.best_f);
    }
  } else {
    s.result = LR_FAIL;
  }
}

// next zoom probe inside [lo, hi]: the cubic step kept 10% away from both ends, else bisection
__device__ void zoom_next(LbState& s, const LbParams& P) {
  if (s.evals >= P.max_ls) {
    finish(s);
    return;
  }
  bool ok;
  double a = cubic_step(s.lo_a, s.lo_f, s.lo_d, s.hi_a, s.hi_f, s.hi_d, ok);
  const double width = s.hi_a - s.lo_a;
  const double left = fmin(s.lo_a, s.hi_a) + 0.1 * fabs(width);
  const double right = fmax(s.lo_a, s.hi_a) - 0.1 * fabs(width);
  if (!ok || !isfinite(a) || a < left || a > right) a = 0.5 * (s.lo_a + s.hi_a);
  s.alpha = a;
  s.phase = LS_ZOOM;
  s.result = LR_CONT;
}

// after a bracketing probe that was not accepted: zoom on a bracket, or expand
__device__ void bracket_next(LbState& s, const LbParams& P) {
  if (s.cur_f > s.f0 + P.c1 * s.cur_a * s.dphi0 || (!s.first && s.cur_f >= s.prev_f)) {
    s.lo_a = s.prev_a, s.lo_f = s.prev_f, s.lo_d = s.prev_d;
    s.hi_a = s.cur_a, s.hi_f = s.cur_f, s.hi_d = s.cur_d;
    zoom_next(s, P);
    return;
  }
  if (s.cur_d >= 0.0) {
    s.lo_a = s.cur_a, s.lo_f = s.cur_f, s.lo_d = s.cur_d;
    s.hi_a = s.prev_a, s.hi_f = s.prev_f, s.hi_d = s.prev_d;
    zoom_next(s, P);
    return;
  }
  // still descending: extrapolate with the cubic, kept within [1.1 a, 4 a]
  bool ok;
  double a_new = cubic_step(s.prev_a, s.prev_f, s.prev_d, s.cur_a, s.cur_f, s.cur_d, ok);
  if (!ok || !isfinite(a_new) || a_new < 1.1 * s.cur_a || a_new > 4.0 * s.cur_a)
    a_new = (!ok || !isfinite(a_new) || a_new > 4.0 * s.cur_a) ? 4.0 * s.cur_a : 1.1 * s.cur_a;
  s.prev_a = s.cur_a, s.prev_f = s.cur_f, s.prev_d = s.cur_d;
  if (s.evals >= P.max_ls) {
    finish(s);
    return;
  }
  s.alpha = a_new;
  s.phase = LS_BRACKET;
  s.result = LR_CONT;
}

__global__ __launch_bounds__(TPB) void search_step(LbState* st, LbParams P, const double* partial,
                                                   const double* E_total, const int* status) {
  if (st->result != LR_CONT) return;
  const double d = sum_partials(partial);
  if (threadIdx.x != 0) return;
  LbState s = *st;
  if (*status != 0) {
    s.status = *status;
    s.result = LR_STATUS;
    *st = s;
    return;
  }
  const double a = s.alpha, f = *E_total;
  ++s.evals;
  s.last_a = a;
  if (f < s.best_f) {
    s.best_a = a;
    s.best_f = f;
  }
  switch (s.phase) {
    case LS_TRIAL:
      s.cur_a = a, s.cur_f = f, s.cur_d = d;
      if (strong_wolfe(s, P, a, f, d)) accept(s, a, f);
      else bracket_next(s, P);
      break;
    case LS_BRACKET:
      s.cur_a = a, s.cur_f = f, s.cur_d = d;
      s.first = 0;
      if (strong_wolfe(s, P, a, f, d) || approx_wolfe(s, P, f, d)) accept(s, a, f);
      else bracket_next(s, P);
      break;
    case LS_ZOOM:
      if (strong_wolfe(s, P, a, f, d) || approx_wolfe(s, P, f, d)) {
        accept(s, a, f);
        break;
      }
      if (f > s.f0 + P.c1 * a * s.dphi0 || f >= s.lo_f) {
        s.hi_a = a, s.hi_f = f, s.hi_d = d;
      } else {
        if (d * (s.hi_a - s.lo_a) >= 0.0) s.hi_a = s.lo_a, s.hi_f = s.lo_f, s.hi_d = s.lo_d;
        s.lo_a = a, s.lo_f = f, s.lo_d = d;
      }
      zoom_next(s, P);
      break;
    default:  // LS_BEST: the re-evaluated lowest point
      accept(s, s.best_a, s.best_f);
      break;
  }
  *st = s;
}

// partials of s.y, y.y and gw.gw for the accepted pair s = a p, y = gw - g
__global__ __launch_bounds__(TPB) void pair_partial(const LbState* st, const double* __restrict__ p,
                                                    const double* __restrict__ gw, const double* __restrict__ g,
                                                    int64_t n, double* partial) {
  if (st->result != LR_ACCEPT) return;
  const double a = st->acc_a;
  __shared__ double red[16];
  double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0, s3 = 0.0, c3 = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const double sj = a * p[j], yj = gw[j] - g[j];
    neumaier_add(s1, c1, sj * yj);
    neumaier_add(s2, c2, yj * yj);
    neumaier_add(s3, c3, gw[j] * gw[j]);
  }
  const double t1 = block_sum_neumaier(s1, c1, red);
  const double t2 = block_sum_neumaier(s2, c2, red);
  const double t3 = block_sum_neumaier(s3, c3, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = t1;
    partial[LB_DOT_BLOCKS + blockIdx.x] = t2;
    partial[2 * LB_DOT_BLOCKS + blockIdx.x] = t3;
  }
}

__global__ __launch_bounds__(TPB) void pair_final(LbState* st, const double* partial) {
  if (st->result != LR_ACCEPT) return;
  const double sy = sum_partials(partial);
  const double yy = sum_partials(partial + LB_DOT_BLOCKS);
  const double gg = sum_partials(partial + 2 * LB_DOT_BLOCKS);
  if (threadIdx.x != 0) return;
  st->sy = sy;
  st->yy = yy;
  st->gg = gg;
  st->E = st->acc_f;
  st->store = sy > 0.0 ? 1 : 0;
  if (st->store) {
    const int i = st->head;
    st->wslot = i;
    st->ys[i] = sy;
    st->head = (i + 1) % st->m;
    st->count = min(st->count + 1, st->m);
    st->beta = yy / sy;
  }
}

// x += a p, g = gw, and the pair into its slot when stored
__global__ void advance(const LbState* st, double* __restrict__ x, double* __restrict__ g,
                        const double* __restrict__ p, const double* __restrict__ gw, double* __restrict__ S,
                        double* __restrict__ Y, int64_t n) {
  if (st->result != LR_ACCEPT) return;
  const double a = st->acc_a;
  const bool store = st->store != 0;
  double* __restrict__ Si = S + (int64_t)st->wslot * n;
  double* __restrict__ Yi = Y + (int64_t)st->wslot * n;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    const double sj = a * p[j], gj = gw[j];
    if (store) {
      Si[j] = sj;
      Yi[j] = gj - g[j];
    }
    x[j] = x[j] + sj;
    g[j] = gj;
  }
}

// |x_k|^2 of each instance's segment, one workgroup per instance
__global__ __launch_bounds__(TPB) void segment_norms(const LbState* st, const double* __restrict__ x,
                                                     const int64_t* __restrict__ off, double* partial) {
  if (st->result != LR_ACCEPT) return;
  __shared__ double red[16];
  double s = 0.0, c = 0.0;
  for (int64_t j = off[blockIdx.x] + threadIdx.x; j < off[blockIdx.x + 1]; j += blockDim.x)
    neumaier_add(s, c, x[j] * x[j]);
  const double t = block_sum_neumaier(s, c, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(TPB) void segment_norm_max(LbState* st, const double* partial, int n_inst) {
  if (st->result != LR_ACCEPT) return;
  __shared__ double red[TPB];
  double m = 0.0;
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) m = fmax(m, partial[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) st->xmax2 = red[0];
}

}  // namespace

void launch_lb_start(LbState* st, const double* g, int64_t n, const double* E_total, double beta0, int set_beta,
                     int m, double* partial, hipStream_t s) {
  dot_partial<<<LB_DOT_BLOCKS, TPB, 0, s>>>(g, g, n, nullptr, partial);
  start_state<<<1, TPB, 0, s>>>(st, E_total, beta0, set_beta, m, partial);
}

void launch_lb_direction(LbState* st, const LbParams& P, const double* x, const double* g, double* p, double* q,
                         const double* S, const double* Y, const double* hd, const double* wv, int64_t n,
                         double* partial, double* xtrial, hipStream_t s) {
  const int vg = vgrid(n);
  for (int t = 0; t <= 2 * P.m; ++t) {
    two_loop_stage<<<LB_DOT_BLOCKS, TPB, 0, s>>>(st, t, g, q, p, S, Y, hd, wv, P.gamma, x, xtrial, n, partial);
    two_loop_scalar<<<1, TPB, 0, s>>>(st, t, partial);
  }
  // preconditioned steepest descent when the two-loop direction does not descend
  precond<<<vg, TPB, 0, s>>>(p, g, hd, wv, n, P.gamma, -1.0, st, &st->steepest);
  dot_partial<<<LB_DOT_BLOCKS, TPB, 0, s>>>(g, p, n, &st->steepest, partial);
  search_begin<<<1, TPB, 0, s>>>(st, partial);
  trial_point<<<vg, TPB, 0, s>>>(xtrial, x, p, n, st, &st->steepest);
}

void launch_lb_restart(LbState* st, const LbParams& P, const double* x, const double* g, double* p,
                       const double* hd, const double* wv, int64_t n, double* partial, double* xtrial,
                       hipStream_t s) {
  const int vg = vgrid(n);
  force_steepest<<<1, 1, 0, s>>>(st);
  precond<<<vg, TPB, 0, s>>>(p, g, hd, wv, n, P.gamma, -1.0, st, nullptr);
  dot_partial<<<LB_DOT_BLOCKS, TPB, 0, s>>>(g, p, n, nullptr, partial);
  search_begin<<<1, TPB, 0, s>>>(st, partial);
  trial_point<<<vg, TPB, 0, s>>>(xtrial, x, p, n, st, nullptr);
}

void launch_lb_after_probe(LbState* st, const LbParams& P, double* x, double* g, const double* p,
                           const double* gw, const double* E_total, const int* status, double* S, double* Y,
                           int64_t n, const int64_t* off, int n_inst, double* partial, double* xtrial,
                           LbState* summary, hipStream_t s) {
  const int vg = vgrid(n);
  dot_partial<<<LB_DOT_BLOCKS, TPB, 0, s>>>(gw, p, n, nullptr, partial);
  search_step<<<1, TPB, 0, s>>>(st, P, partial, E_total, status);
  trial_point<<<vg, TPB, 0, s>>>(xtrial, x, p, n, st, nullptr);
  pair_partial<<<LB_DOT_BLOCKS, TPB, 0, s>>>(st, p, gw, g, n, partial);
  pair_final<<<1, TPB, 0, s>>>(st, partial);
  advance<<<vg, TPB, 0, s>>>(st, x, g, p, gw, S, Y, n);
  if (P.reset_norm > 0.0 && n_inst > 0) {
    segment_norms<<<n_inst, TPB, 0, s>>>(st, x, off, partial);
    segment_norm_max<<<1, TPB, 0, s>>>(st, partial, n_inst);
  }
  (void)hipMemcpyAsync(summary, st, sizeof(LbState), hipMemcpyDeviceToHost, s);
}

}  // namespace etdm
