// Device-resident L-BFGS iteration (Sec. 3.1-3.3): the two-loop recursion over a
// ring of stored pairs, the strong / approximate Wolfe tests and the cubic
// interpolation of the line search, and the memory and beta update all run on
// the device.  The host replays fixed launch sequences and reads one small
// summary per line-search probe.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace etdm {

constexpr int LB_MMAX = 8;           // largest memory length m
constexpr int LB_DOT_BLOCKS = 2048;  // workgroups of the vector reductions (8 per CU)

// outcome of a line-search step
enum LbResult : int32_t { LR_CONT = 0, LR_ACCEPT = 1, LR_FAIL = 2, LR_STATUS = 3 };
// phase of the probe being evaluated
enum LbPhase : int32_t { LS_TRIAL = 0, LS_BRACKET = 1, LS_ZOOM = 2, LS_BEST = 3 };

// Line-search constants (Eq. strw1, strw2, aprw, aprw2) and preconditioner mixing.
struct LbParams {
  double c1, c2, delta, sigma, eps, gamma;
  int32_t max_ls, m;
  double reset_norm;  // > 0: the largest per-instance parameter norm is tracked
};

// All state of one L-BFGS run that lives on the device.  A probe is (step a,
// energy f, slope d = g(a).p).
struct LbState {
  double f0, dphi0;       // energy and slope at a = 0
  double alpha;           // step of the probe being evaluated next
  double prev_a, prev_f, prev_d, cur_a, cur_f, cur_d;
  double lo_a, lo_f, lo_d, hi_a, hi_f, hi_d;
  double best_a, best_f, last_a;
  double acc_a, acc_f;    // the accepted probe
  double E;               // energy at the current point x
  double beta;            // beta^(k) of the preconditioner (Eq. prec_3)
  double gg;              // |g|^2 at x
  double sy, yy;          // of the latest pair
  double coef;            // two-loop scalar of the current step
  double xmax2;           // largest per-instance |x_k|^2 after the last accepted step
  double ys[LB_MMAX];     // s_i . y_i of the stored pairs
  double al[LB_MMAX];     // two-loop alpha_i
  int32_t evals;          // evaluations in this line search
  int32_t phase, first, result;
  int32_t count, head, m; // stored pairs, next slot, ring length
  int32_t status;         // evaluation status word seen by the last step
  int32_t steepest;       // 1 when this iteration's direction is preconditioned steepest descent
  int32_t store, wslot;   // whether the accepted pair is stored, and where
  int32_t pad;
};

// ---- launchers (stream-ordered; every scalar stays in LbState) ----

// State after an evaluation at x: E from E_total, |g|^2, empty memory; beta is
// set to beta0 when set_beta (a first start), kept otherwise (a reference reset).
void launch_lb_start(LbState* st, const double* g, int64_t n, const double* E_total, double beta0, int set_beta,
                     int m, double* partial, hipStream_t s);
// p = -H g by the two-loop recursion (m fixed steps per loop, masked by the pair
// count) with the diagonal preconditioner as H0, then the slope g.p, the switch to
// preconditioned steepest descent when p is not a descent direction, and the
// line-search start with the trial step a = 1 (written to xtrial = x + p).
void launch_lb_direction(LbState* st, const LbParams& P, const double* x, const double* g, double* p, double* q,
                         const double* S, const double* Y, const double* hd, const double* wv, int64_t n,
                         double* partial, double* xtrial, hipStream_t s);
// Erase the memory and restart the line search along preconditioned steepest descent.
void launch_lb_restart(LbState* st, const LbParams& P, const double* x, const double* g, double* p,
                       const double* hd, const double* wv, int64_t n, double* partial, double* xtrial,
                       hipStream_t s);
// After an evaluation at x + alpha p (gradient gw, total energy E_total, status
// word): one line-search step; on CONT the next trial point goes to xtrial, on
// ACCEPT the pair (alpha p, gw - g) is stored when s.y > 0 (beta updated) and
// x, g advance to the accepted point; with P.reset_norm > 0 the largest squared
// norm of the instances' segments of x (offsets off[0..n_inst]) goes to xmax2.
// The state is then copied to `summary`.
void launch_lb_after_probe(LbState* st, const LbParams& P, double* x, double* g, const double* p,
                           const double* gw, const double* E_total, const int* status, double* S, double* Y,
                           int64_t n, const int64_t* off, int n_inst, double* partial, double* xtrial,
                           LbState* summary, hipStream_t s);

}  // namespace etdm
