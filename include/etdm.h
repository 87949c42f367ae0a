/*
 * etdm.h — C ABI of the MI355X (gfx950) library for the hot path of
 * exponential-transformation direct minimization (ETDM).
 *
 * One call of etdm_energy_grad evaluates, for every instance of a batch
 * (independent molecules, or the k-points of one crystal):
 *
 *   U = exp(A)            from the eigendecomposition of iA      (Sec. 3.4, Eq. ed)
 *   C = C0 U              current orbitals                        (Sec. 2, Eq. unit_transf)
 *   rho = C F C^dagger    density matrix                          (Sec. 2)
 *   H(rho), E(rho)        model functional, see below
 *   H_MO = C^dagger H C,  L = w [F, H_MO]                         (Sec. 2, def. of L_mk)
 *   dE/dA                 Eq. gradients, back-transformed through the eigenbasis
 *                         of iA with the divided-difference factors of its
 *                         eigenvalues (Sec. 3.4)
 *
 * Model functional (stands in for the Kohn-Sham functional):
 *   E = sum_k w_k Tr(rho_k H0_k) + (U_hub/2) sum_mu n_mu^2,
 *   n = diag(rho_k) per instance, or sum_k w_k diag(rho_k) when `couple` is set,
 *   H_k = H0_k + U_hub diag(n).
 *
 * Parametrizations (Sec. 2 and Sec. 3.4):
 *   ETDM_REAL_OV       real A = [[0, B], [-B^T, 0]] (Hutter's occupied-virtual form,
 *                      exact for a unitary-invariant functional with equal
 *                      occupations f_occ on the first N columns and 0 elsewhere).
 *                      A is passed as B (N x (M-N), row-major, float64).
 *   ETDM_COMPLEX_FULL  complex skew-Hermitian A (M x M, row-major, interleaved
 *                      complex float64).  Only the upper triangle including the
 *                      diagonal is read; Re of the diagonal is ignored (Sec. 2).
 *
 * Gradient layout (same layout as A):
 *   REAL_OV            G[i][j] = dE/dB_ij
 *   COMPLEX_FULL       G[i][j] = dE/dRe a_ij + i dE/dIm a_ij for i <= j, 0 below
 *                      (Sec. 2, the real-variable derivatives built from the
 *                      derivative with respect to a_ij).
 *
 * Memory: every matrix pointer passed to a call is a DEVICE pointer unless
 * stated otherwise; all descriptor arrays are HOST pointers.  Batches are packed
 * back to back in instance order (instance i starts after all elements of
 * instances < i).  Calls are asynchronous on the given HIP stream (a
 * hipStream_t passed as void*, NULL = default stream); argument errors are
 * returned synchronously; device-side failures (eigensolver not converged,
 * non-finite values) set a status word that etdm_sync_status reports.
 * The handle owns device copies of C0, H0 and f plus all workspaces; no call
 * after etdm_create allocates device memory.  A handle must not be used from
 * two threads at once.  No function throws or aborts.
 */
#ifndef ETDM_H
#define ETDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct etdm_handle etdm_handle;

typedef enum {
  ETDM_OK = 0,
  ETDM_E_ARG = -1,        /* invalid argument (null pointer, bad enum, bad occupations) */
  ETDM_E_SHAPE = -2,      /* inconsistent sizes */
  ETDM_E_HIP = -3,        /* a HIP runtime call failed */
  ETDM_E_NOMEM = -4,      /* device allocation failed in etdm_create */
  ETDM_E_EIGH = -5,       /* FP64 Jacobi eigensolver hit its sweep limit */
  ETDM_E_NONFINITE = -6,  /* NaN/Inf in the energy or gradient */
  ETDM_E_LINESEARCH = -7, /* line search found no acceptable step */
  ETDM_E_STATE = -8       /* call sequence error (e.g. L-BFGS not initialised) */
} etdm_status;

typedef enum { ETDM_REAL_OV = 0, ETDM_COMPLEX_FULL = 1 } etdm_kind;

/* Arithmetic of the dense contractions.  The eigendecomposition, the spectral
 * and divided-difference factors and the energy reduction are FP64 in every mode.
 * REAL_OV: P = B B^T, V = X^T B (X: eigenvectors of P) and the N x N spectral
 * products are FP64 in every mode as well; every later product is taken in the
 * eigenbasis of P, where its terms stay bounded at any rotation angle, so the split
 * modes keep their accuracy for large A. */
typedef enum {
  ETDM_FP64 = 0,   /* FP64 MFMA */
  ETDM_FP32 = 1,   /* operands rounded to FP32, FP32 MFMA, FP64 flush every K chunk */
  ETDM_BF16X3 = 2, /* 2-way BF16 split (hi+lo), 3 products, FP32 MFMA accumulation */
  ETDM_BF16X6 = 3, /* 3-way BF16 split (hi+mid+lo), 6 products */
  ETDM_MIXED = 4   /* by role: the gradient-only contractions (C_virt, L_ov, L_ov V^T,
                      the eigenbasis products of the gradient, G) as ETDM_BF16X6; the
                      ones E depends on (C0_o X, C0_v V^T, C_occ, H0 C_occ) in FP64, or
                      as ETDM_BF16X6 when every instance has N >=
                      ETDM_MIXED_SPLIT_E_MIN_N (the split's rounding of the orbitals
                      then stays far below 1e-8 Ha per electron) */
} etdm_precision;

#define ETDM_MIXED_SPLIT_E_MIN_N 512

typedef struct {
  int32_t n_inst;         /* number of instances (molecules or k-points), >= 1 */
  const int32_t *M;       /* host [n_inst]: basis size, >= 1 */
  const int32_t *N;       /* host [n_inst]: REAL_OV: occupied count 0 <= N <= M;
                             COMPLEX_FULL: ignored */
  int32_t kind;           /* etdm_kind */
  int32_t precision;      /* etdm_precision (COMPLEX_FULL: ETDM_FP64, ETDM_BF16X6 or ETDM_MIXED;
                             its split products are real products of the real views of the
                             interleaved complex operands) */
  double hubbard_U;       /* U_hub of the model functional */
  int32_t couple;         /* 1: Hubbard term on sum_k w_k diag(rho_k) (needs equal M) */
  const double *weights;  /* host [n_inst] k-point weights, NULL = all 1 */
  int32_t h0_format;      /* 0: dense H0 (M x M per instance);
                             1: block-sparse rows (REAL_OV only) */
  int32_t bsr_block;      /* block size when h0_format = 1 (M divisible by it) */
  const int32_t *bsr_row_ptr; /* host, per instance (M/bs + 1) entries, concatenated */
  const int32_t *bsr_col_idx; /* host, per instance row_ptr[last] entries, concatenated */
  int32_t gemm_tuning;    /* kernel choice of the real FP64 and BF16x6 GEMM stages:
                             0 = time the ETDM_GEMM_VARIANTS kernels on the handle's
                             buffers in etdm_create and keep the fastest, once per stage
                             signature (device architecture and compute units, precision,
                             operand ops, every problem's shape) in a process: a later
                             handle with the same stage takes the cached choice and times;
                             with the environment variable ETDM_TUNE_CACHE naming a file,
                             choices are also read from it and appended to it, so they
                             carry over between processes; 1 = fixed rule
                             (packed 128 x 128 tiles when every problem of the stage is at
                             least 128 x 128 with K >= 256, else grouped 64 x 64); forced:
                             2 = packed 128 x 128, 3 = grouped 64 x 64, 4 = packed 64 x 64,
                             5 = packed 128 x 64, 6 = packed 64 x 128.
                             Other values: ETDM_E_ARG */
  int32_t gradient;       /* 0 = exact dE/dA (Eq. gradients, Sec. 3.4); 1 = the approximate
                             gradient G ~ L^T of Eq. app_grad (first term of the expansion,
                             exact at A = 0; keep A small, e.g. by reference updates).
                             Other values: ETDM_E_ARG */
  int32_t expm_method;    /* 0 = exp(A) through the eigendecomposition of iA (Eq. ed, Eq. uinv);
                             1 = scaling and squaring with the [9/9] Pade approximant
                             (Eq. ss), and with gradient = 0 the exact gradient through its
                             Frechet derivative: COMPLEX_FULL with M <= 1024 only
                             (ETDM_E_ARG / ETDM_E_SHAPE otherwise); one stream
                             synchronization per evaluation reads the number of squarings,
                             so its evaluations are not replayed from graphs */
  double odd_lambda;      /* strength of an orbital-dependent model term (the PZ-SIC form of
                             L in Sec. 2): E += -(lambda/2) sum_k w f_k sum_mu |C_mu_k|^4,
                             L_mk += w (f_m conj(V_km) - f_k V_mk), V^k = diag(-lambda
                             |C_mu_k|^2).  0 = off; nonzero needs COMPLEX_FULL (the ov form
                             assumes unitary invariance).  Non-finite: ETDM_E_ARG */
  const void *overlap;    /* NULL: orthonormal basis.  Else device, the overlap S of a
                             non-orthogonal basis (Sec. 2: C^H S C = I), layout of a dense H0
                             (M x M per instance, float64 or complex), Hermitian positive
                             definite; C0 must be S-orthonormal and H0 (dense only) is in the
                             same basis.  The site populations of the Hubbard term become
                             diag(S^1/2 rho S^1/2).  etdm_create applies the Lowdin transform
                             H0 <- S^-1/2 H0 S^-1/2, C0 <- S^1/2 C0 once (Newton-Schulz for
                             S^+-1/2); afterwards the handle works in that orthonormal basis.
                             ETDM_E_ARG if S is not positive definite to working accuracy
                             or with a block-sparse H0 */
  int32_t want_rho;       /* 1: the handle also holds an M x M workspace per instance for
                             etdm_density; 0: etdm_density returns ETDM_E_STATE */
} etdm_desc;

/* Create a handle.  H0: device, dense float64 (REAL_OV) or complex float64
 * (COMPLEX_FULL) M x M per instance, or (h0_format = 1) the concatenated
 * bs x bs row-major blocks in row_ptr/col_idx order.  H0 must be Hermitian.
 * C0: device, M x M per instance, orthonormal columns (float64 or complex).
 * f: host [sum M] occupations.  All inputs are copied; the caller keeps
 * ownership.  `stream` orders the copies. */
etdm_status etdm_create(etdm_handle **h, const etdm_desc *d, const void *H0, const void *C0,
                        const double *f, void *stream);
etdm_status etdm_destroy(etdm_handle *h);

/* U = exp(A) per instance (Eq. ed; for REAL_OV the same U in Hutter's closed
 * form, Eq. uinv).  A: device, parameter layout above.  U: device, M x M per
 * instance (float64 for REAL_OV, complex for COMPLEX_FULL). */
etdm_status etdm_expm(etdm_handle *h, const void *A, void *U, void *stream);

/* E and dE/dA (Eq. gradients), or with desc.gradient = 1 the approximation
 * G ~ L^T of Eq. app_grad in the same layout.  A, G: device, parameter layout.  E: device
 * float64 [n_inst + 1] = per-instance energies (weighted, Hubbard included per
 * instance; with `couple` the Hubbard energy is in the total only) followed
 * by the batch total. */
etdm_status etdm_energy_grad(etdm_handle *h, const void *A, double *E, void *G, void *stream);

/* Density matrix rho = C F C^dagger of the orbitals C = C0 exp(A) (Sec. 2, the
 * definition of rho_mu_nu from the orbitals and their occupations), per instance.
 * REAL_OV: rho = f_occ C_occ C_occ^T, a symmetric rank-N product on the matrix cores
 * (row panels of the upper triangle, then mirrored), in the arithmetic of the
 * contractions E depends on (etdm_precision); COMPLEX_FULL: rho_k = C_k diag(f_k) C_k^H
 * per k-point (k-point weights not applied), FP64.  Only diag(rho) enters E and H(rho)
 * of the model functional; this is the full matrix for inspection and comparison.
 * A: device, parameter layout.  rho: device, M x M per instance packed back to back
 * (float64 / complex float64), overwritten.  Needs desc.want_rho = 1 at creation
 * (ETDM_E_STATE otherwise).  Asynchronous on `stream`. */
etdm_status etdm_density(etdm_handle *h, const void *A, void *rho, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): etdm_energy_grad for ONE real
 * occupied-virtual instance with a dense H0, in FP64, without a handle.  Every
 * intermediate and every launch descriptor lives in a library-owned static device
 * array of ETDM_STATIC_SCRATCH_BYTES (one per GPU, held until the process ends); the
 * call allocates nothing and may be captured in a HIP graph.
 * Sizes: 1 <= N < M <= ETDM_STATIC_MAX_M and N <= ETDM_STATIC_MAX_N, else ETDM_E_SHAPE.
 * H0, C0: device, M x M float64 (H0 symmetric, C0 orthogonal, occupied columns first).
 * B: device, N x (M - N), the parameters of A = [[0, B], [-B^T, 0]].  f_occ: occupation
 * of the first N orbitals (the others are empty).  E: device [2] = the energy and the
 * total (equal for one instance).  G: device N x (M - N), dE/dB.  status: device int32,
 * cleared by the call, then ORed with 1 (eigensolver sweep limit) and 2 (non-finite E
 * or G).  Asynchronous on `stream`.  Calls on one GPU share its array and overwrite
 * it: calls that overlap in time on one GPU (other streams, other threads) race, so
 * the caller must order them. */
#define ETDM_STATIC_SCRATCH_BYTES (4 << 20)
#define ETDM_STATIC_MAX_M 400
#define ETDM_STATIC_MAX_N 88
etdm_status etdm_energy_grad_static(int32_t M, int32_t N, double f_occ, double hubbard_U, const double *H0,
                                    const double *C0, const double *B, double *E, double *G,
                                    int32_t *status, void *stream);

/* Replace the reference orbitals C0 <- C0 exp(A) (Sec. 3.4, reference update).
 * Erases the L-BFGS memory. */
etdm_status etdm_set_reference(etdm_handle *h, const void *A, void *stream);

/* L-BFGS settings (Sec. 3.1-3.3).  etdm_lbfgs_defaults fills the paper's values:
 * m = 3, c1 = 1e-4, c2 = 0.9, delta = 0.1, sigma = 0.9, eps = 1e-6,
 * gamma = 0.25, beta0 = 1, reset_every = 20, max_ls = 20, and reset_norm = 0. */
typedef struct {
  int32_t m;
  double c1, c2, delta, sigma, eps, gamma, beta0;
  int32_t reset_every; /* reference reset period in iterations, 0 = never */
  int32_t max_ls;      /* energy+gradient evaluations per line search */
  double reset_norm;   /* also reset the reference when, after a step, some instance's
                          parameters have a 2-norm above this (Sec. 3.4 suggests resets
                          once the norm of A exceeds 1); 0 = never */
} etdm_lbfgs_params;

typedef struct {
  int32_t iter;      /* iterations done so far */
  int32_t n_evals;   /* energy+gradient evaluations so far (all line searches) */
  double alpha;      /* accepted step length */
  double E;          /* total energy after the step */
  double gnorm;      /* Euclidean norm of the gradient after the step */
  int32_t flags;     /* bit 0: reference reset before this step,
                        bit 1: steepest-descent fallback (memory erased),
                        bit 2: line search failed (state unchanged) */
} etdm_lbfgs_info;

void etdm_lbfgs_defaults(etdm_lbfgs_params *p);

/* One L-BFGS iteration on the whole batch as one vector of free variables.
 * A: device, in/out (current parameters); E: device [n_inst + 1] out; G:
 * device out (gradient at the new A).  On the first call (or after
 * etdm_set_reference) the state is initialised from A.  When a reference reset
 * happens (every reset_every iterations) C0 <- C0 exp(A) and A is set to 0
 * before the step.  params may be NULL (defaults).  info: host, out.
 * The direction, the Wolfe tests and cubic steps of the line search, and the
 * memory and beta updates are decided on the device; the host synchronizes
 * `stream` once per line-search probe to read the outcome.  With etdm_set_graph
 * on, each probe (with the direction for the first) replays one captured graph.
 * ETDM_E_LINESEARCH when neither the L-BFGS direction nor steepest descent
 * yields an acceptable step (state unchanged). */
etdm_status etdm_lbfgs_step(etdm_handle *h, const etdm_lbfgs_params *params, void *A, double *E,
                            void *G, etdm_lbfgs_info *info, void *stream);

/* L-BFGS checkpoint (Sec. 3.4: the state of the minimization is the reference
 * orbitals, A and the L-BFGS memory).  The image lives in caller-owned DEVICE
 * memory of etdm_lbfgs_state_bytes(h) bytes (0 before the first
 * etdm_lbfgs_step): a header, the device-side L-BFGS scalars, A, g, the m
 * stored pairs and every instance's reference orbitals C0.  It is opaque and
 * valid only for a handle created from the same shapes, kind, precision and
 * gradient mode (etdm_lbfgs_set_state returns ETDM_E_SHAPE otherwise).
 * set_state also rebuilds the preconditioner from the restored C0.  On a handle
 * whose kernels are the same (the same gemm_tuning choice), the etdm_lbfgs_step
 * calls after set_state repeat bit for bit those that followed get_state.
 * get_state before the first etdm_lbfgs_step: ETDM_E_ARG.  Both synchronize
 * `stream`. */
size_t etdm_lbfgs_state_bytes(const etdm_handle *h);
etdm_status etdm_lbfgs_get_state(etdm_handle *h, void *state, void *stream);
etdm_status etdm_lbfgs_set_state(etdm_handle *h, const void *state, void *stream);

/* Wait for `stream` and report a device-side failure recorded since the last call. */
etdm_status etdm_sync_status(etdm_handle *h, void *stream);

const char *etdm_status_string(etdm_status s);
/* Human-readable detail of the last error on this handle ("" if none). */
const char *etdm_last_error(const etdm_handle *h);

/* Replay the launch sequence of etdm_energy_grad from a HIP graph (enable = 1)
 * or launch it kernel by kernel (0, the default).  The graph is captured on
 * the first call after enabling (on an internal stream) and launched on the
 * caller's stream; it holds only handle-owned buffers, so A, E and G may
 * change between calls.  While stage timing is on, calls run eagerly. */
etdm_status etdm_set_graph(etdm_handle *h, int32_t enable);

/* Tracing: per-stage HIP-event timing of the launch sequences.  A "stage" is
 * one launch (or grouped launch) of the path: a GEMM group, the eigensolver,
 * an elementwise pass.  `mask` selects stages by index (bit i = stage i,
 * -1 = all, 0 = off); events are recorded on the stream of each call around
 * every selected stage.  Timing adds two event records per selected stage. */
etdm_status etdm_set_timing(etdm_handle *h, int64_t mask);
/* Clear the accumulated times and launch counts. */
etdm_status etdm_reset_timing(etdm_handle *h);
/* Number of stages of this handle's path. */
int32_t etdm_stage_count(const etdm_handle *h);
/* Stage i: its name (static string), launches timed so far, their total
 * duration in ms (waits for the recorded events), and the algorithmic flops
 * and minimum HBM bytes of one launch (operands read once, results written
 * once, float64 storage).  Any output pointer may be NULL. */
etdm_status etdm_stage_info(etdm_handle *h, int32_t i, const char **name, int64_t *launches,
                            double *total_ms, double *flops, double *bytes);

/* GEMM kernels of a real FP64 / BF16x6 stage, in the order of etdm_stage_kernel's
 * tuned_ms: grouped 64 x 64 tiles that read (and split) the operands in every tile;
 * then the operands packed (and split) once per launch into a panel buffer and
 * tiles of 64 x 64, 128 x 64, 64 x 128 and 128 x 128. */
#define ETDM_GEMM_VARIANTS 5

/* GEMM kernel of stage i: *variant = "tile64", "packed64", "packed128x64",
 * "packed64x128" or "packed128" (prefixed "fp64_" for FP64 stages), "zgemm64"
 * (complex), or "" for a stage that is not a GEMM.  tuned_ms (ETDM_GEMM_VARIANTS
 * doubles, or NULL) = the launch times of the kernels measured by the tuning in
 * etdm_create (0 when not timed). */
etdm_status etdm_stage_kernel(const etdm_handle *h, int32_t i, const char **variant, double *tuned_ms);

/* Number of parameters of one A (or G) array in float64 units:
 * REAL_OV sum N(M-N); COMPLEX_FULL 2 sum M^2. */
int64_t etdm_param_count(const etdm_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* ETDM_H */
