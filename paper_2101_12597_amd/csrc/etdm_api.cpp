// Host side of the ETDM library: handle, workspace layout, the launch
// sequences of the energy+gradient path, the matrix exponential, reference
// resets and the L-BFGS driver (Sec. 3.1-3.4).  All device memory is allocated
// in etdm_create; the call paths only launch kernels and copy between buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "etdm.h"
#include "common.h"
#include "ov.h"
#include "eigh_large.h"
#include "lbfgs.h"
#include "expm_ss.h"
#include "overlap.h"

using namespace etdm;

namespace {

constexpr size_t ALIGN = 256;
constexpr int LARGE_EIGH_MAX_SWEEPS = 30;

// Gauss-Legendre nodes and weights on [0, 1] by Newton iteration on the
// Legendre polynomial P_n (three-term recurrence), mapped from [-1, 1].
void gauss_legendre01(int n, double* t, double* w) {
  auto legendre = [n](double x, double& pn, double& dpn) {
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    pn = p1;
    dpn = n * (x * p1 - p0) / (x * x - 1.0);
  };
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), pn, dpn;
    for (int it = 0; it < 100; ++it) {
      legendre(x, pn, dpn);
      const double dx = pn / dpn;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    legendre(x, pn, dpn);
    t[i] = 0.5 * (x + 1.0);
    w[i] = 1.0 / ((1.0 - x * x) * dpn * dpn);  // half of the [-1, 1] weight 2 / ((1 - x^2) P_n'^2)
  }
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// One grouped GEMM launch.  Problems are added at plan time and uploaded once.
// A real FP64 or BF16x6 stage has five kernels:
//   V_TILE64   the grouped 64 x 64 kernel that reads (and splits) the operands
//              inside every tile (gemm.hip);
//   V_P11 .. V_P22  a pack pass into a panel layout shared by all stages, then
//              tiles of tpm x tpn panels of 64 on the packed operands
//              (gemm_split.hip): 64 x 64, 128 x 64, 64 x 128, 128 x 128.
// Which one runs is chosen at plan time (tune_stages).
enum GemmVariant { V_TILE64 = 0, V_P11 = 1, V_P21 = 2, V_P12 = 3, V_P22 = 4, V_COUNT = 5 };
constexpr int kVarTpm[V_COUNT] = {0, 1, 2, 1, 2};
constexpr int kVarTpn[V_COUNT] = {0, 1, 1, 2, 2};

// The launches of one packed variant.
struct PackPlan {
  std::vector<PackJob> jobs;
  std::vector<int32_t> chunk_job;  // pack workgroup -> job
  std::vector<SplitProb> probs;
  std::vector<int32_t> tile_prob;  // GEMM workgroup -> problem
  PackJob* d_jobs = nullptr;
  int32_t* d_chunk_job = nullptr;
  SplitProb* d_probs = nullptr;
  int32_t* d_tile_prob = nullptr;
  int chunks = 0, tiles = 0;
  // operands that change only with the reference orbitals (C0, H0 C0, a dense H0),
  // packed into an arena of their own when the reference changes, not per launch
  std::vector<PackJob> sjobs;
  std::vector<int32_t> schunk_job;
  PackJob* d_sjobs = nullptr;
  int32_t* d_schunk_job = nullptr;
  int schunks = 0;
};

// Address ranges of the operands that change only with the reference orbitals.
struct StaticRanges {
  std::vector<std::pair<const double*, const double*>> r;
  void add(const double* p, int64_t n) {
    if (p && n > 0) r.push_back({p, p + n});
  }
  bool has(const double* p) const {
    if (!p) return true;  // an absent operand does not make its panel dynamic
    for (const auto& x : r)
      if (p >= x.first && p < x.second) return true;
    return false;
  }
};

// Workgroup -> tile order of a packed launch of T tiles, appended to its tile table.
// Workgroup b runs on XCD b mod 8.  The tiles (problem after problem, each in its
// grouped order) are dealt to the XCDs in chunks of 8 consecutive tiles, chunk j to
// XCD j mod 8, so that every XCD gets a share of every problem (the problems of one
// launch can differ several-fold in K) while neighbouring tiles, which share operand
// panels, stay on one XCD's L2; then the lists are evened out to the workgroup count
// of each XCD.
inline void append_tile_order(std::vector<int32_t>& table, int T) {
  constexpr int XCDS = 8, CH = 8;
  std::vector<std::vector<int32_t>> lst(XCDS);
  for (int t = 0; t < T; ++t) lst[(t / CH) % XCDS].push_back(t);
  std::vector<int> want(XCDS);
  for (int x = 0; x < XCDS; ++x) want[x] = T > x ? (T - x + XCDS - 1) / XCDS : 0;
  std::vector<int32_t> spill;
  for (int x = 0; x < XCDS; ++x)
    while ((int)lst[x].size() > want[x]) {
      spill.push_back(lst[x].back());
      lst[x].pop_back();
    }
  for (int x = 0; x < XCDS; ++x)
    while ((int)lst[x].size() < want[x]) {
      lst[x].push_back(spill.back());
      spill.pop_back();
    }
  table.resize((size_t)2 * T);
  for (int b = 0; b < T; ++b) table[(size_t)T + b] = lst[b % XCDS][b / XCDS];
}

struct Stage {
  std::vector<GemmProb> probs;
  std::vector<int32_t> tile_prob;  // workgroup -> problem
  GemmProb* d = nullptr;
  int32_t* d_tile_prob = nullptr;
  int tiles = 0;
  int opA = OP_N, opB = OP_N, prec = GP_FP64;
  bool cplx = false;
  int variant = V_TILE64;
  char* arena = nullptr;                     // shared arena of the per-launch packs
  bool has_static = false;                   // the chosen variant packs static operands apart
  bool no_static = false;                    // forms a static operand itself (H0 C0): packs all per launch
  PackPlan pk[V_COUNT - 1];                  // the packed variants V_P11 .. V_P22
  float tuned_ms[V_COUNT] = {};              // plan-time launch times per variant (0: not timed)
  void init(int a, int b, int p, bool c = false) {
    opA = a;
    opB = b;
    prec = p;
    cplx = c;
  }
  void add(GemmProb p) {
    if (p.m <= 0 || p.n <= 0) return;
    p.tiles_n = ceil_div(p.n, GEMM_BN);
    p.tile_begin = tiles;
    tiles += p.tiles_n * ceil_div(p.m, GEMM_BM);
    tile_prob.resize(tiles, (int32_t)probs.size());
    probs.push_back(p);
  }
  // packed kernels: real FP64 / BF16x6, and complex BF16x6 through the real view of
  // the complex product (the complex FP64 stages keep the grouped complex kernel)
  bool can_pack() const {
    return (cplx ? prec == GP_BF16X6 : (prec == GP_BF16X6 || prec == GP_FP64)) && !probs.empty();
  }
  // the real view of a problem: complex op(A) (m x k) -> m x 2k, op(B) (k x n) ->
  // 2k x 2n, C (m x n) -> m x 2n doubles
  int view_n(const GemmProb& p) const { return cplx ? 2 * p.n : p.n; }
  size_t chunk_bytes() const {
    return prec == GP_FP64 ? (size_t)PK_CHUNK_64 * sizeof(double) : (size_t)PK_CHUNK_X6 * sizeof(__bf16);
  }
  int ktiles(const GemmProb& p) const {
    const int f = cplx ? 2 : 1;
    return ceil_div(f * std::max(p.k, 0), PK_K) + ceil_div(f * std::max(p.k2, 0), PK_K);
  }
  static int panels(int rows, int tp) { return tp * ceil_div(rows, PK_R * tp); }
  // bytes of the packed operands of all problems for packed variant v
  size_t pack_bytes(int v) const {
    size_t n = 0;
    for (const GemmProb& p : probs)
      n += (size_t)(panels(p.m, kVarTpm[v]) + panels(view_n(p), kVarTpn[v])) * ktiles(p) * chunk_bytes();
    return n;
  }
  // an operand panel (both K segments) is static when every source it packs is
  bool a_static(const GemmProb& p, const StaticRanges* sr) const {
    return sr && p.A && sr->has(p.A) && (p.k2 <= 0 || sr->has(p.A2));
  }
  bool b_static(const GemmProb& p, const StaticRanges* sr) const {
    return sr && p.B && sr->has(p.B) && (p.k2 <= 0 || sr->has(p.B2));
  }
  // bytes of the static operand panels of packed variant v
  size_t static_bytes(int v, const StaticRanges* sr) const {
    size_t n = 0;
    for (const GemmProb& p : probs) {
      if (a_static(p, sr)) n += (size_t)panels(p.m, kVarTpm[v]) * ktiles(p) * chunk_bytes();
      if (b_static(p, sr)) n += (size_t)panels(view_n(p), kVarTpn[v]) * ktiles(p) * chunk_bytes();
    }
    return n;
  }
  // pack jobs and packed problems of packed variant v with the operands at arena; with
  // sr, the static operand panels go to sarena and their jobs to the static list
  void plan_pack(int v, char* arena, const StaticRanges* sr = nullptr, char* sarena = nullptr) {
    const int tpm = kVarTpm[v], tpn = kVarTpn[v];
    PackPlan& q = pk[v - 1];
    q = PackPlan();
    const size_t chunk = chunk_bytes();
    size_t off = 0, soff = 0;
    auto job = [&](const double* src, char* dst, int64_t ld, double alpha, bool trans, int rows, int K,
                   int kt0, int kt, int np, int zmode, int zop, bool stat) {
      if (K <= 0) return;
      std::vector<PackJob>& jobs = stat ? q.sjobs : q.jobs;
      std::vector<int32_t>& cj = stat ? q.schunk_job : q.chunk_job;
      int& nch = stat ? q.schunks : q.chunks;
      PackJob j;
      j.src = src;
      j.dst = dst;
      j.ld = ld;
      j.alpha = alpha;
      j.trans = trans ? 1 : 0;
      j.cplx = zmode;
      j.op = zop;
      j.rows = rows;
      j.K = K;
      j.kt0 = kt0;
      j.ktiles = kt;
      j.kt_n = ceil_div(K, PK_K);
      j.begin = nch;
      nch += np * j.kt_n;
      cj.resize(nch, (int32_t)jobs.size());
      jobs.push_back(j);
    };
    // Packed operand regions already planned: a real single-segment operand whose rows
    // are a panel-aligned part of a region's rows of the same source (the same
    // matrix, ld, scale, orientation and K) reads that region instead of packing again
    // (the row panels of P = B B^T, an operand shared by two products of a stage).
    // (rows past the operand's own are read but only feed masked results; every panel
    // read lies inside the region's panels)
    struct Region {
      const double* src;
      int64_t ld;
      double alpha;
      bool trans, stat;
      int rows, panels, K, kt;
      char* dst;
    };
    std::vector<Region> regions;
    auto reuse = [&](const double* src, int64_t ld, double alpha, bool trans, int rows, int np, int K, int kt,
                     bool stat) -> char* {
      for (const Region& r : regions) {
        if (r.ld != ld || r.alpha != alpha || r.trans != trans || r.K != K || r.kt != kt || r.stat != stat) continue;
        const int64_t step = trans ? 1 : ld, d = src - r.src;
        if (d < 0 || d % step != 0) continue;
        const int64_t at = d / step;
        if (at % PK_R != 0 || at + rows > r.rows || at / PK_R + np > r.panels) continue;
        return r.dst + (size_t)(at / PK_R) * kt * chunk;
      }
      return nullptr;
    };
    const int f = cplx ? 2 : 1;  // doubles per element along k and n
    for (const GemmProb& p : probs) {
      const int kt = ktiles(p), kt1 = ceil_div(f * std::max(p.k, 0), PK_K);
      const int nv = view_n(p);
      const int pa = panels(p.m, tpm), pb = panels(nv, tpn);
      const bool sa = sarena && a_static(p, sr), sb = sarena && b_static(p, sr);
      const bool one = !cplx && p.k2 <= 0 && p.k > 0;  // candidates for a shared region
      char* a = one ? reuse(p.A, p.lda, p.alpha, opA == OP_T, p.m, pa, p.k, kt, sa) : nullptr;
      const bool a_new = a == nullptr;
      if (a_new) {
        a = sa ? sarena + soff : arena + off;
        (sa ? soff : off) += (size_t)pa * kt * chunk;
        if (one) regions.push_back(Region{p.A, p.lda, p.alpha, opA == OP_T, sa, p.m, pa, p.k, kt, a});
      }
      char* b = one ? reuse(p.B, p.ldb, 1.0, opB != OP_T, nv, pb, p.k, kt, sb) : nullptr;
      const bool b_new = b == nullptr;
      if (b_new) {
        b = sb ? sarena + soff : arena + off;
        (sb ? soff : off) += (size_t)pb * kt * chunk;
        if (one) regions.push_back(Region{p.B, p.ldb, 1.0, opB != OP_T, sb, nv, pb, p.k, kt, b});
      }
      // op(A)[i][k] = TA ? A[k][i] : A[i][k];  op(B)^T[j][k] = TB ? B[j][k] : B[k][j]
      const int za = cplx ? 1 : 0, zb = cplx ? 2 : 0;
      if (a_new) {
        job(p.A, a, p.lda, p.alpha, opA == OP_T, p.m, f * p.k, 0, kt, pa, za, opA, sa);
        job(p.A2, a, p.lda2, p.alpha2, opA == OP_T, p.m, f * p.k2, kt1, kt, pa, za, opA, sa);
      }
      if (b_new) {
        job(p.B, b, p.ldb, 1.0, opB != OP_T, nv, f * p.k, 0, kt, pb, zb, opB, sb);
        job(p.B2, b, p.ldb2, 1.0, opB != OP_T, nv, f * p.k2, kt1, kt, pb, zb, opB, sb);
      }
      SplitProb sp;
      sp.A = a;
      sp.B = b;
      sp.D = p.D;
      sp.C = p.C;
      sp.ldc = f * p.ldc;
      sp.ldd = f * p.ldd;
      sp.beta = p.beta;
      sp.m = p.m;
      sp.n = nv;
      sp.ktiles = kt;
      sp.tiles_m = ceil_div(p.m, PK_R * tpm);
      sp.tiles_n = ceil_div(nv, PK_R * tpn);
      sp.begin = q.tiles;
      q.tiles += sp.tiles_m * sp.tiles_n;
      q.tile_prob.resize(q.tiles, (int32_t)q.probs.size());
      q.probs.push_back(sp);
    }
    append_tile_order(q.tile_prob, q.tiles);
  }
  // the fixed rule when no timing is wanted: 128 x 128 packed tiles when every
  // problem fills them and its K is long enough to amortize the pack
  int variant_by_size() const {
    for (const GemmProb& p : probs)
      if (p.m < 128 || p.n < 128 || p.k + std::max(p.k2, 0) < 256) return cplx ? V_P11 : V_TILE64;
    return V_P22;
  }
  const char* variant_name() const {
    static const char* real[V_COUNT] = {"tile64", "packed64", "packed128x64", "packed64x128", "packed128"};
    static const char* f64[V_COUNT] = {"fp64_tile64", "fp64_packed64", "fp64_packed128x64", "fp64_packed64x128",
                                       "fp64_packed128"};
    static const char* zx6[V_COUNT] = {"", "zx6_packed64", "zx6_packed128x64", "zx6_packed64x128", "zx6_packed128"};
    if (cplx) return prec == GP_BF16X6 ? zx6[variant] : "zgemm64";
    return prec == GP_FP64 ? f64[variant] : real[variant];
  }
  // the static operand panels of the chosen variant (after a reference change)
  void pack_static(hipStream_t s) const {
    if (!has_static || variant == V_TILE64) return;
    const PackPlan& q = pk[variant - 1];
    if (prec == GP_FP64)
      launch_copy_pack64(q.d_sjobs, q.d_schunk_job, q.schunks, s);
    else
      launch_split_pack(q.d_sjobs, q.d_schunk_job, q.schunks, s);
  }
  void launch(hipStream_t s) const {
    if (probs.empty()) return;
    if (variant != V_TILE64) {
      const PackPlan& q = pk[variant - 1];
      if (prec == GP_FP64) {
        launch_copy_pack64(q.d_jobs, q.d_chunk_job, q.chunks, s);
        launch_gemm_f64_packed(kVarTpm[variant], kVarTpn[variant], q.d_probs, q.d_tile_prob, q.tiles, s);
      } else {
        launch_split_pack(q.d_jobs, q.d_chunk_job, q.chunks, s);
        launch_gemm_x6_packed(kVarTpm[variant], kVarTpn[variant], q.d_probs, q.d_tile_prob, q.tiles, s);
      }
    } else if (cplx) {
      launch_zgemm(d, d_tile_prob, tiles, opA, opB, s);
    } else {
      launch_gemm(d, d_tile_prob, tiles, opA, opB, prec, s);
    }
  }
};

GemmProb prob(int m, int n, int k, const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
              int64_t ldc, double alpha = 1.0) {
  GemmProb p;
  std::memset(&p, 0, sizeof(p));
  p.m = m;
  p.n = n;
  p.k = k;
  p.A = A;
  p.lda = lda;
  p.B = B;
  p.ldb = ldb;
  p.C = C;
  p.ldc = ldc;
  p.alpha = alpha;
  p.alpha2 = 1.0;
  return p;
}

GemmProb with_second(GemmProb p, int k2, const double* A2, int64_t lda2, const double* B2, int64_t ldb2,
                     double alpha2) {
  p.k2 = k2;
  p.A2 = A2;
  p.lda2 = lda2;
  p.B2 = B2;
  p.ldb2 = ldb2;
  p.alpha2 = alpha2;
  return p;
}

GemmProb with_addend(GemmProb p, const double* D, int64_t ldd, double beta) {
  p.D = D;
  p.ldd = ldd;
  p.beta = beta;
  return p;
}

struct OvBuf {
  double *C0, *H0, *f, *B, *G, *U;
  double* eig_ws;  // workspace of the large eigensolver (N > EIGH_LDS_MAX), else null
  EighLargeState* eig_st;
  BsrMat H0_bsr;   // block-sparse H0 (h0_format = 1; then H0 is null)
  int64_t bsr_nnz; // stored entries of H0_bsr
  double *P, *X, *s, *fac, *XT, *XsnT, *tab, *Xcsw, *F3, *mu1, *mu2;
  double *V, *sincP, *CX, *CV, *Cocc, *Cvirt, *T, *d, *e, *Lov, *TCV, *LV, *Gam, *Nm, *XNm;
  double *HC0, *n0, *eps;
  double *HX, *HV;  // dense H0: (H0 C0)_o X and (H0 C0)_v V^T (HC0 is kept for the current C0)
};

struct ZBuf {
  double *wyT, *wyW;  // compact-WY factors and scratch of the tridiagonal eigensolver
  double *C0, *H0, *f, *A, *G;
  double *Hk, *V, *w, *Vp, *Ue, *C, *T, *d, *e, *L, *LV, *W1, *Y;
  double *n0, *eps;
  double *sX, *sX2, *sX4, *sX6, *sX8, *sT, *sU, *sZ;  // scaling and squaring (Eq. ss) workspace
  // its Frechet derivative (exact gradient): scaled direction, power derivatives,
  // combinations, the copies of q(X) and r(X), ping-pong R and L of the squarings
  double *sEs, *sM2, *sM4, *sM6, *sM8, *sLT, *sLV, *sLU, *sZc, *sR0, *sRa, *sLa;
  double *oVC, *oW, *oE;  // orbital-dependent term: -lam |C|^2 o C, (.)^H C, per-row |C|^4 sums
};

// Accumulated HIP-event timing of one stage of the launch sequence.
struct StageTimer {
  const char* name = "";
  double flops = 0.0, bytes = 0.0;  // algorithmic work of one launch
  int64_t launches = 0;
  double total_ms = 0.0;
  std::vector<hipEvent_t> ev0, ev1;
  std::vector<char> pending;
  int next = 0;
};

// stage indices of the two paths
enum OvStage { O_PQ, O_EIGL, O_EIGG, O_SPEC, O_VF, O_CXV, O_ROT, O_C, O_T, O_V, O_ROWS, O_ENERGY, O_LOV, O_LV,
               O_CONG, O_GAM, O_PAIR, O_XNM, O_G, O_SCAN, O_EIGP, O_EIGB, O_COUNT };
const char* kOvNames[O_COUNT] = {"gemm_P",      "eigh_lds",      "eigh_reduce", "spectral",
                                 "gemm_V_funcs", "gemm_CXV",     "eigenbasis_combine", "gemm_Cocc",
                                 "gemm_H0C",    "gemm_TC",       "rows_density_hubbard", "energy_reduce",
                                 "gemm_Lov",    "gemm_LV",       "ov_congruence", "gemm_Gam",
                                 "pair_hadamard", "gemm_XNm",    "gemm_grad",   "nonfinite_scan",
                                 "eigh_tridiag_pairs", "eigh_backtransform"};
enum ZStage { Z_IA, Z_EIG, Z_PHASE, Z_UE, Z_C, Z_T, Z_ROWS, Z_HUBN, Z_APPLY, Z_ENERGY, Z_HMO, Z_COMM, Z_LV, Z_LT,
              Z_DD, Z_W1, Z_Y, Z_GRAD, Z_SS_SCALE, Z_SS_PADE, Z_SS_SOLVE, Z_SS_SQUARE, Z_SS_FRECHET, Z_ODD, Z_COUNT };
const char* kZNames[Z_COUNT] = {"z_build_iA", "z_eigh",   "z_phase",  "zgemm_expA", "zgemm_C",   "zgemm_H0C",
                                "z_rows",     "z_hub_n",  "z_hub_apply", "z_energy", "zgemm_HMO", "z_commutator",
                                "zgemm_LV",   "zgemm_VhLV", "z_divdiff", "zgemm_W1",  "zgemm_Y",   "z_grad",
                                "ss_scaling", "ss_pade",  "ss_solve", "ss_square", "ss_frechet",
                                "z_orbital_term"};

}  // namespace

struct etdm_handle {
  int n_inst = 0, kind = 0, prec = 0, couple = 0, h0_format = 0;
  double U = 0.0;
  std::vector<int> M, N;
  std::vector<double> w, focc;
  std::vector<int64_t> par_off;  // parameter offsets (doubles) of each instance
  int64_t n_param = 0, n_U = 0;
  char* base = nullptr;
  size_t bytes = 0;
  std::vector<OvBuf> ov;
  std::vector<ZBuf> zb;
  double *par_ws = nullptr, *grad_ws = nullptr, *U_ws = nullptr, *E_ws = nullptr, *nvec = nullptr;
  int* status = nullptr;
  double *gl_t = nullptr, *gl_w = nullptr;
  // device descriptor arrays (allocated separately)
  std::vector<void*> dev_allocs;
  int *b_spec = nullptr, *b_rows = nullptr, *b_pair = nullptr, *b_mat = nullptr, *b_rot = nullptr;
  int tot_spec = 0, tot_rows = 0, tot_pair = 0, tot_mat = 0, tot_rot = 0;
  int n_pair = 0;  // entries of d_pair / b_pair: the instances whose gradient chain runs as GEMMs
  OvSpec* d_spec = nullptr;
  OvRot* d_rot = nullptr;
  OvRows* d_rows = nullptr;
  OvEnergy* d_energy = nullptr;
  OvPair* d_pair = nullptr;
  OvCong* d_cong = nullptr;  // gradient chain of the small instances, one workgroup each
  int n_cong = 0;
  ZInst* d_z = nullptr;
  EighProb *d_eig_lds = nullptr, *d_eig_glb = nullptr;
  int n_eig_lds = 0, n_eig_glb = 0, eig_nmax = 1;
  // complex path: tridiagonal solver (M <= HT_MAX), its checks and back-transform
  EighProb* d_eig_herm = nullptr;
  HermCheck* d_hchk = nullptr;
  RealToComplex* d_r2c = nullptr;
  HermWY* d_hwy = nullptr;
  int n_eig_herm = 0, herm_nmax = 1, herm_nblk = 0;
  int* herm_ok = nullptr;
  Stage z_HG, z_HNS;
  // real large path: tridiagonal solver part 2
  Stage s_LG, s_LNS, s_LR, s_LGram;
  std::vector<Stage> s_LWY1, s_LWY2, s_LWY3;
  int cu_count = 1;
  std::string arch;  // device architecture name (tuning cache key)
  std::vector<Stage> z_WY1, z_WY2, z_WY3;  // per block of reflectors: W1 = Y^H V, W2 = T W1, V -= Y W2
  std::vector<EighLarge> eig_large;  // real problems above the LDS size
  const double** d_n0ptr = nullptr;
  double* d_wts = nullptr;
  // preconditioner set-up of the whole batch (per-instance table, element offsets of
  // the free variables), and the ov reference update C0 <- [C_occ | C_virt]
  PrecInst* d_prec = nullptr;
  int* b_prec = nullptr;
  int tot_prec = 0;
  C0Inst* d_c0up = nullptr;
  // grouped GEMM launches
  Stage s_PQ, s_VF, s_CXV, s_C, s_TC, s_Lov, s_LV, s_Gam, s_XNm, s_G;  // real: energy+gradient
  Stage s_V, s_F3, s_Uov, s_Uvv, s_HC0;  // real: C_virt (reference update), expm, preconditioner
  Stage z_Ue, z_C, z_T, z_HMO, z_LV, z_Lt, z_W1, z_Y, z_HC0;                   // complex
  // L-BFGS: scalars and decisions in lb_st (device); the host keeps the iteration
  // and evaluation counts and reads lb_sum (pinned) once per line-search probe
  bool lb_init = false;
  int lb_iter = 0, lb_evals = 0;
  LbParams lbp{};
  bool lbp_set = false;
  LbState* lb_st = nullptr;
  LbState* lb_sum = nullptr;
  int64_t* d_par_off = nullptr;  // n_inst + 1 parameter offsets (device)
  double *x = nullptr, *g = nullptr, *p = nullptr, *q = nullptr;
  double *hd = nullptr, *wv = nullptr, *S = nullptr, *Yv = nullptr, *partial = nullptr;
  // captured L-BFGS probes: [0] direction + probe, [1] probe, [2] steepest restart + probe;
  // with the large solver each ends at its acceptance checks and lbg_back finishes the probe
  hipGraph_t lbg[3] = {nullptr, nullptr, nullptr};
  hipGraphExec_t lbg_exec[3] = {nullptr, nullptr, nullptr};
  hipGraph_t lbg_back = nullptr;
  hipGraphExec_t lbg_back_exec = nullptr;
  // graph replay of the energy+gradient sequence
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph2 = nullptr;          // second part when the large solver splits the sequence
  hipGraphExec_t graph2_exec = nullptr;
  int* ok_host = nullptr;               // pinned: acceptance flags of the large instances
  // packed operands of the FP64 / BF16x6 stages (shared: stages run in order)
  int gemm_tuning = 0;
  int grad_approx = 0;  // 1: G ~ L^T (Eq. app_grad) instead of the exact gradient
  // exp(A) by scaling and squaring (Eq. ss) instead of the eigendecomposition
  int expm_ss = 0;
  SsInst* d_ss = nullptr;
  double* ss_norms = nullptr;
  int* ss_s_dev = nullptr;
  int* ss_s_host = nullptr;  // pinned: the batch's number of squarings
  int ss_max_m = 0;
  int ss_nb = 0;                 // panel width of the solve
  std::vector<Stage> ss_up[2];   // per panel: the rank-nb row updates of the two solves
  PadeB9 ss_b{};
  Stage ss_X2, ss_X4, ss_X68, ss_U, ss_sq0, ss_sq1;  // X6 and X8 in one launch
  // exact gradient on the ss path
  SsDeriv* d_ssd = nullptr;
  SsInst* d_ss2 = nullptr;  // second solve: [q(X) copy | right-hand side]
  const double** d_ss_q = nullptr;
  double** d_ss_qc = nullptr;
  const double** d_ss_r = nullptr;
  double** d_ss_r0 = nullptr;
  const double** d_ss_lu = nullptr;
  Stage fr_M2, fr_M4, fr_M68, fr_LU, fr_N;  // sums of two products: one launch, two K segments (M6, M8 together)
  Stage fr_sq[2];     // per parity of the squaring step: L R + R L and R R in one launch
  Stage fr_Y[2];      // Y = L_s exp(A)^H, by the parity of s
  // full density matrix output (etdm_density): workspace, the SYRK row panels (real)
  // or the complex product, and the symmetric fill / column scaling descriptors
  int want_rho = 0;
  double* rho_ws = nullptr;
  int64_t rho_doubles = 0;
  Stage s_rho, z_rho;
  SymFill* d_fill = nullptr;
  int* b_fill = nullptr;
  int tot_fill = 0;
  // P = B B^T by row panels of the upper triangle (large N): its mirror, in place
  SymFill* d_pfill = nullptr;
  int* b_pfill = nullptr;
  int tot_pfill = 0, n_pfill = 0;
  ScaleCols* d_scale = nullptr;
  int* b_scale = nullptr;
  int tot_scale = 0;
  double odd_lam = 0.0;  // orbital-dependent model term (0: off)
  int has_overlap = 0;   // created from a non-orthogonal basis (H0, C0 Lowdin-transformed)
  Stage z_odd;           // W = VC^H C
  std::vector<Stage*> timer_stage;  // per timed stage: its GEMM launch, or null
  std::vector<Stage*> tune_extra;   // further stages with a kernel choice (inside a timed stage)
  std::vector<Stage*> packed_stages;  // every stage with packed variants
  std::vector<Stage*> static_stages;  // those whose chosen variant packs static operands apart
  StaticRanges static_ranges;         // C0, H0 C0 and a dense H0 of every instance
  // tracing
  std::vector<StageTimer> timers;
  int64_t tmask = 0;
  std::string err;
};

namespace {

etdm_status fail(etdm_handle* h, etdm_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

#define HIPCHK(h, call)                                                               \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(h, ETDM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CHECK(call)                          \
  do {                                       \
    etdm_status st_ = (call);                \
    if (st_ != ETDM_OK) return st_;          \
  } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int TIMER_RING = 64;

void timer_collect(StageTimer& t, int i) {
  if (!t.pending[i]) return;
  float ms = 0.f;
  (void)hipEventSynchronize(t.ev1[i]);
  if (hipEventElapsedTime(&ms, t.ev0[i], t.ev1[i]) == hipSuccess) {
    t.total_ms += ms;
    ++t.launches;
  }
  t.pending[i] = 0;
}

// Records HIP events around one stage when the stage is selected for timing.
struct Timed {
  etdm_handle* h;
  int id;
  hipStream_t s;
  bool on;
  int slot = 0;
  Timed(etdm_handle* h_, int id_, hipStream_t s_) : h(h_), id(id_), s(s_) {
    on = id < (int)h->timers.size() && ((h->tmask >> id) & 1) && !h->timers[id].ev0.empty();
    if (!on) return;
    StageTimer& t = h->timers[id];
    slot = t.next;
    timer_collect(t, slot);
    (void)hipEventRecord(t.ev0[slot], s);
  }
  ~Timed() {
    if (!on) return;
    StageTimer& t = h->timers[id];
    (void)hipEventRecord(t.ev1[slot], s);
    t.pending[slot] = 1;
    t.next = (slot + 1) % TIMER_RING;
  }
};

double stage_flops(const Stage& st) {
  double f = 0.0;
  for (const GemmProb& p : st.probs) f += (st.cplx ? 8.0 : 2.0) * p.m * (double)p.n * (p.k + p.k2);
  return f;
}

double stage_bytes(const Stage& st) {
  const double e = st.cplx ? 16.0 : 8.0;
  double b = 0.0;
  for (const GemmProb& p : st.probs)
    b += e * ((double)p.m * (p.k + p.k2) + (double)(p.k + p.k2) * p.n + (double)p.m * p.n * (p.beta != 0.0 ? 2 : 1));
  return b;
}

struct Planner {
  char* base;
  size_t off = 0;
  double* take(int64_t n_doubles) {
    char* p = base + off;
    off += ((size_t)std::max<int64_t>(n_doubles, 1) * sizeof(double) + ALIGN - 1) / ALIGN * ALIGN;
    return reinterpret_cast<double*>(p);
  }
};

// Lay out every workspace buffer; with base == nullptr it only measures.
size_t plan_buffers(etdm_handle* h, char* base) {
  Planner pl{base};
  const bool real = h->kind == ETDM_REAL_OV;
  h->par_ws = pl.take(h->n_param);
  h->grad_ws = pl.take(h->n_param);
  h->U_ws = real ? pl.take(h->n_U) : nullptr;
  h->E_ws = pl.take(h->n_inst + 1);
  h->status = reinterpret_cast<int*>(pl.take(1));
  h->gl_t = pl.take(OV_NQ);
  h->gl_w = pl.take(OV_NQ);
  int maxM = 0;
  for (int i = 0; i < h->n_inst; ++i) maxM = std::max(maxM, h->M[i]);
  h->nvec = pl.take(maxM);
  int64_t uoff = 0;
  if (real) {
    h->ov.resize(h->n_inst);
    for (int i = 0; i < h->n_inst; ++i) {
      const int64_t M = h->M[i], N = h->N[i], Nv = M - N;
      OvBuf& b = h->ov[i];
      b.B = h->par_ws + h->par_off[i];
      b.G = h->grad_ws + h->par_off[i];
      b.U = h->U_ws + uoff;
      uoff += M * M;
      b.C0 = pl.take(M * M);
      b.H0 = h->h0_format == 0 ? pl.take(M * M) : nullptr;
      b.H0_bsr = BsrMat{nullptr, nullptr, nullptr, 0, 0};
      b.bsr_nnz = 0;
      b.f = pl.take(M);
      b.P = pl.take(N * N);
      b.X = pl.take(N * N);
      b.s = pl.take(N);
      b.fac = pl.take(3 * N);
      b.XT = pl.take(N * N);
      b.XsnT = pl.take(N * N);
      b.tab = pl.take(4 * N * OV_NQ);
      b.Xcsw = pl.take(3 * N * N);
      b.F3 = pl.take(3 * N * N);
      b.mu1 = pl.take(N * N);
      b.mu2 = pl.take(N * N);
      b.V = pl.take(N * Nv);
      b.sincP = pl.take(N * N);
      b.CX = pl.take(M * N);
      b.CV = pl.take(M * N);
      b.Cocc = pl.take(M * N);
      b.Cvirt = pl.take(M * Nv);
      b.T = pl.take(M * N);
      b.d = pl.take(M);
      b.e = pl.take(M);
      b.Lov = pl.take(N * Nv);
      b.TCV = pl.take(N * N);
      b.LV = pl.take(N * N);
      b.Gam = pl.take(N * N);
      b.Nm = pl.take(N * N);
      b.XNm = pl.take(N * N);
      // Dense H0: HC0 = H0 C0 is kept for the current reference (T = H0 C_occ is formed
      // from it); block-sparse H0: the preconditioner's H0 C0 shares the expm output
      b.HC0 = h->h0_format == 0 ? pl.take(M * M) : b.U;
      h->static_ranges.add(b.C0, (int64_t)M * M);
      if (h->h0_format == 0) {
        h->static_ranges.add(b.H0, (int64_t)M * M);
        h->static_ranges.add(b.HC0, (int64_t)M * M);
      }
      b.HX = h->h0_format == 0 ? pl.take(M * N) : nullptr;
      b.HV = h->h0_format == 0 ? pl.take(M * N) : nullptr;
      b.n0 = pl.take(M);
      b.eps = pl.take(M);
      b.eig_ws = nullptr;
      b.eig_st = nullptr;
      if (N > EIGH_LDS_MAX) {
        b.eig_ws = pl.take((int64_t)eigh_large_workspace((int)N, nullptr));
        b.eig_st = reinterpret_cast<EighLargeState*>(pl.take(8));
      }
    }
  } else {
    h->herm_ok = reinterpret_cast<int*>(pl.take(h->n_inst / 2 + 1));
    h->zb.resize(h->n_inst);
    for (int i = 0; i < h->n_inst; ++i) {
      const int64_t M = h->M[i], MM2 = 2 * M * M;
      ZBuf& b = h->zb[i];
      b.A = h->par_ws + h->par_off[i];
      b.G = h->grad_ws + h->par_off[i];
      b.C0 = pl.take(MM2);
      b.H0 = pl.take(MM2);
      h->static_ranges.add(b.C0, (int64_t)MM2);
      h->static_ranges.add(b.H0, (int64_t)MM2);
      b.f = pl.take(M);
      b.Hk = pl.take(MM2);
      b.V = pl.take(MM2);
      b.w = pl.take(M);
      b.Vp = pl.take(MM2);
      b.Ue = pl.take(MM2);
      b.C = pl.take(MM2);
      b.T = pl.take(MM2);
      b.d = pl.take(M);
      b.e = pl.take(M);
      b.L = pl.take(MM2);
      b.LV = pl.take(MM2);
      b.W1 = pl.take(MM2);
      b.Y = pl.take(MM2);
      b.n0 = pl.take(M);
      b.eps = pl.take(M);
      const int64_t nblk = M <= HT_MAX ? (M - 1 + HT_NB - 1) / HT_NB : 0;
      b.wyT = pl.take(2 * nblk * HT_NB * HT_NB);
      b.wyW = pl.take(M <= HT_MAX ? 2 * 2 * HT_NB * M : 0);
      const int64_t ssz = h->expm_ss ? MM2 : 0;
      b.sX = pl.take(ssz);
      b.sX2 = pl.take(ssz);
      b.sX4 = pl.take(ssz);
      b.sX6 = pl.take(ssz);
      b.sX8 = pl.take(ssz);
      b.sT = pl.take(ssz);
      b.sU = pl.take(ssz);
      b.sZ = pl.take(ssz);
      const int64_t fz = h->expm_ss && !h->grad_approx ? MM2 : 0;
      for (double** q : {&b.sEs, &b.sM2, &b.sM4, &b.sM6, &b.sM8, &b.sLT, &b.sLV, &b.sLU, &b.sZc, &b.sR0, &b.sRa,
                         &b.sLa})
        *q = pl.take(fz);
      const bool odd = h->odd_lam != 0.0;
      b.oVC = pl.take(odd ? MM2 : 0);
      b.oW = pl.take(odd ? MM2 : 0);
      b.oE = pl.take(odd ? M : 0);
    }
    h->ss_norms = pl.take(h->expm_ss ? (int64_t)h->n_inst * SS_NORM_TILES : 0);
    h->ss_s_dev = reinterpret_cast<int*>(pl.take(h->expm_ss ? 1 : 0));
  }
  const int64_t np = h->n_param;
  h->x = pl.take(np);
  h->g = pl.take(np);
  h->p = pl.take(np);
  h->q = pl.take(np);
  h->hd = pl.take(np);
  h->wv = pl.take(np);
  h->S = pl.take(np * LB_MMAX);
  h->Yv = pl.take(np * LB_MMAX);
  h->partial = pl.take(std::max<int64_t>(3 * LB_DOT_BLOCKS, h->n_inst));
  h->lb_st = reinterpret_cast<LbState*>(pl.take((sizeof(LbState) + 7) / 8));
  h->rho_doubles = 0;
  if (h->want_rho)
    for (int i = 0; i < h->n_inst; ++i) h->rho_doubles += (real ? 1 : 2) * (int64_t)h->M[i] * h->M[i];
  h->rho_ws = h->want_rho ? pl.take(h->rho_doubles) : nullptr;
  return pl.off;
}

template <typename T>
etdm_status upload(etdm_handle* h, T** dst, const std::vector<T>& v) {
  *dst = nullptr;
  if (v.empty()) return ETDM_OK;
  void* p = nullptr;
  HIPCHK(h, hipMalloc(&p, v.size() * sizeof(T)));
  h->dev_allocs.push_back(p);
  HIPCHK(h, hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *dst = reinterpret_cast<T*>(p);
  return ETDM_OK;
}

etdm_status upload_stage(etdm_handle* h, Stage& s) {
  CHECK(upload(h, &s.d, s.probs));
  return upload(h, &s.d_tile_prob, s.tile_prob);
}

// Packed operands for every FP64 / BF16x6 stage of the list: one arena of the largest
// stage's size (the stages of one stream run one after another, and a stage runs one
// variant at a time).  Stages that can run on different streams at the same time take
// arenas of their own (one call each).
etdm_status plan_packed_stages(etdm_handle* h, Stage* const* stages, size_t n) {
  size_t bytes = 0;
  for (size_t i = 0; i < n; ++i)
    if (stages[i]->can_pack())
      for (int v = V_P11; v < V_COUNT; ++v) bytes = std::max(bytes, stages[i]->pack_bytes(v));
  if (bytes == 0) return ETDM_OK;
  void* p = nullptr;
  HIPCHK(h, hipMalloc(&p, bytes));
  h->dev_allocs.push_back(p);
  char* arena = reinterpret_cast<char*>(p);
  for (size_t i = 0; i < n; ++i) {
    Stage& sg = *stages[i];
    if (!sg.can_pack()) continue;
    sg.arena = arena;
    h->packed_stages.push_back(&sg);
    for (int v = V_P11; v < V_COUNT; ++v) {
      sg.plan_pack(v, arena);
      PackPlan& q = sg.pk[v - 1];
      CHECK(upload(h, &q.d_jobs, q.jobs));
      CHECK(upload(h, &q.d_chunk_job, q.chunk_job));
      CHECK(upload(h, &q.d_probs, q.probs));
      CHECK(upload(h, &q.d_tile_prob, q.tile_prob));
    }
    switch (h->gemm_tuning) {
      case 2: sg.variant = V_P22; break;
      case 3: sg.variant = sg.cplx ? V_P11 : V_TILE64; break;  // complex BF16x6: packed only
      case 4: sg.variant = V_P11; break;
      case 5: sg.variant = V_P21; break;
      case 6: sg.variant = V_P12; break;
      default: sg.variant = sg.variant_by_size();
    }
  }
  return ETDM_OK;
}

// Tuning cache: the kernel choice of a stage keyed by the device (architecture
// name, compute units) and the stage signature (precision, operand ops, real or
// complex, and every problem's m, n, k, k2 and beta != 0, hashed with FNV-1a).
// Process-wide; with ETDM_TUNE_CACHE naming a file, entries are also read from it
// (once per file name) and appended to it, one line each:
//   <key> <variant> <ms of the ETDM_GEMM_VARIANTS kernels>
struct TuneEntry {
  int variant;
  float ms[V_COUNT];
};
static_assert(V_COUNT == 5, "the cache line format lists five kernel times");
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
std::string g_tune_file;  // the file already read

std::string tune_key(const etdm_handle* h, const Stage& sg) {
  uint64_t x = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int b = 0; b < 8; ++b) {
      x ^= (uint64_t)((v >> (8 * b)) & 0xff);
      x *= 1099511628211ull;
    }
  };
  mix(sg.prec);
  mix(sg.opA);
  mix(sg.opB);
  mix(sg.cplx);
  mix((int64_t)sg.probs.size());
  for (const GemmProb& p : sg.probs) {
    mix(p.m);
    mix(p.n);
    mix(p.k);
    mix(p.k2);
    mix(p.beta != 0.0);
  }
  char buf[64];
  // t2: packed variants timed with their static operands packed apart
  snprintf(buf, sizeof buf, "/%d/t2/%016llx", h->cu_count, (unsigned long long)x);
  return (h->arch.empty() ? std::string("unknown") : h->arch) + buf;
}

// with g_tune_mu held
void tune_file_load() {
  const char* path = getenv("ETDM_TUNE_CACHE");
  if (!path || !*path || g_tune_file == path) return;
  g_tune_file = path;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char key[256];
  TuneEntry e;
  while (fscanf(f, "%255s %d %f %f %f %f %f", key, &e.variant, &e.ms[0], &e.ms[1], &e.ms[2], &e.ms[3], &e.ms[4]) ==
         2 + V_COUNT)
    if (e.variant >= 0 && e.variant < V_COUNT) g_tune[key] = e;
  fclose(f);
}

void tune_file_append(const std::string& key, const TuneEntry& e) {
  const char* path = getenv("ETDM_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %.6g %.6g %.6g %.6g %.6g\n", key.c_str(), e.variant, e.ms[0], e.ms[1], e.ms[2], e.ms[3], e.ms[4]);
  fclose(f);
}

// The pack plan of packed variant v of a stage and its device copies; with sarena, the
// static operand panels go there (their jobs are not part of a launch).
etdm_status replan(etdm_handle* h, Stage& sg, int v, char* sarena) {
  sg.plan_pack(v, sg.arena, sarena ? &h->static_ranges : nullptr, sarena);
  PackPlan& q = sg.pk[v - 1];
  CHECK(upload(h, &q.d_jobs, q.jobs));
  CHECK(upload(h, &q.d_chunk_job, q.chunk_job));
  CHECK(upload(h, &q.d_probs, q.probs));
  return upload(h, &q.d_tile_prob, q.tile_prob);
}

// Plan-time choice among the kernels of an FP64 / BF16x6 stage: each runs on the
// handle's own buffers (every evaluation overwrites what they write), one warm-up
// and three timed launches, and the fastest is kept, unless the tuning cache holds
// the stage already.  A packed variant is timed as it will run: operands that change
// only with the reference orbitals packed apart (into a scratch arena here, whose
// contents do not matter for the timing), the others packed by each launch.
etdm_status tune_stages(etdm_handle* h, hipStream_t s) {
  if (h->gemm_tuning != 0) return ETDM_OK;
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  etdm_status st = ETDM_OK;
  std::vector<Stage*> all(h->timer_stage);
  all.insert(all.end(), h->tune_extra.begin(), h->tune_extra.end());
  for (Stage* sg : all) {
    if (!sg || !sg->can_pack()) continue;
    const std::string key = tune_key(h, *sg);
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      tune_file_load();
      const auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        sg->variant = it->second.variant;
        std::copy(it->second.ms, it->second.ms + V_COUNT, sg->tuned_ms);
        continue;
      }
    }
    // a complex BF16x6 stage has no grouped split kernel: its packed variants only
    const int v0 = sg->cplx ? V_P11 : V_TILE64;
    size_t sbytes = 0;
    if (!sg->no_static)
      for (int v = V_P11; v < V_COUNT; ++v) sbytes = std::max(sbytes, sg->static_bytes(v, &h->static_ranges));
    char* sarena = nullptr;
    if (sbytes > 0 && hipMalloc(reinterpret_cast<void**>(&sarena), sbytes) != hipSuccess) sarena = nullptr;
    int best = v0;
    for (int v = v0; v < V_COUNT && st == ETDM_OK; ++v) {
      if (sarena && v >= V_P11) st = replan(h, *sg, v, sarena);
      if (st != ETDM_OK) break;
      sg->variant = v;
      sg->launch(s);
      float ms = 0.f;
      if (hipEventRecord(e0, s) != hipSuccess) st = ETDM_E_HIP;
      for (int r = 0; r < 3; ++r) sg->launch(s);
      if (st == ETDM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = ETDM_E_HIP;
      sg->tuned_ms[v] = ms / 3.f;
      if (sg->tuned_ms[v] < sg->tuned_ms[best]) best = v;
    }
    if (sarena) {
      // back to the plans that pack every operand per launch (plan_static re-plans the
      // chosen variant once the static panels have their own arena)
      if (hipStreamSynchronize(s) != hipSuccess) st = ETDM_E_HIP;
      for (int v = V_P11; v < V_COUNT && st == ETDM_OK; ++v) st = replan(h, *sg, v, nullptr);
      (void)hipFree(sarena);
    }
    if (st != ETDM_OK) break;
    sg->variant = best;
    TuneEntry e;
    e.variant = best;
    std::copy(sg->tuned_ms, sg->tuned_ms + V_COUNT, e.ms);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (g_tune.emplace(key, e).second) tune_file_append(key, e);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ETDM_OK) return fail(h, st, "GEMM kernel tuning failed");
  HIPCHK(h, hipGetLastError());
  return ETDM_OK;
}

// After the kernel choice: the stages whose chosen packed variant reads operands that
// change only with the reference orbitals get those panels packed into an arena of
// their own, once per reference (pack_static), instead of on every launch.
etdm_status plan_static(etdm_handle* h) {
  for (Stage* sg : h->packed_stages) {
    if (sg->variant == V_TILE64 || sg->probs.empty() || sg->no_static) continue;
    const size_t sb = sg->static_bytes(sg->variant, &h->static_ranges);
    if (sb == 0) continue;
    void* p = nullptr;
    HIPCHK(h, hipMalloc(&p, sb));
    h->dev_allocs.push_back(p);
    sg->plan_pack(sg->variant, sg->arena, &h->static_ranges, reinterpret_cast<char*>(p));
    PackPlan& q = sg->pk[sg->variant - 1];
    CHECK(upload(h, &q.d_jobs, q.jobs));
    CHECK(upload(h, &q.d_chunk_job, q.chunk_job));
    CHECK(upload(h, &q.d_probs, q.probs));
    CHECK(upload(h, &q.d_tile_prob, q.tile_prob));
    CHECK(upload(h, &q.d_sjobs, q.sjobs));
    CHECK(upload(h, &q.d_schunk_job, q.schunk_job));
    sg->has_static = true;
    h->static_stages.push_back(sg);
  }
  return ETDM_OK;
}

void pack_static(etdm_handle* h, hipStream_t s) {
  for (const Stage* sg : h->static_stages) sg->pack_static(s);
}

// ----- plan of the real occupied-virtual path ------------------------------
// Every product after the eigendecomposition is taken in the eigenbasis of P (see
// ov.hip): V = X^T B, CX = C0_o X, CV = C0_v V^T, then the combination kernel and
// C_occ = CX' X^T, L_ov = w f (T^T C0_v + (T^T CV') V), and on the gradient side LV = L_ov V^T,
// Gam = X^T LV, XNm = X Nm, dE/dB = -2 (sinc sqrt(P) L_ov + XNm V).
etdm_status build_ov_plan(etdm_handle* h) {
  // precision by role: ep for the contractions E depends on, gp for the gradient-only
  // ones.  P = B B^T, V = X^T B and the N x N spectral products stay FP64 in every
  // mode (the eigendecomposition and every later product depend on them).  In the
  // mixed mode the energy side runs split when every instance is large enough for the
  // split's rounding of the orbitals to stay far below 1e-8 Ha per electron.
  bool all_large = h->n_inst > 0;
  for (int i = 0; i < h->n_inst; ++i) all_large = all_large && h->N[i] >= ETDM_MIXED_SPLIT_E_MIN_N;
  const int ep = h->prec == ETDM_MIXED ? (all_large ? GP_BF16X6 : GP_FP64) : h->prec;
  const int gp = h->prec == ETDM_MIXED ? GP_BF16X6 : h->prec;
  h->s_PQ.init(OP_N, OP_T, GP_FP64);
  h->s_VF.init(OP_T, OP_N, GP_FP64);
  h->s_CXV.init(OP_N, OP_T, ep);
  h->s_C.init(OP_N, OP_T, ep);
  h->s_V.init(OP_N, OP_N, gp);
  h->s_TC.init(OP_T, OP_N, gp);
  h->s_Lov.init(OP_N, OP_N, gp);
  h->s_LV.init(OP_N, OP_T, gp);
  h->s_Gam.init(OP_T, OP_N, gp);
  h->s_XNm.init(OP_N, OP_N, gp);
  h->s_G.init(OP_N, OP_N, gp);
  h->s_F3.init(OP_N, OP_T, GP_FP64);
  h->s_Uov.init(OP_N, OP_N, GP_FP64);
  h->s_Uvv.init(OP_T, OP_N, GP_FP64);
  h->s_HC0.init(OP_N, OP_N, GP_FP64);
  h->s_HC0.no_static = true;  // it forms H0 C0 from C0 right after C0 changes
  h->s_rho.init(OP_N, OP_T, ep);
  std::vector<SymFill> fill, pfill;
  std::vector<int> bfill, bpfill;
  int64_t rho_off = 0;
  std::vector<OvSpec> spec;
  std::vector<OvRot> rot;
  std::vector<OvRows> rows;
  std::vector<OvEnergy> en;
  std::vector<OvPair> pair;
  std::vector<OvCong> cong;
  std::vector<int> bspec, brot, brows, bpair;
  std::vector<EighProb> el, eg;
  for (int i = 0; i < h->n_inst; ++i) {
    const int M = h->M[i], N = h->N[i], Nv = M - N;
    const OvBuf& b = h->ov[i];
    const double* Fc = b.F3;
    const double* Fs = b.F3 + (size_t)N * N;
    const double* Wm = b.F3 + 2 * (size_t)N * N;
    // P = B B^T; for large N only the row panels of the upper triangle, mirrored after
    // the product (the eigensolvers read both triangles)
    if (N >= 512) {
      constexpr int RB = 512;
      for (int r0 = 0; r0 < N; r0 += RB)
        h->s_PQ.add(prob(std::min(RB, N - r0), N - r0, Nv, b.B + (size_t)r0 * Nv, Nv, b.B + (size_t)r0 * Nv, Nv,
                         b.P + (size_t)r0 * N + r0, N));
      pfill.push_back(SymFill{b.P, (int64_t)(b.P - reinterpret_cast<double*>(h->base)), N});
      bpfill.push_back(h->tot_pfill);
      h->tot_pfill += ceil_div(N, 32) * ceil_div(N, 32);
    } else {
      h->s_PQ.add(prob(N, N, Nv, b.B, Nv, b.B, Nv, b.P, N));
    }
    // P = X diag(s) X^T
    if (N <= EIGH_LDS_MAX) {
      el.push_back(EighProb{b.P, b.X, b.s, N, 1});
    } else {
      EighLarge e;
      std::memset(&e, 0, sizeof(e));
      e.P = b.P;
      e.X = b.X;
      e.w = b.s;
      e.n = N;
      eigh_large_layout(e, b.eig_ws, b.eig_st, h->cu_count);
      h->eig_large.push_back(e);
      // tridiagonal path, part 2: Z^T Z (into the free work matrix), its check and
      // one Newton-Schulz step into X = Z + Z (I - G) / 2, then X <- Q X in compact-WY
      // blocks
      h->s_LG.add(prob(N, N, N, e.Zw, N, e.Zw, N, e.Aw, N));
      h->s_LNS.add(with_addend(prob(N, N, N, e.Zw, N, e.Aw, N, e.X, N), e.Zw, N, 1.0));
      h->s_LR.add(prob(N, N, N, e.Ps, N, e.X, N, e.Aw, N));  // R = sym(P) X for the final check
      // X <- Q X: one fused launch when the panel fits its registers, else grouped
      // GEMMs per compact-WY block
      const int nblk = (N - 1 + TB_NBW - 1) / TB_NBW;
      const bool fused_wy = tb_apply_wy_fits(N);
      if (!fused_wy && (int)h->s_LWY1.size() < nblk) {
        h->s_LWY1.resize(nblk);
        h->s_LWY2.resize(nblk);
        h->s_LWY3.resize(nblk);
      }
      const int ldT = e.nkc * TB_NBW;
      for (int bk = 0; bk < nblk; ++bk) {
        const int k0 = bk * TB_NBW, mb = std::min(TB_NBW, N - 1 - k0), R = N - 1 - k0;
        const double* Yb = e.Vw + (size_t)(k0 + 1) * N + k0;
        h->s_LGram.add(prob(mb, mb, R, Yb, N, Yb, N, e.Gw + (size_t)bk * TB_NBW * TB_NBW, mb));
        if (fused_wy) continue;
        double* Xr = e.X + (size_t)(k0 + 1) * N;
        // W1 = Y_b^T X in K chunks of TB_KC rows (partial c at rows c mb), then
        // W2 = [T_b ... T_b] [W1_0; W1_1; ...] = T_b W1
        int nc = 0;
        for (int r0 = 0; r0 < R; r0 += TB_KC, ++nc)
          h->s_LWY1[bk].add(prob(mb, N, std::min(TB_KC, R - r0), Yb + (size_t)r0 * N, N, Xr + (size_t)r0 * N, N,
                                 e.W1 + (size_t)nc * mb * N, N));
        h->s_LWY2[bk].add(prob(mb, N, nc * mb, e.Tw + (size_t)bk * TB_NBW * ldT, ldT, e.W1, N, e.W2, N));
        GemmProb up = prob(R, N, mb, Yb, N, e.W2, N, Xr, N, -1.0);
        up.beta = 1.0;
        up.D = Xr;
        up.ldd = N;
        h->s_LWY3[bk].add(up);
      }
    }
    spec.push_back(OvSpec{b.s, b.X, b.fac, b.XT, b.XsnT, b.tab, b.Xcsw, N});
    bspec.push_back(h->tot_spec);
    h->tot_spec += ov_spectral_blocks(N);
    // V = X^T B; sinc sqrt(P) = (X diag sinc) X^T and the two quadrature products of
    // the pair integrals (tables node-major): the exact gradient only
    h->s_VF.add(prob(N, Nv, N, b.X, N, b.B, Nv, b.V, Nv));
    if (!h->grad_approx) {
      const double* tq = b.tab;
      const size_t q = (size_t)OV_NQ * N;
      h->s_VF.add(prob(N, N, N, b.XsnT, N, b.XT, N, b.sincP, N));
      h->s_VF.add(prob(N, N, OV_NQ, tq, N, tq + q, N, b.mu1, N));
      h->s_VF.add(prob(N, N, OV_NQ, tq + 2 * q, N, tq + 3 * q, N, b.mu2, N));
    }
    // CX = C0_o X (B operand X^T), CV = C0_v V^T; dense H0 also (H0 C0)_o X, (H0 C0)_v V^T
    h->s_CXV.add(prob(M, N, N, b.C0, M, b.XT, N, b.CX, N));
    h->s_CXV.add(prob(M, N, Nv, b.C0 + N, M, b.V, Nv, b.CV, N));
    if (b.H0) {
      h->s_CXV.add(prob(M, N, N, b.HC0, M, b.XT, N, b.HX, N));
      h->s_CXV.add(prob(M, N, Nv, b.HC0 + N, M, b.V, Nv, b.HV, N));
    }
    rot.push_back(OvRot{b.CX, b.CV, b.HX, b.HV, b.fac, M, N});
    brot.push_back(h->tot_rot);
    h->tot_rot += M * N;
    // C_occ = CX' X^T (dense H0: T = H0 C_occ = HX' X^T in the same launch);
    // C_virt = C0_v + CV' V is formed only for a reference update (L_ov below does
    // not need it)
    h->s_C.add(prob(M, N, N, b.CX, N, b.X, N, b.Cocc, N));
    if (b.H0) h->s_C.add(prob(M, N, N, b.HX, N, b.X, N, b.T, N));
    h->s_V.add(with_addend(prob(M, Nv, N, b.CV, N, b.V, Nv, b.Cvirt, Nv), b.C0 + N, M, 1.0));

    rows.push_back(OvRows{b.Cocc, b.T, b.d, b.e, M, N, h->focc[i]});
    brows.push_back(h->tot_rows);
    h->tot_rows += M;
    en.push_back(OvEnergy{b.d, b.e, M, h->focc[i], h->w[i]});
    // L_ov = w f_occ T^T C_virt (the weight makes this the gradient of w E) without
    // C_virt: T^T C_virt = T^T C0_v + (T^T CV') V, so T^T [C0_v | CV'] (one launch,
    // into Lov and TCV), then L_ov = w f_occ (TCV V + T^T C0_v)
    h->s_TC.add(prob(N, Nv, M, b.T, N, b.C0 + N, M, b.Lov, Nv));
    h->s_TC.add(prob(N, N, M, b.T, N, b.CV, N, b.TCV, N));
    if (h->grad_approx) {
      // G ~ L^T (Eq. app_grad): g = -2 L_ov, straight from the L_ov product
      const double a = -2.0 * h->w[i] * h->focc[i];
      h->s_Lov.add(with_addend(prob(N, Nv, N, b.TCV, N, b.V, Nv, b.G, Nv, a), b.Lov, Nv, a));
    } else {
      const double a = h->w[i] * h->focc[i];
      h->s_Lov.add(with_addend(prob(N, Nv, N, b.TCV, N, b.V, Nv, b.Lov, Nv, a), b.Lov, Nv, a));
      // LV = L_ov V^T; Gam = X^T LV, Nm = Gam o mu1 + Gam^T o mu2, XNm = X Nm: one
      // workgroup per instance where X fits the LDS, else grouped GEMMs around the
      // pair kernel
      h->s_LV.add(prob(N, N, Nv, b.Lov, Nv, b.V, Nv, b.LV, N));
      if (N <= EIGH_LDS_MAX) {
        cong.push_back(OvCong{b.s, b.X, b.LV, b.mu1, b.mu2, b.XNm, N});
      } else {
        h->s_Gam.add(prob(N, N, N, b.X, N, b.LV, N, b.Gam, N));
        pair.push_back(OvPair{b.s, b.Gam, b.mu1, b.mu2, b.Nm, N});
        bpair.push_back(h->tot_pair);
        h->tot_pair += N * N;
        h->s_XNm.add(prob(N, N, N, b.X, N, b.Nm, N, b.XNm, N));
      }
      // G = -2 (sinc sqrt(P) L_ov + XNm V)
      h->s_G.add(with_second(prob(N, Nv, N, b.sincP, N, b.Lov, Nv, b.G, Nv, -2.0), N, b.XNm, N, b.V, Nv, -2.0));
    }
    // exp(A): [cos; sinc; W](sqrt P) = Xcsw X^T, U_ov = sinc B, W B (into Lov),
    // U_vo = -B^T sinc, U_vv = I + B^T (W B)
    h->s_F3.add(prob(3 * N, N, N, b.Xcsw, N, b.X, N, b.F3, N));
    h->s_Uov.add(prob(N, Nv, N, Fs, N, b.B, Nv, b.U + N, M));
    h->s_Uov.add(prob(N, Nv, N, Wm, N, b.B, Nv, b.Lov, Nv));
    h->s_Uvv.add(prob(Nv, N, N, b.B, Nv, Fs, N, b.U + (size_t)N * M, M, -1.0));
    h->s_Uvv.add(with_addend(prob(Nv, Nv, N, b.B, Nv, b.Lov, Nv, b.U + (size_t)N * M + N, M),
                             b.U + (size_t)N * M + N, M, 1.0));
    (void)Fc;
    // preconditioner: H0 C0
    if (b.H0) h->s_HC0.add(prob(M, M, M, b.H0, M, b.C0, M, b.HC0, M));
    // density output: rho = f_occ C_occ C_occ^T by row panels of the upper triangle
    // (panel r: rows [r0, r0 + RB) against columns [r0, M)), then the symmetric fill
    if (h->want_rho) {
      constexpr int RB = 512;
      double* rho = h->rho_ws + rho_off;
      for (int r0 = 0; r0 < M; r0 += RB)
        h->s_rho.add(prob(std::min(RB, M - r0), M - r0, N, b.Cocc + (size_t)r0 * N, N, b.Cocc + (size_t)r0 * N, N,
                          rho + (size_t)r0 * M + r0, M, h->focc[i]));
      fill.push_back(SymFill{rho, rho_off, M});
      bfill.push_back(h->tot_fill);
      h->tot_fill += ceil_div(M, 32) * ceil_div(M, 32);
      rho_off += (int64_t)M * M;
    }
  }
  h->n_eig_lds = (int)el.size();
  h->n_eig_glb = (int)eg.size();
  for (const EighProb& e : eg) h->eig_nmax = std::max(h->eig_nmax, e.n);
  {
    h->timers.assign(O_COUNT, StageTimer());
    for (int i = 0; i < O_COUNT; ++i) h->timers[i].name = kOvNames[i];
    Stage* gs[O_COUNT] = {};
    gs[O_PQ] = &h->s_PQ;
    gs[O_VF] = &h->s_VF;
    gs[O_CXV] = &h->s_CXV;
    gs[O_C] = &h->s_C;
    gs[O_V] = &h->s_TC;
    gs[O_LOV] = &h->s_Lov;
    gs[O_LV] = &h->s_LV;
    gs[O_GAM] = &h->s_Gam;
    gs[O_XNM] = &h->s_XNm;
    gs[O_G] = &h->s_G;
    h->timer_stage.assign(gs, gs + O_COUNT);
    for (int i = 0; i < O_COUNT; ++i)
      if (gs[i]) {
        h->timers[i].flops = stage_flops(*gs[i]);
        h->timers[i].bytes = stage_bytes(*gs[i]);
      }
    for (const EighProb& e : el) {
      h->timers[O_EIGL].flops += 9.0 * e.n * (double)e.n * e.n;
      h->timers[O_EIGL].bytes += 16.0 * e.n * (double)e.n + 8.0 * e.n;
    }
    // the large solver in three stages: the reduction to tridiagonal form (4/3 n^3, P
    // read and T written), the eigenpairs of T (O(n^2): the vectors written), and the
    // back-transform with its checks (the GEMMs' own counts)
    for (const EighLarge& e : h->eig_large) {
      const double n = e.n;
      h->timers[O_EIGG].flops += 4.0 / 3.0 * n * n * n;
      h->timers[O_EIGG].bytes += 8.0 * n * n + 16.0 * n;
      h->timers[O_EIGP].bytes += 8.0 * n * n + 24.0 * n;
    }
    {
      std::vector<const Stage*> bt = {&h->s_LG, &h->s_LNS, &h->s_LR, &h->s_LGram};
      for (size_t bk = 0; bk < h->s_LWY1.size(); ++bk)
        for (const Stage* st : {&h->s_LWY1[bk], &h->s_LWY2[bk], &h->s_LWY3[bk]}) bt.push_back(st);
      for (const Stage* st : bt) {
        h->timers[O_EIGB].flops += stage_flops(*st);
        h->timers[O_EIGB].bytes += stage_bytes(*st);
      }
      // the fused compact-WY product: W = Y_b^T X, T_b W and X -= Y_b W2 per block; X
      // read and written once, each Y_b read once
      for (const EighLarge& e : h->eig_large) {
        if (!tb_apply_wy_fits(e.n)) continue;
        const double n = e.n;
        for (int k0 = 0; k0 < e.n - 1; k0 += TB_NBW) {
          const double R = e.n - 1 - k0, mb = std::min(TB_NBW, e.n - 1 - k0);
          h->timers[O_EIGB].flops += 4.0 * R * mb * n + mb * mb * n;
          h->timers[O_EIGB].bytes += 8.0 * R * mb;
        }
        h->timers[O_EIGB].bytes += 16.0 * n * n;
      }
    }
    for (int i = 0; i < h->n_inst; ++i) {
      const double M = h->M[i], N = h->N[i];
      const bool dense = h->h0_format == 0;
      h->timers[O_ROWS].flops += 6.0 * M * N;
      if (h->h0_format == 1) {
        h->timers[O_T].flops += 2.0 * (double)h->ov[i].bsr_nnz * N;
        h->timers[O_T].bytes += 8.0 * ((double)h->ov[i].bsr_nnz + 2.0 * M * N);
      }
      h->timers[O_ROWS].bytes += 8.0 * (3.0 * M * N + 2.0 * M);
      // X read; X^T, (X diag sinc)^T, the four node-major tables and the factors written
      h->timers[O_SPEC].bytes += 8.0 * (3.0 * N * N + 4.0 * N * OV_NQ + 4.0 * N);
      // CX, CV (and HX, HV) read and written
      h->timers[O_ROT].flops += (dense ? 6.0 : 4.0) * M * N;
      h->timers[O_ROT].bytes += 8.0 * (dense ? 7.0 : 4.0) * M * N;
      if (!h->grad_approx && N <= EIGH_LDS_MAX) {  // two N^3 products; X LV mu1 mu2 in, XNm out
        h->timers[O_CONG].flops += 4.0 * N * N * N + 3.0 * N * N;
        h->timers[O_CONG].bytes += 8.0 * 5.0 * N * N;
      } else {
        h->timers[O_PAIR].flops += 3.0 * N * N;
        h->timers[O_PAIR].bytes += 8.0 * 4.0 * N * N;
      }
      h->timers[O_ENERGY].bytes += 16.0 * M;
    }
    h->timers[O_SCAN].bytes = 8.0 * h->n_param;
  }
  Stage* stages[] = {&h->s_PQ, &h->s_VF, &h->s_CXV, &h->s_C,   &h->s_TC,  &h->s_Lov, &h->s_LV, &h->s_Gam,
                     &h->s_XNm, &h->s_G, &h->s_V,   &h->s_F3, &h->s_Uov, &h->s_Uvv, &h->s_HC0, &h->s_rho};
  for (Stage* sg : stages) CHECK(upload_stage(h, *sg));
  std::vector<Stage*> packable(stages, stages + sizeof(stages) / sizeof(stages[0]));
  if (!h->eig_large.empty()) {
    h->s_LG.init(OP_T, OP_N, GP_FP64);
    // the Newton-Schulz correction Z (I - G) / 2 is of the order of the orthogonality
    // error (at most 1e-6 when accepted), so a split product's relative error of 1e-7
    // on it stays below FP64 rounding of X: split outside the FP64 mode
    h->s_LNS.init(OP_N, OP_N, h->prec == ETDM_FP64 ? GP_FP64 : GP_BF16X6);
    h->s_LR.init(OP_N, OP_N, GP_FP64);
    h->s_LGram.init(OP_T, OP_N, GP_FP64);
    CHECK(upload_stage(h, h->s_LGram));
    CHECK(upload_stage(h, h->s_LG));
    CHECK(upload_stage(h, h->s_LNS));
    CHECK(upload_stage(h, h->s_LR));
    // the three N^3 products of the checks and the Gram matrices also get the
    // kernel choice (the compact-WY blocks keep the grouped kernel: small m)
    h->tune_extra = {&h->s_LG, &h->s_LNS, &h->s_LR, &h->s_LGram};
    packable.insert(packable.end(), h->tune_extra.begin(), h->tune_extra.end());
    for (size_t bk = 0; bk < h->s_LWY1.size(); ++bk) {
      h->s_LWY1[bk].init(OP_T, OP_N, GP_FP64);
      h->s_LWY2[bk].init(OP_N, OP_N, GP_FP64);
      h->s_LWY3[bk].init(OP_N, OP_N, GP_FP64);
      CHECK(upload_stage(h, h->s_LWY1[bk]));
      CHECK(upload_stage(h, h->s_LWY2[bk]));
      CHECK(upload_stage(h, h->s_LWY3[bk]));
    }
  }
  CHECK(plan_packed_stages(h, packable.data(), packable.size()));
  CHECK(upload(h, &h->d_spec, spec));
  CHECK(upload(h, &h->b_spec, bspec));
  CHECK(upload(h, &h->d_rot, rot));
  CHECK(upload(h, &h->b_rot, brot));
  CHECK(upload(h, &h->d_fill, fill));
  CHECK(upload(h, &h->b_fill, bfill));
  CHECK(upload(h, &h->d_pfill, pfill));
  h->n_pfill = (int)pfill.size();
  CHECK(upload(h, &h->b_pfill, bpfill));
  CHECK(upload(h, &h->d_rows, rows));
  CHECK(upload(h, &h->b_rows, brows));
  {
    // preconditioner set-up and reference update of the whole batch
    std::vector<PrecInst> pi;
    std::vector<C0Inst> ci;
    std::vector<int> bprec, bmm;
    for (int i = 0; i < h->n_inst; ++i) {
      const int M = h->M[i], N = h->N[i];
      const OvBuf& b = h->ov[i];
      pi.push_back(PrecInst{b.C0, b.HC0, b.f, b.n0, b.n0, b.eps, h->hd + h->par_off[i], h->wv + h->par_off[i], M, N,
                            h->w[i]});
      ci.push_back(C0Inst{b.C0, b.Cocc, b.Cvirt, M, N});
      bprec.push_back(h->tot_prec);
      h->tot_prec += N * (M - N);
      bmm.push_back(h->tot_mat);
      h->tot_mat += M * M;
    }
    CHECK(upload(h, &h->d_prec, pi));
    CHECK(upload(h, &h->b_prec, bprec));
    CHECK(upload(h, &h->d_c0up, ci));
    CHECK(upload(h, &h->b_mat, bmm));
  }
  CHECK(upload(h, &h->d_energy, en));
  CHECK(upload(h, &h->d_pair, pair));
  h->n_pair = (int)pair.size();
  CHECK(upload(h, &h->d_cong, cong));
  h->n_cong = (int)cong.size();
  CHECK(upload(h, &h->b_pair, bpair));
  CHECK(upload(h, &h->d_eig_lds, el));
  CHECK(upload(h, &h->d_eig_glb, eg));
  return ETDM_OK;
}

// ----- plan of the complex full path -----------------------------------------
etdm_status build_z_plan(etdm_handle* h) {
  std::vector<ZInst> zi;
  std::vector<int> bmat, brows;
  std::vector<EighProb> eg, eh;
  std::vector<HermCheck> hchk;
  std::vector<RealToComplex> r2c;
  std::vector<HermWY> hwy;
  std::vector<const double*> n0ptr;
  h->z_HG.init(OP_T, OP_N, GP_FP64, false);
  h->z_HNS.init(OP_N, OP_N, GP_FP64, false);
  // precision by role, as on the real path: the gradient-only products (L V, V^H L V,
  // the divided-difference product and Y) split in the mixed mode; the ones E depends
  // on (exp(A), C, H0 C, H_MO) when every k-point has M >= ETDM_MIXED_SPLIT_E_MIN_N
  bool all_large = h->n_inst > 0;
  for (int i = 0; i < h->n_inst; ++i) all_large = all_large && h->M[i] >= ETDM_MIXED_SPLIT_E_MIN_N;
  const int zep = h->prec == ETDM_BF16X6 || (h->prec == ETDM_MIXED && all_large) ? GP_BF16X6 : GP_FP64;
  const int zgp = h->prec == ETDM_BF16X6 || h->prec == ETDM_MIXED ? GP_BF16X6 : GP_FP64;
  h->z_Ue.init(OP_N, OP_C, zep, true);
  h->z_C.init(OP_N, OP_N, zep, true);
  h->z_T.init(OP_N, OP_N, zep, true);
  h->z_HMO.init(OP_C, OP_N, zep, true);
  h->z_LV.init(OP_N, OP_N, zgp, true);
  h->z_Lt.init(OP_C, OP_N, zgp, true);
  h->z_W1.init(OP_N, OP_C, zgp, true);
  h->z_Y.init(OP_N, OP_N, zgp, true);
  h->z_HC0.init(OP_N, OP_N, GP_FP64, true);
  h->z_HC0.no_static = true;  // it forms H0 C0 from C0 right after C0 changes
  h->z_odd.init(OP_C, OP_N, GP_FP64, true);
  h->z_rho.init(OP_N, OP_C, GP_FP64, true);
  std::vector<ScaleCols> scale;
  std::vector<SymFill> fill;
  std::vector<int> bscale, bfill;
  int64_t rho_off = 0;
  for (Stage* st : {&h->ss_X2, &h->ss_X4, &h->ss_X68, &h->ss_U, &h->ss_sq0, &h->ss_sq1})
    st->init(OP_N, OP_N, GP_FP64, true);
  const bool ss_exact = h->expm_ss && !h->grad_approx;
  std::vector<Stage*> fr_all = {&h->fr_M2, &h->fr_M4, &h->fr_M68, &h->fr_LU, &h->fr_N, &h->fr_sq[0], &h->fr_sq[1]};
  for (Stage* st : fr_all) st->init(OP_N, OP_N, GP_FP64, true);
  h->fr_Y[0].init(OP_N, OP_C, GP_FP64, true);
  h->fr_Y[1].init(OP_N, OP_C, GP_FP64, true);
  std::vector<SsInst> ss, ss2;
  std::vector<SsDeriv> ssd;
  std::vector<const double*> ss_q, ss_r, ss_lu;
  std::vector<double*> ss_qc, ss_r0;
  for (int i = 0; i < h->n_inst; ++i) {
    const int M = h->M[i];
    const ZBuf& b = h->zb[i];
    ZInst z;
    std::memset(&z, 0, sizeof(z));
    z.A = b.A;
    z.Hk = b.Hk;
    z.V = b.V;
    z.w = b.w;
    z.Vp = b.Vp;
    z.C = b.C;
    z.T = b.T;
    z.d = b.d;
    z.e = b.e;
    z.n = h->couple ? h->nvec : b.d;
    z.L = b.L;
    z.G = b.G;
    z.Y = h->grad_approx ? b.L : b.Y;  // G ~ L^T: the gradient kernel reads L itself
    z.f = b.f;
    z.M = M;
    z.weight = h->w[i];
    if (h->odd_lam != 0.0) {
      z.VC = b.oVC;
      z.W = b.oW;
      z.eodd = b.oE;
      z.lam = h->odd_lam;
      h->z_odd.add(prob(M, M, M, b.oVC, M, b.C, M, b.oW, M));  // W[m][k] = <m|V^m|k>
    }
    zi.push_back(z);
    bmat.push_back(h->tot_mat);
    h->tot_mat += M * M;
    if (h->want_rho) {
      // rho_k = (C diag f) C^H: the scaled copy in W1 (free outside the gradient)
      scale.push_back(ScaleCols{b.C, b.f, b.W1, M});
      bscale.push_back(h->tot_scale);
      h->tot_scale += M * M;
      h->z_rho.add(prob(M, M, M, b.W1, M, b.C, M, h->rho_ws + rho_off, M));
      fill.push_back(SymFill{h->rho_ws + rho_off, rho_off, M});
      bfill.push_back(h->tot_fill);
      h->tot_fill += ceil_div(M, 32) * ceil_div(M, 32);
      rho_off += 2 * (int64_t)M * M;
    }
    brows.push_back(h->tot_rows);
    h->tot_rows += M;
    if (M <= HT_MAX) {
      // tridiagonal solver: reflectors in Ue, Z (real) in V, G and the Newton-Schulz
      // factor in C, Z (3 I - G) / 2 in the second half of C, its complex copy in V,
      // then V <- Q_b V for the blocks of reflectors, last block first
      eh.push_back(EighProb{b.Hk, b.V, b.w, M, 0, b.Ue, h->herm_ok + i});
      hchk.push_back(HermCheck{b.C, h->herm_ok + i, M});
      r2c.push_back(RealToComplex{b.C + (size_t)M * M, b.V, M});
      hwy.push_back(HermWY{b.Ue, b.wyT, M});
      h->z_HG.add(prob(M, M, M, b.V, M, b.V, M, b.C, M));
      h->z_HNS.add(prob(M, M, M, b.V, M, b.C, M, b.C + (size_t)M * M, M));
      h->herm_nmax = std::max(h->herm_nmax, M);
      const int nblk = (M - 1 + HT_NB - 1) / HT_NB;
      h->herm_nblk = std::max(h->herm_nblk, nblk);
      if ((int)h->z_WY1.size() < nblk) {
        h->z_WY1.resize(nblk);
        h->z_WY2.resize(nblk);
        h->z_WY3.resize(nblk);
      }
      double* W1 = b.wyW;
      double* W2 = b.wyW + 2 * (size_t)HT_NB * M;
      for (int bk = 0; bk < nblk; ++bk) {
        const int k0 = bk * HT_NB, mb = std::min(HT_NB, M - 1 - k0), R = M - 1 - k0;
        const double* Yb = b.Ue + 2 * ((size_t)(k0 + 1) * M + k0);  // rows k0+1.., columns k0..
        double* Vr = b.V + 2 * (size_t)(k0 + 1) * M;                 // rows k0+1..
        h->z_WY1[bk].add(prob(mb, M, R, Yb, M, Vr, M, W1, M));
        h->z_WY2[bk].add(prob(mb, M, mb, b.wyT + 2 * (size_t)bk * HT_NB * HT_NB, HT_NB, W1, M, W2, M));
        GemmProb up = prob(R, M, mb, Yb, M, W2, M, Vr, M, -1.0);
        up.beta = 1.0;
        up.D = Vr;
        up.ldd = M;
        h->z_WY3[bk].add(up);
      }
    }
    // the Jacobi sweeps take the matrices the tridiagonal solver did not accept
    eg.push_back(EighProb{b.Hk, b.V, b.w, M, 0, nullptr, M <= HT_MAX ? h->herm_ok + i : nullptr});
    n0ptr.push_back(b.n0);
    h->z_Ue.add(prob(M, M, M, b.Vp, M, b.V, M, b.Ue, M));    // exp(A) = (V e^{-iw}) V^H
    h->z_C.add(prob(M, M, M, b.C0, M, b.Ue, M, b.C, M));     // C = C0 exp(A)
    h->z_T.add(prob(M, M, M, b.H0, M, b.C, M, b.T, M));      // H0 C
    h->z_HMO.add(prob(M, M, M, b.C, M, b.T, M, b.L, M));     // H_MO = C^H H C
    if (!h->grad_approx && !h->expm_ss) {  // Y through the eigenbasis (the exact gradient only)
      h->z_LV.add(prob(M, M, M, b.L, M, b.V, M, b.LV, M));     // L V
      h->z_Lt.add(prob(M, M, M, b.V, M, b.LV, M, b.L, M));     // V^H L V
      h->z_W1.add(prob(M, M, M, b.L, M, b.V, M, b.W1, M));     // (. o D) V^H
      h->z_Y.add(prob(M, M, M, b.V, M, b.W1, M, b.Y, M));      // Y = V (.) V^H
    }
    h->z_HC0.add(prob(M, M, M, b.H0, M, b.C0, M, b.LV, M));  // preconditioner: H0 C0 (into LV)
    if (h->expm_ss) {
      // Eq. ss: the even powers, U = X T, the squarings (ping-pong between Ue and X, or a
      // buffer of the derivative phase when X is still needed there)
      double* sq = ss_exact ? b.sRa : b.sX;
      ss.push_back(SsInst{b.A, b.sX, b.sX2, b.sX4, b.sX6, b.sX8, b.sT, b.sU, b.sZ, b.Ue, sq, M});
      h->ss_X2.add(prob(M, M, M, b.sX, M, b.sX, M, b.sX2, M));
      h->ss_X4.add(prob(M, M, M, b.sX2, M, b.sX2, M, b.sX4, M));
      h->ss_X68.add(prob(M, M, M, b.sX4, M, b.sX2, M, b.sX6, M));
      h->ss_X68.add(prob(M, M, M, b.sX4, M, b.sX4, M, b.sX8, M));
      h->ss_U.add(prob(M, M, M, b.sX, M, b.sT, M, b.sU, M));  // U = X (b9 X8 + ... + b1 I)
      h->ss_sq0.add(prob(M, M, M, b.Ue, M, b.Ue, M, sq, M));
      h->ss_sq1.add(prob(M, M, M, sq, M, sq, M, b.Ue, M));
      h->ss_max_m = std::max(h->ss_max_m, M);
    }
    if (ss_exact) {
      // Frechet derivative of exp at A in the direction L; Y = L_s exp(A)^H
      ss2.push_back(SsInst{b.A, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, b.sZc, b.sLV, nullptr, M});
      ssd.push_back(SsDeriv{b.L, b.sEs, b.sM2, b.sM4, b.sM6, b.sM8, b.sLT, b.sLV, M});
      ss_q.push_back(b.sZ);
      ss_qc.push_back(b.sZc);
      ss_r.push_back(b.Ue);
      ss_r0.push_back(b.sR0);
      ss_lu.push_back(b.sLU);
      auto acc = [&](GemmProb p, double* D) {  // C = A B + D (D may be C)
        p.beta = 1.0;
        p.D = D;
        p.ldd = M;
        return p;
      };
      // C = A B + A2 B2 in one launch (the second product as the second K segment)
      auto sum2 = [&](const double* A, const double* B, const double* A2, const double* B2, double* C) {
        GemmProb p = prob(M, M, M, A, M, B, M, C, M);
        p.A2 = A2;
        p.B2 = B2;
        p.lda2 = p.ldb2 = M;
        p.k2 = M;
        p.alpha2 = 1.0;
        return p;
      };
      h->fr_M2.add(sum2(b.sX, b.sEs, b.sEs, b.sX, b.sM2));
      h->fr_M4.add(sum2(b.sX2, b.sM2, b.sM2, b.sX2, b.sM4));
      h->fr_M68.add(sum2(b.sX4, b.sM2, b.sM4, b.sX2, b.sM6));
      h->fr_M68.add(sum2(b.sX4, b.sM4, b.sM4, b.sX4, b.sM8));
      h->fr_LU.add(sum2(b.sX, b.sLT, b.sEs, b.sT, b.sLU));
      // right-hand side (LU + LV) - (LV - LU) r, with LT = LV - LU and LV = LU + LV
      h->fr_N.add(acc(prob(M, M, M, b.sLT, M, b.sR0, M, b.sLV, M, -1.0), b.sLV));
      double* Rb[2] = {b.sR0, b.sRa};
      double* Lb[2] = {b.sLV, b.sLa};
      for (int k = 0; k < 2; ++k) {
        double *R = Rb[k], *L = Lb[k], *Rn = Rb[1 - k], *Ln = Lb[1 - k];
        h->fr_sq[k].add(sum2(R, L, L, R, Ln));
        h->fr_sq[k].add(prob(M, M, M, R, M, R, M, Rn, M));
        h->fr_Y[k].add(prob(M, M, M, L, M, b.Ue, M, b.Y, M));
      }
    }
  }
  if (h->expm_ss) {
    // Gauss-Jordan row updates of each panel: the rows above and below it take
    // -Z[rows, panel] (reduced panel rows) over the Z columns right of the panel and
    // over all of R, in place (C = -A B + C); no problem writes what another reads
    h->ss_nb = ss_solve_panel(h->ss_max_m);
    auto solve_updates = [&](const std::vector<SsInst>& v, std::vector<Stage>& ups) -> etdm_status {
      const int nb = h->ss_nb;
      ups.assign(ceil_div(h->ss_max_m, nb), Stage());
      for (size_t pn = 0; pn < ups.size(); ++pn) {
        Stage& st = ups[pn];
        st.init(OP_N, OP_N, GP_FP64, true);
        const int k0 = (int)pn * nb;
        for (const SsInst& z : v) {
          const int M = z.M;
          if (k0 >= M) continue;
          const int w = std::min(nb, M - k0), e = k0 + w;
          const int r0[2] = {0, e}, nr[2] = {k0, M - e};
          for (int q = 0; q < 2; ++q) {
            const double* F = z.Z + 2 * ((size_t)r0[q] * M + k0);
            double* cz = z.Z + 2 * ((size_t)r0[q] * M + e);
            double* cr = z.R + 2 * (size_t)r0[q] * M;
            GemmProb pz = prob(nr[q], M - e, w, F, M, z.Z + 2 * ((size_t)k0 * M + e), M, cz, M, -1.0);
            GemmProb pr = prob(nr[q], M, w, F, M, z.R + 2 * (size_t)k0 * M, M, cr, M, -1.0);
            pz.beta = pr.beta = 1.0;
            pz.D = cz;
            pr.D = cr;
            pz.ldd = pr.ldd = M;
            st.add(pz);
            st.add(pr);
          }
        }
        CHECK(upload_stage(h, st));
      }
      return ETDM_OK;
    };
    CHECK(solve_updates(ss, h->ss_up[0]));
    if (ss_exact) CHECK(solve_updates(ss2, h->ss_up[1]));
    CHECK(upload(h, &h->d_ss, ss));
    // numerator coefficients of the [9/9] approximant: b_0 = 1, b_{j+1} = b_j (m - j) / ((2m - j)(j + 1))
    h->ss_b.b[0] = 1.0;
    for (int j = 0; j < 9; ++j) h->ss_b.b[j + 1] = h->ss_b.b[j] * (9 - j) / ((18.0 - j) * (j + 1));
    for (Stage* st : {&h->ss_X2, &h->ss_X4, &h->ss_X68, &h->ss_U, &h->ss_sq0, &h->ss_sq1})
      CHECK(upload_stage(h, *st));
  }
  if (ss_exact) {
    CHECK(upload(h, &h->d_ss2, ss2));
    CHECK(upload(h, &h->d_ssd, ssd));
    CHECK(upload(h, &h->d_ss_q, ss_q));
    CHECK(upload(h, &h->d_ss_qc, ss_qc));
    CHECK(upload(h, &h->d_ss_r, ss_r));
    CHECK(upload(h, &h->d_ss_r0, ss_r0));
    CHECK(upload(h, &h->d_ss_lu, ss_lu));
    for (Stage* st : fr_all) CHECK(upload_stage(h, *st));
    CHECK(upload_stage(h, h->fr_Y[0]));
    CHECK(upload_stage(h, h->fr_Y[1]));
  }
  h->n_eig_glb = (int)eg.size();
  for (const EighProb& e : eg) h->eig_nmax = std::max(h->eig_nmax, e.n);
  h->n_eig_herm = (int)eh.size();
  {
    h->timers.assign(Z_COUNT, StageTimer());
    for (int i = 0; i < Z_COUNT; ++i) h->timers[i].name = kZNames[i];
    Stage* gs[Z_COUNT] = {};
    gs[Z_UE] = &h->z_Ue;
    gs[Z_C] = &h->z_C;
    gs[Z_T] = &h->z_T;
    gs[Z_HMO] = &h->z_HMO;
    gs[Z_LV] = &h->z_LV;
    gs[Z_LT] = &h->z_Lt;
    gs[Z_W1] = &h->z_W1;
    gs[Z_Y] = &h->z_Y;
    gs[Z_ODD] = &h->z_odd;
    h->timer_stage.assign(gs, gs + Z_COUNT);
    for (int i = 0; i < Z_COUNT; ++i)
      if (gs[i]) {
        h->timers[i].flops = stage_flops(*gs[i]);
        h->timers[i].bytes = stage_bytes(*gs[i]);
      }
    for (int i = 0; i < h->n_inst; ++i) {
      const double M = h->M[i];
      h->timers[Z_EIG].flops += 36.0 * M * M * M;  // complex Hermitian eigensystem (4 x the real count)
      h->timers[Z_EIG].bytes += 32.0 * M * M + 8.0 * M;
      h->timers[Z_IA].bytes += 32.0 * M * M;
      h->timers[Z_PHASE].bytes += 32.0 * M * M;
      h->timers[Z_ROWS].bytes += 32.0 * M * M;
      h->timers[Z_APPLY].bytes += 48.0 * M * M;
      h->timers[Z_COMM].bytes += 32.0 * M * M;
      h->timers[Z_DD].bytes += 32.0 * M * M;
      h->timers[Z_GRAD].bytes += 32.0 * M * M;
      if (h->expm_ss) {
        h->timers[Z_SS_SCALE].bytes += 16.0 * M * M;
        h->timers[Z_SS_SOLVE].flops += 12.0 * M * M * M;  // Gauss-Jordan on [q(X) | p(X)], complex
        h->timers[Z_SS_SOLVE].bytes += 32.0 * M * M;
      }
    }
    for (Stage* st : {&h->ss_X2, &h->ss_X4, &h->ss_X68, &h->ss_U}) {
      h->timers[Z_SS_PADE].flops += stage_flops(*st);
      h->timers[Z_SS_PADE].bytes += stage_bytes(*st);
    }
    h->timers[Z_SS_SQUARE].flops = stage_flops(h->ss_sq0);  // per squaring
    h->timers[Z_SS_SQUARE].bytes = stage_bytes(h->ss_sq0);
    // Frechet phase without its squaring steps (three products per halving on top)
    for (Stage* st : {&h->fr_M2, &h->fr_M4, &h->fr_M68, &h->fr_LU, &h->fr_N, &h->fr_Y[0]}) {
      h->timers[Z_SS_FRECHET].flops += stage_flops(*st);
      h->timers[Z_SS_FRECHET].bytes += stage_bytes(*st);
    }
    h->timers[Z_SS_FRECHET].flops += h->timers[Z_SS_SOLVE].flops;
  }
  Stage* stages[] = {&h->z_Ue, &h->z_C,   &h->z_T,  &h->z_HMO, &h->z_LV,  &h->z_Lt, &h->z_W1,
                     &h->z_Y,  &h->z_HC0, &h->z_HG, &h->z_HNS, &h->z_odd, &h->z_rho};
  for (Stage* sg : stages) CHECK(upload_stage(h, *sg));
  {
    // the split complex stages run packed (real view of the complex product)
    Stage* zs[] = {&h->z_Ue, &h->z_C, &h->z_T, &h->z_HMO, &h->z_LV, &h->z_Lt, &h->z_W1, &h->z_Y};
    CHECK(plan_packed_stages(h, zs, sizeof(zs) / sizeof(zs[0])));
  }
  CHECK(upload(h, &h->d_scale, scale));
  CHECK(upload(h, &h->b_scale, bscale));
  CHECK(upload(h, &h->d_fill, fill));
  CHECK(upload(h, &h->b_fill, bfill));
  for (int bk = 0; bk < h->herm_nblk; ++bk) {
    h->z_WY1[bk].init(OP_C, OP_N, GP_FP64, true);
    h->z_WY2[bk].init(OP_N, OP_N, GP_FP64, true);
    h->z_WY3[bk].init(OP_N, OP_N, GP_FP64, true);
    CHECK(upload_stage(h, h->z_WY1[bk]));
    CHECK(upload_stage(h, h->z_WY2[bk]));
    CHECK(upload_stage(h, h->z_WY3[bk]));
  }
  CHECK(upload(h, &h->d_z, zi));
  CHECK(upload(h, &h->b_mat, bmat));
  CHECK(upload(h, &h->b_rows, brows));
  {
    // preconditioner set-up of the whole batch (H0 C0 lands in LV)
    std::vector<PrecInst> pi;
    for (int i = 0; i < h->n_inst; ++i) {
      const ZBuf& b = h->zb[i];
      pi.push_back(PrecInst{b.C0, b.LV, b.f, b.n0, h->couple ? h->nvec : b.n0, b.eps, h->hd + h->par_off[i],
                            h->wv + h->par_off[i], h->M[i], h->N[i], h->w[i]});
    }
    h->tot_prec = h->tot_mat;
    h->b_prec = h->b_mat;
    CHECK(upload(h, &h->d_prec, pi));
  }
  CHECK(upload(h, &h->d_eig_glb, eg));
  if (!eh.empty()) {
    CHECK(upload(h, &h->d_eig_herm, eh));
    CHECK(upload(h, &h->d_hchk, hchk));
    CHECK(upload(h, &h->d_r2c, r2c));
    CHECK(upload(h, &h->d_hwy, hwy));
  }
  CHECK(upload(h, &h->d_n0ptr, n0ptr));
  CHECK(upload(h, &h->d_wts, h->w));
  return ETDM_OK;
}

void free_timers(etdm_handle* h) {
  for (StageTimer& t : h->timers) {
    for (hipEvent_t e : t.ev0) (void)hipEventDestroy(e);
    for (hipEvent_t e : t.ev1) (void)hipEventDestroy(e);
    t.ev0.clear();
    t.ev1.clear();
    t.pending.clear();
  }
}

void free_lb_graphs(etdm_handle* h) {
  for (int i = 0; i < 3; ++i) {
    if (h->lbg_exec[i]) (void)hipGraphExecDestroy(h->lbg_exec[i]);
    if (h->lbg[i]) (void)hipGraphDestroy(h->lbg[i]);
    h->lbg_exec[i] = nullptr;
    h->lbg[i] = nullptr;
  }
  if (h->lbg_back_exec) (void)hipGraphExecDestroy(h->lbg_back_exec);
  if (h->lbg_back) (void)hipGraphDestroy(h->lbg_back);
  h->lbg_back_exec = nullptr;
  h->lbg_back = nullptr;
}

void free_graph(etdm_handle* h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->graph2_exec) (void)hipGraphExecDestroy(h->graph2_exec);
  if (h->graph2) (void)hipGraphDestroy(h->graph2);
  h->graph_exec = h->graph2_exec = nullptr;
  h->graph = h->graph2 = nullptr;
  free_lb_graphs(h);
}

void free_handle(etdm_handle* h) {
  if (!h) return;
  free_graph(h);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->ok_host) (void)hipHostFree(h->ok_host);
  if (h->ss_s_host) (void)hipHostFree(h->ss_s_host);
  if (h->lb_sum) (void)hipHostFree(h->lb_sum);
  free_timers(h);
  if (h->base) (void)hipFree(h->base);
  for (void* p : h->dev_allocs) (void)hipFree(p);
  delete h;
}

// ----- launch sequences --------------------------------------------------------

#define TIMED(id) Timed timed_scope_(h, id, s)

// Exponential part, front: P, the small eigensolver and the tridiagonal path of
// the large instances up to their acceptance checks.  fallback selects what
// follows for the large instances: 0 nothing (the caller decides), 1 the Jacobi
// sweeps launched until the host sees them converge, 2 all sweeps launched (each
// returns at once when the tridiagonal result was accepted; for graph capture).
void ov_front(etdm_handle* h, hipStream_t s, int fallback) {
  {
    TIMED(O_PQ);
    h->s_PQ.launch(s);
    launch_sym_fill(h->d_pfill, h->b_pfill, h->n_pfill, h->tot_pfill, reinterpret_cast<double*>(h->base), 0, s);
  }
  { TIMED(O_EIGL); launch_eigh_real_lds(h->d_eig_lds, h->n_eig_lds, h->status, s); }
  if (!h->eig_large.empty()) {
    // reduction to tridiagonal form and its eigenpairs, the orthogonality check and
    // one Newton-Schulz step, the compact-WY back-transform, the residual against P
    {
      TIMED(O_EIGG);
      for (const EighLarge& e : h->eig_large) launch_tb_reduce(e, s);
    }
    {
      TIMED(O_EIGP);
      for (const EighLarge& e : h->eig_large) launch_tb_eigenpairs(e, s);
    }
    TIMED(O_EIGB);
    h->s_LG.launch(s);
    for (const EighLarge& e : h->eig_large) launch_tb_orth_check(e, s);
    h->s_LNS.launch(s);
    h->s_LGram.launch(s);
    for (const EighLarge& e : h->eig_large) launch_tb_wy_t(e, s);
    for (const EighLarge& e : h->eig_large) launch_tb_apply_wy(e, s);
    for (int bk = (int)h->s_LWY1.size() - 1; bk >= 0; --bk) {
      h->s_LWY1[bk].launch(s);
      h->s_LWY2[bk].launch(s);
      h->s_LWY3[bk].launch(s);
    }
    h->s_LR.launch(s);
    for (const EighLarge& e : h->eig_large) launch_tb_final_check(e, s);
    // the block Jacobi fallback, which returns at once when the tridiagonal result
    // was accepted
    if (fallback)
      for (const EighLarge& e : h->eig_large) launch_eigh_large(e, LARGE_EIGH_MAX_SWEEPS, h->status, s, fallback == 1);
  }
}

// After the eigendecomposition: the spectral factors and eigenbasis copies, then
// V = X^T B with sinc sqrt(P) and the pair-integral products (energy and gradient),
// or the matrix functions [cos; sinc; W](sqrt P) of exp(A) itself.
void ov_basis(etdm_handle* h, hipStream_t s, int want_exp) {
  {
    TIMED(O_SPEC);
    launch_ov_spectral(h->d_spec, h->b_spec, h->n_inst, h->tot_spec, h->gl_t, h->gl_w, want_exp, s);
  }
  if (want_exp) {
    h->s_F3.launch(s);
  } else {
    TIMED(O_VF);
    h->s_VF.launch(s);
  }
}

void ov_front_fallback(etdm_handle* h, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cs);
  ov_front(h, s, cs == hipStreamCaptureStatusNone ? 1 : 2);
}

// The rotated orbitals: CX = C0_o X, CV = C0_v V^T, their combination, then C_occ
// (and dense T), and C_virt when asked (a reference update).
void ov_orbitals(etdm_handle* h, hipStream_t s, bool want_cvirt) {
  { TIMED(O_CXV); h->s_CXV.launch(s); }
  { TIMED(O_ROT); launch_ov_rot(h->d_rot, h->b_rot, h->n_inst, h->tot_rot, s); }
  { TIMED(O_C); h->s_C.launch(s); }
  if (want_cvirt) h->s_V.launch(s);
}

void ov_energy_grad_rest(etdm_handle* h, hipStream_t s);

void ov_energy_grad(etdm_handle* h, hipStream_t s) {
  ov_front_fallback(h, s);
  ov_basis(h, s, 0);
  ov_energy_grad_rest(h, s);
}

// After the spectral products: C, H0 C_occ, the energy, L and the gradient.
void ov_energy_grad_rest(etdm_handle* h, hipStream_t s) {
  ov_orbitals(h, s, false);
  if (h->h0_format == 1) {
    // block-sparse H0: T = H0 C_occ here (dense H0: T was formed with C_occ)
    TIMED(O_T);
    for (int i = 0; i < h->n_inst; ++i) {
      const OvBuf& b = h->ov[i];
      launch_bsr_spmm(b.H0_bsr, b.Cocc, h->N[i], h->N[i], b.T, h->N[i], s);
    }
  }
  { TIMED(O_ROWS); launch_ov_rows(h->d_rows, h->b_rows, h->n_inst, h->tot_rows, h->U, s); }
  {
    TIMED(O_ENERGY);
    launch_ov_energy(h->d_energy, h->n_inst, h->U, h->E_ws, s);
    launch_total_energy(h->E_ws, h->n_inst, 0.0, nullptr, 0, h->U, h->status, s);
  }
  { TIMED(O_V); h->s_TC.launch(s); }
  { TIMED(O_LOV); h->s_Lov.launch(s); }
  if (!h->s_LV.probs.empty()) {
    TIMED(O_LV);
    h->s_LV.launch(s);
  }
  if (h->n_cong > 0) {
    TIMED(O_CONG);
    launch_ov_congruence(h->d_cong, h->n_cong, s);
  }
  if (!h->s_Gam.probs.empty()) {
    TIMED(O_GAM);
    h->s_Gam.launch(s);
  }
  if (h->tot_pair > 0) {
    TIMED(O_PAIR);
    launch_ov_pair(h->d_pair, h->b_pair, h->n_pair, h->tot_pair, s);
  }
  if (!h->s_XNm.probs.empty()) {
    TIMED(O_XNM);
    h->s_XNm.launch(s);
  }
  if (!h->s_G.probs.empty()) {
    TIMED(O_G);
    h->s_G.launch(s);
  }
  { TIMED(O_SCAN); launch_nonfinite_scan(h->grad_ws, h->n_param, h->status, s); }
}

void ov_expm(etdm_handle* h, hipStream_t s) {
  ov_front_fallback(h, s);
  ov_basis(h, s, 1);
  for (int i = 0; i < h->n_inst; ++i) {
    const OvBuf& b = h->ov[i];
    const int M = h->M[i], N = h->N[i];
    launch_copy_block(b.U, M, b.F3, N, N, N, 1.0, s);                    // U_oo = cos sqrt(P)
    launch_set_identity(b.U + (size_t)N * M + N, M, M - N, 1.0, s);     // U_vv = I (+ below)
  }
  h->s_Uov.launch(s);
  h->s_Uvv.launch(s);
}

void ov_new_reference(etdm_handle* h, hipStream_t s) {
  ov_front_fallback(h, s);
  ov_basis(h, s, 0);
  ov_orbitals(h, s, true);
  launch_c0_update(h->d_c0up, h->b_mat, h->n_inst, h->tot_mat, s);
  if (h->h0_format == 0) h->s_HC0.launch(s);  // H0 C0 for the new reference
  pack_static(h, s);
}

// exp(A) by scaling and squaring (Eq. ss) into Ue.  The number of squarings is the
// batch's, read by the host (one synchronization).
// R <- Z^-1 R of every instance: per panel the panel rows are reduced, then the
// other rows take the rank-nb update on the matrix cores
void ss_solve(etdm_handle* h, const SsInst* d, std::vector<Stage>& ups, hipStream_t s) {
  for (size_t pn = 0; pn < ups.size(); ++pn) {
    launch_ss_panel(d, h->n_inst, h->ss_max_m, (int)pn * h->ss_nb, h->ss_nb, s);
    ups[pn].launch(s);
  }
}

void ss_exponential(etdm_handle* h, hipStream_t s) {
  {
    TIMED(Z_SS_SCALE);
    launch_ss_scaling(h->d_ss, h->n_inst, h->ss_norms, h->ss_s_dev, s);
    (void)hipMemcpyAsync(h->ss_s_host, h->ss_s_dev, sizeof(int), hipMemcpyDeviceToHost, s);
  }
  (void)hipStreamSynchronize(s);
  const int sq = *h->ss_s_host;
  {
    TIMED(Z_SS_PADE);
    launch_ss_build(h->d_ss, h->b_mat, h->n_inst, h->tot_mat, h->ss_s_dev, s);
    h->ss_X2.launch(s);
    h->ss_X4.launch(s);
    h->ss_X68.launch(s);
    launch_ss_combine_odd(h->d_ss, h->b_mat, h->n_inst, h->tot_mat, h->ss_b, s);
    h->ss_U.launch(s);
    launch_ss_combine_even(h->d_ss, h->b_mat, h->n_inst, h->tot_mat, h->ss_b, s);
  }
  {
    TIMED(Z_SS_SOLVE);
    const bool exact = !h->grad_approx;  // keep q(X) and r(X) for the Frechet derivative
    if (exact) launch_ss_copy(h->d_ss_q, h->d_ss_qc, h->b_mat, h->n_inst, h->tot_mat, s);
    ss_solve(h, h->d_ss, h->ss_up[0], s);
    if (exact) launch_ss_copy(h->d_ss_r, h->d_ss_r0, h->b_mat, h->n_inst, h->tot_mat, s);
  }
  {
    TIMED(Z_SS_SQUARE);
    for (int k = 0; k < sq; ++k) (k % 2 == 0 ? h->ss_sq0 : h->ss_sq1).launch(s);
    if (sq % 2) launch_ss_copy_back(h->d_ss, h->b_mat, h->n_inst, h->tot_mat, s);
  }
}

void z_exponential_part(etdm_handle* h, hipStream_t s) {
  if (h->expm_ss) {
    ss_exponential(h, s);
    return;
  }
  { TIMED(Z_IA); launch_z_build_iA(h->d_z, h->b_mat, h->n_inst, h->tot_mat, s); }
  {
    TIMED(Z_EIG);
    if (h->n_eig_herm > 0) {
      // tridiagonal solver, orthogonality check of Z, one Newton-Schulz step,
      // V = Q Z in compact-WY blocks; then iA is rebuilt (the reduction consumed it) for the Jacobi
      // sweeps, which return at once on the accepted matrices
      launch_eigh_herm_tridiag(h->d_eig_herm, h->n_eig_herm, h->herm_nmax, h->status, s);
      h->z_HG.launch(s);
      launch_herm_check(h->d_hchk, h->n_eig_herm, s);
      h->z_HNS.launch(s);
      launch_real_to_complex(h->d_r2c, h->n_eig_herm, s);
      launch_herm_wy_t(h->d_hwy, h->n_eig_herm, h->herm_nblk, s);
      for (int bk = h->herm_nblk - 1; bk >= 0; --bk) {
        h->z_WY1[bk].launch(s);
        h->z_WY2[bk].launch(s);
        h->z_WY3[bk].launch(s);
      }
      launch_z_build_iA(h->d_z, h->b_mat, h->n_inst, h->tot_mat, s);
    }
    launch_eigh_complex(h->d_eig_glb, h->n_eig_glb, h->eig_nmax, h->status, s);
  }
  { TIMED(Z_PHASE); launch_z_phase(h->d_z, h->b_mat, h->n_inst, h->tot_mat, s); }
  { TIMED(Z_UE); h->z_Ue.launch(s); }
}

void z_energy_grad(etdm_handle* h, hipStream_t s) {
  z_exponential_part(h, s);
  { TIMED(Z_C); h->z_C.launch(s); }
  { TIMED(Z_T); h->z_T.launch(s); }
  { TIMED(Z_ROWS); launch_z_rows(h->d_z, h->b_rows, h->n_inst, h->tot_rows, s); }
  if (h->odd_lam != 0.0) {
    TIMED(Z_ODD);
    launch_z_odd_rows(h->d_z, h->b_rows, h->n_inst, h->tot_rows, s);
    h->z_odd.launch(s);
  }
  if (h->couple) {
    TIMED(Z_HUBN);
    launch_z_hubbard_density(h->d_z, h->n_inst, 1, h->nvec, h->M[0], s);
  }
  { TIMED(Z_APPLY); launch_z_apply_hubbard(h->d_z, h->b_rows, h->n_inst, h->tot_rows, h->U, s); }
  {
    TIMED(Z_ENERGY);
    launch_z_energy(h->d_z, h->n_inst, h->couple, h->U, h->E_ws, s);
    launch_total_energy(h->E_ws, h->n_inst, 0.0, h->couple ? h->nvec : nullptr, h->couple ? h->M[0] : 0, h->U,
                        h->status, s);
  }
  { TIMED(Z_HMO); h->z_HMO.launch(s); }
  { TIMED(Z_COMM); launch_z_commutator(h->d_z, h->b_mat, h->n_inst, h->tot_mat, s); }
  if (h->odd_lam != 0.0) {
    TIMED(Z_ODD);
    launch_z_odd_L(h->d_z, h->b_mat, h->n_inst, h->tot_mat, s);
  }
  if (h->expm_ss && !h->grad_approx) {
    // Y = L(A, L) exp(A)^H through the Frechet derivative of the scaling and squaring
    TIMED(Z_SS_FRECHET);
    const int sq = *h->ss_s_host;  // this evaluation's halvings
    launch_ss_deriv_scale(h->d_ssd, h->b_mat, h->n_inst, h->tot_mat, h->ss_s_dev, s);
    for (Stage* st : {&h->fr_M2, &h->fr_M4, &h->fr_M68}) st->launch(s);
    launch_ss_deriv_combine(h->d_ssd, h->b_mat, h->n_inst, h->tot_mat, h->ss_b, s);
    h->fr_LU.launch(s);
    launch_ss_deriv_rhs(h->d_ssd, h->d_ss_lu, h->b_mat, h->n_inst, h->tot_mat, s);
    h->fr_N.launch(s);
    ss_solve(h, h->d_ss2, h->ss_up[1], s);
    for (int k = 0; k < sq; ++k) h->fr_sq[k % 2].launch(s);
    h->fr_Y[sq % 2].launch(s);
  }
  if (!h->z_LV.probs.empty()) {
    TIMED(Z_LV);
    h->z_LV.launch(s);
  }
  if (!h->z_Lt.probs.empty()) {
    TIMED(Z_LT);
    h->z_Lt.launch(s);
  }
  if (!h->grad_approx && !h->expm_ss) {
    TIMED(Z_DD);
    launch_z_divdiff(h->d_z, h->b_mat, h->n_inst, h->tot_mat, s);
  }
  if (!h->z_W1.probs.empty()) {
    TIMED(Z_W1);
    h->z_W1.launch(s);
  }
  if (!h->z_Y.probs.empty()) {
    TIMED(Z_Y);
    h->z_Y.launch(s);
  }
  { TIMED(Z_GRAD); launch_z_grad(h->d_z, h->b_mat, h->n_inst, h->tot_mat, h->status, s); }
}

void run_energy_grad_eager(etdm_handle* h, hipStream_t s) {
  if (h->kind == ETDM_REAL_OV) ov_energy_grad(h, s);
  else z_energy_grad(h, s);
}

// Energy+gradient launch sequence, from the captured graphs when enabled.  With
// large real instances the sequence is captured in two graphs around the block
// Jacobi fallback: after the first, the host reads the acceptance flags of the
// tridiagonal path (one stream synchronization) and launches the fallback only
// for an instance that failed; a graph would replay all its sweeps.
etdm_status capture(etdm_handle* h, hipGraph_t* g, hipGraphExec_t* x, void (*seq)(etdm_handle*, hipStream_t)) {
  HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  seq(h, h->cap_stream);
  HIPCHK(h, hipStreamEndCapture(h->cap_stream, g));
  HIPCHK(h, hipGraphInstantiate(x, *g, nullptr, nullptr, 0));
  return ETDM_OK;
}

// Between the two graphs of a split sequence: read the acceptance flags of the
// large instances and run the block Jacobi fallback for those that failed.
etdm_status large_fallback(etdm_handle* h, hipStream_t s) {
  if (!h->ok_host) HIPCHK(h, hipHostMalloc(reinterpret_cast<void**>(&h->ok_host), h->eig_large.size() * sizeof(int)));
  for (size_t i = 0; i < h->eig_large.size(); ++i)
    HIPCHK(h, hipMemcpyAsync(&h->ok_host[i], h->eig_large[i].ok, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  for (size_t i = 0; i < h->eig_large.size(); ++i)
    if (!h->ok_host[i]) launch_eigh_large(h->eig_large[i], LARGE_EIGH_MAX_SWEEPS, h->status, s, true);
  return ETDM_OK;
}

bool split_sequence(const etdm_handle* h) { return h->kind == ETDM_REAL_OV && !h->eig_large.empty(); }

etdm_status run_energy_grad(etdm_handle* h, hipStream_t s) {
  if (!h->use_graph || h->tmask != 0 || h->expm_ss) {
    run_energy_grad_eager(h, s);
    return ETDM_OK;
  }
  const bool split = split_sequence(h);
  if (!h->graph_exec) {
    if (split) {
      CHECK(capture(h, &h->graph, &h->graph_exec, [](etdm_handle* hh, hipStream_t ss) { ov_front(hh, ss, 0); }));
      CHECK(capture(h, &h->graph2, &h->graph2_exec, [](etdm_handle* hh, hipStream_t ss) {
        ov_basis(hh, ss, 0);
        ov_energy_grad_rest(hh, ss);
      }));
    } else {
      CHECK(capture(h, &h->graph, &h->graph_exec, run_energy_grad_eager));
    }
  }
  HIPCHK(h, hipGraphLaunch(h->graph_exec, s));
  if (split) {
    CHECK(large_fallback(h, s));
    HIPCHK(h, hipGraphLaunch(h->graph2_exec, s));
  }
  return ETDM_OK;
}

// Read and clear the device status word.
etdm_status check_status(etdm_handle* h, hipStream_t s) {
  HIPCHK(h, hipStreamSynchronize(s));
  int st = 0;
  HIPCHK(h, hipMemcpy(&st, h->status, sizeof(int), hipMemcpyDeviceToHost));
  if (st) {
    HIPCHK(h, hipMemset(h->status, 0, sizeof(int)));
    if (st & ST_EIGH) return fail(h, ETDM_E_EIGH, "Jacobi eigensolver hit its sweep limit");
    if (st & ST_NONFINITE) return fail(h, ETDM_E_NONFINITE, "non-finite energy or gradient");
  }
  return ETDM_OK;
}

// Diagonal Hessian model of the preconditioner (Sec. 3.3) for the current
// reference orbitals: eps_i = diag(C0^H H(rho0) C0),
// h_ij = w * max(0, -2 (eps_i - eps_j)(f_i - f_j)).
void build_hdiag(etdm_handle* h, hipStream_t s) {
  const bool real = h->kind == ETDM_REAL_OV;
  if (real) {
    h->s_HC0.launch(s);
    if (h->h0_format == 1)
      for (int i = 0; i < h->n_inst; ++i)
        launch_bsr_spmm(h->ov[i].H0_bsr, h->ov[i].C0, h->M[i], h->M[i], h->ov[i].HC0, h->M[i], s);
  } else {
    h->z_HC0.launch(s);
  }
  const bool coupled = !real && h->couple;
  launch_prec_setup(h->d_prec, h->b_rows, h->tot_rows, h->b_prec, h->tot_prec, h->n_inst, real ? 0 : 1, h->U,
                    coupled ? h->d_n0ptr : nullptr, h->d_wts, h->nvec, coupled ? h->M[0] : 0, s);
}

void new_reference(etdm_handle* h, hipStream_t s) {
  if (h->kind == ETDM_REAL_OV) {
    ov_new_reference(h, s);
    return;
  }
  z_exponential_part(h, s);
  h->z_C.launch(s);
  for (int i = 0; i < h->n_inst; ++i)
    (void)hipMemcpyAsync(h->zb[i].C0, h->zb[i].C, 2 * sizeof(double) * h->M[i] * h->M[i], hipMemcpyDeviceToDevice, s);
  pack_static(h, s);
}

// ----- L-BFGS driver ---------------------------------------------------------------
//
// One probe of the line search is: [pre] evaluation at xtrial (= par_ws) [post].
// pre is the direction and the line-search start (which 0), nothing (which 1), or
// the steepest-descent restart (which 2); post is launch_lb_after_probe, which
// ends with the state copied to lb_sum.  With graphs on, each probe is one graph
// replay (two around the block Jacobi fallback of the large solver) and one
// stream synchronization.

void lb_pre(etdm_handle* h, int which, hipStream_t s) {
  const int64_t n = h->n_param;
  if (which == 0)
    launch_lb_direction(h->lb_st, h->lbp, h->x, h->g, h->p, h->q, h->S, h->Yv, h->hd, h->wv, n, h->partial,
                        h->par_ws, s);
  else if (which == 2)
    launch_lb_restart(h->lb_st, h->lbp, h->x, h->g, h->p, h->hd, h->wv, n, h->partial, h->par_ws, s);
}

void lb_post(etdm_handle* h, hipStream_t s) {
  launch_lb_after_probe(h->lb_st, h->lbp, h->x, h->g, h->p, h->grad_ws, h->E_ws + h->n_inst, h->status, h->S,
                        h->Yv, h->n_param, h->d_par_off, h->n_inst, h->partial, h->par_ws, h->lb_sum, s);
}

template <int W>
void lb_seq_whole(etdm_handle* h, hipStream_t s) {
  lb_pre(h, W, s);
  run_energy_grad_eager(h, s);
  lb_post(h, s);
}

template <int W>
void lb_seq_front(etdm_handle* h, hipStream_t s) {
  lb_pre(h, W, s);
  ov_front(h, s, 0);
}

void lb_seq_back(etdm_handle* h, hipStream_t s) {
  ov_basis(h, s, 0);
  ov_energy_grad_rest(h, s);
  lb_post(h, s);
}

// one probe: launch, wait, and read the device decision from lb_sum
etdm_status lb_probe(etdm_handle* h, int which, hipStream_t s) {
  if (!h->use_graph || h->tmask != 0 || h->expm_ss) {
    lb_pre(h, which, s);
    run_energy_grad_eager(h, s);
    lb_post(h, s);
  } else if (split_sequence(h)) {
    if (!h->lbg_exec[which]) {
      void (*seq)(etdm_handle*, hipStream_t) =
          which == 0 ? lb_seq_front<0> : which == 1 ? lb_seq_front<1> : lb_seq_front<2>;
      CHECK(capture(h, &h->lbg[which], &h->lbg_exec[which], seq));
    }
    if (!h->lbg_back_exec) CHECK(capture(h, &h->lbg_back, &h->lbg_back_exec, lb_seq_back));
    HIPCHK(h, hipGraphLaunch(h->lbg_exec[which], s));
    CHECK(large_fallback(h, s));
    HIPCHK(h, hipGraphLaunch(h->lbg_back_exec, s));
  } else {
    if (!h->lbg_exec[which]) {
      void (*seq)(etdm_handle*, hipStream_t) =
          which == 0 ? lb_seq_whole<0> : which == 1 ? lb_seq_whole<1> : lb_seq_whole<2>;
      CHECK(capture(h, &h->lbg[which], &h->lbg_exec[which], seq));
    }
    HIPCHK(h, hipGraphLaunch(h->lbg_exec[which], s));
  }
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(s));
  ++h->lb_evals;
  return ETDM_OK;
}

// Line search started by `which` (0 or 2): probes until the device accepts or
// gives up; lb_sum then holds the final state.
etdm_status lb_search(etdm_handle* h, int which, hipStream_t s) {
  CHECK(lb_probe(h, which, s));
  while (h->lb_sum->result == LR_CONT) CHECK(lb_probe(h, 1, s));
  if (h->lb_sum->result == LR_STATUS) {
    CHECK(check_status(h, s));
    return fail(h, ETDM_E_HIP, "device status word set during the line search");
  }
  return ETDM_OK;
}

// Evaluation at x, then a fresh memory (beta reset to beta0 when set_beta) and the
// preconditioner of the current reference orbitals.
etdm_status lb_start(etdm_handle* h, double beta0, int set_beta, hipStream_t s) {
  const size_t pb = (size_t)h->n_param * sizeof(double);
  if (pb) HIPCHK(h, hipMemcpyAsync(h->par_ws, h->x, pb, hipMemcpyDeviceToDevice, s));
  CHECK(run_energy_grad(h, s));
  if (pb) HIPCHK(h, hipMemcpyAsync(h->g, h->grad_ws, pb, hipMemcpyDeviceToDevice, s));
  launch_lb_start(h->lb_st, h->g, h->n_param, h->E_ws + h->n_inst, beta0, set_beta, h->lbp.m, h->partial, s);
  build_hdiag(h, s);
  HIPCHK(h, hipMemcpyAsync(h->lb_sum, h->lb_st, sizeof(LbState), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipGetLastError());
  CHECK(check_status(h, s));
  ++h->lb_evals;
  return ETDM_OK;
}

// Lowdin transform of a non-orthogonal basis (overlap S, device, dense-H0 layout):
// S^1/2 and S^-1/2 by the coupled Newton-Schulz iteration on S / c, then
// H0 <- S^-1/2 H0 S^-1/2 and C0 <- S^1/2 C0 in the instance buffers.  Creation-time
// work with its own workspace, freed before returning.
etdm_status apply_overlap(etdm_handle* h, const void* S, hipStream_t s) {
  const bool cplx = h->kind != ETDM_REAL_OV;
  const int64_t esz = cplx ? 2 : 1;  // doubles per element
  int64_t doubles = 0;
  int total = 0;
  std::vector<int> begin;
  for (int i = 0; i < h->n_inst; ++i) {
    doubles += 7 * (int64_t)h->M[i] * h->M[i] * esz + 1;
    begin.push_back(total);
    total += h->M[i] * h->M[i];
  }
  double* ws = nullptr;
  double* resid_host = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&ws), (size_t)(doubles + h->n_inst) * sizeof(double)) != hipSuccess)
    return fail(h, ETDM_E_NOMEM, "overlap workspace");
  if (hipHostMalloc(reinterpret_cast<void**>(&resid_host), h->n_inst * sizeof(double)) != hipSuccess) {
    (void)hipFree(ws);
    return fail(h, ETDM_E_NOMEM, "overlap workspace");
  }
  struct Release {  // waits for the stream, also on an early error return
    double *a, *b;
    hipStream_t s;
    ~Release() {
      (void)hipStreamSynchronize(s);
      (void)hipFree(a);
      (void)hipHostFree(b);
    }
  } release{ws, resid_host, s};
  double* resid_dev = ws + doubles;
  std::vector<OvlInst> tab[2];
  Stage prodP[2], prodY[2], prodZ[2], finW[2], finH[2], finC[2];
  for (int p = 0; p < 2; ++p)
    for (Stage* st : {&prodP[p], &prodY[p], &prodZ[p], &finW[p], &finH[p], &finC[p]})
      st->init(OP_N, OP_N, GP_FP64, cplx);
  std::vector<double*> c0s, pbuf;
  const double* Sp = static_cast<const double*>(S);
  double* cur = ws;
  for (int i = 0; i < h->n_inst; ++i) {
    const int M = h->M[i];
    const int64_t mm = (int64_t)M * M * esz;
    double *Y0 = cur, *Y1 = cur + mm, *Z0 = cur + 2 * mm, *Z1 = cur + 3 * mm, *P = cur + 4 * mm, *T = cur + 5 * mm,
           *W = cur + 6 * mm, *c = cur + 7 * mm;
    cur += 7 * mm + 1;
    double* H0 = cplx ? h->zb[i].H0 : h->ov[i].H0;
    double* C0 = cplx ? h->zb[i].C0 : h->ov[i].C0;
    tab[0].push_back(OvlInst{Sp, Y0, Z0, P, T, c, M});
    tab[1].push_back(OvlInst{Sp, Y1, Z1, P, T, c, M});
    Sp += mm;
    double* Yb[2] = {Y0, Y1};
    double* Zb[2] = {Z0, Z1};
    for (int p = 0; p < 2; ++p) {
      prodP[p].add(prob(M, M, M, Zb[p], M, Yb[p], M, P, M));          // P = Z Y
      prodY[p].add(prob(M, M, M, Yb[p], M, T, M, Yb[1 - p], M));      // Y <- Y T
      prodZ[p].add(prob(M, M, M, T, M, Zb[p], M, Zb[1 - p], M));      // Z <- T Z
      finW[p].add(prob(M, M, M, Zb[p], M, H0, M, W, M));              // S^-1/2 H0
      finH[p].add(prob(M, M, M, W, M, Zb[p], M, H0, M));              // (.) S^-1/2
      finC[p].add(prob(M, M, M, Yb[p], M, C0, M, P, M));              // S^1/2 C0, via P
    }
    c0s.push_back(C0);
    pbuf.push_back(P);
  }
  OvlInst* d_tab[2] = {nullptr, nullptr};
  int* d_begin = nullptr;
  for (int p = 0; p < 2; ++p) {
    CHECK(upload(h, &d_tab[p], tab[p]));
    for (Stage* st : {&prodP[p], &prodY[p], &prodZ[p], &finW[p], &finH[p], &finC[p]}) CHECK(upload_stage(h, *st));
  }
  CHECK(upload(h, &d_begin, begin));
  launch_ovl_start(d_tab[0], d_begin, h->n_inst, total, cplx, s);
  int p = 0;
  bool converged = false;
  for (int it = 0; it < 80 && !converged; ++it) {
    prodP[p].launch(s);
    launch_ovl_step(d_tab[p], h->n_inst, cplx, resid_dev, s);
    HIPCHK(h, hipMemcpyAsync(resid_host, resid_dev, h->n_inst * sizeof(double), hipMemcpyDeviceToHost, s));
    prodY[p].launch(s);
    prodZ[p].launch(s);
    HIPCHK(h, hipStreamSynchronize(s));
    p = 1 - p;
    double r = 0.0;
    for (int i = 0; i < h->n_inst; ++i) r = std::isfinite(resid_host[i]) ? std::max(r, resid_host[i]) : 1e300;
    if (r > 1e6) break;  // diverging: not positive definite
    converged = r <= 1e-10;
  }
  if (!converged) return fail(h, ETDM_E_ARG, "overlap not positive definite to working accuracy");
  launch_ovl_finish(d_tab[p], d_begin, h->n_inst, total, cplx, s);
  finW[p].launch(s);
  finH[p].launch(s);
  finC[p].launch(s);
  for (int i = 0; i < h->n_inst; ++i)
    HIPCHK(h, hipMemcpyAsync(c0s[i], pbuf[i], (size_t)h->M[i] * h->M[i] * esz * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(s));
  return ETDM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* etdm_status_string(etdm_status s) {
  switch (s) {
    case ETDM_OK: return "ok";
    case ETDM_E_ARG: return "invalid argument";
    case ETDM_E_SHAPE: return "inconsistent shape";
    case ETDM_E_HIP: return "HIP runtime error";
    case ETDM_E_NOMEM: return "device allocation failed";
    case ETDM_E_EIGH: return "eigensolver did not converge";
    case ETDM_E_NONFINITE: return "non-finite energy or gradient";
    case ETDM_E_LINESEARCH: return "line search failed";
    case ETDM_E_STATE: return "invalid call sequence";
  }
  return "unknown status";
}

const char* etdm_last_error(const etdm_handle* h) { return h ? h->err.c_str() : ""; }

int64_t etdm_param_count(const etdm_handle* h) { return h ? h->n_param : 0; }

void etdm_lbfgs_defaults(etdm_lbfgs_params* p) {
  if (!p) return;
  p->m = 3;
  p->c1 = 1e-4;
  p->c2 = 0.9;
  p->delta = 0.1;
  p->sigma = 0.9;
  p->eps = 1e-6;
  p->gamma = 0.25;
  p->beta0 = 1.0;
  p->reset_every = 20;
  p->max_ls = 20;
  p->reset_norm = 0.0;
}

etdm_status etdm_create(etdm_handle** out, const etdm_desc* d, const void* H0, const void* C0, const double* f,
                        void* stream) {
  if (!out) return ETDM_E_ARG;
  *out = nullptr;
  if (!d || !H0 || !C0 || !f) return ETDM_E_ARG;
  if (d->n_inst < 1 || !d->M) return ETDM_E_ARG;
  if (d->kind != ETDM_REAL_OV && d->kind != ETDM_COMPLEX_FULL) return ETDM_E_ARG;
  if (d->precision < ETDM_FP64 || d->precision > ETDM_MIXED) return ETDM_E_ARG;
  if (d->kind == ETDM_COMPLEX_FULL && d->precision != ETDM_FP64 && d->precision != ETDM_BF16X6 &&
      d->precision != ETDM_MIXED)
    return ETDM_E_ARG;
  if (d->gemm_tuning < 0 || d->gemm_tuning > 6) return ETDM_E_ARG;
  if (d->gradient != 0 && d->gradient != 1) return ETDM_E_ARG;
  if (d->expm_method != 0 && d->expm_method != 1) return ETDM_E_ARG;
  if (d->expm_method == 1 && d->kind != ETDM_COMPLEX_FULL) return ETDM_E_ARG;
  if (!std::isfinite(d->odd_lambda) || (d->odd_lambda != 0.0 && d->kind != ETDM_COMPLEX_FULL)) return ETDM_E_ARG;
  if (d->overlap && d->h0_format != 0) return ETDM_E_ARG;
  if (d->want_rho != 0 && d->want_rho != 1) return ETDM_E_ARG;
  if (d->kind == ETDM_REAL_OV && (!d->N || d->couple)) return ETDM_E_ARG;
  if (d->h0_format != 0 && d->h0_format != 1) return ETDM_E_ARG;
  if (d->h0_format == 1 && (d->kind != ETDM_REAL_OV || d->bsr_block < 1 || d->bsr_block > BSR_MAX_BS ||
                            !d->bsr_row_ptr || !d->bsr_col_idx))
    return ETDM_E_ARG;
  if (!std::isfinite(d->hubbard_U)) return ETDM_E_ARG;
  hipStream_t s = S(stream);
  etdm_handle* h = new etdm_handle();
  auto bail = [&](etdm_status st) {
    free_handle(h);
    return st;
  };
  h->n_inst = d->n_inst;
  h->kind = d->kind;
  {
    int dev = 0, cus = 1;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
      h->cu_count = std::max(1, cus);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) h->arch = prop.gcnArchName;
    for (char& c : h->arch)
      if (c == ' ') c = '_';
  }
  h->prec = d->precision;
  h->gemm_tuning = d->gemm_tuning;
  h->grad_approx = d->gradient;
  h->expm_ss = d->expm_method;
  h->odd_lam = d->odd_lambda;
  h->has_overlap = d->overlap != nullptr;
  h->want_rho = d->want_rho ? 1 : 0;
  h->U = d->hubbard_U;
  h->couple = d->couple ? 1 : 0;
  h->h0_format = d->h0_format;
  int64_t off = 0;
  for (int i = 0; i < d->n_inst; ++i) {
    const int M = d->M[i];
    const int N = d->kind == ETDM_REAL_OV ? d->N[i] : M;
    if (M < 1 || M > 32768 || N < 0 || N > M) return bail(ETDM_E_SHAPE);
    if (d->kind == ETDM_REAL_OV && N > 4096) return bail(ETDM_E_SHAPE);
    if (d->kind == ETDM_COMPLEX_FULL && M > 4000) return bail(ETDM_E_SHAPE);
    if (d->expm_method == 1 && M > SS_MAX_M) return bail(ETDM_E_SHAPE);
    if (d->h0_format == 1 && M % d->bsr_block != 0) return bail(ETDM_E_SHAPE);
    const double wi = d->weights ? d->weights[i] : 1.0;
    if (!(wi > 0.0) || !std::isfinite(wi)) return bail(ETDM_E_ARG);
    h->M.push_back(M);
    h->N.push_back(N);
    h->w.push_back(wi);
    h->par_off.push_back(off);
    off += d->kind == ETDM_REAL_OV ? (int64_t)N * (M - N) : 2 * (int64_t)M * M;
    h->n_U += (int64_t)M * M;
  }
  if (h->couple)
    for (int i = 1; i < h->n_inst; ++i)
      if (h->M[i] != h->M[0]) return bail(ETDM_E_SHAPE);
  // occupations: REAL_OV needs f_occ > 0 on the first N columns and 0 on the rest
  {
    int64_t o = 0;
    for (int i = 0; i < h->n_inst; ++i) {
      const int M = h->M[i], N = h->N[i];
      for (int j = 0; j < M; ++j)
        if (!std::isfinite(f[o + j]) || f[o + j] < 0.0) return bail(ETDM_E_ARG);
      double fo = 0.0;
      if (d->kind == ETDM_REAL_OV) {
        fo = N > 0 ? f[o] : 0.0;
        if (N > 0 && !(fo > 0.0)) return bail(ETDM_E_ARG);
        for (int j = 0; j < M; ++j)
          if (f[o + j] != (j < N ? fo : 0.0)) return bail(ETDM_E_ARG);
      }
      h->focc.push_back(fo);
      o += M;
    }
  }
  h->n_param = off;
  h->bytes = plan_buffers(h, nullptr);
  if (hipMalloc(reinterpret_cast<void**>(&h->base), h->bytes) != hipSuccess) return bail(ETDM_E_NOMEM);
  plan_buffers(h, h->base);
  if (hipMemsetAsync(h->base, 0, h->bytes, s) != hipSuccess) return bail(ETDM_E_HIP);
  {
    double t[OV_NQ], wq[OV_NQ];
    gauss_legendre01(OV_NQ, t, wq);
    if (hipMemcpyAsync(h->gl_t, t, sizeof(t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(h->gl_w, wq, sizeof(wq), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return bail(ETDM_E_HIP);
  }
  // copies of C0, H0 and f
  const bool real = d->kind == ETDM_REAL_OV;
  const size_t esz = real ? sizeof(double) : 2 * sizeof(double);
  const char* c0 = static_cast<const char*>(C0);
  const char* h0 = static_cast<const char*>(H0);
  int64_t fo = 0, row_off = 0, blk_off = 0;
  for (int i = 0; i < h->n_inst; ++i) {
    const int64_t M = h->M[i];
    double* dC0 = real ? h->ov[i].C0 : h->zb[i].C0;
    double* dH0 = real ? h->ov[i].H0 : h->zb[i].H0;
    double* df = real ? h->ov[i].f : h->zb[i].f;
    if (hipMemcpyAsync(dC0, c0, M * M * esz, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(df, f + fo, M * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
      return bail(ETDM_E_HIP);
    c0 += M * M * esz;
    fo += M;
    if (d->h0_format == 0) {
      if (hipMemcpyAsync(dH0, h0, M * M * esz, hipMemcpyDeviceToDevice, s) != hipSuccess) return bail(ETDM_E_HIP);
      h0 += M * M * esz;
      continue;
    }
    // block-sparse H0 stays block-sparse on the device: rebased row pointers,
    // column indices (validated here) and a copy of the blocks
    const int bs = d->bsr_block, nbr = (int)(M / bs);
    const int32_t* rp = d->bsr_row_ptr + row_off;
    const int nnzb = rp[nbr] - rp[0];
    if (nnzb < 0) return bail(ETDM_E_ARG);
    std::vector<int> rows(nbr + 1), cols(std::max(nnzb, 1));
    for (int r = 0; r <= nbr; ++r) {
      if (r < nbr && rp[r + 1] < rp[r]) return bail(ETDM_E_ARG);
      rows[r] = rp[r] - rp[0];
    }
    for (int p = 0; p < nnzb; ++p) {
      const int c = d->bsr_col_idx[blk_off + p];
      if (c < 0 || c >= nbr) return bail(ETDM_E_ARG);
      cols[p] = c;
    }
    int *drp = nullptr, *dci = nullptr;
    double* dblk = nullptr;
    const size_t blk_bytes = std::max<size_t>((size_t)nnzb * bs * bs, 1) * sizeof(double);
    if (hipMalloc(&drp, rows.size() * sizeof(int)) != hipSuccess) return bail(ETDM_E_NOMEM);
    h->dev_allocs.push_back(drp);
    if (hipMalloc(&dci, cols.size() * sizeof(int)) != hipSuccess) return bail(ETDM_E_NOMEM);
    h->dev_allocs.push_back(dci);
    if (hipMalloc(&dblk, blk_bytes) != hipSuccess) return bail(ETDM_E_NOMEM);
    h->dev_allocs.push_back(dblk);
    if (hipMemcpy(drp, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dci, cols.data(), cols.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpyAsync(dblk, h0, (size_t)nnzb * bs * bs * sizeof(double), hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
      return bail(ETDM_E_HIP);
    h->ov[i].H0_bsr = BsrMat{dblk, drp, dci, nbr, bs};
    h->ov[i].bsr_nnz = (int64_t)nnzb * bs * bs;
    h0 += (size_t)nnzb * bs * bs * sizeof(double);
    row_off += nbr + 1;
    blk_off += nnzb;
  }
  if (d->overlap) {
    const etdm_status so = apply_overlap(h, d->overlap, s);
    if (so != ETDM_OK) return bail(so);
  }
  etdm_status st = real ? build_ov_plan(h) : build_z_plan(h);
  if (st == ETDM_OK) {
    std::vector<int64_t> offs(h->par_off);
    offs.push_back(h->n_param);
    st = upload(h, &h->d_par_off, offs);
  }
  if (st == ETDM_OK) st = tune_stages(h, s);
  if (st == ETDM_OK && h->expm_ss &&
      hipHostMalloc(reinterpret_cast<void**>(&h->ss_s_host), sizeof(int)) != hipSuccess)
    st = ETDM_E_NOMEM;
  if (st == ETDM_OK && real && h->h0_format == 0) h->s_HC0.launch(s);  // H0 C0 of the reference
  if (st == ETDM_OK) st = plan_static(h);
  if (st == ETDM_OK) pack_static(h, s);
  if (st != ETDM_OK) return bail(st);
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) return bail(ETDM_E_HIP);
  *out = h;
  return ETDM_OK;
}

etdm_status etdm_destroy(etdm_handle* h) {
  if (!h) return ETDM_E_ARG;
  (void)hipDeviceSynchronize();
  free_handle(h);
  return ETDM_OK;
}

etdm_status etdm_energy_grad(etdm_handle* h, const void* A, double* E, void* G, void* stream) {
  if (!h) return ETDM_E_ARG;
  if ((!A || !G) && h->n_param > 0) return fail(h, ETDM_E_ARG, "null A or G");
  if (!E) return fail(h, ETDM_E_ARG, "null E");
  hipStream_t s = S(stream);
  const size_t pb = (size_t)h->n_param * sizeof(double);
  if (pb) HIPCHK(h, hipMemcpyAsync(h->par_ws, A, pb, hipMemcpyDeviceToDevice, s));
  CHECK(run_energy_grad(h, s));
  if (pb) HIPCHK(h, hipMemcpyAsync(G, h->grad_ws, pb, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(E, h->E_ws, (h->n_inst + 1) * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipGetLastError());
  return ETDM_OK;
}

etdm_status etdm_expm(etdm_handle* h, const void* A, void* U, void* stream) {
  if (!h) return ETDM_E_ARG;
  if ((!A && h->n_param > 0) || !U) return fail(h, ETDM_E_ARG, "null A or U");
  hipStream_t s = S(stream);
  const size_t pb = (size_t)h->n_param * sizeof(double);
  if (pb) HIPCHK(h, hipMemcpyAsync(h->par_ws, A, pb, hipMemcpyDeviceToDevice, s));
  if (h->kind == ETDM_REAL_OV) {
    ov_expm(h, s);
    HIPCHK(h, hipMemcpyAsync(U, h->U_ws, h->n_U * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    z_exponential_part(h, s);
    char* u = static_cast<char*>(U);
    for (int i = 0; i < h->n_inst; ++i) {
      const size_t b = 2 * sizeof(double) * h->M[i] * h->M[i];
      HIPCHK(h, hipMemcpyAsync(u, h->zb[i].Ue, b, hipMemcpyDeviceToDevice, s));
      u += b;
    }
  }
  HIPCHK(h, hipGetLastError());
  return ETDM_OK;
}

etdm_status etdm_density(etdm_handle* h, const void* A, void* rho, void* stream) {
  if (!h) return ETDM_E_ARG;
  if (!h->want_rho) return fail(h, ETDM_E_STATE, "the handle was created without want_rho");
  if ((!A && h->n_param > 0) || !rho) return fail(h, ETDM_E_ARG, "null A or rho");
  hipStream_t s = S(stream);
  const size_t pb = (size_t)h->n_param * sizeof(double);
  if (pb) HIPCHK(h, hipMemcpyAsync(h->par_ws, A, pb, hipMemcpyDeviceToDevice, s));
  if (h->kind == ETDM_REAL_OV) {
    ov_front_fallback(h, s);
    ov_basis(h, s, 0);
    ov_orbitals(h, s, false);
    h->s_rho.launch(s);
    launch_sym_fill(h->d_fill, h->b_fill, h->n_inst, h->tot_fill, static_cast<double*>(rho), 0, s);
  } else {
    z_exponential_part(h, s);
    h->z_C.launch(s);
    launch_scale_cols(h->d_scale, h->b_scale, h->n_inst, h->tot_scale, s);
    h->z_rho.launch(s);
    launch_sym_fill(h->d_fill, h->b_fill, h->n_inst, h->tot_fill, static_cast<double*>(rho), 1, s);
  }
  HIPCHK(h, hipGetLastError());
  return ETDM_OK;
}

etdm_status etdm_set_reference(etdm_handle* h, const void* A, void* stream) {
  if (!h) return ETDM_E_ARG;
  if (!A && h->n_param > 0) return fail(h, ETDM_E_ARG, "null A");
  hipStream_t s = S(stream);
  const size_t pb = (size_t)h->n_param * sizeof(double);
  if (pb) HIPCHK(h, hipMemcpyAsync(h->par_ws, A, pb, hipMemcpyDeviceToDevice, s));
  new_reference(h, s);
  HIPCHK(h, hipGetLastError());
  h->lb_init = false;
  return ETDM_OK;
}

etdm_status etdm_sync_status(etdm_handle* h, void* stream) {
  if (!h) return ETDM_E_ARG;
  return check_status(h, S(stream));
}

etdm_status etdm_set_graph(etdm_handle* h, int32_t enable) {
  if (!h) return ETDM_E_ARG;
  if (enable && !h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  if (!enable) free_graph(h);
  h->use_graph = enable != 0;
  return ETDM_OK;
}

etdm_status etdm_set_timing(etdm_handle* h, int64_t mask) {
  if (!h) return ETDM_E_ARG;
  for (size_t i = 0; i < h->timers.size(); ++i) {
    StageTimer& t = h->timers[i];
    const bool want = (mask >> i) & 1;
    if (want && t.ev0.empty()) {
      t.ev0.resize(TIMER_RING);
      t.ev1.resize(TIMER_RING);
      t.pending.assign(TIMER_RING, 0);
      for (int k = 0; k < TIMER_RING; ++k) {
        HIPCHK(h, hipEventCreate(&t.ev0[k]));
        HIPCHK(h, hipEventCreate(&t.ev1[k]));
      }
    }
  }
  h->tmask = mask;
  return ETDM_OK;
}

etdm_status etdm_reset_timing(etdm_handle* h) {
  if (!h) return ETDM_E_ARG;
  for (StageTimer& t : h->timers) {
    for (size_t k = 0; k < t.pending.size(); ++k) timer_collect(t, (int)k);
    t.total_ms = 0.0;
    t.launches = 0;
  }
  return ETDM_OK;
}

int32_t etdm_stage_count(const etdm_handle* h) { return h ? (int32_t)h->timers.size() : 0; }

etdm_status etdm_stage_info(etdm_handle* h, int32_t i, const char** name, int64_t* launches, double* total_ms,
                            double* flops, double* bytes) {
  if (!h || i < 0 || i >= (int32_t)h->timers.size()) return ETDM_E_ARG;
  StageTimer& t = h->timers[i];
  for (size_t k = 0; k < t.pending.size(); ++k) timer_collect(t, (int)k);
  if (name) *name = t.name;
  if (launches) *launches = t.launches;
  if (total_ms) *total_ms = t.total_ms;
  if (flops) *flops = t.flops;
  if (bytes) *bytes = t.bytes;
  return ETDM_OK;
}

etdm_status etdm_stage_kernel(const etdm_handle* h, int32_t i, const char** variant, double* tuned_ms) {
  if (!h || i < 0 || i >= (int32_t)h->timers.size()) return ETDM_E_ARG;
  const Stage* sg = i < (int32_t)h->timer_stage.size() ? h->timer_stage[i] : nullptr;
  if (variant) *variant = sg && !sg->probs.empty() ? sg->variant_name() : "";
  if (tuned_ms)
    for (int v = 0; v < V_COUNT; ++v) tuned_ms[v] = sg ? sg->tuned_ms[v] : 0.0;
  return ETDM_OK;
}

}  // extern "C"

// ----- L-BFGS checkpoint -----------------------------------------------------------

namespace {

constexpr size_t LB_CKPT_HEADER = 256;

struct LbCheckpoint {
  char magic[8];
  uint64_t layout;      // FNV-1a of kind, precision, gradient mode and every (M, N)
  int64_t n_param, c0_doubles;
  int32_t iter, evals, m, pad;
  LbParams lbp;
};
static_assert(sizeof(LbCheckpoint) <= LB_CKPT_HEADER, "checkpoint header too large");
const char kCkptMagic[8] = {'E', 'T', 'D', 'M', 'L', 'B', 'S', '1'};

uint64_t ckpt_layout(const etdm_handle* h) {
  uint64_t v = 1469598103934665603ull;
  auto mix = [&](int64_t x) {
    for (int b = 0; b < 8; ++b) {
      v ^= (uint64_t)((x >> (8 * b)) & 0xff);
      v *= 1099511628211ull;
    }
  };
  mix(h->kind);
  mix(h->prec);
  mix(h->grad_approx);
  mix(h->expm_ss);
  mix(h->has_overlap);
  {
    int64_t bits;
    std::memcpy(&bits, &h->odd_lam, sizeof(bits));
    mix(bits);
  }
  mix(h->n_inst);
  for (int i = 0; i < h->n_inst; ++i) {
    mix(h->M[i]);
    mix(h->N[i]);
  }
  return v;
}

int64_t c0_doubles(const etdm_handle* h, int i) {
  const int64_t MM = (int64_t)h->M[i] * h->M[i];
  return h->kind == ETDM_REAL_OV ? MM : 2 * MM;
}

double* c0_ptr(etdm_handle* h, int i) { return h->kind == ETDM_REAL_OV ? h->ov[i].C0 : h->zb[i].C0; }

size_t state_scalars_bytes() { return (sizeof(LbState) + 7) / 8 * 8; }

}  // namespace

extern "C" {

size_t etdm_lbfgs_state_bytes(const etdm_handle* h) {
  if (!h || !h->lb_init) return 0;
  int64_t c0 = 0;
  for (int i = 0; i < h->n_inst; ++i) c0 += c0_doubles(h, i);
  const int64_t n = h->n_param;
  return LB_CKPT_HEADER + state_scalars_bytes() + sizeof(double) * (size_t)(2 * n + 2 * h->lbp.m * n + c0);
}

etdm_status etdm_lbfgs_get_state(etdm_handle* h, void* state, void* stream) {
  if (!h) return ETDM_E_ARG;
  if (!h->lb_init) return fail(h, ETDM_E_ARG, "no L-BFGS state before the first etdm_lbfgs_step");
  if (!state) return fail(h, ETDM_E_ARG, "null state buffer");
  hipStream_t s = S(stream);
  LbCheckpoint hd{};
  std::memcpy(hd.magic, kCkptMagic, 8);
  hd.layout = ckpt_layout(h);
  hd.n_param = h->n_param;
  for (int i = 0; i < h->n_inst; ++i) hd.c0_doubles += c0_doubles(h, i);
  hd.iter = h->lb_iter;
  hd.evals = h->lb_evals;
  hd.m = h->lbp.m;
  hd.lbp = h->lbp;
  char* out = static_cast<char*>(state);
  const int64_t n = h->n_param;
  const size_t vb = (size_t)n * sizeof(double);
  HIPCHK(h, hipMemcpyAsync(out, &hd, sizeof(hd), hipMemcpyHostToDevice, s));
  out += LB_CKPT_HEADER;
  HIPCHK(h, hipMemcpyAsync(out, h->lb_st, sizeof(LbState), hipMemcpyDeviceToDevice, s));
  out += state_scalars_bytes();
  const std::pair<const double*, size_t> parts[] = {
      {h->x, vb}, {h->g, vb}, {h->S, vb * hd.m}, {h->Yv, vb * hd.m}};
  for (const auto& pr : parts) {
    if (pr.second) HIPCHK(h, hipMemcpyAsync(out, pr.first, pr.second, hipMemcpyDeviceToDevice, s));
    out += pr.second;
  }
  for (int i = 0; i < h->n_inst; ++i) {
    const size_t b = (size_t)c0_doubles(h, i) * sizeof(double);
    if (b) HIPCHK(h, hipMemcpyAsync(out, c0_ptr(h, i), b, hipMemcpyDeviceToDevice, s));
    out += b;
  }
  HIPCHK(h, hipStreamSynchronize(s));  // the header is copied from this stack frame
  return ETDM_OK;
}

etdm_status etdm_lbfgs_set_state(etdm_handle* h, const void* state, void* stream) {
  if (!h) return ETDM_E_ARG;
  if (!state) return fail(h, ETDM_E_ARG, "null state buffer");
  hipStream_t s = S(stream);
  LbCheckpoint hd{};
  const char* in = static_cast<const char*>(state);
  HIPCHK(h, hipMemcpyAsync(&hd, in, sizeof(hd), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  int64_t c0 = 0;
  for (int i = 0; i < h->n_inst; ++i) c0 += c0_doubles(h, i);
  if (std::memcmp(hd.magic, kCkptMagic, 8) != 0) return fail(h, ETDM_E_ARG, "not an L-BFGS checkpoint");
  if (hd.layout != ckpt_layout(h) || hd.n_param != h->n_param || hd.c0_doubles != c0)
    return fail(h, ETDM_E_SHAPE, "checkpoint from a handle with other shapes or modes");
  if (hd.m < 1 || hd.m > LB_MMAX || hd.lbp.m != hd.m) return fail(h, ETDM_E_ARG, "corrupt checkpoint header");
  if (!h->lb_sum) HIPCHK(h, hipHostMalloc(reinterpret_cast<void**>(&h->lb_sum), sizeof(LbState)));
  const int64_t n = h->n_param;
  const size_t vb = (size_t)n * sizeof(double);
  in += LB_CKPT_HEADER;
  HIPCHK(h, hipMemcpyAsync(h->lb_st, in, sizeof(LbState), hipMemcpyDeviceToDevice, s));
  in += state_scalars_bytes();
  const std::pair<double*, size_t> parts[] = {{h->x, vb}, {h->g, vb}, {h->S, vb * hd.m}, {h->Yv, vb * hd.m}};
  for (const auto& pr : parts) {
    if (pr.second) HIPCHK(h, hipMemcpyAsync(pr.first, in, pr.second, hipMemcpyDeviceToDevice, s));
    in += pr.second;
  }
  for (int i = 0; i < h->n_inst; ++i) {
    const size_t b = (size_t)c0_doubles(h, i) * sizeof(double);
    if (b) HIPCHK(h, hipMemcpyAsync(c0_ptr(h, i), in, b, hipMemcpyDeviceToDevice, s));
    in += b;
  }
  build_hdiag(h, s);  // preconditioner (and H0 C0) of the restored reference orbitals
  pack_static(h, s);   // and the packed panels of the restored reference
  HIPCHK(h, hipMemcpyAsync(h->lb_sum, h->lb_st, sizeof(LbState), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(s));
  free_lb_graphs(h);
  h->lbp = hd.lbp;
  h->lbp_set = true;
  h->lb_iter = hd.iter;
  h->lb_evals = hd.evals;
  h->lb_init = true;
  return ETDM_OK;
}

etdm_status etdm_lbfgs_step(etdm_handle* h, const etdm_lbfgs_params* params, void* A, double* E, void* G,
                            etdm_lbfgs_info* info, void* stream) {
  if (!h) return ETDM_E_ARG;
  if ((!A || !G) && h->n_param > 0) return fail(h, ETDM_E_ARG, "null A or G");
  if (!E || !info) return fail(h, ETDM_E_ARG, "null E or info");
  etdm_lbfgs_params P;
  if (params) P = *params;
  else etdm_lbfgs_defaults(&P);
  if (P.m < 1 || P.m > LB_MMAX || P.max_ls < 1 || !(P.c1 > 0.0) || !(P.c2 > P.c1) || !(P.c2 < 1.0) ||
      !(P.gamma >= 0.0) || !(P.gamma <= 1.0) || !(P.beta0 > 0.0) || P.reset_every < 0 ||
      !(P.reset_norm >= 0.0))
    return fail(h, ETDM_E_ARG, "invalid L-BFGS parameters");
  hipStream_t s = S(stream);
  const int64_t n = h->n_param;
  const size_t pb = (size_t)n * sizeof(double);
  std::memset(info, 0, sizeof(*info));
  if (!h->lb_sum) HIPCHK(h, hipHostMalloc(reinterpret_cast<void**>(&h->lb_sum), sizeof(LbState)));
  const LbParams lp{P.c1, P.c2, P.delta, P.sigma, P.eps, P.gamma, P.max_ls, P.m, P.reset_norm};
  const bool m_changed = h->lbp_set && h->lbp.m != lp.m;
  if (!h->lbp_set || std::memcmp(&lp, &h->lbp, sizeof(lp)) != 0) {
    free_lb_graphs(h);  // the constants are part of the captured launches
    h->lbp = lp;
    h->lbp_set = true;
  }
  if (!h->lb_init) {
    if (pb) HIPCHK(h, hipMemcpyAsync(h->x, A, pb, hipMemcpyDeviceToDevice, s));
    h->lb_iter = 0;
    h->lb_evals = 0;
    CHECK(lb_start(h, P.beta0, 1, s));
    h->lb_init = true;
  } else if ((P.reset_every > 0 && h->lb_iter > 0 && h->lb_iter % P.reset_every == 0) ||
             (P.reset_norm > 0.0 && h->lb_sum->xmax2 > P.reset_norm * P.reset_norm)) {
    // reference reset (Sec. 3.4): C0 <- C0 exp(A), A <- 0, memory erased, beta kept
    HIPCHK(h, hipMemcpyAsync(h->par_ws, h->x, pb, hipMemcpyDeviceToDevice, s));
    new_reference(h, s);
    launch_fill(h->x, n, 0.0, s);
    CHECK(lb_start(h, P.beta0, 0, s));
    info->flags |= 1;
  } else if (m_changed) {
    CHECK(lb_start(h, P.beta0, 0, s));  // a new memory length starts an empty memory
  }
  CHECK(lb_search(h, 0, s));
  if (h->lb_sum->steepest) info->flags |= 2;
  if (h->lb_sum->result == LR_FAIL) {
    info->flags |= 2;
    CHECK(lb_search(h, 2, s));
    if (h->lb_sum->result != LR_ACCEPT) {
      info->flags |= 4;
      info->iter = h->lb_iter;
      info->n_evals = h->lb_evals;
      info->E = h->lb_sum->E;
      return fail(h, ETDM_E_LINESEARCH, "no acceptable step along the search direction");
    }
  }
  ++h->lb_iter;
  if (pb) {
    HIPCHK(h, hipMemcpyAsync(A, h->x, pb, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipMemcpyAsync(G, h->g, pb, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(h, hipMemcpyAsync(E, h->E_ws, (h->n_inst + 1) * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipStreamSynchronize(s));
  const LbState& r = *h->lb_sum;
  info->iter = h->lb_iter;
  info->n_evals = h->lb_evals;
  info->alpha = r.acc_a;
  info->E = r.acc_f;
  info->gnorm = std::sqrt(std::max(r.gg, 0.0));
  return ETDM_OK;
}

}  // extern "C"
