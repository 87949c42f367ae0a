// etdm_energy_grad_static: the energy and exact gradient of ONE real occupied-virtual
// instance (dense H0, FP64) for callers that cannot allocate device memory.  Every
// intermediate and every launch descriptor lives in `scratch`, a file-scope device
// array of a fixed size, instead of a handle's workspace.  The launch sequence and the
// kernels are those of etdm_energy_grad's real path in the eigenbasis of P (ov.hip):
//   P = B B^T, eigendecomposition (LDS solver, N <= EIGH_LDS_MAX), spectral pass,
//   V = X^T B with sinc sqrt(P) and the pair-integral products, C0_o X and C0_v V^T,
//   their combination, C_occ, T = H0 C_occ, C_virt, rows and energy, L_ov, L_ov V^T,
//   the one-workgroup gradient chain, G = -2 (sinc sqrt(P) L_ov + (X Nm) V).
// The descriptors are assembled on the host per call and written into the array by a
// small kernel that takes them by value, so a call allocates nothing and can be
// captured in a HIP graph.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "common.h"
#include "etdm.h"
#include "ov.h"

using namespace etdm;

// One array per GPU that runs the library, held until the process ends.  Calls on one
// GPU share it: calls that overlap in time on one GPU race.
static __device__ __align__(256) unsigned char scratch[ETDM_STATIC_SCRATCH_BYTES];

namespace {

constexpr size_t DESC_BYTES = 64 << 10;  // descriptors at the start of the array
constexpr int MAX_DEVICES = 64;
constexpr int BLOB_WORDS = 256;  // 2 KB of descriptors per write launch

// Device address of `scratch` per device, from hipGetSymbolAddress on the first call
// with that device current (in host code the array's name is not a device address).
void* g_ptr[MAX_DEVICES] = {};
std::mutex g_mu;

etdm_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return ETDM_E_HIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ETDM_E_HIP;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return ETDM_OK;
}

struct Blob {
  uint64_t w[BLOB_WORDS];
};

// dst[0 .. nwords) = blob; the first thread also clears *zero (the caller's status)
__global__ void blob_write_kernel(Blob b, int nwords, uint64_t* __restrict__ dst, int32_t* zero) {
  const int t = threadIdx.x;
  if (t < nwords) dst[t] = b.w[t];
  if (zero && t == 0) *zero = 0;
}

// Host image of the descriptor area: a bump layout whose offsets are also the device
// offsets from the start of `scratch`.
struct HostDesc {
  alignas(16) unsigned char bytes[DESC_BYTES];
  size_t off = 0;
  bool overflow = false;
  template <typename T>
  size_t put(const T* v, size_t n) {
    const size_t a = (off + 15) & ~size_t(15);
    const size_t sz = n * sizeof(T);
    if (a + sz > DESC_BYTES) {
      overflow = true;
      return 0;
    }
    std::memcpy(bytes + a, v, sz);
    off = a + sz;
    return a;
  }
};

GemmProb mk(int m, int n, int k, const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
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

// One grouped GEMM launch: its problems and workgroup -> problem table in the
// descriptor area.
struct StaticStage {
  GemmProb probs[4];
  int n = 0, tiles = 0;
  int tile_prob[256];
  const GemmProb* d_probs = nullptr;
  const int* d_tile = nullptr;
  int opA = OP_N, opB = OP_N;
  bool ok = true;
  void add(GemmProb p) {
    if (p.m <= 0 || p.n <= 0) return;
    p.tiles_n = (p.n + GEMM_BN - 1) / GEMM_BN;
    p.tile_begin = tiles;
    const int t = p.tiles_n * ((p.m + GEMM_BM - 1) / GEMM_BM);
    if (n >= 4 || tiles + t > 256) {
      ok = false;
      return;
    }
    for (int i = 0; i < t; ++i) tile_prob[tiles + i] = n;
    tiles += t;
    probs[n++] = p;
  }
  void place(HostDesc& hd, unsigned char* base) {
    d_probs = reinterpret_cast<const GemmProb*>(base + hd.put(probs, n > 0 ? n : 1));
    d_tile = reinterpret_cast<const int*>(base + hd.put(tile_prob, tiles > 0 ? tiles : 1));
  }
  void launch(hipStream_t s) const { launch_gemm(d_probs, d_tile, tiles, opA, opB, GP_FP64, s); }
};

// Gauss-Legendre nodes and weights on [0, 1] (Newton on the three-term recurrence).
void gauss_legendre_01(int n, double* t, double* w) {
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), p0 = 1.0, p1 = x;
    for (int it = 0; it < 100; ++it) {
      p0 = 1.0;
      p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    p0 = 1.0;
    p1 = x;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double dp = n * (x * p1 - p0) / (x * x - 1.0);
    t[i] = 0.5 * (x + 1.0);
    w[i] = 1.0 / ((1.0 - x * x) * dp * dp);
  }
}

thread_local HostDesc t_desc;

}  // namespace

extern "C" etdm_status etdm_energy_grad_static(int32_t M, int32_t N, double f_occ, double hubbard_U,
                                               const double* H0, const double* C0, const double* B, double* E,
                                               double* G, int32_t* status, void* stream) {
  if (!H0 || !C0 || !B || !E || !G || !status) return ETDM_E_ARG;
  if (!std::isfinite(f_occ) || !std::isfinite(hubbard_U)) return ETDM_E_ARG;
  if (M < 2 || M > ETDM_STATIC_MAX_M || N < 1 || N >= M || N > ETDM_STATIC_MAX_N) return ETDM_E_SHAPE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  void* vbase = nullptr;
  if (scratch_address(&vbase) != ETDM_OK) return ETDM_E_HIP;
  unsigned char* base = static_cast<unsigned char*>(vbase);

  // workspace after the descriptor area, in doubles
  const int64_t Nv = M - N, NN = (int64_t)N * N, MN = (int64_t)M * N, q = (int64_t)OV_NQ * N;
  double* ws = reinterpret_cast<double*>(base + DESC_BYTES);
  int64_t o = 0;
  auto take = [&](int64_t n) {
    double* p = ws + o;
    o += (n + 31) & ~int64_t(31);  // 256-byte steps
    return p;
  };
  double *P = take(NN), *X = take(NN), *sv = take(N), *fac = take(3 * N), *XT = take(NN), *XsnT = take(NN);
  double *tab = take(4 * q), *mu1 = take(NN), *mu2 = take(NN), *V = take(N * Nv), *sincP = take(NN);
  double *CX = take(MN), *CV = take(MN), *Cocc = take(MN), *Cvirt = take(M * Nv), *T = take(MN);
  double *d = take(M), *e = take(M), *Lov = take(N * Nv), *LV = take(NN), *XNm = take(NN);
  double* gl = take(2 * OV_NQ);  // Gauss-Legendre nodes, then weights
  if (DESC_BYTES + (size_t)o * sizeof(double) > (size_t)ETDM_STATIC_SCRATCH_BYTES) return ETDM_E_SHAPE;

  // launch descriptors
  StaticStage sP, sVF, sCXV, sC, sT, sV, sL, sLV, sG;
  sP.opB = OP_T;
  sP.add(mk(N, N, (int)Nv, B, Nv, B, Nv, P, N));
  sVF.opA = OP_T;
  sVF.add(mk(N, (int)Nv, N, X, N, B, Nv, V, Nv));
  sVF.add(mk(N, N, N, XsnT, N, XT, N, sincP, N));
  sVF.add(mk(N, N, OV_NQ, tab, N, tab + q, N, mu1, N));
  sVF.add(mk(N, N, OV_NQ, tab + 2 * q, N, tab + 3 * q, N, mu2, N));
  sCXV.opB = OP_T;
  sCXV.add(mk(M, N, N, C0, M, XT, N, CX, N));
  sCXV.add(mk(M, N, (int)Nv, C0 + N, M, V, Nv, CV, N));
  sC.opB = OP_T;
  sC.add(mk(M, N, N, CX, N, X, N, Cocc, N));
  sT.add(mk(M, N, M, H0, M, Cocc, N, T, N));
  {
    GemmProb p = mk(M, (int)Nv, N, CV, N, V, Nv, Cvirt, Nv);
    p.D = C0 + N;
    p.ldd = M;
    p.beta = 1.0;
    sV.add(p);
  }
  sL.opA = OP_T;
  sL.add(mk(N, (int)Nv, M, T, N, Cvirt, Nv, Lov, Nv, f_occ));
  sLV.opB = OP_T;
  sLV.add(mk(N, N, (int)Nv, Lov, Nv, V, Nv, LV, N));
  {
    GemmProb p = mk(N, (int)Nv, N, sincP, N, Lov, Nv, G, Nv, -2.0);
    p.k2 = N;
    p.A2 = XNm;
    p.lda2 = N;
    p.B2 = V;
    p.ldb2 = Nv;
    p.alpha2 = -2.0;
    sG.add(p);
  }
  StaticStage* all[] = {&sP, &sVF, &sCXV, &sC, &sT, &sV, &sL, &sLV, &sG};
  HostDesc& hd = t_desc;
  hd.off = 0;
  hd.overflow = false;
  for (StaticStage* st : all) {
    if (!st->ok) return ETDM_E_SHAPE;
    st->place(hd, base);
  }
  const int zero = 0;
  const EighProb eig{P, X, sv, N, 1, nullptr, nullptr};
  const OvSpec spec{sv, X, fac, XT, XsnT, tab, P /* exp(A) copies not written */, N};
  const OvRot rot{CX, CV, nullptr, nullptr, fac, M, N};
  const OvRows rows{Cocc, T, d, e, M, N, f_occ};
  const OvEnergy en{d, e, M, f_occ, 1.0};
  const OvCong cong{sv, X, LV, mu1, mu2, XNm, N};
  const EighProb* d_eig = reinterpret_cast<const EighProb*>(base + hd.put(&eig, 1));
  const OvSpec* d_spec = reinterpret_cast<const OvSpec*>(base + hd.put(&spec, 1));
  const OvRot* d_rot = reinterpret_cast<const OvRot*>(base + hd.put(&rot, 1));
  const OvRows* d_rows = reinterpret_cast<const OvRows*>(base + hd.put(&rows, 1));
  const OvEnergy* d_en = reinterpret_cast<const OvEnergy*>(base + hd.put(&en, 1));
  const OvCong* d_cong = reinterpret_cast<const OvCong*>(base + hd.put(&cong, 1));
  const int* d_zero = reinterpret_cast<const int*>(base + hd.put(&zero, 1));  // begin offsets {0}
  double t_h[OV_NQ], w_h[OV_NQ];
  gauss_legendre_01(OV_NQ, t_h, w_h);
  if (hd.overflow) return ETDM_E_SHAPE;
  const size_t words = (hd.off + 7) / 8;

  // descriptors into the array (the first launch also clears the status word), then
  // the quadrature nodes into the workspace
  for (size_t w0 = 0; w0 < words; w0 += BLOB_WORDS) {
    Blob b;
    const int nw = (int)std::min<size_t>(BLOB_WORDS, words - w0);
    std::memcpy(b.w, hd.bytes + 8 * w0, 8 * (size_t)nw);
    blob_write_kernel<<<1, BLOB_WORDS, 0, s>>>(b, nw, reinterpret_cast<uint64_t*>(base) + w0,
                                               w0 == 0 ? status : nullptr);
  }
  {
    Blob b;
    std::memcpy(b.w, t_h, sizeof(t_h));
    std::memcpy(b.w + OV_NQ, w_h, sizeof(w_h));
    blob_write_kernel<<<1, BLOB_WORDS, 0, s>>>(b, 2 * OV_NQ, reinterpret_cast<uint64_t*>(gl), nullptr);
  }

  // the launch sequence of the real path (see ov.hip)
  sP.launch(s);
  launch_eigh_real_lds(d_eig, 1, status, s);
  launch_ov_spectral(d_spec, d_zero, 1, ov_spectral_blocks(N), gl, gl + OV_NQ, 0, s);
  sVF.launch(s);
  sCXV.launch(s);
  launch_ov_rot(d_rot, d_zero, 1, M * N, s);
  sC.launch(s);
  sT.launch(s);
  sV.launch(s);
  launch_ov_rows(d_rows, d_zero, 1, M, hubbard_U, s);
  launch_ov_energy(d_en, 1, hubbard_U, E, s);
  launch_total_energy(E, 1, 0.0, nullptr, 0, hubbard_U, status, s);
  sL.launch(s);
  sLV.launch(s);
  launch_ov_congruence(d_cong, 1, s);
  sG.launch(s);
  launch_nonfinite_scan(G, (int64_t)N * Nv, status, s);
  return hipGetLastError() == hipSuccess ? ETDM_OK : ETDM_E_HIP;
}
