// Host side of the space-time multigrid library: parameter validation, the
// level hierarchy (coarsening rule of Sec. 4), per-level constant tables for
// the fast-diagonalisation block solve, workspace binding, the V-cycle /
// solve / adjoint drivers, and the C ABI declared in st_mg.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "st_mg.h"
#include "stmg_internal.h"
#include "stmg_mesh.h"

using namespace stmg;

namespace {

constexpr double PI = 3.14159265358979323846;

// ------------------------------------------------------------ small dense helpers
// Legendre P_l(s) by the three-term recurrence.
double legendre(int l, double s) {
  if (l == 0) return 1.0;
  double p0 = 1.0, p1 = s;
  for (int k = 2; k <= l; ++k) {
    const double p2 = ((2.0 * k - 1.0) * s * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Gauss-Legendre nodes/weights on [-1,1] (Newton on P_q).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double s = std::cos(PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      const double p = legendre(q, s), pm = legendre(q - 1, s);
      const double dp = q * (s * p - pm) / (s * s - 1.0);
      const double ds = p / dp;
      s -= ds;
      if (std::fabs(ds) < 1e-16) break;
    }
    const double p = legendre(q, s), pm = legendre(q - 1, s);
    const double dp = q * (s * p - pm) / (s * s - 1.0);
    x[i] = s;
    w[i] = 2.0 / ((1.0 - s * s) * dp * dp);
  }
}

// In-place inverse of a small dense matrix (Gauss-Jordan, partial pivoting).
bool invert(int n, double* A) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[c * n + k], A[piv * n + k]);
        std::swap(I[c * n + k], I[piv * n + k]);
      }
    const double d = A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] /= d;
      I[c * n + k] /= d;
    }
    for (int r = 0; r < n; ++r)
      if (r != c) {
        const double f = A[r * n + c];
        if (f == 0.0) continue;
        for (int k = 0; k < n; ++k) {
          A[r * n + k] -= f * A[c * n + k];
          I[r * n + k] -= f * I[c * n + k];
        }
      }
  }
  std::memcpy(A, I.data(), sizeof(double) * n * n);
  return true;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Nearest bfloat16 (ties to even) of a double, via the nearest float.
uint16_t bf16_round(double v) {
  const float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct Level {
  int n = 0, N = 0;
  long long nx = 0;
  double tau = 0, h = 0, mu = 0;
  char kind = 0;          // transition to the next coarser level: 'f' or 's'; 0 on the coarsest
  int hb = 0;             // folded transform: 16-row blocks per half
  double* S64 = nullptr;  // folded DST-I in MFMA fragment order
  float* S32 = nullptr;
  void* S16 = nullptr;    // folded DST-I in bf16 16x16x16 operand order [dir][half][kb][c][lane][4]
  double* G64 = nullptr;  // per-mode inverse blocks [nx][nt][nt]
  float* G32 = nullptr;
  double* Sp64 = nullptr; // plain DST-I (n x n), used by the small-level smoother
  double* S2_64 = nullptr; // twice-folded fragments (FP64: n = 63, 127) [dir][mat][kb][ib][lane]
  float* S2_32 = nullptr;  // the same for FP32 (n = 63, 127, 255), FP32 contraction order
  void* S2_16 = nullptr;   // the same in bf16 for the BF16 inner cycle: [dir][mat][kb][c][lane][4]
  double* eig64 = nullptr; // 1-D eigenvalues m_s then kappa_s in spectral order (2n)
  float* eig32 = nullptr;
  float* Sp32 = nullptr;
  int impl = -1;          // transform family chosen for this level (-1: handle default)
  int small = -1;         // small-level smoother on (1) / off (0) for this level (-1: handle default)
  int rx = -1;            // residual fused with the forward x pass (1) / separate (0) (-1: handle default)
  int rr = -1;            // pre-restriction defect restricted by the residual kernel (1) / two passes (0)
  float tuned_ms = 0.f;   // autotuned smoothing-step time
  PassShape shape{};      // launch shape of the twice-folded passes (autotuned)
  void* u = nullptr;      // workspace vectors (inner precision), coarse levels only
  void* u2 = nullptr;     // second iterate buffer for the small-level smoother
  void* F = nullptr;
  void* r = nullptr;
  // spatial cycle of the inexact smoother: sub-level j has n_j = (n_{j-1}-1)/2
  // interior nodes per dimension down to one; X/Y are the Jacobi ping-pong
  // iterates, F the restricted defect (j >= 1)
  struct Sub {
    int n = 0;
    long long nx = 0;
    double h = 0;
    void *X = nullptr, *Y = nullptr, *F = nullptr;
  };
  std::vector<Sub> sub;
  // P1 meshes: n is the refinement level; D = dense inverse of the slab matrix
  // on the coarse mesh at this level's tau (m = N_t x its interior nodes), C =
  // the same for this level's own mesh on the coarsest level
  double* D64 = nullptr;
  float* D32 = nullptr;
  int dm = 0;
  double* C64 = nullptr;
  float* C32 = nullptr;
  int cm = 0;
  long long dof(int nt, int b) const { return (long long)b * N * nt * nx; }
};

// One refinement level of a P1 mesh on the device (CSR of M_h / K_h with their
// diagonals; interpolation from the next coarser level when level > 0).
struct MeshDev {
  long long nx = 0, nnz = 0, nxc = 0;
  int *rowptr = nullptr, *col = nullptr;
  int ew = 0;                                   // ELL width (longest row)
  int* ecol = nullptr;                          // [ew][nx]
  double* emk64 = nullptr;                      // [ew][nx][2] (M_h, K_h)
  float* emk32 = nullptr;
  int hmax = 0;                                 // largest tile halo
  int *hoff = nullptr, *hcol = nullptr;         // tile halos (256-row tiles)
  unsigned short* lcol = nullptr;               // [ew][nx] halo-local columns
  unsigned short* ldiag = nullptr;              // [nx] halo-local position of the node itself

  double *mv64 = nullptr, *kv64 = nullptr, *dg64 = nullptr, *w64 = nullptr;
  float *mv32 = nullptr, *kv32 = nullptr, *dg32 = nullptr, *w32 = nullptr;
  int *p = nullptr, *rrow = nullptr, *rcol = nullptr;
  int* rell = nullptr;                          // [rw][nxc] transpose of the interpolation, ELL
  int rw = 0;
  int *rhoff = nullptr, *rhcol = nullptr;       // coarse-tile halos of the transpose
  unsigned short* rloc = nullptr;
  int rhmax = 0;
};

struct GraphCache {
  hipGraphExec_t exec = nullptr;
  const void* u = nullptr;
  const void* F = nullptr;
  int transpose = -1;
  hipStream_t stream = nullptr;
};

}  // namespace

struct st_mg {
  st_mg_params p{};
  int nt = 0;
  double mu_star = 0;
  std::vector<Level> lv;
  bool mesh = false;                 // P1 mesh in space (st_mg_setup_mesh)
  std::vector<stmg::MeshLevel> mh;   // host meshes, refinement levels 0..R
  std::vector<MeshDev> md;           // their device copies
  double Kt[NT_BIG * NT_BIG] = {};   // K_tau (independent of tau for the Legendre basis)
  double Mh[NT_BIG * NT_BIG] = {};   // M_tau / tau
  double ca[NT_BIG] = {};            // psi_l(t_{n-1}^+): N_tau = ca cb^T
  double cb[NT_BIG] = {};            // psi_l(t_n^-)
  double ints[NT_BIG] = {};          // int_slab psi_l dt / tau
  double R1T[NT_BIG * NT_BIG] = {};  // time prolongation blocks (independent of tau)
  double R2T[NT_BIG * NT_BIG] = {};
  // device copies of the time matrices for N_t > NT_MAX:
  // [K | K^T | M/tau | ca | cb | ints | R1T | R2T], double and float
  double* gen64 = nullptr;
  float* gen32 = nullptr;
  // workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  void* tmp = nullptr;   // transform buffer, inner precision, fine size
  void* r0 = nullptr;    // fine residual, inner precision
  void* F32 = nullptr;   // mixed: inner right-hand side (fine, float)
  void* e32 = nullptr;   // mixed: inner correction (fine, float)
  double *cu64 = nullptr, *cF64 = nullptr, *cr64 = nullptr, *ct64 = nullptr;  // mixed: coarsest in double
  double* partial = nullptr;
  long long partial_per_batch = 0;
  double* norm_dev = nullptr;
  int graph = 0;
  int cus = 0;            // compute units of the device (caps of persistent grids)
  int impl = TRANSFORM_AUTO;
  bool small = true;      // one-kernel smoothing steps on levels whose slabs fit in LDS
  bool rx = false;        // residual fused with the forward x pass where it applies (autotuned per level)
  bool rr = true;         // residual and full restriction in one pass where it applies
  // coarse end of every cycle in one workgroup from level `tail` down (-1: off);
  // argument blocks in device memory for the forward and the adjoint cycle
  int tail = -1;
  size_t tail_lds = 0;
  void* tail_args[2] = {nullptr, nullptr};
  GraphCache gc;
  // per-launch event pairs while profiling is on
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  // this device's copy of the static scratch array (st_mg_residual_noalloc),
  // or nullptr with the reason in scratch_err
  double* scratch = nullptr;
  std::string scratch_err;
  size_t ev_used = 0;
  struct ProfRec { int kind, level; size_t e0, e1; };
  std::vector<ProfRec> prof_recs;
  std::string err;
};

// Static scratch of st_mg_residual_noalloc: per-workgroup partial sums of
// r^2 (NOALLOC_PARTIALS doubles), then one sum per right-hand side
// (NOALLOC_BATCH doubles); 8 MiB + 2 KiB.  Every GPU the library runs on
// holds its own copy until the process ends.  Host code never names the
// array: it uses the address hipGetSymbolAddress returns for the current
// device (scratch_address below).
constexpr long long NOALLOC_PARTIALS = 1LL << 20;
constexpr int NOALLOC_BATCH = 256;
static __device__ __align__(256) double scratch[NOALLOC_PARTIALS + NOALLOC_BATCH];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The current device's address of `scratch`, looked up once per device.
hipError_t scratch_address(double** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int fail(st_mg_t h, int code, const char* fmt, ...) {
  if (h) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    h->err = buf;
  }
  return code;
}

#define HIPCHK(h, call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) return fail(h, ST_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define CHK(call)              \
  do {                         \
    int rc_ = (call);          \
    if (rc_ != ST_OK) return rc_; \
  } while (0)

bool is_pow2(long long x) { return x > 0 && (x & (x - 1)) == 0; }

// FP64 outer refinement around an FP32 inner cycle (FP32 or BF16 transforms).
bool is_mixed(const st_mg* h) { return h->p.precision == ST_MIXED || h->p.precision == ST_MIXED_BF16; }

// High DG orders run the runtime-N_t kernels (time matrices in device memory).
bool high_order(const st_mg* h) { return h->nt > NT_MAX; }

// ------------------------------------------------------------------ profiling
// Event pair around one launch: begin() returns a ticket, end() closes it.
size_t prof_event(st_mg* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return (size_t)-1;
    h->ev_pool.push_back(e);
  }
  return h->ev_used++;
}

struct ProfScope {
  st_mg* h;
  int kind, level;
  hipStream_t s;
  size_t e0 = (size_t)-1;
  ProfScope(st_mg* h_, int kind_, int level_, hipStream_t s_) : h(h_), kind(kind_), level(level_), s(s_) {
    if (h->prof) {
      e0 = prof_event(h);
      if (e0 != (size_t)-1) (void)hipEventRecord(h->ev_pool[e0], s);
    }
  }
  ~ProfScope() {
    if (h->prof && e0 != (size_t)-1) {
      const size_t e1 = prof_event(h);
      if (e1 == (size_t)-1) return;
      (void)hipEventRecord(h->ev_pool[e1], s);
      h->prof_recs.push_back({kind, level, e0, e1});
    }
  }
};

// ---------------------------------------------------------------- time basis
// Shifted Legendre basis on a slab: M_tau = tau diag(1/(2l+1));
// K_tau[k][l] = 1 - 2 [l < k and k - l odd] (from -int psi_l psi_k' + psi_l(t_n) psi_k(t_n));
// psi_l(t_n^-) = 1, psi_l(t_{n-1}^+) = (-1)^l.
void time_basis(st_mg* h) {
  const int nt = h->nt;
  for (int k = 0; k < nt; ++k) {
    for (int l = 0; l < nt; ++l) {
      h->Kt[k * nt + l] = 1.0 - ((l < k && ((k - l) & 1)) ? 2.0 : 0.0);
      h->Mh[k * nt + l] = (k == l) ? 1.0 / (2.0 * k + 1.0) : 0.0;
    }
    h->ca[k] = (k & 1) ? -1.0 : 1.0;
    h->cb[k] = 1.0;
    h->ints[k] = (k == 0) ? 1.0 : 0.0;
  }
  // R_s^T[k][l]: Legendre coefficient k (fine slab s) of the coarse basis
  // function P_l restricted to that half: P_l((x + 2s - 1)/2), x in [-1,1].
  std::vector<double> gx, gw;
  gauss_legendre(nt + 2, gx, gw);
  for (int s = 0; s < 2; ++s) {
    double* RT = s == 0 ? h->R1T : h->R2T;
    for (int k = 0; k < nt; ++k)
      for (int l = 0; l < nt; ++l) {
        double acc = 0.0;
        for (size_t q = 0; q < gx.size(); ++q)
          acc += gw[q] * legendre(k, gx[q]) * legendre(l, 0.5 * (gx[q] + 2.0 * s - 1.0));
        RT[k * nt + l] = 0.5 * (2.0 * k + 1.0) * acc;
      }
  }
}

// Stability function R(z) = b^T (K - z M/tau)^{-1} a (trace of the rank-one
// matrix (K + lam M)^{-1} N with lam tau = -z; Lemma chap4_theorem2).
double stability(const st_mg* h, double z) {
  const int nt = h->nt;
  double A[NT_BIG * NT_BIG];
  for (int i = 0; i < nt * nt; ++i) A[i] = h->Kt[i] - z * h->Mh[i];
  if (!invert(nt, A)) return NAN;
  double r = 0.0;
  for (int i = 0; i < nt; ++i)
    for (int j = 0; j < nt; ++j) r += h->cb[i] * A[i * nt + j] * h->ca[j];
  return r;
}

// mu*: first root of R(-3 mu) = sqrt(2) - 1 on (0, 5]
// (Remark chap4_remarkCriticalDiscretizationParameter).
double critical_mu(const st_mg* h) {
  const double target = std::sqrt(2.0) - 1.0;
  double lo = 0.0, hi = -1.0;
  const int steps = 5000;
  double prev = stability(h, 0.0) - target;
  for (int i = 1; i <= steps; ++i) {
    const double m = 5.0 * i / steps;
    const double v = stability(h, -3.0 * m) - target;
    if (prev > 0.0 && v <= 0.0) {
      lo = 5.0 * (i - 1) / steps;
      hi = m;
      break;
    }
    prev = v;
  }
  if (hi < 0) return NAN;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (stability(h, -3.0 * mid) - target > 0.0) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Spectral order along one axis: the h odd sine modes first, then the h-1 even
// ones.  Returns the 1-based mode number k of spectral index s.
int spectral_mode(int s, int n) {
  const int h = (n + 1) / 2;
  return s < h ? 2 * s + 1 : 2 * (s - h) + 2;
}

// Upload the level's folded DST fragments and the per-mode blocks G.
int build_level_tables(st_mg* h, Level& L) {
  const int n = L.n, nt = h->nt, d = h->p.dim;
  const int HB = L.hb, HP = 16 * HB, half = (n + 1) / 2;
  const double sc = std::sqrt(2.0 / (n + 1));
  // folded blocks: fwd_odd[s][i] = S[2s+1][i+1] (s, i < h), fwd_even[s][i] = S[2s+2][i+1] (s, i < h-1);
  // the inverse blocks are their transposes.
  auto blk = [&](int dir, int hf, int r, int c) -> double {
    const int lim = hf == 0 ? half : half - 1;
    if (r >= lim || c >= lim) return 0.0;
    const int s = dir == 0 ? r : c, i = dir == 0 ? c : r;
    const int k = hf == 0 ? 2 * s + 1 : 2 * s + 2;
    return sc * std::sin(PI * (double)k * (i + 1.0) / (n + 1));
  };
  const size_t per = (size_t)HB * (HP / 4) * 64;
  std::vector<double> frag(4 * per);
  std::vector<float> frag32(4 * per);
  for (int dir = 0; dir < 2; ++dir)
    for (int hf = 0; hf < 2; ++hf)
      for (int kb = 0; kb < HB; ++kb)
        for (int ib = 0; ib < HP / 4; ++ib)
          for (int lane = 0; lane < 64; ++lane) {
            const size_t o = (size_t)(dir * 2 + hf) * per + ((size_t)kb * (HP / 4) + ib) * 64 + lane;
            frag[o] = blk(dir, hf, kb * 16 + (lane & 15), ib * 4 + (lane >> 4));
            frag32[o] = (float)frag[o];
          }
  // bf16 operands of v_mfma_f32_16x16x16_bf16: lane supplies A[lane%16][4(lane/16)+q]
  std::vector<uint16_t> frag16((size_t)4 * HB * HB * 64 * 4);
  for (int dir = 0; dir < 2; ++dir)
    for (int hf = 0; hf < 2; ++hf)
      for (int kb = 0; kb < HB; ++kb)
        for (int c = 0; c < HB; ++c)
          for (int lane = 0; lane < 64; ++lane)
            for (int q = 0; q < 4; ++q) {
              const size_t o = (((((size_t)dir * 2 + hf) * HB + kb) * HB + c) * 64 + lane) * 4 + q;
              frag16[o] = bf16_round(blk(dir, hf, kb * 16 + (lane & 15), c * 16 + 4 * (lane >> 4) + q));
            }
  // per-mode blocks: mu_k K + nu_k M with mu_k = prod m, nu_k = sum_a kappa_a prod_{b!=a} m_b,
  // m = h/3 (2 + cos), kappa = 2/h (1 - cos) at angle (k+1) pi h
  const double hh = L.h;
  std::vector<double> m1(n), k1(n);
  for (int s = 0; s < n; ++s) {
    const double c = std::cos(spectral_mode(s, n) * PI * hh);
    m1[s] = hh / 3.0 * (2.0 + c);
    k1[s] = 2.0 / hh * (1.0 - c);
  }
  {
    std::vector<double> e64(2 * (size_t)n);
    std::vector<float> e32(2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
      e64[i] = m1[i];
      e64[n + i] = k1[i];
      e32[i] = (float)m1[i];
      e32[n + i] = (float)k1[i];
    }
    HIPCHK(h, hipMalloc(&L.eig64, e64.size() * sizeof(double)));
    HIPCHK(h, hipMalloc(&L.eig32, e32.size() * sizeof(float)));
    HIPCHK(h, hipMemcpy(L.eig64, e64.data(), e64.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(h, hipMemcpy(L.eig32, e32.data(), e32.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  const long long nx = L.nx;
  std::vector<double> G((size_t)nx * nt * nt);
  std::vector<float> G32((size_t)nx * nt * nt);
  for (long long j = 0; j < nx; ++j) {
    int idx[3] = {(int)(j % n), d >= 2 ? (int)((j / n) % n) : 0, d == 3 ? (int)(j / ((long long)n * n)) : 0};
    double mu = 1.0;
    for (int a = 0; a < d; ++a) mu *= m1[idx[a]];
    double nu = 0.0;
    for (int a = 0; a < d; ++a) {
      double t = k1[idx[a]];
      for (int b = 0; b < d; ++b)
        if (b != a) t *= m1[idx[b]];
      nu += t;
    }
    double blk[NT_BIG * NT_BIG];
    for (int i = 0; i < nt * nt; ++i) blk[i] = mu * h->Kt[i] + nu * L.tau * h->Mh[i];
    if (!invert(nt, blk)) return fail(h, ST_EINVAL, "singular slab block at mode %lld", j);
    for (int i = 0; i < nt * nt; ++i) {
      G[(size_t)j * nt * nt + i] = blk[i];
      G32[(size_t)j * nt * nt + i] = (float)blk[i];
    }
  }
  std::vector<double> Sp((size_t)n * n);
  std::vector<float> Sp32((size_t)n * n);
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < n; ++i) {
      Sp[(size_t)k * n + i] = sc * std::sin(PI * (k + 1.0) * (i + 1.0) / (n + 1));
      Sp32[(size_t)k * n + i] = (float)Sp[(size_t)k * n + i];
    }
  if (twice_folded_ok(n, 4)) {
    // twice-folded blocks: odd modes O[s][i] = S[2s+1][i+1], even E[s][i] = S[2s+2][i+1] on even i = 2p (mat 0, 2)
    // and odd i = 2p + 1 (mat 1, 3), rows s < h/2 and contraction p < h/2; the even block has no column
    // i = h - 1 and its middle row s = h/2 - 1 vanishes on odd i (both stored as exact zeros)
    const int q = half / 2, KB = q / 16, NC = q / 4;
    auto M = [&](int mat, int srow, int p) -> double {
      const int i = mat & 1 ? 2 * p + 1 : 2 * p;
      const int k = mat < 2 ? 2 * srow + 1 : 2 * srow + 2;
      if (mat == 3 && (i >= half - 1 || srow == q - 1)) return 0.0;
      return sc * std::sin(PI * (double)k * (i + 1.0) / (n + 1));
    };
    const size_t len2 = (size_t)2 * 4 * KB * NC * 64;
    std::vector<double> f2(len2);
    std::vector<float> f2_32(len2);
    for (int dir = 0; dir < 2; ++dir)
      for (int mat = 0; mat < 4; ++mat)
        for (int kb = 0; kb < KB; ++kb)
          for (int ib = 0; ib < NC; ++ib)
            for (int lane = 0; lane < 64; ++lane) {
              const size_t o = ((((size_t)dir * 4 + mat) * KB + kb) * NC + ib) * 64 + lane;
              // operand lane: row lane % 16 of block kb, contraction index 4 ib + lane / 16
              const int cc = ib * 4 + (lane >> 4);
              const int r8 = kb * 16 + twice_fold_row(8, lane & 15), r4 = kb * 16 + twice_fold_row(4, lane & 15);
              f2[o] = dir == 0 ? M(mat, r8, cc) : M(mat, cc, r8);
              f2_32[o] = (float)(dir == 0 ? M(mat, r4, cc) : M(mat, cc, r4));
            }
    if (twice_folded_ok(n, 8)) {
      HIPCHK(h, hipMalloc(&L.S2_64, len2 * sizeof(double)));
      HIPCHK(h, hipMemcpy(L.S2_64, f2.data(), len2 * sizeof(double), hipMemcpyHostToDevice));
    }
    HIPCHK(h, hipMalloc(&L.S2_32, len2 * sizeof(float)));
    HIPCHK(h, hipMemcpy(L.S2_32, f2_32.data(), len2 * sizeof(float), hipMemcpyHostToDevice));
    // bf16 operands of v_mfma_f32_16x16x16_bf16: lane supplies operand row lane % 16 (logical row
    // twice_fold_row) and the four contraction indices 4 (4 c + e) + lane / 16, e < 4, of chunk c
    std::vector<uint16_t> f2_16((size_t)2 * 4 * KB * KB * 64 * 4);
    for (int dir = 0; dir < 2; ++dir)
      for (int mat = 0; mat < 4; ++mat)
        for (int kb = 0; kb < KB; ++kb)
          for (int c = 0; c < KB; ++c)
            for (int lane = 0; lane < 64; ++lane)
              for (int e = 0; e < 4; ++e) {
                const size_t o = (((((size_t)dir * 4 + mat) * KB + kb) * KB + c) * 64 + lane) * 4 + e;
                const int rr = kb * 16 + twice_fold_row(4, lane & 15);
                const int cc = 4 * (4 * c + e) + (lane >> 4);
                f2_16[o] = bf16_round(dir == 0 ? M(mat, rr, cc) : M(mat, cc, rr));
              }
    HIPCHK(h, hipMalloc(&L.S2_16, f2_16.size() * sizeof(uint16_t)));
    HIPCHK(h, hipMemcpy(L.S2_16, f2_16.data(), f2_16.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  }
  HIPCHK(h, hipMalloc(&L.Sp64, Sp.size() * sizeof(double)));
  HIPCHK(h, hipMalloc(&L.Sp32, Sp32.size() * sizeof(float)));
  HIPCHK(h, hipMemcpy(L.Sp64, Sp.data(), Sp.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(L.Sp32, Sp32.data(), Sp32.size() * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(h, hipMalloc(&L.S16, frag16.size() * sizeof(uint16_t)));
  HIPCHK(h, hipMemcpy(L.S16, frag16.data(), frag16.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  HIPCHK(h, hipMalloc(&L.S64, frag.size() * sizeof(double)));
  HIPCHK(h, hipMalloc(&L.S32, frag32.size() * sizeof(float)));
  HIPCHK(h, hipMalloc(&L.G64, G.size() * sizeof(double)));
  HIPCHK(h, hipMalloc(&L.G32, G32.size() * sizeof(float)));
  HIPCHK(h, hipMemcpy(L.S64, frag.data(), frag.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(L.S32, frag32.data(), frag32.size() * sizeof(float), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(L.G64, G.data(), G.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(L.G32, G32.data(), G32.size() * sizeof(float), hipMemcpyHostToDevice));
  return ST_OK;
}

// --------------------------------------------------------------- precisions
template <typename T> const T* Sof(const Level& L);
template <> const double* Sof<double>(const Level& L) { return L.S64; }
template <> const float* Sof<float>(const Level& L) { return L.S32; }
template <typename T> const T* Eigof(const Level& L);
template <> const double* Eigof<double>(const Level& L) { return L.eig64; }
template <> const float* Eigof<float>(const Level& L) { return L.eig32; }
template <typename T> const T* S2of(const Level& L);
template <> const double* S2of<double>(const Level& L) { return L.S2_64; }
template <> const float* S2of<float>(const Level& L) { return L.S2_32; }
template <typename T> const T* SPof(const Level& L);
template <> const double* SPof<double>(const Level& L) { return L.Sp64; }
template <> const float* SPof<float>(const Level& L) { return L.Sp32; }
template <typename T> const T* Gof(const Level& L);
template <> const double* Gof<double>(const Level& L) { return L.G64; }
template <> const float* Gof<float>(const Level& L) { return L.G32; }

template <typename T>
ResidArgs<T> resid_args(const st_mg* h, const Level& L, bool transpose) {
  ResidArgs<T> a{};
  const int nt = h->nt;
  for (int l = 0; l < nt; ++l)
    for (int k = 0; k < nt; ++k) {
      a.K[l * nt + k] = (T)(transpose ? h->Kt[k * nt + l] : h->Kt[l * nt + k]);
      a.M[l * nt + k] = (T)(L.tau * h->Mh[l * nt + k]);
    }
  for (int l = 0; l < nt; ++l) {
    a.ca[l] = (T)(transpose ? h->cb[l] : h->ca[l]);
    a.cb[l] = (T)(transpose ? h->ca[l] : h->cb[l]);
  }
  a.wm[0] = a.wm[2] = (T)(L.h / 6.0);
  a.wm[1] = (T)(4.0 * L.h / 6.0);
  a.wk[0] = a.wk[2] = (T)(-1.0 / L.h);
  a.wk[1] = (T)(2.0 / L.h);
  a.n = L.n;
  a.nx = L.nx;
  a.N = L.N;
  a.batch = h->p.batch;
  a.dir = transpose ? +1 : -1;
  return a;
}

template <typename T>
TransferArgs<T> transfer_args(const st_mg* h, int lf) {
  const Level& F = h->lv[lf];
  const Level& C = h->lv[lf + 1];
  TransferArgs<T> a{};
  for (int i = 0; i < h->nt * h->nt; ++i) {
    a.R1T[i] = (T)h->R1T[i];
    a.R2T[i] = (T)h->R2T[i];
  }
  a.nf = F.n;
  a.nc = C.n;
  a.nxf = F.nx;
  a.nxc = C.nx;
  a.Nc = C.N;
  a.batch = h->p.batch;
  return a;
}

template <typename T>
RhsArgs<T> rhs_args(const st_mg* h) {
  const Level& L = h->lv[0];
  RhsArgs<T> a{};
  for (int l = 0; l < h->nt; ++l) {
    a.ints[l] = (T)(L.tau * h->ints[l]);
    a.ca[l] = (T)h->ca[l];
  }
  a.wm[0] = a.wm[2] = (T)(L.h / 6.0);
  a.wm[1] = (T)(4.0 * L.h / 6.0);
  a.n = L.n;
  a.nx = L.nx;
  a.N = L.N;
  a.batch = h->p.batch;
  return a;
}

template <typename T>
MeshRhsArgs<T> mesh_rhs_args(const st_mg* h);

template <typename T>
const T* gen_table(const st_mg* h);
template <>
const double* gen_table<double>(const st_mg* h) { return h->gen64; }
template <>
const float* gen_table<float>(const st_mg* h) { return h->gen32; }

template <typename T>
GenArgs<T> gen_args(const st_mg* h, const Level& L, bool transpose) {
  const int nt = h->nt, q = nt * nt;
  const T* t = gen_table<T>(h);
  GenArgs<T> a{};
  a.K = t + (transpose ? q : 0);
  a.M = t + 2 * q;
  a.ca = t + 3 * q + (transpose ? nt : 0);
  a.cb = t + 3 * q + (transpose ? 0 : nt);
  a.ints = t + 3 * q + 2 * nt;
  a.tau = (T)L.tau;
  a.wm[0] = a.wm[2] = (T)(L.h / 6.0);
  a.wm[1] = (T)(4.0 * L.h / 6.0);
  a.wk[0] = a.wk[2] = (T)(-1.0 / L.h);
  a.wk[1] = (T)(2.0 / L.h);
  a.n = L.n;
  a.nx = L.nx;
  a.N = L.N;
  a.batch = h->p.batch;
  a.dir = transpose ? +1 : -1;
  a.nt = nt;
  return a;
}

template <typename T>
GenTransfer<T> gen_transfer(const st_mg* h, int lf) {
  const Level& F = h->lv[lf];
  const Level& C = h->lv[lf + 1];
  const int nt = h->nt, q = nt * nt;
  const T* t = gen_table<T>(h);
  GenTransfer<T> a{};
  a.R1T = t + 3 * q + 3 * nt;
  a.R2T = t + 4 * q + 3 * nt;
  a.nf = F.n;
  a.nc = C.n;
  a.nxf = F.nx;
  a.nxc = C.nx;
  a.Nc = C.N;
  a.batch = h->p.batch;
  a.nt = nt;
  return a;
}

unsigned resid_blocks(const st_mg* h, const Level& L) {
  if (h->mesh) return mesh_blocks_per_slab(L.nx);
  return high_order(h) ? residual_gen_blocks_per_slab(L.nx) : residual_blocks_per_slab(h->p.dim, L.n, L.nx, h->nt, (long long)h->p.batch * L.N);
}

// ------------------------------------------------------------ P1 mesh data
template <typename T>
MeshOp<T> mesh_op(const st_mg* h, int rx);
template <>
MeshOp<double> mesh_op<double>(const st_mg* h, int rx) {
  const MeshDev& m = h->md[(size_t)rx];
  return {m.rowptr, m.col, m.mv64, m.kv64, m.dg64, m.nx, m.ecol, m.emk64, m.ew, m.hoff, m.hcol, m.lcol, m.ldiag, m.hmax};
}
template <>
MeshOp<float> mesh_op<float>(const st_mg* h, int rx) {
  const MeshDev& m = h->md[(size_t)rx];
  return {m.rowptr, m.col, m.mv32, m.kv32, m.dg32, m.nx, m.ecol, m.emk32, m.ew, m.hoff, m.hcol, m.lcol, m.ldiag, m.hmax};
}
template <typename T>
const T* mesh_w(const st_mg* h, int rx);
template <>
const double* mesh_w<double>(const st_mg* h, int rx) { return h->md[(size_t)rx].w64; }
template <>
const float* mesh_w<float>(const st_mg* h, int rx) { return h->md[(size_t)rx].w32; }
// interpolation from refinement level rx - 1 to rx
MeshXfer mesh_xfer(const st_mg* h, int rx) {
  const MeshDev& m = h->md[(size_t)rx];
  return {m.p, m.rrow, m.rcol, m.nx, m.nxc, m.rell, m.rw, m.rhoff, m.rhcol, m.rloc, m.rhmax};
}
template <typename T>
const T* dense_inv(const Level& L, bool own);
template <>
const double* dense_inv<double>(const Level& L, bool own) { return own && L.C64 ? L.C64 : L.D64; }
template <>
const float* dense_inv<float>(const Level& L, bool own) { return own && L.C32 ? L.C32 : L.D32; }

template <typename T>
MeshRhsArgs<T> mesh_rhs_args(const st_mg* h) {
  const Level& L = h->lv[0];
  MeshRhsArgs<T> a{};
  a.op = mesh_op<T>(h, L.n);
  for (int l = 0; l < h->nt; ++l) {
    a.ints[l] = (T)(L.tau * h->ints[l]);
    a.ca[l] = (T)h->ca[l];
  }
  a.N = L.N;
  a.batch = h->p.batch;
  return a;
}

// ------------------------------------------------------------------ operators
// partial / norm_out: where the per-workgroup partial sums of r^2 and the
// per-RHS sums go when norms is set (nullptr: the workspace's buffers).
template <typename Tin, typename Tout>
int op_residual(st_mg* h, int l, bool transpose, const Tin* u, const Tin* F, Tout* r, bool norms,
                hipStream_t s, double* partial = nullptr, double* norm_out = nullptr) {
  const Level& L = h->lv[l];
  if (partial == nullptr) partial = h->partial;
  if (norm_out == nullptr) norm_out = h->norm_dev;
  if (h->mesh) {
    const ResidArgs<Tin> ra = resid_args<Tin>(h, L, transpose);
    MeshResidArgs<Tin> a{};
    a.op = mesh_op<Tin>(h, L.n);
    for (int i = 0; i < NT_MAX * NT_MAX; ++i) {
      a.K[i] = ra.K[i];
      a.M[i] = ra.M[i];
    }
    for (int i = 0; i < NT_MAX; ++i) {
      a.ca[i] = ra.ca[i];
      a.cb[i] = ra.cb[i];
    }
    a.N = L.N;
    a.batch = h->p.batch;
    a.dir = ra.dir;
    ProfScope ps(h, ST_PROF_RESIDUAL, l, s);
    HIPCHK(h, (launch_mesh_residual<Tin, Tout>(h->nt, u, F, r, a, norms ? partial : nullptr, s)));
  } else if (high_order(h)) {
    ProfScope ps(h, ST_PROF_RESIDUAL, l, s);
    HIPCHK(h, (launch_residual_gen<Tin, Tout>(h->p.dim, u, F, r, gen_args<Tin>(h, L, transpose),
                                              norms ? partial : nullptr, s)));
  } else {
    const ResidArgs<Tin> a = resid_args<Tin>(h, L, transpose);
    ProfScope ps(h, ST_PROF_RESIDUAL, l, s);
    HIPCHK(h, (launch_residual<Tin, Tout>(h->p.dim, h->nt, u, F, r, a, norms ? partial : nullptr, s)));
  }
  if (norms) {
    ProfScope ps(h, ST_PROF_OTHER, l, s);
    const long long per = (long long)resid_blocks(h, L) * L.N;
    HIPCHK(h, launch_norm_final(partial, per, h->p.batch, norm_out, s));
  }
  return ST_OK;
}

// The level's launch shape of the twice-folded passes with the device's CU count.
PassShape level_shape(const st_mg* h, const Level& L) {
  PassShape sh = L.shape;
  sh.cus = h->cus;
  return sh;
}

// Inner-cycle levels of ST_MIXED_BF16 run their transforms on the bf16 matrix cores.
template <typename T>
bool bf16_level(const st_mg* h, const Level& L) {
  return sizeof(T) == 4 && h->p.precision == ST_MIXED_BF16 && L.hb <= 8;
}

// The slab-resident kernel applies to this level (2-D, twice-folded sizes, N_t <= 2, not a BF16 level)
// and is its chosen family.
template <typename T>
bool slab_capable(const st_mg* h, const Level& L) {
  return h->p.dim == 2 && !high_order(h) && !bf16_level<T>(h, L) && S2of<T>(L) != nullptr &&
         slab_solve2_lds(2, L.n, h->nt, (int)sizeof(T)) > 0;
}
// 3-D levels whose (slab, x-mode) planes fit the slab-resident kernel: forward
// x pass into the x-mode-major layout, one workgroup per plane, inverse x pass.
template <typename T>
bool xslab_capable(const st_mg* h, const Level& L) {
  return h->p.dim == 3 && !high_order(h) && !bf16_level<T>(h, L) && S2of<T>(L) != nullptr &&
         slab_solve2_lds(3, L.n, h->nt, (int)sizeof(T)) > 0;
}
template <typename T>
bool xslab_level(const st_mg* h, const Level& L) {
  const int impl = L.impl >= 0 ? L.impl : h->impl;
  return impl == TRANSFORM_XSLAB && xslab_capable<T>(h, L);
}
template <typename T>
bool slab_level(const st_mg* h, const Level& L) {
  const int impl = L.impl >= 0 ? L.impl : h->impl;
  return impl == TRANSFORM_SLAB && slab_capable<T>(h, L);
}

// x = D^{-1} src written into dst with `mode` (store / += omega x / = omega x):
// folded DST passes along the leading axes, the fused forward/time-solve/inverse
// pass along the slowest axis, then the inverse passes.  Intermediate data
// alternate between the buffers A and B; src is only read.
template <typename T>
int op_block_solve(st_mg* h, int l, bool transpose, const T* src, T* dst, int mode, T omega, T* A,
                   T* B, hipStream_t s, bool x_done = false) {
  const Level& L = h->lv[l];
  const int d = h->p.dim, n = L.n, nt = h->nt;
  const long long slabs = (long long)h->p.batch * L.N;
  const long long nn = n;
  auto pass = [&](int axis, bool inv, const T* in, T* out, int md, T om) -> int {
    long long inner = 1;
    for (int i = 0; i < axis; ++i) inner *= nn;
    long long rest = 1;
    for (int i = axis + 1; i < d; ++i) rest *= nn;
    const long long ncols = slabs * nt * rest * inner;
    const int kind = axis == 0 ? (inv ? ST_PROF_PASS_INV : ST_PROF_PASS_FWD)
                               : (inv ? ST_PROF_PASS_INV_Y : ST_PROF_PASS_FWD_Y);
    ProfScope ps(h, kind, l, s);
    if (bf16_level<T>(h, L) && L.S2_16) {
      HIPCHK(h, launch_pass_reg2<float>(n, inv, (const float*)in, (float*)out, (const float*)L.S2_16, inner, ncols,
                                        (float)om, md, s, true, level_shape(h, L)));
      return ST_OK;
    }
    if (bf16_level<T>(h, L)) {
      HIPCHK(h, launch_pass_bf16(L.hb, inv, (const float*)in, (float*)out, L.S16, n, inner, ncols, (float)om, md, s));
      return ST_OK;
    }
    int impl = L.impl >= 0 ? L.impl : h->impl;
    if (impl == TRANSFORM_SLAB || impl == TRANSFORM_XSLAB) impl = TRANSFORM_AUTO;   // levels the slab kernel does not take
    if ((impl == TRANSFORM_REG2 || impl == TRANSFORM_AUTO) && S2of<T>(L)) {
      HIPCHK(h, launch_pass_reg2<T>(n, inv, in, out, S2of<T>(L), inner, ncols, om, md, s, false, level_shape(h, L)));
      return ST_OK;
    }
    HIPCHK(h, launch_dst_pass<T>(impl, L.hb, axis == 0, inv, in, out, Sof<T>(L), n, inner, ncols, om, md, s));
    return ST_OK;
  };
  // per-mode blocks from the eigenvalues for the twice-folded fused pass
  ModeEig<T> me{};
  const ModeEig<T>* mep = nullptr;
  if (nt <= NT_MAX) {
    me.eig = Eigof<T>(L);
    for (int i = 0; i < nt * nt; ++i) {
      me.K[i] = (T)h->Kt[i];
      me.M[i] = (T)(L.tau * h->Mh[i]);
    }
    mep = &me;
  }
  auto fused = [&](const T* in, T* out, int md, T om) -> int {
    long long inner = 1;
    for (int i = 0; i < d - 1; ++i) inner *= nn;
    ProfScope ps(h, ST_PROF_FUSED, l, s);
    if (bf16_level<T>(h, L) && L.S2_16) {
      HIPCHK(h, launch_fused_pair2<float>(n, nt, (const float*)in, (float*)out, (const float*)L.S2_16,
                                          (const float*)Gof<T>(L), inner, slabs, transpose ? 1 : 0, (float)om, md, s,
                                          true, (const ModeEig<float>*)mep, level_shape(h, L)));
      return ST_OK;
    }
    if (bf16_level<T>(h, L)) {
      HIPCHK(h, launch_fused_bf16(L.hb, nt, (const float*)in, (float*)out, L.S16, (const float*)Gof<T>(L), n, inner,
                                  slabs, transpose ? 1 : 0, (float)om, md, s));
      return ST_OK;
    }
    int impl = L.impl >= 0 ? L.impl : h->impl;
    if (impl == TRANSFORM_SLAB || impl == TRANSFORM_XSLAB) impl = TRANSFORM_AUTO;
    if ((impl == TRANSFORM_REG2 || impl == TRANSFORM_AUTO) && S2of<T>(L)) {
      HIPCHK(h, launch_fused_pair2<T>(n, nt, in, out, S2of<T>(L), Gof<T>(L), inner, slabs, transpose ? 1 : 0, om, md,
                                      s, false, mep, level_shape(h, L)));
      return ST_OK;
    }
    HIPCHK(h, launch_dst_fused<T>(impl, L.hb, nt, in, out, Sof<T>(L), Gof<T>(L), n, inner, slabs,
                                  transpose ? 1 : 0, om, md, s));
    return ST_OK;
  };
  if (xslab_level<T>(h, L)) {
    // x pass into [slab][kx][l][z][y], a (z, y) block solve per (slab, kx) in LDS, inverse x pass (+ update)
    // (x_done: src already holds the x-transformed values in that layout, in A)
    const long long lps = (long long)nt * nn * nn;
    const long long ncols = slabs * lps;
    if (!x_done) {
      ProfScope ps(h, ST_PROF_PASS_FWD, l, s);
      HIPCHK(h, launch_pass_reg2<T>(n, false, src, A, S2of<T>(L), 1, ncols, T(1), MODE_STORE, s, false,
                                    level_shape(h, L), lps));
    }
    {
      ProfScope ps(h, ST_PROF_FUSED, l, s);
      HIPCHK(h, launch_slab_solve2<T>(n, nt, A, A, S2of<T>(L), Gof<T>(L), slabs, transpose ? 1 : 0, T(1), MODE_STORE,
                                      s, &me));
    }
    ProfScope ps(h, ST_PROF_PASS_INV, l, s);
    HIPCHK(h, launch_pass_reg2<T>(n, true, A, dst, S2of<T>(L), 1, ncols, omega, mode, s, false, level_shape(h, L),
                                  lps));
    return ST_OK;
  }
  if (slab_level<T>(h, L)) {
    ProfScope ps(h, ST_PROF_FUSED, l, s);
    HIPCHK(h, launch_slab_solve2<T>(n, nt, src, dst, S2of<T>(L), Gof<T>(L), slabs, transpose ? 1 : 0, omega, mode,
                                    s));
    return ST_OK;
  }
  if (high_order(h)) {
    // N_t > NT_MAX: transform every axis, per-mode time solve, inverse transforms
    const T* cur = src;
    T* bufs[2] = {A, B};
    for (int ax = 0; ax < d; ++ax) {
      CHK(pass(ax, false, cur, bufs[ax & 1], MODE_STORE, T(1)));
      cur = bufs[ax & 1];
    }
    T* spec = bufs[(d - 1) & 1];
    {
      ProfScope ps(h, ST_PROF_FUSED, l, s);
      HIPCHK(h, launch_time_solve_gen<T>(spec, spec, Gof<T>(L), L.nx, nt, slabs, transpose ? 1 : 0, T(1),
                                         MODE_STORE, s));
    }
    cur = spec;
    for (int ax = d - 1; ax >= 0; --ax) {
      if (ax == 0) return pass(0, true, cur, dst, mode, omega);
      T* nxt = (cur == A) ? B : A;
      CHK(pass(ax, true, cur, nxt, MODE_STORE, T(1)));
      cur = nxt;
    }
    return ST_OK;
  }
  if (d == 1) return fused(src, dst, mode, omega);
  if (d == 2) {
    // x_done: src already holds the forward x pass of the right-hand side, in A
    if (!x_done) CHK(pass(0, false, src, A, MODE_STORE, T(1)));
    CHK(fused(A, A, MODE_STORE, T(1)));
    return pass(0, true, A, dst, mode, omega);
  }
  CHK(pass(0, false, src, A, MODE_STORE, T(1)));
  CHK(pass(1, false, A, B, MODE_STORE, T(1)));
  CHK(fused(B, B, MODE_STORE, T(1)));
  CHK(pass(1, true, B, A, MODE_STORE, T(1)));
  return pass(0, true, A, dst, mode, omega);
}

// Space-time transfer between level lf and lf + 1 on a mesh: the mesh
// interpolation in space for full coarsening, none for semi-coarsening.
template <typename T>
MeshTransferArgs<T> mesh_transfer(const st_mg* h, int lf) {
  const Level& F = h->lv[lf];
  const Level& C = h->lv[lf + 1];
  MeshTransferArgs<T> a{};
  for (int i = 0; i < h->nt * h->nt; ++i) {
    a.R1T[i] = (T)h->R1T[i];
    a.R2T[i] = (T)h->R2T[i];
  }
  a.full = F.kind == 'f' ? 1 : 0;
  if (a.full) {
    a.x = mesh_xfer(h, F.n);
    a.w = mesh_w<T>(h, F.n);
  } else {
    a.x = MeshXfer{nullptr, nullptr, nullptr, F.nx, F.nx, nullptr, 0, nullptr, nullptr, nullptr, 0};
    a.w = nullptr;
  }
  a.Nc = C.N;
  a.batch = h->p.batch;
  return a;
}

template <typename T>
int op_restrict(st_mg* h, int l, const T* rf, T* Fc, hipStream_t s) {
  ProfScope ps(h, ST_PROF_RESTRICT, l, s);
  if (h->mesh) {
    HIPCHK(h, launch_mesh_restrict<T>(h->nt, rf, Fc, mesh_transfer<T>(h, l), s));
    return ST_OK;
  }
  if (high_order(h)) {
    HIPCHK(h, launch_restrict_gen<T>(h->p.dim, h->lv[l].kind == 'f', rf, Fc, gen_transfer<T>(h, l), s));
    return ST_OK;
  }
  const TransferArgs<T> a = transfer_args<T>(h, l);
  HIPCHK(h, launch_restrict<T>(h->p.dim, h->nt, h->lv[l].kind == 'f', rf, Fc, a, s));
  return ST_OK;
}

// F_c = P^T (F - L u) from level l to l + 1: on fully coarsened 2-D/3-D levels
// the residual kernel restricts its own output (per-slab parts in r, n_c^d /
// n^d of its size, then the pair sums), else the residual into r followed by
// the restriction.
template <typename T>
bool rr_level(const st_mg* h, int l) {
  if (h->mesh || high_order(h) || l + 1 >= (int)h->lv.size() || h->lv[l].kind != 'f') return false;
  if (!(h->lv[l].rr >= 0 ? h->lv[l].rr != 0 : h->rr)) return false;
  ResRestrictShape sh;
  return resid_restrict_shape(h->p.dim, h->nt, h->lv[l].n, h->lv[l + 1].n, (long long)h->p.batch * h->lv[l].N,
                              (int)sizeof(T), sh);
}

template <typename T>
int op_resid_restrict(st_mg* h, int l, bool transpose, const T* u, const T* F, T* r, T* Fc, hipStream_t s) {
  if (rr_level<T>(h, l)) {
    const ResidArgs<T> a = resid_args<T>(h, h->lv[l], transpose);
    const TransferArgs<T> t = transfer_args<T>(h, l);
    ProfScope ps(h, ST_PROF_RESID_RESTRICT, l, s);
    HIPCHK(h, launch_resid_restrict<T>(h->p.dim, h->nt, u, F, Fc, r, a, t, s));
    return ST_OK;
  }
  CHK((op_residual<T, T>(h, l, transpose, u, F, r, false, s)));
  return op_restrict<T>(h, l, r, Fc, s);
}

template <typename T>
int op_prolong(st_mg* h, int l, const T* ec, T* uf, hipStream_t s) {
  ProfScope ps(h, ST_PROF_PROLONG, l, s);
  if (h->mesh) {
    HIPCHK(h, launch_mesh_prolong<T>(h->nt, ec, uf, mesh_transfer<T>(h, l), s));
    return ST_OK;
  }
  if (high_order(h)) {
    HIPCHK(h, launch_prolong_gen<T>(h->p.dim, h->lv[l].kind == 'f', ec, uf, gen_transfer<T>(h, l), s));
    return ST_OK;
  }
  const TransferArgs<T> a = transfer_args<T>(h, l);
  HIPCHK(h, launch_prolong<T>(h->p.dim, h->nt, h->lv[l].kind == 'f', ec, uf, a, s));
  return ST_OK;
}

// ------------------------------------------------------ spatial multigrid
// Coefficients of the slab matrix on spatial sub-level j of level l and the
// inverse of its N_t x N_t node block D^x = M_jj K + K_jj M (M_jj = (2h/3)^d,
// K_jj = d (2/h) (2h/3)^(d-1): the diagonals of the Q1 matrices), transposed
// for the adjoint.  On a one-node sub-level D^x is the whole of A.
template <typename T>
SpatialArgs<T> spatial_args(const st_mg* h, const Level& L, const Level::Sub& S, bool transpose, int op,
                            int upd, T scale, bool x_zero, T omega) {
  SpatialArgs<T> a{};
  const int nt = h->nt, d = h->p.dim;
  double K[NT_MAX * NT_MAX], M[NT_MAX * NT_MAX], Dm[NT_MAX * NT_MAX];
  const double mjj = std::pow(2.0 * S.h / 3.0, d);
  const double kjj = d * (2.0 / S.h) * std::pow(2.0 * S.h / 3.0, d - 1);
  for (int l = 0; l < nt; ++l)
    for (int k = 0; k < nt; ++k) {
      K[l * nt + k] = transpose ? h->Kt[k * nt + l] : h->Kt[l * nt + k];
      M[l * nt + k] = L.tau * h->Mh[l * nt + k];
      Dm[l * nt + k] = mjj * K[l * nt + k] + kjj * M[l * nt + k];
    }
  invert(nt, Dm);
  for (int i = 0; i < nt * nt; ++i) {
    a.K[i] = (T)K[i];
    a.M[i] = (T)M[i];
    a.Dinv[i] = (T)Dm[i];
  }
  a.wm[0] = a.wm[2] = (T)(S.h / 6.0);
  a.wm[1] = (T)(4.0 * S.h / 6.0);
  a.wk[0] = a.wk[2] = (T)(-1.0 / S.h);
  a.wk[1] = (T)(2.0 / S.h);
  a.n = S.n;
  a.nx = S.nx;
  a.slabs = (long long)h->p.batch * L.N;
  a.omega = omega;
  a.scale = scale;
  a.op = op;
  a.upd = upd;
  a.x_zero = x_zero ? 1 : 0;
  return a;
}

template <typename T>
int op_spatial(st_mg* h, int l, int j, bool transpose, const T* x, const T* f, const T* base, T* out, int op,
               int upd, T scale, bool x_zero, T omega, hipStream_t s) {
  const Level& L = h->lv[l];
  const SpatialArgs<T> a = spatial_args<T>(h, L, L.sub[j], transpose, op, upd, scale, x_zero, omega);
  ProfScope ps(h, ST_PROF_JACOBI, l, s);
  HIPCHK(h, launch_spatial<T>(h->p.dim, h->nt, x, f, base, out, a, s));
  return ST_OK;
}

// One spatial cycle on sub-level j of level l for every slab, from x = 0:
// x = (I - M^x) A_j^{-1} f.  When `dst` is given (j = 0) the result is written
// there as dst = x (MODE_STORE), dst = omega x (MODE_SET_SCALED) or
// dst += omega x (MODE_ADD_SCALED), fused into the last Jacobi step;
// otherwise *res points at the sub-level buffer holding x.
template <typename T>
int spatial_cycle(st_mg* h, int l, int j, bool transpose, const T* f, T* dst, int mode, T omega_t, T** res,
                  hipStream_t s) {
  Level& L = h->lv[l];
  const Level::Sub& S = L.sub[j];
  const int d = h->p.dim, nt = h->nt;
  const T om = (T)h->p.omega_x;
  const long long slabs = (long long)h->p.batch * L.N;
  const long long len = slabs * nt * S.nx;
  const int upd_last = mode == MODE_ADD_SCALED ? UPD_ADD : UPD_SET;
  const T sc_last = mode == MODE_STORE ? T(1) : omega_t;
  // The one-kernel tail runs only with nu1x, nu2x >= 2: with nu1x = 1, nu2x = 0
  // it once ended in a memory-aperture fault whose cause is not understood, so
  // the other step counts keep the kernel-per-step path below.
  const bool tail_ok = h->p.nu1x >= 2 && h->p.nu2x >= 2;
  if (tail_ok && spatial_tail_lds(d, S.n, nt, sizeof(T)) > 0 && (int)(L.sub.size() - j) <= TAIL_MAX) {
    // the rest of the cycle fits in LDS: one kernel, one workgroup per slab
    TailArgs<T> ta{};
    const SpatialArgs<T> a0 = spatial_args<T>(h, L, S, transpose, SP_JACOBI, UPD_NONE, T(1), false, om);
    for (int i = 0; i < nt * nt; ++i) {
      ta.K[i] = a0.K[i];
      ta.M[i] = a0.M[i];
    }
    ta.levels = (int)L.sub.size() - j;
    for (int q = 0; q < ta.levels; ++q) {
      const SpatialArgs<T> aq = spatial_args<T>(h, L, L.sub[j + q], transpose, SP_JACOBI, UPD_NONE, T(1), false, om);
      for (int i = 0; i < nt * nt; ++i) ta.Dinv[q][i] = aq.Dinv[i];
      for (int i = 0; i < 3; ++i) {
        ta.wm[q][i] = aq.wm[i];
        ta.wk[q][i] = aq.wk[i];
      }
      ta.n[q] = L.sub[j + q].n;
    }
    ta.slabs = slabs;
    ta.omega = om;
    ta.nu1 = h->p.nu1x;
    ta.nu2 = h->p.nu2x;
    T* target = dst ? dst : (T*)S.X;
    ta.upd = dst ? upd_last : UPD_NONE;
    ta.scale = dst ? sc_last : T(1);
    ProfScope ps(h, ST_PROF_JACOBI, l, s);
    HIPCHK(h, launch_spatial_tail<T>(d, nt, f, dst, target, ta, s));
    if (!dst) *res = (T*)S.X;
    return ST_OK;
  }
  if (S.n == 1) {   // one node: exact N_t x N_t solve per slab
    if (dst) return op_spatial<T>(h, l, j, transpose, nullptr, f, dst, dst, SP_JACOBI, upd_last, sc_last, true, T(1), s);
    CHK(op_spatial<T>(h, l, j, transpose, nullptr, f, nullptr, (T*)S.X, SP_JACOBI, UPD_NONE, T(1), true, T(1), s));
    *res = (T*)S.X;
    return ST_OK;
  }
  T* cur = (T*)S.X;
  T* oth = (T*)S.Y;
  const int nu1 = h->p.nu1x, nu2 = h->p.nu2x;
  for (int i = 0; i < nu1; ++i) {
    CHK(op_spatial<T>(h, l, j, transpose, cur, f, nullptr, i == 0 ? cur : oth, SP_JACOBI, UPD_NONE, T(1), i == 0,
                      om, s));
    if (i > 0) std::swap(cur, oth);
  }
  const Level::Sub& C = L.sub[j + 1];
  if (nu1 == 0) {
    HIPCHK(h, launch_fill<T>(cur, len, s));
    ProfScope ps(h, ST_PROF_XFER_X, l, s);
    HIPCHK(h, launch_restrict_space<T>(d, nt, f, (T*)C.F, S.n, C.n, slabs, s));
  } else {
    CHK(op_spatial<T>(h, l, j, transpose, cur, f, nullptr, oth, SP_DEFECT, UPD_NONE, T(1), false, om, s));
    ProfScope ps(h, ST_PROF_XFER_X, l, s);
    HIPCHK(h, launch_restrict_space<T>(d, nt, oth, (T*)C.F, S.n, C.n, slabs, s));
  }
  T* ec = nullptr;
  CHK(spatial_cycle<T>(h, l, j + 1, transpose, (const T*)C.F, nullptr, MODE_STORE, T(1), &ec, s));
  {
    ProfScope ps(h, ST_PROF_XFER_X, l, s);
    HIPCHK(h, launch_prolong_space<T>(d, nt, ec, cur, S.n, C.n, slabs, s));
  }
  for (int i = 0; i < nu2; ++i) {
    if (dst && i == nu2 - 1)
      return op_spatial<T>(h, l, j, transpose, cur, f, dst, dst, SP_JACOBI, upd_last, sc_last, false, om, s);
    CHK(op_spatial<T>(h, l, j, transpose, cur, f, nullptr, oth, SP_JACOBI, UPD_NONE, T(1), false, om, s));
    std::swap(cur, oth);
  }
  if (dst) {   // no post-smoothing: combine the prolongated iterate into dst
    return op_spatial<T>(h, l, j, transpose, cur, cur, dst, dst, SP_JACOBI, upd_last, sc_last, false, T(0), s);
  }
  *res = cur;
  return ST_OK;
}

bool inexact_level(const st_mg* h, int l) {
  if (h->mesh) return true;
  return h->p.smoother == ST_SMOOTH_SPATIAL_MG && h->lv[l].n > 1;
}

// Exact slab solves on a mesh level by its dense inverse (the coarse mesh, or
// the coarsest level's own mesh), written with `mode` as op_block_solve does.
template <typename T>
int mesh_exact_solve(st_mg* h, int l, bool transpose, const T* src, T* dst, int mode, T omega, hipStream_t s) {
  const Level& L = h->lv[l];
  const bool own = l + 1 == (int)h->lv.size();
  if (L.n != 0 && !own)
    return fail(h, ST_EINVAL, "exact slab solves on a mesh exist on refinement level 0 and on the coarsest level");
  const int m = own && L.cm > 0 ? L.cm : L.dm;
  const int upd = mode == MODE_ADD_SCALED ? UPD_ADD : UPD_SET;
  const T sc = mode == MODE_STORE ? T(1) : omega;
  ProfScope ps(h, ST_PROF_OTHER, l, s);
  HIPCHK(h, launch_mesh_dense<T>(dense_inv<T>(L, own), m, transpose ? 1 : 0, src, dst, dst, upd, sc,
                                 (long long)h->p.batch * L.N, s));
  return ST_OK;
}

// One spatial cycle on a mesh level (sub-level j = refinement level L.n - j),
// from x = 0, with the conventions of spatial_cycle: node-block Jacobi steps,
// P^T / P between refinement levels, the dense slab inverse on the coarse mesh.
template <typename T>
int mesh_spatial_cycle(st_mg* h, int l, int j, bool transpose, const T* f, T* dst, int mode, T omega_t, T** res,
                       hipStream_t s) {
  Level& L = h->lv[l];
  const Level::Sub& S = L.sub[j];
  const int nt = h->nt, rx = S.n;
  const long long slabs = (long long)h->p.batch * L.N;
  const long long len = slabs * nt * S.nx;
  const int upd_last = mode == MODE_ADD_SCALED ? UPD_ADD : UPD_SET;
  const T sc_last = mode == MODE_STORE ? T(1) : omega_t;
  if (rx == 0) {
    ProfScope ps(h, ST_PROF_JACOBI, l, s);
    if (dst) {
      HIPCHK(h, launch_mesh_dense<T>(dense_inv<T>(L, false), L.dm, transpose ? 1 : 0, f, dst, dst, upd_last, sc_last,
                                     slabs, s));
      return ST_OK;
    }
    HIPCHK(h, launch_mesh_dense<T>(dense_inv<T>(L, false), L.dm, transpose ? 1 : 0, f, nullptr, (T*)S.X, UPD_NONE,
                                   T(1), slabs, s));
    *res = (T*)S.X;
    return ST_OK;
  }
  const T om = (T)h->p.omega_x;
  MeshSmoothArgs<T> a{};
  a.op = mesh_op<T>(h, rx);
  for (int l2 = 0; l2 < nt; ++l2)
    for (int k = 0; k < nt; ++k) {
      a.K[l2 * nt + k] = (T)(transpose ? h->Kt[k * nt + l2] : h->Kt[l2 * nt + k]);
      a.M[l2 * nt + k] = (T)(L.tau * h->Mh[l2 * nt + k]);
    }
  a.slabs = slabs;
  auto smooth = [&](const T* x, const T* ff, const T* base, T* out, int op, int upd, T scale, bool x_zero,
                    T omega) -> int {
    MeshSmoothArgs<T> b = a;
    b.omega = omega;
    b.scale = scale;
    b.op_kind = op;
    b.upd = upd;
    b.x_zero = x_zero ? 1 : 0;
    ProfScope ps(h, ST_PROF_JACOBI, l, s);
    HIPCHK(h, launch_mesh_smooth<T>(nt, x, ff, base, out, b, s));
    return ST_OK;
  };
  T* cur = (T*)S.X;
  T* oth = (T*)S.Y;
  const int nu1 = h->p.nu1x, nu2 = h->p.nu2x;
  for (int i = 0; i < nu1; ++i) {
    CHK(smooth(cur, f, nullptr, i == 0 ? cur : oth, SP_JACOBI, UPD_NONE, T(1), i == 0, om));
    if (i > 0) std::swap(cur, oth);
  }
  const Level::Sub& C = L.sub[j + 1];
  const MeshXfer xf = mesh_xfer(h, rx);
  const T* w = mesh_w<T>(h, rx);
  if (nu1 == 0) {
    HIPCHK(h, launch_fill<T>(cur, len, s));
    ProfScope ps(h, ST_PROF_XFER_X, l, s);
    HIPCHK(h, launch_mesh_restrict_space<T>(nt, f, (T*)C.F, xf, w, slabs, s));
  } else {
    CHK(smooth(cur, f, nullptr, oth, SP_DEFECT, UPD_NONE, T(1), false, om));
    ProfScope ps(h, ST_PROF_XFER_X, l, s);
    HIPCHK(h, launch_mesh_restrict_space<T>(nt, oth, (T*)C.F, xf, w, slabs, s));
  }
  T* ec = nullptr;
  CHK(mesh_spatial_cycle<T>(h, l, j + 1, transpose, (const T*)C.F, nullptr, MODE_STORE, T(1), &ec, s));
  {
    ProfScope ps(h, ST_PROF_XFER_X, l, s);
    HIPCHK(h, launch_mesh_prolong_space<T>(nt, ec, cur, xf, w, slabs, s));
  }
  for (int i = 0; i < nu2; ++i) {
    if (dst && i == nu2 - 1) return smooth(cur, f, dst, dst, SP_JACOBI, upd_last, sc_last, false, om);
    CHK(smooth(cur, f, nullptr, oth, SP_JACOBI, UPD_NONE, T(1), false, om));
    std::swap(cur, oth);
  }
  if (dst) {   // no post-smoothing: combine the prolongated iterate into dst
    return smooth(cur, cur, dst, dst, SP_JACOBI, upd_last, sc_last, false, T(0));
  }
  *res = cur;
  return ST_OK;
}

// x = D^{-1} src (exact) or (I - M^x) D^{-1} src (spatial cycle), written into
// dst with `mode` as op_block_solve does.
template <typename T>
int op_smoother_solve(st_mg* h, int l, bool transpose, const T* src, T* dst, int mode, T omega, T* A, T* B,
                      hipStream_t s) {
  if (h->mesh) return mesh_spatial_cycle<T>(h, l, 0, transpose, src, dst, mode, omega, nullptr, s);
  if (inexact_level(h, l)) return spatial_cycle<T>(h, l, 0, transpose, src, dst, mode, omega, nullptr, s);
  return op_block_solve<T>(h, l, transpose, src, dst, mode, omega, A, B, s);
}

// One damped block-Jacobi step of a small level in one kernel: u_out = u_in +
// omega D^{-1}(F - L u_in), u_in treated as zero when u_zero.
template <typename T>
bool small_level(const st_mg* h, int l) {
  const Level& L = h->lv[l];
  if (h->mesh || inexact_level(h, l) || high_order(h)) return false;
  const bool on = L.small >= 0 ? L.small != 0 : h->small;
  return on && smooth_small_lds(h->p.dim, L.n, L.nx, h->nt, sizeof(T)) > 0;
}

template <typename T>
int op_smooth_small(st_mg* h, int l, bool transpose, const T* u_in, T* u_out, const T* F, bool u_zero,
                    hipStream_t s) {
  const Level& L = h->lv[l];
  SmallArgs<T> a{};
  a.r = resid_args<T>(h, L, transpose);
  a.omega = (T)h->p.omega;
  a.transpose = transpose ? 1 : 0;
  a.u_zero = u_zero ? 1 : 0;
  ProfScope ps(h, ST_PROF_SMALL, l, s);
  HIPCHK(h, launch_smooth_small<T>(h->p.dim, h->nt, u_zero ? F : u_in, u_out, F, SPof<T>(L), Gof<T>(L), a, s));
  return ST_OK;
}

// ------------------------------------------------------------------- V-cycle
template <typename T>
T* level_r(st_mg* h, int l) { return (T*)(l == 0 ? h->r0 : h->lv[l].r); }

template <typename T>
int coarsest_solve(st_mg* h, bool transpose, T* u, const T* F, hipStream_t s);

template <>
int coarsest_solve<double>(st_mg* h, bool transpose, double* u, const double* F, hipStream_t s) {
  const int l = (int)h->lv.size() - 1;
  if (h->mesh) return mesh_exact_solve<double>(h, l, transpose, F, u, MODE_SET_SCALED, 1.0, s);
  return op_block_solve<double>(h, l, transpose, F, u, MODE_SET_SCALED, 1.0, (double*)h->tmp,
                                level_r<double>(h, l), s);
}

template <>
int coarsest_solve<float>(st_mg* h, bool transpose, float* u, const float* F, hipStream_t s) {
  const int l = (int)h->lv.size() - 1;
  if (h->mesh && !is_mixed(h)) return mesh_exact_solve<float>(h, l, transpose, F, u, MODE_SET_SCALED, 1.0f, s);
  if (is_mixed(h)) {
    // exact coarsest solve kept in double
    const long long len = h->lv[l].dof(h->nt, h->p.batch);
    HIPCHK(h, launch_cast_f32_f64(F, h->cF64, len, s));
    if (h->mesh)
      CHK(mesh_exact_solve<double>(h, l, transpose, h->cF64, h->cu64, MODE_SET_SCALED, 1.0, s));
    else
      CHK(op_block_solve<double>(h, l, transpose, h->cF64, h->cu64, MODE_SET_SCALED, 1.0, h->ct64,
                                 h->cr64, s));
    HIPCHK(h, launch_cast_f64_f32(h->cu64, u, len, s));
    return ST_OK;
  }
  return op_block_solve<float>(h, l, transpose, F, u, MODE_SET_SCALED, 1.0f, (float*)h->tmp,
                               level_r<float>(h, l), s);
}

template <typename T>
int vcycle(st_mg* h, int l, bool transpose, T* u, const T* F, bool u_zero, bool r_ready, hipStream_t s);

// The residual of this level is fused with the forward x pass of the block solve: 2-D, N_t = 2, the twice-folded
// family (n = 63, 127), exact smoother, and chosen for the level.
template <typename T>
bool rx_level(const st_mg* h, int l) {
  const Level& L = h->lv[l];
  if (h->mesh || inexact_level(h, l) || high_order(h) || bf16_level<T>(h, L) || slab_level<T>(h, L) ||
      small_level<T>(h, l))
    return false;
  const int impl = L.impl >= 0 ? L.impl : h->impl;
  if (impl != TRANSFORM_AUTO && impl != TRANSFORM_REG2) return false;
  const bool on = L.rx >= 0 ? L.rx != 0 : h->rx;
  return on && S2of<T>(L) != nullptr && resid_xfwd_ok(h->p.dim, L.n, h->nt, (int)sizeof(T));
}

// 3-D x-mode-major levels: the residual kernel applies the forward x pass and
// writes the slab solve's layout (autotuned per level like the 2-D fusion).
template <typename T>
bool rx3_level(const st_mg* h, int l) {
  const Level& L = h->lv[l];
  if (h->mesh || inexact_level(h, l) || !xslab_level<T>(h, L)) return false;
  const bool on = L.rx >= 0 ? L.rx != 0 : h->rx;
  return on && resid_xfwd3_ok(L.n, h->nt, (int)sizeof(T));
}

// The fine-level residual norm kernel also applies the forward x pass and leaves the result in the transform
// buffer (in the x-mode-major layout on 3-D levels), where the first pre-smoothing step of the next cycle takes it
// (FP64/FP32 handles, nu1 >= 1).
template <typename T>
bool norm_xhat(const st_mg* h) {
  return !is_mixed(h) && h->p.nu1 >= 1 && (rx_level<T>(h, 0) || rx3_level<T>(h, 0));
}

// One damped block-Jacobi step u += omega D^{-1}(F - L u) on level l (r and A are scratch).
template <typename T>
int smooth_step(st_mg* h, int l, bool transpose, T* u, const T* F, T* r, T* A, hipStream_t s) {
  const T om = (T)h->p.omega;
  if (rx3_level<T>(h, l)) {
    const Level& L = h->lv[l];
    {
      ProfScope ps(h, ST_PROF_RESID_X, l, s);
      HIPCHK(h, launch_resid_xfwd3<T>(L.n, h->nt, u, F, A, resid_args<T>(h, L, transpose), S2of<T>(L), nullptr, s));
    }
    return op_block_solve<T>(h, l, transpose, A, u, MODE_ADD_SCALED, om, A, r, s, true);
  }
  if (rx_level<T>(h, l)) {
    const Level& L = h->lv[l];
    const ResidArgs<T> a = resid_args<T>(h, L, transpose);
    {
      ProfScope ps(h, ST_PROF_RESID_X, l, s);
      HIPCHK(h, launch_resid_xfwd<T>(L.n, u, F, A, a, S2of<T>(L), nullptr, s));
    }
    return op_block_solve<T>(h, l, transpose, A, u, MODE_ADD_SCALED, om, A, r, s, true);
  }
  CHK((op_residual<T, T>(h, l, transpose, u, F, r, false, s)));
  return op_smoother_solve<T>(h, l, transpose, r, u, MODE_ADD_SCALED, om, A, r, s);
}

// V-cycle on a small level: each smoothing step is one kernel that reads one
// iterate buffer and writes the other (level 0 borrows the transform buffer);
// the result is copied back when the step count leaves it in the other buffer.
template <typename T>
int vcycle_small(st_mg* h, int l, bool transpose, T* u, const T* F, bool u_zero, hipStream_t s) {
  const long long len = h->lv[l].dof(h->nt, h->p.batch);
  T* buf[2] = {u, l == 0 ? (T*)h->tmp : (T*)h->lv[l].u2};
  int cur = 0;
  for (int i = 0; i < h->p.nu1; ++i) {
    CHK(op_smooth_small<T>(h, l, transpose, buf[cur], buf[1 - cur], F, u_zero && i == 0, s));
    cur ^= 1;
  }
  if (cur) {
    HIPCHK(h, launch_copy<T>(buf[1], u, len, s));
    cur = 0;
  }
  const Level& C = h->lv[l + 1];
  T* uc = (T*)C.u;
  T* Fc = (T*)C.F;
  T* r = level_r<T>(h, l);
  if (h->p.nu1 == 0 && u_zero) {
    CHK(op_restrict<T>(h, l, F, Fc, s));
    HIPCHK(h, launch_fill<T>(u, len, s));
  } else {
    CHK(op_resid_restrict<T>(h, l, transpose, u, F, r, Fc, s));
  }
  for (int g = 0; g < h->p.gamma; ++g) CHK(vcycle<T>(h, l + 1, transpose, uc, Fc, g == 0, false, s));
  CHK(op_prolong<T>(h, l, uc, u, s));
  for (int i = 0; i < h->p.nu2; ++i) {
    CHK(op_smooth_small<T>(h, l, transpose, buf[cur], buf[1 - cur], F, false, s));
    cur ^= 1;
  }
  if (cur) HIPCHK(h, launch_copy<T>(buf[1], u, len, s));
  return ST_OK;
}

// One cycle on level l (gamma coarse-grid cycles: V or W).  u_zero: u holds no valid data and is treated as 0
// (coarse-level corrections).  r_ready: level_r already holds F - L u.
template <typename T>
int vcycle(st_mg* h, int l, bool transpose, T* u, const T* F, bool u_zero, bool r_ready,
           hipStream_t s) {
  const int last = (int)h->lv.size() - 1;
  if (l == h->tail && l > 0) {
    ProfScope ps(h, ST_PROF_SMALL, l, s);
    HIPCHK(h, launch_coarse_cycle<T>(h->p.dim, h->nt, (const CoarseArgs<T>*)h->tail_args[transpose ? 1 : 0],
                                     h->tail_lds, F, u, h->p.batch, u_zero ? 1 : 0, s));
    return ST_OK;
  }
  if (l == last) return coarsest_solve<T>(h, transpose, u, F, s);
  const T om = (T)h->p.omega;
  T* r = level_r<T>(h, l);
  T* A = (T*)h->tmp;
  if (small_level<T>(h, l)) return vcycle_small<T>(h, l, transpose, u, F, u_zero, s);
  for (int i = 0; i < h->p.nu1; ++i) {
    if (i == 0 && u_zero) {
      CHK(op_smoother_solve<T>(h, l, transpose, F, u, MODE_SET_SCALED, om, A, r, s));
    } else if (i == 0 && r_ready) {
      if (l == 0 && norm_xhat<T>(h))   // the norm kernel left the x-transformed residual in A
        CHK(op_block_solve<T>(h, l, transpose, A, u, MODE_ADD_SCALED, om, A, r, s, true));
      else
        CHK(op_smoother_solve<T>(h, l, transpose, r, u, MODE_ADD_SCALED, om, A, r, s));
    } else {
      CHK(smooth_step<T>(h, l, transpose, u, F, r, A, s));
    }
  }
  const Level& C = h->lv[l + 1];
  T* uc = (T*)C.u;
  T* Fc = (T*)C.F;
  if (h->p.nu1 == 0 && u_zero) {
    CHK(op_restrict<T>(h, l, F, Fc, s));
  } else if (h->p.nu1 == 0 && r_ready) {
    CHK(op_restrict<T>(h, l, r, Fc, s));
  } else {
    CHK(op_resid_restrict<T>(h, l, transpose, u, F, r, Fc, s));
  }
  for (int g = 0; g < h->p.gamma; ++g) CHK(vcycle<T>(h, l + 1, transpose, uc, Fc, g == 0, false, s));
  if (h->p.nu1 == 0 && u_zero) {
    const long long len = h->lv[l].dof(h->nt, h->p.batch);
    // u has no defined content yet: start the correction from zero (a fill
    // kernel rather than a memset node, so the cycle stays graph-capturable)
    HIPCHK(h, launch_fill<T>(u, len, s));
  }
  CHK(op_prolong<T>(h, l, uc, u, s));
  for (int i = 0; i < h->p.nu2; ++i) CHK(smooth_step<T>(h, l, transpose, u, F, r, A, s));
  return ST_OK;
}

int read_norms(st_mg* h, double* out, hipStream_t s) {
  HIPCHK(h, hipMemcpyAsync(out, h->norm_dev, sizeof(double) * h->p.batch, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  for (int b = 0; b < h->p.batch; ++b) out[b] = std::sqrt(out[b]);
  return ST_OK;
}

// Fine-level residual norms ||F - L u|| into h->norm_dev (squared); leaves the
// residual in the buffer the next cycle starts from.
template <typename T>
int fine_residual_norm(st_mg* h, bool transpose, const void* u, const void* F, hipStream_t s) {
  if (is_mixed(h))
    return op_residual<double, float>(h, 0, transpose, (const double*)u, (const double*)F,
                                      (float*)h->F32, true, s);
  if (norm_xhat<T>(h)) {
    const Level& L = h->lv[0];
    const bool x3 = rx3_level<T>(h, 0);
    {
      ProfScope ps(h, ST_PROF_RESID_X, 0, s);
      if (x3)
        HIPCHK(h, launch_resid_xfwd3<T>(L.n, h->nt, (const T*)u, (const T*)F, (T*)h->tmp,
                                        resid_args<T>(h, L, transpose), S2of<T>(L), h->partial, s));
      else
        HIPCHK(h, launch_resid_xfwd<T>(L.n, (const T*)u, (const T*)F, (T*)h->tmp, resid_args<T>(h, L, transpose),
                                       S2of<T>(L), h->partial, s));
    }
    ProfScope ps(h, ST_PROF_OTHER, 0, s);
    const long long per =
        (long long)(x3 ? resid_xfwd3_blocks_per_slab(L.n, h->nt, (long long)h->p.batch * L.N, (int)sizeof(T))
                       : resid_blocks(h, L)) * L.N;
    HIPCHK(h, launch_norm_final(h->partial, per, h->p.batch, h->norm_dev, s));
    return ST_OK;
  }
  return op_residual<T, T>(h, 0, transpose, (const T*)u, (const T*)F, level_r<T>(h, 0), true, s);
}

// One cycle of the outer iteration given that the fine residual is ready:
// FP64/FP32: V-cycle reusing r; mixed: inner float V-cycle on L e = r, u += e.
template <typename T>
int cycle_body(st_mg* h, bool transpose, void* u, const void* F, hipStream_t s) {
  if (is_mixed(h)) {
    CHK(vcycle<float>(h, 0, transpose, (float*)h->e32, (const float*)h->F32, true, false, s));
    const long long len = h->lv[0].dof(h->nt, h->p.batch);
    HIPCHK(h, launch_axpy_f32_f64((double*)u, (const float*)h->e32, len, s));
    return ST_OK;
  }
  return vcycle<T>(h, 0, transpose, (T*)u, (const T*)F, false, true, s);
}

int check_ready(st_mg* h) {
  if (!h) return ST_EINVAL;
  if (!h->ws) return fail(h, ST_EWORKSPACE, "no workspace bound (st_mg_bind_workspace)");
  return ST_OK;
}

// cycle + residual norm, replayed from a hipGraph when graph mode is on
template <typename T>
int cycle_and_norm(st_mg* h, bool transpose, void* u, const void* F, hipStream_t s) {
  if (!h->graph) {
    CHK(cycle_body<T>(h, transpose, u, F, s));
    return fine_residual_norm<T>(h, transpose, u, F, s);
  }
  if (s == nullptr) return fail(h, ST_EINVAL, "graph mode needs a non-default stream");
  GraphCache& g = h->gc;
  if (!(g.exec && g.u == u && g.F == F && g.transpose == (int)transpose && g.stream == s)) {
    if (g.exec) {
      (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
    }
    hipGraph_t graph;
    HIPCHK(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = cycle_body<T>(h, transpose, u, F, s);
    if (rc == ST_OK) rc = fine_residual_norm<T>(h, transpose, u, F, s);
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc != ST_OK) return rc;
    if (e != hipSuccess) return fail(h, ST_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(h, ST_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    g.u = u;
    g.F = F;
    g.transpose = (int)transpose;
    g.stream = s;
  }
  HIPCHK(h, hipGraphLaunch(g.exec, s));
  return ST_OK;
}

template <typename T>
int solve_impl(st_mg* h, bool transpose, void* u, const void* F, double rtol, int maxit, int* iters,
               double* hist, hipStream_t s) {
  const int b = h->p.batch;
  std::vector<double> nrm(b), scale(b), rel(b);
  CHK(fine_residual_norm<T>(h, transpose, u, F, s));
  CHK(read_norms(h, nrm.data(), s));
  for (int i = 0; i < b; ++i) {
    if (!std::isfinite(nrm[i])) {
      if (iters) *iters = 0;
      return fail(h, ST_ENAN, "initial residual norm is not finite (rhs %d)", i);
    }
    scale[i] = nrm[i] > 0 ? nrm[i] : 1.0;
    rel[i] = nrm[i] > 0 ? 1.0 : 0.0;
    if (hist) hist[i] = rel[i];
  }
  int k = 0;
  auto converged = [&]() {
    for (int i = 0; i < b; ++i)
      if (!(rel[i] <= rtol)) return false;
    return true;
  };
  while (k < maxit && !converged()) {
    CHK(cycle_and_norm<T>(h, transpose, u, F, s));
    CHK(read_norms(h, nrm.data(), s));
    ++k;
    for (int i = 0; i < b; ++i) {
      rel[i] = nrm[i] / scale[i];
      if (hist) hist[(size_t)k * b + i] = rel[i];
      if (!std::isfinite(rel[i])) {
        if (iters) *iters = k;
        return fail(h, ST_ENAN, "residual norm is not finite after cycle %d (rhs %d)", k, i);
      }
    }
  }
  if (iters) *iters = k;
  if (!converged()) return fail(h, ST_ENOCONV, "not converged to %g in %d cycles", rtol, maxit);
  return ST_OK;
}

int inner_bytes(const st_mg* h) { return h->p.precision == ST_FP64 ? 8 : 4; }

// Workspace layout (every piece 256-byte aligned).  Returns total bytes and,
// when base != NULL, assigns the pointers.
size_t layout(st_mg* h, char* base) {
  const int b = h->p.batch, nt = h->nt;
  const size_t ib = (size_t)inner_bytes(h);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const long long fine = h->lv[0].dof(nt, b);
  h->tmp = take(fine * ib);
  h->r0 = take(fine * ib);
  for (size_t l = 1; l < h->lv.size(); ++l) {
    Level& L = h->lv[l];
    const long long len = L.dof(nt, b);
    L.u = take(len * ib);
    L.u2 = take(len * ib);
    L.F = take(len * ib);
    L.r = take(len * ib);
  }
  for (size_t l = 0; l < h->lv.size(); ++l) {
    Level& L = h->lv[l];
    if (h->p.smoother != ST_SMOOTH_SPATIAL_MG || (h->mesh ? L.n == 0 : L.n == 1)) continue;
    for (size_t j = 0; j < L.sub.size(); ++j) {
      Level::Sub& S = L.sub[j];
      const long long len = (long long)b * L.N * nt * S.nx;
      S.X = take(len * ib);
      S.Y = (h->mesh ? j + 1 < L.sub.size() : S.n > 1) ? take(len * ib) : nullptr;
      S.F = j > 0 ? take(len * ib) : nullptr;
    }
  }
  if (is_mixed(h)) {
    h->F32 = take(fine * 4);
    h->e32 = take(fine * 4);
    const long long cl = h->lv.back().dof(nt, b);
    h->cu64 = (double*)take(cl * 8);
    h->cF64 = (double*)take(cl * 8);
    h->cr64 = (double*)take(cl * 8);
    h->ct64 = (double*)take(cl * 8);
  }
  const Level& L0 = h->lv[0];
  h->partial_per_batch = std::max<long long>(
      (long long)std::max(resid_blocks(h, L0),
                          h->p.dim == 3 ? resid_xfwd3_blocks_per_slab(L0.n, nt, (long long)b * L0.N, (int)ib) : 0u) *
          L0.N,
      1024);
  h->partial = (double*)take(sizeof(double) * h->partial_per_batch * b);
  h->norm_dev = (double*)take(sizeof(double) * b);
  return off;
}

// Level index and arithmetic of a level operator (no workspace needed).
int check_level_args(st_mg* h, int level, int prec, bool need_next) {
  if (!h) return ST_EINVAL;
  if (level < 0 || level >= (int)h->lv.size() || (need_next && level + 1 >= (int)h->lv.size()))
    return fail(h, ST_EINVAL, "level %d out of range (levels: %zu)", level, h->lv.size());
  if (prec != ST_FP64 && prec != ST_FP32) return fail(h, ST_EINVAL, "prec must be ST_FP64 or ST_FP32");
  if (prec == ST_FP64 && h->p.precision != ST_FP64)
    return fail(h, ST_EINVAL, "FP64 level operators need a handle set up with ST_FP64");
  if (prec == ST_FP32 && h->p.precision == ST_FP64)
    return fail(h, ST_EINVAL, "FP32 level operators need a handle set up with ST_FP32 or ST_MIXED(_BF16)");
  return ST_OK;
}

int check_level(st_mg* h, int level, int prec, bool need_next) {
  if (!h) return ST_EINVAL;
  CHK(check_ready(h));
  return check_level_args(h, level, prec, need_next);
}

// ------------------------------------------------------------------ autotune
// Time one smoothing step of level l (residual + block solve + update, or the
// one-kernel small-level step) for every applicable kernel family and keep the
// fastest.  u, F, r, alt are level-sized scratch buffers; contents are destroyed.
template <typename T>
int tune_level(st_mg* h, int l, T* u, T* F, T* r, T* alt, hipStream_t s) {
  Level& L = h->lv[l];
  const long long len = L.dof(h->nt, h->p.batch);
  HIPCHK(h, launch_fill<T>(u, len, s));
  HIPCHK(h, launch_fill<T>(F, len, s));
  L.shape = PassShape{};
  struct Cand { int small, impl, rx; };
  std::vector<Cand> cands;
  const bool can_small = !high_order(h) && smooth_small_lds(h->p.dim, L.n, L.nx, h->nt, sizeof(T)) > 0;
  if (can_small) cands.push_back({1, TRANSFORM_AUTO, 0});
  cands.push_back({0, TRANSFORM_LDS, 0});
  if (sizeof(T) == 8 && L.hb <= 4) {
    cands.push_back({0, TRANSFORM_AUTO, 0});
    cands.push_back({0, TRANSFORM_REG, 0});   // AUTO is the twice-folded family where it exists
  } else if (sizeof(T) == 4 && L.hb <= 8) {
    cands.push_back({0, TRANSFORM_AUTO, 0});
    cands.push_back({0, TRANSFORM_REG, 0});
  }
  if (slab_capable<T>(h, L)) cands.push_back({0, TRANSFORM_SLAB, 0});
  if (xslab_capable<T>(h, L)) {
    cands.push_back({0, TRANSFORM_XSLAB, 0});
    if (resid_xfwd3_ok(L.n, h->nt, (int)sizeof(T))) cands.push_back({0, TRANSFORM_XSLAB, 1});
  }
  if (!high_order(h) && !bf16_level<T>(h, L) && S2of<T>(L) && resid_xfwd_ok(h->p.dim, L.n, h->nt, (int)sizeof(T)))
    cands.push_back({0, TRANSFORM_AUTO, 1});
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  float best = 1e30f;
  Cand pick = cands.front();
  const bool prof = h->prof;
  h->prof = false;
  // best of five smoothing steps of the level's current choice (ms; 1e30 on failure)
  auto time_step = [&]() -> float {
    auto step = [&]() -> int {
      if (L.small == 1) return op_smooth_small<T>(h, l, false, u, alt, F, false, s);
      return smooth_step<T>(h, l, false, u, F, r, (T*)h->tmp, s);
    };
    int rc = step();
    float ms = 1e30f;
    for (int rep = 0; rep < 5 && rc == ST_OK; ++rep) {
      // the spin holds the stream while the host queues the step, so the
      // events time the kernels and not the launch latency between them
      if (launch_spin(200.0, s) != hipSuccess) {
        rc = ST_EHIP;
        break;
      }
      (void)hipEventRecord(e0, s);
      rc = step();
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      if (rc != ST_OK) break;
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      ms = std::min(ms, t);
    }
    return rc == ST_OK ? ms : 1e30f;
  };
  for (const Cand& c : cands) {
    L.small = c.small;
    L.impl = c.impl;
    L.rx = c.rx;
    const float ms = time_step();
    if (ms < best) {
      best = ms;
      pick = c;
    }
  }
  L.small = pick.small;
  L.impl = pick.impl;
  L.rx = pick.rx;
  // launch shape of the twice-folded passes the pick runs: waves per workgroup
  // of the line passes, persistent grids (workgroups per compute unit) and
  // column groups per workgroup of the fused pass, one knob at a time
  const int impl_pick = pick.impl >= 0 ? pick.impl : h->impl;
  const bool uses_reg2 = !pick.small && !high_order(h) && !slab_level<T>(h, L) &&
                         ((bf16_level<T>(h, L) && L.S2_16) ||
                          ((impl_pick == TRANSFORM_AUTO || impl_pick == TRANSFORM_REG2 ||
                            impl_pick == TRANSFORM_XSLAB) && S2of<T>(L)));
  if (uses_reg2) {
    PassShape bsh = L.shape;
    auto try_shape = [&](const PassShape& c) {
      L.shape = c;
      const float ms = time_step();
      if (ms < best) {
        best = ms;
        bsh = c;
      }
    };
    for (int wpg : {2, 1}) {
      PassShape c = bsh;
      c.wpg = wpg;
      try_shape(c);
    }
    for (int pc : {2, 4, 8}) {
      PassShape c = bsh;
      c.pass_per_cu = pc;
      try_shape(c);
    }
    const int cgmax = h->nt >= 3 ? 1 : 4 / h->nt;
    for (int cg = 1; cg < cgmax; cg *= 2) {
      PassShape c = bsh;
      c.fused_cg = cg;
      try_shape(c);
    }
    for (int pc : {2, 4, 8}) {
      PassShape c = bsh;
      c.fused_per_cu = pc;
      try_shape(c);
    }
    L.shape = bsh;
  }
  // the cycle's pre-restriction defect: residual kernel with the restricting
  // epilogue, or the residual stored and restricted in a second pass
  L.rr = -1;
  T* Fc = l + 1 < (int)h->lv.size() ? (T*)h->lv[l + 1].F : nullptr;
  if (h->rr && Fc != nullptr && rr_level<T>(h, l)) {
    float t2[2] = {1e30f, 1e30f};
    for (int v = 0; v < 2; ++v) {
      L.rr = v;
      int rc = op_resid_restrict<T>(h, l, false, u, F, r, Fc, s);
      for (int rep = 0; rep < 5 && rc == ST_OK; ++rep) {
        if (launch_spin(200.0, s) != hipSuccess) {
          rc = ST_EHIP;
          break;
        }
        (void)hipEventRecord(e0, s);
        rc = op_resid_restrict<T>(h, l, false, u, F, r, Fc, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        if (rc == ST_OK) t2[v] = std::min(t2[v], t);
      }
    }
    L.rr = t2[1] <= t2[0] ? 1 : 0;
  }
  h->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  L.tuned_ms = best;
  return ST_OK;
}

template <typename T>
int autotune_all(st_mg* h, void* u0, void* F0, hipStream_t s) {
  const int last = (int)h->lv.size() - 1;
  for (int l = 0; l < last; ++l) {
    Level& L = h->lv[l];
    if (l == 0) {
      T* alt = (T*)h->tmp;
      // level 0: caller scratch for u and F; the transform buffer doubles as the
      // second iterate of the small-level step only when the regular path is not timed
      CHK(tune_level<T>(h, 0, (T*)u0, (T*)F0, (T*)h->r0, alt, s));
    } else {
      CHK(tune_level<T>(h, l, (T*)L.u, (T*)L.F, (T*)L.r, (T*)L.u2, s));
    }
  }
  return ST_OK;
}

// The coarse end of the cycle in one workgroup: the first level l >= 1 from
// which every level's iterate, right-hand side and tables, plus two scratch
// vectors, fit in 64 KB of LDS (exact smoother, N_t <= 4, FP64 or FP32 handles;
// STMG_COARSE_TAIL=0 turns it off).
template <typename T>
int setup_coarse_tail_t(st_mg* h) {
  const int last = (int)h->lv.size() - 1, nt = h->nt, b = h->p.batch;
  auto need = [&](int top) -> size_t {
    size_t e = 0, mx = 0;
    for (int l = top; l <= last; ++l) {
      const Level& L = h->lv[l];
      const size_t dof = (size_t)b * L.N * nt * L.nx;
      e += (size_t)L.n * L.n + (size_t)L.nx * nt * nt + 2 * dof;
      mx = std::max(mx, dof);
    }
    return (e + 2 * mx) * sizeof(T);
  };
  int top = -1;
  for (int l = 1; l < last; ++l)
    if (last - l + 1 <= CT_MAX && need(l) <= 65536) {
      top = l;
      break;
    }
  if (top < 0) return ST_OK;
  for (int tr = 0; tr < 2; ++tr) {
    CoarseArgs<T> a{};
    int off = 0;
    a.levels = last - top + 1;
    for (int q = 0; q < a.levels; ++q) {
      const Level& L = h->lv[top + q];
      const ResidArgs<T> ra = resid_args<T>(h, L, tr != 0);
      CoarseLevel<T>& c = a.lv[q];
      for (int i = 0; i < NT_MAX * NT_MAX; ++i) {
        c.K[i] = ra.K[i];
        c.M[i] = ra.M[i];
      }
      for (int i = 0; i < NT_MAX; ++i) {
        c.ca[i] = ra.ca[i];
        c.cb[i] = ra.cb[i];
      }
      for (int i = 0; i < 3; ++i) {
        c.wm[i] = ra.wm[i];
        c.wk[i] = ra.wk[i];
      }
      c.gS = SPof<T>(L);
      c.gG = Gof<T>(L);
      c.n = L.n;
      c.N = L.N;
      c.nx = (int)L.nx;
      c.rn = 1.0f / (float)L.n;
      c.rN = 1.0f / (float)L.N;
      c.rnx = 1.0f / (float)L.nx;
      c.full = L.kind == 'f' ? 1 : 0;
      const int dof = b * L.N * nt * (int)L.nx;
      c.offS = off;
      off += L.n * L.n;
      c.offG = off;
      off += (int)L.nx * nt * nt;
      c.offU = off;
      off += dof;
      c.offF = off;
      off += dof;
    }
    int mx = 0;
    for (int q = 0; q < a.levels; ++q) mx = std::max(mx, b * a.lv[q].N * nt * a.lv[q].nx);
    a.offR = off;
    a.offQ = off + mx;
    for (int i = 0; i < nt * nt; ++i) {
      a.R1T[i] = (T)h->R1T[i];
      a.R2T[i] = (T)h->R2T[i];
    }
    a.omega = (T)h->p.omega;
    a.nu1 = h->p.nu1;
    a.nu2 = h->p.nu2;
    a.gamma = h->p.gamma;
    a.transpose = tr;
    a.dir = tr ? +1 : -1;
    HIPCHK(h, hipMalloc(&h->tail_args[tr], sizeof(a)));
    HIPCHK(h, hipMemcpy(h->tail_args[tr], &a, sizeof(a), hipMemcpyHostToDevice));
  }
  h->tail = top;
  h->tail_lds = need(top);
  return ST_OK;
}

int setup_coarse_tail(st_mg* h) {
  if (const char* e = std::getenv("STMG_COARSE_TAIL"))
    if (std::atoi(e) == 0) return ST_OK;
  if (h->mesh || high_order(h) || h->p.smoother != ST_SMOOTH_EXACT || is_mixed(h)) return ST_OK;
  return h->p.precision == ST_FP32 ? setup_coarse_tail_t<float>(h) : setup_coarse_tail_t<double>(h);
}

// Device copy of a host array (nullptr for an empty one).
template <typename D, typename S>
int upload(st_mg* h, D** dst, const std::vector<S>& src) {
  *dst = nullptr;
  if (src.empty()) return ST_OK;
  std::vector<D> tmp(src.begin(), src.end());
  if (hipMalloc((void**)dst, tmp.size() * sizeof(D)) != hipSuccess)
    return fail(h, ST_ENOMEM, "hipMalloc of %zu bytes failed", tmp.size() * sizeof(D));
  HIPCHK(h, hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(D), hipMemcpyHostToDevice));
  return ST_OK;
}

// Dense inverse of the slab matrix A = K_tau (x) M_h + M_tau (x) K_h of mesh
// level `rx` (rows l * nx + i), uploaded in double and float.
int dense_slab_inverse(st_mg* h, int rx, double tau, double** d64, float** d32, int* m_out) {
  const stmg::MeshLevel& M = h->mh[(size_t)rx];
  const int nt = h->nt;
  const long long nx = M.nx(), m = nt * nx;
  if (m > 1024)
    return fail(h, ST_EINVAL,
                "an exact slab solve on refinement level %d needs a dense %lld x %lld inverse (limit 1024): "
                "refine less or use more time slabs so that space is coarsened further",
                rx, m, m);
  std::vector<double> A((size_t)(m * m), 0.0);
  for (long long i = 0; i < nx; ++i)
    for (int e = M.rowptr[(size_t)i]; e < M.rowptr[(size_t)i + 1]; ++e) {
      const long long c = M.col[(size_t)e];
      for (int l = 0; l < nt; ++l)
        for (int k = 0; k < nt; ++k)
          A[(size_t)((l * nx + i) * m + k * nx + c)] =
              h->Kt[l * nt + k] * M.mval[(size_t)e] + tau * h->Mh[l * nt + k] * M.kval[(size_t)e];
    }
  if (!invert((int)m, A.data())) return fail(h, ST_EINVAL, "singular slab matrix on refinement level %d", rx);
  CHK(upload(h, d64, A));
  CHK(upload(h, d32, A));
  *m_out = (int)m;
  return ST_OK;
}

// Levels on a P1 mesh: the Sec. 4 rule with the refinement level in place of
// the grid size (space coarsens while the level is above 0) and h_L = h0 2^-L;
// the spatial cycle of a level runs over its refinement levels down to 0.
int setup_mesh_levels(st_mg* h, const st_mesh* mesh, int refinements) {
  const st_mg_params* p = &h->p;
  std::string err;
  int rc = stmg::mesh_hierarchy(mesh, refinements, h->mh, err);
  if (rc != ST_OK) return fail(h, rc, "%s", err.c_str());
  h->mesh = true;
  const double h0 = mesh->h0 > 0.0 ? mesh->h0 : h->mh[0].longest_edge;
  for (size_t r = 0; r < h->mh.size(); ++r)
    if (h->mh[r].nx() < 1)
      return fail(h, ST_EINVAL, "refinement level %zu of the mesh has no interior node", r);
  int rx = refinements, N = p->N;
  double tau = p->T / p->N;
  while (true) {
    Level L;
    L.n = rx;
    L.N = N;
    L.nx = h->mh[(size_t)rx].nx();
    L.tau = tau;
    L.h = h0 * std::ldexp(1.0, -rx);
    L.mu = tau / (L.h * L.h);
    for (int j = rx; j >= 0; --j) {
      Level::Sub S;
      S.n = j;
      S.nx = h->mh[(size_t)j].nx();
      S.h = h0 * std::ldexp(1.0, -j);
      L.sub.push_back(S);
    }
    if (N == 1) {
      h->lv.push_back(L);
      break;
    }
    bool full;
    if (p->coarsen == ST_COARSEN_FULL) full = rx > 0;
    else if (p->coarsen == ST_COARSEN_SEMI) full = false;
    else full = rx > 0 && L.mu >= h->mu_star * (1.0 - 1e-12);
    L.kind = full ? 'f' : 's';
    h->lv.push_back(L);
    if (full) rx -= 1;
    N /= 2;
    tau *= 2.0;
  }
  h->md.resize(h->mh.size());
  for (size_t r = 0; r < h->mh.size(); ++r) {
    const stmg::MeshLevel& M = h->mh[r];
    MeshDev& D = h->md[r];
    D.nx = M.nx();
    D.nnz = (long long)M.col.size();
    std::vector<double> dg((size_t)D.nx * 2, 0.0);
    for (long long i = 0; i < D.nx; ++i)
      for (int e = M.rowptr[(size_t)i]; e < M.rowptr[(size_t)i + 1]; ++e)
        if (M.col[(size_t)e] == i) {
          dg[(size_t)i * 2] = M.mval[(size_t)e];
          dg[(size_t)i * 2 + 1] = M.kval[(size_t)e];
        }
    CHK(upload(h, &D.rowptr, M.rowptr));
    CHK(upload(h, &D.col, M.col));
    CHK(upload(h, &D.mv64, M.mval));
    CHK(upload(h, &D.kv64, M.kval));
    CHK(upload(h, &D.mv32, M.mval));
    CHK(upload(h, &D.kv32, M.kval));
    CHK(upload(h, &D.dg64, dg));
    CHK(upload(h, &D.dg32, dg));
    for (long long i = 0; i < D.nx; ++i) D.ew = std::max(D.ew, M.rowptr[(size_t)i + 1] - M.rowptr[(size_t)i]);
    std::vector<int> ecol((size_t)D.ew * D.nx);
    std::vector<double> emk((size_t)D.ew * D.nx * 2, 0.0);
    for (long long i = 0; i < D.nx; ++i)
      for (int e = 0; e < D.ew; ++e) {
        const int q = M.rowptr[(size_t)i] + e;
        const size_t at = (size_t)e * D.nx + i;
        if (q < M.rowptr[(size_t)i + 1]) {
          ecol[at] = M.col[(size_t)q];
          emk[2 * at] = M.mval[(size_t)q];
          emk[2 * at + 1] = M.kval[(size_t)q];
        } else {
          ecol[at] = (int)i;
        }
      }
    CHK(upload(h, &D.ecol, ecol));
    CHK(upload(h, &D.emk64, emk));
    CHK(upload(h, &D.emk32, emk));
    {
      const long long tiles = (D.nx + MESH_TILE - 1) / MESH_TILE;
      std::vector<int> hoff((size_t)tiles + 1, 0), hcol;
      std::vector<unsigned short> lcol((size_t)D.ew * D.nx, 0), ldiag((size_t)D.nx, 0);
      for (long long t = 0; t < tiles; ++t) {
        const long long i0 = t * MESH_TILE, i1 = std::min(D.nx, i0 + MESH_TILE);
        std::vector<int> cols;
        for (long long i = i0; i < i1; ++i)
          for (int e = 0; e < D.ew; ++e) cols.push_back(ecol[(size_t)e * D.nx + i]);
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        if (cols.size() > 65535) return fail(h, ST_EINVAL, "mesh rows touch too many distinct nodes");
        for (long long i = i0; i < i1; ++i) {
          for (int e = 0; e < D.ew; ++e) {
            const size_t at = (size_t)e * D.nx + i;
            lcol[at] = (unsigned short)(std::lower_bound(cols.begin(), cols.end(), ecol[at]) - cols.begin());
          }
          // every row holds its diagonal entry, so the node is in its own tile's halo
          ldiag[(size_t)i] = (unsigned short)(std::lower_bound(cols.begin(), cols.end(), (int)i) - cols.begin());
        }
        D.hmax = std::max(D.hmax, (int)cols.size());
        hcol.insert(hcol.end(), cols.begin(), cols.end());
        hoff[(size_t)t + 1] = (int)hcol.size();
      }
      CHK(upload(h, &D.hoff, hoff));
      CHK(upload(h, &D.hcol, hcol));
      CHK(upload(h, &D.lcol, lcol));
      CHK(upload(h, &D.ldiag, ldiag));
    }
    if (r > 0) {
      std::vector<int> pp, rrow, rcol;
      std::vector<double> w;
      stmg::mesh_interpolation(h->mh[r - 1], M, pp, w, rrow, rcol);
      D.nxc = h->mh[r - 1].nx();
      CHK(upload(h, &D.p, pp));
      CHK(upload(h, &D.rrow, rrow));
      CHK(upload(h, &D.rcol, rcol));
      CHK(upload(h, &D.w64, w));
      CHK(upload(h, &D.w32, w));
      for (long long I = 0; I < D.nxc; ++I) D.rw = std::max(D.rw, rrow[(size_t)I + 1] - rrow[(size_t)I]);
      std::vector<int> rell((size_t)D.rw * D.nxc, -1);
      for (long long I = 0; I < D.nxc; ++I)
        for (int e = rrow[(size_t)I]; e < rrow[(size_t)I + 1]; ++e)
          rell[(size_t)(e - rrow[(size_t)I]) * D.nxc + I] = rcol[(size_t)e];
      CHK(upload(h, &D.rell, rell));
      {
        const long long tiles = (D.nxc + MESH_TILE - 1) / MESH_TILE;
        std::vector<int> hoff((size_t)tiles + 1, 0), hcol;
        std::vector<unsigned short> loc((size_t)D.rw * D.nxc, 0);
        for (long long t = 0; t < tiles; ++t) {
          const long long i0 = t * MESH_TILE, i1 = std::min(D.nxc, i0 + MESH_TILE);
          std::vector<int> cols;
          for (long long I = i0; I < i1; ++I)
            for (int e = rrow[(size_t)I]; e < rrow[(size_t)I + 1]; ++e) cols.push_back(rcol[(size_t)e]);
          std::sort(cols.begin(), cols.end());
          cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
          if (cols.size() > 65535) return fail(h, ST_EINVAL, "interpolation rows touch too many distinct nodes");
          for (long long I = i0; I < i1; ++I)
            for (int e = 0; e < D.rw; ++e) {
              const size_t at = (size_t)e * D.nxc + I;
              if (rell[at] >= 0)
                loc[at] = (unsigned short)(std::lower_bound(cols.begin(), cols.end(), rell[at]) - cols.begin());
            }
          D.rhmax = std::max(D.rhmax, (int)cols.size());
          hcol.insert(hcol.end(), cols.begin(), cols.end());
          hoff[(size_t)t + 1] = (int)hcol.size();
        }
        CHK(upload(h, &D.rhoff, hoff));
        CHK(upload(h, &D.rhcol, hcol));
        CHK(upload(h, &D.rloc, loc));
      }
    }
  }
  for (size_t l = 0; l < h->lv.size(); ++l) {
    Level& L = h->lv[l];
    CHK(dense_slab_inverse(h, 0, L.tau, &L.D64, &L.D32, &L.dm));
    if (l + 1 == h->lv.size() && L.n > 0) CHK(dense_slab_inverse(h, L.n, L.tau, &L.C64, &L.C32, &L.cm));
  }
  return ST_OK;
}

int setup_impl(const st_mg_params* p, st_mg_t* out, const st_mesh* mesh, int refinements) {
  if (!p || !out) return ST_EINVAL;
  *out = nullptr;
  st_mg* h = new (std::nothrow) st_mg();
  if (!h) return ST_ENOMEM;
  h->p = *p;
  auto bad = [&](const char* msg) {
    h->err = msg;
    return ST_EINVAL;
  };
  int rc = ST_OK;
  if (p->dim < 1 || p->dim > 3) rc = bad("dim must be 1, 2 or 3");
  else if (!mesh && (p->n < 1 || p->n > 255 || !is_pow2((long long)p->n + 1)))
    rc = bad("n must be 2^m - 1 with 1 <= n <= 255");
  else if (mesh && mesh->dim != p->dim) rc = bad("params dim and mesh dim differ");
  else if (mesh && p->smoother != ST_SMOOTH_SPATIAL_MG)
    rc = bad("P1 meshes need the spatial-cycle smoother (ST_SMOOTH_SPATIAL_MG)");
  else if (mesh && p->precision == ST_MIXED_BF16)
    rc = bad("P1 meshes have no sine transforms: use ST_FP64, ST_FP32 or ST_MIXED");
  else if (!(p->T > 0.0) || !std::isfinite(p->T)) rc = bad("T must be positive");
  else if (!is_pow2(p->N) || p->N > (1 << 20)) rc = bad("N must be a power of two (<= 2^20)");
  else if (p->pt < 0 || p->pt > NT_BIG - 1) rc = bad("p_t must be in 0..47");
  else if (!(p->omega > 0.0 && p->omega <= 1.0)) rc = bad("omega must be in (0, 1]");
  else if (p->nu1 < 0 || p->nu2 < 0 || p->nu1 + p->nu2 > 64) rc = bad("nu1, nu2 must be >= 0");
  else if (p->coarsen < ST_COARSEN_AUTO || p->coarsen > ST_COARSEN_FULL) rc = bad("unknown coarsening rule");
  else if (p->precision < ST_FP64 || p->precision > ST_MIXED_BF16) rc = bad("unknown precision");
  else if (p->batch < 1) rc = bad("batch must be >= 1");
  else if (p->smoother != ST_SMOOTH_EXACT && p->smoother != ST_SMOOTH_SPATIAL_MG) rc = bad("unknown smoother");
  else if (p->smoother == ST_SMOOTH_SPATIAL_MG &&
           (p->nu1x < 0 || p->nu2x < 0 || p->nu1x > 16 || p->nu2x > 16 || !(p->omega_x > 0.0 && p->omega_x <= 1.0)))
    rc = bad("spatial cycle needs 0 <= nu1x, nu2x <= 16 and omega_x in (0, 1]");
  else if (p->gamma != 1 && p->gamma != 2) rc = bad("gamma must be 1 (V-cycle) or 2 (W-cycle)");
  else if (p->smoother == ST_SMOOTH_SPATIAL_MG && p->pt > NT_MAX - 1)
    rc = bad("the spatial-cycle smoother supports p_t <= 3");
  if (rc != ST_OK) {
    // keep the handle alive only to report the message: return it so the caller can read it
    *out = h;
    return rc;
  }
  h->nt = p->pt + 1;
  // tuning knob: STMG_TRANSFORM=1 forces the LDS-staged transforms, =2 the register ones
  // tuning knob: STMG_SMALL=0 turns the one-kernel small-level smoother off
  if (const char* sm = std::getenv("STMG_SMALL")) h->small = std::atoi(sm) != 0;
  if (const char* rx = std::getenv("STMG_RX")) h->rx = std::atoi(rx) != 0;
  // tuning knob: STMG_RR=0 stores the fine defect and restricts it in a second pass
  if (const char* rr = std::getenv("STMG_RR")) h->rr = std::atoi(rr) != 0;
  if (const char* ti = std::getenv("STMG_TRANSFORM")) {
    const int v = std::atoi(ti);
    h->impl = ((v >= TRANSFORM_AUTO && v <= TRANSFORM_SLAB) || v == TRANSFORM_XSLAB) ? v : TRANSFORM_AUTO;
  }
  time_basis(h);
  {
    const int nt = h->nt, q = nt * nt;
    std::vector<double> t(5 * q + 3 * nt);
    for (int l = 0; l < nt; ++l)
      for (int k = 0; k < nt; ++k) {
        t[l * nt + k] = h->Kt[l * nt + k];
        t[q + l * nt + k] = h->Kt[k * nt + l];
        t[2 * q + l * nt + k] = h->Mh[l * nt + k];
        t[3 * q + 3 * nt + l * nt + k] = h->R1T[l * nt + k];
        t[4 * q + 3 * nt + l * nt + k] = h->R2T[l * nt + k];
      }
    for (int l = 0; l < nt; ++l) {
      t[3 * q + l] = h->ca[l];
      t[3 * q + nt + l] = h->cb[l];
      t[3 * q + 2 * nt + l] = h->ints[l];
    }
    std::vector<float> t32(t.begin(), t.end());
    if (hipMalloc(&h->gen64, t.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&h->gen32, t32.size() * sizeof(float)) != hipSuccess ||
        hipMemcpy(h->gen64, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->gen32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      h->err = "could not upload the time matrices";
      *out = h;
      return ST_EHIP;
    }
  }
  h->mu_star = p->mu_star > 0.0 ? p->mu_star : critical_mu(h);
  if (!std::isfinite(h->mu_star)) {
    h->err = "could not compute mu*";
    *out = h;
    return ST_EINVAL;
  }
  if (mesh) {
    rc = setup_mesh_levels(h, mesh, refinements);
    *out = h;
    return rc;
  }
  // hierarchy: Sec. 4 rule; space down to one node, time down to one slab
  int n = p->n, N = p->N;
  double tau = p->T / p->N;
  while (true) {
    Level L;
    L.n = n;
    L.N = N;
    L.nx = 1;
    for (int i = 0; i < p->dim; ++i) L.nx *= n;
    L.tau = tau;
    L.h = 1.0 / (n + 1);
    L.mu = tau / (L.h * L.h);
    L.hb = transform_half_blocks(n);
    if (N == 1) {
      h->lv.push_back(L);
      break;
    }
    bool full;
    if (p->coarsen == ST_COARSEN_FULL) full = n > 1;
    else if (p->coarsen == ST_COARSEN_SEMI) full = false;
    else full = n > 1 && L.mu >= h->mu_star * (1.0 - 1e-12);
    L.kind = full ? 'f' : 's';
    h->lv.push_back(L);
    if (full) n = (n - 1) / 2;
    N /= 2;
    tau *= 2.0;
  }
  if (p->smoother == ST_SMOOTH_SPATIAL_MG) {
    for (auto& L : h->lv) {
      for (int m = L.n; m >= 1; m = (m - 1) / 2) {
        Level::Sub S;
        S.n = m;
        S.nx = 1;
        for (int i = 0; i < p->dim; ++i) S.nx *= m;
        S.h = 1.0 / (m + 1);
        L.sub.push_back(S);
        if (m == 1) break;
      }
    }
  }
  for (auto& L : h->lv) {
    rc = build_level_tables(h, L);
    if (rc != ST_OK) {
      *out = h;
      return rc;
    }
  }
  rc = setup_coarse_tail(h);
  if (rc == ST_OK) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      h->cus = 0;
  }
  if (rc == ST_OK) {
    const hipError_t e = scratch_address(&h->scratch);
    if (e != hipSuccess) h->scratch_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
  }
  *out = h;
  return rc;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

void st_mg_default_params(st_mg_params* p) {
  if (!p) return;
  p->dim = 1;
  p->n = 31;
  p->T = 1.0;
  p->N = 16;
  p->pt = 1;
  p->omega = 0.5;
  p->nu1 = 2;
  p->nu2 = 2;
  p->coarsen = ST_COARSEN_AUTO;
  p->mu_star = 0.0;
  p->precision = ST_FP64;
  p->batch = 1;
  p->smoother = ST_SMOOTH_EXACT;
  p->nu1x = 2;
  p->nu2x = 2;
  p->omega_x = 2.0 / 3.0;
  p->gamma = 1;
}

int st_mg_setup(const st_mg_params* p, st_mg_t* out) { return setup_impl(p, out, nullptr, 0); }

int st_mg_setup_mesh(const st_mg_params* p, const st_mesh* coarse, int refinements, st_mg_t* out) {
  if (!coarse) return ST_EINVAL;
  return setup_impl(p, out, coarse, refinements);
}

int st_mg_destroy(st_mg_t h) {
  if (!h) return ST_OK;
  if (h->gc.exec) (void)hipGraphExecDestroy(h->gc.exec);
  for (auto& L : h->lv) {
    (void)hipFree(L.S64);
    (void)hipFree(L.S32);
    (void)hipFree(L.S16);
    (void)hipFree(L.G64);
    (void)hipFree(L.G32);
    (void)hipFree(L.Sp64);
    (void)hipFree(L.Sp32);
    (void)hipFree(L.S2_64);
    (void)hipFree(L.S2_32);
    (void)hipFree(L.S2_16);
    (void)hipFree(L.eig64);
    (void)hipFree(L.eig32);
    (void)hipFree(L.D64);
    (void)hipFree(L.D32);
    (void)hipFree(L.C64);
    (void)hipFree(L.C32);
  }
  for (auto& D : h->md) {
    for (void* q : {(void*)D.ldiag, (void*)D.rhoff, (void*)D.rhcol, (void*)D.rloc, (void*)D.rell, (void*)D.hoff, (void*)D.hcol, (void*)D.lcol, (void*)D.ecol, (void*)D.emk64, (void*)D.emk32, (void*)D.rowptr, (void*)D.col, (void*)D.mv64, (void*)D.kv64, (void*)D.dg64, (void*)D.w64,
                    (void*)D.mv32, (void*)D.kv32, (void*)D.dg32, (void*)D.w32, (void*)D.p, (void*)D.rrow,
                    (void*)D.rcol})
      (void)hipFree(q);
  }
  if (h->ws_owned && h->ws) (void)hipFree(h->ws);
  (void)hipFree(h->tail_args[0]);
  (void)hipFree(h->tail_args[1]);
  (void)hipFree(h->gen64);
  (void)hipFree(h->gen32);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  delete h;
  return ST_OK;
}

const char* st_mg_last_error(st_mg_t h) { return h ? h->err.c_str() : "null handle"; }

int st_mg_workspace_bytes(st_mg_t h, size_t* bytes) {
  if (!h || !bytes) return ST_EINVAL;
  if (h->lv.empty()) return fail(h, ST_ESTATE, "handle was not set up");
  *bytes = layout(h, nullptr);
  return ST_OK;
}

int st_mg_bind_workspace(st_mg_t h, void* dptr, size_t bytes) {
  if (!h) return ST_EINVAL;
  if (h->lv.empty()) return fail(h, ST_ESTATE, "handle was not set up");
  const size_t need = layout(h, nullptr);
  if (h->gc.exec) {
    (void)hipGraphExecDestroy(h->gc.exec);
    h->gc.exec = nullptr;
  }
  if (h->ws_owned && h->ws) {
    (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_owned = false;
  }
  if (dptr == nullptr) {
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) return fail(h, ST_ENOMEM, "hipMalloc(%zu) failed", need);
    h->ws = p;
    h->ws_owned = true;
    h->ws_bytes = need;
  } else {
    if (bytes < need) return fail(h, ST_EWORKSPACE, "workspace of %zu bytes < %zu needed", bytes, need);
    if (((uintptr_t)dptr & 255) != 0) return fail(h, ST_EWORKSPACE, "workspace must be 256-byte aligned");
    h->ws = dptr;
    h->ws_bytes = bytes;
  }
  layout(h, (char*)h->ws);
  return ST_OK;
}

int st_mg_levels(st_mg_t h, int* nlev, char* schedule, int cap) {
  if (!h || h->lv.empty()) return ST_EINVAL;
  const int nl = (int)h->lv.size();
  if (nlev) *nlev = nl;
  if (schedule) {
    if (cap < nl) return fail(h, ST_EINVAL, "schedule buffer needs %d bytes", nl);
    for (int i = 0; i < nl - 1; ++i) schedule[i] = h->lv[i].kind;
    schedule[nl - 1] = '\0';
  }
  return ST_OK;
}

int st_mg_level_info(st_mg_t h, int level, int* n, int* N, double* tau, double* mu) {
  if (!h || level < 0 || level >= (int)h->lv.size()) return ST_EINVAL;
  const Level& L = h->lv[level];
  if (n) *n = L.n;
  if (N) *N = L.N;
  if (tau) *tau = L.tau;
  if (mu) *mu = L.mu;
  return ST_OK;
}

int st_mg_level_nx(st_mg_t h, int level, long long* nx) {
  if (!h || !nx || level < 0 || level >= (int)h->lv.size()) return ST_EINVAL;
  *nx = h->lv[level].nx;
  return ST_OK;
}

int st_mg_sizes(st_mg_t h, long long* dof, long long* f_len, long long* u0_len) {
  if (!h || h->lv.empty()) return ST_EINVAL;
  const Level& L = h->lv[0];
  if (dof) *dof = (long long)L.N * h->nt * L.nx;
  if (f_len) *f_len = (long long)L.N * L.nx;
  if (u0_len) *u0_len = L.nx;
  return ST_OK;
}

int st_mg_rhs(st_mg_t h, const void* f, const void* u0, void* F, void* stream) {
  if (!h || h->lv.empty() || !f || !F) return h ? fail(h, ST_EINVAL, "null argument") : ST_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (h->mesh) {
    if (h->p.precision == ST_FP32)
      HIPCHK(h, launch_mesh_rhs<float>(h->nt, (const float*)f, (const float*)u0, (float*)F, mesh_rhs_args<float>(h), s));
    else
      HIPCHK(h, launch_mesh_rhs<double>(h->nt, (const double*)f, (const double*)u0, (double*)F,
                                        mesh_rhs_args<double>(h), s));
    return ST_OK;
  }
  if (high_order(h)) {
    if (h->p.precision == ST_FP32)
      HIPCHK(h, launch_rhs_gen<float>(h->p.dim, (const float*)f, (const float*)u0, (float*)F,
                                      gen_args<float>(h, h->lv[0], false), s));
    else
      HIPCHK(h, launch_rhs_gen<double>(h->p.dim, (const double*)f, (const double*)u0, (double*)F,
                                       gen_args<double>(h, h->lv[0], false), s));
  } else if (h->p.precision == ST_FP32) {
    HIPCHK(h, launch_rhs<float>(h->p.dim, h->nt, (const float*)f, (const float*)u0, (float*)F,
                                rhs_args<float>(h), s));
  } else {
    HIPCHK(h, launch_rhs<double>(h->p.dim, h->nt, (const double*)f, (const double*)u0, (double*)F,
                                 rhs_args<double>(h), s));
  }
  return ST_OK;
}

int st_mg_rhs_adjoint(st_mg_t h, const void* lam, void* grad_f, void* grad_u0, void* stream) {
  if (!h || h->lv.empty() || !lam) return h ? fail(h, ST_EINVAL, "null argument") : ST_EINVAL;
  if (!grad_f && !grad_u0) return ST_OK;
  hipStream_t s = (hipStream_t)stream;
  if (h->mesh) {
    if (h->p.precision == ST_FP32)
      HIPCHK(h, launch_mesh_rhs_adjoint<float>(h->nt, (const float*)lam, (float*)grad_f, (float*)grad_u0,
                                               mesh_rhs_args<float>(h), s));
    else
      HIPCHK(h, launch_mesh_rhs_adjoint<double>(h->nt, (const double*)lam, (double*)grad_f, (double*)grad_u0,
                                                mesh_rhs_args<double>(h), s));
    return ST_OK;
  }
  if (high_order(h)) {
    if (h->p.precision == ST_FP32)
      HIPCHK(h, launch_rhs_adjoint_gen<float>(h->p.dim, (const float*)lam, (float*)grad_f, (float*)grad_u0,
                                              gen_args<float>(h, h->lv[0], false), s));
    else
      HIPCHK(h, launch_rhs_adjoint_gen<double>(h->p.dim, (const double*)lam, (double*)grad_f, (double*)grad_u0,
                                               gen_args<double>(h, h->lv[0], false), s));
  } else if (h->p.precision == ST_FP32) {
    HIPCHK(h, launch_rhs_adjoint<float>(h->p.dim, h->nt, (const float*)lam, (float*)grad_f,
                                        (float*)grad_u0, rhs_args<float>(h), s));
  } else {
    HIPCHK(h, launch_rhs_adjoint<double>(h->p.dim, h->nt, (const double*)lam, (double*)grad_f,
                                         (double*)grad_u0, rhs_args<double>(h), s));
  }
  return ST_OK;
}

int st_mg_residual(st_mg_t h, int level, int prec, int transpose, const void* u, const void* F,
                   void* r, double* norms2, void* stream) {
  CHK(check_level(h, level, prec, false));
  if (!u || !F || !r) return fail(h, ST_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)stream;
  const bool nrm = norms2 != nullptr && level == 0;
  if (norms2 != nullptr && level != 0) return fail(h, ST_EINVAL, "norms only on level 0");
  if (prec == ST_FP64)
    CHK((op_residual<double, double>(h, level, transpose != 0, (const double*)u, (const double*)F,
                                     (double*)r, nrm, s)));
  else
    CHK((op_residual<float, float>(h, level, transpose != 0, (const float*)u, (const float*)F,
                                   (float*)r, nrm, s)));
  if (nrm) {
    HIPCHK(h, hipMemcpyAsync(norms2, h->norm_dev, sizeof(double) * h->p.batch, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
  }
  return ST_OK;
}

int st_mg_residual_noalloc(st_mg_t h, int level, int prec, int transpose, const void* u, const void* F,
                           void* r, double* norms2, void* stream) {
  CHK(check_level_args(h, level, prec, false));
  if (!u || !F || !r) return fail(h, ST_EINVAL, "null vector");
  if (norms2 != nullptr && level != 0) return fail(h, ST_EINVAL, "norms only on level 0");
  const bool nrm = norms2 != nullptr;
  hipStream_t s = (hipStream_t)stream;
  double* partial = nullptr;
  double* sums = nullptr;
  if (nrm) {
    if (h->scratch == nullptr) return fail(h, ST_EHIP, "static scratch unavailable: %s", h->scratch_err.c_str());
    const Level& L = h->lv[0];
    const long long per = (long long)resid_blocks(h, L) * L.N;
    if (h->p.batch > NOALLOC_BATCH || per * h->p.batch > NOALLOC_PARTIALS)
      return fail(h, ST_EINVAL,
                  "static scratch too small: %lld partial sums for %d right-hand sides (limits %lld and %d)",
                  per * h->p.batch, h->p.batch, NOALLOC_PARTIALS, NOALLOC_BATCH);
    partial = h->scratch;
    sums = h->scratch + NOALLOC_PARTIALS;
  }
  // no profiling events here: creating them could allocate
  const bool prof = h->prof;
  h->prof = false;
  int rc;
  if (prec == ST_FP64)
    rc = op_residual<double, double>(h, level, transpose != 0, (const double*)u, (const double*)F, (double*)r, nrm,
                                     s, partial, sums);
  else
    rc = op_residual<float, float>(h, level, transpose != 0, (const float*)u, (const float*)F, (float*)r, nrm, s,
                                   partial, sums);
  h->prof = prof;
  CHK(rc);
  if (nrm) {
    HIPCHK(h, hipMemcpyAsync(norms2, sums, sizeof(double) * h->p.batch, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
  }
  return ST_OK;
}

int st_mg_block_solve(st_mg_t h, int level, int prec, int transpose, const void* r, void* x,
                      void* stream) {
  CHK(check_level(h, level, prec, false));
  if (!r || !x) return fail(h, ST_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)stream;
  if (h->mesh) {
    if (prec == ST_FP64)
      return mesh_exact_solve<double>(h, level, transpose != 0, (const double*)r, (double*)x, MODE_STORE, 1.0, s);
    return mesh_exact_solve<float>(h, level, transpose != 0, (const float*)r, (float*)x, MODE_STORE, 1.0f, s);
  }
  if (prec == ST_FP64)
    return op_block_solve<double>(h, level, transpose != 0, (const double*)r, (double*)x, MODE_STORE,
                                  1.0, (double*)h->tmp, level_r<double>(h, level), s);
  return op_block_solve<float>(h, level, transpose != 0, (const float*)r, (float*)x, MODE_STORE, 1.0f,
                               (float*)h->tmp, level_r<float>(h, level), s);
}

int st_mg_spatial_cycle(st_mg_t h, int level, int prec, int transpose, const void* r, void* x,
                        void* stream) {
  CHK(check_level(h, level, prec, false));
  if (!r || !x) return fail(h, ST_EINVAL, "null vector");
  if (h->p.smoother != ST_SMOOTH_SPATIAL_MG)
    return fail(h, ST_ESTATE, "the spatial cycle needs a handle set up with ST_SMOOTH_SPATIAL_MG");
  hipStream_t s = (hipStream_t)stream;
  if (h->mesh) {
    if (prec == ST_FP64)
      return mesh_spatial_cycle<double>(h, level, 0, transpose != 0, (const double*)r, (double*)x, MODE_STORE, 1.0,
                                        nullptr, s);
    return mesh_spatial_cycle<float>(h, level, 0, transpose != 0, (const float*)r, (float*)x, MODE_STORE, 1.0f,
                                     nullptr, s);
  }
  if (prec == ST_FP64)
    return spatial_cycle<double>(h, level, 0, transpose != 0, (const double*)r, (double*)x, MODE_STORE, 1.0,
                                 nullptr, s);
  return spatial_cycle<float>(h, level, 0, transpose != 0, (const float*)r, (float*)x, MODE_STORE, 1.0f,
                              nullptr, s);
}

int st_mg_smooth(st_mg_t h, int level, int prec, int transpose, void* u, const void* F, void* stream) {
  CHK(check_level(h, level, prec, false));
  if (!u || !F) return fail(h, ST_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)stream;
  if (prec == ST_FP64)
    return smooth_step<double>(h, level, transpose != 0, (double*)u, (const double*)F, level_r<double>(h, level),
                               (double*)h->tmp, s);
  return smooth_step<float>(h, level, transpose != 0, (float*)u, (const float*)F, level_r<float>(h, level),
                            (float*)h->tmp, s);
}

int st_mg_restrict(st_mg_t h, int level, int prec, const void* r_fine, void* F_coarse, void* stream) {
  CHK(check_level(h, level, prec, true));
  if (!r_fine || !F_coarse) return fail(h, ST_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)stream;
  if (prec == ST_FP64) return op_restrict<double>(h, level, (const double*)r_fine, (double*)F_coarse, s);
  return op_restrict<float>(h, level, (const float*)r_fine, (float*)F_coarse, s);
}

int st_mg_residual_restrict(st_mg_t h, int level, int prec, int transpose, const void* u, const void* F,
                            void* F_coarse, void* stream) {
  CHK(check_level(h, level, prec, true));
  if (!u || !F || !F_coarse) return fail(h, ST_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)stream;
  if (prec == ST_FP64)
    return op_resid_restrict<double>(h, level, transpose != 0, (const double*)u, (const double*)F,
                                     level_r<double>(h, level), (double*)F_coarse, s);
  return op_resid_restrict<float>(h, level, transpose != 0, (const float*)u, (const float*)F,
                                  level_r<float>(h, level), (float*)F_coarse, s);
}

int st_mg_prolong_add(st_mg_t h, int level, int prec, const void* e_coarse, void* u_fine, void* stream) {
  CHK(check_level(h, level, prec, true));
  if (!e_coarse || !u_fine) return fail(h, ST_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)stream;
  if (prec == ST_FP64) return op_prolong<double>(h, level, (const double*)e_coarse, (double*)u_fine, s);
  return op_prolong<float>(h, level, (const float*)e_coarse, (float*)u_fine, s);
}

int st_mg_vcycle(st_mg_t h, void* u, const void* F, double* relres, void* stream) {
  CHK(check_ready(h));
  if (!u || !F) return fail(h, ST_EINVAL, "null vector");
  hipStream_t s = (hipStream_t)stream;
  const int b = h->p.batch;
  std::vector<double> n0(b), n1(b);
  if (h->p.precision == ST_FP32) {
    CHK(fine_residual_norm<float>(h, false, u, F, s));
    if (relres) CHK(read_norms(h, n0.data(), s));
    CHK(cycle_and_norm<float>(h, false, u, F, s));
  } else {
    CHK(fine_residual_norm<double>(h, false, u, F, s));
    if (relres) CHK(read_norms(h, n0.data(), s));
    CHK(cycle_and_norm<double>(h, false, u, F, s));
  }
  if (relres) {
    CHK(read_norms(h, n1.data(), s));
    for (int i = 0; i < b; ++i) relres[i] = n0[i] > 0 ? n1[i] / n0[i] : 0.0;
  }
  return ST_OK;
}

int st_mg_solve(st_mg_t h, void* u, const void* F, double rtol, int maxit, int* iters, double* hist,
                void* stream) {
  CHK(check_ready(h));
  if (!u || !F || maxit < 0 || !(rtol >= 0.0)) return fail(h, ST_EINVAL, "invalid argument");
  hipStream_t s = (hipStream_t)stream;
  if (h->p.precision == ST_FP32) return solve_impl<float>(h, false, u, F, rtol, maxit, iters, hist, s);
  return solve_impl<double>(h, false, u, F, rtol, maxit, iters, hist, s);
}

int st_mg_adjoint(st_mg_t h, const void* g, void* lam, void* grad_f, void* grad_u0, double rtol,
                  int maxit, int* iters, double* hist, void* stream) {
  CHK(check_ready(h));
  if (!g || !lam || maxit < 0 || !(rtol >= 0.0)) return fail(h, ST_EINVAL, "invalid argument");
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if (h->p.precision == ST_FP32) rc = solve_impl<float>(h, true, lam, g, rtol, maxit, iters, hist, s);
  else rc = solve_impl<double>(h, true, lam, g, rtol, maxit, iters, hist, s);
  if (rc != ST_OK && rc != ST_ENOCONV) return rc;
  const int rc2 = st_mg_rhs_adjoint(h, lam, grad_f, grad_u0, stream);
  return rc2 != ST_OK ? rc2 : rc;
}

int st_mg_autotune(st_mg_t h, void* u_scratch, void* F_scratch, void* stream) {
  CHK(check_ready(h));
  if (h->p.precision == ST_FP64 && (!u_scratch || !F_scratch))
    return fail(h, ST_EINVAL, "FP64 autotuning needs two fine-level scratch vectors");
  hipStream_t s = (hipStream_t)stream;
  if (h->gc.exec) {
    (void)hipGraphExecDestroy(h->gc.exec);
    h->gc.exec = nullptr;
  }
  if (h->p.smoother == ST_SMOOTH_SPATIAL_MG) return ST_OK;   // transforms only on the coarsest level
  if (h->p.precision == ST_FP64) return autotune_all<double>(h, u_scratch, F_scratch, s);
  // float paths: level 0 of the inner cycle lives in workspace buffers
  void* u0 = is_mixed(h) ? h->e32 : u_scratch;
  void* F0 = is_mixed(h) ? h->F32 : F_scratch;
  if (!u0 || !F0) return fail(h, ST_EINVAL, "FP32 autotuning needs two fine-level scratch vectors");
  return autotune_all<float>(h, u0, F0, s);
}

int st_mg_level_tuning(st_mg_t h, int level, int* small, int* impl, float* ms) {
  if (!h || level < 0 || level >= (int)h->lv.size()) return ST_EINVAL;
  const Level& L = h->lv[level];
  if (small) *small = L.small >= 0 ? L.small : (h->small ? 1 : 0);
  if (impl) {
    const int f = L.impl >= 0 ? L.impl : h->impl;
    // 5: twice folded, residual fused in; 7: x-mode-major slab solve, residual fused in
    *impl = L.rx == 1 ? (f == TRANSFORM_XSLAB ? 7 : 5) : f;
  }
  if (ms) *ms = L.tuned_ms;
  return ST_OK;
}

int st_mg_level_shape(st_mg_t h, int level, int* wpg, int* pass_per_cu, int* fused_cg, int* fused_per_cu) {
  if (!h || level < 0 || level >= (int)h->lv.size()) return ST_EINVAL;
  const PassShape& sh = h->lv[level].shape;
  if (wpg) *wpg = sh.wpg;
  if (pass_per_cu) *pass_per_cu = sh.pass_per_cu;
  if (fused_cg) *fused_cg = sh.fused_cg != 0 ? sh.fused_cg : (h->nt >= 3 ? 1 : 4 / h->nt);
  if (fused_per_cu) *fused_per_cu = sh.fused_per_cu;
  return ST_OK;
}

int st_mg_set_level_shape(st_mg_t h, int level, int wpg, int pass_per_cu, int fused_cg, int fused_per_cu) {
  if (!h || level < 0 || level >= (int)h->lv.size()) return ST_EINVAL;
  const int cgmax = h->nt >= 3 ? 1 : 4 / h->nt;
  if (!(wpg == 1 || wpg == 2 || wpg == 4) || pass_per_cu < 0 || fused_per_cu < 0 || fused_cg < 0 ||
      fused_cg > cgmax || (fused_cg & (fused_cg - 1)) != 0)
    return fail(h, ST_EINVAL, "shape: wpg in {1,2,4}, fused_cg a power of two <= %d (0 = default), caps >= 0", cgmax);
  PassShape& sh = h->lv[level].shape;
  sh.wpg = wpg;
  sh.pass_per_cu = pass_per_cu;
  sh.fused_cg = fused_cg;
  sh.fused_per_cu = fused_per_cu;
  if (h->gc.exec) {   // a recorded graph holds the old launch shapes
    (void)hipGraphExecDestroy(h->gc.exec);
    h->gc.exec = nullptr;
  }
  return ST_OK;
}

int st_mg_set_graph(st_mg_t h, int enable) {
  if (!h) return ST_EINVAL;
  if (enable && h->prof) return fail(h, ST_ESTATE, "stop profiling before enabling graph mode");
  h->graph = enable ? 1 : 0;
  if (!h->graph && h->gc.exec) {
    (void)hipGraphExecDestroy(h->gc.exec);
    h->gc.exec = nullptr;
  }
  return ST_OK;
}

int st_mg_profile_start(st_mg_t h) {
  if (!h) return ST_EINVAL;
  if (h->graph) return fail(h, ST_ESTATE, "profiling needs eager mode (graph mode is on)");
  h->prof = true;
  h->ev_used = 0;
  h->prof_recs.clear();
  return ST_OK;
}

int st_mg_profile_stop(st_mg_t h) {
  if (!h) return ST_EINVAL;
  h->prof = false;
  return ST_OK;
}

int st_mg_profile_read(st_mg_t h, int kind, int level, double* total_ms, int* count) {
  if (!h || kind < 0 || kind >= ST_PROF_KINDS) return ST_EINVAL;
  double tot = 0.0;
  int cnt = 0;
  if (!h->prof_recs.empty()) HIPCHK(h, hipEventSynchronize(h->ev_pool[h->prof_recs.back().e1]));
  for (const auto& r : h->prof_recs) {
    if (r.kind != kind || (level >= 0 && r.level != level)) continue;
    float ms = 0.0f;
    HIPCHK(h, hipEventElapsedTime(&ms, h->ev_pool[r.e0], h->ev_pool[r.e1]));
    tot += ms;
    ++cnt;
  }
  if (total_ms) *total_ms = tot;
  if (count) *count = cnt;
  return ST_OK;
}

}  // extern "C"
