// libqoc host side: C ABI, validation, device memory and the launch plan of
// one cost (+ gradient) evaluation.  See include/qoc.h for the contract.
#include "../../include/qoc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "qoc_kernels.h"

namespace {

thread_local std::string g_err;

qoc_status fail(qoc_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return fail(QOC_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// (p, n) reading of the paper's "conservative global choice" (Sec. III):
// fewest products p-1+n such that the Taylor remainder bound, amplified by
// the 2^n squarings, is at most tol.
double taylor_bound(double theta, int p, int n) {
  const double x = std::ldexp(theta, -n);
  double f = 1.0;
  for (int k = 2; k <= p + 1; ++k) f *= k;
  return std::ldexp(1.0, n) * std::pow(x, p + 1) / f * std::exp(x);
}

bool taylor_select(double theta, double tol, int *p_out, int *n_out) {
  int bestG = -1, bp = 0, bn = 0;
  for (int n = 0; n < 60; ++n) {
    for (int p = 2; p <= 30; ++p) {
      if (taylor_bound(theta, p, n) <= tol) {
        const int G = p - 1 + n;
        if (bestG < 0 || G < bestG) {
          bestG = G;
          bp = p;
          bn = n;
        }
        break;
      }
    }
  }
  if (bestG < 0) return false;
  *p_out = bp;
  *n_out = bn;
  return true;
}

// The action form's pair (U_j psi by p 2^n products with H_j): the fewest
// products within the same bound, with theta / 2^n <= 1 so that the series
// terms do not grow (no cancellation between large terms in FP32); ties
// toward fewer squarings.
bool action_select(double theta, double tol, int *p_out, int *n_out) {
  long best = -1;
  int bp = 0, bn = 0;
  for (int n = 0; n < 60; ++n) {
    if (std::ldexp(theta, -n) > 1.0) continue;
    if (best >= 0 && (2L << n) >= best) break;  // p >= 2: no later n does better
    for (int p = 2; p <= 30; ++p) {
      if (taylor_bound(theta, p, n) <= tol) {
        const long c = (long)p << n;
        if (best < 0 || c < best) {
          best = c;
          bp = p;
          bn = n;
        }
        break;
      }
    }
  }
  if (best < 0) return false;
  *p_out = bp;
  *n_out = bn;
  return true;
}

// Largest theta whose truncation bound a fixed (p, n) still meets (the
// bound grows with theta): what a fixed pair admits without a warning.
double theta_admitted(int p, int n, double tol) {
  double lo = 0.0, hi = 1.0;
  while (taylor_bound(hi, p, n) <= tol && hi < 1e6) hi *= 2.0;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    (taylor_bound(mid, p, n) <= tol ? lo : hi) = mid;
  }
  return lo;
}

// Error index of the bf16x3 split products in the step propagators: the
// l2 error they add to the propagated states, up to a calibration factor.
// A split product (bf16 hi/lo halves, the lo x lo term dropped) errs by
// about eps = 2^-17 of the product of its operand norms, where an FP32
// product errs by 2^-24.  Per step, the first Taylor product (X X, |X| =
// theta / 2^n) is amplified by the n squarings after it (2^n), squaring i
// (|D^(i)| = min(2, theta 2^(i - n))) by 2^(n - i - 1); a block product
// (|E| <= 2) errs by 4 eps once per tree level and block.  Independent
// errors add in quadrature over the N steps (and the N / L blocks).  Only
// the classes in `cls` count (the FP32 products are the reference).
// Measured on MI355X, the state error stayed within 0.7 times the index.
double bf3_error_index(double theta, int n, int N, int L, int cls) {
  const double eps = std::ldexp(1.0, -17);
  const double x = std::ldexp(theta, -n);
  double step = 0.0;
  if (cls & QOC_BF3_TAYLOR) step += eps * x * x * std::ldexp(1.0, n);
  if (cls & QOC_BF3_SQUARING)
    for (int i = 0; i < n; ++i) {
      const double di = std::min(2.0, std::ldexp(theta, i - n));
      step += eps * di * di * std::ldexp(1.0, n - i - 1);
    }
  double blocks = 0.0;
  if (cls & QOC_BF3_BLOCKPROD) {
    int levels = 0;
    while ((1 << levels) < L) ++levels;
    blocks = std::sqrt(std::ceil((double)N / L)) * 4.0 * eps * levels;
  }
  return std::sqrt((double)N) * step + blocks;
}

// Classes the automatic bf16x3 policy runs as split products.  Measured on
// MI355X (transmon-cavity d = 128, N = 5000, theta_max 5.5, n = 5; spin chain
// d = 512, N = 1000, theta_max 0.81, n = 2; each chain class split alone and
// all together), the fidelity error stayed within 0.24 |z| times the index
// and the gradient's relative error within 1.4 times the index, where |z|
// <= 1 is the final overlap.  The budget 4e-5 therefore keeps |dF| <= 1e-5
// at any fidelity and the gradient within 1e-3.  The per-step derivative's
// products do not feed the states or the fidelity and, measured, leave the
// gradient error at its FP32 level, so they are always split; of the chain
// classes, all three are split when the index allows, else the Taylor
// products and squarings, else the Taylor products alone, else none.
constexpr double kBf3Budget = 4e-5;
int bf3_auto_classes(double theta, int n, int N, int L) {
  const int tries[3] = {QOC_BF3_TAYLOR | QOC_BF3_SQUARING | QOC_BF3_BLOCKPROD,
                        QOC_BF3_TAYLOR | QOC_BF3_SQUARING, QOC_BF3_TAYLOR};
  for (int cls : tries)
    if (bf3_error_index(theta, n, N, L, cls) <= kBf3Budget) return cls | QOC_BF3_ADJOINT;
  return QOC_BF3_ADJOINT;
}

// Capacity of the device-side (p, n) choice on the small-d path.
constexpr int kSmallNCap = 16, kSmallPCap = 16;
// Padding (elements) of the state buffers read by fixed-size prefetch slots.
constexpr size_t kRingSlack = 1024;

// Static device scratch of the no-alloc entry point: the per-call work
// space (Taylor / squaring levels, derivative scratch and partial sums) of
// calls that may not allocate.  Every GPU the library runs on holds its own
// copy until the process ends; host code reaches it only through the
// per-device address from hipGetSymbolAddress (the array's name is a host
// stand-in, not a device address).
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch`; `dev` must be the current device.
qoc_status scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(QOC_ERR_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(QOC_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return QOC_OK;
}

int pow2_at_least(long v) {
  int l = 1;
  while (l < v) l <<= 1;
  return l;
}

}  // namespace

struct qoc_handle {
  // problem
  int d = 0, dp = 0, M = 0, N = 0, S = 0, prec = QOC_FP32, fid_mode = 0;
  int bf3 = 0;  // bf16x3 split products in the batched chains (padded d >= 64)
  int bf3_req = -1;  // classes allowed bf16x3 products (QOC_BF3_* bits), -1 automatic
  int bf3_used = 0;  // classes the last call asked to run as bf16x3 products
  int bf3_adj_ran = 0;  // the last call launched split products in the derivative
  int bf3_fallback = 0;  // the automatic choice moved some classes to FP32
  bool capturing = false;  // the current call's stream is capturing a HIP graph
  // FP64 unitarity check of the step propagators: every `unit_stride`-th
  // step (0: off); its result word carries the call's epoch
  int unit_stride = 0;
  int grad_mode = QOC_GRAD_EXACT;
  unsigned epoch = 0, unit_epoch = 0;
  double last_unitarity = -1.0;
  // per-call work space carved from the static device scratch instead of
  // the handle's own allocations (the no-alloc entry point)
  unsigned char *ws_base = nullptr;
  size_t ws_cap = 0, ws_used = 0;
  int last_flags = 0;  // warning bits of the last call
  int sweep_mode[4] = {0, 0, 0, 0};  // per sweep: 0 auto, 1 per-block, 2 per-step launches,
                                     // 3 four-wavefront LDS (small d), 4 chain workgroup
  double dt = 0, a_fid = 0, a_amp = 0, a_var = 0, a_pen = 0, tol = 0, drift_warn = 0;
  bool has_pen = false;
  // per-step terms beyond the level penalty: forbidden states (C5) and the
  // time-optimal term (C6 / C7); they run on the generic per-block sweeps
  int nf = 0;
  double a_time = 0;
  bool has_ext = false;
  double *forb64 = nullptr;   // nf x d complex interleaved
  void *src = nullptr;        // (N + 1) state sets of costate sources
  double *ext_part = nullptr; // 2 x next
  int next = 1;
  // structured (sparse) Hamiltonians on the batched path: the union pattern
  // in compressed columns for the norm, and per-control nonzero lists for
  // the gradient contraction; built when the union has at most d^2 / 4
  // entries, and then used by default (qoc_set_structure)
  bool sp_built = false, sp_auto = false;
  int sp_mode = -1;  // -1 automatic, 0 dense, 1 structured
  bool sp_used = false;
  long nnz_union = 0, nev = 0;
  int *sp_colptr = nullptr, *sp_rowidx = nullptr;
  double *sp_vals = nullptr;
  int *sp_rptr = nullptr, *sp_rcol = nullptr, *sp_eptr = nullptr, *sp_ek = nullptr;
  void *sp_eval = nullptr;
  int fixed_p = 0, fixed_n = 0;
  int L = 1, nb = 1, device = 0;
  size_t esize = 4;  // sizeof(T) of the chain precision
  hipStream_t stream = nullptr;
  // device buffers (chain precision T unless noted)
  void *Hf = nullptr;         // (M+1) x 2 dp^2
  double *H64 = nullptr;      // (M+1) x d^2 complex interleaved
  double *u_dev = nullptr;    // M x N
  double *out_dev = nullptr;  // 2 + N
  double *grad_dev = nullptr; // M x N
  void *psi0 = nullptr;       // state set [2][S][dp]
  double *psiT64 = nullptr;   // S x d complex interleaved
  double *w64 = nullptr;      // dp
  void *pw = nullptr;         // dp, a_pen / S * w
  // action form (QOC_PROP_ACTION): H_j in an ELL layout (actK slots per
  // row), every matrix's slot values, per-step values, product inputs and
  // cotangents of gradient calls, and the controls' entries
  int prop = QOC_PROP_MATRIX, actK = 0;
  int *act_ecol = nullptr;       // actK x dp
  double *act_hm = nullptr;      // (M+1) x actK x 2 x dp
  void *act_hv = nullptr;        // N x actK x 2 x dp
  void *act_A = nullptr, *act_Y = nullptr;  // N x S x P x 2 x dp each
  long act_P = 0;                // P of act_A / act_Y
  double *act_part = nullptr;    // N x S x M
  int act_nent = 0;
  int *act_erow = nullptr, *act_ecol2 = nullptr, *act_cptr = nullptr, *act_cent = nullptr;
  void *act_cval = nullptr;
  long act_npairs = 0;
  // memory-lean mode: time segments of Ns steps (a multiple of L; Ns = N
  // and nseg = 1 when off); every per-step stack holds Ns steps
  int Ns = 0, nseg = 1;
  double *u_seg = nullptr;    // M x Ns: the controls of one segment
  void *X = nullptr, *Qa = nullptr, *Qb = nullptr;  // Ns x 2 dp^2 each
  void *Eh = nullptr;  // nb x 2 dp^2: E_b^H for the single-wavefront sweeps
  // padded d 16, L a multiple of SUB16 above it: sub-block products, their
  // ^H (ceil(N / SUB16) x 2 dp^2 each) and partial penalty costates
  void *Es = nullptr, *Ehs = nullptr, *nu = nullptr;
  void *Dlev = nullptr;       // levels x Ns x 2 dp^2
  int levels_alloc = 0;
  void *ckpt = nullptr, *lam_ckpt = nullptr, *mu = nullptr;  // (nb+1) sets
  void *psi_buf = nullptr, *lam_buf = nullptr;                // N+1, N sets
  unsigned long long *bits = nullptr;  // [theta, drift, norm ticket, unitarity, norm accumulator]
  double *zinfo = nullptr;    // 3 + 2S
  double *part = nullptr;     // 4 x npart
  int *pn_dev = nullptr;      // device-side (p, n, status)
  double *sc_dev = nullptr;   // device-side (dt / 2^n, theta)
  int npart = 1;
  void *adj = nullptr;
  double *adj_part = nullptr;  // batched large-d adjoint partial sums
  long adj_part_alloc = 0;
  long adj_elems_alloc = 0;   // total elements
  int adj_blocks = 0;
  // pinned host staging
  double *h_u = nullptr, *h_out = nullptr, *h_grad = nullptr;
  size_t bytes = 0;
  // diagnostics
  int last_p = 0, last_n = 0;
  double last_theta = 0, last_drift = 0;
  // profiling
  bool prof = false;
  double prof_ms[QOC_PHASE_COUNT] = {0};
  long long prof_calls[QOC_PHASE_COUNT] = {0};
  struct Pending {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
};

namespace {

struct DeviceGuard {
  int prev = 0;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
  }
  ~DeviceGuard() {
    if (ok) (void)hipSetDevice(prev);
  }
};

qoc_status dalloc(qoc_handle *h, void **p, size_t bytes) {
  *p = nullptr;
  if (h->capturing)
    return fail(QOC_ERR_UNSUPPORTED,
                "this call needs " + std::to_string(bytes) +
                    " more bytes of device work space, which cannot be allocated while its "
                    "stream captures a HIP graph: run one call with the same (p, n) before "
                    "capturing");
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(QOC_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                   hipGetErrorString(e));
  }
  h->bytes += bytes;
  return QOC_OK;
}

void dfree(qoc_handle *h, void **p, size_t bytes) {
  if (*p) {
    (void)hipFree(*p);
    h->bytes -= std::min(h->bytes, bytes);
  }
  *p = nullptr;
}

void release(qoc_handle *h) {
  void **ptrs[] = {&h->Hf, (void **)&h->H64, (void **)&h->u_dev, (void **)&h->out_dev,
                   (void **)&h->grad_dev, &h->psi0, (void **)&h->psiT64, (void **)&h->w64,
                   &h->pw, &h->X, &h->Qa, &h->Qb, &h->Eh, &h->Es, &h->Ehs, &h->nu, &h->Dlev,
                   (void **)&h->forb64, &h->src, (void **)&h->ext_part, (void **)&h->u_seg,
                   (void **)&h->act_ecol, (void **)&h->act_hm, &h->act_hv, &h->act_A, &h->act_Y,
                   (void **)&h->act_part, (void **)&h->act_erow, (void **)&h->act_ecol2,
                   (void **)&h->act_cptr, (void **)&h->act_cent, &h->act_cval,
                   (void **)&h->sp_colptr, (void **)&h->sp_rowidx, (void **)&h->sp_vals,
                   (void **)&h->sp_rptr, (void **)&h->sp_rcol, (void **)&h->sp_eptr,
                   (void **)&h->sp_ek, &h->sp_eval,
                   &h->ckpt, &h->lam_ckpt, &h->mu,
                   &h->psi_buf, &h->lam_buf, (void **)&h->bits,
                   (void **)&h->zinfo, (void **)&h->part, (void **)&h->pn_dev,
                   (void **)&h->sc_dev, &h->adj, (void **)&h->adj_part};
  for (void **p : ptrs)
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  if (h->h_u) (void)hipHostFree(h->h_u);
  if (h->h_out) (void)hipHostFree(h->h_out);
  if (h->h_grad) (void)hipHostFree(h->h_grad);
  h->h_u = h->h_out = h->h_grad = nullptr;
  for (auto &pe : h->pending) {
    (void)hipEventDestroy(pe.a);
    (void)hipEventDestroy(pe.b);
  }
  h->pending.clear();
  for (auto e : h->event_pool) (void)hipEventDestroy(e);
  h->event_pool.clear();
  if (h->stream) (void)hipStreamDestroy(h->stream);
  h->stream = nullptr;

  h->bytes = 0;
}

bool all_finite(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// ||H - H^dagger||_max <= 1e-12 max(1, ||H||_max), H d x d interleaved
bool hermitian(const double *H, int d) {
  double mx = 0.0, dev = 0.0;
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      const double ar = H[2 * ((size_t)r * d + c)], ai = H[2 * ((size_t)r * d + c) + 1];
      const double br = H[2 * ((size_t)c * d + r)], bi = -H[2 * ((size_t)c * d + r) + 1];
      mx = std::max(mx, std::hypot(ar, ai));
      dev = std::max(dev, std::hypot(ar - br, ai - bi));
    }
  return dev <= 1e-12 * std::max(1.0, mx);
}

// ------------------------------------------------------------------ timing
hipEvent_t pool_event(qoc_handle *h) {
  if (!h->event_pool.empty()) {
    hipEvent_t e = h->event_pool.back();
    h->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct PhaseTimer {
  qoc_handle *h;
  int phase;
  hipStream_t st;
  hipEvent_t a = nullptr;
  PhaseTimer(qoc_handle *h_, int ph, hipStream_t s) : h(h_), phase(ph), st(s) {
    if (h->prof) {
      a = pool_event(h);
      if (a) (void)hipEventRecord(a, st);
    }
  }
  void done() {
    if (h->prof && a) {
      hipEvent_t b = pool_event(h);
      if (b) {
        (void)hipEventRecord(b, st);
        h->pending.push_back({phase, a, b});
      }
      a = nullptr;
    }
  }
  ~PhaseTimer() { done(); }
};

qoc_status drain_pending(qoc_handle *h) {
  for (auto &pe : h->pending) {
    HIP_TRY(hipEventSynchronize(pe.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, pe.a, pe.b));
    h->prof_ms[pe.phase] += ms;
    h->prof_calls[pe.phase] += 1;
    h->event_pool.push_back(pe.a);
    h->event_pool.push_back(pe.b);
  }
  h->pending.clear();
  return QOC_OK;
}

// ------------------------------------------------------------------ buffers
// A slice of `bytes` of the static device scratch (256-byte aligned) for
// the no-alloc entry point, or QOC_ERR_UNSUPPORTED when it does not fit.
qoc_status carve(qoc_handle *h, void **p, size_t bytes) {
  const size_t off = (h->ws_used + 255) & ~(size_t)255;
  if (off > h->ws_cap || bytes > h->ws_cap - off)
    return fail(QOC_ERR_UNSUPPORTED,
                "this call needs more than the " + std::to_string(h->ws_cap) +
                    " bytes of static device scratch the no-alloc entry point may use (" +
                    std::to_string(off + bytes) + " bytes so far): use qoc_cost_grad_device");
  *p = h->ws_base + off;
  h->ws_used = off + bytes;
  return QOC_OK;
}

template <typename T> qoc_status ensure_levels(qoc_handle *h, int levels) {
  const size_t mat = 2 * (size_t)h->dp * h->dp;
  if (h->ws_base) return carve(h, &h->Dlev, (size_t)levels * h->Ns * mat * sizeof(T));
  if (levels <= h->levels_alloc) return QOC_OK;
  dfree(h, &h->Dlev, (size_t)h->levels_alloc * h->Ns * mat * sizeof(T));
  h->levels_alloc = 0;
  qoc_status s = dalloc(h, &h->Dlev, (size_t)levels * h->Ns * mat * sizeof(T));
  if (s) return s;
  h->levels_alloc = levels;
  return QOC_OK;
}

template <typename T> qoc_status ensure_adjoint(qoc_handle *h, int p, int Rcap, bool big) {
  long total;
  if (big) {
    // batched large-d adjoint: scratch per step, partial sums per tile
    total = qoc::adjoint_big_scratch_per_step<T>(h->dp, p, Rcap) * (long)h->Ns;
    const long parts = (long)h->Ns * qoc::adjoint_big_slices(h->dp) * std::max(h->M, 1);
    if (h->ws_base) {
      qoc_status s = carve(h, (void **)&h->adj_part, (size_t)parts * sizeof(double));
      if (s) return s;
    } else if (parts > h->adj_part_alloc) {
      dfree(h, (void **)&h->adj_part, (size_t)h->adj_part_alloc * sizeof(double));
      h->adj_part_alloc = 0;
      qoc_status s = dalloc(h, (void **)&h->adj_part, (size_t)parts * sizeof(double));
      if (s) return s;
      h->adj_part_alloc = parts;
    }
  } else {
    const int gpb = qoc::adjoint_groups_per_block<T>(h->dp);
    h->adj_blocks = std::min((h->N + gpb - 1) / gpb, 1024);
    total = qoc::adjoint_scratch_elems<T>(h->dp, p, Rcap) * (long)h->adj_blocks * gpb;
  }
  if (h->ws_base) return carve(h, &h->adj, (size_t)total * sizeof(T));
  if (total <= h->adj_elems_alloc) return QOC_OK;
  dfree(h, &h->adj, (size_t)h->adj_elems_alloc * sizeof(T));
  h->adj_elems_alloc = 0;
  qoc_status s = dalloc(h, &h->adj, (size_t)total * sizeof(T));
  if (s) return s;
  h->adj_elems_alloc = total;
  return QOC_OK;
}

// Partial sums of the first-order gradient contraction: Ns x slices x M.
qoc_status ensure_part(qoc_handle *h) {
  const long parts = (long)h->Ns * qoc::adjoint_big_slices(h->dp) * std::max(h->M, 1);
  if (h->ws_base) return carve(h, (void **)&h->adj_part, (size_t)parts * sizeof(double));
  if (parts <= h->adj_part_alloc) return QOC_OK;
  dfree(h, (void **)&h->adj_part, (size_t)h->adj_part_alloc * sizeof(double));
  h->adj_part_alloc = 0;
  qoc_status s = dalloc(h, (void **)&h->adj_part, (size_t)parts * sizeof(double));
  if (s) return s;
  h->adj_part_alloc = parts;
  return QOC_OK;
}

// In-block passes split over sub-blocks of SUB16 steps: FP32 chains at
// padded d 16 on the single-wavefront sweeps, with L a multiple of SUB16
// (at most 8 of them).
template <typename T> bool split_sweeps(const qoc_handle *h) {
  return sizeof(T) == 4 && h->dp == 16 && qoc::wave_sweep_ok<T>(h->dp, h->S) && h->L > qoc::SUB16 &&
         h->L % qoc::SUB16 == 0 && h->L <= 8 * qoc::SUB16;
}

// Union pattern and per-control nonzero lists of the (Hermitian parts of
// the) Hamiltonians, for the structured kernels of the batched path.
template <typename T>
qoc_status build_structure(qoc_handle *h, const std::vector<double> &h64) {
  const int d = h->d, M = h->M;
  if (h->dp < 64) return QOC_OK;  // the small-d path keeps dense tiles
  const size_t dd = (size_t)d * d;
  auto nz = [&](int k, size_t rc) { return h64[(k * dd + rc) * 2] != 0.0 || h64[(k * dd + rc) * 2 + 1] != 0.0; };
  std::vector<int> colptr(d + 1, 0), rowidx;
  for (int c = 0; c < d; ++c) {
    for (int r = 0; r < d; ++r) {
      bool any = false;
      for (int k = 0; k <= M && !any; ++k) any = nz(k, (size_t)r * d + c);
      if (any) rowidx.push_back(r);
    }
    colptr[c + 1] = (int)rowidx.size();
  }
  h->nnz_union = (long)rowidx.size();
  if (h->nnz_union * 4 > (long)dd) return QOC_OK;  // dense enough for the dense kernels
  std::vector<double> vals((size_t)h->nnz_union * (M + 1) * 2);
  for (int c = 0; c < d; ++c)
    for (int e = colptr[c]; e < colptr[c + 1]; ++e)
      for (int k = 0; k <= M; ++k) {
        const size_t rc = (size_t)rowidx[e] * d + c;
        vals[((size_t)e * (M + 1) + k) * 2] = h64[(k * dd + rc) * 2];
        vals[((size_t)e * (M + 1) + k) * 2 + 1] = h64[(k * dd + rc) * 2 + 1];
      }
  // union of the controls' patterns by rows, with the controls at each entry
  std::vector<int> rptr(d + 1, 0), rcol, eptr(1, 0), ek;
  std::vector<double> ev;
  for (int r = 0; r < d; ++r) {
    for (int c = 0; c < d; ++c) {
      const size_t rc = (size_t)r * d + c;
      bool any = false;
      for (int k = 1; k <= M; ++k)
        if (nz(k, rc)) {
          any = true;
          ek.push_back(k - 1);
          ev.push_back(h64[(k * dd + rc) * 2]);
          ev.push_back(h64[(k * dd + rc) * 2 + 1]);
        }
      if (any) {
        rcol.push_back(c);
        eptr.push_back((int)ek.size());
      }
    }
    rptr[r + 1] = (int)rcol.size();
  }
  h->nev = (long)ek.size();
  std::vector<T> eval(2 * std::max<long>(1, h->nev), (T)0);
  for (long q = 0; q < h->nev; ++q) {
    eval[q] = (T)ev[2 * q];
    eval[h->nev + q] = (T)ev[2 * q + 1];
  }
  qoc_status s;
#define ALLOC(ptr, bytes)                                        \
  if ((s = dalloc(h, (void **)&(ptr), (bytes))) != QOC_OK) return s;
  ALLOC(h->sp_colptr, (d + 1) * sizeof(int));
  ALLOC(h->sp_rowidx, std::max<long>(1, h->nnz_union) * sizeof(int));
  ALLOC(h->sp_vals, vals.size() * sizeof(double) + 16);
  ALLOC(h->sp_rptr, (d + 1) * sizeof(int));
  ALLOC(h->sp_rcol, std::max<size_t>(1, rcol.size()) * sizeof(int));
  ALLOC(h->sp_eptr, eptr.size() * sizeof(int));
  ALLOC(h->sp_ek, std::max<long>(1, h->nev) * sizeof(int));
  ALLOC(h->sp_eval, eval.size() * sizeof(T));
#undef ALLOC
  HIP_TRY(hipMemcpy(h->sp_colptr, colptr.data(), (d + 1) * sizeof(int), hipMemcpyHostToDevice));
  if (h->nnz_union) {
    HIP_TRY(hipMemcpy(h->sp_rowidx, rowidx.data(), rowidx.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->sp_vals, vals.data(), vals.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(h->sp_rptr, rptr.data(), (d + 1) * sizeof(int), hipMemcpyHostToDevice));
  if (!rcol.empty())
    HIP_TRY(hipMemcpy(h->sp_rcol, rcol.data(), rcol.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->sp_eptr, eptr.data(), eptr.size() * sizeof(int), hipMemcpyHostToDevice));
  if (h->nev) HIP_TRY(hipMemcpy(h->sp_ek, ek.data(), ek.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->sp_eval, eval.data(), eval.size() * sizeof(T), hipMemcpyHostToDevice));
  h->sp_built = true;
  // by default whenever recorded: on the batched transmon-chain instances
  // with a pattern (unions up to d^2 / 4) the structured contraction was
  // faster than the dense one on every instance measured
  h->sp_auto = true;
  return QOC_OK;
}

// Action form: the ELL layout of the union pattern of H_0 .. H_M over the
// padded rows (K slots per row, zero-valued padding slots at the row's own
// column), every matrix's slot values in FP64, the per-step value and
// partial-sum buffers, and for the gradient the union of the controls'
// patterns (rows, columns) with each control's entries and values.
template <typename T>
qoc_status build_action(qoc_handle *h, const std::vector<double> &h64) {
  const int d = h->d, dp = h->dp, M = h->M, N = h->N, S = h->S;
  const size_t dd = (size_t)d * d * 2;
  auto at = [&](int k, int r, int c) { return h64.data() + k * dd + 2 * ((size_t)r * d + c); };
  auto nz = [&](int k, int r, int c) {
    const double *x = at(k, r, c);
    return x[0] != 0.0 || x[1] != 0.0;
  };
  std::vector<std::vector<int>> rows(dp);
  size_t width = 1;
  for (int r = 0; r < d; ++r) {
    for (int c = 0; c < d; ++c)
      for (int k = 0; k <= M; ++k)
        if (nz(k, r, c)) {
          rows[r].push_back(c);
          break;
        }
    width = std::max(width, rows[r].size());
  }
  int K = 4;  // slot counts the chains are built for: 4, 8, 12, 16, 24, 32
  while ((size_t)K < width) K = K < 8 ? 8 : (K < 16 ? K + 4 : K + 8);
  if (!qoc::act_shape_ok<T>(dp, K))
    return fail(QOC_ERR_UNSUPPORTED,
                "the action form keeps each row's nonzeros in registers: the union pattern of "
                "H_0 .. H_M has " + std::to_string(width) + " per row (at most 32 in FP32 and 16 "
                "in FP64 for padded d <= 512, half that up to 1024)");
  h->actK = K;
  std::vector<int> ecol((size_t)K * dp);
  std::vector<double> hm((size_t)(M + 1) * K * 2 * dp, 0.0);
  for (int r = 0; r < dp; ++r)
    for (int kk = 0; kk < K; ++kk) {
      const bool real = kk < (int)rows[r].size();
      const int c = real ? rows[r][kk] : r;
      ecol[(size_t)kk * dp + r] = c;
      if (!real) continue;
      for (int k = 0; k <= M; ++k) {
        const double *x = at(k, r, c);
        double *o = hm.data() + (((size_t)k * K + kk) * 2) * dp;
        o[r] = x[0];
        o[dp + r] = x[1];
      }
    }
  // the controls' entries and each control's (entry, value) pairs
  std::vector<int> erow, ecol2, cptr(M + 1, 0), cent;
  std::vector<std::vector<std::pair<int, int>>> per(M);  // (entry, (r, c) index)
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      int e = -1;
      for (int k = 1; k <= M; ++k)
        if (nz(k, r, c)) {
          if (e < 0) {
            e = (int)erow.size();
            erow.push_back(r);
            ecol2.push_back(c);
          }
          per[k - 1].push_back({e, r * d + c});
        }
    }
  h->act_nent = (int)erow.size();
  for (int k = 0; k < M; ++k) cptr[k + 1] = cptr[k] + (int)per[k].size();
  h->act_npairs = cptr[M];
  std::vector<T> cval(2 * std::max<long>(1, h->act_npairs));
  for (int k = 0; k < M; ++k)
    for (size_t i = 0; i < per[k].size(); ++i) {
      const long pi = cptr[k] + (long)i;
      const int rc = per[k][i].second;
      const double *x = at(k + 1, rc / d, rc % d);
      cent.push_back(per[k][i].first);
      cval[pi] = (T)x[0];
      cval[h->act_npairs + pi] = (T)x[1];
    }
  if (M > 0 && qoc::act_grad_lds<T>(dp, h->act_nent) > 64 * 1024)
    return fail(QOC_ERR_UNSUPPORTED,
                "the action form's gradient keeps the controls' " +
                    std::to_string(h->act_nent) +
                    " pattern entries in LDS: too many for 64 KB at this d");
  qoc_status s;
#define ALLOC(ptr, bytes)                                        \
  if ((s = dalloc(h, (void **)&(ptr), (bytes))) != QOC_OK) return s;
  ALLOC(h->act_ecol, ecol.size() * sizeof(int));
  ALLOC(h->act_hm, hm.size() * sizeof(double));
  ALLOC(h->act_hv, (size_t)N * K * 2 * dp * sizeof(T));
  ALLOC(h->act_part, (size_t)N * S * std::max(1, M) * sizeof(double));
  ALLOC(h->act_erow, std::max<size_t>(1, erow.size()) * sizeof(int));
  ALLOC(h->act_ecol2, std::max<size_t>(1, ecol2.size()) * sizeof(int));
  ALLOC(h->act_cptr, cptr.size() * sizeof(int));
  ALLOC(h->act_cent, std::max<size_t>(1, cent.size()) * sizeof(int));
  ALLOC(h->act_cval, cval.size() * sizeof(T));
#undef ALLOC
  HIP_TRY(hipMemcpy(h->act_ecol, ecol.data(), ecol.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->act_hm, hm.data(), hm.size() * sizeof(double), hipMemcpyHostToDevice));
  if (!erow.empty()) {
    HIP_TRY(hipMemcpy(h->act_erow, erow.data(), erow.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->act_ecol2, ecol2.data(), ecol2.size() * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->act_cent, cent.data(), cent.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  HIP_TRY(hipMemcpy(h->act_cptr, cptr.data(), cptr.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->act_cval, cval.data(), cval.size() * sizeof(T), hipMemcpyHostToDevice));
  return QOC_OK;
}

template <typename T>
qoc_status alloc_all(qoc_handle *h, const qoc_problem_desc *desc) {
  const int d = h->d, dp = h->dp, M = h->M, N = h->N, S = h->S;
  const size_t mat = 2 * (size_t)dp * dp, set = 2 * (size_t)S * dp;
  qoc_status s;
#define ALLOC(ptr, bytes)                                        \
  if ((s = dalloc(h, (void **)&(ptr), (bytes))) != QOC_OK) return s;
  ALLOC(h->Hf, (M + 1) * mat * sizeof(T));
  ALLOC(h->H64, (size_t)(M + 1) * d * d * 2 * sizeof(double));
  ALLOC(h->u_dev, (size_t)std::max(1, M * N) * sizeof(double));
  ALLOC(h->out_dev, (size_t)(2 + N) * sizeof(double));
  ALLOC(h->grad_dev, (size_t)std::max(1, M * N) * sizeof(double));
  ALLOC(h->psi0, set * sizeof(T));
  ALLOC(h->psiT64, (size_t)S * d * 2 * sizeof(double));
  if (h->has_pen) {
    ALLOC(h->w64, (size_t)dp * sizeof(double));
    ALLOC(h->pw, (size_t)dp * sizeof(T));
  }
  // the action form forms no step propagator: no per-step matrix stacks
  const size_t Ns = h->prop == QOC_PROP_ACTION ? 0 : (size_t)h->Ns;
  ALLOC(h->X, Ns * mat * sizeof(T));
  ALLOC(h->Qa, Ns * mat * sizeof(T));
  ALLOC(h->Qb, Ns * mat * sizeof(T));
  if (h->nseg > 1) ALLOC(h->u_seg, (size_t)std::max(1, M) * Ns * sizeof(double));
  if (qoc::wave_sweep_ok<T>(dp, S)) ALLOC(h->Eh, (size_t)h->nb * mat * sizeof(T));
  // state buffers carry kRingSlack elements of padding: the small-d sweeps
  // load fixed-size ring slots that may run past the last state set
  const size_t slack = kRingSlack;
  if (split_sweeps<T>(h)) {
    const size_t nsub = ((size_t)N + qoc::SUB16 - 1) / qoc::SUB16;
    ALLOC(h->Es, nsub * mat * sizeof(T));
    ALLOC(h->Ehs, nsub * mat * sizeof(T));
    if (h->has_pen) ALLOC(h->nu, (nsub * set + slack) * sizeof(T));
  }
  ALLOC(h->ckpt, ((size_t)(h->nb + 1) * set + slack) * sizeof(T));
  ALLOC(h->lam_ckpt, ((size_t)(h->nb + 1) * set + slack) * sizeof(T));
  if (h->has_pen || h->has_ext) ALLOC(h->mu, ((size_t)h->nb * set + slack) * sizeof(T));
  ALLOC(h->psi_buf, ((size_t)(N + 1) * set + slack) * sizeof(T));
  ALLOC(h->lam_buf, ((size_t)N * set + slack) * sizeof(T));
  // theta, drift, norm ticket, (unused), norm accumulator
  ALLOC(h->bits, 8 * sizeof(unsigned long long));
  HIP_TRY(hipMemset(h->bits, 0, 8 * sizeof(unsigned long long)));  // ticket, accumulator start at zero
  ALLOC(h->zinfo, (size_t)(3 + 2 * S) * sizeof(double));
  h->npart = std::max(1, std::min(1024, (N + 3) / 4));
  ALLOC(h->part, (size_t)4 * h->npart * sizeof(double));
  if (h->has_ext) {
    if (h->nf > 0) ALLOC(h->forb64, (size_t)h->nf * d * 2 * sizeof(double));
    ALLOC(h->src, (size_t)(N + 1) * set * sizeof(T));
    h->next = std::max(1, std::min(1024, (N + 3) / 4));
    ALLOC(h->ext_part, (size_t)2 * h->next * sizeof(double));
  }
  ALLOC(h->pn_dev, 4 * sizeof(int));
  ALLOC(h->sc_dev, 2 * sizeof(double));
  // no pair yet: the first speculative pass of the padded-d-16 kernel is redone
  HIP_TRY(hipMemset(h->pn_dev, 0, 4 * sizeof(int)));
  HIP_TRY(hipMemset(h->sc_dev, 0, 2 * sizeof(double)));
#undef ALLOC
  if (hipHostMalloc((void **)&h->h_u, (size_t)std::max(1, M * N) * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void **)&h->h_out, (size_t)(2 + N + 2 * S * d) * sizeof(double)) !=
          hipSuccess ||
      hipHostMalloc((void **)&h->h_grad, (size_t)std::max(1, M * N) * sizeof(double)) !=
          hipSuccess)
    return fail(QOC_ERR_NOMEM, "pinned host staging allocation failed");

  // upload problem data (padded planar copies in the chain precision)
  // Hermitian parts (H + H^dagger) / 2 of the (validated, Hermitian to
  // 1e-12) inputs: the device copies are exactly Hermitian, so every
  // assembled X_j = -i s H_j is exactly anti-Hermitian in the chain
  // precision (the per-step derivative relies on X^H = -X)
  std::vector<double> h64((size_t)(M + 1) * d * d * 2);
  for (int k = 0; k <= M; ++k) {
    const double *src = (k == 0) ? desc->H0 : desc->Hk + (size_t)(k - 1) * d * d * 2;
    double *dst = h64.data() + (size_t)k * d * d * 2;
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c) {
        const size_t rc = 2 * ((size_t)r * d + c), cr = 2 * ((size_t)c * d + r);
        dst[rc] = 0.5 * (src[rc] + src[cr]);
        dst[rc + 1] = r == c ? 0.0 : 0.5 * (src[rc + 1] - src[cr + 1]);
      }
  }
  std::vector<T> hf((M + 1) * mat, (T)0);
  for (int k = 0; k <= M; ++k) {
    const double *src = h64.data() + (size_t)k * d * d * 2;
    T *re = hf.data() + k * mat, *im = re + (size_t)dp * dp;
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c) {
        re[(size_t)r * dp + c] = (T)src[2 * ((size_t)r * d + c)];
        im[(size_t)r * dp + c] = (T)src[2 * ((size_t)r * d + c) + 1];
      }
  }
  HIP_TRY(hipMemcpy(h->Hf, hf.data(), hf.size() * sizeof(T), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->H64, h64.data(), h64.size() * sizeof(double), hipMemcpyHostToDevice));
  if ((s = build_structure<T>(h, h64)) != QOC_OK) return s;
  if (h->prop == QOC_PROP_ACTION && (s = build_action<T>(h, h64)) != QOC_OK) return s;
  std::vector<T> ps(set, (T)0);
  for (int s2 = 0; s2 < S; ++s2)
    for (int m = 0; m < d; ++m) {
      ps[(size_t)s2 * dp + m] = (T)desc->psi0[2 * ((size_t)s2 * d + m)];
      ps[(size_t)S * dp + (size_t)s2 * dp + m] = (T)desc->psi0[2 * ((size_t)s2 * d + m) + 1];
    }
  HIP_TRY(hipMemcpy(h->psi0, ps.data(), set * sizeof(T), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->psiT64, desc->psiT, (size_t)S * d * 2 * sizeof(double),
                    hipMemcpyHostToDevice));
  if (h->nf > 0)
    HIP_TRY(hipMemcpy(h->forb64, desc->forbidden, (size_t)h->nf * d * 2 * sizeof(double),
                      hipMemcpyHostToDevice));
  if (h->has_pen) {
    std::vector<double> w(dp, 0.0);
    std::vector<T> pw(dp, (T)0);
    for (int m = 0; m < d; ++m) {
      w[m] = desc->penalty_w[m];
      pw[m] = (T)(h->a_pen / S * desc->penalty_w[m]);
    }
    HIP_TRY(hipMemcpy(h->w64, w.data(), dp * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->pw, pw.data(), dp * sizeof(T), hipMemcpyHostToDevice));
  }
  return QOC_OK;
}

// ------------------------------------------------------------------ pipeline
// Paterson-Stockmeyer evaluation of D^(0) = T_p(X) - I = sum_{k=1..p} X^k/k!
// (the same polynomial as the Horner form, fewer products): powers
// X^2 .. X^s (s - 1 products), then Horner in Y = X^s over the blocks
// B_q = sum_{r<s} c_{qs+r} X^r (X^0 = I, c_0 = 0, c_k = 0 beyond p):
// W_Q = B_Q, W_q = B_q + Y W_{q+1}, D^(0) = W_0.  When s divides p,
// B_Q = c_p I and W_{Q-1} = B_{Q-1} + c_p Y needs no product.
struct PsPlan {
  int s, Q, rem, cost;
};
PsPlan ps_plan(int p) {
  PsPlan best{0, 0, 0, 1 << 30};
  for (int s = 2; s <= std::min(p, 4); ++s) {
    const int Q = p / s, rem = p - Q * s;
    const int cost = (s - 1) + Q - (rem == 0 ? 1 : 0);
    if (cost < best.cost) best = PsPlan{s, Q, rem, cost};
  }
  return best;
}

// Products that evaluate T_p(X) on the batched path: Paterson-Stockmeyer
// when it takes fewer than Horner's p - 1.
int batched_products(int p) { return std::min(p - 1, ps_plan(p).cost); }

// The batched path's pair: the fewest evaluated products
// batched_products(p) + n within the bound, with theta / 2^n <= 1 (the
// series terms do not grow), ties toward the lower order p (the exact
// derivative runs p - 1 reverse Horner stages; measured at d 96 - 128, N
// 1500, S 2: (13, 0) 8 % slower per call than (8, 2) at equal products).
bool taylor_select_ps(double theta, double tol, int *p_out, int *n_out) {
  int best = -1, bp = 0, bn = 0;
  for (int n = 0; n < 60; ++n) {
    if (std::ldexp(theta, -n) > 1.0) continue;
    if (best >= 0 && n >= best) break;  // n alone already costs as much
    for (int p = 2; p <= 30; ++p) {
      if (taylor_bound(theta, p, n) <= tol) {
        const int c = batched_products(p) + n;
        if (best < 0 || c < best || (c == best && p < bp)) {
          best = c;
          bp = p;
          bn = n;
        }
        break;
      }
    }
  }
  if (best < 0) return false;
  *p_out = bp;
  *n_out = bn;
  return true;
}

// bf16x3 handles under the automatic class policy: the pair whose Taylor
// products and squarings take the least modelled time, a split product
// counting bf3_product_cost(d_pad) of an FP32 one (the measured ratio of the
// stage kernels, every class split, pair (8, 2): d_pad 64 0.79, 128 0.56,
// 256 0.48, 512 0.42; 1 where the chain has no split kernel), with the
// classes the policy allows at that pair (fewer squarings raise
// theta / 2^n and with it the split's error index, so the cheapest pair in
// products may run unsplit); ties toward the lower order p.
double bf3_product_cost(int dp) {
  if (!qoc::stage_bf3_ok(dp)) return 1.0;
  return dp <= 64 ? 0.79 : dp <= 128 ? 0.56 : dp <= 256 ? 0.48 : 0.42;
}
bool taylor_select_bf3(double theta, double tol, int N, int L, int dp, int *p_out, int *n_out) {
  const double cost = bf3_product_cost(dp);
  double best = -1.0;
  int bp = 0, bn = 0;
  for (int n = 0; n < 60; ++n) {
    if (std::ldexp(theta, -n) > 1.0) continue;
    if (best >= 0.0 && n * cost >= best) break;
    for (int p = 2; p <= 30; ++p) {
      if (taylor_bound(theta, p, n) <= tol) {
        const int cls = bf3_auto_classes(theta, n, N, L);
        const double t = batched_products(p) * ((cls & QOC_BF3_TAYLOR) ? cost : 1.0) +
                         n * ((cls & QOC_BF3_SQUARING) ? cost : 1.0);
        if (best < 0.0 || t < best - 1e-9 || (t <= best + 1e-9 && p < bp)) {
          best = t;
          bp = p;
          bn = n;
        }
        break;
      }
    }
  }
  if (best < 0.0) return false;
  *p_out = bp;
  *n_out = bn;
  return true;
}

template <typename T>
hipError_t taylor_ps(qoc_handle *h, const PsPlan &ps, int p, int nslots, T *X, T *Qa, T *Qb,
                     T *Dl, long lev, long mat, int N, int dp, int bf3, hipStream_t st) {
  const int s = ps.s;
  std::vector<double> c(p + s + 1, 0.0);
  {
    double f = 1.0;
    for (int k = 1; k <= p; ++k) {
      f *= k;
      c[k] = 1.0 / f;
    }
  }
  // storage: P[1] = X, P[2] = Qa, P[3] = Qb, P[4] and the two Horner
  // panels in level slots 1.. (free until the squarings)
  std::vector<T *> tmp;
  for (int i = 1; i < nslots; ++i) tmp.push_back(Dl + (long)i * lev);
  size_t ti = 0;
  T *P[5] = {nullptr, X, Qa, Qb, nullptr};
  if (s == 4) P[4] = tmp[ti++];
  T *Wa = tmp[ti++], *Wb = tmp[ti++];
  const int H = ps.rem == 0 ? ps.Q - 1 : ps.Q;  // Horner products
  // destination of the Horner output i (i = -1: the panel formed with the
  // last power); the last one is D^(0) in level slot 0
  auto dest = [&](int i) -> T * {
    if (i == H - 1) return Dl;
    return ((H - 1 - i) & 1) ? Wa : Wb;
  };
  auto B = [&](int q, qoc::StageArgs<T> &a, bool second) {
    // addends of B_q: X^0 -> gamma, X^1 .. X^(s-1) -> extra addends
    T *g = second ? &a.g2 : &a.gamma;
    *g = (T)c[q * s];
    for (int r = 1; r < s; ++r) {
      a.xadd[r - 1] = P[r];
      (second ? a.xc2 : a.xc)[r - 1] = (T)c[q * s + r];
    }
    a.nx = s - 1;
  };
  for (int r = 2; r <= s; ++r) {
    qoc::StageArgs<T> a{P[r - 1], mat, X, mat, P[r], mat, N, dp, (T)1, (T)0, (T)0, (T)0, bf3};
    if (r == s) {
      // second output: W_Q = B_Q, or W_{Q-1} = B_{Q-1} + c_p Y when s | p
      a.C2 = dest(-1);
      if (ps.rem == 0) {
        B(ps.Q - 1, a, true);
        a.c2P = (T)c[p];
      } else {
        B(ps.Q, a, true);
      }
    }
    PhaseTimer tm(h, QOC_PHASE_TAYLOR, st);
    hipError_t e = qoc::launch_stage<T>(0, a, st);
    if (e != hipSuccess) return e;
  }
  const int q0 = ps.rem == 0 ? ps.Q - 2 : ps.Q - 1;
  for (int i = 0; i < H; ++i) {
    const int q = q0 - i;
    qoc::StageArgs<T> a{P[s], mat, dest(i - 1), mat, dest(i), mat, N, dp, (T)1, (T)0, (T)0,
                        (T)0, bf3};
    B(q, a, false);
    PhaseTimer tm(h, QOC_PHASE_TAYLOR, st);
    hipError_t e = qoc::launch_stage<T>(0, a, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Whether a handle runs the small-d path (device-side (p, n), chains in LDS).
bool on_small_path(const qoc_handle *h) {
  return h->prec == QOC_FP64
             ? (qoc::small_expm_ok<double>(h->dp) && qoc::small_sweep_ok<double>(h->dp, h->S))
             : (qoc::small_expm_ok<float>(h->dp) && qoc::small_sweep_ok<float>(h->dp, h->S));
}

// A fixed pair within the capacity of the handle's path: p <= 16 and
// n <= 16 on the small-d path (its preallocated levels and chains), p <= 30
// and n <= 60 on the batched path (the device-side check of the pair).
qoc_status check_fixed_pair(const qoc_handle *h, int p, int n) {
  if (p == 0) return QOC_OK;
  const bool sp = on_small_path(h);
  const int pc = sp ? kSmallPCap : 30, nc = sp ? kSmallNCap : 60;
  if (p > pc || n > nc)
    return fail(QOC_ERR_UNSUPPORTED, "fixed (p, n) = (" + std::to_string(p) + ", " +
                                         std::to_string(n) + ") exceeds this path's capacity (p <= " +
                                         std::to_string(pc) + ", n <= " + std::to_string(nc) + ")");
  return QOC_OK;
}

// A fixed (p, n) on the small-d path, as the device applies it (clamped to
// the preallocated capacity), and the cotangent rank bound it implies.
std::pair<int, int> small_fixed_pn(const qoc_handle *h) {
  return {std::min(h->fixed_p, kSmallPCap), std::min(h->fixed_n, kSmallNCap)};
}
int small_fixed_rcap(const qoc_handle *h) {
  const int n = small_fixed_pn(h).second;
  const long raw = n >= 30 ? h->dp : std::min<long>((long)h->S << n, h->dp);
  return (int)std::min<long>((raw + 15) & ~15L, h->dp);
}
template <typename T> bool small_big_adjoint(const qoc_handle *h) {
  return h->fixed_p >= 2 && h->dp >= 32 && !qoc::adjoint16_ok<T>(h->dp, kSmallPCap);
}

// Block products for a checkpoint interval L that is not a power of two:
// a pairwise tree inside every block (the blocks' trees side by side),
// E_b = U_{bL+L-1} ... U_{bL} - I in D-form (C = A + B + A B).  At each
// level the c elements of a full block pair up as (2i, 2i + 1) -> i, one
// stage launch over all full blocks (segments of c / 2 products), an odd
// last element carried by a strided copy; the shorter last block runs its
// own launches into the slot after the full blocks, so every level's
// results are contiguous per block and the final E_b are contiguous.
template <typename T>
hipError_t block_tree_any(qoc_handle *h, const T *D, long N, T *Qa, T *Qb, long mat, int bf3,
                          hipStream_t st, const T **E_out) {
  const long L = h->L, nb = (N + L - 1) / L;
  const long nfull = N / L, clast = N - nfull * L;  // clast: steps of a short last block
  long c = L, cl = clast;  // elements per full block and in the short block at this level
  const T *in = D;
  long in_stride = L * mat;  // between full blocks at this level
  long in_last = nfull * L * mat;  // offset of the short block's elements
  T *out = Qa;
  while (c > 1 || cl > 1) {
    const long c2 = (c + 1) / 2, cl2 = (cl + 1) / 2;
    const long out_stride = c2 * mat, out_last = nfull * c2 * mat;
    if (c > 1 && nfull > 0) {
      qoc::StageArgs<T> a{in + mat, 2 * mat, in, 2 * mat, out, mat, (int)(nfull * (c / 2)),
                          h->dp, (T)1, (T)1, (T)1, (T)0, bf3};
      a.seg = (int)(c / 2);
      a.segA = a.segB = in_stride;
      a.segC = out_stride;
      PhaseTimer tm(h, QOC_PHASE_BLOCKPROD, st);
      hipError_t e = qoc::launch_stage<T>(0, a, st);
      if (e != hipSuccess) return e;
    }
    if (nfull > 0 && (c & 1)) {
      // the odd element of every full block, carried (c == 1: the block's
      // product is already complete and moves to this level's buffer)
      hipError_t e = qoc::launch_copy_strided<T>(out + (c2 - 1) * mat, out_stride,
                                                 in + (c - 1) * mat, in_stride, mat, nfull, st);
      if (e != hipSuccess) return e;
    }
    if (cl > 1) {
      qoc::StageArgs<T> a{in + in_last + mat, 2 * mat, in + in_last, 2 * mat, out + out_last,
                          mat, (int)(cl / 2), h->dp, (T)1, (T)1, (T)1, (T)0, bf3};
      PhaseTimer tm(h, QOC_PHASE_BLOCKPROD, st);
      hipError_t e = qoc::launch_stage<T>(0, a, st);
      if (e != hipSuccess) return e;
    }
    if (cl > 0 && (cl & 1)) {
      hipError_t e = qoc::launch_copy<T>(out + out_last + (cl2 - 1) * mat,
                                         in + in_last + (cl - 1) * mat, mat, st);
      if (e != hipSuccess) return e;
    }
    c = c2;
    cl = cl2;
    in = out;
    in_stride = out_stride;
    in_last = out_last;
    out = (out == Qa) ? Qb : Qa;
  }
  (void)nb;
  *E_out = in;
  return hipSuccess;
}

// Batched path: the FP64 norms of all N steps and the global (p, n) (fixed,
// or chosen on the host from theta_max read back).
template <typename T>
qoc_status choose_pn_large(qoc_handle *h, const double *u_dev, hipStream_t st,
                           const qoc::SparseU *spu, int *p, int *n, bool action = false) {
  {
    PhaseTimer tm(h, QOC_PHASE_NORM, st);
    // a fixed (p, n) is checked against the tolerance on the device
    // (status 2 in pn_dev), so the call needs no host round trip
    qoc::SelectArgs sel{nullptr, nullptr, (unsigned *)(h->bits + 2), h->tol, 60, 30, 0, 0,
                        h->bits + 4};
    if (h->fixed_p >= 2)
      sel = qoc::SelectArgs{h->pn_dev, h->sc_dev, (unsigned *)(h->bits + 2), h->tol, 60, 30,
                            h->fixed_p, h->fixed_n, h->bits + 4};
    HIP_TRY(qoc::launch_norm(h->H64, u_dev, h->d, h->M, h->N, h->dt, h->bits, sel, st, spu));
  }
  if (h->fixed_p >= 2) {
    *p = h->fixed_p;
    *n = h->fixed_n;
    return QOC_OK;
  }
  if (h->capturing)
    return fail(QOC_ERR_UNSUPPORTED,
                "choosing (p, n) per call reads theta_max back to the host, which a stream "
                "that captures a HIP graph cannot do: fix the pair with qoc_set_taylor "
                "before capturing");
  unsigned long long tb = 0;
  HIP_TRY(hipMemcpyAsync(&tb, h->bits, sizeof(tb), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double theta;
  std::memcpy(&theta, &tb, sizeof(theta));
  h->last_theta = theta;
  if (!std::isfinite(theta)) return fail(QOC_ERR_NONFINITE, "non-finite step norm");
  const bool ok = action ? action_select(theta, h->tol, p, n)
                  : (h->bf3 && h->bf3_req < 0)
                      ? taylor_select_bf3(theta, h->tol, h->N, h->L, h->dp, p, n)
                      : taylor_select_ps(theta, h->tol, p, n);
  if (!ok)
    return fail(QOC_ERR_UNSUPPORTED, "no (p, n) meets the tolerance for theta_max = " +
                                         std::to_string(theta));
  return QOC_OK;
}

// Paterson-Stockmeyer temporaries beyond the levels 1..n: the two ping-pong
// panels and, for s = 4, the fourth power.
int ps_extra_levels(int p, int n) {
  const PsPlan ps = ps_plan(p);
  const bool use_ps = ps.cost < p - 1;
  const int need = use_ps ? 2 + (ps.s == 4 ? 1 : 0) : 0;
  return std::max(0, need - n);
}

// Batched path, once (p, n) is known: the work space of this call and the
// product classes that run as bf16x3 split products.
template <typename T>
qoc_status prepare_large(qoc_handle *h, int p, int n, bool want_grad, int Rcap) {
  qoc_status s = ensure_levels<T>(h, n + 1 + ps_extra_levels(p, n));
  if (s) return s;
  if (want_grad && (s = ensure_adjoint<T>(h, p, Rcap, qoc::adjoint_big_ok<T>(h->dp))) != QOC_OK)
    return s;
  h->last_p = p;
  h->last_n = n;
  int cls = 0;
  h->bf3_fallback = 0;
  if (h->bf3) {
    if (h->bf3_req >= 0) {
      cls = h->bf3_req;
    } else {
      const double th = h->fixed_p >= 2 ? theta_admitted(p, n, h->tol) : h->last_theta;
      cls = bf3_auto_classes(th, n, h->N, h->L);
      h->bf3_fallback = cls != QOC_BF3_ALL;
    }
  }
  // the chain classes have split kernels only for padded d a multiple of 64
  if (!qoc::stage_bf3_ok(h->dp)) cls &= QOC_BF3_ADJOINT;
  h->bf3_used = cls;
  h->bf3_adj_ran = 0;
  return QOC_OK;
}

// Batched path: the step exponentials D_j = U_j - I of Nloc consecutive
// steps with controls u_loc (M x Nloc) -- assembly, Taylor (Horner or
// Paterson-Stockmeyer) in D-form, n squarings -- and their block products
// E_b (blocks of L).  Stacks of Nloc matrices, levels at stride Nloc.
template <typename T>
hipError_t exps_large(qoc_handle *h, const double *u_loc, int Nloc, int p, int n, hipStream_t st,
                      const T **D_out, const T **E_out) {
  const int dp = h->dp, M = h->M;
  const long mat = 2L * dp * dp, lev = (long)Nloc * mat;
  T *X = (T *)h->X, *Qa = (T *)h->Qa, *Qb = (T *)h->Qb, *Dl = (T *)h->Dlev;
  const int cls = h->bf3_used;
  const int bT = (cls & QOC_BF3_TAYLOR) ? 1 : 0, bS = (cls & QOC_BF3_SQUARING) ? 1 : 0,
            bB = (cls & QOC_BF3_BLOCKPROD) ? 1 : 0;
  const PsPlan ps = ps_plan(p);
  const bool use_ps = ps.cost < p - 1;
  const int ps_extra = ps_extra_levels(p, n);
  hipError_t e;
  const double sc = std::ldexp(h->dt, -n);
  {
    PhaseTimer tm(h, QOC_PHASE_ASSEMBLE, st);
    if ((e = qoc::launch_assemble<T>((const T *)h->Hf, u_loc, dp, M, Nloc, (T)sc, (T)(1.0 / p), X,
                                     use_ps ? nullptr : Qa, st)) != hipSuccess)
      return e;
  }
  if (use_ps) {
    if ((e = taylor_ps<T>(h, ps, p, n + 1 + ps_extra, X, Qa, Qb, Dl, lev, mat, Nloc, dp, bT, st)) !=
        hipSuccess)
      return e;
  } else {
    T *cur = Qa, *nxt = Qb;
    for (int k = p - 1; k >= 2; --k) {
      qoc::StageArgs<T> a{X, mat, cur, mat, nxt, mat, Nloc, dp, (T)(1.0 / k), (T)0, (T)0, (T)1,
                          bT};
      PhaseTimer tm(h, QOC_PHASE_TAYLOR, st);
      if ((e = qoc::launch_stage<T>(0, a, st)) != hipSuccess) return e;
      std::swap(cur, nxt);
    }
    qoc::StageArgs<T> a{X, mat, cur, mat, Dl, mat, Nloc, dp, (T)1, (T)0, (T)0, (T)0, bT};
    PhaseTimer tm(h, QOC_PHASE_TAYLOR, st);
    if ((e = qoc::launch_stage<T>(0, a, st)) != hipSuccess) return e;
  }
  for (int i = 0; i < n; ++i) {
    qoc::StageArgs<T> a{Dl + i * lev, mat, Dl + i * lev, mat, Dl + (i + 1) * lev, mat, Nloc, dp,
                        (T)1, (T)0, (T)2, (T)0, bS};
    PhaseTimer tm(h, QOC_PHASE_TAYLOR, st);
    if ((e = qoc::launch_stage<T>(0, a, st)) != hipSuccess) return e;
  }
  const T *D = Dl + (long)n * lev;
  *D_out = D;
  // ---- block products E_b (pairwise tree, D-form: C = A + B + A B)
  if (h->L & (h->L - 1)) return block_tree_any<T>(h, D, Nloc, Qa, Qb, mat, bB, st, E_out);
  long cnt = Nloc;
  const T *in = D;
  T *outb = Qa;
  for (int span = 2; span <= h->L; span <<= 1) {
    const long pairs = cnt / 2;
    qoc::StageArgs<T> a{in + mat, 2 * mat, in, 2 * mat, outb, mat, (int)pairs, dp,
                        (T)1, (T)1, (T)1, (T)0, bB};
    PhaseTimer tm(h, QOC_PHASE_BLOCKPROD, st);
    if ((e = qoc::launch_stage<T>(0, a, st)) != hipSuccess) return e;
    tm.done();
    if (cnt & 1)
      if ((e = qoc::launch_copy<T>(outb + pairs * mat, in + (cnt - 1) * mat, mat, st)) !=
          hipSuccess)
        return e;
    cnt = (cnt + 1) / 2;
    in = outb;
    outb = (outb == Qa) ? Qb : Qa;
  }
  *E_out = in;
  return hipSuccess;
}

// Sweep and cost arguments over the whole horizon.
template <typename T>
qoc::SweepArgs<T> sweep_args(const qoc_handle *h, const T *D, const T *E, const double *u_dev,
                             double *out_dev) {
  qoc::SweepArgs<T> sw{};
  sw.N = h->N; sw.L = h->L; sw.nb = h->nb; sw.dp = h->dp; sw.d = h->d; sw.S = h->S; sw.M = h->M;
  sw.D = D; sw.E = E; sw.psi0 = (const T *)h->psi0; sw.ckpt = (T *)h->ckpt;
  sw.psi_buf = (T *)h->psi_buf; sw.lam_ckpt = (T *)h->lam_ckpt; sw.mu = (T *)h->mu;
  sw.lam_buf = (T *)h->lam_buf; sw.w64 = h->w64; sw.pw = (const T *)h->pw;
  sw.drift_bits = h->bits + 1; sw.psiT64 = h->psiT64; sw.u = u_dev;
  sw.alpha_fid = h->a_fid; sw.alpha_pen = h->a_pen; sw.alpha_amp = h->a_amp;
  sw.alpha_var = h->a_var; sw.fid_mode = h->fid_mode; sw.out = out_dev; sw.zinfo = h->zinfo;
  sw.part = h->part; sw.npart = h->npart;
  if (h->has_ext) {
    sw.src = (const T *)h->src;
    sw.ext_part = h->ext_part;
    sw.next = h->next;
    sw.alpha_time = h->a_time;
  }
  return sw;
}

// The cost from the states of the whole horizon: fidelity and lambda_N
// beside the penalties in one launch, then (with source terms) the
// forbidden-state occupancies, time-optimal fidelities and costate sources,
// then the total.
template <typename T>
hipError_t launch_cost_all(qoc_handle *h, const qoc::SweepArgs<T> &sw, bool total, hipStream_t st) {
  PhaseTimer tm(h, QOC_PHASE_COST, st);
  hipError_t e = qoc::launch_cost<T>(sw, st);
  if (e != hipSuccess) return e;
  if (h->has_ext) {
    const long set = 2L * h->S * h->dp;
    const qoc::ExtArgs<T> ea{h->forb64, h->nf, h->a_time, (T *)h->src,
                             (T *)h->lam_ckpt + (long)h->nb * set, h->ext_part, h->next};
    if ((e = qoc::launch_ext<T>(sw, ea, st)) != hipSuccess) return e;
  }
  return total ? qoc::launch_total<T>(sw, st) : hipSuccess;
}

// The sweep kernels of a call: one wavefront (S d_pad <= 64), one workgroup
// with a prefetch ring (d_pad <= 64), chain workgroups, per-step launches of
// many workgroups, or the generic per-block kernels, which alone carry the
// per-step source terms (forbidden states, time-optimal term).
struct SweepPick {
  bool ext, wave, small, wide_ok;
};

template <typename T>
hipError_t launch_sweep(const qoc_handle *h, const SweepPick &k, int which,
                        const qoc::SweepArgs<T> &sw, hipStream_t st) {
  const int dp = h->dp, S = h->S;
  const int mode = h->sweep_mode[which];
  if (k.ext) {
    switch (which) {
      case 0: return qoc::launch_fwd_blocks<T>(sw, st);
      case 1: return qoc::launch_fwd_replay<T>(sw, st);
      case 2: return qoc::launch_bwd_blocks<T>(sw, st);
      default: return qoc::launch_bwd_pairs<T>(sw, st);
    }
  }
  if (k.wave && !(mode == 3 && qoc::small_sweep_ok<T>(dp, S)))
    return qoc::launch_wave_sweep<T>(which, sw, st);
  // chain workgroups: by default for FP32 padded d 64 .. 128 (measured at
  // padded d 64, S = 2, N ~ 2900: 1.8 ms per call against 3.7 ms with the
  // four-wavefront LDS sweeps)
  if (qoc::chain_sweep_ok<T>(dp, S) && (mode == 4 || (mode == 0 && dp >= 64)))
    return qoc::launch_chain_sweep<T>(which, sw, st);
  if (k.wave || k.small) return qoc::launch_small_sweep<T>(which, sw, st);
  // per-step launches: the block sweeps (F2, B2) from padded d 80, the
  // in-block passes (F3, B3) from 256, unless set per handle; by default
  // (and as variant 5) their products run on the MFMA (measured at padded
  // d 512, S = 8, N = 1000: the four sweeps 2.2 ms per call against 6.3 ms
  // with the VALU products of variant 2)
  if (k.wide_ok && mode == 5) return qoc::launch_wide_sweep<T>(which, sw, st, true);
  const bool wide =
      k.wide_ok && (mode == 2 || (mode == 0 && (which == 0 || which == 2 || dp >= 256)));
  if (wide) return qoc::launch_wide_sweep<T>(which, sw, st, mode == 0);
  switch (which) {
    case 0: return qoc::launch_fwd_blocks<T>(sw, st);
    case 1: return qoc::launch_fwd_replay<T>(sw, st);
    case 2: return qoc::launch_bwd_blocks<T>(sw, st);
    default: return qoc::launch_bwd_pairs<T>(sw, st);
  }
}

template <typename T>
qoc_status run(qoc_handle *h, const double *u_dev, double *out_dev, double *grad_dev,
               hipStream_t st, bool want_grad) {
  const int dp = h->dp, N = h->N, M = h->M, S = h->S;
  // structured Hamiltonians (batched path): norm and gradient contraction
  // over their nonzeros
  const bool sp_on = h->sp_built && (h->sp_mode == 1 || (h->sp_mode < 0 && h->sp_auto));
  h->sp_used = sp_on;
  const qoc::SparseU spu{h->sp_colptr, h->sp_rowidx, h->sp_vals};
  const long mat = 2L * dp * dp;
  const long lev = (long)N * mat;
  const bool small_path = qoc::small_expm_ok<T>(dp) && qoc::small_sweep_ok<T>(dp, S);
  T *X = (T *)h->X, *Qa = (T *)h->Qa, *Qb = (T *)h->Qb;
  const T *D = nullptr, *E = nullptr;
  int p = 0, n = 0, Rcap_used = dp;
  // the single-wavefront sweeps read D^H / E^H (written by the small-path
  // kernels into Qb, unused there, and Eh)
  T *Dh_small = (small_path && h->Eh) ? Qb : nullptr;
  if (small_path) {
    // ---- no host round trip: (p, n) chosen on the device, fused chains
    const int n_cap = kSmallNCap, p_cap = kSmallPCap;
    qoc_status s = ensure_levels<T>(h, n_cap + 1);
    if (s) return s;
    if (want_grad && !qoc::adjoint16_ok<T>(dp, p_cap)) {
      if (small_big_adjoint<T>(h))
        s = ensure_adjoint<T>(h, small_fixed_pn(h).first, small_fixed_rcap(h), true);
      else
        s = ensure_adjoint<T>(h, p_cap, dp, false);
      if (s) return s;
    }
    const qoc::SelectArgs sel{h->pn_dev, h->sc_dev, (unsigned *)(h->bits + 2), h->tol, n_cap,
                              p_cap, h->fixed_p, h->fixed_n, h->bits + 4};
    // padded d 16: the norms ride along the exponential pass (its workgroup
    // maxima kept in `part`, free until the cost kernel), the (p, n) choice
    // and any recompute along the block products
    const qoc::Norm16 nm{h->H64, h->d, h->dt, h->bits, (unsigned long long *)h->part, sel};
    const bool subs = h->Es && Dh_small;
    const qoc::Pick16<T> pick{nm, (int)qoc::expm16_blocks<T>(N), (const T *)h->Hf, u_dev, M, X,
                              (T *)h->Dlev, Dh_small, subs ? (T *)h->Es : nullptr,
                              subs ? (T *)h->Ehs : nullptr};
    if (dp == 16) {
      PhaseTimer tm(h, QOC_PHASE_TAYLOR, st);
      HIP_TRY(qoc::launch_expm16<T>((const T *)h->Hf, u_dev, M, N, X, (T *)h->Dlev, Dh_small, nm,
                                    st));
    } else {
      {
        PhaseTimer tm(h, QOC_PHASE_NORM, st);
        HIP_TRY(qoc::launch_norm(h->H64, u_dev, h->d, M, N, h->dt, h->bits, sel, st));
      }
      PhaseTimer tm(h, QOC_PHASE_TAYLOR, st);
      HIP_TRY(qoc::launch_expm_small<T>((const T *)h->Hf, u_dev, dp, M, N, h->pn_dev, h->sc_dev,
                                        X, (T *)h->Dlev, Dh_small, st));
    }
    D = (const T *)h->Dlev;  // slot 0 = D^(n)
    {
      PhaseTimer tm(h, QOC_PHASE_BLOCKPROD, st);
      HIP_TRY(qoc::launch_blockprod_small<T>(D, dp, N, h->L, h->nb, Qa, (T *)h->Eh,
                                             dp == 16 ? &pick : nullptr, st));
    }
    E = Qa;
  } else {
    // ---- (p, n): fixed, or from theta_max (FP64 norms on the device)
    qoc_status s = choose_pn_large<T>(h, u_dev, st, sp_on ? &spu : nullptr, &p, &n);
    if (s) return s;
    const int Rraw = (long)S << std::min(n, 30) > dp ? dp : (S << n);
    Rcap_used = std::min((Rraw + 15) & ~15, dp);
    if ((s = prepare_large<T>(h, p, n, want_grad, Rcap_used)) != QOC_OK) return s;
    HIP_TRY(exps_large<T>(h, u_dev, N, p, n, st, &D, &E));
  }
  // FP64 unitarity drift of the final propagators (a diagnostic; at padded
  // d 16 after the block products, which may recompute D with the chosen pair)
  h->unit_epoch = 0;
  if (h->unit_stride > 0) {
    h->unit_epoch = ++h->epoch;
    HIP_TRY(qoc::launch_unitarity<T>(D, dp, h->d, N, h->unit_stride, h->unit_epoch, h->bits + 3, st));
  }
  qoc::SweepArgs<T> sw = sweep_args<T>(h, D, E, u_dev, out_dev);
  sw.Dh = Dh_small;
  sw.Eh = Dh_small ? (const T *)h->Eh : nullptr;
  if (h->Es && Dh_small) {  // sub-block products written by the block-product kernel
    sw.Es = (const T *)h->Es; sw.Ehs = (const T *)h->Ehs; sw.nu = (T *)h->nu;
  }
  // sweep kernels: one wavefront (S d_pad <= 64), one workgroup with a
  // prefetch ring (d_pad <= 64), or the generic streaming kernels; the
  // per-step source terms (forbidden states, time-optimal) run on the
  // generic per-block kernels only
  const bool ext = h->has_ext;
  const bool wave = !ext && qoc::wave_sweep_ok<T>(dp, S) && sw.Dh && sw.Eh;
  // padded d 16 with a gradient: the total runs as an extra workgroup of
  // the derivative kernel instead of a launch of its own, and (single-
  // wavefront block sweep) lambda_N, the fidelity and the penalty pass run
  // inside the backward block sweep's launch instead of the cost launch
  const bool first_order = h->grad_mode == QOC_GRAD_FIRST_ORDER;
  const bool total_in_adjoint = !ext && !first_order && want_grad && M > 0 && small_path &&
                                !small_big_adjoint<T>(h) && qoc::adjoint16_ok<T>(dp, kSmallPCap);
  sw.fuse_cost = (total_in_adjoint && wave && h->sweep_mode[2] != 3) ? 1 : 0;
  const bool small = !ext && !wave && qoc::small_sweep_ok<T>(dp, S);
  const bool wide_ok = !ext && !wave && !small && qoc::wide_sweep_ok<T>(dp, S);
  const SweepPick pick{ext, wave, small, wide_ok};
  auto sweep = [&](int which) { return launch_sweep<T>(h, pick, which, sw, st); };
  {
    PhaseTimer tm(h, QOC_PHASE_FWD_BLOCKS, st);
    HIP_TRY(sweep(0));
  }
  {
    PhaseTimer tm(h, QOC_PHASE_FWD_REPLAY, st);
    // with source terms the block penalty costates wait for them: replay only
    sw.replay_mode = ext ? 1 : 0;
    HIP_TRY(sweep(1));
    sw.replay_mode = 0;
  }
  // penalties beside fidelity / lambda_N in one launch, then the total cost
  // and drift (a side stream for the penalties measured slower here, its
  // events costing more than the overlap gained)
  if (!sw.fuse_cost) HIP_TRY(launch_cost_all<T>(h, sw, !total_in_adjoint, st));
  if (!want_grad) return QOC_OK;
  if (ext) {
    // the block-local penalty costates mu_b with the sources
    PhaseTimer tm(h, QOC_PHASE_FWD_REPLAY, st);
    sw.replay_mode = 2;
    HIP_TRY(qoc::launch_fwd_replay<T>(sw, st));
    sw.replay_mode = 0;
  }
  {
    PhaseTimer tm(h, QOC_PHASE_BWD_BLOCKS, st);
    HIP_TRY(sweep(2));
  }
  {
    PhaseTimer tm(h, QOC_PHASE_BWD_PAIRS, st);
    HIP_TRY(sweep(3));
  }
  if (M > 0 && first_order) {
    // the paper's first-order gradient from the pairs (lambda_{j+1}, psi_{j+1})
    PhaseTimer tm(h, QOC_PHASE_ADJOINT, st);
    qoc_status s = ensure_part(h);
    if (s) return s;
    qoc::AdjointArgs<T> ad{};
    ad.N = N; ad.dp = dp; ad.M = M; ad.S = S;
    ad.lam_buf = (const T *)h->lam_buf; ad.psi_buf = (const T *)h->psi_buf;
    ad.Hf = (const T *)h->Hf; ad.u = u_dev; ad.alpha_amp = h->a_amp; ad.alpha_var = h->a_var;
    ad.grad = grad_dev; ad.part = h->adj_part; ad.xbar = Qa;
    HIP_TRY(qoc::launch_grad_first<T>(ad, h->dt, st));
  } else if (M > 0) {
    PhaseTimer tm(h, QOC_PHASE_ADJOINT, st);
    qoc::AdjointArgs<T> ad{};
    // batched per-step derivative for padded d >= 64, and for d >= 32 on the
    // small-d path when a fixed (p, n) makes the pair known on the host
    const bool sbig = small_path && small_big_adjoint<T>(h);
    const bool big = sbig || (!small_path && qoc::adjoint_big_ok<T>(dp));
    if (sbig) {
      p = small_fixed_pn(h).first;
      n = small_fixed_pn(h).second;
      Rcap_used = small_fixed_rcap(h);
    }
    ad.N = N; ad.dp = dp; ad.M = M; ad.S = S; ad.p = small_path && !sbig ? kSmallPCap : p;
    ad.n = n; ad.Rcap = Rcap_used; ad.nblocks = h->adj_blocks;
    ad.pn = small_path ? h->pn_dev : nullptr; ad.sc = small_path ? h->sc_dev : nullptr;
    ad.X = X; ad.Dlev = (const T *)h->Dlev; ad.lam_buf = (const T *)h->lam_buf; ad.psi_buf = (const T *)h->psi_buf;
    ad.Hf = (const T *)h->Hf; ad.u = u_dev; ad.s_scale = std::ldexp(h->dt, -n);
    ad.alpha_amp = h->a_amp; ad.alpha_var = h->a_var; ad.scratch = (T *)h->adj;
    ad.scratch_elems = qoc::adjoint_scratch_elems<T>(dp, ad.p, ad.Rcap); ad.grad = grad_dev;
    ad.part = h->adj_part;
    ad.xbar = Qa;  // the Taylor work space is free once the sweeps are done
    ad.bf3 = (h->bf3_used & QOC_BF3_ADJOINT) ? 1 : 0;
    ad.bf3_launched = &h->bf3_adj_ran;
    ad.with_total = total_in_adjoint ? 1 : 0;
    ad.total = qoc::total_args(sw);
    if (sp_on && big) {
      ad.rptr = h->sp_rptr; ad.rcol = h->sp_rcol; ad.eptr = h->sp_eptr; ad.ek = h->sp_ek;
      ad.eval = (const T *)h->sp_eval; ad.nev = h->nev; ad.d = h->d;
    }
    if (!big && qoc::adjoint16_ok<T>(dp, ad.p))
      HIP_TRY(qoc::launch_adjoint16<T>(ad, st));
    else if (big)
      HIP_TRY(qoc::launch_adjoint_big<T>(ad, st));
    else
      HIP_TRY(qoc::launch_adjoint<T>(ad, st));
  }
  return QOC_OK;
}

// Memory-lean mode (App. A: the propagators formed again in the backward
// pass instead of stored): the horizon in time segments of Ns steps, whole
// checkpoint blocks each, and every per-step stack one segment long.  The
// forward pass forms each segment's exponentials and sweeps its states; the
// cost runs over the whole horizon; the backward pass visits the segments
// last to first, forms each segment's exponentials again (the same kernels
// on the same controls: the same values), sweeps its costates from the
// costate at the following segment's first step, writes the costate at its
// own first step, and contracts its derivative.  The states, checkpoints and
// costates stay whole (O(N S d), against the O(N d^2) stacks).
template <typename T>
qoc_status run_segmented(qoc_handle *h, const double *u_dev, double *out_dev, double *grad_dev,
                         hipStream_t st, bool want_grad) {
  const int dp = h->dp, N = h->N, M = h->M, S = h->S, L = h->L, Ns = h->Ns;
  const long set = 2L * S * dp;
  const bool sp_on = h->sp_built && (h->sp_mode == 1 || (h->sp_mode < 0 && h->sp_auto));
  h->sp_used = sp_on;
  const qoc::SparseU spu{h->sp_colptr, h->sp_rowidx, h->sp_vals};
  int p = 0, n = 0;
  qoc_status s = choose_pn_large<T>(h, u_dev, st, sp_on ? &spu : nullptr, &p, &n);
  if (s) return s;
  const int Rraw = (long)S << std::min(n, 30) > dp ? dp : (S << n);
  const int Rcap = std::min((Rraw + 15) & ~15, dp);
  if ((s = prepare_large<T>(h, p, n, want_grad, Rcap)) != QOC_OK) return s;
  h->unit_epoch = h->unit_stride > 0 ? ++h->epoch : 0;
  const bool ext = h->has_ext;
  const bool small = !ext && qoc::small_sweep_ok<T>(dp, S);
  const SweepPick pick{ext, false, small, !ext && !small && qoc::wide_sweep_ok<T>(dp, S)};
  const qoc::SweepArgs<T> all = sweep_args<T>(h, nullptr, nullptr, u_dev, out_dev);
  auto seg_len = [&](int g) { return (int)std::min<long>(Ns, N - (long)g * Ns); };
  // the segment's exponentials D_j and block products E_b, from its controls
  auto exps = [&](int g, const T **D, const T **E) -> hipError_t {
    const int Nloc = seg_len(g);
    hipError_t e = qoc::launch_copy_strided<double>(h->u_seg, Nloc, u_dev + (long)g * Ns, N,
                                                     Nloc, M, st);
    if (e != hipSuccess) return e;
    return exps_large<T>(h, h->u_seg, Nloc, p, n, st, D, E);
  };
  // sweep arguments of segment g: its steps and blocks, the global buffers
  // at its offsets (its first state: psi_0, or the previous segment's last)
  auto segment = [&](int g, const T *D, const T *E) {
    qoc::SweepArgs<T> sw = all;
    const long s0 = (long)g * Ns, b0 = s0 / L;
    sw.N = seg_len(g);
    sw.nb = (sw.N + L - 1) / L;
    sw.D = D;
    sw.E = E;
    sw.psi0 = g == 0 ? all.psi0 : all.psi_buf + s0 * set;
    sw.ckpt = all.ckpt + b0 * set;
    sw.psi_buf = all.psi_buf + s0 * set;
    sw.lam_ckpt = all.lam_ckpt + b0 * set;
    sw.mu = all.mu ? all.mu + b0 * set : nullptr;
    sw.lam_buf = all.lam_buf + s0 * set;
    sw.src = all.src ? all.src + s0 * set : nullptr;
    return sw;
  };
  const T *D = nullptr, *E = nullptr;
  for (int g = 0; g < h->nseg; ++g) {
    HIP_TRY(exps(g, &D, &E));
    if (h->unit_stride > 0)
      HIP_TRY(qoc::launch_unitarity<T>(D, dp, h->d, seg_len(g), h->unit_stride, h->unit_epoch,
                                       h->bits + 3, st));
    qoc::SweepArgs<T> sw = segment(g, D, E);
    {
      PhaseTimer tm(h, QOC_PHASE_FWD_BLOCKS, st);
      HIP_TRY(launch_sweep<T>(h, pick, 0, sw, st));
    }
    PhaseTimer tm(h, QOC_PHASE_FWD_REPLAY, st);
    sw.replay_mode = ext ? 1 : 0;  // with source terms the block costates wait for them
    HIP_TRY(launch_sweep<T>(h, pick, 1, sw, st));
  }
  HIP_TRY(launch_cost_all<T>(h, all, true, st));
  if (!want_grad) return QOC_OK;
  const bool first_order = h->grad_mode == QOC_GRAD_FIRST_ORDER;
  if (M > 0 && first_order && (s = ensure_part(h)) != QOC_OK) return s;
  for (int g = h->nseg - 1; g >= 0; --g) {
    HIP_TRY(exps(g, &D, &E));
    qoc::SweepArgs<T> sw = segment(g, D, E);
    if (ext) {
      PhaseTimer tm(h, QOC_PHASE_FWD_REPLAY, st);
      sw.replay_mode = 2;
      HIP_TRY(qoc::launch_fwd_replay<T>(sw, st));
      sw.replay_mode = 0;
    }
    {
      PhaseTimer tm(h, QOC_PHASE_BWD_BLOCKS, st);
      HIP_TRY(launch_sweep<T>(h, pick, 2, sw, st));
    }
    {
      PhaseTimer tm(h, QOC_PHASE_BWD_PAIRS, st);
      HIP_TRY(launch_sweep<T>(h, pick, 3, sw, st));
      if (g > 0) HIP_TRY(qoc::launch_seg_lambda<T>(sw, st));
    }
    if (M == 0) continue;
    PhaseTimer tm(h, QOC_PHASE_ADJOINT, st);
    qoc::AdjointArgs<T> ad{};
    ad.N = sw.N; ad.dp = dp; ad.M = M; ad.S = S; ad.p = p; ad.n = n; ad.Rcap = Rcap;
    ad.nblocks = h->adj_blocks;
    ad.X = (const T *)h->X; ad.Dlev = (const T *)h->Dlev;
    ad.lam_buf = sw.lam_buf; ad.psi_buf = sw.psi_buf;
    ad.Hf = (const T *)h->Hf; ad.u = u_dev; ad.s_scale = std::ldexp(h->dt, -n);
    ad.alpha_amp = h->a_amp; ad.alpha_var = h->a_var; ad.scratch = (T *)h->adj;
    ad.scratch_elems = qoc::adjoint_scratch_elems<T>(dp, p, Rcap);
    ad.grad = grad_dev; ad.part = h->adj_part;
    ad.xbar = (T *)h->Qa;  // the Taylor work space is free once the sweeps are done
    ad.bf3 = (h->bf3_used & QOC_BF3_ADJOINT) ? 1 : 0;
    ad.bf3_launched = &h->bf3_adj_ran;
    ad.total = qoc::total_args(all);
    ad.j0 = (long)g * Ns;
    ad.ldN = N;
    if (first_order) {
      HIP_TRY(qoc::launch_grad_first<T>(ad, h->dt, st));
      continue;
    }
    if (sp_on) {
      ad.rptr = h->sp_rptr; ad.rcol = h->sp_rcol; ad.eptr = h->sp_eptr; ad.ek = h->sp_ek;
      ad.eval = (const T *)h->sp_eval; ad.nev = h->nev; ad.d = h->d;
    }
    HIP_TRY(qoc::launch_adjoint_big<T>(ad, st));
  }
  return QOC_OK;
}

// Product inputs and cotangents of the action form's gradient for P
// products per step and column.
template <typename T> qoc_status ensure_action_work(qoc_handle *h, long P) {
  const size_t bytes = (size_t)h->N * h->S * P * 2 * h->dp * sizeof(T);
  if (h->ws_base) {
    qoc_status s = carve(h, &h->act_A, bytes);
    return s ? s : carve(h, &h->act_Y, bytes);
  }
  if (P <= h->act_P) return QOC_OK;
  const size_t old = (size_t)h->N * h->S * h->act_P * 2 * h->dp * sizeof(T);
  dfree(h, &h->act_A, old);
  dfree(h, &h->act_Y, old);
  h->act_P = 0;
  qoc_status s = dalloc(h, &h->act_A, bytes);
  if (s || (s = dalloc(h, &h->act_Y, bytes)) != QOC_OK) return s;
  h->act_P = P;
  return QOC_OK;
}

// State-mode action form (Sec. IV): no step propagator is formed.  The
// per-step values of H_j (parallel over steps), the forward chain of
// matrix-vector products (one workgroup per column; it keeps every
// product's input for the gradient), the cost over the whole horizon, the
// backward chain (the reverse pass of the same products: the costates, and
// every product's output cotangent), then the derivative for all controls
// at once, parallel over (step, column).  The first-order mode contracts
// (lambda_{j+1}, psi_{j+1}) instead.
template <typename T>
qoc_status run_action(qoc_handle *h, const double *u_dev, double *out_dev, double *grad_dev,
                      hipStream_t st, bool want_grad) {
  const int dp = h->dp, N = h->N, M = h->M, S = h->S;
  const long set = 2L * S * dp;
  const bool sp_on = h->sp_built && (h->sp_mode == 1 || (h->sp_mode < 0 && h->sp_auto));
  h->sp_used = sp_on;
  const qoc::SparseU spu{h->sp_colptr, h->sp_rowidx, h->sp_vals};
  int p = 0, n = 0;
  qoc_status s = choose_pn_large<T>(h, u_dev, st, sp_on ? &spu : nullptr, &p, &n, true);
  if (s) return s;
  if (p > 32 || n > 16 || ((long)p << n) > 4096)
    return fail(QOC_ERR_UNSUPPORTED, "the action form runs at most 4096 products per step (p 2^n "
                                     "with n <= 16); theta_max or the fixed pair asks for more");
  const long P = (long)p << n;
  h->last_p = p;
  h->last_n = n;
  h->bf3_used = 0;
  h->bf3_adj_ran = 0;
  h->bf3_fallback = 0;
  h->unit_epoch = 0;  // no step propagator to check
  const bool first_order = h->grad_mode == QOC_GRAD_FIRST_ORDER;
  const bool keep = want_grad && M > 0 && !first_order;
  if (keep && (s = ensure_action_work<T>(h, P)) != QOC_OK) return s;
  {
    PhaseTimer tm(h, QOC_PHASE_ASSEMBLE, st);
    const qoc::ActValArgs<T> va{h->act_hm, u_dev, M, N, h->actK, dp, (T *)h->act_hv};
    HIP_TRY(qoc::launch_act_values<T>(va, st));
  }
  qoc::ActionArgs<T> a{};
  a.N = N; a.dp = dp; a.S = S; a.K = h->actK; a.p = p; a.n = n; a.P = (int)P;
  a.s = (T)std::ldexp(h->dt, -n);
  for (int k = 1; k <= p; ++k) {
    a.coef[k] = (T)(std::ldexp(h->dt, -n) / k);
    a.inv[k] = (T)(1.0 / k);
  }
  a.ecol = h->act_ecol; a.hv = (const T *)h->act_hv; a.psi0 = (const T *)h->psi0;
  a.psi_buf = (T *)h->psi_buf; a.A = keep ? (T *)h->act_A : nullptr;
  a.lamN = (const T *)h->lam_ckpt + (long)h->nb * set; a.lam_buf = (T *)h->lam_buf;
  a.pw = (const T *)h->pw; a.src = h->has_ext ? (const T *)h->src : nullptr;
  a.Ybar = keep ? (T *)h->act_Y : nullptr;
  {
    PhaseTimer tm(h, QOC_PHASE_FWD_REPLAY, st);
    HIP_TRY(qoc::launch_act_chain<T>(0, a, st));
  }
  const qoc::SweepArgs<T> all = sweep_args<T>(h, nullptr, nullptr, u_dev, out_dev);
  HIP_TRY(launch_cost_all<T>(h, all, true, st));
  if (!want_grad) return QOC_OK;
  {
    PhaseTimer tm(h, QOC_PHASE_BWD_PAIRS, st);
    HIP_TRY(qoc::launch_act_chain<T>(1, a, st));
  }
  if (M == 0) return QOC_OK;
  PhaseTimer tm(h, QOC_PHASE_ADJOINT, st);
  qoc::ActGradArgs<T> g{};
  if (first_order) {
    // eq. (7): one product per step, (lambda_{j+1}, psi_{j+1}) in set layout
    g.A = (const T *)h->psi_buf + set; g.aj = set; g.as = dp; g.aq = 0; g.aplane = (long)S * dp;
    g.Y = (const T *)h->lam_buf; g.yj = set; g.ys = dp; g.yq = 0; g.yplane = (long)S * dp;
    g.P = 1;
  } else {
    const long vec = 2L * dp;
    g.A = (const T *)h->act_A; g.aj = S * P * vec; g.as = P * vec; g.aq = vec; g.aplane = dp;
    g.Y = (const T *)h->act_Y; g.yj = S * P * vec; g.ys = P * vec; g.yq = vec; g.yplane = dp;
    g.P = (int)P;
  }
  g.N = N; g.S = S; g.dp = dp; g.M = M;
  g.nent = h->act_nent; g.erow = h->act_erow; g.ecol = h->act_ecol2;
  g.cptr = h->act_cptr; g.cent = h->act_cent; g.cval = (const T *)h->act_cval;
  g.npairs = h->act_npairs; g.part = h->act_part;
  HIP_TRY(qoc::launch_act_grad<T>(g, st));
  const double two_s = 2.0 * (first_order ? h->dt : std::ldexp(h->dt, -n));
  HIP_TRY(qoc::launch_grad_finish(h->act_part, u_dev, grad_dev, two_s, h->a_amp, h->a_var, N, M,
                                  S, 0, N, st));
  return QOC_OK;
}

qoc_status run_any(qoc_handle *h, const double *u_dev, double *out_dev, double *grad_dev,
                   hipStream_t st, bool want_grad) {
  if (h->prop == QOC_PROP_ACTION) {
    if (h->prec == QOC_FP64) return run_action<double>(h, u_dev, out_dev, grad_dev, st, want_grad);
    return run_action<float>(h, u_dev, out_dev, grad_dev, st, want_grad);
  }
  if (h->nseg > 1) {
    if (h->prec == QOC_FP64)
      return run_segmented<double>(h, u_dev, out_dev, grad_dev, st, want_grad);
    return run_segmented<float>(h, u_dev, out_dev, grad_dev, st, want_grad);
  }
  if (h->prec == QOC_FP64) return run<double>(h, u_dev, out_dev, grad_dev, st, want_grad);
  return run<float>(h, u_dev, out_dev, grad_dev, st, want_grad);
}

// The unitarity word of the last call: (epoch << 32 | FP32 bits); -1 when
// the call ran no check.
double unitarity_of(const qoc_handle *h, unsigned long long word) {
  if (h->unit_epoch == 0 || (unsigned)(word >> 32) != h->unit_epoch) return -1.0;
  const unsigned bitsf = (unsigned)(word & 0xffffffffu);
  float f;
  std::memcpy(&f, &bitsf, sizeof(f));
  return (double)f;
}

qoc_status finish_diag(qoc_handle *h, hipStream_t st, int *flags) {
  unsigned long long b[4] = {0, 0, 0, 0};
  int pn[3] = {0, 0, 0};
  HIP_TRY(hipMemcpyAsync(b, h->bits, sizeof(b), hipMemcpyDeviceToHost, st));
  const bool small_path = h->prop != QOC_PROP_ACTION && on_small_path(h);
  const bool dev_pn = small_path || h->fixed_p >= 2;
  if (dev_pn) HIP_TRY(hipMemcpyAsync(pn, h->pn_dev, sizeof(pn), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (dev_pn) {
    h->last_p = pn[0];
    h->last_n = pn[1];
    if (pn[2] == 1) return fail(QOC_ERR_UNSUPPORTED, "the (p, n) required by theta_max exceeds the "
                                                     "preallocated capacity of the small-d path");
  }
  double th, dr;
  std::memcpy(&th, &b[0], 8);
  std::memcpy(&dr, &b[1], 8);
  h->last_theta = th;
  h->last_drift = dr;
  h->last_unitarity = unitarity_of(h, b[3]);
  h->last_flags = ((dr > h->drift_warn) ? QOC_WARN_DRIFT : 0) |
                  ((dev_pn && pn[2] == 2) ? QOC_WARN_TAYLOR : 0) |
                  (h->bf3_fallback ? QOC_WARN_PRECISION : 0) |
                  ((h->last_unitarity > h->drift_warn) ? QOC_WARN_UNITARITY : 0);
  if (flags) *flags = h->last_flags;
  if (h->prof) return drain_pending(h);
  return QOC_OK;
}

qoc_status check_u(qoc_handle *h, const double *u) {
  if (h->M > 0 && !u) return fail(QOC_ERR_ARG, "u is NULL");
  if (h->M > 0 && !all_finite(u, (size_t)h->M * h->N))
    return fail(QOC_ERR_NONFINITE, "u contains NaN or Inf");
  return QOC_OK;
}

}  // namespace

extern "C" {

const char *qoc_version(void) { return "libqoc 0.1 (gfx950)"; }

const char *qoc_last_error(void) { return g_err.c_str(); }

const char *qoc_status_string(qoc_status s) {
  switch (s) {
    case QOC_OK: return "ok";
    case QOC_ERR_ARG: return "invalid argument";
    case QOC_ERR_SHAPE: return "invalid shape";
    case QOC_ERR_NOT_HERMITIAN: return "Hamiltonian not Hermitian";
    case QOC_ERR_NONFINITE: return "non-finite input";
    case QOC_ERR_NOMEM: return "out of memory";
    case QOC_ERR_DEVICE: return "device error";
    case QOC_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

qoc_status qoc_taylor_select(double theta, double tol, int *p, int *n) {
  if (!p || !n) return fail(QOC_ERR_ARG, "null output pointer");
  if (!(theta >= 0.0) || !std::isfinite(theta) || !(tol > 0.0))
    return fail(QOC_ERR_ARG, "theta must be finite and >= 0, tol > 0");
  if (!taylor_select(theta, tol, p, n)) return fail(QOC_ERR_UNSUPPORTED, "no (p, n) meets tol");
  return QOC_OK;
}

qoc_status qoc_select_pair(double theta, double tol, int form, int *p, int *n) {
  if (!p || !n) return fail(QOC_ERR_ARG, "null output pointer");
  if (!(theta >= 0.0) || !std::isfinite(theta) || !(tol > 0.0))
    return fail(QOC_ERR_ARG, "theta must be finite and >= 0, tol > 0");
  bool ok;
  switch (form) {
    case QOC_FORM_HORNER: ok = taylor_select(theta, tol, p, n); break;
    case QOC_FORM_BATCHED: ok = taylor_select_ps(theta, tol, p, n); break;
    case QOC_FORM_ACTION: ok = action_select(theta, tol, p, n); break;
    default: return fail(QOC_ERR_ARG, "form must be QOC_FORM_HORNER, _BATCHED or _ACTION");
  }
  if (!ok) return fail(QOC_ERR_UNSUPPORTED, "no (p, n) meets tol");
  return QOC_OK;
}

qoc_status qoc_pair_for(const qoc_handle *h, double theta, int *p, int *n) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  if (h->prop != QOC_PROP_ACTION && !on_small_path(h) && h->bf3 && h->bf3_req < 0) {
    if (!p || !n) return fail(QOC_ERR_ARG, "null output pointer");
    if (!(theta >= 0.0) || !std::isfinite(theta))
      return fail(QOC_ERR_ARG, "theta must be finite and >= 0");
    if (!taylor_select_bf3(theta, h->tol, h->N, h->L, h->dp, p, n))
      return fail(QOC_ERR_UNSUPPORTED, "no (p, n) meets tol");
    return QOC_OK;
  }
  const int form = h->prop == QOC_PROP_ACTION ? QOC_FORM_ACTION
                   : on_small_path(h)         ? QOC_FORM_HORNER
                                              : QOC_FORM_BATCHED;
  return qoc_select_pair(theta, h->tol, form, p, n);
}

qoc_status qoc_set_taylor(qoc_handle *h, int p, int n) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  if (!(p == 0 || (p >= 2 && p <= 64 && n >= 0 && n <= 60)))
    return fail(QOC_ERR_ARG, "p must be 0 (automatic) or in [2, 64] with n in [0, 60]");
  const qoc_status s = check_fixed_pair(h, p, n);
  if (s) return s;
  h->fixed_p = p;
  h->fixed_n = p ? n : 0;
  return QOC_OK;
}

qoc_status qoc_set_gradient(qoc_handle *h, int mode) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  if (mode != QOC_GRAD_EXACT && mode != QOC_GRAD_FIRST_ORDER)
    return fail(QOC_ERR_ARG, "mode must be QOC_GRAD_EXACT or QOC_GRAD_FIRST_ORDER");
  h->grad_mode = mode;
  return QOC_OK;
}

qoc_status qoc_set_structure(qoc_handle *h, int mode) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  if (mode < -1 || mode > 1) return fail(QOC_ERR_ARG, "mode must be -1, 0 or 1");
  if (mode == 1 && !h->sp_built)
    return fail(QOC_ERR_UNSUPPORTED,
                "structured kernels need padded d >= 64 and a union of nonzero patterns of at "
                "most d^2 / 4 entries");
  h->sp_mode = mode;
  return QOC_OK;
}

qoc_status qoc_set_unitarity_check(qoc_handle *h, int stride) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  if (stride < 0) return fail(QOC_ERR_ARG, "stride must be >= 0");
  h->unit_stride = stride;
  return QOC_OK;
}

qoc_status qoc_set_bf16x3(qoc_handle *h, int classes) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  if (classes < -1 || classes > QOC_BF3_ALL)
    return fail(QOC_ERR_ARG, "classes must be -1 (automatic) or a mask of QOC_BF3_* bits");
  h->bf3_req = classes;
  return QOC_OK;
}

qoc_status qoc_set_sweep(qoc_handle *h, int which, int variant) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  if (which < -1 || which > 3 || variant < 0 || variant > 5)
    return fail(QOC_ERR_ARG, "which must be -1..3 and variant 0..5");
  for (int w = 0; w < 4; ++w)
    if (which == -1 || which == w) h->sweep_mode[w] = variant;
  return QOC_OK;
}

qoc_status qoc_create(const qoc_problem_desc *desc, qoc_handle **out) {
  if (!out) return fail(QOC_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(QOC_ERR_ARG, "desc is NULL");
  const qoc_problem_desc &D = *desc;
  if (D.d < 1 || D.d > 1024) return fail(QOC_ERR_SHAPE, "d must be in [1, 1024]");
  if (D.M < 0 || D.M > 64) return fail(QOC_ERR_SHAPE, "M must be in [0, 64]");
  if (D.N < 1 || D.N > (1 << 22)) return fail(QOC_ERR_SHAPE, "N must be in [1, 2^22]");
  if (D.S < 1 || D.S > D.d) return fail(QOC_ERR_SHAPE, "S must be in [1, d]");
  if (!(D.dt > 0.0) || !std::isfinite(D.dt)) return fail(QOC_ERR_ARG, "dt must be finite and > 0");
  if (!D.H0 || !D.psi0 || !D.psiT || (D.M > 0 && !D.Hk))
    return fail(QOC_ERR_ARG, "H0, Hk (M > 0), psi0 and psiT must be non-NULL");
  if (D.fid_mode != QOC_FID_COHERENT && D.fid_mode != QOC_FID_INCOHERENT)
    return fail(QOC_ERR_ARG, "fid_mode must be QOC_FID_COHERENT or QOC_FID_INCOHERENT");
  if (D.precision != QOC_FP32 && D.precision != QOC_FP64 && D.precision != QOC_BF16X3)
    return fail(QOC_ERR_ARG, "precision must be QOC_FP32, QOC_FP64 or QOC_BF16X3");
  if (D.checkpoint_every < 0) return fail(QOC_ERR_ARG, "checkpoint_every must be >= 0");
  if (!(D.pad_multiple == 0 || D.pad_multiple == 16 || D.pad_multiple == 32 ||
        D.pad_multiple == 64))
    return fail(QOC_ERR_ARG, "pad_multiple must be 0, 16, 32 or 64");
  if (D.segment_steps < 0) return fail(QOC_ERR_ARG, "segment_steps must be >= 0");
  if (!(D.propagation == QOC_PROP_MATRIX || D.propagation == QOC_PROP_ACTION))
    return fail(QOC_ERR_ARG, "propagation must be QOC_PROP_MATRIX or QOC_PROP_ACTION");
  if (D.propagation == QOC_PROP_ACTION && D.precision == QOC_BF16X3)
    return fail(QOC_ERR_UNSUPPORTED, "the action form runs no matrix products: FP32 or FP64");
  if (D.propagation == QOC_PROP_ACTION && D.segment_steps > 0)
    return fail(QOC_ERR_UNSUPPORTED, "the action form keeps no per-step matrix stacks to "
                                     "segment");
  if (!(D.taylor_tol >= 0.0) || !std::isfinite(D.taylor_tol))
    return fail(QOC_ERR_ARG, "taylor_tol must be finite and >= 0");
  if (!(D.taylor_p == 0 || (D.taylor_p >= 2 && D.taylor_p <= 64 && D.taylor_n >= 0 &&
                            D.taylor_n <= 60)))
    return fail(QOC_ERR_ARG, "taylor_p must be 0 (automatic) or in [2, 64] with taylor_n in [0, 60]");
  if (!(D.drift_warn >= 0.0)) return fail(QOC_ERR_ARG, "drift_warn must be >= 0");
  if (D.n_forbidden < 0 || D.n_forbidden > qoc::QOC_MAX_FORBIDDEN)
    return fail(QOC_ERR_SHAPE, "n_forbidden must be in [0, " +
                                   std::to_string(qoc::QOC_MAX_FORBIDDEN) + "]");
  if (D.n_forbidden > 0 && !D.forbidden)
    return fail(QOC_ERR_ARG, "forbidden must be non-NULL when n_forbidden > 0");
  if (!std::isfinite(D.alpha_time)) return fail(QOC_ERR_NONFINITE, "alpha_time must be finite");
  if (D.n_forbidden > 0 && !all_finite(D.forbidden, (size_t)D.n_forbidden * D.d * 2))
    return fail(QOC_ERR_NONFINITE, "forbidden states contain NaN or Inf");
  const double alphas[4] = {D.alpha_fid, D.alpha_amp, D.alpha_var, D.alpha_pen};
  if (!all_finite(alphas, 4)) return fail(QOC_ERR_NONFINITE, "cost weights must be finite");
  const size_t dd = (size_t)D.d * D.d * 2;
  if (!all_finite(D.H0, dd) || (D.M > 0 && !all_finite(D.Hk, dd * D.M)))
    return fail(QOC_ERR_NONFINITE, "Hamiltonian contains NaN or Inf");
  if (!all_finite(D.psi0, (size_t)D.S * D.d * 2) || !all_finite(D.psiT, (size_t)D.S * D.d * 2))
    return fail(QOC_ERR_NONFINITE, "states contain NaN or Inf");
  if (D.penalty_w) {
    if (!all_finite(D.penalty_w, D.d)) return fail(QOC_ERR_NONFINITE, "penalty_w has NaN or Inf");
    for (int m = 0; m < D.d; ++m)
      if (D.penalty_w[m] < 0.0) return fail(QOC_ERR_ARG, "penalty_w must be >= 0");
  }
  if (!hermitian(D.H0, D.d)) return fail(QOC_ERR_NOT_HERMITIAN, "H0 is not Hermitian");
  for (int k = 0; k < D.M; ++k)
    if (!hermitian(D.Hk + dd * k, D.d))
      return fail(QOC_ERR_NOT_HERMITIAN, "H_" + std::to_string(k + 1) + " is not Hermitian");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(QOC_ERR_DEVICE, "no HIP device available");
  }
  if (D.device < 0 || D.device >= ndev) return fail(QOC_ERR_ARG, "device ordinal out of range");

  qoc_handle *h = new (std::nothrow) qoc_handle();
  if (!h) return fail(QOC_ERR_NOMEM, "host allocation failed");
  h->d = D.d;
  {
    // padding of d: a multiple of 16 by default (16 / 32-wide tiles and the
    // small-d chains for d <= 48), or of 32 / 64 on request (64 x 64 tiles
    // for every product at the price of more zero padding; a tile-shape
    // choice that bench and Batch leave to the measuring tuner)
    const int pm = D.pad_multiple > 0 ? D.pad_multiple : 16;
    h->dp = (D.d + pm - 1) / pm * pm;
  }
  h->M = D.M;
  h->N = D.N;
  h->S = D.S;
  h->prop = D.propagation;
  h->dt = D.dt;
  h->prec = D.precision;
  h->bf3 = D.precision == QOC_BF16X3 ? 1 : 0;
  h->esize = (D.precision == QOC_FP64) ? 8 : 4;
  h->fid_mode = D.fid_mode;
  h->a_fid = D.alpha_fid;
  h->a_amp = D.alpha_amp;
  h->a_var = D.alpha_var;
  h->a_pen = D.alpha_pen;
  h->has_pen = D.penalty_w != nullptr;
  h->nf = (D.alpha_pen != 0.0) ? D.n_forbidden : 0;
  h->a_time = D.alpha_time;
  h->has_ext = h->nf > 0 || h->a_time != 0.0;
  h->tol = D.taylor_tol > 0 ? D.taylor_tol : (D.precision == QOC_FP64 ? 1e-15 : 1e-10);
  h->drift_warn = D.drift_warn > 0 ? D.drift_warn : 1e-4;
  h->fixed_p = D.taylor_p;
  h->fixed_n = D.taylor_n;
  if (check_fixed_pair(h, h->fixed_p, h->fixed_n) != QOC_OK) {
    const std::string msg = g_err;
    delete h;
    return fail(QOC_ERR_UNSUPPORTED, msg);
  }
  h->device = D.device;
  if (D.checkpoint_every > 0) {
    h->L = D.checkpoint_every;
  } else {
    const double r = std::sqrt((double)D.N);
    int l = 1;
    while (l * 2 <= r) l <<= 1;                   // l <= sqrt(N) < 2l
    h->L = (r / l > (2.0 * l) / r) ? 2 * l : l;   // nearer in ratio
  }
  h->nb = (int)((D.N + h->L - 1) / h->L);
  h->adj_blocks = std::min(D.N, 1024);
  // memory-lean mode: segments of whole checkpoint blocks
  h->Ns = D.N;
  if (D.segment_steps > 0) {
    const long len = ((long)D.segment_steps + h->L - 1) / h->L * h->L;
    if (len < D.N) {
      h->Ns = (int)len;
      h->nseg = (int)((D.N + len - 1) / len);
    }
  }
  if (h->nseg > 1 && (on_small_path(h) || h->dp < 64)) {
    delete h;
    return fail(QOC_ERR_UNSUPPORTED,
                "time segments apply to the batched path with its batched derivative (padded "
                "d >= 64); smaller problems keep their stacks whole");
  }
  DeviceGuard g(h->device);
  if (!g.ok) {
    delete h;
    return fail(QOC_ERR_DEVICE, "hipSetDevice failed");
  }
  if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
    delete h;
    return fail(QOC_ERR_DEVICE, "hipStreamCreate failed");
  }
  {
    // the device's static scratch address, once per device (for the
    // no-alloc entry point)
    void *sp = nullptr;
    const qoc_status ss = scratch_address(h->device, &sp);
    if (ss != QOC_OK) {
      const std::string msg = g_err;
      release(h);
      delete h;
      return fail(ss, msg);
    }
  }
  qoc_status s = (h->prec == QOC_FP64) ? alloc_all<double>(h, desc) : alloc_all<float>(h, desc);
  if (s != QOC_OK) {
    std::string msg = g_err;
    release(h);
    delete h;
    return fail(s, msg);
  }
  *out = h;
  return QOC_OK;
}

void qoc_destroy(qoc_handle *h) {
  if (!h) return;
  DeviceGuard g(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  release(h);
  delete h;
}

qoc_status qoc_forward(qoc_handle *h, const double *u, double *cost_fid, double *step_penalty,
                       double *psiN, int *flags_out) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  qoc_status s = check_u(h, u);
  if (s) return s;
  DeviceGuard g(h->device);
  if (!g.ok) return fail(QOC_ERR_DEVICE, "hipSetDevice failed");
  hipStream_t st = h->stream;
  const size_t mn = (size_t)h->M * h->N;
  if (mn) {
    std::memcpy(h->h_u, u, mn * sizeof(double));
    HIP_TRY(hipMemcpyAsync(h->u_dev, h->h_u, mn * sizeof(double), hipMemcpyHostToDevice, st));
  }
  if ((s = run_any(h, h->u_dev, h->out_dev, h->grad_dev, st, false)) != QOC_OK) return s;
  HIP_TRY(hipMemcpyAsync(h->h_out, h->out_dev, (2 + h->N) * sizeof(double),
                         hipMemcpyDeviceToHost, st));
  // final states: psi_buf[N] (padded planar, chain precision)
  const size_t set = 2 * (size_t)h->S * h->dp;
  std::vector<unsigned char> tmp(set * h->esize);
  HIP_TRY(hipMemcpyAsync(tmp.data(), (unsigned char *)h->psi_buf + (size_t)h->N * set * h->esize,
                         set * h->esize, hipMemcpyDeviceToHost, st));
  int flags = 0;
  if ((s = finish_diag(h, st, &flags)) != QOC_OK) return s;
  if (cost_fid) *cost_fid = h->h_out[1];
  if (step_penalty) std::memcpy(step_penalty, h->h_out + 2, h->N * sizeof(double));
  if (psiN) {
    for (int s2 = 0; s2 < h->S; ++s2)
      for (int m = 0; m < h->d; ++m) {
        const size_t ir = (size_t)s2 * h->dp + m, ii = (size_t)h->S * h->dp + ir;
        double vr, vi;
        if (h->esize == 8) {
          vr = ((double *)tmp.data())[ir];
          vi = ((double *)tmp.data())[ii];
        } else {
          vr = ((float *)tmp.data())[ir];
          vi = ((float *)tmp.data())[ii];
        }
        psiN[2 * ((size_t)s2 * h->d + m)] = vr;
        psiN[2 * ((size_t)s2 * h->d + m) + 1] = vi;
      }
  }
  if (flags_out) *flags_out = flags;
  return QOC_OK;
}

qoc_status qoc_cost_grad(qoc_handle *h, const double *u, double *cost, double *cost_fid,
                         double *step_penalty, double *grad, int *flags_out) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  if (h->M > 0 && !grad) return fail(QOC_ERR_ARG, "grad is NULL");
  qoc_status s = check_u(h, u);
  if (s) return s;
  DeviceGuard g(h->device);
  if (!g.ok) return fail(QOC_ERR_DEVICE, "hipSetDevice failed");
  hipStream_t st = h->stream;
  const size_t mn = (size_t)h->M * h->N;
  if (mn) {
    std::memcpy(h->h_u, u, mn * sizeof(double));
    HIP_TRY(hipMemcpyAsync(h->u_dev, h->h_u, mn * sizeof(double), hipMemcpyHostToDevice, st));
  }
  if ((s = run_any(h, h->u_dev, h->out_dev, h->grad_dev, st, true)) != QOC_OK) return s;
  HIP_TRY(hipMemcpyAsync(h->h_out, h->out_dev, (2 + h->N) * sizeof(double),
                         hipMemcpyDeviceToHost, st));
  if (mn)
    HIP_TRY(hipMemcpyAsync(h->h_grad, h->grad_dev, mn * sizeof(double), hipMemcpyDeviceToHost, st));
  int flags = 0;
  if ((s = finish_diag(h, st, &flags)) != QOC_OK) return s;
  if (cost) *cost = h->h_out[0];
  if (cost_fid) *cost_fid = h->h_out[1];
  if (step_penalty) std::memcpy(step_penalty, h->h_out + 2, h->N * sizeof(double));
  if (mn) std::memcpy(grad, h->h_grad, mn * sizeof(double));
  if (flags_out) *flags_out = flags;
  return QOC_OK;
}

qoc_status qoc_cost_grad_device(qoc_handle *h, const double *u_dev, double *out_dev,
                                double *grad_dev, void *stream) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  if ((h->M > 0 && (!u_dev || !grad_dev)) || !out_dev)
    return fail(QOC_ERR_ARG, "u_dev, out_dev and grad_dev must be non-NULL");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(QOC_ERR_DEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(st, &cs));
  h->capturing = cs != hipStreamCaptureStatusNone;
  if (h->capturing && h->prof)
    return fail(QOC_ERR_UNSUPPORTED,
                "per-phase profiling records events that a captured graph cannot hold: "
                "disable qoc_profile_enable before capturing");
  const qoc_status s = run_any(h, h->M > 0 ? u_dev : h->u_dev, out_dev, grad_dev, st, true);
  h->capturing = false;
  return s;
}

qoc_status qoc_cost_grad_device_noalloc(qoc_handle *h, const double *u_dev, double *out_dev,
                                        double *grad_dev, void *stream) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  if ((h->M > 0 && (!u_dev || !grad_dev)) || !out_dev)
    return fail(QOC_ERR_ARG, "u_dev, out_dev and grad_dev must be non-NULL");
  if (h->prof)
    return fail(QOC_ERR_UNSUPPORTED,
                "per-phase profiling creates events: disable qoc_profile_enable for the no-alloc "
                "entry point");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(QOC_ERR_DEVICE, "hipSetDevice failed");
  void *base = nullptr;
  qoc_status s = scratch_address(h->device, &base);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(st, &cs));
  h->capturing = cs != hipStreamCaptureStatusNone;
  // the per-call buffers come from the scratch for this call only; the
  // handle's own ones (if an allocating call made them) are kept aside
  void *own_lev = h->Dlev, *own_adj = h->adj;
  double *own_part = h->adj_part;
  h->ws_base = (unsigned char *)base;
  h->ws_cap = kScratchBytes;
  h->ws_used = 0;
  s = run_any(h, h->M > 0 ? u_dev : h->u_dev, out_dev, grad_dev, st, true);
  h->Dlev = own_lev;
  h->adj = own_adj;
  h->adj_part = own_part;
  h->ws_base = nullptr;
  h->ws_cap = h->ws_used = 0;
  h->capturing = false;
  return s;
}

qoc_status qoc_adam_step(long n, double *u_dev, const double *grad_dev, double *m_dev,
                         double *v_dev, double *t_dev, double lr, double beta1, double beta2,
                         double eps, void *stream) {
  if (n < 0 || (n > 0 && (!u_dev || !grad_dev || !m_dev || !v_dev)) || !t_dev)
    return fail(QOC_ERR_ARG, "n must be >= 0 and the device arrays non-NULL");
  if (!(lr >= 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0) || !std::isfinite(lr) || !std::isfinite(eps))
    return fail(QOC_ERR_ARG, "need lr >= 0, 0 <= beta1, beta2 < 1 and eps > 0");
  HIP_TRY(qoc::launch_adam(n, u_dev, grad_dev, m_dev, v_dev, t_dev, lr, beta1, beta2, eps,
                           (hipStream_t)stream));
  return QOC_OK;
}

qoc_status qoc_cost_grad_batched(int B, qoc_handle *const *hs, const double *const *u_dev,
                                 double *const *out_dev, double *const *grad_dev, void *stream) {
  if (B < 0 || (B > 0 && (!hs || !u_dev || !out_dev || !grad_dev)))
    return fail(QOC_ERR_ARG, "invalid batch arrays");
  for (int b = 0; b < B; ++b) {
    if (!hs[b]) return fail(QOC_ERR_ARG, "null handle in batch");
    if (hs[b]->device != hs[0]->device) return fail(QOC_ERR_ARG, "batch spans several devices");
  }
  for (int b = 0; b < B; ++b) {
    qoc_status s = qoc_cost_grad_device(hs[b], u_dev[b], out_dev[b], grad_dev[b], stream);
    if (s) return s;
  }
  return QOC_OK;
}

qoc_status qoc_get_info(const qoc_handle *hc, qoc_info *info) {
  if (!hc || !info) return fail(QOC_ERR_ARG, "null argument");
  qoc_handle *h = const_cast<qoc_handle *>(hc);
  {
    // refresh from the device (the device-pointer entry points do not read
    // their diagnostics back)
    DeviceGuard g(h->device);
    if (!g.ok) return fail(QOC_ERR_DEVICE, "hipSetDevice failed");
    HIP_TRY(hipDeviceSynchronize());
    unsigned long long b[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpy(b, h->bits, sizeof(b), hipMemcpyDeviceToHost));
    std::memcpy(&h->last_theta, &b[0], 8);
    std::memcpy(&h->last_drift, &b[1], 8);
    h->last_unitarity = unitarity_of(h, b[3]);
    int pn[3] = {0, 0, 0};
    HIP_TRY(hipMemcpy(pn, h->pn_dev, sizeof(pn), hipMemcpyDeviceToHost));
    if (pn[0] >= 2 && h->fixed_p == 0 && h->last_p == 0) {
      h->last_p = pn[0];
      h->last_n = pn[1];
    }
    const bool small_path = h->prop != QOC_PROP_ACTION && on_small_path(h);
    if (small_path && pn[0] >= 2) {
      h->last_p = pn[0];
      h->last_n = pn[1];
    }
    h->last_flags = ((h->last_drift > h->drift_warn) ? QOC_WARN_DRIFT : 0) |
                    (((small_path || h->fixed_p >= 2) && pn[2] == 2) ? QOC_WARN_TAYLOR : 0) |
                    (((small_path || h->fixed_p >= 2) && pn[2] == 1) ? QOC_WARN_NO_PAIR : 0) |
                    (h->bf3_fallback ? QOC_WARN_PRECISION : 0) |
                    ((h->last_unitarity > h->drift_warn) ? QOC_WARN_UNITARITY : 0);
  }
  info->flags = h->last_flags;
  info->p = h->last_p;
  info->n = h->last_n;
  info->theta_max = h->last_theta;
  info->norm_drift = h->last_drift;
  info->block_len = h->L;
  info->n_blocks = h->nb;
  info->d_pad = h->dp;
  info->device_bytes = h->bytes;
  // classes that ran split products: the derivative's only where a split
  // product was launched (narrow thin products and the sparse contraction
  // have FP32 kernels only)
  info->bf16x3_classes = h->bf3_adj_ran ? h->bf3_used : (h->bf3_used & ~QOC_BF3_ADJOINT);
  info->unitarity_drift = h->last_unitarity;
  info->structured = h->sp_used ? 1 : 0;
  info->segments = h->nseg;
  info->propagation = h->prop;
  return QOC_OK;
}

qoc_status qoc_profile_enable(qoc_handle *h, int on) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  h->prof = on != 0;
  return QOC_OK;
}

qoc_status qoc_profile_read(qoc_handle *h, double *ms, long long *calls, int reset) {
  if (!h) return fail(QOC_ERR_ARG, "handle is NULL");
  DeviceGuard g(h->device);
  qoc_status s = drain_pending(h);
  if (s) return s;
  for (int i = 0; i < QOC_PHASE_COUNT; ++i) {
    if (ms) ms[i] = h->prof_ms[i];
    if (calls) calls[i] = h->prof_calls[i];
    if (reset) {
      h->prof_ms[i] = 0;
      h->prof_calls[i] = 0;
    }
  }
  return QOC_OK;
}

}  // extern "C"
