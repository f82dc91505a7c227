// Latency-oriented sweeps for small Hilbert spaces (padded d <= 64).
//
// Same blocked two-level scan as kernels_sweep.hip (F2 / F3 / B2 / B3), but
// each workgroup carries all S columns at once and the step matrices are
// staged through LDS from a register ring that is PD steps ahead: the global
// loads for step j + PD are issued before the product of step j, so HBM
// latency is off the sequential critical path.  For the costate sweeps the
// matrix is stored transposed in LDS, so both directions read rows.
//
// Per step: y = x + op(D) x (+ add) for the S columns, op = identity or ^H.
// Thread t handles output o = t / KC (o = s * DP + m) and the k-chunk
// t % KC of length DP / KC; partial sums are combined across the KC
// consecutive lanes with cross-lane shuffles.
#include "qoc_device.h"
#include "qoc_kernels.h"

namespace qoc {

template <typename T, int DP> struct SmallPlan {
  static constexpr int PF = (2 * DP * DP + 255) / 256;  // step-matrix elements per thread
  static constexpr int PA = 4;                          // state-set elements per thread
  static constexpr int PD = DP <= 16 ? 8 : (DP <= 32 ? 4 : 2);  // prefetch depth (steps)
  int S, OUT, KC, CH;
  __device__ void init(int S_) {
    S = S_;
    OUT = DP * S;
    int kc = 1;
    if (OUT <= 256) {
      while (kc * 2 * OUT <= 256 && kc * 2 <= DP) kc *= 2;
    }
    KC = kc;
    CH = DP / KC;
  }
};

// Ring loads and stores are branch-free so that the compiler's wait counts
// stay exact (a conditional load makes it wait for every load in flight).
// Every load is in bounds because the device buffers carry kRingSlack
// elements of padding and ring indices are clamped.
template <typename T, int N>
__device__ __forceinline__ void pf_load(const T *__restrict__ g, T (&reg)[N]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < N; ++q) reg[q] = g[q * 256 + t];
}

template <typename T, int DP, int N, bool TRANS>
__device__ __forceinline__ void pf_store(T *dst, const T (&reg)[N]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const int e = q * 256 + t;
    if (TRANS) {
      const int pl = e / (DP * DP), rem = e - pl * DP * DP;
      const int r = rem / DP, c = rem - r * DP;
      dst[pl * DP * DP + c * DP + r] = reg[q];
    } else {
      dst[e] = reg[q];
    }
  }
}

// y = x + op(D) x (+ wl o add), op(D)[m][k] = Ds[m][k] (CONJ = false) or
// conj(Ds[m][k]) with Ds holding D^T (CONJ = true); add is a state set in
// LDS, wl per-level weights in LDS (null: unit weights).
template <typename T, int DP, bool CONJ>
__device__ __forceinline__ void sm_apply(const SmallPlan<T, DP> &P, const T *Ds, const T *x,
                                         T *y, const T *add, const T *wl) {
  const int t = threadIdx.x;
  const int SD = P.S * DP;
  const T *Dr = Ds, *Di = Ds + DP * DP;
  for (int base = 0; base < P.OUT * P.KC; base += 256) {
    const int tt = base + t;
    const int o = tt / P.KC, kc = tt - o * P.KC;
    T sr = 0, si = 0;
    int s = 0, m = 0;
    if (o < P.OUT) {
      s = o / DP;
      m = o - s * DP;
      const T *dr = Dr + m * DP + kc * P.CH, *di = Di + m * DP + kc * P.CH;
      const T *xr = x + s * DP + kc * P.CH, *xi = x + SD + s * DP + kc * P.CH;
      for (int i = 0; i < P.CH; ++i) {
        const T a = dr[i], b = CONJ ? -di[i] : di[i];
        sr += a * xr[i] - b * xi[i];
        si += a * xi[i] + b * xr[i];
      }
    }
    for (int off = 1; off < P.KC; off <<= 1) {
      sr += __shfl_xor(sr, off, 64);
      si += __shfl_xor(si, off, 64);
    }
    if (o < P.OUT && kc == 0) {
      T vr = x[s * DP + m] + sr, vi = x[SD + s * DP + m] + si;
      if (add) {
        const T wgt = wl ? wl[m] : (T)1;
        vr += wgt * add[s * DP + m];
        vi += wgt * add[SD + s * DP + m];
      }
      y[s * DP + m] = vr;
      y[SD + s * DP + m] = vi;
    }
  }
}

// These kernels always run 256 threads per workgroup.  The constant (and not
// blockDim.x, which is read from the dispatch packet with a global load)
// keeps the prefetch ring's loads in flight.
constexpr int kThreads = 256;

template <typename T>
__device__ __forceinline__ void copy_set(T *dst, const T *src, int n) {
  for (int e = threadIdx.x; e < n; e += kThreads) dst[e] = src[e];
}

// Software pipeline over `count` steps: the step matrix (and, with AUX, one
// state set) of step i + PD is loaded into registers while step i runs, so
// global-memory latency stays off the sequential path.  step(i) must end
// with a barrier after its last LDS read of Ds / As.  The barriers inside
// the pipeline order LDS only (lds_barrier), so loads in flight stay in
// flight; the global stores a step makes are read only by later kernels.
template <typename T, int DP, bool TRANS, bool AUX, class DPtr, class APtr, class Step>
__device__ __forceinline__ void sm_pipeline(int count, DPtr dptr, APtr aptr, T *Ds, T *As,
                                            Step step) {
  typedef SmallPlan<T, DP> P;
  constexpr int PD = P::PD, PF = P::PF, PA = AUX ? P::PA : 1;
  static_assert(PF * 256 == 2 * DP * DP, "step matrix must fill the ring slot exactly");
  if (count <= 0) return;
  T rd[PD][PF];
  T ra[PD][PA];
#pragma unroll
  for (int q = 0; q < PD; ++q) {
    const int i = q < count ? q : count - 1;
    pf_load<T, PF>(dptr(i), rd[q]);
    if (AUX) pf_load<T, PA>(aptr(i), ra[q]);
  }
  for (int i0 = 0; i0 < count; i0 += PD) {
#pragma unroll
    for (int q = 0; q < PD; ++q) {
      const int i = i0 + q;
      if (i < count) {
        pf_store<T, DP, PF, TRANS>(Ds, rd[q]);
        if (AUX) pf_store<T, DP, PA, false>(As, ra[q]);
        lds_barrier();
        const int nx = (i + PD < count) ? i + PD : count - 1;
        pf_load<T, PF>(dptr(nx), rd[q]);
        if (AUX) pf_load<T, PA>(aptr(nx), ra[q]);
        step(i);
      }
    }
  }
}

// LDS: Ds (2 DP^2) | x, y (2 S DP each) | As (4 * 256, one full ring slot)
// | wl (DP)
#define SM_SETUP                                                   \
  extern __shared__ unsigned char shraw[];                         \
  T *Ds = (T *)shraw;                                              \
  const int set = 2 * a.S * DP;                                    \
  T *x = Ds + 2 * DP * DP, *y = x + set, *As = y + set;            \
  T *wl = As + 4 * 256;                                            \
  SmallPlan<T, DP> P;                                              \
  P.init(a.S);                                                     \
  const long mat = 2L * DP * DP;                                   \
  (void)mat;

// ------------------------------------------------------------------ F2
template <typename T, int DP> __global__ __launch_bounds__(256) void k_smF2(SweepArgs<T> a) {
  SM_SETUP
  copy_set(x, a.psi0, set);
  copy_set(a.ckpt, a.psi0, set);
  __syncthreads();
  auto dptr = [&](int i) -> const T * { return a.E + i * mat; };
  auto nop = [&](int) -> const T * { return nullptr; };
  sm_pipeline<T, DP, false, false>(a.nb, dptr, nop, Ds, As, [&](int b) {
    sm_apply<T, DP, false>(P, Ds, x, y, nullptr, nullptr);
    lds_barrier();
    copy_set(a.ckpt + (long)(b + 1) * set, y, set);
    T *tmp = x; x = y; y = tmp;
  });
}

// ------------------------------------------------------------------ F3
template <typename T, int DP> __global__ __launch_bounds__(256) void k_smF3(SweepArgs<T> a) {
  SM_SETUP
  const int b = blockIdx.x;
  const int start = b * a.L, end = min(a.N, start + a.L), cnt = end - start;
  copy_set(x, a.ckpt + (long)b * set, set);
  copy_set(a.psi_buf + (long)start * set, a.ckpt + (long)b * set, set);
  if (a.pw) copy_set(wl, a.pw, DP);
  __syncthreads();
  auto fptr = [&](int i) -> const T * { return a.D + (start + i) * mat; };
  auto nop = [&](int) -> const T * { return nullptr; };
  sm_pipeline<T, DP, false, false>(cnt, fptr, nop, Ds, As, [&](int i) {
    sm_apply<T, DP, false>(P, Ds, x, y, nullptr, nullptr);
    lds_barrier();
    const int j = start + i;
    if (j + 1 < end || j + 1 == a.N) copy_set(a.psi_buf + (long)(j + 1) * set, y, set);
    T *tmp = x; x = y; y = tmp;
  });
  if (!a.pw) return;  // block-uniform
  // block-local penalty costate from zero at the block end, over the states
  // this workgroup just wrote:  mu <- mu + D_j^H mu + pw o psi_j  (j >= 1)
  __syncthreads();  // last state copy-out done before x is reused
  for (int e = threadIdx.x; e < set; e += kThreads) x[e] = (T)0;
  __syncthreads();
  auto bptr = [&](int i) -> const T * { return a.D + (end - 1 - i) * mat; };
  auto pptr = [&](int i) -> const T * { return a.psi_buf + (long)(end - 1 - i) * set; };
  sm_pipeline<T, DP, true, true>(cnt, bptr, pptr, Ds, As, [&](int i) {
    const int j = end - 1 - i;
    sm_apply<T, DP, true>(P, Ds, x, y, j >= 1 ? As : nullptr, wl);
    lds_barrier();
    T *tmp = x; x = y; y = tmp;
  });
  copy_set(a.mu + (long)b * set, x, set);
}

// ------------------------------------------------------------------ B2
template <typename T, int DP> __global__ __launch_bounds__(256) void k_smB2(SweepArgs<T> a) {
  SM_SETUP
  copy_set(x, a.lam_ckpt + (long)a.nb * set, set);
  __syncthreads();
  // steps b = nb-1 .. 1:  lambda_{bL} = lambda + E_b^H lambda + mu_b
  auto dptr = [&](int i) -> const T * { return a.E + (a.nb - 1 - i) * mat; };
  auto mptr = [&](int i) -> const T * {
    return a.mu ? a.mu + (long)(a.nb - 1 - i) * set : a.lam_ckpt;  // dummy when no penalty
  };
  sm_pipeline<T, DP, true, true>(a.nb - 1, dptr, mptr, Ds, As, [&](int i) {
    sm_apply<T, DP, true>(P, Ds, x, y, a.mu ? As : nullptr, nullptr);
    lds_barrier();
    copy_set(a.lam_ckpt + (long)(a.nb - 1 - i) * set, y, set);
    T *tmp = x; x = y; y = tmp;
  });
}

// ------------------------------------------------------------------ B3
template <typename T, int DP> __global__ __launch_bounds__(256) void k_smB3(SweepArgs<T> a) {
  SM_SETUP
  const int b = blockIdx.x;
  const int start = b * a.L, end = min(a.N, start + a.L);
  copy_set(x, a.lam_ckpt + (long)(b + 1) * set, set);
  if (a.pw) copy_set(wl, a.pw, DP);
  __syncthreads();
  // steps j = end-1 .. start+1: emit lambda_{j+1}, then
  // lambda_j = lambda_{j+1} + D_j^H lambda_{j+1} + pw o psi_j
  auto dptr = [&](int i) -> const T * { return a.D + (end - 1 - i) * mat; };
  auto pptr = [&](int i) -> const T * { return a.psi_buf + (long)(end - 1 - i) * set; };
  sm_pipeline<T, DP, true, true>(end - 1 - start, dptr, pptr, Ds, As, [&](int i) {
    const int j = end - 1 - i;
    copy_set(a.lam_buf + (long)j * set, x, set);
    sm_apply<T, DP, true>(P, Ds, x, y, (a.pw && j >= 1) ? As : nullptr, wl);
    lds_barrier();
    T *tmp = x; x = y; y = tmp;
  });
  copy_set(a.lam_buf + (long)start * set, x, set);
}

template <typename T, int DP> size_t sm_lds_bytes(int S) {
  return sizeof(T) * (2 * DP * DP + 4 * (size_t)S * DP + 4 * 256 + DP);
}

template <typename T, int DP> hipError_t sm_launch(int which, const SweepArgs<T> &a, hipStream_t st) {
  const size_t shm = sm_lds_bytes<T, DP>(a.S);
  switch (which) {
    case 0: hipLaunchKernelGGL((k_smF2<T, DP>), dim3(1), dim3(256), shm, st, a); break;
    case 1: hipLaunchKernelGGL((k_smF3<T, DP>), dim3(a.nb), dim3(256), shm, st, a); break;
    case 2: hipLaunchKernelGGL((k_smB2<T, DP>), dim3(1), dim3(256), shm, st, a); break;
    default: hipLaunchKernelGGL((k_smB3<T, DP>), dim3(a.nb), dim3(256), shm, st, a); break;
  }
  return hipGetLastError();
}

template <typename T> bool small_sweep_ok(int dp, int S) {
  if (dp > 64 || dp % 16) return false;
  if (2 * S * dp > 4 * 256) return false;  // one state set per 4 elements per thread
  const size_t bytes = sizeof(T) * (2 * (size_t)dp * dp + 4 * (size_t)S * dp + 4 * 256 + dp);
  return bytes <= 60 * 1024;
}

template <typename T> hipError_t launch_small_sweep(int which, const SweepArgs<T> &a, hipStream_t st) {
  switch (a.dp) {
    case 16: return sm_launch<T, 16>(which, a, st);
    case 32: return sm_launch<T, 32>(which, a, st);
    case 48: return sm_launch<T, 48>(which, a, st);
    case 64: return sm_launch<T, 64>(which, a, st);
  }
  return hipErrorInvalidValue;
}

template bool small_sweep_ok<float>(int, int);
template bool small_sweep_ok<double>(int, int);
template hipError_t launch_small_sweep<float>(int, const SweepArgs<float> &, hipStream_t);
template hipError_t launch_small_sweep<double>(int, const SweepArgs<double> &, hipStream_t);

}  // namespace qoc
