// Single-wavefront sweeps for the smallest problems (S * d_pad <= 64).
//
// The blocked two-level scan of kernels_sweep.hip (F2 / F3 / B2 / B3) with
// the whole state set in one wavefront: lane l owns output (s, m) with
// l mod (S d_pad) = s d_pad + m.  Each lane keeps its row of op(D_j) for the
// next RD steps in registers (a prefetch ring), reads its column of the
// state from LDS (a broadcast within the lanes of one column) and writes
// its new entry back; there is no workgroup barrier on the sequential path.
// Lanes beyond S d_pad duplicate an owner lane exactly, so every store is
// unconditional and the compiler's wait counts stay exact.
#include <type_traits>

#include "qoc_device.h"
#include "qoc_kernels.h"

namespace qoc {

#ifndef QOC_WAVE_RD16
#define QOC_WAVE_RD16 4
#endif
#ifndef QOC_WAVE_RD32
#define QOC_WAVE_RD32 2
#endif
template <int DP> struct WaveRing {
  static constexpr int RD = DP <= 16 ? QOC_WAVE_RD16 : QOC_WAVE_RD32;  // steps prefetched ahead
};

__device__ __forceinline__ void wave_lds_fence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// Row m of op(D): D itself (ADJ = false) or D^H (ADJ = true).
template <typename T, int DP, bool ADJ>
__device__ __forceinline__ void w_load_row(const T *__restrict__ D, int m, T (&r)[2 * DP]) {
  if (!ADJ) {
#pragma unroll
    for (int k = 0; k < DP; ++k) {
      r[k] = D[m * DP + k];
      r[DP + k] = D[DP * DP + m * DP + k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < DP; ++k) {
      r[k] = D[k * DP + m];
      r[DP + k] = -D[DP * DP + k * DP + m];
    }
  }
}

struct WLane {
  int s, m, SD, S;
};

// y = x + op(D) x (+ w o aux) for this lane's output; x lives in LDS xs.
// The dot product runs as WA independent partial sums (a short dependency
// chain on the sequential path), the state column read in 16-byte pieces.
template <typename T, int DP>
__device__ __forceinline__ void w_apply(const WLane &L, const T (&r)[2 * DP], const T *xs,
                                        T aux_r, T aux_i, T wgt, T &yr, T &yi) {
  constexpr int WA = 4;
  typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type V;
  constexpr int VN = 16 / sizeof(T);
  const T *xr = xs + L.s * DP, *xi = xs + L.SD + L.s * DP;
  T pr[WA], pi[WA];
#pragma unroll
  for (int q = 0; q < WA; ++q) {
    pr[q] = 0;
    pi[q] = 0;
  }
#pragma unroll
  for (int k0 = 0; k0 < DP; k0 += VN) {
    const V xv = *reinterpret_cast<const V *>(xr + k0);
    const V yv = *reinterpret_cast<const V *>(xi + k0);
    const T *xa = reinterpret_cast<const T *>(&xv), *ya = reinterpret_cast<const T *>(&yv);
#pragma unroll
    for (int e = 0; e < VN; ++e) {
      const int k = k0 + e, q = k % WA;
      pr[q] += r[k] * xa[e] - r[DP + k] * ya[e];
      pi[q] += r[k] * ya[e] + r[DP + k] * xa[e];
    }
  }
  T ar = 0, ai = 0;
#pragma unroll
  for (int q = 0; q < WA; ++q) {
    ar += pr[q];
    ai += pi[q];
  }
  // select, not multiply: an unused auxiliary operand is never touched
  yr = xr[L.m] + ar + (wgt != (T)0 ? wgt * aux_r : (T)0);
  yi = xi[L.m] + ai + (wgt != (T)0 ? wgt * aux_i : (T)0);
}

// Ring-pipelined loop over `count` steps.  step(i, row, aux_r, aux_i).
template <typename T, int DP, bool ADJ, class DPtr, class APtr, class Step>
__device__ __forceinline__ void w_pipeline(const WLane &L, int count, DPtr dptr, APtr aptr,
                                           Step step) {
  constexpr int RD = WaveRing<DP>::RD;
  if (count <= 0) return;
  T r[RD][2 * DP];
  T ar[RD], ai[RD];
  const int o = L.s * DP + L.m;
#pragma unroll
  for (int q = 0; q < RD; ++q) {
    const int i = q < count ? q : count - 1;
    w_load_row<T, DP, ADJ>(dptr(i), L.m, r[q]);
    const T *a = aptr(i);
    ar[q] = a[o];
    ai[q] = a[L.SD + o];
  }
  for (int i0 = 0; i0 < count; i0 += RD) {
#pragma unroll
    for (int q = 0; q < RD; ++q) {
      const int i = i0 + q;
      if (i < count) {
        step(i, r[q], ar[q], ai[q]);
        const int nx = (i + RD < count) ? i + RD : count - 1;
        w_load_row<T, DP, ADJ>(dptr(nx), L.m, r[q]);
        const T *a = aptr(nx);
        ar[q] = a[o];
        ai[q] = a[L.SD + o];
      }
    }
  }
}

#define W_SETUP                                                        \
  __shared__ __align__(16) T xs[2][128];                               \
  WLane L;                                                             \
  L.S = a.S;                                                           \
  L.SD = a.S * DP;                                                     \
  {                                                                    \
    const int l = threadIdx.x % L.SD;                                  \
    L.s = l / DP;                                                      \
    L.m = l - L.s * DP;                                                \
  }                                                                    \
  const int o = L.s * DP + L.m;                                        \
  const long set = 2L * a.S * DP, mat = 2L * DP * DP;                  \
  int cur = 0;                                                         \
  (void)mat;

template <typename T>
__device__ __forceinline__ void w_put(T *xs, const WLane &L, int o, T vr, T vi) {
  xs[o] = vr;
  xs[L.SD + o] = vi;
}

// ------------------------------------------------------------------ F2
template <typename T, int DP> __global__ __launch_bounds__(64) void k_wF2(SweepArgs<T> a) {
  W_SETUP
  T vr = a.psi0[o], vi = a.psi0[L.SD + o];
  w_put(xs[0], L, o, vr, vi);
  a.ckpt[o] = vr;
  a.ckpt[L.SD + o] = vi;
  wave_lds_fence();
  auto dptr = [&](int i) -> const T * { return a.E + i * mat; };
  auto aptr = [&](int) -> const T * { return a.psi0; };  // unused
  w_pipeline<T, DP, false>(L, a.nb, dptr, aptr, [&](int b, const T (&r)[2 * DP], T, T) {
    T yr, yi;
    w_apply<T, DP>(L, r, xs[cur], (T)0, (T)0, (T)0, yr, yi);
    w_put(xs[cur ^ 1], L, o, yr, yi);
    T *c = a.ckpt + (long)(b + 1) * set;
    c[o] = yr;
    c[L.SD + o] = yi;
    cur ^= 1;
    wave_lds_fence();
  });
}

// ------------------------------------------------------------------ F3
template <typename T, int DP> __global__ __launch_bounds__(64) void k_wF3(SweepArgs<T> a) {
  W_SETUP
  const int b = blockIdx.x;
  const int start = b * a.L, end = min(a.N, start + a.L), cnt = end - start;
  const T *ck = a.ckpt + (long)b * set;
  T vr = ck[o], vi = ck[L.SD + o];
  w_put(xs[0], L, o, vr, vi);
  a.psi_buf[(long)start * set + o] = vr;
  a.psi_buf[(long)start * set + L.SD + o] = vi;
  wave_lds_fence();
  auto fptr = [&](int i) -> const T * { return a.D + (start + i) * mat; };
  auto dummy = [&](int) -> const T * { return ck; };
  w_pipeline<T, DP, false>(L, cnt, fptr, dummy, [&](int i, const T (&r)[2 * DP], T, T) {
    T yr, yi;
    w_apply<T, DP>(L, r, xs[cur], (T)0, (T)0, (T)0, yr, yi);
    w_put(xs[cur ^ 1], L, o, yr, yi);
    const int j = start + i;
    if (j + 1 < end || j + 1 == a.N) {  // wave-uniform
      a.psi_buf[(long)(j + 1) * set + o] = yr;
      a.psi_buf[(long)(j + 1) * set + L.SD + o] = yi;
    }
    cur ^= 1;
    wave_lds_fence();
  });
  if (!a.pw) return;  // uniform
  // block-local penalty costate from zero at the block end:
  // mu <- mu + D_j^H mu + pw o psi_j (j >= 1), over the states written above
  __threadfence_block();
  const T wgt = a.pw[L.m];
  w_put(xs[cur], L, o, (T)0, (T)0);
  wave_lds_fence();
  auto bptr = [&](int i) -> const T * { return a.D + (end - 1 - i) * mat; };
  auto pptr = [&](int i) -> const T * { return a.psi_buf + (long)(end - 1 - i) * set; };
  w_pipeline<T, DP, true>(L, cnt, bptr, pptr, [&](int i, const T (&r)[2 * DP], T pr, T pi) {
    const int j = end - 1 - i;
    T yr, yi;
    w_apply<T, DP>(L, r, xs[cur], pr, pi, j >= 1 ? wgt : (T)0, yr, yi);
    w_put(xs[cur ^ 1], L, o, yr, yi);
    cur ^= 1;
    wave_lds_fence();
  });
  T *mu = a.mu + (long)b * set;
  mu[o] = xs[cur][o];
  mu[L.SD + o] = xs[cur][L.SD + o];
}

// ------------------------------------------------------------------ B2
template <typename T, int DP> __global__ __launch_bounds__(64) void k_wB2(SweepArgs<T> a) {
  W_SETUP
  const T *lN = a.lam_ckpt + (long)a.nb * set;
  w_put(xs[0], L, o, lN[o], lN[L.SD + o]);
  wave_lds_fence();
  const T one = a.mu ? (T)1 : (T)0;
  auto dptr = [&](int i) -> const T * { return a.E + (a.nb - 1 - i) * mat; };
  auto mptr = [&](int i) -> const T * {
    return a.mu ? a.mu + (long)(a.nb - 1 - i) * set : a.psi0;  // psi0: finite placeholder
  };
  w_pipeline<T, DP, true>(L, a.nb - 1, dptr, mptr, [&](int i, const T (&r)[2 * DP], T mr, T mi) {
    T yr, yi;
    w_apply<T, DP>(L, r, xs[cur], mr, mi, one, yr, yi);
    w_put(xs[cur ^ 1], L, o, yr, yi);
    T *c = a.lam_ckpt + (long)(a.nb - 1 - i) * set;
    c[o] = yr;
    c[L.SD + o] = yi;
    cur ^= 1;
    wave_lds_fence();
  });
}

// ------------------------------------------------------------------ B3
template <typename T, int DP> __global__ __launch_bounds__(64) void k_wB3(SweepArgs<T> a) {
  W_SETUP
  const int b = blockIdx.x;
  const int start = b * a.L, end = min(a.N, start + a.L);
  const T *c = a.lam_ckpt + (long)(b + 1) * set;
  w_put(xs[0], L, o, c[o], c[L.SD + o]);
  wave_lds_fence();
  const T wgt = a.pw ? a.pw[L.m] : (T)0;
  auto dptr = [&](int i) -> const T * { return a.D + (end - 1 - i) * mat; };
  auto pptr = [&](int i) -> const T * { return a.psi_buf + (long)(end - 1 - i) * set; };
  w_pipeline<T, DP, true>(L, end - 1 - start, dptr, pptr,
                          [&](int i, const T (&r)[2 * DP], T pr, T pi) {
    const int j = end - 1 - i;
    T *lb = a.lam_buf + (long)j * set;
    lb[o] = xs[cur][o];  // lambda_{j+1}
    lb[L.SD + o] = xs[cur][L.SD + o];
    T yr, yi;
    w_apply<T, DP>(L, r, xs[cur], pr, pi, j >= 1 ? wgt : (T)0, yr, yi);
    w_put(xs[cur ^ 1], L, o, yr, yi);
    cur ^= 1;
    wave_lds_fence();
  });
  T *lb = a.lam_buf + (long)start * set;
  lb[o] = xs[cur][o];
  lb[L.SD + o] = xs[cur][L.SD + o];
}

template <typename T> bool wave_sweep_ok(int dp, int S) {
  return (dp == 16 && S * dp <= 64) || (dp == 32 && S * dp <= 64);
}

template <typename T, int DP> hipError_t w_launch(int which, const SweepArgs<T> &a, hipStream_t st) {
  switch (which) {
    case 0: hipLaunchKernelGGL((k_wF2<T, DP>), dim3(1), dim3(64), 0, st, a); break;
    case 1: hipLaunchKernelGGL((k_wF3<T, DP>), dim3(a.nb), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_wB2<T, DP>), dim3(1), dim3(64), 0, st, a); break;
    default: hipLaunchKernelGGL((k_wB3<T, DP>), dim3(a.nb), dim3(64), 0, st, a); break;
  }
  return hipGetLastError();
}

template <typename T> hipError_t launch_wave_sweep(int which, const SweepArgs<T> &a, hipStream_t st) {
  if (a.dp == 16) return w_launch<T, 16>(which, a, st);
  if (a.dp == 32) return w_launch<T, 32>(which, a, st);
  return hipErrorInvalidValue;
}

template bool wave_sweep_ok<float>(int, int);
template bool wave_sweep_ok<double>(int, int);
template hipError_t launch_wave_sweep<float>(int, const SweepArgs<float> &, hipStream_t);
template hipError_t launch_wave_sweep<double>(int, const SweepArgs<double> &, hipStream_t);

}  // namespace qoc
