// Chain-workgroup sweeps for padded d 64 .. 128 (sweep variant 4).
//
// The blocked two-level scan of kernels_sweep.hip (F2 / F3 / B2 / B3), one
// workgroup of 8 d_pad threads per (block, state) -- a whole compute unit
// on one sequential chain of matrix-vector products.  Each thread owns a
// fixed slice of every step matrix and keeps the slices of the next RD
// steps in registers (a prefetch ring), so the chain waits on HBM only for
// the first steps; the barriers order LDS only (no wait on the loads in
// flight).
//
//   y = x + op(M) x (+ aux)
//   forward (op = 1): thread (r, g) = (t / 8, t % 8) takes row r, columns
//     g KC .. g KC + KC - 1 (KC = d_pad / 8); the eight partial sums of a
//     row meet through lane swizzles, lane g = 0 owns y_r.
//   adjoint (op = ^H): thread (c, s) = (t % G, t / G) takes the VN
//     columns c VN .. of rows s, s + SL, ... (G = d_pad / VN column groups,
//     SL = 8 d_pad / G row slices); partial sums meet in LDS, thread c' <
//     d_pad owns y_c'.
#include <type_traits>

#include "qoc_device.h"
#include "qoc_kernels.h"

namespace qoc {

// steps prefetched ahead (3 keeps d_pad 128 within the 128 registers of a
// 16-wavefront workgroup; 4 spills)
#ifndef QOC_CHAIN_RD
#define QOC_CHAIN_RD 3
#endif

template <typename T, int DP> struct ChainGeo {
  static constexpr int NT = 8 * DP;                  // threads
  static constexpr int KC = DP / 8;                  // forward columns per thread
  static constexpr int FV = (KC % 4 == 0 && sizeof(T) == 4) ? 4 : 2;  // forward vector (elems)
  static constexpr int AV = 16 / sizeof(T);          // adjoint vector (elems)
  static constexpr int G = DP / AV;                  // adjoint column groups
  static constexpr int SL = NT / G;                  // adjoint row slices
  static constexpr int RS = (DP + SL - 1) / SL;      // adjoint rows per slice
  static constexpr int FE = 2 * KC;                  // forward ring elements per step
  static constexpr int AE = 2 * RS * AV;             // adjoint ring elements per step
  static constexpr int RD = QOC_CHAIN_RD;
};

template <typename T, int N> struct VecN;
template <> struct VecN<float, 4> { typedef float4 type; };
template <> struct VecN<float, 2> { typedef float2 type; };
template <> struct VecN<double, 2> { typedef double2 type; };

template <int CTRL> __device__ __forceinline__ float c_swz(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double c_swz(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// sum over the 8 lanes t & ~7 .. (t & ~7) + 7; every lane gets the total
// (each swizzle adds the same two values in either order)
template <typename T> __device__ __forceinline__ T sum8(T v) {
  v += c_swz<0xB1>(v);         // lane ^ 1
  v += c_swz<0x4E>(v);         // lane ^ 2
  v += __shfl_xor(v, 4, 64);   // lane ^ 4
  return v;
}

// ---- slices of one step matrix M (planar re, im; dp x dp row-major)
template <typename T, int DP>
__device__ __forceinline__ void fwd_load(const T *__restrict__ M, int t, T (&r)[ChainGeo<T, DP>::FE]) {
  typedef ChainGeo<T, DP> G;
  typedef typename VecN<T, G::FV>::type V;
  const int row = t >> 3, g = t & 7;
  const T *p = M + row * DP + g * G::KC;
#pragma unroll
  for (int k = 0; k < G::KC; k += G::FV) {
    const V a = *reinterpret_cast<const V *>(p + k);
    const V b = *reinterpret_cast<const V *>(p + DP * DP + k);
    const T *ea = reinterpret_cast<const T *>(&a), *eb = reinterpret_cast<const T *>(&b);
#pragma unroll
    for (int e = 0; e < G::FV; ++e) {
      r[k + e] = ea[e];
      r[G::KC + k + e] = eb[e];
    }
  }
}
template <typename T, int DP>
__device__ __forceinline__ void adj_load(const T *__restrict__ M, int t, T (&r)[ChainGeo<T, DP>::AE]) {
  typedef ChainGeo<T, DP> G;
  typedef typename VecN<T, G::AV>::type V;
  const int c = t % G::G, s = t / G::G;
#pragma unroll
  for (int i = 0; i < G::RS; ++i) {
    const int k = s + i * G::SL;
    const int kk = k < DP ? k : DP - 1;  // rows beyond dp: a valid address, weight 0 below
    const V a = *reinterpret_cast<const V *>(M + kk * DP + c * G::AV);
    const V b = *reinterpret_cast<const V *>(M + DP * DP + kk * DP + c * G::AV);
    const T *ea = reinterpret_cast<const T *>(&a), *eb = reinterpret_cast<const T *>(&b);
#pragma unroll
    for (int e = 0; e < G::AV; ++e) {
      r[(2 * i) * G::AV + e] = ea[e];
      r[(2 * i + 1) * G::AV + e] = eb[e];
    }
  }
}

// ---- one step.  x, y: LDS [re dp][im dp]; red: LDS scratch of the adjoint
// (2 * SL * dp elements).  The owner thread of an output row (fwd: g == 0,
// adj: t < dp) writes it to y and gets it in (or_, oi); returns ownership.
template <typename T, int DP>
__device__ __forceinline__ bool fwd_step(int t, const T (&r)[ChainGeo<T, DP>::FE], const T *x,
                                         T *y, T aux_r, T aux_i, T &or_, T &oi) {
  typedef ChainGeo<T, DP> G;
  const int row = t >> 3, g = t & 7;
  const T *xr = x + g * G::KC, *xi = x + DP + g * G::KC;
  // two partial sums, each started from its first term (an added zero
  // cannot be dropped by the compiler)
  T pr0, pr1, pi0, pi1;
#pragma unroll
  for (int k = 0; k < G::KC; ++k) {
    const T a = xr[k], b = xi[k];
    const T tr = r[k] * a - r[G::KC + k] * b, ti = r[k] * b + r[G::KC + k] * a;
    if (k == 0) {
      pr0 = tr;
      pi0 = ti;
    } else if (k == 1) {
      pr1 = tr;
      pi1 = ti;
    } else if (k & 1) {
      pr1 += tr;
      pi1 += ti;
    } else {
      pr0 += tr;
      pi0 += ti;
    }
  }
  const T sr = sum8(pr0 + pr1), si = sum8(pi0 + pi1);
  if (g == 0) {
    or_ = x[row] + sr + aux_r;
    oi = x[DP + row] + si + aux_i;
    y[row] = or_;
    y[DP + row] = oi;
    return true;
  }
  return false;
}

template <typename T, int DP>
__device__ __forceinline__ bool adj_step(int t, const T (&r)[ChainGeo<T, DP>::AE], const T *x,
                                         T *y, T *red, T aux_r, T aux_i, T &or_, T &oi) {
  typedef ChainGeo<T, DP> G;
  const int c = t % G::G, s = t / G::G;
  T pr[G::AV], pi[G::AV];
#pragma unroll
  for (int i = 0; i < G::RS; ++i) {
    const int k = s + i * G::SL;
    if (i == 0 || k < DP) {  // row s < SL <= DP always exists
      const T a = x[k], b = x[DP + k];
#pragma unroll
      for (int e = 0; e < G::AV; ++e) {
        const T mr = r[(2 * i) * G::AV + e], mi = -r[(2 * i + 1) * G::AV + e];  // conj
        const T tr = mr * a - mi * b, ti = mr * b + mi * a;
        pr[e] = i == 0 ? tr : pr[e] + tr;
        pi[e] = i == 0 ? ti : pi[e] + ti;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < G::AV; ++e) {
    red[s * DP + c * G::AV + e] = pr[e];
    red[(G::SL + s) * DP + c * G::AV + e] = pi[e];
  }
  lds_barrier();
  bool own = false;
  if (t < DP) {
    // the SL slices' partial sums in four interleaved chains
    static_assert(G::SL % 4 == 0, "slices");
    T sr4[4], si4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sr4[u] = red[u * DP + t];
      si4[u] = red[(G::SL + u) * DP + t];
    }
#pragma unroll
    for (int q = 4; q < G::SL; q += 4)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        sr4[u] += red[(q + u) * DP + t];
        si4[u] += red[(G::SL + q + u) * DP + t];
      }
    const T sr = (sr4[0] + sr4[1]) + (sr4[2] + sr4[3]);
    const T si = (si4[0] + si4[1]) + (si4[2] + si4[3]);
    or_ = x[t] + sr + aux_r;
    oi = x[DP + t] + si + aux_i;
    y[t] = or_;
    y[DP + t] = oi;
    own = true;
  }
  return own;
}

// Ring-pipelined chain of `count` steps: step i uses the slices loaded RD
// steps earlier (loads clamped to the last step, none under a condition);
// step(i, slices, aux_r, aux_i) with the owner thread's addend, read at
// aptr(i)[orow] and aptr(i)[imoff + orow] (null: none).
template <typename T, int DP, bool ADJ, class MPtr, class APtr, class Step>
__device__ __forceinline__ void c_pipeline(int t, int count, MPtr mptr, APtr aptr, int orow,
                                           long imoff, Step step) {
  typedef ChainGeo<T, DP> G;
  constexpr int RD = G::RD, E = ADJ ? G::AE : G::FE;
  if (count <= 0) return;
  T r[RD][E];
  T ar[RD], ai[RD];
  auto load = [&](int q, int i) {
    if constexpr (ADJ)
      adj_load<T, DP>(mptr(i), t, r[q]);
    else
      fwd_load<T, DP>(mptr(i), t, r[q]);
    const T *a = aptr(i);
    ar[q] = a ? a[orow] : (T)0;
    ai[q] = a ? a[imoff + orow] : (T)0;
  };
#pragma unroll
  for (int q = 0; q < RD; ++q) load(q, q < count ? q : count - 1);
  int i0 = 0;
  for (; i0 + RD <= count; i0 += RD) {
#pragma unroll
    for (int q = 0; q < RD; ++q) {
      step(i0 + q, r[q], ar[q], ai[q]);
      load(q, i0 + q + RD < count ? i0 + q + RD : count - 1);
    }
  }
#pragma unroll
  for (int q = 0; q < RD - 1; ++q)
    if (i0 + q < count) step(i0 + q, r[q], ar[q], ai[q]);
}

// state s of a set [2][S][dp]: re at s dp + m, im at (S + s) dp + m
#define C_SETUP                                                              \
  typedef ChainGeo<T, DP> G;                                                 \
  __shared__ __align__(16) T xs[2][2 * DP];                                  \
  __shared__ __align__(16) T red[2 * G::SL * DP];                            \
  const int t = threadIdx.x;                                                 \
  const int S = a.S;                                                         \
  const long set = 2L * S * DP, mat = 2L * DP * DP;                          \
  int cur = 0;                                                               \
  (void)red;

// y to global: a state-set entry (owner thread only)
template <typename T>
__device__ __forceinline__ void c_put(T *setp, int S, int dp, int s, int m, T vr, T vi) {
  setp[(long)s * dp + m] = vr;
  setp[(long)(S + s) * dp + m] = vi;
}

// ------------------------------------------------------------------ F2
template <typename T, int DP> __global__ __launch_bounds__(8 * DP) void k_cF2(SweepArgs<T> a) {
  C_SETUP
  const int s = blockIdx.x;
  if (t < DP) {
    const T vr = a.psi0[(long)s * DP + t], vi = a.psi0[(long)(S + s) * DP + t];
    xs[0][t] = vr;
    xs[0][DP + t] = vi;
    c_put(a.ckpt, S, DP, s, t, vr, vi);
  }
  lds_barrier();
  auto mptr = [&](int i) -> const T * { return a.E + (long)i * mat; };
  auto aptr = [&](int) -> const T * { return nullptr; };
  c_pipeline<T, DP, false>(t, a.nb, mptr, aptr, 0, 0, [&](int b, const T(&r)[G::FE], T, T) {
    T vr = 0, vi = 0;
    if (fwd_step<T, DP>(t, r, xs[cur], xs[cur ^ 1], (T)0, (T)0, vr, vi))
      c_put(a.ckpt + (long)(b + 1) * set, S, DP, s, t >> 3, vr, vi);
    cur ^= 1;
    lds_barrier();
  });
}

// ------------------------------------------------------------------ F3
template <typename T, int DP> __global__ __launch_bounds__(8 * DP) void k_cF3(SweepArgs<T> a) {
  C_SETUP
  // (block, state) from the XCD-grouped 1-D grid (xcd_grid in the launch)
  const long lg_ = xcd_logical_block(blockIdx.x, gridDim.x);
  if (lg_ >= (long)a.nb * S) return;  // padding of the grid
  const int b = (int)(lg_ / S), s = (int)(lg_ - lg_ / S * S);
  const int start = b * a.L, end = min(a.N, start + a.L), cnt = end - start;
  if (t < DP) {
    const T *c = a.ckpt + (long)b * set;
    const T vr = c[(long)s * DP + t], vi = c[(long)(S + s) * DP + t];
    xs[0][t] = vr;
    xs[0][DP + t] = vi;
    c_put(a.psi_buf + (long)start * set, S, DP, s, t, vr, vi);
  }
  lds_barrier();
  auto fptr = [&](int i) -> const T * { return a.D + (long)(start + i) * mat; };
  auto none = [&](int) -> const T * { return nullptr; };
  c_pipeline<T, DP, false>(t, cnt, fptr, none, 0, 0, [&](int i, const T(&r)[G::FE], T, T) {
    T vr = 0, vi = 0;
    const int j = start + i;
    if (fwd_step<T, DP>(t, r, xs[cur], xs[cur ^ 1], (T)0, (T)0, vr, vi))
      if (j + 1 < end || j + 1 == a.N)
        c_put(a.psi_buf + (long)(j + 1) * set, S, DP, s, t >> 3, vr, vi);
    cur ^= 1;
    lds_barrier();
  });
  if (!a.pw) return;  // uniform
  // block-local penalty costate from zero at the block end:
  // mu <- mu + D_j^H mu + pw o psi_j (j >= 1), over the states written above
  __threadfence_block();
  if (t < DP) {
    xs[cur][t] = (T)0;
    xs[cur][DP + t] = (T)0;
  }
  __syncthreads();
  const int orow = t < DP ? t : 0;
  const T wgt = a.pw[orow];
  auto bptr = [&](int i) -> const T * { return a.D + (long)(end - 1 - i) * mat; };
  auto pptr = [&](int i) -> const T * { return a.psi_buf + (long)(end - 1 - i) * set + (long)s * DP; };
  T mr = 0, mi = 0;
  c_pipeline<T, DP, true>(t, cnt, bptr, pptr, orow, (long)S * DP,
                          [&](int i, const T(&r)[G::AE], T pr, T pi) {
    const int j = end - 1 - i;
    const T w = j >= 1 ? wgt : (T)0;
    T vr = 0, vi = 0;
    adj_step<T, DP>(t, r, xs[cur], xs[cur ^ 1], red, w * pr, w * pi, vr, vi);
    mr = vr;
    mi = vi;
    cur ^= 1;
    lds_barrier();
  });
  if (t < DP) {
    T *mu = a.mu + (long)b * set;
    mu[(long)s * DP + t] = cnt > 0 ? mr : (T)0;
    mu[(long)(S + s) * DP + t] = cnt > 0 ? mi : (T)0;
  }
}

// ------------------------------------------------------------------ B2
template <typename T, int DP> __global__ __launch_bounds__(8 * DP) void k_cB2(SweepArgs<T> a) {
  C_SETUP
  const int s = blockIdx.x;
  if (t < DP) {
    const T *lN = a.lam_ckpt + (long)a.nb * set;
    xs[0][t] = lN[(long)s * DP + t];
    xs[0][DP + t] = lN[(long)(S + s) * DP + t];
  }
  lds_barrier();
  const int orow = t < DP ? t : 0;
  auto mptr = [&](int i) -> const T * { return a.E + (long)(a.nb - 1 - i) * mat; };
  auto aptr = [&](int i) -> const T * {
    return a.mu ? a.mu + (long)(a.nb - 1 - i) * set + (long)s * DP : nullptr;
  };
  c_pipeline<T, DP, true>(t, a.nb - 1, mptr, aptr, orow, (long)S * DP,
                          [&](int i, const T(&r)[G::AE], T mr, T mi) {
    T vr = 0, vi = 0;
    if (adj_step<T, DP>(t, r, xs[cur], xs[cur ^ 1], red, mr, mi, vr, vi))
      c_put(a.lam_ckpt + (long)(a.nb - 1 - i) * set, S, DP, s, t, vr, vi);
    cur ^= 1;
    lds_barrier();
  });
}

// ------------------------------------------------------------------ B3
template <typename T, int DP> __global__ __launch_bounds__(8 * DP) void k_cB3(SweepArgs<T> a) {
  C_SETUP
  // (block, state) from the XCD-grouped 1-D grid (xcd_grid in the launch)
  const long lg_ = xcd_logical_block(blockIdx.x, gridDim.x);
  if (lg_ >= (long)a.nb * S) return;  // padding of the grid
  const int b = (int)(lg_ / S), s = (int)(lg_ - lg_ / S * S);
  const int start = b * a.L, end = min(a.N, start + a.L);
  if (t < DP) {
    const T *c = a.lam_ckpt + (long)(b + 1) * set;
    xs[0][t] = c[(long)s * DP + t];
    xs[0][DP + t] = c[(long)(S + s) * DP + t];
  }
  lds_barrier();
  const int orow = t < DP ? t : 0;
  const T wgt = a.pw ? a.pw[orow] : (T)0;
  auto mptr = [&](int i) -> const T * { return a.D + (long)(end - 1 - i) * mat; };
  auto pptr = [&](int i) -> const T * {
    return a.pw ? a.psi_buf + (long)(end - 1 - i) * set + (long)s * DP : nullptr;
  };
  T lr = t < DP ? xs[0][t] : (T)0, li = t < DP ? xs[0][DP + t] : (T)0;
  c_pipeline<T, DP, true>(t, end - 1 - start, mptr, pptr, orow, (long)S * DP,
                          [&](int i, const T(&r)[G::AE], T pr, T pi) {
    const int j = end - 1 - i;
    if (t < DP) c_put(a.lam_buf + (long)j * set, S, DP, s, t, lr, li);  // lambda_{j+1}
    const T w = j >= 1 ? wgt : (T)0;
    T vr = 0, vi = 0;
    adj_step<T, DP>(t, r, xs[cur], xs[cur ^ 1], red, w * pr, w * pi, vr, vi);
    lr = vr;
    li = vi;
    cur ^= 1;
    lds_barrier();
  });
  if (t < DP) c_put(a.lam_buf + (long)start * set, S, DP, s, t, lr, li);
}

// FP32 only: at 8 d_pad threads a wavefront has 128 registers, which an
// FP64 ring would not fit.
template <typename T> bool chain_sweep_ok(int dp, int S) {
  (void)S;
  return sizeof(T) == 4 && dp >= 64 && dp <= 128 && dp % 16 == 0;
}

template <typename T, int DP> hipError_t c_launch(int which, const SweepArgs<T> &a, hipStream_t st) {
  const dim3 blk(8 * DP);
  switch (which) {
    case 0: hipLaunchKernelGGL((k_cF2<T, DP>), dim3(a.S), blk, 0, st, a); break;
    case 1: hipLaunchKernelGGL((k_cF3<T, DP>), dim3(xcd_grid((long)a.nb * a.S, a.S)), blk, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_cB2<T, DP>), dim3(a.S), blk, 0, st, a); break;
    default: hipLaunchKernelGGL((k_cB3<T, DP>), dim3(xcd_grid((long)a.nb * a.S, a.S)), blk, 0, st, a); break;
  }
  return hipGetLastError();
}

template <typename T> hipError_t launch_chain_sweep(int which, const SweepArgs<T> &a, hipStream_t st) {
  if constexpr (sizeof(T) != 4) {
    (void)which;
    (void)a;
    (void)st;
    return hipErrorInvalidValue;
  } else {
    switch (a.dp) {
      case 64: return c_launch<T, 64>(which, a, st);
      case 80: return c_launch<T, 80>(which, a, st);
      case 96: return c_launch<T, 96>(which, a, st);
      case 112: return c_launch<T, 112>(which, a, st);
      case 128: return c_launch<T, 128>(which, a, st);
      default: return hipErrorInvalidValue;
    }
  }
}

template bool chain_sweep_ok<float>(int, int);
template bool chain_sweep_ok<double>(int, int);
template hipError_t launch_chain_sweep<float>(int, const SweepArgs<float> &, hipStream_t);
template hipError_t launch_chain_sweep<double>(int, const SweepArgs<double> &, hipStream_t);

}  // namespace qoc
