// Single-wavefront sweeps for the smallest problems (padded d 16 or 32).
//
// The blocked two-level scan of kernels_sweep.hip (F2 / F3 / B2 / B3) with
// one wavefront per state (the S states of a set never mix, so they run as
// independent wavefronts, grid dimension y).  Output row m of a step is
// shared by KQ = 64 / d_pad adjacent lanes: lane (m, kq) takes the inner
// indices kq KC .. kq KC + KC - 1 (KC = d_pad / KQ) of
//   y_m = x_m + sum_k op(D)[m][k] x_k  (+ w_m aux_m),
// and the KQ partial sums are combined with DPP lane swizzles, which leave
// the bitwise identical total in every lane of the group (each swizzle adds
// the same two values in either order).  Each lane keeps its KC-wide slice
// of row m for the next RD steps in registers (a prefetch ring), reads its
// KC entries of the state from LDS and, after the update, the group writes
// y_m back; there is no workgroup barrier on the sequential path.  The
// costate passes read rows of D^H and E^H, written by the small-path
// kernels, so every pass streams contiguous 16-byte pieces and no
// arithmetic waits on a load in flight.  All lanes of a group store the
// same value to the same address, so every store is unconditional and the
// compiler's wait counts stay exact.
#include <type_traits>

#include "qoc_device.h"
#include "qoc_cost.h"
#include "qoc_kernels.h"

namespace qoc {

#ifndef QOC_WAVE_RD16
#define QOC_WAVE_RD16 8
#endif
#ifndef QOC_WAVE_RD32
#define QOC_WAVE_RD32 4
#endif
template <int DP> struct WaveGeo {
  static constexpr int KQ = 64 / DP;  // lanes per output row
  static constexpr int KC = DP / KQ;  // inner indices per lane
  static constexpr int RD = DP <= 16 ? QOC_WAVE_RD16 : QOC_WAVE_RD32;  // steps prefetched ahead
};

__device__ __forceinline__ void wave_lds_fence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// v from lane l ^ 1 (CTRL 0xB1) or l ^ 2 (CTRL 0x4E): DPP quad permutations
template <int CTRL> __device__ __forceinline__ float dpp_swz(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_swz(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <typename T, int KQ> __device__ __forceinline__ T group_sum(T v) {
  v += dpp_swz<0xB1>(v);
  if (KQ == 4) v += dpp_swz<0x4E>(v);
  return v;
}

struct WLane {
  int m, kq;  // output row, inner-index slice
  int o, oi;  // (s, m) in a state set: real and imaginary entries
};

// Slice kq of row m of a step matrix (D, or D^H for the costate passes).
template <typename T, int DP>
__device__ __forceinline__ void w_load(const T *__restrict__ D, const WLane &L,
                                       T (&r)[2 * WaveGeo<DP>::KC]) {
  constexpr int KC = WaveGeo<DP>::KC;
  const T *p = D + L.m * DP + L.kq * KC;
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    r[k] = p[k];
    r[KC + k] = p[DP * DP + k];
  }
}

// sum_k row[k] x_k over the whole row (all KQ lanes of the group); xs is
// this wavefront's state in LDS, [re DP][im DP].  The slice's dot product
// runs as WA independent partial sums, the state read in 16-byte pieces.
template <typename T, int DP>
__device__ __forceinline__ void w_dot(const WLane &L, const T (&r)[2 * WaveGeo<DP>::KC],
                                      const T *xs, T &sr, T &si) {
  constexpr int KC = WaveGeo<DP>::KC, KQ = WaveGeo<DP>::KQ;
  constexpr int WA = KC < 4 ? KC : 4;
  typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type V;
  constexpr int VN = 16 / sizeof(T);
  const T *xr = xs + L.kq * KC, *xi = xs + DP + L.kq * KC;
  // each partial sum starts from its first term (an added zero cannot be
  // dropped by the compiler and would lengthen the chain)
  T pr[WA], pi[WA];
#pragma unroll
  for (int k0 = 0; k0 < KC; k0 += VN) {
    const V xv = *reinterpret_cast<const V *>(xr + k0);
    const V yv = *reinterpret_cast<const V *>(xi + k0);
    const T *xa = reinterpret_cast<const T *>(&xv), *ya = reinterpret_cast<const T *>(&yv);
#pragma unroll
    for (int e = 0; e < VN; ++e) {
      const int k = k0 + e, q = k % WA;
      const T tr = r[k] * xa[e] - r[KC + k] * ya[e];
      const T ti = r[k] * ya[e] + r[KC + k] * xa[e];
      if (k < WA) {  // compile-time
        pr[q] = tr;
        pi[q] = ti;
      } else {
        pr[q] += tr;
        pi[q] += ti;
      }
    }
  }
  T ar = pr[0], ai = pi[0];
#pragma unroll
  for (int q = 1; q < WA; ++q) {
    ar += pr[q];
    ai += pi[q];
  }
  sr = group_sum<T, KQ>(ar);
  si = group_sum<T, KQ>(ai);
}

// Ring-pipelined loop over `count` steps: step i uses the slice loaded RD
// steps earlier.  Whole chunks of RD steps run with no condition around
// the loads (the index is clamped to the last step), so the compiler can
// count the loads in flight exactly and wait only for the slot it reads;
// a last partial chunk only drains the ring.  step(i, slice, aux_r, aux_i).
template <typename T, int DP, class DPtr, class APtr, class Step>
__device__ __forceinline__ void w_pipeline(const WLane &L, int count, DPtr dptr, APtr aptr,
                                           Step step) {
  constexpr int RD = WaveGeo<DP>::RD, KC = WaveGeo<DP>::KC;
  if (count <= 0) return;
  T r[RD][2 * KC];
  T ar[RD], ai[RD];
#pragma unroll
  for (int q = 0; q < RD; ++q) {
    const int i = q < count ? q : count - 1;
    w_load<T, DP>(dptr(i), L, r[q]);
    const T *a = aptr(i);
    ar[q] = a[L.o];
    ai[q] = a[L.oi];
  }
  int i0 = 0;
  for (; i0 + RD <= count; i0 += RD) {
#pragma unroll
    for (int q = 0; q < RD; ++q) {
      step(i0 + q, r[q], ar[q], ai[q]);
      const int nx = (i0 + q + RD < count) ? i0 + q + RD : count - 1;
      w_load<T, DP>(dptr(nx), L, r[q]);
      const T *a = aptr(nx);
      ar[q] = a[L.o];
      ai[q] = a[L.oi];
    }
  }
#pragma unroll
  for (int q = 0; q < RD - 1; ++q)
    if (i0 + q < count) step(i0 + q, r[q], ar[q], ai[q]);
}

// One wavefront: state ws (blockIdx.y unless given) of a set [2][S][DP].
#define W_SETUP_STATE(state)                                     \
  constexpr int KC = WaveGeo<DP>::KC;                            \
  __shared__ __align__(16) T xs[2][2 * DP];                      \
  const int ws = (state);                                        \
  WLane L;                                                       \
  L.m = threadIdx.x / WaveGeo<DP>::KQ;                           \
  L.kq = threadIdx.x - L.m * WaveGeo<DP>::KQ;                    \
  L.o = ws * DP + L.m;                                           \
  L.oi = (a.S + ws) * DP + L.m;                                  \
  const long set = 2L * a.S * DP, mat = 2L * DP * DP;            \
  int cur = 0;                                                   \
  (void)mat;
#define W_SETUP W_SETUP_STATE((int)blockIdx.y)

template <typename T> __device__ __forceinline__ void w_put(T *xs, int m, int dp, T vr, T vi) {
  xs[m] = vr;
  xs[dp + m] = vi;
}

// ------------------------------------------------------------------ F2
template <typename T, int DP> __global__ __launch_bounds__(64) void k_wF2(SweepArgs<T> a) {
  W_SETUP
  T xr = a.psi0[L.o], xi = a.psi0[L.oi];
  w_put(xs[0], L.m, DP, xr, xi);
  a.ckpt[L.o] = xr;
  a.ckpt[L.oi] = xi;
  wave_lds_fence();
  auto dptr = [&](int i) -> const T * { return a.E + i * mat; };
  auto aptr = [&](int) -> const T * { return a.psi0; };  // unused
  w_pipeline<T, DP>(L, a.nb, dptr, aptr, [&](int b, const T (&r)[2 * KC], T, T) {
    T sr, si;
    w_dot<T, DP>(L, r, xs[cur], sr, si);
    xr += sr;
    xi += si;
    w_put(xs[cur ^ 1], L.m, DP, xr, xi);
    T *c = a.ckpt + (long)(b + 1) * set;
    c[L.o] = xr;
    c[L.oi] = xi;
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
  T xr = ck[L.o], xi = ck[L.oi];
  w_put(xs[0], L.m, DP, xr, xi);
  a.psi_buf[(long)start * set + L.o] = xr;
  a.psi_buf[(long)start * set + L.oi] = xi;
  wave_lds_fence();
  auto fptr = [&](int i) -> const T * { return a.D + (start + i) * mat; };
  auto dummy = [&](int) -> const T * { return ck; };
  w_pipeline<T, DP>(L, cnt, fptr, dummy, [&](int i, const T (&r)[2 * KC], T, T) {
    T sr, si;
    w_dot<T, DP>(L, r, xs[cur], sr, si);
    xr += sr;
    xi += si;
    w_put(xs[cur ^ 1], L.m, DP, xr, xi);
    const int j = start + i;
    if (j + 1 < end || j + 1 == a.N) {  // wave-uniform
      a.psi_buf[(long)(j + 1) * set + L.o] = xr;
      a.psi_buf[(long)(j + 1) * set + L.oi] = xi;
    }
    cur ^= 1;
    wave_lds_fence();
  });
  if (!a.pw) return;  // uniform
  // block-local penalty costate from zero at the block end:
  // mu <- mu + D_j^H mu + pw o psi_j (j >= 1), over the states written above
  __threadfence_block();
  const T wgt = a.pw[L.m];
  T mr = (T)0, mi = (T)0;
  w_put(xs[cur], L.m, DP, mr, mi);
  wave_lds_fence();
  auto bptr = [&](int i) -> const T * { return a.Dh + (end - 1 - i) * mat; };
  auto pptr = [&](int i) -> const T * { return a.psi_buf + (long)(end - 1 - i) * set; };
  w_pipeline<T, DP>(L, cnt, bptr, pptr, [&](int i, const T (&r)[2 * KC], T pr, T pi) {
    const int j = end - 1 - i;
    T sr, si;
    w_dot<T, DP>(L, r, xs[cur], sr, si);
    // select, not multiply: an unused auxiliary operand is never touched
    mr += sr + (j >= 1 ? wgt * pr : (T)0);
    mi += si + (j >= 1 ? wgt * pi : (T)0);
    w_put(xs[cur ^ 1], L.m, DP, mr, mi);
    cur ^= 1;
    wave_lds_fence();
  });
  T *mu = a.mu + (long)b * set;
  mu[L.o] = mr;
  mu[L.oi] = mi;
}

// ------------------------------------------------------------------ B2
// With fuse_cost (a 1-D grid of S + npart wavefronts): wavefronts 0..S-1
// form lambda_N of their state themselves (fidelity included) and run the
// chain; the others run the penalty pass beside them, each storing its
// partials for the total.  Otherwise (grid 1 x S) lambda_N is read.
template <typename T, int DP> __global__ __launch_bounds__(64) void k_wB2(SweepArgs<T> a) {
  if (a.fuse_cost && (int)blockIdx.x >= a.S) {  // block-uniform: a penalty wavefront
    const long wi = (long)blockIdx.x - a.S;
    double cpen, camp, cvar, dmax;
    pen_wave(a, wi, (long)a.npart, cpen, camp, cvar, dmax);
    if (threadIdx.x == 0) {
      a.part[wi] = cpen;
      a.part[a.npart + wi] = camp;
      a.part[2 * a.npart + wi] = cvar;
      a.part[3 * a.npart + wi] = dmax;
    }
    return;
  }
  W_SETUP_STATE(a.fuse_cost ? (int)blockIdx.x : (int)blockIdx.y)
  T *lN = a.lam_ckpt + (long)a.nb * set;
  T xr, xi;
  if (a.fuse_cost) {
    lam_wave<T, DP>(a, ws, L.m, L.kq, xr, xi);
    lN[L.o] = xr;  // lambda_N for the in-block costate pass
    lN[L.oi] = xi;
  } else {
    xr = lN[L.o];
    xi = lN[L.oi];
  }
  w_put(xs[0], L.m, DP, xr, xi);
  wave_lds_fence();
  const bool has_mu = a.mu != nullptr;
  auto dptr = [&](int i) -> const T * { return a.Eh + (a.nb - 1 - i) * mat; };
  // chosen once: without penalties psi0 (finite) stands in, at stride zero
  const T *mbase = has_mu ? a.mu : a.psi0;
  const long mstride = has_mu ? set : 0;
  auto mptr = [&](int i) -> const T * { return mbase + (long)(a.nb - 1 - i) * mstride; };
  w_pipeline<T, DP>(L, a.nb - 1, dptr, mptr, [&](int i, const T (&r)[2 * KC], T mr, T mi) {
    T sr, si;
    w_dot<T, DP>(L, r, xs[cur], sr, si);
    xr += sr + (has_mu ? mr : (T)0);
    xi += si + (has_mu ? mi : (T)0);
    w_put(xs[cur ^ 1], L.m, DP, xr, xi);
    T *c = a.lam_ckpt + (long)(a.nb - 1 - i) * set;
    c[L.o] = xr;
    c[L.oi] = xi;
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
  T xr = c[L.o], xi = c[L.oi];
  w_put(xs[0], L.m, DP, xr, xi);
  wave_lds_fence();
  const T wgt = a.pw ? a.pw[L.m] : (T)0;
  auto dptr = [&](int i) -> const T * { return a.Dh + (end - 1 - i) * mat; };
  auto pptr = [&](int i) -> const T * { return a.psi_buf + (long)(end - 1 - i) * set; };
  w_pipeline<T, DP>(L, end - 1 - start, dptr, pptr,
                    [&](int i, const T (&r)[2 * KC], T pr, T pi) {
    const int j = end - 1 - i;
    T *lb = a.lam_buf + (long)j * set;
    lb[L.o] = xr;  // lambda_{j+1}
    lb[L.oi] = xi;
    T sr, si;
    w_dot<T, DP>(L, r, xs[cur], sr, si);
    xr += sr + (j >= 1 ? wgt * pr : (T)0);
    xi += si + (j >= 1 ? wgt * pi : (T)0);
    w_put(xs[cur ^ 1], L.m, DP, xr, xi);
    cur ^= 1;
    wave_lds_fence();
  });
  T *lb = a.lam_buf + (long)start * set;
  lb[L.o] = xr;
  lb[L.oi] = xi;
}

// ------------------------------------------------------------ F3 / B3 split
// The in-block passes over sub-blocks of SUB16 steps (FP32, padded d 16,
// given the sub-block products Es / Ehs): one workgroup per (block, state)
// with one wavefront per sub-block.
//
// F3: wavefront 0 walks the sub-block starts, x <- x + Es_q x (at most
// L / SUB16 - 1 steps); then every wavefront replays its own sub-block
// from its start and, with a penalty, forms its sub-block's partial
// costate nu_q from zero at the sub-block end (nu <- nu + D_j^H nu +
// pw o psi_j, j >= 1), and wavefront 0 combines them into the block's
// mu = nu_first + (I + Ehs_first) (... (nu_last)).
// B3: wavefront 0 walks the costate back over the sub-block ends,
// lambda <- lambda + Ehs_q lambda + nu_q; then every wavefront replays its
// own sub-block backwards.  The values are those of the sequential passes
// (the same recursions, regrouped).
//
// Every loop runs over the SUB16 slots of a sub-block, fully unrolled and
// guarded by a uniform count, so the matrix slices, states and auxiliary
// terms sit in registers indexed by constants; each pass's loads are
// issued before the previous pass (or the workgroup barrier) is waited
// for, and the states and partial costates a later pass needs are kept in
// registers or LDS instead of being read back from global memory.
constexpr int WSPLIT_MAX = 8;  // wavefronts per workgroup: L <= 8 SUB16

template <typename T, int DP> struct WSlices {
  T r[SUB16][2 * WaveGeo<DP>::KC];
};
// slot s < count: slice of matrix base + idx(s) * mat (other slots: slot 0's)
template <typename T, int DP, class Idx>
__device__ __forceinline__ void ws_load(WSlices<T, DP> &S, const WLane &L, const T *base,
                                        int count, Idx idx) {
  constexpr long mat = 2L * DP * DP;
#pragma unroll
  for (int t = 0; t < SUB16; ++t) w_load<T, DP>(base + idx(t < count ? t : 0) * mat, L, S.r[t]);
}

#define WS_SETUP                                                     \
  constexpr int KQ = WaveGeo<DP>::KQ;                                \
  __shared__ __align__(16) T xs[WSPLIT_MAX][2][2 * DP];              \
  __shared__ __align__(16) T xb[WSPLIT_MAX][2 * DP];                 \
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;           \
  const long lg_ = xcd_logical_block(blockIdx.x, gridDim.x);         \
  if (lg_ >= (long)a.nb * a.S) return; /* padding of the 1-D grid */ \
  const int ws = (int)(lg_ % a.S), b = (int)(lg_ / a.S);             \
  WLane L;                                                           \
  L.m = lane / KQ;                                                   \
  L.kq = lane - L.m * KQ;                                            \
  L.o = ws * DP + L.m;                                               \
  L.oi = (a.S + ws) * DP + L.m;                                      \
  const long set = 2L * a.S * DP;                                    \
  const int start = b * a.L, end = min(a.N, start + a.L);            \
  const int nsub = (end - start + SUB16 - 1) / SUB16;                \
  const long sb0 = start / SUB16;                                    \
  const int a0 = start + q * SUB16;                                  \
  const int cnt = max(0, min(end, a0 + SUB16) - a0);                 \
  const long a0c = cnt > 0 ? a0 : a.N - 1; /* loads of idle slots */ \
  T(*x2)[2 * DP] = xs[q];                                            \
  int cur = 0;                                                       \
  auto wstep = [&](const T(&r)[2 * WaveGeo<DP>::KC], T &xr, T &xi, T ar, T ai) { \
    T sr, si;                                                        \
    w_dot<T, DP>(L, r, x2[cur], sr, si);                             \
    xr += sr + ar;                                                   \
    xi += si + ai;                                                   \
    w_put(x2[cur ^ 1], L.m, DP, xr, xi);                             \
    cur ^= 1;                                                        \
    wave_lds_fence();                                                \
  };                                                                 \
  auto wset = [&](T xr, T xi) {                                      \
    cur = 0;                                                         \
    w_put(x2[0], L.m, DP, xr, xi);                                   \
    wave_lds_fence();                                                \
  };

template <typename T, int DP> __global__ __launch_bounds__(64 * WSPLIT_MAX) void k_wF3s(SweepArgs<T> a) {
  WS_SETUP
  const bool pen = a.pw != nullptr;  // uniform
  // ---- loads: this sub-block's D_j; for wavefront 0 also the Es of the walk
  WSlices<T, DP> rd, re;
  ws_load(rd, L, a.D, cnt, [&](int t) { return a0c + t; });
  const T *ck = a.ckpt + (long)b * set;
  T xr = ck[L.o], xi = ck[L.oi];
  // ---- sub-block starts (wavefront 0)
  if (q == 0) {
    ws_load(re, L, a.Es, nsub - 1, [&](int t) { return sb0 + t; });
    w_put(xb[0], L.m, DP, xr, xi);
    wset(xr, xi);
#pragma unroll
    for (int t = 0; t < SUB16 - 1; ++t)
      if (t < nsub - 1) {
        wstep(re.r[t], xr, xi, (T)0, (T)0);
        w_put(xb[t + 1], L.m, DP, xr, xi);
      }
  }
  // the penalty pass's D_j^H, in flight across the barrier
  WSlices<T, DP> rh;
  if (pen) ws_load(rh, L, a.Dh, cnt, [&](int t) { return a0c + t; });
  const T wgt = pen ? a.pw[L.m] : (T)0;
  __syncthreads();
  // ---- replay of sub-block q; its states kept for the penalty pass
  T pr[SUB16 + 1], pi[SUB16 + 1];
  if (cnt > 0) {
    xr = xb[q][L.m];
    xi = xb[q][DP + L.m];
    pr[0] = xr;
    pi[0] = xi;
    wset(xr, xi);
    a.psi_buf[(long)a0 * set + L.o] = xr;
    a.psi_buf[(long)a0 * set + L.oi] = xi;
#pragma unroll
    for (int t = 0; t < SUB16; ++t)
      if (t < cnt) {
        wstep(rd.r[t], xr, xi, (T)0, (T)0);
        pr[t + 1] = xr;
        pi[t + 1] = xi;
        const int j = a0 + t;
        if (j + 1 < a0 + cnt || j + 1 == a.N) {  // wave-uniform
          a.psi_buf[(long)(j + 1) * set + L.o] = xr;
          a.psi_buf[(long)(j + 1) * set + L.oi] = xi;
        }
      }
  }
  if (!pen) return;  // uniform
  // wavefront 0: the combination's Ehs, in flight during the penalty pass
  WSlices<T, DP> rc;
  if (q == 0) ws_load(rc, L, a.Ehs, nsub - 1, [&](int t) { return sb0 + t; });
  // ---- partial penalty costate of sub-block q, from zero at its end
  if (cnt > 0) {
    T mr = (T)0, mi = (T)0;
    wset(mr, mi);
#pragma unroll
    for (int t = SUB16 - 1; t >= 0; --t)
      if (t < cnt) {
        const bool on = a0 + t >= 1;
        wstep(rh.r[t], mr, mi, on ? wgt * pr[t] : (T)0, on ? wgt * pi[t] : (T)0);
      }
    w_put(xb[q], L.m, DP, mr, mi);  // the sub-block's start state is no longer needed
    T *nu = a.nu + (sb0 + q) * set;
    nu[L.o] = mr;
    nu[L.oi] = mi;
  }
  __syncthreads();
  // ---- the block's penalty costate from the sub-blocks' (wavefront 0)
  if (q == 0) {
    T mr = xb[nsub - 1][L.m], mi = xb[nsub - 1][DP + L.m];
    wset(mr, mi);
#pragma unroll
    for (int t = SUB16 - 2; t >= 0; --t)
      if (t < nsub - 1) wstep(rc.r[t], mr, mi, xb[t][L.m], xb[t][DP + L.m]);
    T *mu = a.mu + (long)b * set;
    mu[L.o] = mr;
    mu[L.oi] = mi;
  }
}

template <typename T, int DP> __global__ __launch_bounds__(64 * WSPLIT_MAX) void k_wB3s(SweepArgs<T> a) {
  WS_SETUP
  const bool pen = a.pw != nullptr;  // uniform
  // ---- loads: this sub-block's D_j^H and states (slots 1 .. cnt - 1), and
  // for wavefront 0 the Ehs and nu of the walk (sub-blocks 1 .. nsub - 1)
  // (read unconditionally: without a penalty the states are finite and
  // weighted by zero, and the states stand in for nu)
  WSlices<T, DP> rd, re;
  ws_load(rd, L, a.Dh, cnt, [&](int t) { return a0c + t; });
  T pr[SUB16], pi[SUB16];
#pragma unroll
  for (int t = 0; t < SUB16; ++t) {
    const long j = a0c + (t < cnt ? t : 0);
    pr[t] = a.psi_buf[j * set + L.o];
    pi[t] = a.psi_buf[j * set + L.oi];
  }
  T nr[SUB16], ni[SUB16];
  if (q == 0) {
    ws_load(re, L, a.Ehs, nsub, [&](int t) { return sb0 + t; });
    const T *nub = pen ? a.nu : a.psi_buf;
#pragma unroll
    for (int t = 0; t < SUB16; ++t) {
      const long sb = sb0 + (t < nsub ? t : 0);
      nr[t] = nub[sb * set + L.o];
      ni[t] = nub[sb * set + L.oi];
    }
  }
  // ---- costates at the sub-block ends (wavefront 0): xb[t] = lambda at
  // the end of sub-block t
  if (q == 0) {
    const T *c = a.lam_ckpt + (long)(b + 1) * set;
    T xr = c[L.o], xi = c[L.oi];
    w_put(xb[nsub - 1], L.m, DP, xr, xi);
    wset(xr, xi);
#pragma unroll
    for (int t = SUB16 - 1; t >= 1; --t)
      if (t < nsub) {
        wstep(re.r[t], xr, xi, pen ? nr[t] : (T)0, pen ? ni[t] : (T)0);
        w_put(xb[t - 1], L.m, DP, xr, xi);
      }
  }
  __syncthreads();
  if (cnt == 0) return;
  // ---- sub-block q backwards: lam_buf[j] = lambda_{j+1}
  T xr = xb[q][L.m], xi = xb[q][DP + L.m];
  wset(xr, xi);
  const T wgt = pen ? a.pw[L.m] : (T)0;
#pragma unroll
  for (int t = SUB16 - 1; t >= 1; --t)
    if (t < cnt) {
      const int j = a0 + t;
      T *lb = a.lam_buf + (long)j * set;
      lb[L.o] = xr;  // lambda_{j+1}
      lb[L.oi] = xi;
      wstep(rd.r[t], xr, xi, wgt * pr[t], wgt * pi[t]);  // j >= 1 here
    }
  T *lb = a.lam_buf + (long)a0 * set;
  lb[L.o] = xr;
  lb[L.oi] = xi;
}

template <typename T> bool wave_sweep_ok(int dp, int S) {
  return (dp == 16 && S * dp <= 64) || (dp == 32 && S * dp <= 64);
}

// Grid of the split in-block passes: one workgroup per (block, state) on a
// 1-D launch padded to a multiple of 8 S, with the S states of a block at
// consecutive logical indices of one XCD (xcd_logical_block), so that the
// block's step matrices come from HBM once into that XCD's L2 and are read
// there by all S state workgroups.
template <typename T> unsigned ws_grid(const SweepArgs<T> &a) {
  return xcd_grid((long)a.nb * a.S, a.S);
}

template <typename T, int DP> hipError_t w_launch(int which, const SweepArgs<T> &a, hipStream_t st) {
  const unsigned S = (unsigned)a.S;
  switch (which) {
    case 0: hipLaunchKernelGGL((k_wF2<T, DP>), dim3(1, S), dim3(64), 0, st, a); break;
    case 1:
      if constexpr (DP == 16 && sizeof(T) == 4) {
        if (a.Es) {
          hipLaunchKernelGGL((k_wF3s<T, DP>), dim3(ws_grid(a)), dim3(64 * (a.L / SUB16)), 0, st, a);
          break;
        }
      }
      hipLaunchKernelGGL((k_wF3<T, DP>), dim3(a.nb, S), dim3(64), 0, st, a);
      break;
    case 2:
      if (a.fuse_cost)
        hipLaunchKernelGGL((k_wB2<T, DP>), dim3(a.S + a.npart), dim3(64), 0, st, a);
      else
        hipLaunchKernelGGL((k_wB2<T, DP>), dim3(1, S), dim3(64), 0, st, a);
      break;
    default:
      if constexpr (DP == 16 && sizeof(T) == 4) {
        if (a.Es) {
          hipLaunchKernelGGL((k_wB3s<T, DP>), dim3(ws_grid(a)), dim3(64 * (a.L / SUB16)), 0, st, a);
          break;
        }
      }
      hipLaunchKernelGGL((k_wB3<T, DP>), dim3(a.nb, S), dim3(64), 0, st, a);
      break;
  }
  return hipGetLastError();
}

template <typename T> hipError_t launch_wave_sweep(int which, const SweepArgs<T> &a, hipStream_t st) {
  if (!a.Dh || !a.Eh) return hipErrorInvalidValue;
  if (a.Es && (a.dp != 16 || sizeof(T) != 4 || !a.Ehs || a.L % SUB16 || a.L > WSPLIT_MAX * SUB16 ||
               (a.pw && !a.nu)))
    return hipErrorInvalidValue;
  if (a.dp == 16) return w_launch<T, 16>(which, a, st);
  if (a.dp == 32) return w_launch<T, 32>(which, a, st);
  return hipErrorInvalidValue;
}

template bool wave_sweep_ok<float>(int, int);
template bool wave_sweep_ok<double>(int, int);
template hipError_t launch_wave_sweep<float>(int, const SweepArgs<float> &, hipStream_t);
template hipError_t launch_wave_sweep<double>(int, const SweepArgs<double> &, hipStream_t);

}  // namespace qoc
