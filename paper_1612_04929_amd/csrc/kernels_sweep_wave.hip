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
  T pr[WA], pi[WA];
#pragma unroll
  for (int q = 0; q < WA; ++q) {
    pr[q] = 0;
    pi[q] = 0;
  }
#pragma unroll
  for (int k0 = 0; k0 < KC; k0 += VN) {
    const V xv = *reinterpret_cast<const V *>(xr + k0);
    const V yv = *reinterpret_cast<const V *>(xi + k0);
    const T *xa = reinterpret_cast<const T *>(&xv), *ya = reinterpret_cast<const T *>(&yv);
#pragma unroll
    for (int e = 0; e < VN; ++e) {
      const int k = k0 + e, q = k % WA;
      pr[q] += r[k] * xa[e] - r[KC + k] * ya[e];
      pi[q] += r[k] * ya[e] + r[KC + k] * xa[e];
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
  auto mptr = [&](int i) -> const T * {
    return has_mu ? a.mu + (long)(a.nb - 1 - i) * set : a.psi0;  // psi0: finite placeholder
  };
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
// The in-block passes over sub-blocks of SUB16 steps (padded d 16, given
// the sub-block products Es / Ehs): one workgroup per (block, state) with
// one wavefront per sub-block.
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
constexpr int WSPLIT_MAX = 16;  // wavefronts per workgroup: L <= 16 SUB16

#define WS_SETUP                                                     \
  constexpr int KC = WaveGeo<DP>::KC, KQ = WaveGeo<DP>::KQ;          \
  __shared__ __align__(16) T xs[WSPLIT_MAX][2][2 * DP];              \
  __shared__ __align__(16) T xb[WSPLIT_MAX][2 * DP];                 \
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;           \
  const int ws = blockIdx.y, b = blockIdx.x;                         \
  WLane L;                                                           \
  L.m = lane / KQ;                                                   \
  L.kq = lane - L.m * KQ;                                            \
  L.o = ws * DP + L.m;                                               \
  L.oi = (a.S + ws) * DP + L.m;                                      \
  const long set = 2L * a.S * DP, mat = 2L * DP * DP;                \
  const int start = b * a.L, end = min(a.N, start + a.L);            \
  const int nsub = (end - start + SUB16 - 1) / SUB16;                \
  const long sb0 = start / SUB16;                                    \
  T(*x2)[2 * DP] = xs[q];                                            \
  int cur = 0;

template <typename T, int DP> __global__ __launch_bounds__(64 * WSPLIT_MAX) void k_wF3s(SweepArgs<T> a) {
  WS_SETUP
  // ---- sub-block starts (wavefront 0)
  if (q == 0) {
    const T *ck = a.ckpt + (long)b * set;
    T xr = ck[L.o], xi = ck[L.oi];
    w_put(xb[0], L.m, DP, xr, xi);
    w_put(x2[0], L.m, DP, xr, xi);
    wave_lds_fence();
    auto eptr = [&](int i) -> const T * { return a.Es + (sb0 + i) * mat; };
    auto dummy = [&](int) -> const T * { return ck; };
    w_pipeline<T, DP>(L, nsub - 1, eptr, dummy, [&](int i, const T (&r)[2 * KC], T, T) {
      T sr, si;
      w_dot<T, DP>(L, r, x2[cur], sr, si);
      xr += sr;
      xi += si;
      w_put(x2[cur ^ 1], L.m, DP, xr, xi);
      w_put(xb[i + 1], L.m, DP, xr, xi);
      cur ^= 1;
      wave_lds_fence();
    });
  }
  __syncthreads();
  // ---- replay of sub-block q, then its partial penalty costate
  if (q < nsub) {
    const int a0 = start + q * SUB16, e0 = min(end, a0 + SUB16);
    T xr = xb[q][L.m], xi = xb[q][DP + L.m];
    cur = 0;
    w_put(x2[0], L.m, DP, xr, xi);
    a.psi_buf[(long)a0 * set + L.o] = xr;
    a.psi_buf[(long)a0 * set + L.oi] = xi;
    wave_lds_fence();
    auto fptr = [&](int i) -> const T * { return a.D + (a0 + i) * mat; };
    auto dummy = [&](int) -> const T * { return a.psi0; };
    w_pipeline<T, DP>(L, e0 - a0, fptr, dummy, [&](int i, const T (&r)[2 * KC], T, T) {
      T sr, si;
      w_dot<T, DP>(L, r, x2[cur], sr, si);
      xr += sr;
      xi += si;
      w_put(x2[cur ^ 1], L.m, DP, xr, xi);
      const int j = a0 + i;
      if (j + 1 < e0 || j + 1 == a.N) {  // wave-uniform
        a.psi_buf[(long)(j + 1) * set + L.o] = xr;
        a.psi_buf[(long)(j + 1) * set + L.oi] = xi;
      }
      cur ^= 1;
      wave_lds_fence();
    });
    if (a.pw) {  // uniform
      __threadfence_block();
      const T wgt = a.pw[L.m];
      T mr = (T)0, mi = (T)0;
      w_put(x2[cur], L.m, DP, mr, mi);
      wave_lds_fence();
      auto bptr = [&](int i) -> const T * { return a.Dh + (e0 - 1 - i) * mat; };
      auto pptr = [&](int i) -> const T * { return a.psi_buf + (long)(e0 - 1 - i) * set; };
      w_pipeline<T, DP>(L, e0 - a0, bptr, pptr, [&](int i, const T (&r)[2 * KC], T pr, T pi) {
        const int j = e0 - 1 - i;
        T sr, si;
        w_dot<T, DP>(L, r, x2[cur], sr, si);
        mr += sr + (j >= 1 ? wgt * pr : (T)0);
        mi += si + (j >= 1 ? wgt * pi : (T)0);
        w_put(x2[cur ^ 1], L.m, DP, mr, mi);
        cur ^= 1;
        wave_lds_fence();
      });
      T *nu = a.nu + (sb0 + q) * set;
      nu[L.o] = mr;
      nu[L.oi] = mi;
    }
  }
  if (!a.pw) return;  // uniform
  __threadfence_block();
  __syncthreads();
  // ---- the block's penalty costate from the sub-blocks' (wavefront 0)
  if (q == 0) {
    const T *nl = a.nu + (sb0 + nsub - 1) * set;
    T mr = nl[L.o], mi = nl[L.oi];
    cur = 0;
    w_put(x2[0], L.m, DP, mr, mi);
    wave_lds_fence();
    auto hptr = [&](int i) -> const T * { return a.Ehs + (sb0 + nsub - 2 - i) * mat; };
    auto nptr = [&](int i) -> const T * { return a.nu + (sb0 + nsub - 2 - i) * set; };
    w_pipeline<T, DP>(L, nsub - 1, hptr, nptr, [&](int, const T (&r)[2 * KC], T nr, T ni) {
      T sr, si;
      w_dot<T, DP>(L, r, x2[cur], sr, si);
      mr += sr + nr;
      mi += si + ni;
      w_put(x2[cur ^ 1], L.m, DP, mr, mi);
      cur ^= 1;
      wave_lds_fence();
    });
    T *mu = a.mu + (long)b * set;
    mu[L.o] = mr;
    mu[L.oi] = mi;
  }
}

template <typename T, int DP> __global__ __launch_bounds__(64 * WSPLIT_MAX) void k_wB3s(SweepArgs<T> a) {
  WS_SETUP
  const bool has_nu = a.pw != nullptr;
  // ---- costates at the sub-block ends (wavefront 0), xb[q] = lambda at the
  // end of sub-block q
  if (q == 0) {
    const T *c = a.lam_ckpt + (long)(b + 1) * set;
    T xr = c[L.o], xi = c[L.oi];
    w_put(xb[nsub - 1], L.m, DP, xr, xi);
    w_put(x2[0], L.m, DP, xr, xi);
    wave_lds_fence();
    auto hptr = [&](int i) -> const T * { return a.Ehs + (sb0 + nsub - 1 - i) * mat; };
    auto nptr = [&](int i) -> const T * {
      return has_nu ? a.nu + (sb0 + nsub - 1 - i) * set : a.psi0;  // psi0: finite placeholder
    };
    w_pipeline<T, DP>(L, nsub - 1, hptr, nptr, [&](int i, const T (&r)[2 * KC], T nr, T ni) {
      T sr, si;
      w_dot<T, DP>(L, r, x2[cur], sr, si);
      xr += sr + (has_nu ? nr : (T)0);
      xi += si + (has_nu ? ni : (T)0);
      w_put(x2[cur ^ 1], L.m, DP, xr, xi);
      w_put(xb[nsub - 2 - i], L.m, DP, xr, xi);
      cur ^= 1;
      wave_lds_fence();
    });
  }
  __syncthreads();
  if (q >= nsub) return;
  // ---- sub-block q backwards: lam_buf[j] = lambda_{j+1}
  const int a0 = start + q * SUB16, e0 = min(end, a0 + SUB16);
  T xr = xb[q][L.m], xi = xb[q][DP + L.m];
  cur = 0;
  w_put(x2[0], L.m, DP, xr, xi);
  wave_lds_fence();
  const T wgt = a.pw ? a.pw[L.m] : (T)0;
  auto dptr = [&](int i) -> const T * { return a.Dh + (e0 - 1 - i) * mat; };
  auto pptr = [&](int i) -> const T * { return a.psi_buf + (long)(e0 - 1 - i) * set; };
  w_pipeline<T, DP>(L, e0 - 1 - a0, dptr, pptr, [&](int i, const T (&r)[2 * KC], T pr, T pi) {
    const int j = e0 - 1 - i;
    T *lb = a.lam_buf + (long)j * set;
    lb[L.o] = xr;  // lambda_{j+1}
    lb[L.oi] = xi;
    T sr, si;
    w_dot<T, DP>(L, r, x2[cur], sr, si);
    xr += sr + (j >= 1 ? wgt * pr : (T)0);
    xi += si + (j >= 1 ? wgt * pi : (T)0);
    w_put(x2[cur ^ 1], L.m, DP, xr, xi);
    cur ^= 1;
    wave_lds_fence();
  });
  T *lb = a.lam_buf + (long)a0 * set;
  lb[L.o] = xr;
  lb[L.oi] = xi;
}

template <typename T> bool wave_sweep_ok(int dp, int S) {
  return (dp == 16 && S * dp <= 64) || (dp == 32 && S * dp <= 64);
}

template <typename T, int DP> hipError_t w_launch(int which, const SweepArgs<T> &a, hipStream_t st) {
  const unsigned S = (unsigned)a.S;
  switch (which) {
    case 0: hipLaunchKernelGGL((k_wF2<T, DP>), dim3(1, S), dim3(64), 0, st, a); break;
    case 1:
      if (DP == 16 && a.Es)
        hipLaunchKernelGGL((k_wF3s<T, DP>), dim3(a.nb, S), dim3(64 * (a.L / SUB16)), 0, st, a);
      else
        hipLaunchKernelGGL((k_wF3<T, DP>), dim3(a.nb, S), dim3(64), 0, st, a);
      break;
    case 2:
      if (a.fuse_cost)
        hipLaunchKernelGGL((k_wB2<T, DP>), dim3(a.S + a.npart), dim3(64), 0, st, a);
      else
        hipLaunchKernelGGL((k_wB2<T, DP>), dim3(1, S), dim3(64), 0, st, a);
      break;
    default:
      if (DP == 16 && a.Es)
        hipLaunchKernelGGL((k_wB3s<T, DP>), dim3(a.nb, S), dim3(64 * (a.L / SUB16)), 0, st, a);
      else
        hipLaunchKernelGGL((k_wB3<T, DP>), dim3(a.nb, S), dim3(64), 0, st, a);
      break;
  }
  return hipGetLastError();
}

template <typename T> hipError_t launch_wave_sweep(int which, const SweepArgs<T> &a, hipStream_t st) {
  if (!a.Dh || !a.Eh) return hipErrorInvalidValue;
  if (a.Es && (a.dp != 16 || !a.Ehs || a.L % SUB16 || a.L > WSPLIT_MAX * SUB16 ||
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
