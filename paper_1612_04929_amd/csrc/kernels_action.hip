// State-mode action form (Sec. IV: U_j |psi> as a series of matrix-vector
// products; no step propagator is formed).  The approximant is the one of
// Sec. III, T_p(X_j)^(2^n) with X_j = -i (dt / 2^n) H_j, applied to each
// propagated column by Horner's rule, w <- v + X_j w / k for k = p .. 1,
// 2^n times per step: p 2^n products with H_j per step and column.
//
// H_j is held in an ELL layout over the union of the nonzero patterns of
// H_0 .. H_M: K slots per row (padded with zero values), slot (kk, r) at
// column ecol[kk dp + r].  The per-step values hv_j = H_0 + sum_k u_kj H_k
// are formed for every step up front (k_act_values, parallel over steps);
// the sequential chains keep the values of their rows in registers, with
// the next step's prefetched, and the vector being multiplied in LDS.
//
//   k_act_fwd   one workgroup per column: psi_{j+1} = T_p(X_j)^(2^n) psi_j,
//               and (gradient calls) every product's input vector a_q
//   k_act_bwd   one workgroup per column: the reverse pass of the same
//               products, lambda_j = (T_p(X_j)^(2^n))^H lambda_{j+1} +
//               pw o psi_j + src_j (j >= 1), lambda_{j+1} to lam_buf[j],
//               and every product's output cotangent ybar_q
//   k_act_grad  one workgroup per (step, column): the exact derivative of
//               the step's action for every control at once,
//               sum_q Im(ybar_q^H H_k a_q) -- the Xbar_j = sum_q ybar_q a_q^H
//               of the reverse pass sampled at the controls' nonzeros --
//               into per-column partial sums
#include <type_traits>

#include "qoc_device.h"
#include "qoc_kernels.h"

namespace qoc {

// ------------------------------------------------------------------ values
template <typename T> __global__ __launch_bounds__(256) void k_act_values(ActValArgs<T> a) {
  const long slots = (long)a.K * a.dp;
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  if (q >= slots) return;
  const long kk = q / a.dp, r = q - kk * a.dp;
  const long mstride = 2 * slots;  // one matrix's planes
  for (long j = blockIdx.y; j < a.N; j += gridDim.y) {
    double re = a.hm[kk * 2 * a.dp + r], im = a.hm[kk * 2 * a.dp + a.dp + r];
    for (int m = 1; m <= a.M; ++m) {
      const double c = a.u[(long)(m - 1) * a.N + j];
      const double *hm = a.hm + m * mstride + kk * 2 * a.dp;
      re += c * hm[r];
      im += c * hm[a.dp + r];
    }
    T *o = a.hv + (j * a.K + kk) * 2 * a.dp;
    o[r] = (T)re;
    o[a.dp + r] = (T)im;
  }
}

template <typename T> hipError_t launch_act_values(const ActValArgs<T> &a, hipStream_t st) {
  const long slots = (long)a.K * a.dp;
  const unsigned gx = (unsigned)((slots + 255) / 256);
  const unsigned gy = (unsigned)std::max(1, std::min(a.N, 4096));
  hipLaunchKernelGGL(k_act_values<T>, dim3(gx, gy), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ chains
// Row-owner layout: thread t owns rows t + i * blockDim (i < RPT) and keeps
// their K slot values and columns in registers.  The vector being
// multiplied sits in LDS as interleaved complex pairs (one 8- or 16-byte
// read per slot).
template <typename T> struct Cplx;
template <> struct Cplx<float> { typedef float2 type; };
template <> struct Cplx<double> { typedef double2 type; };
template <typename T, int K, int RPT, int TPR> struct ActRows {
  // TPR consecutive lanes share a row, each holding K / TPR of its slots;
  // thread t's rows are t / TPR + i nt / TPR
  static constexpr int KT = K / TPR;
  int col[RPT][KT];
  T hr[RPT][KT], hi[RPT][KT];   // values of the current step
  T nr[RPT][KT], ni[RPT][KT];   // prefetched values of the next step
  int h, rb, rs;
  __device__ __forceinline__ void init(int t, int nt) {
    h = t % TPR;
    rb = t / TPR;
    rs = nt / TPR;
  }
  __device__ __forceinline__ int row(int i) const { return rb + i * rs; }
  __device__ __forceinline__ bool lead() const { return h == 0; }
  __device__ __forceinline__ void load_cols(const ActionArgs<T> &a) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = row(i);
#pragma unroll
      for (int m = 0; m < KT; ++m) {
        const int kk = h + TPR * m;
        col[i][m] = r < a.dp ? a.ecol[kk * a.dp + r] : 0;
      }
    }
  }
  __device__ __forceinline__ void prefetch(const ActionArgs<T> &a, long j) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = row(i);
#pragma unroll
      for (int m = 0; m < KT; ++m) {
        const int kk = h + TPR * m;
        const T *hp = a.hv + (j * K + kk) * 2 * a.dp;
        nr[i][m] = r < a.dp ? hp[r] : (T)0;
        ni[i][m] = r < a.dp ? hp[a.dp + r] : (T)0;
      }
    }
  }
  __device__ __forceinline__ void advance() {
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
      for (int m = 0; m < KT; ++m) {
        hr[i][m] = nr[i][m];
        hi[i][m] = ni[i][m];
      }
  }
  // (H_j x)_r for the thread's rows, x interleaved complex in LDS; the
  // TPR lanes of a row add their partial sums (both hold the result)
  __device__ __forceinline__ void mv(const typename Cplx<T>::type *x, T (&ar)[RPT],
                                     T (&ai)[RPT]) const {
    typename Cplx<T>::type v[RPT][KT];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
      for (int m = 0; m < KT; ++m) v[i][m] = x[col[i][m]];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      // two partial sums per component (even / odd slots): half the
      // dependent chain of a row's multiply-adds
      T sr[2] = {0, 0}, si[2] = {0, 0};
#pragma unroll
      for (int m = 0; m < KT; ++m) {
        sr[m & 1] += hr[i][m] * v[i][m].x - hi[i][m] * v[i][m].y;
        si[m & 1] += hr[i][m] * v[i][m].y + hi[i][m] * v[i][m].x;
      }
      T r0 = sr[0] + sr[1], i0 = si[0] + si[1];
#pragma unroll
      for (int o = 1; o < TPR; o <<= 1) {
        r0 += __shfl_xor(r0, o, 64);
        i0 += __shfl_xor(i0, o, 64);
      }
      ar[i] = r0;
      ai[i] = i0;
    }
  }
};

template <typename T>
__device__ __forceinline__ long act_off(const ActionArgs<T> &a, long j, int s, int q) {
  return ((j * a.S + s) * (long)a.P + q) * 2 * a.dp;
}

template <typename T, int K, int RPT, int TPR>
__global__ __launch_bounds__(512 * TPR) void k_act_fwd(ActionArgs<T> a) {
  typedef typename Cplx<T>::type C2;
  extern __shared__ unsigned char shraw[];
  C2 *buf = (C2 *)shraw;  // [2 buffers][dp]
  const int s = blockIdx.x, t = threadIdx.x, nt = blockDim.x, dp = a.dp, S = a.S;
  const long set = 2L * S * dp;
  ActRows<T, K, RPT, TPR> R;
  R.init(t, nt);
  R.load_cols(a);
  R.prefetch(a, 0);
  T vr[RPT], vi[RPT], wr[RPT], wi[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = R.row(i);
    vr[i] = r < dp ? a.psi0[(long)s * dp + r] : (T)0;
    vi[i] = r < dp ? a.psi0[(long)(S + s) * dp + r] : (T)0;
    if (r < dp && R.lead()) {
      a.psi_buf[(long)s * dp + r] = vr[i];
      a.psi_buf[(long)(S + s) * dp + r] = vi[i];
    }
  }
  int cur = 0;
  const int subs = 1 << a.n;
  for (long j = 0; j < a.N; ++j) {
    R.advance();
    if (j + 1 < a.N) R.prefetch(a, j + 1);
    for (int sub = 0; sub < subs; ++sub) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        wr[i] = vr[i];
        wi[i] = vi[i];
      }
      for (int k = a.p; k >= 1; --k) {
        C2 *x = buf + cur * dp;
        const long off = a.A ? act_off(a, j, s, sub * a.p + (a.p - k)) : 0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int r = R.row(i);
          if (r < dp && R.lead()) {
            C2 v;
            v.x = wr[i];
            v.y = wi[i];
            x[r] = v;
            if (a.A) {
              a.A[off + r] = wr[i];
              a.A[off + dp + r] = wi[i];
            }
          }
        }
        lds_barrier();
        T ar[RPT], ai[RPT];
        R.mv(x, ar, ai);
        const T c = a.coef[k];  // s / k; y = -i s (H w): w <- v + y / k
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          wr[i] = vr[i] + c * ai[i];
          wi[i] = vi[i] - c * ar[i];
        }
        cur ^= 1;
      }
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        vr[i] = wr[i];
        vi[i] = wi[i];
      }
    }
    T *o = a.psi_buf + (j + 1) * set;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = R.row(i);
      if (r < dp && R.lead()) {
        o[(long)s * dp + r] = vr[i];
        o[(long)(S + s) * dp + r] = vi[i];
      }
    }
  }
}

template <typename T, int K, int RPT, int TPR>
__global__ __launch_bounds__(512 * TPR) void k_act_bwd(ActionArgs<T> a) {
  typedef typename Cplx<T>::type C2;
  extern __shared__ unsigned char shraw[];
  C2 *buf = (C2 *)shraw;
  const int s = blockIdx.x, t = threadIdx.x, nt = blockDim.x, dp = a.dp, S = a.S;
  const long set = 2L * S * dp;
  ActRows<T, K, RPT, TPR> R;
  R.init(t, nt);
  R.load_cols(a);
  R.prefetch(a, a.N - 1);
  T lr[RPT], li[RPT], br[RPT], bi[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = R.row(i);
    lr[i] = r < dp ? a.lamN[(long)s * dp + r] : (T)0;
    li[i] = r < dp ? a.lamN[(long)(S + s) * dp + r] : (T)0;
  }
  int cur = 0;
  const int subs = 1 << a.n;
  for (long j = a.N - 1; j >= 0; --j) {
    R.advance();
    if (j >= 1) R.prefetch(a, j - 1);
    // the step's own costate source (pw o psi_j + src_j), loaded ahead of use
    T qr[RPT], qi[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = R.row(i);
      qr[i] = 0;
      qi[i] = 0;
      if (j >= 1 && r < dp) {
        if (a.pw) {
          const T *ps = a.psi_buf + j * set;
          qr[i] = a.pw[r] * ps[(long)s * dp + r];
          qi[i] = a.pw[r] * ps[(long)(S + s) * dp + r];
        }
        if (a.src) {
          const T *sr = a.src + j * set;
          qr[i] += sr[(long)s * dp + r];
          qi[i] += sr[(long)(S + s) * dp + r];
        }
      }
    }
    T *lb = a.lam_buf + j * set;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = R.row(i);
      if (r < dp && R.lead()) {
        lb[(long)s * dp + r] = lr[i];
        lb[(long)(S + s) * dp + r] = li[i];
      }
    }
    for (int sub = subs - 1; sub >= 0; --sub) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        br[i] = 0;
        bi[i] = 0;
      }
      for (int k = 1; k <= a.p; ++k) {
        // w = v + y / k: vbar += wbar, ybar = wbar / k; y = X a: abar = X^H ybar
        C2 *x = buf + cur * dp;
        const T ik = a.inv[k];
        const long off = a.Ybar ? act_off(a, j, s, sub * a.p + (a.p - k)) : 0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int r = R.row(i);
          br[i] += lr[i];
          bi[i] += li[i];
          const T yr = lr[i] * ik, yi = li[i] * ik;
          if (r < dp && R.lead()) {
            C2 v;
            v.x = yr;
            v.y = yi;
            x[r] = v;
            if (a.Ybar) {
              a.Ybar[off + r] = yr;
              a.Ybar[off + dp + r] = yi;
            }
          }
        }
        lds_barrier();
        T ar[RPT], ai[RPT];
        R.mv(x, ar, ai);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {  // X^H = i s H
          lr[i] = -a.s * ai[i];
          li[i] = a.s * ar[i];
        }
        cur ^= 1;
      }
#pragma unroll
      for (int i = 0; i < RPT; ++i) {  // the substep's input cotangent
        lr[i] += br[i];
        li[i] += bi[i];
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      lr[i] += qr[i];
      li[i] += qi[i];
    }
  }
}

template <typename T, int K, int RPT, int TPR = 1>
hipError_t act_chain(int which, const ActionArgs<T> &a, hipStream_t st) {
  const int rows = (a.dp + RPT - 1) / RPT;
  const int nt = std::max(64, (TPR * rows + 63) / 64 * 64);
  const size_t sh = 4 * (size_t)a.dp * sizeof(T);  // two buffers of dp complex
  if (which == 0)
    hipLaunchKernelGGL((k_act_fwd<T, K, RPT, TPR>), dim3(a.S), dim3(nt), sh, st, a);
  else
    hipLaunchKernelGGL((k_act_bwd<T, K, RPT, TPR>), dim3(a.S), dim3(nt), sh, st, a);
  return hipGetLastError();
}

template <typename T> bool act_shape_ok(int dp, int K) {
  if (dp > 1024 || !(K == 4 || K == 8 || K == 12 || K == 16 || K == 24 || K == 32)) return false;
  const int rpt = dp <= 512 ? 1 : 2;
  return (long)K * rpt * (long)(sizeof(T) / 4) <= 32;
}

template <typename T> hipError_t launch_act_chain(int which, const ActionArgs<T> &a,
                                                  hipStream_t st) {
  if (!act_shape_ok<T>(a.dp, a.K)) return hipErrorInvalidValue;
  const bool two = a.dp > 512;
  if constexpr (std::is_same<T, float>::value) {
    // lanes per row: the most that keep a padded d <= 32 within one
    // wavefront (more lanes per row shorten each product's dependent chain;
    // beyond one wavefront the wider barrier costs more, measured at
    // padded d 512: 16.2 against 14.0 ms per call with two lanes)
    const int tpr = (a.dp <= 16 && a.K >= 8) ? 4 : (a.dp <= 32 ? 2 : 1);
    switch (a.K) {
      case 4:
        if (tpr >= 2) return act_chain<T, 4, 1, 2>(which, a, st);
        return two ? act_chain<T, 4, 2>(which, a, st) : act_chain<T, 4, 1>(which, a, st);
      case 8:
        if (tpr == 4) return act_chain<T, 8, 1, 4>(which, a, st);
        if (tpr == 2) return act_chain<T, 8, 1, 2>(which, a, st);
        return two ? act_chain<T, 8, 2>(which, a, st) : act_chain<T, 8, 1>(which, a, st);
      case 12:
        if (tpr == 4) return act_chain<T, 12, 1, 4>(which, a, st);
        if (tpr == 2) return act_chain<T, 12, 1, 2>(which, a, st);
        return two ? act_chain<T, 12, 2>(which, a, st) : act_chain<T, 12, 1>(which, a, st);
      case 16:
        if (tpr == 4) return act_chain<T, 16, 1, 4>(which, a, st);
        if (tpr == 2) return act_chain<T, 16, 1, 2>(which, a, st);
        return two ? act_chain<T, 16, 2>(which, a, st) : act_chain<T, 16, 1>(which, a, st);
      case 24:
        if (tpr >= 2) return act_chain<T, 24, 1, 2>(which, a, st);
        return act_chain<T, 24, 1>(which, a, st);
      case 32:
        if (tpr >= 2) return act_chain<T, 32, 1, 2>(which, a, st);
        return act_chain<T, 32, 1>(which, a, st);
    }
  } else {
    switch (a.K) {
      case 4: return two ? act_chain<T, 4, 2>(which, a, st) : act_chain<T, 4, 1>(which, a, st);
      case 8: return two ? act_chain<T, 8, 2>(which, a, st) : act_chain<T, 8, 1>(which, a, st);
      case 12: return act_chain<T, 12, 1>(which, a, st);
      case 16: return act_chain<T, 16, 1>(which, a, st);
    }
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ gradient
// One workgroup per (step j, column s): g_e = sum_q conj(ybar_q[row_e])
// a_q[col_e] at every entry e of the union of the controls' patterns (LDS,
// each entry owned by one thread), then per control k the fixed-order sum
// sum_{e in H_k} Im(H_k[e] g_e) (FP64) into part[(j S + s) M + k].
template <typename T> __global__ __launch_bounds__(256) void k_act_grad(ActGradArgs<T> a) {
  extern __shared__ unsigned char shraw[];
  T *vec = (T *)shraw;                 // a_q (re, im), ybar_q (re, im): 4 dp
  T *gre = vec + 4 * a.dp, *gim = gre + a.nent;
  __shared__ double red[4];
  const int t = threadIdx.x, dp = a.dp;
  const long js = blockIdx.x;
  const long j = js / a.S;
  const int s = (int)(js - j * a.S);
  for (int e = t; e < a.nent; e += 256) {
    gre[e] = 0;
    gim[e] = 0;
  }
  for (int q = 0; q < a.P; ++q) {
    const T *av = a.A + j * a.aj + s * a.as + q * a.aq;
    const T *yv = a.Y + j * a.yj + s * a.ys + q * a.yq;
    __syncthreads();
    for (int r = t; r < dp; r += 256) {
      vec[r] = av[r];
      vec[dp + r] = av[a.aplane + r];
      vec[2 * dp + r] = yv[r];
      vec[3 * dp + r] = yv[a.yplane + r];
    }
    __syncthreads();
    for (int e = t; e < a.nent; e += 256) {
      const int rr = a.erow[e], cc = a.ecol[e];
      const T xr = vec[cc], xi = vec[dp + cc];
      const T yr = vec[2 * dp + rr], yi = vec[3 * dp + rr];
      gre[e] += yr * xr + yi * xi;  // conj(y) x
      gim[e] += yr * xi - yi * xr;
    }
  }
  __syncthreads();
  for (int k = 0; k < a.M; ++k) {
    double acc = 0.0;
    for (int i = a.cptr[k] + t; i < a.cptr[k + 1]; i += 256) {
      const int e = a.cent[i];
      const double hr = (double)a.cval[i], hi = (double)a.cval[a.npairs + i];
      acc += hr * (double)gim[e] + hi * (double)gre[e];  // Im(h g)
    }
    acc = block_sum(acc, red);
    if (t == 0) a.part[js * a.M + k] = acc;
  }
}

template <typename T> hipError_t launch_act_grad(const ActGradArgs<T> &a, hipStream_t st) {
  const size_t sh = (4 * (size_t)a.dp + 2 * (size_t)a.nent) * sizeof(T);
  const long blocks = (long)a.N * a.S;
  if (blocks <= 0 || a.M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_act_grad<T>, dim3((unsigned)blocks), dim3(256), sh, st, a);
  return hipGetLastError();
}

template <typename T> long act_grad_lds(int dp, long nent) {
  return (4L * dp + 2L * nent) * (long)sizeof(T);
}

#define QOC_INST(T)                                                                      \
  template hipError_t launch_act_values<T>(const ActValArgs<T> &, hipStream_t);          \
  template hipError_t launch_act_chain<T>(int, const ActionArgs<T> &, hipStream_t);      \
  template hipError_t launch_act_grad<T>(const ActGradArgs<T> &, hipStream_t);           \
  template bool act_shape_ok<T>(int, int);                                               \
  template long act_grad_lds<T>(int, long);
QOC_INST(float)
QOC_INST(double)
#undef QOC_INST

}  // namespace qoc
