// Forward and costate sweeps as a blocked two-level scan.
//
// The product of propagators (Sec. II, eqs. 2-4) is inherently sequential
// over time steps.  Instead of N dependent matrix-vector steps on one
// compute unit, the steps are cut into nb blocks of L (a power of two near
// sqrt(N)):
//   F2  sequential over blocks: psi_{(b+1)L} = (I + E_b) psi_{bL} with the
//       block product E_b = U_{bL+L-1} ... U_{bL} - I (state checkpoints);
//   F3  parallel over blocks and columns: replay psi_j inside each block
//       from its checkpoint, and the block-local penalty costate mu_b
//       (the per-step penalties c_j of Table I, C5, are then reduced in
//       parallel over all steps by k_cost);
//   cost: fidelity overlap in FP64 and the final costate lambda_N;
//   B2  sequential over blocks: lambda_{bL} = (I + E_b)^H lambda_{(b+1)L} + mu_b;
//   B3  parallel over blocks and columns: lambda_{j+1} for every step, the
//       cotangent partner of psi_j for the per-step derivative.
// Columns (states) propagate independently, so every sweep runs one
// workgroup per column (F2, B2) or per (block, column) (F3, B3).
// All updates are in D-form: y = x + D x.
#include <algorithm>

#include "qoc_device.h"
#include "qoc_kernels.h"
#include "qoc_cost.h"
#include "qoc_total.h"

namespace qoc {

// 16-byte vector of T (4 floats or 2 doubles) for wide global loads.
template <typename T> struct Vec16;
template <> struct Vec16<float> {
  typedef float4 type;
  static constexpr int n = 4;
};
template <> struct Vec16<double> {
  typedef double2 type;
  static constexpr int n = 2;
};
template <typename T> __device__ __forceinline__ T vget(const typename Vec16<T>::type &v, int q);
template <> __device__ __forceinline__ float vget<float>(const float4 &v, int q) {
  return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}
template <> __device__ __forceinline__ double vget<double>(const double2 &v, int q) {
  return q == 0 ? v.x : v.y;
}

// y = x + D x, D row-major planar (dp x dp) in global memory, x and y in
// LDS.  Each wavefront takes 8 output rows at a time with the lanes along
// the rows in 16-byte vectors (coalesced, 8 rows x 2 planes of loads in
// flight), then reduces the 16 partial sums across the wavefront.  dp is a
// multiple of 16; the matrices are 16-byte aligned.
template <typename T>
__device__ __forceinline__ void mv_plus(const T *__restrict__ Dr, const T *__restrict__ Di,
                                        int dp, const T *xr, const T *xi, T *yr, T *yi) {
  typedef typename Vec16<T>::type V;
  constexpr int VN = Vec16<T>::n;
  constexpr int RB = 8;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = 4;
  const int nv = dp / VN;
  for (int m0 = w * RB; m0 < dp; m0 += nw * RB) {
    T sr[RB], si[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      sr[q] = 0;
      si[q] = 0;
    }
    for (int kv = lane; kv < nv; kv += 64) {
      const int k = kv * VN;
      V dr[RB], di[RB];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        dr[q] = *reinterpret_cast<const V *>(Dr + (long)(m0 + q) * dp + k);
        di[q] = *reinterpret_cast<const V *>(Di + (long)(m0 + q) * dp + k);
      }
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        const T a = xr[k + e], b = xi[k + e];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const T vr = vget<T>(dr[q], e), vi = vget<T>(di[q], e);
          sr[q] += vr * a - vi * b;
          si[q] += vr * b + vi * a;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      sr[q] = wave_sum(sr[q]);
      si[q] = wave_sum(si[q]);
    }
    if (lane < RB) {
      T vr = 0, vi = 0;
#pragma unroll
      for (int q = 0; q < RB; ++q)
        if (q == lane) {
          vr = sr[q];
          vi = si[q];
        }
      yr[m0 + lane] = xr[m0 + lane] + vr;
      yi[m0 + lane] = xi[m0 + lane] + vi;
    }
  }
}

// y = x + D^H x (+ add).  Thread t owns the VN consecutive output rows of
// column group t % G (G = dp / VN) and the inner-dimension slice t / G of
// the 256 / G slices; each reads 16-byte vectors of D's rows (coalesced
// across the column groups).  Slice partial sums meet in LDS scratch `red`
// (2 * 256 * VN elements) with one barrier.
template <typename T>
__device__ __forceinline__ void mv_plus_adj(const T *__restrict__ Dr, const T *__restrict__ Di,
                                            int dp, const T *xr, const T *xi, T *yr, T *yi,
                                            const T *addr, const T *addi, T *red) {
  typedef typename Vec16<T>::type V;
  constexpr int VN = Vec16<T>::n;
  const int t = threadIdx.x;
  const int G = dp / VN;                       // column groups
  const int SL = G >= 256 ? 1 : 256 / G;       // inner-dimension slices
  const int kper = (dp + SL - 1) / SL;
  for (int g0 = 0; g0 < G; g0 += 256 / SL) {
    const int cg = g0 + t % (256 / SL), sl = t / (256 / SL);
    T sr[VN], si[VN];
#pragma unroll
    for (int e = 0; e < VN; ++e) {
      sr[e] = 0;
      si[e] = 0;
    }
    if (cg < G && sl < SL) {
      const int k0 = sl * kper, k1 = min(dp, k0 + kper);
      for (int k = k0; k < k1; ++k) {
        const V dr = *reinterpret_cast<const V *>(Dr + (long)k * dp + cg * VN);
        const V di = *reinterpret_cast<const V *>(Di + (long)k * dp + cg * VN);
        const T a = xr[k], b = xi[k];
#pragma unroll
        for (int e = 0; e < VN; ++e) {
          const T vr = vget<T>(dr, e), vi = -vget<T>(di, e);
          sr[e] += vr * a - vi * b;
          si[e] += vr * b + vi * a;
        }
      }
    }
    if (SL > 1) {
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        red[(2 * t) * VN + e] = sr[e];
        red[(2 * t + 1) * VN + e] = si[e];
      }
      __syncthreads();
      if (sl == 0 && cg < G) {
        for (int s2 = 1; s2 < SL; ++s2) {
          const int tt = t + s2 * (256 / SL);
#pragma unroll
          for (int e = 0; e < VN; ++e) {
            sr[e] += red[(2 * tt) * VN + e];
            si[e] += red[(2 * tt + 1) * VN + e];
          }
        }
      }
      __syncthreads();
    }
    if (sl == 0 && cg < G) {
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        const int m = cg * VN + e;
        T vr = xr[m] + sr[e], vi = xi[m] + si[e];
        if (addr) {
          vr += addr[m];
          vi += addi[m];
        }
        yr[m] = vr;
        yi[m] = vi;
      }
    }
  }
}

template <typename T> __device__ __forceinline__ const T *set_re(const T *base, int S, int dp, int s) {
  return base + (long)s * dp;
}
template <typename T> __device__ __forceinline__ const T *set_im(const T *base, int S, int dp, int s) {
  return base + (long)S * dp + (long)s * dp;
}
template <typename T> __device__ __forceinline__ T *set_rew(T *base, int S, int dp, int s) {
  return base + (long)s * dp;
}
template <typename T> __device__ __forceinline__ T *set_imw(T *base, int S, int dp, int s) {
  return base + (long)S * dp + (long)s * dp;
}

// ------------------------------------------------------------------ F2
template <typename T> __global__ __launch_bounds__(256) void k_fwd_blocks(SweepArgs<T> a) {
  extern __shared__ unsigned char shraw[];
  T *buf = (T *)shraw;
  const int dp = a.dp, S = a.S, s = blockIdx.x;
  const long set = 2L * S * dp, mat = 2L * dp * dp;
  T *xr = buf, *xi = buf + dp, *yr = buf + 2 * dp, *yi = buf + 3 * dp;
  for (int m = threadIdx.x; m < dp; m += blockDim.x) {
    xr[m] = set_re(a.psi0, S, dp, s)[m];
    xi[m] = set_im(a.psi0, S, dp, s)[m];
    set_rew(a.ckpt, S, dp, s)[m] = xr[m];
    set_imw(a.ckpt, S, dp, s)[m] = xi[m];
  }
  __syncthreads();
  for (int b = 0; b < a.nb; ++b) {
    const T *E = a.E + (long)b * mat;
    mv_plus(E, E + (long)dp * dp, dp, xr, xi, yr, yi);
    __syncthreads();
    T *c = a.ckpt + (long)(b + 1) * set;
    for (int m = threadIdx.x; m < dp; m += blockDim.x) {
      set_rew(c, S, dp, s)[m] = yr[m];
      set_imw(c, S, dp, s)[m] = yi[m];
    }
    T *tr = xr, *ti = xi;
    xr = yr; xi = yi; yr = tr; yi = ti;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ F3
template <typename T> __global__ __launch_bounds__(256) void k_fwd_replay(SweepArgs<T> a) {
  extern __shared__ unsigned char shraw[];
  T *buf = (T *)shraw;
  const int dp = a.dp, S = a.S;
  // (block, state) from the XCD-grouped 1-D grid (xcd_grid in the launch)
  const long lg_ = xcd_logical_block(blockIdx.x, gridDim.x);
  if (lg_ >= (long)a.nb * S) return;  // padding of the grid
  const int b = (int)(lg_ / S), s = (int)(lg_ - lg_ / S * S);
  const long set = 2L * S * dp, mat = 2L * dp * dp;
  const int start = b * a.L, end = min(a.N, start + a.L);
  T *xr = buf, *xi = buf + dp, *yr = buf + 2 * dp, *yi = buf + 3 * dp;
  const T *c = a.ckpt + (long)b * set;
  if (a.replay_mode != 2) {  // grid-uniform
  for (int m = threadIdx.x; m < dp; m += blockDim.x) {
    const T vr = set_re(c, S, dp, s)[m], vi = set_im(c, S, dp, s)[m];
    xr[m] = vr; xi[m] = vi;
    set_rew(a.psi_buf + (long)start * set, S, dp, s)[m] = vr;
    set_imw(a.psi_buf + (long)start * set, S, dp, s)[m] = vi;
  }
  __syncthreads();
  for (int j = start; j < end; ++j) {
    const T *D = a.D + (long)j * mat;
    mv_plus(D, D + (long)dp * dp, dp, xr, xi, yr, yi);
    __syncthreads();
    if ((j + 1 < end) || (j + 1 == a.N)) {
      for (int m = threadIdx.x; m < dp; m += blockDim.x) {
        set_rew(a.psi_buf + (long)(j + 1) * set, S, dp, s)[m] = yr[m];
        set_imw(a.psi_buf + (long)(j + 1) * set, S, dp, s)[m] = yi[m];
      }
    }
    T *tr = xr, *ti = xi;
    xr = yr; xi = yi; yr = tr; yi = ti;
    __syncthreads();
  }
  }
  if ((!a.pw && !a.src) || a.replay_mode == 1) return;  // block-uniform
  // block-local penalty costate from zero at the block end:
  // mu <- mu + D_j^H mu + pw o psi_j + src_j   (per-step terms only for j >= 1)
  T *mr = xr, *mi = xi, *nr = yr, *ni = yi;
  T *pr = buf + 4 * dp, *pi = buf + 5 * dp;
  for (int m = threadIdx.x; m < dp; m += blockDim.x) {
    mr[m] = 0;
    mi[m] = 0;
  }
  __syncthreads();
  for (int j = end - 1; j >= start; --j) {
    const T *ps = a.psi_buf + (long)j * set;
    for (int m = threadIdx.x; m < dp; m += blockDim.x) {
      const T wgt = (a.pw && j >= 1) ? a.pw[m] : (T)0;
      T vr = wgt * set_re(ps, S, dp, s)[m], vi = wgt * set_im(ps, S, dp, s)[m];
      if (a.src && j >= 1) {
        vr += set_re(a.src + (long)j * set, S, dp, s)[m];
        vi += set_im(a.src + (long)j * set, S, dp, s)[m];
      }
      pr[m] = vr;
      pi[m] = vi;
    }
    __syncthreads();
    const T *D = a.D + (long)j * mat;
    mv_plus_adj(D, D + (long)dp * dp, dp, mr, mi, nr, ni, pr, pi, buf + 6 * dp);
    __syncthreads();
    T *tr = mr, *ti = mi;
    mr = nr; mi = ni; nr = tr; ni = ti;
  }
  T *mu = a.mu + (long)b * set;
  for (int m = threadIdx.x; m < dp; m += blockDim.x) {
    set_rew(mu, S, dp, s)[m] = mr[m];
    set_imw(mu, S, dp, s)[m] = mi[m];
  }
}

// ------------------------------------------------------------------ cost
// FP64.  One launch (k_cost): its last workgroup computes the fidelity
// overlaps, F, C_fid and the final costate lambda_N (rounded to the chain
// precision) -- all the costate sweeps need -- while the other workgroups
// run the penalty pass below.  k_total: the weighted total cost from F and
// the per-workgroup partial sums of the penalty pass (penalties, |u|^2,
// variations) and the norm drift from its per-workgroup maxima, in a fixed
// order.
template <typename T> __device__ void lam_block(const SweepArgs<T> &a) {
  __shared__ double red[4];
  const int dp = a.dp, d = a.d, S = a.S, N = a.N;
  const long set = 2L * S * dp;
  const T *psiN = a.psi_buf + (long)N * set;
  double zr = 0.0, zi = 0.0, Finc = 0.0;
  for (int s = 0; s < S; ++s) {
    double pr = 0.0, pi = 0.0;
    for (int m = threadIdx.x; m < d; m += blockDim.x) {
      const double tr = a.psiT64[((long)s * d + m) * 2], ti = a.psiT64[((long)s * d + m) * 2 + 1];
      const double xr = (double)set_re(psiN, S, dp, s)[m], xi = (double)set_im(psiN, S, dp, s)[m];
      pr += tr * xr + ti * xi;  // conj(T) psi
      pi += tr * xi - ti * xr;
    }
    pr = block_sum(pr, red);
    pi = block_sum(pi, red);
    zr += pr;
    zi += pi;
    Finc += pr * pr + pi * pi;
    if (threadIdx.x == 0) {
      a.zinfo[3 + 2 * s] = pr;
      a.zinfo[4 + 2 * s] = pi;
    }
  }
  zr /= S;
  zi /= S;
  const double F = (a.fid_mode == 0) ? (zr * zr + zi * zi) : Finc / S;
  if (threadIdx.x == 0) {
    a.out[1] = 1.0 - F;
    a.zinfo[0] = zr;
    a.zinfo[1] = zi;
    a.zinfo[2] = F;
  }
  __syncthreads();
  // lambda_N^s = -a_fid coef_s T_s + pw o psi_N^s, coef = z/S or o_s/S
  T *lamN = a.lam_ckpt + (long)a.nb * set;
  for (int s = 0; s < S; ++s) {
    double cr, ci;
    if (a.fid_mode == 0) {
      cr = zr / S;
      ci = zi / S;
    } else {
      cr = a.zinfo[3 + 2 * s] / S;
      ci = a.zinfo[4 + 2 * s] / S;
    }
    for (int m = threadIdx.x; m < dp; m += blockDim.x) {
      double tr = 0.0, ti = 0.0;
      if (m < d) {
        tr = a.psiT64[((long)s * d + m) * 2];
        ti = a.psiT64[((long)s * d + m) * 2 + 1];
      }
      double lr = -a.alpha_fid * (cr * tr - ci * ti);
      double li = -a.alpha_fid * (cr * ti + ci * tr);
      if (a.pw) {
        lr += (double)a.pw[m] * (double)set_re(psiN, S, dp, s)[m];
        li += (double)a.pw[m] * (double)set_im(psiN, S, dp, s)[m];
      }
      set_rew(lamN, S, dp, s)[m] = (T)lr;
      set_imw(lamN, S, dp, s)[m] = (T)li;
    }
  }
}

template <typename T> __global__ __launch_bounds__(256) void k_total(SweepArgs<T> a) {
  cost_total_block(total_args(a));
}

// ------------------------------------------------------------------ penalties
// One wavefront per step transition j -> j+1 (FP64): c_{j+1} =
// (1/S) sum_s sum_m w_m |psi_{j+1}^s[m]|^2 written to out, the norm drift
// max_{j,s} | ||psi_{j+1}^s||^2 - ||psi_j^s||^2 |, and per-workgroup partial
// sums of the penalties and of the regularisers C3 (|u|^2) and C4 (control
// variations) and of the drift for the final reduction (fixed order) in
// k_total.  The last workgroup of the launch is the fidelity block.
template <typename T> __global__ __launch_bounds__(256) void k_cost(SweepArgs<T> a) {
  if (blockIdx.x == gridDim.x - 1) {  // block-uniform
    lam_block(a);
    return;
  }
  __shared__ double red[3][4];
  __shared__ double dred[4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double cpen, camp, cvar, dmax;
  pen_wave(a, (long)blockIdx.x * 4 + w, (long)a.npart * 4, cpen, camp, cvar, dmax);
  if (lane == 0) {
    red[0][w] = cpen;  // identical on all lanes of the wave
    red[1][w] = camp;
    red[2][w] = cvar;
    dred[w] = dmax;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int q = threadIdx.x;
    a.part[q * a.npart + blockIdx.x] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
  }
  if (threadIdx.x == 0)
    a.part[3 * a.npart + blockIdx.x] = fmax(fmax(dred[0], dred[1]), fmax(dred[2], dred[3]));
}


template <typename T> hipError_t launch_cost(const SweepArgs<T> &a, hipStream_t st) {
  hipLaunchKernelGGL(k_cost<T>, dim3(a.npart + 1), dim3(256), 0, st, a);
  return hipGetLastError();
}
template <typename T> hipError_t launch_total(const SweepArgs<T> &a, hipStream_t st) {
  hipLaunchKernelGGL(k_total<T>, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ B2
template <typename T> __global__ __launch_bounds__(256) void k_bwd_blocks(SweepArgs<T> a) {
  extern __shared__ unsigned char shraw[];
  T *buf = (T *)shraw;
  const int dp = a.dp, S = a.S, s = blockIdx.x;
  const long set = 2L * S * dp, mat = 2L * dp * dp;
  T *xr = buf, *xi = buf + dp, *yr = buf + 2 * dp, *yi = buf + 3 * dp;
  const T *lN = a.lam_ckpt + (long)a.nb * set;
  for (int m = threadIdx.x; m < dp; m += blockDim.x) {
    xr[m] = set_re(lN, S, dp, s)[m];
    xi[m] = set_im(lN, S, dp, s)[m];
  }
  __syncthreads();
  for (int b = a.nb - 1; b >= 1; --b) {
    const T *E = a.E + (long)b * mat;
    const T *mur = a.mu ? set_re(a.mu + (long)b * set, S, dp, s) : nullptr;
    const T *mui = a.mu ? set_im(a.mu + (long)b * set, S, dp, s) : nullptr;
    mv_plus_adj(E, E + (long)dp * dp, dp, xr, xi, yr, yi, mur, mui, buf + 6 * dp);
    __syncthreads();
    T *c = a.lam_ckpt + (long)b * set;
    for (int m = threadIdx.x; m < dp; m += blockDim.x) {
      set_rew(c, S, dp, s)[m] = yr[m];
      set_imw(c, S, dp, s)[m] = yi[m];
    }
    T *tr = xr, *ti = xi;
    xr = yr; xi = yi; yr = tr; yi = ti;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ B3
template <typename T> __global__ __launch_bounds__(256) void k_bwd_pairs(SweepArgs<T> a) {
  extern __shared__ unsigned char shraw[];
  T *buf = (T *)shraw;
  const int dp = a.dp, S = a.S;
  // (block, state) from the XCD-grouped 1-D grid (xcd_grid in the launch)
  const long lg_ = xcd_logical_block(blockIdx.x, gridDim.x);
  if (lg_ >= (long)a.nb * S) return;  // padding of the grid
  const int b = (int)(lg_ / S), s = (int)(lg_ - lg_ / S * S);
  const long set = 2L * S * dp, mat = 2L * dp * dp;
  const int start = b * a.L, end = min(a.N, start + a.L);
  T *xr = buf, *xi = buf + dp, *yr = buf + 2 * dp, *yi = buf + 3 * dp;
  T *pr = buf + 4 * dp, *pi = buf + 5 * dp;
  const T *c = a.lam_ckpt + (long)(b + 1) * set;
  for (int m = threadIdx.x; m < dp; m += blockDim.x) {
    xr[m] = set_re(c, S, dp, s)[m];
    xi[m] = set_im(c, S, dp, s)[m];
  }
  __syncthreads();
  for (int j = end - 1; j >= start; --j) {
    T *lb = a.lam_buf + (long)j * set;
    const T *ps = a.psi_buf + (long)j * set;
    for (int m = threadIdx.x; m < dp; m += blockDim.x) {
      set_rew(lb, S, dp, s)[m] = xr[m];
      set_imw(lb, S, dp, s)[m] = xi[m];
      const T wgt = (a.pw && j >= 1) ? a.pw[m] : (T)0;
      T vr = wgt * set_re(ps, S, dp, s)[m], vi = wgt * set_im(ps, S, dp, s)[m];
      if (a.src && j >= 1) {
        vr += set_re(a.src + (long)j * set, S, dp, s)[m];
        vi += set_im(a.src + (long)j * set, S, dp, s)[m];
      }
      pr[m] = vr;
      pi[m] = vi;
    }
    if (j == start) break;  // lambda_start belongs to the previous block
    __syncthreads();
    const T *D = a.D + (long)j * mat;
    mv_plus_adj(D, D + (long)dp * dp, dp, xr, xi, yr, yi, pr, pi, buf + 6 * dp);
    __syncthreads();
    T *tr = xr, *ti = xi;
    xr = yr; xi = yi; yr = tr; yi = ti;
  }
}

// ------------------------------------------------------------------ segment start
// Time segments (memory-lean mode): the costate at a segment's first step
// j0 >= 1, lambda_j0 = lambda_{j0+1} + D_j0^H lambda_{j0+1} + pw o psi_j0 +
// src_j0, written to the segment's first checkpoint lam_ckpt[0].  The
// arguments are the segment's own (lam_buf[0] = lambda_{j0+1}, D[0],
// psi_buf[0], src[0]); the preceding segment's block sweep starts from it.
template <typename T> __global__ __launch_bounds__(256) void k_seg_lambda(SweepArgs<T> a) {
  extern __shared__ unsigned char shraw[];
  T *buf = (T *)shraw;
  const int dp = a.dp, S = a.S, s = blockIdx.x;
  T *xr = buf, *xi = buf + dp, *yr = buf + 2 * dp, *yi = buf + 3 * dp;
  T *pr = buf + 4 * dp, *pi = buf + 5 * dp;
  for (int m = threadIdx.x; m < dp; m += blockDim.x) {
    xr[m] = set_re(a.lam_buf, S, dp, s)[m];
    xi[m] = set_im(a.lam_buf, S, dp, s)[m];
    const T wgt = a.pw ? a.pw[m] : (T)0;
    T vr = wgt * set_re(a.psi_buf, S, dp, s)[m], vi = wgt * set_im(a.psi_buf, S, dp, s)[m];
    if (a.src) {
      vr += set_re(a.src, S, dp, s)[m];
      vi += set_im(a.src, S, dp, s)[m];
    }
    pr[m] = vr;
    pi[m] = vi;
  }
  __syncthreads();
  mv_plus_adj(a.D, a.D + (long)dp * dp, dp, xr, xi, yr, yi, pr, pi, buf + 6 * dp);
  __syncthreads();
  for (int m = threadIdx.x; m < dp; m += blockDim.x) {
    set_rew(a.lam_ckpt, S, dp, s)[m] = yr[m];
    set_imw(a.lam_ckpt, S, dp, s)[m] = yi[m];
  }
}

template <typename T> hipError_t launch_seg_lambda(const SweepArgs<T> &a, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_lambda<T>, dim3(a.S), dim3(256), 6 * a.dp * sizeof(T) + 8192, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ wide
// Large d: one launch per step of a sequential chain, the step's matrix
// spread over many workgroups (the chains above keep one workgroup per
// column and stream a d x d matrix per step through one compute unit).
//   F2   per block b:        ckpt[b+1] = ckpt[b] + E_b ckpt[b]
//   F3   per offset t:       psi[j+1] = psi[j] + D_j psi[j], j = bL + t, all blocks
//   F3mu per offset t (down): mu_b <- mu_b + D_j^H mu_b + pw o psi_j
//   B2   per block b (down): lam_ckpt[b] = lam_ckpt[b+1] + E_b^H lam_ckpt[b+1] + mu_b
//   B3   per offset t (down): lam[j-1] = lam[j] + D_j^H lam[j] + pw o psi_j
// A launch covers all blocks (grid y) for one offset t.  Forward products
// give each wavefront WR_ROWS output rows (lanes along the row, 16-byte
// loads, wavefront reductions); adjoint products give each workgroup 64
// output columns (lane = column, coalesced row reads) with the rows split
// over the 4 wavefronts.  States are staged in LDS, SW columns at a time.
constexpr int WR_ROWS = 2, WA_UNR = 8;

template <typename T> struct WideStep {
  int mode;  // 0 F2, 1 F3, 2 F3mu, 3 B2, 4 B3
  int t;     // block (F2, B2) or offset inside the block (F3, F3mu, B3)
  T *mu_in, *mu_out;  // F3mu ping-pong sets (nb each)
  int sw;             // state columns staged in LDS at a time (<= WIDE_SWM)
};
constexpr int WIDE_SWM = 8;
// Columns per LDS chunk so that states and partial sums fit in 64 KB.
template <typename T> int wide_sw(int dp) {
  const long per = (long)sizeof(T) * (2L * dp + 512);
  long sw = 65536 / per;
  return (int)std::max(1L, std::min<long>(WIDE_SWM, sw));
}

// Operands of one (mode, t, block) job; false if the block has no work.
template <typename T>
__device__ __forceinline__ bool wide_job(const SweepArgs<T> &a, const WideStep<T> &w, int b,
                                         const T *&D, const T *&X, T *&Y, const T *&add,
                                         bool &addw) {
  const long set = 2L * a.S * a.dp, mat = 2L * a.dp * a.dp;
  add = nullptr;
  addw = false;
  if (w.mode == 0 || w.mode == 3) {
    if (b != 0) return false;
    const int blk = w.t;
    D = a.E + (long)blk * mat;
    if (w.mode == 0) {
      X = blk == 0 ? a.psi0 : a.ckpt + (long)blk * set;
      Y = a.ckpt + (long)(blk + 1) * set;
    } else {
      X = a.lam_ckpt + (long)(blk + 1) * set;
      Y = a.lam_ckpt + (long)blk * set;
      add = a.mu ? a.mu + (long)blk * set : nullptr;
    }
    return true;
  }
  const int start = b * a.L, end = min(a.N, start + a.L);
  const int j = start + w.t;
  if (j >= end) return false;
  D = a.D + (long)j * mat;
  if (w.mode == 1) {
    if (!((j + 1 < end) || (j + 1 == a.N))) return false;  // block ends come from F2
    X = a.psi_buf + (long)j * set;
    Y = a.psi_buf + (long)(j + 1) * set;
    return true;
  }
  if (w.mode == 2) {
    X = w.mu_in + (long)b * set;
    Y = w.mu_out + (long)b * set;
    add = a.psi_buf + (long)j * set;
    addw = j >= 1;
    return true;
  }
  // B3: lambda_j from lambda_{j+1} (stored at lam_buf[j]), j > start
  if (w.t == 0) return false;
  X = a.lam_buf + (long)j * set;
  Y = a.lam_buf + (long)(j - 1) * set;
  add = a.psi_buf + (long)j * set;
  addw = a.pw != nullptr;
  return true;
}

// Y = X + D X on WR_ROWS rows per wavefront, all columns of the set.
template <typename T> __global__ __launch_bounds__(256) void k_wide_fwd(SweepArgs<T> a, WideStep<T> w) {
  extern __shared__ unsigned char shraw[];
  typedef typename Vec16<T>::type V;
  constexpr int VN = Vec16<T>::n, SW = WIDE_SWM;
  const int swr = w.sw;
  T *xs = (T *)shraw, *xsi = xs + (long)swr * a.dp;  // [2][swr][dp]
  const T *D, *X, *add;
  T *Y;
  bool addw;
  if (!wide_job(a, w, blockIdx.y, D, X, Y, add, addw)) return;  // block-uniform
  const int dp = a.dp, S = a.S;
  const long plane = (long)dp * dp;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r0 = (blockIdx.x * 4 + wv) * WR_ROWS;
  const int nv = dp / VN;
  for (int s0 = 0; s0 < S; s0 += swr) {
    const int sc = min(swr, S - s0);
    __syncthreads();
    for (int e = threadIdx.x; e < sc * dp; e += 256) {
      const int s = e / dp, m = e - s * dp;
      xs[s * dp + m] = X[(long)(s0 + s) * dp + m];
      xsi[s * dp + m] = X[(long)S * dp + (long)(s0 + s) * dp + m];
    }
    __syncthreads();
    if (r0 >= dp) continue;  // wave-uniform, no barrier until the next chunk
    T ar[WR_ROWS][SW], ai[WR_ROWS][SW];
#pragma unroll
    for (int q = 0; q < WR_ROWS; ++q)
#pragma unroll
      for (int s = 0; s < SW; ++s) {
        ar[q][s] = 0;
        ai[q][s] = 0;
      }
    for (int kv = lane; kv < nv; kv += 64) {
      const int k = kv * VN;
      V dr[WR_ROWS], di[WR_ROWS];
#pragma unroll
      for (int q = 0; q < WR_ROWS; ++q) {
        dr[q] = *reinterpret_cast<const V *>(D + (long)(r0 + q) * dp + k);
        di[q] = *reinterpret_cast<const V *>(D + plane + (long)(r0 + q) * dp + k);
      }
#pragma unroll
      for (int s = 0; s < SW; ++s) {
        if (s < sc) {
#pragma unroll
          for (int e = 0; e < VN; ++e) {
            const T xr = xs[s * dp + k + e], xi = xsi[s * dp + k + e];
#pragma unroll
            for (int q = 0; q < WR_ROWS; ++q) {
              const T vr = vget<T>(dr[q], e), vi = vget<T>(di[q], e);
              ar[q][s] += vr * xr - vi * xi;
              ai[q][s] += vr * xi + vi * xr;
            }
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < WR_ROWS; ++q)
#pragma unroll
      for (int s = 0; s < SW; ++s) {
        if (s < sc) {
          const T vr = wave_sum(ar[q][s]), vi = wave_sum(ai[q][s]);
          if (lane == 0) {
            const int m = r0 + q;
            Y[(long)(s0 + s) * dp + m] = xs[s * dp + m] + vr;
            Y[(long)S * dp + (long)(s0 + s) * dp + m] = xsi[s * dp + m] + vi;
          }
        }
      }
  }
}

// Y = X + D^H X (+ ADD): workgroup = 64 output columns, 4 row slices.
template <typename T> __global__ __launch_bounds__(256) void k_wide_adj(SweepArgs<T> a, WideStep<T> w) {
  extern __shared__ unsigned char shraw[];
  constexpr int SW = WIDE_SWM;
  const int swr = w.sw;
  T *xs = (T *)shraw, *xsi = xs + (long)swr * a.dp;  // [2][swr][dp]
  T *red = xs + 2L * swr * a.dp;                      // [4][2][swr][64]
  const T *D, *X, *add;
  T *Y;
  bool addw;
  if (!wide_job(a, w, blockIdx.y, D, X, Y, add, addw)) return;  // block-uniform
  const int dp = a.dp, S = a.S;
  const long plane = (long)dp * dp;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const bool cok = c < dp;
  const int rper = (dp + 3) / 4, rb = wv * rper, re = min(dp, rb + rper);
  for (int s0 = 0; s0 < S; s0 += swr) {
    const int sc = min(swr, S - s0);
    __syncthreads();
    for (int e = threadIdx.x; e < sc * dp; e += 256) {
      const int s = e / dp, m = e - s * dp;
      xs[s * dp + m] = X[(long)(s0 + s) * dp + m];
      xsi[s * dp + m] = X[(long)S * dp + (long)(s0 + s) * dp + m];
    }
    __syncthreads();
    T yr[SW], yi[SW];
#pragma unroll
    for (int s = 0; s < SW; ++s) {
      yr[s] = 0;
      yi[s] = 0;
    }
    if (cok) {
      // WA_UNR rows of loads in flight per step of the loop (rper is a
      // multiple of 4, dp of 16; the tail loop takes the rest)
      int r = rb;
      for (; r + WA_UNR <= re; r += WA_UNR) {
        T dr[WA_UNR], di[WA_UNR];
#pragma unroll
        for (int q = 0; q < WA_UNR; ++q) {
          dr[q] = D[(long)(r + q) * dp + c];
          di[q] = -D[plane + (long)(r + q) * dp + c];  // conj(D[r][c])
        }
#pragma unroll
        for (int q = 0; q < WA_UNR; ++q)
#pragma unroll
          for (int s = 0; s < SW; ++s) {
            if (s < sc) {
              const T xr = xs[s * dp + r + q], xi = xsi[s * dp + r + q];
              yr[s] += dr[q] * xr - di[q] * xi;
              yi[s] += dr[q] * xi + di[q] * xr;
            }
          }
      }
      for (; r < re; ++r) {
        const T dr = D[(long)r * dp + c], di = -D[plane + (long)r * dp + c];
#pragma unroll
        for (int s = 0; s < SW; ++s) {
          if (s < sc) {
            const T xr = xs[s * dp + r], xi = xsi[s * dp + r];
            yr[s] += dr * xr - di * xi;
            yi[s] += dr * xi + di * xr;
          }
        }
      }
    }
#pragma unroll
    for (int s = 0; s < SW; ++s) {
      if (s < sc) {
        red[((wv * 2 + 0) * swr + s) * 64 + lane] = yr[s];
        red[((wv * 2 + 1) * swr + s) * 64 + lane] = yi[s];
      }
    }
    __syncthreads();
    if (wv == 0 && cok) {
      for (int s = 0; s < sc; ++s) {
        T vr = xs[s * dp + c], vi = xsi[s * dp + c];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          vr += red[((q * 2 + 0) * swr + s) * 64 + lane];
          vi += red[((q * 2 + 1) * swr + s) * 64 + lane];
        }
        if (add) {
          if (w.mode == 3) {
            vr += add[(long)(s0 + s) * dp + c];
            vi += add[(long)S * dp + (long)(s0 + s) * dp + c];
          } else if (addw) {
            const T wg = a.pw[c];
            vr += wg * add[(long)(s0 + s) * dp + c];
            vi += wg * add[(long)S * dp + (long)(s0 + s) * dp + c];
          }
        }
        Y[(long)(s0 + s) * dp + c] = vr;
        Y[(long)S * dp + (long)(s0 + s) * dp + c] = vi;
      }
    }
  }
}

// ------------------------------------------------------------------ wide, MFMA
// The same per-step products as thin matrix products on the MFMA (sweep
// variant 5): Y = X + op(M) X (+ addend) with the state set X (S x d_pad,
// state-major) taken as the d_pad x S panel X^T.  A workgroup owns 16
// output rows and 16 states; its 4 wavefronts split the inner dimension in
// quarters and multiply straight from global memory (no LDS staging: each
// lane reads 16-byte vectors of 4 consecutive inner indices, and the inner
// index of MFMA step q at lane group kk is 4 kk + q so that both operands
// come from those vectors), then meet in LDS.  Small tiles put the
// sequential chain's per-step matrix read on many compute units.
template <typename T>
__device__ __forceinline__ void wm_vec4(const T *p, T (&v)[4]) {
  typedef typename Vec16<T>::type V;
  if constexpr (Vec16<T>::n == 4) {
    const V x = *reinterpret_cast<const V *>(p);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = vget<T>(x, e);
  } else {
    const V x0 = *reinterpret_cast<const V *>(p), x1 = *reinterpret_cast<const V *>(p + 2);
    v[0] = vget<T>(x0, 0);
    v[1] = vget<T>(x0, 1);
    v[2] = vget<T>(x1, 0);
    v[3] = vget<T>(x1, 1);
  }
}

template <typename T, int OPA>
__global__ __launch_bounds__(256) void k_wide_mm(SweepArgs<T> a, WideStep<T> w) {
  __shared__ T red[4][2][4][64];  // [wave][re, im][acc element][lane]
  const T *D, *X, *add;
  T *Y;
  bool addw;
  if (!wide_job(a, w, blockIdx.y, D, X, Y, add, addw)) return;  // block-uniform
  const int dp = a.dp, S = a.S;
  const long plane = (long)dp * dp;
  const int rt = dp / 16;
  const int r0 = (blockIdx.x % rt) * 16, s0 = (blockIdx.x / rt) * 16;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int kq = dp / 4, kb = wv * kq, ke = kb + kq;  // this wavefront's inner range
  const bool sok = s0 + i < S;
  const long xo = sok ? (long)(s0 + i) * dp : 0;  // state row (index 0 if none)
  v4<T> cr = vzero<T>(), ci = vzero<T>();
  for (int k0 = kb; k0 < ke; k0 += 16) {
    // this lane's 4 inner indices k .. k+3 (a quarter of dp is a multiple of
    // 4, not always of 16: lanes past the range read at its start, add zero)
    const bool kok = k0 + 4 * kk < ke;
    const int k = kok ? k0 + 4 * kk : kb;
    T ar[4], ai[4], br[4], bi[4];
    if (OPA == 0) {  // M[r0 + i][k .. k+3]
      wm_vec4<T>(D + (long)(r0 + i) * dp + k, ar);
      wm_vec4<T>(D + plane + (long)(r0 + i) * dp + k, ai);
    } else {  // conj(M[k .. k+3][r0 + i])
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ar[q] = D[(long)(k + q) * dp + r0 + i];
        ai[q] = -D[plane + (long)(k + q) * dp + r0 + i];
      }
    }
    wm_vec4<T>(X + xo + k, br);
    wm_vec4<T>(X + (long)S * dp + xo + k, bi);
    if (!sok || !kok) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        br[q] = 0;
        bi[q] = 0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cr = mfma4(ar[q], br[q], cr);
      cr = mfma4(-ai[q], bi[q], cr);
      ci = mfma4(ar[q], bi[q], ci);
      ci = mfma4(ai[q], br[q], ci);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    red[wv][0][v][lane] = cr[v];
    red[wv][1][v][lane] = ci[v];
  }
  __syncthreads();
  if (wv != 0) return;
  // y[s][m] = x[s][m] + (op(M) x^s)[m] (+ mu, or pw o psi, by mode)
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = r0 + acc_row<T>(lane, v), sidx = s0 + (lane & 15);
    if (sidx >= S) continue;
    const T sr = red[0][0][v][lane] + red[1][0][v][lane] + red[2][0][v][lane] + red[3][0][v][lane];
    const T si = red[0][1][v][lane] + red[1][1][v][lane] + red[2][1][v][lane] + red[3][1][v][lane];
    const long o = (long)sidx * dp + m, oi = (long)S * dp + o;
    T vr = X[o] + sr, vi = X[oi] + si;
    if (add) {
      if (w.mode == 3) {
        vr += add[o];
        vi += add[oi];
      } else if (addw) {
        const T wg = a.pw[m];
        vr += wg * add[o];
        vi += wg * add[oi];
      }
    }
    Y[o] = vr;
    Y[oi] = vi;
  }
}

template <typename T> bool wide_sweep_ok(int dp, int S) {
  (void)S;
  return dp >= 80;
}

// The four sweeps of the blocked scan as per-step launches.  Scratch: the
// F3mu ping-pong partner of mu uses lam_buf (free until B3).
template <typename T> hipError_t launch_wide_sweep(int which, const SweepArgs<T> &a,
                                                   hipStream_t st, bool mm) {
  const int SW = wide_sw<T>(a.dp);
  // MFMA variant: 16-row x 16-state tiles
  const unsigned mmg = (unsigned)((a.dp / 16) * ((a.S + 15) / 16));
  auto fwd = [&](const WideStep<T> &w, unsigned gy) -> hipError_t {
    if (mm)
      hipLaunchKernelGGL((k_wide_mm<T, 0>), dim3(mmg, gy), dim3(256), 0, st, a, w);
    else
      hipLaunchKernelGGL(k_wide_fwd<T>, dim3((unsigned)((a.dp + 4 * WR_ROWS - 1) / (4 * WR_ROWS)), gy),
                         dim3(256), 2 * SW * a.dp * sizeof(T), st, a, w);
    return hipGetLastError();
  };
  auto adj = [&](const WideStep<T> &w, unsigned gy) -> hipError_t {
    if (mm)
      hipLaunchKernelGGL((k_wide_mm<T, 1>), dim3(mmg, gy), dim3(256), 0, st, a, w);
    else
      hipLaunchKernelGGL(k_wide_adj<T>, dim3((unsigned)((a.dp + 63) / 64), gy), dim3(256),
                         2 * SW * a.dp * sizeof(T) + 4 * 2 * SW * 64 * sizeof(T), st, a, w);
    return hipGetLastError();
  };
  const long set = 2L * a.S * a.dp;
  const int Lmax = a.nb > 1 ? a.L : a.N;  // longest block
  hipError_t e;
  WideStep<T> w{};
  w.sw = SW;
  switch (which) {
    case 0:  // F2
      if ((e = launch_copy<T>(a.ckpt, a.psi0, set, st)) != hipSuccess) return e;
      for (int b = 0; b < a.nb; ++b) {
        w.mode = 0;
        w.t = b;
        if ((e = fwd(w, 1)) != hipSuccess) return e;
      }
      return hipSuccess;
    case 1: {  // F3: block starts from the checkpoints (one strided copy), then every offset
      if ((e = launch_copy_strided<T>(a.psi_buf, (long)a.L * set, a.ckpt, set, set, a.nb, st)) !=
          hipSuccess)
        return e;
      for (int t = 0; t < Lmax; ++t) {
        w.mode = 1;
        w.t = t;
        if ((e = fwd(w, a.nb)) != hipSuccess) return e;
      }
      if (!a.pw) return hipSuccess;
      // block-local penalty costates, from zero at each block end
      T *bufs[2] = {a.mu, a.lam_buf};
      if ((e = launch_fill<T>(a.mu, (long)a.nb * set, (T)0, st)) != hipSuccess) return e;
      if ((e = launch_fill<T>(a.lam_buf, (long)a.nb * set, (T)0, st)) != hipSuccess) return e;
      for (int t = Lmax - 1; t >= 0; --t) {
        // the launch for offset t writes the buffer that t = 0 ends in (mu)
        w.mode = 2;
        w.t = t;
        w.mu_out = bufs[t & 1];
        w.mu_in = bufs[(t + 1) & 1];
        if ((e = adj(w, a.nb)) != hipSuccess) return e;
      }
      return hipSuccess;
    }
    case 2:  // B2
      for (int b = a.nb - 1; b >= 1; --b) {
        w.mode = 3;
        w.t = b;
        if ((e = adj(w, 1)) != hipSuccess) return e;
      }
      return hipSuccess;
    default: {  // B3: lam_buf[end-1] = lambda_end (the full blocks in one strided copy), then every offset downwards
      const int full = a.N / a.L;  // blocks of length L; a ragged last one apart
      if (full > 0 &&
          (e = launch_copy_strided<T>(a.lam_buf + (long)(a.L - 1) * set, (long)a.L * set,
                                      a.lam_ckpt + set, set, set, full, st)) != hipSuccess)
        return e;
      if (full < a.nb &&
          (e = launch_copy<T>(a.lam_buf + (long)(a.N - 1) * set, a.lam_ckpt + (long)a.nb * set,
                              set, st)) != hipSuccess)
        return e;
      for (int t = Lmax - 1; t >= 1; --t) {
        w.mode = 4;
        w.t = t;
        if ((e = adj(w, a.nb)) != hipSuccess) return e;
      }
      return hipSuccess;
    }
  }
}

template <typename T> hipError_t launch_fwd_blocks(const SweepArgs<T> &a, hipStream_t st) {
  hipLaunchKernelGGL(k_fwd_blocks<T>, dim3(a.S), dim3(256), 4 * a.dp * sizeof(T), st, a);
  return hipGetLastError();
}
template <typename T> hipError_t launch_fwd_replay(const SweepArgs<T> &a, hipStream_t st) {
  hipLaunchKernelGGL(k_fwd_replay<T>, dim3(xcd_grid((long)a.nb * a.S, a.S)), dim3(256), 6 * a.dp * sizeof(T) + 8192, st, a);
  return hipGetLastError();
}

template <typename T> hipError_t launch_bwd_blocks(const SweepArgs<T> &a, hipStream_t st) {
  hipLaunchKernelGGL(k_bwd_blocks<T>, dim3(a.S), dim3(256), 6 * a.dp * sizeof(T) + 8192, st, a);
  return hipGetLastError();
}
template <typename T> hipError_t launch_bwd_pairs(const SweepArgs<T> &a, hipStream_t st) {
  hipLaunchKernelGGL(k_bwd_pairs<T>, dim3(xcd_grid((long)a.nb * a.S, a.S)), dim3(256), 6 * a.dp * sizeof(T) + 8192, st, a);
  return hipGetLastError();
}

#define QOC_INST(T)                                                                   \
  template bool wide_sweep_ok<T>(int, int);                                           \
  template hipError_t launch_wide_sweep<T>(int, const SweepArgs<T> &, hipStream_t, bool); \
  template hipError_t launch_fwd_blocks<T>(const SweepArgs<T> &, hipStream_t);       \
  template hipError_t launch_seg_lambda<T>(const SweepArgs<T> &, hipStream_t);       \
  template hipError_t launch_fwd_replay<T>(const SweepArgs<T> &, hipStream_t);       \
  template hipError_t launch_cost<T>(const SweepArgs<T> &, hipStream_t);             \
  template hipError_t launch_total<T>(const SweepArgs<T> &, hipStream_t);            \
  template hipError_t launch_bwd_blocks<T>(const SweepArgs<T> &, hipStream_t);       \
  template hipError_t launch_bwd_pairs<T>(const SweepArgs<T> &, hipStream_t);
QOC_INST(float)
QOC_INST(double)
#undef QOC_INST

}  // namespace qoc
