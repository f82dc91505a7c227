// Per-step cost terms beyond the diagonal level penalty (Table I):
//   C5 with general forbidden states F_f (Sec. II.A: a set of forbidden
//      states enters upon summation):
//        c_j += (1/S) sum_s sum_f |<F_f|psi_j^s>|^2,            j = 1..N
//   C6 / C7, the time-optimal term: the fidelity of every intermediate
//      state set against the targets, in the mode of the final fidelity
//      (coherent for a target gate on a basis, C6; incoherent for target
//      states, C7):  C_time = 1 - (1/N) sum_{j=1..N} F_j.
// Both are functions of psi_j alone, so their derivatives enter the costate
// recursion as per-step sources (Sec. II.B, reverse accumulation):
//   src_j^s = a_pen/S sum_f <F_f|psi_j^s> F_f - (a_time/N) coef_j^s T_s,
//   coef_j^s = z_j / S (coherent, z_j = (1/S) sum_s <T_s|psi_j^s>) or
//              <T_s|psi_j^s> / S (incoherent),
// and lambda_j = U_j^H lambda_{j+1} + (level penalty) + src_j for j >= 1,
// lambda_N picking up src_N.  One wavefront per step, all overlaps in FP64.
#include <algorithm>

#include "qoc_device.h"
#include "qoc_kernels.h"

namespace qoc {

namespace {

template <typename T> __device__ __forceinline__ double ld_re(const T *set, int S, int dp, int s, int m) {
  return (double)set[(long)s * dp + m];
}
template <typename T> __device__ __forceinline__ double ld_im(const T *set, int S, int dp, int s, int m) {
  return (double)set[(long)S * dp + (long)s * dp + m];
}

// <V|psi^s> over the true dimension d, V interleaved complex FP64; every
// lane of the wavefront returns the same sum.
template <typename T>
__device__ __forceinline__ void overlap(const double *V, const T *set, int S, int dp, int d,
                                       int s, double &orr, double &oi) {
  const int lane = threadIdx.x & 63;
  double pr = 0.0, pi = 0.0;
  for (int m = lane; m < d; m += 64) {
    const double vr = V[2 * m], vi = V[2 * m + 1];
    const double xr = ld_re(set, S, dp, s, m), xi = ld_im(set, S, dp, s, m);
    pr += vr * xr + vi * xi;  // conj(V) psi
    pi += vr * xi - vi * xr;
  }
  orr = wave_sum(pr);
  oi = wave_sum(pi);
}

}  // namespace

template <typename T> __global__ __launch_bounds__(256) void k_ext(SweepArgs<T> a, ExtArgs<T> e) {
  __shared__ double red[2][4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int dp = a.dp, d = a.d, S = a.S, N = a.N, nf = e.nf;
  const long set = 2L * S * dp;
  const bool coherent = a.fid_mode == 0, timed = e.alpha_time != 0.0;
  double pen_sum = 0.0, f_sum = 0.0;
  for (long j = 1 + (long)blockIdx.x * 4 + w; j <= N; j += (long)gridDim.x * 4) {
    const T *psi = a.psi_buf + j * set;
    T *src = e.src + j * set;
    // coherent time term: z_j over all columns first
    double zr = 0.0, zi = 0.0, finc = 0.0;
    if (timed) {
      for (int s = 0; s < S; ++s) {
        double orr, oi;
        overlap(a.psiT64 + (long)s * d * 2, psi, S, dp, d, s, orr, oi);
        zr += orr;
        zi += oi;
        finc += orr * orr + oi * oi;
      }
      zr /= S;
      zi /= S;
    }
    double pen = 0.0;
    for (int s = 0; s < S; ++s) {
      double fr[QOC_MAX_FORBIDDEN], fi[QOC_MAX_FORBIDDEN];
#pragma unroll
      for (int f = 0; f < QOC_MAX_FORBIDDEN; ++f) {
        fr[f] = 0.0;
        fi[f] = 0.0;
        if (f < nf) {
          overlap(e.forb64 + (long)f * d * 2, psi, S, dp, d, s, fr[f], fi[f]);
          pen += fr[f] * fr[f] + fi[f] * fi[f];
        }
      }
      double cr = 0.0, ci = 0.0;  // coefficient of T_s in the source
      if (timed) {
        if (coherent) {
          cr = zr / S;
          ci = zi / S;
        } else {
          overlap(a.psiT64 + (long)s * d * 2, psi, S, dp, d, s, cr, ci);
          cr /= S;
          ci /= S;
        }
      }
      const double kt = -e.alpha_time / N, kf = a.alpha_pen / S;
      T *sr = src + (long)s * dp, *si = src + (long)S * dp + (long)s * dp;
      T *lr = nullptr, *li = nullptr;
      if (j == N && e.lamN) {
        lr = e.lamN + (long)s * dp;
        li = e.lamN + (long)S * dp + (long)s * dp;
      }
      for (int m = lane; m < dp; m += 64) {
        double vr = 0.0, vi = 0.0;
        if (m < d) {
#pragma unroll
          for (int f = 0; f < QOC_MAX_FORBIDDEN; ++f) {
            if (f < nf) {
              const double Fr = e.forb64[((long)f * d + m) * 2], Fi = e.forb64[((long)f * d + m) * 2 + 1];
              vr += kf * (fr[f] * Fr - fi[f] * Fi);
              vi += kf * (fr[f] * Fi + fi[f] * Fr);
            }
          }
          if (timed) {
            const double Tr = a.psiT64[((long)s * d + m) * 2], Ti = a.psiT64[((long)s * d + m) * 2 + 1];
            vr += kt * (cr * Tr - ci * Ti);
            vi += kt * (cr * Ti + ci * Tr);
          }
        }
        sr[m] = (T)vr;
        si[m] = (T)vi;
        if (lr) {
          // lambda_N (written by the cost launch before this one) gains src_N
          lr[m] = (T)((double)lr[m] + vr);
          li[m] = (T)((double)li[m] + vi);
        }
      }
    }
    pen /= S;
    if (lane == 0 && nf > 0) a.out[1 + j] += pen;  // out[2 + (j - 1)] = c_j
    pen_sum += pen;
    if (timed) f_sum += coherent ? (zr * zr + zi * zi) : finc / S;
  }
  if (lane == 0) {
    red[0][w] = pen_sum;
    red[1][w] = f_sum;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int q = threadIdx.x;
    e.part[q * e.nblk + blockIdx.x] = red[q][0] + red[q][1] + red[q][2] + red[q][3];
  }
}

template <typename T>
hipError_t launch_ext(const SweepArgs<T> &a, const ExtArgs<T> &e, hipStream_t st) {
  hipLaunchKernelGGL(k_ext<T>, dim3(e.nblk), dim3(256), 0, st, a, e);
  return hipGetLastError();
}

template hipError_t launch_ext<float>(const SweepArgs<float> &, const ExtArgs<float> &,
                                      hipStream_t);
template hipError_t launch_ext<double>(const SweepArgs<double> &, const ExtArgs<double> &,
                                       hipStream_t);


// ---------------------------------------------------------------------------
// Unitarity drift of the step propagators (Sec. III: the truncated series
// with scaling and squaring is only approximately unitary): with U = I + D,
//   U^H U - I = D + D^H + D^H D,
// whose largest entry magnitude over the checked steps is accumulated in
// FP64 (products on the FP64 MFMA from operands converted to FP64).  One
// wavefront per 16 x 16 tile of one checked step; the checked steps are
// j = N-1, N-1-stride, ...  The result is folded into *acc with one atomic
// maximum per wavefront on (epoch << 32 | FP32 bits of the tile maximum):
// a later call (larger epoch) supersedes every earlier value without a
// clearing launch, and positive FP32 values order like their bit patterns.
namespace {
template <typename T>
__global__ __launch_bounds__(256) void k_unitarity(const T *__restrict__ D, int dp, int d, int N,
                                                   int stride, int nchk, unsigned epoch,
                                                   unsigned long long *acc) {
  const int tdim = dp / 16, tiles = tdim * tdim;
  const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wave >= (long)nchk * tiles) return;  // wavefront-uniform; no barrier below
  const int q = (int)(wave / tiles), t = (int)(wave - (long)q * tiles);
  const int r0 = (t / tdim) * 16, c0 = (t % tdim) * 16;
  const long j = (long)N - 1 - (long)q * stride;
  const long plane = (long)dp * dp;
  const T *Dr = D + j * 2 * plane, *Di = Dr + plane;
  const int lane = threadIdx.x & 63, i = lane & 15, kk = lane >> 4;
  f64x4 cr = vzero<double>(), ci = vzero<double>();
  // (D^H D)_{rc} = sum_k conj(D_{kr}) D_{kc}: A = D^H, B = D
  for (int k = 0; k < dp; k += 4) {
    const long oa = (long)(k + kk) * dp + (r0 + i), ob = (long)(k + kk) * dp + (c0 + i);
    const double ar = (double)Dr[oa], ai = -(double)Di[oa];
    const double br = (double)Dr[ob], bi = (double)Di[ob];
    cr = mfma4(ar, br, cr);
    cr = mfma4(-ai, bi, cr);
    ci = mfma4(ar, bi, ci);
    ci = mfma4(ai, br, ci);
  }
  double m = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = r0 + acc_row<double>(lane, v), c = c0 + i;
    if (r < d && c < d) {
      // + D_{rc} + conj(D_{cr})
      const double er = cr[v] + (double)Dr[(long)r * dp + c] + (double)Dr[(long)c * dp + r];
      const double ei = ci[v] + (double)Di[(long)r * dp + c] - (double)Di[(long)c * dp + r];
      m = fmax(m, sqrt(er * er + ei * ei));
    }
  }
  m = wave_max(m);
  if (lane == 0) {
    const float mf = (float)m;
    atomicMax(acc, ((unsigned long long)epoch << 32) | (unsigned long long)__float_as_uint(mf));
  }
}
}  // namespace

template <typename T>
hipError_t launch_unitarity(const T *D, int dp, int d, int N, int stride, unsigned epoch,
                            unsigned long long *acc, hipStream_t st) {
  if (N <= 0 || stride <= 0) return hipSuccess;
  const int nchk = (N + stride - 1) / stride;
  const long waves = (long)nchk * (dp / 16) * (dp / 16);
  hipLaunchKernelGGL(k_unitarity<T>, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, D, dp, d,
                     N, stride, nchk, epoch, acc);
  return hipGetLastError();
}

template hipError_t launch_unitarity<float>(const float *, int, int, int, int, unsigned,
                                            unsigned long long *, hipStream_t);
template hipError_t launch_unitarity<double>(const double *, int, int, int, int, unsigned,
                                             unsigned long long *, hipStream_t);


// ---------------------------------------------------------------------------
// Adam update of the control amplitudes (the optimiser of the paper's
// examples, Sec. IV), flat over any number of instances' amplitudes, in FP64:
//   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,  t' = t + 1,
//   u <- u - lr (m / (1 - b1^t')) / (sqrt(v / (1 - b2^t')) + eps).
// The step count lives on the device (graph replays advance it): k_adam
// reads t, and k_adam_count increments it afterwards.
namespace {
__global__ __launch_bounds__(256) void k_adam(long n, double *__restrict__ u,
                                              const double *__restrict__ g, double *__restrict__ m,
                                              double *__restrict__ v, const double *__restrict__ t,
                                              double lr, double b1, double b2, double eps) {
  const double tn = t[0] + 1.0;
  const double bc1 = 1.0 - pow(b1, tn), bc2 = 1.0 - pow(b2, tn);
  const double step = lr / bc1, rbc2 = 1.0 / sqrt(bc2);
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const double gi = g[i];
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    u[i] -= step * mi / (sqrt(vi) * rbc2 + eps);
  }
}
__global__ void k_adam_count(double *t) {
  if (threadIdx.x == 0) t[0] += 1.0;
}
}  // namespace

hipError_t launch_adam(long n, double *u, const double *g, double *m, double *v, double *t,
                       double lr, double b1, double b2, double eps, hipStream_t st) {
  if (n > 0) {
    const long blocks = std::min<long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, st, n, u, g, m, v, t, lr, b1,
                       b2, eps);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adam_count, dim3(1), dim3(64), 0, st, t);
  return hipGetLastError();
}

}  // namespace qoc
