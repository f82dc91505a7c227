// Latency-oriented sweeps for small Hilbert spaces (padded d <= 64).
//
// Same blocked two-level scan as kernels_sweep.hip (F2 / F3 / B2 / B3), but
// each workgroup carries all S columns at once and the step matrix is
// staged through LDS with a one-step register prefetch: the global loads of
// D_{j+1} are issued before the product with D_j, so the HBM latency is
// off the sequential critical path.  For the costate sweeps the matrix is
// stored transposed in LDS, so both directions read rows.
//
// Per step: y = x + op(D) x (+ add) for the S columns, op = identity or ^H.
// Thread t handles output o = t / KC (o = s * DP + m) and the k-chunk
// t % KC of length DP / KC; partial sums are combined across the KC
// consecutive lanes with cross-lane shuffles.
#include "qoc_device.h"
#include "qoc_kernels.h"

namespace qoc {

template <typename T, int DP> struct SmallPlan {
  static constexpr int PF = (2 * DP * DP + 255) / 256;  // prefetched elements per thread
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

template <typename T, int DP>
__device__ __forceinline__ void sm_prefetch(const T *__restrict__ g, T (&reg)[SmallPlan<T, DP>::PF]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < SmallPlan<T, DP>::PF; ++q) {
    const int e = q * 256 + t;
    reg[q] = (e < 2 * DP * DP) ? g[e] : (T)0;
  }
}

template <typename T, int DP, bool TRANS>
__device__ __forceinline__ void sm_store(T *Ds, const T (&reg)[SmallPlan<T, DP>::PF]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < SmallPlan<T, DP>::PF; ++q) {
    const int e = q * 256 + t;
    if (e < 2 * DP * DP) {
      if (TRANS) {
        const int pl = e / (DP * DP), rem = e - pl * DP * DP;
        const int r = rem / DP, c = rem - r * DP;
        Ds[pl * DP * DP + c * DP + r] = reg[q];
      } else {
        Ds[e] = reg[q];
      }
    }
  }
}

// y = x + op(D) x + add, with op(D)[m][k] = Ds[m][k] (CONJ = false) or
// conj(Ds[m][k]) where Ds holds D^T (CONJ = true).  add (optional) is
// given per output as (ar, ai) from the caller's registers.
template <typename T, int DP, bool CONJ>
__device__ __forceinline__ void sm_apply(const SmallPlan<T, DP> &P, const T *Ds, const T *x,
                                         T *y, const T *addr_g, const T *addi_g,
                                         const T *pw, bool use_add) {
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
      if (use_add) {
        vr += pw[m] * addr_g[s * DP + m];
        vi += pw[m] * addi_g[s * DP + m];
      }
      y[s * DP + m] = vr;
      y[SD + s * DP + m] = vi;
    }
  }
}

template <typename T>
__device__ __forceinline__ void copy_set(T *dst, const T *src, int n) {
  for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
}

// ------------------------------------------------------------------ F2
template <typename T, int DP> __global__ __launch_bounds__(256) void k_smF2(SweepArgs<T> a) {
  extern __shared__ unsigned char shraw[];
  T *Ds = (T *)shraw;
  T *x = Ds + 2 * DP * DP, *y = x + 2 * a.S * DP;
  SmallPlan<T, DP> P;
  P.init(a.S);
  const int set = 2 * a.S * DP;
  const long mat = 2L * DP * DP;
  T reg[SmallPlan<T, DP>::PF];
  copy_set(x, a.psi0, set);
  copy_set(a.ckpt, a.psi0, set);
  sm_prefetch<T, DP>(a.E, reg);
  for (int b = 0; b < a.nb; ++b) {
    sm_store<T, DP, false>(Ds, reg);
    __syncthreads();
    if (b + 1 < a.nb) sm_prefetch<T, DP>(a.E + (b + 1) * mat, reg);
    sm_apply<T, DP, false>(P, Ds, x, y, nullptr, nullptr, nullptr, false);
    __syncthreads();
    copy_set(a.ckpt + (long)(b + 1) * set, y, set);
    T *tmp = x; x = y; y = tmp;
  }
}

// ------------------------------------------------------------------ F3
template <typename T, int DP> __global__ __launch_bounds__(256) void k_smF3(SweepArgs<T> a) {
  extern __shared__ unsigned char shraw[];
  T *Ds = (T *)shraw;
  T *x = Ds + 2 * DP * DP, *y = x + 2 * a.S * DP;
  SmallPlan<T, DP> P;
  P.init(a.S);
  const int set = 2 * a.S * DP;
  const long mat = 2L * DP * DP;
  const int b = blockIdx.x;
  const int start = b * a.L, end = min(a.N, start + a.L);
  T reg[SmallPlan<T, DP>::PF];
  copy_set(x, a.ckpt + (long)b * set, set);
  copy_set(a.psi_buf + (long)start * set, a.ckpt + (long)b * set, set);
  sm_prefetch<T, DP>(a.D + start * mat, reg);
  for (int j = start; j < end; ++j) {
    sm_store<T, DP, false>(Ds, reg);
    __syncthreads();
    if (j + 1 < end) sm_prefetch<T, DP>(a.D + (j + 1) * mat, reg);
    sm_apply<T, DP, false>(P, Ds, x, y, nullptr, nullptr, nullptr, false);
    __syncthreads();
    if (j + 1 < end || j + 1 == a.N) copy_set(a.psi_buf + (long)(j + 1) * set, y, set);
    T *tmp = x; x = y; y = tmp;
  }
  if (!a.pw) return;  // block-uniform
  // block-local penalty costate from zero at the block end (states of this
  // block were written above by this workgroup):
  // mu <- mu + D_j^H mu + pw o psi_j   (penalty only for j >= 1)
  for (int e = threadIdx.x; e < set; e += blockDim.x) x[e] = (T)0;
  sm_prefetch<T, DP>(a.D + (end - 1) * mat, reg);
  __syncthreads();
  for (int j = end - 1; j >= start; --j) {
    sm_store<T, DP, true>(Ds, reg);
    __syncthreads();
    if (j - 1 >= start) sm_prefetch<T, DP>(a.D + (j - 1) * mat, reg);
    const T *ps = a.psi_buf + (long)j * set;
    sm_apply<T, DP, true>(P, Ds, x, y, ps, ps + a.S * DP, a.pw, j >= 1);
    __syncthreads();
    T *tmp = x; x = y; y = tmp;
  }
  copy_set(a.mu + (long)b * set, x, set);
}

// ------------------------------------------------------------------ B2
template <typename T, int DP> __global__ __launch_bounds__(256) void k_smB2(SweepArgs<T> a) {
  extern __shared__ unsigned char shraw[];
  T *Ds = (T *)shraw;
  T *x = Ds + 2 * DP * DP, *y = x + 2 * a.S * DP;
  SmallPlan<T, DP> P;
  P.init(a.S);
  const int set = 2 * a.S * DP;
  const long mat = 2L * DP * DP;
  T reg[SmallPlan<T, DP>::PF];
  copy_set(x, a.lam_ckpt + (long)a.nb * set, set);
  if (a.nb >= 2) sm_prefetch<T, DP>(a.E + (a.nb - 1) * mat, reg);
  for (int b = a.nb - 1; b >= 1; --b) {
    sm_store<T, DP, true>(Ds, reg);
    __syncthreads();
    if (b - 1 >= 1) sm_prefetch<T, DP>(a.E + (b - 1) * mat, reg);
    const T *mu = a.mu ? a.mu + (long)b * set : nullptr;
    T *yy = y;
    if (mu) {
      // y = x + E^H x + mu : use the add path with unit weights via pw = null
      sm_apply<T, DP, true>(P, Ds, x, yy, nullptr, nullptr, nullptr, false);
      __syncthreads();
      for (int e = threadIdx.x; e < set; e += blockDim.x) yy[e] += mu[e];
    } else {
      sm_apply<T, DP, true>(P, Ds, x, yy, nullptr, nullptr, nullptr, false);
    }
    __syncthreads();
    copy_set(a.lam_ckpt + (long)b * set, yy, set);
    T *tmp = x; x = y; y = tmp;
  }
}

// ------------------------------------------------------------------ B3
template <typename T, int DP> __global__ __launch_bounds__(256) void k_smB3(SweepArgs<T> a) {
  extern __shared__ unsigned char shraw[];
  T *Ds = (T *)shraw;
  T *x = Ds + 2 * DP * DP, *y = x + 2 * a.S * DP;
  SmallPlan<T, DP> P;
  P.init(a.S);
  const int set = 2 * a.S * DP;
  const long mat = 2L * DP * DP;
  const int b = blockIdx.x;
  const int start = b * a.L, end = min(a.N, start + a.L);
  T reg[SmallPlan<T, DP>::PF];
  copy_set(x, a.lam_ckpt + (long)(b + 1) * set, set);
  if (end - 1 > start) sm_prefetch<T, DP>(a.D + (end - 1) * mat, reg);
  __syncthreads();
  for (int j = end - 1; j >= start; --j) {
    copy_set(a.lam_buf + (long)j * set, x, set);  // lambda_{j+1}
    if (j == start) break;                        // block-uniform
    sm_store<T, DP, true>(Ds, reg);
    __syncthreads();
    if (j - 1 > start) sm_prefetch<T, DP>(a.D + (j - 1) * mat, reg);
    const T *ps = a.psi_buf + (long)j * set;
    sm_apply<T, DP, true>(P, Ds, x, y, ps, ps + a.S * DP, a.pw, a.pw != nullptr && j >= 1);
    __syncthreads();
    T *tmp = x; x = y; y = tmp;
  }
}

template <typename T, int DP> size_t sm_lds_bytes(int S) {
  return sizeof(T) * (2 * DP * DP + 4 * (size_t)S * DP);
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
  const size_t bytes = sizeof(T) * (2 * (size_t)dp * dp + 4 * (size_t)S * dp);
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

// ------------------------------------------------------------------ penalties
// c_part[j][s] = sum_m w_m |psi_j^s[m]|^2 (FP64) for j = 1..N and the norm
// drift max_{j,s} | ||psi_{j+1}^s||^2 - ||psi_j^s||^2 |, all in parallel.
template <typename T> __global__ __launch_bounds__(256) void k_pen(SweepArgs<T> a) {
  __shared__ double red[4];
  const long pairs = (long)a.N * a.S;
  const int dp = a.dp, S = a.S;
  const long set = 2L * S * dp;
  double dmax = 0.0;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < pairs;
       q += (long)gridDim.x * blockDim.x) {
    const long j = q / S;            // step j -> j + 1
    const int s = (int)(q - j * S);
    const T *p0r = a.psi_buf + j * set + (long)s * dp, *p0i = p0r + (long)S * dp;
    const T *p1r = a.psi_buf + (j + 1) * set + (long)s * dp, *p1i = p1r + (long)S * dp;
    double n0 = 0.0, n1 = 0.0, pen = 0.0;
    for (int m = 0; m < dp; ++m) {
      const double ar = p0r[m], ai = p0i[m], br = p1r[m], bi = p1i[m];
      const double q1 = br * br + bi * bi;
      n0 += ar * ar + ai * ai;
      n1 += q1;
      if (a.w64) pen += a.w64[m] * q1;
    }
    if (a.w64) a.c_part[(j + 1) * S + s] = pen;
    dmax = fmax(dmax, fabs(n1 - n0));
  }
  dmax = wave_max(dmax);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(a.drift_bits, (unsigned long long)__double_as_longlong(m));
  }
}

template <typename T> hipError_t launch_pen(const SweepArgs<T> &a, hipStream_t st) {
  const long pairs = (long)a.N * a.S;
  long blocks = (pairs + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_pen<T>, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

template bool small_sweep_ok<float>(int, int);
template bool small_sweep_ok<double>(int, int);
template hipError_t launch_small_sweep<float>(int, const SweepArgs<float> &, hipStream_t);
template hipError_t launch_small_sweep<double>(int, const SweepArgs<double> &, hipStream_t);
template hipError_t launch_pen<float>(const SweepArgs<float> &, hipStream_t);
template hipError_t launch_pen<double>(const SweepArgs<double> &, hipStream_t);

}  // namespace qoc
