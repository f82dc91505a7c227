// theta_max = max_j || dt H_j ||_1 (maximum column absolute sum), in FP64.
//
// The paper fixes one conservative truncation order p and squaring count n
// for all steps instead of estimating each step's spectral radius
// (Sec. III); this kernel supplies the global norm that choice is made
// from.  Each workgroup covers 16 columns x 16 steps; the Hamiltonian
// entries of a 2-row chunk are staged once in LDS and reused by all 16
// steps, so H is read from L2 N/16 times instead of N times.
#include "qoc_device.h"
#include "qoc_kernels.h"

namespace qoc {

constexpr int NRM_COLS = 16, NRM_STEPS = 16, NRM_ROWS = 2;

// (p, n) from theta by the rule of qoc_taylor_select, one wavefront, one
// lane per squaring count n; returns {p, n, status} and dt / 2^n.
__device__ void select_pn(double theta, double dt, double tol, int n_cap, int p_cap, int fixed_p,
                          int fixed_n, int *pn, double *sc) {
  const int lane = threadIdx.x & 63;
  long key = 0x7fffffffffffL;  // G * 64 + n, smallest wins (ties to fewer squarings)
  int my_p = 0;
  if (lane < 60 && theta >= 0.0) {
    const int n = lane;
    const double x = ldexp(theta, -n);
    double f = 1.0, pw = x;
    for (int p = 1; p <= 30; ++p) {
      f *= (p + 1);
      pw *= x;  // x^(p+1)
      if (p >= 2 && ldexp(1.0, n) * pw / f * exp(x) <= tol) {
        my_p = p;
        key = (long)(p - 1 + n) * 64 + n;
        break;
      }
    }
  }
  long best = key;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const long other = __shfl_xor(best, o, 64);
    best = other < best ? other : best;
  }
  const int bn = (int)(best % 64);
  const int bp = __shfl(my_p, bn, 64);
  if (lane == 0) {
    int p = bp, n = bn, status = 0;
    bool found = best != 0x7fffffffffffL;
    if (fixed_p >= 2) {
      p = fixed_p;
      n = fixed_n;
      found = true;
    }
    if (!found || !(theta >= 0.0)) {
      status = 1;
      p = 2;
      n = 0;
    } else if (n > n_cap || p > p_cap) {
      status = 1;
      n = min(n, n_cap);
      p = min(p, p_cap);
    }
    pn[0] = p;
    pn[1] = n;
    pn[2] = status;
    sc[0] = ldexp(dt, -n);
    sc[1] = theta;
  }
}

__global__ __launch_bounds__(256) void k_norm(const double *__restrict__ H64,
                                              const double *__restrict__ u, int d, int M, int N,
                                              double dt, unsigned long long *theta_bits,
                                              SelectArgs sel) {
  extern __shared__ double sh[];
  // sh layout: coef[NRM_STEPS][M] then Hs[(M+1)][NRM_ROWS][NRM_COLS][2]
  double *coef = sh;
  double *Hs = sh + NRM_STEPS * M;
  __shared__ double red[4];
  const int t = threadIdx.x;
  const int cc = t & (NRM_COLS - 1), jj = t >> 4;
  const int c0 = blockIdx.y * NRM_COLS, j0 = blockIdx.x * NRM_STEPS;
  const int col = c0 + cc, j = j0 + jj;
  for (int e = t; e < NRM_STEPS * M; e += 256) {
    const int sj = e / M, k = e - sj * M;
    coef[e] = (j0 + sj < N) ? u[(long)k * N + j0 + sj] : 0.0;
  }
  double acc = 0.0;
  const int hs_elems = (M + 1) * NRM_ROWS * NRM_COLS;
  for (int r0 = 0; r0 < d; r0 += NRM_ROWS) {
    __syncthreads();
    for (int e = t; e < hs_elems; e += 256) {
      const int k = e / (NRM_ROWS * NRM_COLS);
      const int rem = e - k * NRM_ROWS * NRM_COLS;
      const int rr = rem / NRM_COLS, c = rem - rr * NRM_COLS;
      const int row = r0 + rr, cl = c0 + c;
      double vr = 0.0, vi = 0.0;
      if (row < d && cl < d) {
        const long o = ((long)k * d * d + (long)row * d + cl) * 2;
        vr = H64[o];
        vi = H64[o + 1];
      }
      Hs[2 * e] = vr;
      Hs[2 * e + 1] = vi;
    }
    __syncthreads();
    if (col < d && j < N) {
      for (int rr = 0; rr < NRM_ROWS; ++rr) {
        const int e0 = rr * NRM_COLS + cc;
        double hr = Hs[2 * e0], hi = Hs[2 * e0 + 1];
        for (int k = 0; k < M; ++k) {
          const double c = coef[jj * M + k];
          const int e = (k + 1) * NRM_ROWS * NRM_COLS + e0;
          hr += c * Hs[2 * e];
          hi += c * Hs[2 * e + 1];
        }
        acc += sqrt(hr * hr + hi * hi);
      }
    }
  }
  double v = (col < d && j < N) ? dt * acc : 0.0;
  v = wave_max(v);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  __shared__ int last;
  if (t == 0) {
    double m = red[0];
    for (int i = 1; i < 4; ++i) m = red[i] > m ? red[i] : m;
    atomicMax(theta_bits, (unsigned long long)__double_as_longlong(m));
    last = 0;
    if (sel.pn) {
      __threadfence();
      const unsigned total = gridDim.x * gridDim.y;
      last = atomicAdd(sel.ticket, 1u) == total - 1;
    }
  }
  __syncthreads();
  if (last && t < 64) {  // the last workgroup to finish chooses (p, n)
    __threadfence();
    const double theta =
        __longlong_as_double((long long)atomicAdd(theta_bits, 0ull));
    select_pn(theta, dt, sel.tol, sel.n_cap, sel.p_cap, sel.fixed_p, sel.fixed_n, sel.pn, sel.sc);
  }
}

hipError_t launch_norm(const double *H64, const double *u, int d, int M, int N, double dt,
                       unsigned long long *theta_bits, const SelectArgs &sel, hipStream_t st) {
  dim3 grid((N + NRM_STEPS - 1) / NRM_STEPS, (d + NRM_COLS - 1) / NRM_COLS);
  const size_t shm =
      sizeof(double) * (NRM_STEPS * M + 2 * (M + 1) * NRM_ROWS * NRM_COLS);
  hipLaunchKernelGGL(k_norm, grid, dim3(256), shm, st, H64, u, d, M, N, dt, theta_bits, sel);
  return hipGetLastError();
}

}  // namespace qoc
