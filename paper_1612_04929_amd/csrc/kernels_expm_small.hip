// Whole Taylor + squaring chain of one step in LDS, for padded d <= 48.
//
// Same D-form recurrences as kernels_expm.hip (Sec. III, eq. 6):
//   X = -i (dt/2^n) H_j,  Q <- I + X/p,  Q <- I + (1/k) X Q (k = p-1..2),
//   D^(0) = X Q,  D^(i+1) = 2 D^(i) + D^(i) D^(i),
// but one group of GW wavefronts keeps X and the running matrix in LDS for
// all p - 1 + n products of its step, so a step costs one launch and no
// HBM round trips between products.  GW = 1 (a wavefront per step) for
// d_pad = 16; GW = 4 otherwise.  X and every D^(i) are written to global
// memory for the sweeps and the adjoint.
//
// Also: block products E_b = U_{end-1} ... U_{start} - I of the two-level
// sweep, one group per block, accumulated in LDS in D-form
// (E <- D + E + D E).
//
// When asked for (Dh / Eh not null), both kernels also write the conjugate
// transposes D^H and E^H, read from the LDS copy they already hold: the
// costate sweeps then stream rows of D^H with the same contiguous 16-byte
// loads as the state sweeps stream rows of D.
#include "qoc_device.h"
#include "qoc_kernels.h"

namespace qoc {

template <int GW> __device__ __forceinline__ void gsync() {
  if (GW == 4) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// acc[t] (t-th tile owned by this wave) = A * B over LDS matrices (DP x DP
// planar, row stride DP).  Tiles of the DP/16 x DP/16 grid are dealt to the
// GW waves round robin.
template <typename T, int DP, int GW>
__device__ __forceinline__ void lds_product(const T *Ar, const T *Ai, const T *Br, const T *Bi,
                                            v4<T> (&cr)[(DP / 16) * (DP / 16) / GW + 1],
                                            v4<T> (&ci)[(DP / 16) * (DP / 16) / GW + 1]) {
  constexpr int T1 = DP / 16, NT = T1 * T1;
  constexpr int MAXT = NT / GW + 1;
  const int gw = (threadIdx.x >> 6) % GW, lane = threadIdx.x & 63;
  const int i = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = gw + q * GW;
    cr[q] = vzero<T>();
    ci[q] = vzero<T>();
    if (t < NT) {
      const int r0 = (t / T1) * 16, c0 = (t % T1) * 16;
#pragma unroll
      for (int k = 0; k < DP; k += 4) {
        const T ar = Ar[(r0 + i) * DP + k + kk], ai = Ai[(r0 + i) * DP + k + kk];
        const T br = Br[(k + kk) * DP + c0 + i], bi = Bi[(k + kk) * DP + c0 + i];
        cr[q] = mfma4(ar, br, cr[q]);
        cr[q] = mfma4(-ai, bi, cr[q]);
        ci[q] = mfma4(ar, bi, ci[q]);
        ci[q] = mfma4(ai, br, ci[q]);
      }
    }
  }
}

// out = alpha * acc + betaB * B + gamma * I written to LDS (and optionally
// to global), for the tiles owned by this wave.
template <typename T, int DP, int GW>
__device__ __forceinline__ void lds_epilogue(const v4<T> (&cr)[(DP / 16) * (DP / 16) / GW + 1],
                                             const v4<T> (&ci)[(DP / 16) * (DP / 16) / GW + 1],
                                             T alpha, const T *Br, const T *Bi, T betaB, T gamma,
                                             T *Or, T *Oi, T *gr, T *gi) {
  constexpr int T1 = DP / 16, NT = T1 * T1;
  constexpr int MAXT = NT / GW + 1;
  const int gw = (threadIdx.x >> 6) % GW, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < MAXT; ++q) {
    const int t = gw + q * GW;
    if (t < NT) {
      const int r0 = (t / T1) * 16, c0 = (t % T1) * 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + acc_row<T>(lane, v), col = c0 + (lane & 15);
        const int o = row * DP + col;
        T vr = alpha * cr[q][v], vi = alpha * ci[q][v];
        if (betaB != (T)0) {
          vr += betaB * Br[o];
          vi += betaB * Bi[o];
        }
        if (row == col) vr += gamma;
        Or[o] = vr;
        Oi[o] = vi;
        if (gr) {
          gr[o] = vr;
          gi[o] = vi;
        }
      }
    }
  }
}

template <typename T, int DP, int GW>
__global__ __launch_bounds__(256) void k_expm_small(const T *__restrict__ Hf,
                                                    const double *__restrict__ u, int M, int N,
                                                    const int *__restrict__ pn,
                                                    const double *__restrict__ sc, T *X,
                                                    T *Dlev, T *Dh) {
  constexpr int GS = 64 * GW, GPB = 4 / GW;
  constexpr int PL = DP * DP;
  constexpr int MAXT = (DP / 16) * (DP / 16) / GW + 1;
  __shared__ T lds[GPB][4 * PL];
  const int w = threadIdx.x >> 6, gt = threadIdx.x % GS;
  const int p = pn[0], n = pn[1];
  const T s = (T)sc[0];
  T *Xr = lds[w / GW], *Xi = Xr + PL, *Qr = Xi + PL, *Qi = Qr + PL;
  const long lev = (long)N * 2 * PL;
  for (long j = (long)blockIdx.x * GPB + w / GW; j < N; j += (long)gridDim.x * GPB) {
    // X_j and the innermost Horner factor Q = I + X/p
    const T inv_p = (T)1 / (T)p;
    for (int e = gt; e < PL; e += GS) {
      T hr = Hf[e], hi = Hf[PL + e];
      for (int k = 0; k < M; ++k) {
        const T c = (T)u[(long)k * N + j];
        hr += c * Hf[(long)(k + 1) * 2 * PL + e];
        hi += c * Hf[(long)(k + 1) * 2 * PL + PL + e];
      }
      const T xr = s * hi, xi = -s * hr;
      Xr[e] = xr;
      Xi[e] = xi;
      X[j * 2 * PL + e] = xr;
      X[j * 2 * PL + PL + e] = xi;
      const int r = e / DP, c = e - r * DP;
      Qr[e] = (r == c ? (T)1 : (T)0) + xr * inv_p;
      Qi[e] = xi * inv_p;
    }
    gsync<GW>();
    v4<T> cr[MAXT], ci[MAXT];
    for (int k = p - 1; k >= 2; --k) {
      lds_product<T, DP, GW>(Xr, Xi, Qr, Qi, cr, ci);
      gsync<GW>();
      lds_epilogue<T, DP, GW>(cr, ci, (T)1 / (T)k, nullptr, nullptr, (T)0, (T)1, Qr, Qi,
                              nullptr, nullptr);
      gsync<GW>();
    }
    // D^(0) = X Q.  Level i is stored at slot n - i, so the final D^(n) is
    // always slot 0 whatever n the device chose.
    T *D0 = Dlev + (long)n * lev + j * 2 * PL;
    lds_product<T, DP, GW>(Xr, Xi, Qr, Qi, cr, ci);
    gsync<GW>();
    lds_epilogue<T, DP, GW>(cr, ci, (T)1, nullptr, nullptr, (T)0, (T)0, Qr, Qi, D0, D0 + PL);
    gsync<GW>();
    for (int i = 0; i < n; ++i) {
      T *Di = Dlev + (long)(n - i - 1) * lev + j * 2 * PL;
      lds_product<T, DP, GW>(Qr, Qi, Qr, Qi, cr, ci);
      gsync<GW>();
      lds_epilogue<T, DP, GW>(cr, ci, (T)1, Qr, Qi, (T)2, (T)0, Qr, Qi, Di, Di + PL);
      gsync<GW>();
    }
    if (Dh) {  // uniform
      T *o = Dh + j * 2 * PL;
      for (int e = gt; e < PL; e += GS) {
        const int r = e / DP, c = e - r * DP;
        o[e] = Qr[c * DP + r];
        o[PL + e] = -Qi[c * DP + r];
      }
      gsync<GW>();
    }
  }
}

// E_b = U_{end-1} ... U_{start} - I, D-form E <- D_j + E + D_j E, with the
// step matrices of the next RD steps held in a register ring.
template <typename T, int DP, int GW>
__global__ __launch_bounds__(256) void k_blockprod_small(const T *__restrict__ D, int N, int L,
                                                         int nb, T *E, T *Eh) {
  constexpr int GS = 64 * GW, GPB = 4 / GW;
  constexpr int PL = DP * DP;
  constexpr int MAXT = (DP / 16) * (DP / 16) / GW + 1;
  constexpr int EPL = (2 * PL + GS - 1) / GS;  // ring elements per lane per step
  constexpr int RD = 4;
  __shared__ T lds[GPB][4 * PL];
  const int w = threadIdx.x >> 6, gt = threadIdx.x % GS;
  T *Er = lds[w / GW], *Ei = Er + PL, *Dr = Ei + PL, *Di = Dr + PL;
  constexpr int T1 = DP / 16, NT = T1 * T1;
  const int gw = (threadIdx.x >> 6) % GW, lane = threadIdx.x & 63;
  for (long b = (long)blockIdx.x * GPB + w / GW; b < nb; b += (long)gridDim.x * GPB) {
    const long start = b * L, end = min((long)N, start + L);
    T ring[RD][EPL];
#pragma unroll
    for (int q = 0; q < RD; ++q)
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int idx = e * GS + gt;
        const long j = start + 1 + q;
        ring[q][e] = (j < end && idx < 2 * PL) ? D[j * 2 * PL + idx] : (T)0;
      }
    for (int e = gt; e < 2 * PL; e += GS) Er[e] = D[start * 2 * PL + e];
    for (long j0 = start + 1; j0 < end; j0 += RD) {
#pragma unroll
      for (int q = 0; q < RD; ++q) {
        const long j = j0 + q;
        if (j < end) {
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            const int idx = e * GS + gt;
            if (idx < 2 * PL) Dr[idx] = ring[q][e];
          }
          gsync<GW>();
          if (j + RD < end) {
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
              const int idx = e * GS + gt;
              ring[q][e] = (idx < 2 * PL) ? D[(j + RD) * 2 * PL + idx] : (T)0;
            }
          }
          v4<T> cr[MAXT], ci[MAXT];
          lds_product<T, DP, GW>(Dr, Di, Er, Ei, cr, ci);
          gsync<GW>();
#pragma unroll
          for (int qq = 0; qq < MAXT; ++qq) {
            const int t = gw + qq * GW;
            if (t < NT) {
              const int r0 = (t / T1) * 16, c0 = (t % T1) * 16;
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int o = (r0 + acc_row<T>(lane, v)) * DP + c0 + (lane & 15);
                Er[o] = cr[qq][v] + Er[o] + Dr[o];
                Ei[o] = ci[qq][v] + Ei[o] + Di[o];
              }
            }
          }
          gsync<GW>();
        }
      }
    }
    for (int e = gt; e < 2 * PL; e += GS) E[b * 2 * PL + e] = Er[e];
    if (Eh) {  // uniform
      for (int e = gt; e < PL; e += GS) {
        const int r = e / DP, c = e - r * DP;
        Eh[b * 2 * PL + e] = Er[c * DP + r];
        Eh[b * 2 * PL + PL + e] = -Ei[c * DP + r];
      }
    }
    gsync<GW>();
  }
}

template <typename T> bool small_expm_ok(int dp) {
  return dp == 16 || dp == 32 || (dp == 48 && sizeof(T) == 4);
}

template <typename T>
hipError_t launch_expm_small(const T *Hf, const double *u, int dp, int M, int N, const int *pn,
                             const double *sc, T *X, T *Dlev, T *Dh, hipStream_t st) {
  switch (dp) {
    case 16: {
      const long blocks = std::min<long>((N + 3) / 4, 4096);
      hipLaunchKernelGGL((k_expm_small<T, 16, 1>), dim3(blocks), dim3(256), 0, st, Hf, u, M, N,
                         pn, sc, X, Dlev, Dh);
      break;
    }
    case 32: {
      const long blocks = std::min<long>(N, 4096);
      hipLaunchKernelGGL((k_expm_small<T, 32, 4>), dim3(blocks), dim3(256), 0, st, Hf, u, M, N,
                         pn, sc, X, Dlev, Dh);
      break;
    }
    case 48: {
      if constexpr (sizeof(T) == 4) {
        const long blocks = std::min<long>(N, 4096);
        hipLaunchKernelGGL((k_expm_small<T, 48, 4>), dim3(blocks), dim3(256), 0, st, Hf, u, M,
                           N, pn, sc, X, Dlev, Dh);
        break;
      }
      return hipErrorInvalidValue;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_blockprod_small(const T *D, int dp, int N, int L, int nb, T *E, T *Eh,
                                  hipStream_t st) {
  switch (dp) {
    case 16:
      hipLaunchKernelGGL((k_blockprod_small<T, 16, 1>), dim3((nb + 3) / 4), dim3(256), 0, st, D,
                         N, L, nb, E, Eh);
      break;
    case 32:
      hipLaunchKernelGGL((k_blockprod_small<T, 32, 4>), dim3(nb), dim3(256), 0, st, D, N, L, nb,
                         E, Eh);
      break;
    case 48:
      if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL((k_blockprod_small<T, 48, 4>), dim3(nb), dim3(256), 0, st, D, N, L,
                           nb, E, Eh);
        break;
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template bool small_expm_ok<float>(int);
template bool small_expm_ok<double>(int);
template hipError_t launch_expm_small<float>(const float *, const double *, int, int, int,
                                             const int *, const double *, float *, float *,
                                             float *, hipStream_t);
template hipError_t launch_expm_small<double>(const double *, const double *, int, int, int,
                                              const int *, const double *, double *, double *,
                                              double *, hipStream_t);
template hipError_t launch_blockprod_small<float>(const float *, int, int, int, int, float *,
                                                  float *, hipStream_t);
template hipError_t launch_blockprod_small<double>(const double *, int, int, int, int, double *,
                                                   double *, hipStream_t);

}  // namespace qoc
