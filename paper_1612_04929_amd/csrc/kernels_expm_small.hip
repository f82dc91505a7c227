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
#include <type_traits>

#include "qoc_device.h"
#include "qoc_kernels.h"
#include "qoc_select.h"
#include "qoc_tile16.h"

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
      // every addend read before the first write (the output may be the
      // addend's own matrix), so the reads are not serialised behind writes
      T br[4], bi[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = (r0 + acc_row<T>(lane, v)) * DP + c0 + (lane & 15);
        br[v] = betaB != (T)0 ? Br[o] : (T)0;
        bi[v] = betaB != (T)0 ? Bi[o] : (T)0;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + acc_row<T>(lane, v), col = c0 + (lane & 15);
        const int o = row * DP + col;
        T vr = alpha * cr[q][v] + betaB * br[v], vi = alpha * ci[q][v] + betaB * bi[v];
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
    // X_j and the innermost Horner factor Q = I + X/p.  Each lane keeps its
    // EPL entries in registers across the control loop (no store inside
    // it), so the loads of several controls are in flight together.
    const T inv_p = (T)1 / (T)p;
    constexpr int EPL = (PL + GS - 1) / GS;
    T hr[EPL], hi[EPL];
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      const int e = gt + q * GS;
      hr[q] = e < PL ? Hf[e] : (T)0;
      hi[q] = e < PL ? Hf[PL + e] : (T)0;
    }
#pragma unroll 4
    for (int k = 0; k < M; ++k) {
      const T c = (T)u[(long)k * N + j];
      const T *Hk = Hf + (long)(k + 1) * 2 * PL;
#pragma unroll
      for (int q = 0; q < EPL; ++q) {
        const int e = gt + q * GS;
        if (e < PL) {
          hr[q] += c * Hk[e];
          hi[q] += c * Hk[PL + e];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
      const int e = gt + q * GS;
      if (e < PL) {
        const T xr = s * hi[q], xi = -s * hr[q];
        Xr[e] = xr;
        Xi[e] = xi;
        X[j * 2 * PL + e] = xr;
        X[j * 2 * PL + PL + e] = xi;
        const int r = e / DP, c = e - r * DP;
        Qr[e] = (r == c ? (T)1 : (T)0) + xr * inv_p;
        Qi[e] = xi * inv_p;
      }
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

// Padded d 16: one wavefront per step with the whole chain in registers.
// X is assembled into LDS once (its left-operand fragments are read from
// there); the Horner factor Q and the D levels stay in MFMA result layout
// and feed the next product directly as its right-hand operand (operand
// order of qoc_tile16.h); each squaring D^2 stages D once as a left operand.
//
// The same pass takes each step's FP64 1-norm ||dt H_j||_1 (true d, from
// the FP64 copies of the Hamiltonians), so no norm pass precedes it.  It
// runs speculatively with the pair held in sel.pn, the previous call's
// (recorded in pn[3]); every workgroup stores the largest norm of its
// steps, and the block-product kernel that follows reduces them, chooses
// this call's (p, n) and, only where that differs from the pair used,
// recomputes the steps it owns.  The results are those of choosing first.
template <typename T, bool NORM>
__device__ __forceinline__ unsigned long long expm16_step(long j, int p, int n, T s,
                                                          const T *__restrict__ Hf,
                                                          const double *__restrict__ u, int M,
                                                          int N, T *X, T *Dlev, T *Dh,
                                                          const Norm16 &nm, T *Xr, T *Xi, T *tr,
                                                          T *ti) {
  constexpr int PL = 256;
  const int lane = threadIdx.x & 63, col = lane & 15;
  const long lev = (long)N * 2 * PL;
  const int d = nm.d;
  const long dd = (long)d * d;
  // X_j = -i s H_j: entries lane + 64 q of each plane (row lane / 16 + 4 q,
  // column lane % 16); with NORM also H_j in FP64.  The FP64 entries are
  // read at clamped (always valid) positions, summed, and masked only at
  // the end: a load under a lane-dependent condition would sit in a branch
  // of its own, and a mask applied at once would wait for the load there,
  // before the control terms' loads are issued.
  // The drift term's offset is an opaque zero, so its loads are issued here
  // beside the others rather than hoisted out of the caller's step loop
  // (where the copy into the accumulators would wait for them on their own).
  int z0;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z0));
  T hr[4], hi[4];
  double gr[4], gi[4];
  int go[4];     // FP64 entry offset (complex pairs) of row, column
  bool gin[4];   // inside the true d x d block
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hr[q] = Hf[z0 + lane + 64 * q];
    hi[q] = Hf[z0 + PL + lane + 64 * q];
    const int row = (lane >> 4) + 4 * q;
    gin[q] = row < d && col < d;
    go[q] = ((row < d ? row : d - 1) * d + (col < d ? col : d - 1)) * 2;
    if (NORM) {
      const double2 g = *reinterpret_cast<const double2 *>(nm.H64 + z0 + go[q]);
      gr[q] = g.x;
      gi[q] = g.y;
    }
  }
  // controls in groups of four: every load of a group is issued before the
  // first use (a short group reads the last control again with a zero
  // amplitude, which adds exact zeros)
  for (int k0 = 0; k0 < M; k0 += 4) {
    double cu[4];
    T ar[4][4], ai[4][4];
    double2 ag[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = k0 + t < M ? k0 + t : M - 1;
      cu[t] = u[(long)k * N + j];
      const T *Hk = Hf + (long)(k + 1) * 2 * PL;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ar[t][q] = Hk[lane + 64 * q];
        ai[t][q] = Hk[PL + lane + 64 * q];
        if (NORM) ag[t][q] = *reinterpret_cast<const double2 *>(nm.H64 + (k + 1) * dd * 2 + go[q]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double cd = k0 + t < M ? cu[t] : 0.0;
      const T c = (T)cd;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        hr[q] += c * ar[t][q];
        hi[q] += c * ai[t][q];
        if (NORM) {
          gr[q] += cd * ag[t][q].x;
          gi[q] += cd * ag[t][q].y;
        }
      }
    }
  }
  if (NORM) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      gr[q] = gin[q] ? gr[q] : 0.0;
      gi[q] = gin[q] ? gi[q] : 0.0;
    }
  }
  unsigned long long bits = 0ull;
  if (NORM) {
    // column sums over the four rows of this lane, then over the four
    // lanes of the column; the largest column sum of the step
    double cs = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) cs += sqrt(gr[q] * gr[q] + gi[q] * gi[q]);
    cs += __shfl_xor(cs, 16, 64);
    cs += __shfl_xor(cs, 32, 64);
    const double x = nm.dt * cs;
    bits = (x != x) ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(x);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = lane + 64 * q;
    const T xr = s * hi[q], xi = -s * hr[q];
    Xr[e] = xr;
    Xi[e] = xi;
    X[j * 2 * PL + e] = xr;
    X[j * 2 * PL + PL + e] = xi;
  }
  wave_lds_sync();
  Frag<T> fX;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    fX.r[t] = Xr[col * 16 + acc_row<T>(lane, t)];
    fX.i[t] = Xi[col * 16 + acc_row<T>(lane, t)];
  }
  // Q = I + X / p, in result layout
  const T inv_p = (T)1 / (T)p;
  CTile<T> Q;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = acc_row<T>(lane, v);
    Q.r[v] = (row == col ? (T)1 : (T)0) + Xr[row * 16 + col] * inv_p;
    Q.i[v] = Xi[row * 16 + col] * inv_p;
  }
  // Q <- I + (1/k) X Q, k = p-1 .. 2
  for (int k = p - 1; k >= 2; --k) {
    CTile<T> acc = ctile_zero<T>();
    cmma(fX, asB(Q), acc);
    const T ik = (T)1 / (T)k;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Q.r[v] = acc.r[v] * ik + (acc_row<T>(lane, v) == col ? (T)1 : (T)0);
      Q.i[v] = acc.i[v] * ik;
    }
  }
  // D^(0) = X Q at slot n, D^(i+1) = 2 D^(i) + D^(i) D^(i) at slot n - i - 1
  CTile<T> Dt = ctile_zero<T>();
  cmma(fX, asB(Q), Dt);
  auto put = [&](T *g) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int o = acc_row<T>(lane, v) * 16 + col;
      g[o] = Dt.r[v];
      g[PL + o] = Dt.i[v];
    }
  };
  put(Dlev + (long)n * lev + j * 2 * PL);
  for (int i = 0; i < n; ++i) {
    wave_lds_sync();
    stage(tr, ti, Dt);
    wave_lds_sync();
    const Frag<T> aD = fragA(tr, ti);
    CTile<T> acc = ctile_zero<T>();
    cmma(aD, asB(Dt), acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Dt.r[v] = (T)2 * Dt.r[v] + acc.r[v];
      Dt.i[v] = (T)2 * Dt.i[v] + acc.i[v];
    }
    put(Dlev + (long)(n - i - 1) * lev + j * 2 * PL);
  }
  if (Dh) {  // uniform: D^H[col][row] = conj(D[row][col])
    T *o = Dh + j * 2 * PL;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = acc_row<T>(lane, v);
      o[col * 16 + row] = Dt.r[v];
      o[PL + col * 16 + row] = -Dt.i[v];
    }
  }
  wave_lds_sync();  // X and the staging tile are rewritten by the next step
  return bits;
}

constexpr int E16_WAVES = 4;  // wavefronts (steps in flight) per workgroup of k_expm16

// LDS of one wavefront's step: X (two planes) and a staging tile
template <typename T> struct Expm16Lds {
  T x[2][256];
  T t[2][16 * A16_LD];
};

template <typename T>
__global__ __launch_bounds__(64 * E16_WAVES) void k_expm16(const T *__restrict__ Hf,
                                                const double *__restrict__ u, int M, int N,
                                                T *X, T *Dlev, T *Dh, Norm16 nm) {
  __shared__ __align__(16) Expm16Lds<T> lds[E16_WAVES];
  __shared__ unsigned long long red[E16_WAVES];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int *pn = nm.sel.pn;
  const int p0 = pn[0], n0 = pn[1];
  // no pair yet (first call): a placeholder whose results are redone
  const int p = p0 >= 2 ? p0 : 2, n = p0 >= 2 ? n0 : 0;
  const T s = (T)nm.sel.sc[0];
  Expm16Lds<T> &L = lds[w];
  unsigned long long vmax = 0ull;  // largest ||dt H_j||_1 bit pattern of this wavefront
  for (long j = (long)blockIdx.x * E16_WAVES + w; j < N; j += (long)gridDim.x * E16_WAVES) {
    const unsigned long long b = expm16_step<T, true>(j, p, n, s, Hf, u, M, N, X, Dlev, Dh, nm,
                                                      L.x[0], L.x[1], L.t[0], L.t[1]);
    vmax = b > vmax ? b : vmax;
  }
  vmax = wave_max(vmax);
  if (lane == 0) red[w] = vmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = red[0];
    for (int i = 1; i < E16_WAVES; ++i) m = red[i] > m ? red[i] : m;
    nm.part[blockIdx.x] = m;
    if (blockIdx.x == 0) pn[3] = (p0 & 0xffff) | (n0 << 16);  // the pair used
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

// Block products for padded d 16 as a pairwise tree: one workgroup per
// block, the block's step matrices staged in LDS TCH at a time and reduced
// pairwise (later factor on the left, D-form P = A + B + A B, each product
// written over its earlier factor's slot), a wavefront per pair; each
// chunk's product is then folded into the running E the same way.  The
// dependent chain is about log2(L) + L / (4 TCH) products instead of L - 1.
template <typename T> struct TreeCh {
  // chunk slots + the running product in 64 KB of LDS
  static constexpr int value = (64 * 1024) / (2 * 256 * (int)sizeof(T)) - 1;
};

// O = P + A + B for one 16 x 16 tile (P = A B in MFMA result layout, LDS
// matrices with row stride 16); all reads before the writes, so O may be B.
template <typename T>
__device__ __forceinline__ void dform_store(int lane, const v4<T> &pr, const v4<T> &pi,
                                            const T *A, const T *B, T *O) {
  constexpr int PL = 256;
  T ar[4], ai[4], br[4], bi[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int o = acc_row<T>(lane, v) * 16 + (lane & 15);
    ar[v] = A[o];
    ai[v] = A[PL + o];
    br[v] = B[o];
    bi[v] = B[PL + o];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int o = acc_row<T>(lane, v) * 16 + (lane & 15);
    O[o] = pr[v] + ar[v] + br[v];
    O[PL + o] = pi[v] + ai[v] + bi[v];
  }
}

//
// With pick.nm.part set, the workgroup first reduces the norm maxima of the
// exponential pass, chooses (p, n) (workgroup 0 publishes it), and, if the
// pair differs from the one that pass used, recomputes the exponentials of
// its own steps before forming their product.
template <typename T> struct TreeWaves {  // wavefronts per block-product workgroup
  // FP64: four, so their recompute buffers fit in the product slots
  static constexpr int value = sizeof(T) == 4 ? 8 : 4;
};
template <typename T>
__global__ __launch_bounds__(64 * TreeWaves<T>::value) void k_blockprod_tree16(
    const T *__restrict__ D, int N, int L, T *E, T *Eh, Pick16<T> pick) {
  constexpr int PL = 256, CH = TreeCh<T>::value;
  constexpr int TW = TreeWaves<T>::value, NT = 64 * TW;
  static_assert(TW * sizeof(Expm16Lds<T>) <= sizeof(T) * (CH + 1) * 2 * PL, "recompute buffers");
  constexpr int MAXT = 2;  // lds_product<T, 16, 1> tile slots (one used)
  __shared__ __align__(16) T m[CH + 1][2 * PL];  // slot CH: the running product
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long b = blockIdx.x;
  const long start = b * L, end = min((long)N, start + L);
  if (pick.nm.part) {  // uniform
    __shared__ unsigned long long tred[TW];
    __shared__ int spn[4];
    __shared__ double ssc[2];
    const Norm16 &nm = pick.nm;
    unsigned long long v = 0ull;
    for (int i = threadIdx.x; i < pick.nparts; i += NT) v = nm.part[i] > v ? nm.part[i] : v;
    v = wave_max(v);
    if (lane == 0) tred[w] = v;
    __syncthreads();
    unsigned long long tb = tred[0];
    for (int i = 1; i < TW; ++i) tb = tred[i] > tb ? tred[i] : tb;
    if (w == 0)
      select_pn(__longlong_as_double((long long)tb), nm.dt, nm.sel.tol, nm.sel.n_cap,
                nm.sel.p_cap, nm.sel.fixed_p, nm.sel.fixed_n, spn, ssc);
    __syncthreads();
    const int p = spn[0], n = spn[1];
    const int used = nm.sel.pn[3];
    if (b == 0 && threadIdx.x == 0) {
      nm.sel.pn[0] = spn[0];
      nm.sel.pn[1] = spn[1];
      nm.sel.pn[2] = spn[2];
      nm.sel.sc[0] = ssc[0];
      nm.sel.sc[1] = ssc[1];
      nm.theta_bits[0] = tb;
    }
    if (p != (used & 0xffff) || n != (used >> 16)) {  // uniform: redo this block's steps
      Expm16Lds<T> &S = reinterpret_cast<Expm16Lds<T> *>(&m[0][0])[w];
      const T sc = (T)ssc[0];
      for (long j = start + w; j < end; j += TW)
        expm16_step<T, false>(j, p, n, sc, pick.Hf, pick.u, pick.M, N, pick.X, pick.Dlev,
                              pick.Dh, nm, S.x[0], S.x[1], S.t[0], S.t[1]);
      __threadfence_block();
      __syncthreads();
    }
  }
  // with sub-block products wanted, chunks hold whole sub-blocks, and the
  // products of the first tree levels (SUB16 steps) are stored on the way;
  // a block that fits all CH + 1 slots is one chunk (the running-product
  // slot is free until its tree is done)
  const bool subs = pick.Es != nullptr;  // uniform
  const int chunk = L <= CH + 1 ? L : (subs ? (CH / SUB16) * SUB16 : CH);
  auto store_subs = [&](long c0, int cnt) {
    const int ns = (cnt + SUB16 - 1) / SUB16;
    const long s0 = c0 / SUB16;
    for (int e = threadIdx.x; e < ns * PL; e += NT) {
      const int q = e / PL, o = e - q * PL, r = o >> 4, c = o & 15;
      const T *src = m[q * SUB16];
      T *es = pick.Es + (s0 + q) * 2 * PL, *eh = pick.Ehs + (s0 + q) * 2 * PL;
      es[o] = src[o];
      es[PL + o] = src[PL + o];
      eh[o] = src[c * 16 + r];
      eh[PL + o] = -src[PL + c * 16 + r];
    }
    __syncthreads();  // before the next level overwrites the slots
  };
  for (long c0 = start; c0 < end; c0 += chunk) {
    const int cnt = (int)min((long)chunk, end - c0);
    {
      typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type V;
      constexpr int VN = 16 / sizeof(T);
      const V *src = reinterpret_cast<const V *>(D + c0 * 2 * PL);
      V *dst = reinterpret_cast<V *>(&m[0][0]);
      const int nv = cnt * 2 * PL / VN;
      // eight 16-byte loads in flight per lane before the LDS stores (at a
      // clamped index, the stores masked: no load under a condition)
      for (int e = threadIdx.x; e < nv; e += 8 * NT) {
        V t[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) t[q] = src[min(e + q * NT, nv - 1)];
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (e + q * NT < nv) dst[e + q * NT] = t[q];
      }
    }
    __syncthreads();
    bool stored = !subs;
    for (int stride = 1; stride < cnt; stride *= 2) {
      const int npair = (cnt - stride + 2 * stride - 1) / (2 * stride);
      for (int q = w; q < npair; q += TW) {
        T *B = m[q * 2 * stride], *A = m[q * 2 * stride + stride];
        v4<T> cr[MAXT], ci[MAXT];
        lds_product<T, 16, 1>(A, A + PL, B, B + PL, cr, ci);
        dform_store(lane, cr[0], ci[0], A, B, B);
      }
      __syncthreads();
      if (!stored && 2 * stride == SUB16) {  // slot q SUB16: sub-block q's product
        store_subs(c0, cnt);
        stored = true;
      }
    }
    if (!stored) store_subs(c0, cnt);  // a chunk of at most half a sub-block
    if (c0 == start) {  // uniform: the first chunk's product starts E
      for (int e = threadIdx.x; e < 2 * PL; e += NT) m[CH][e] = m[0][e];
    } else if (w == 0) {  // E <- C + E + C E, C the later chunk
      T *C = m[0], *R = m[CH];
      v4<T> cr[MAXT], ci[MAXT];
      lds_product<T, 16, 1>(C, C + PL, R, R + PL, cr, ci);
      dform_store(lane, cr[0], ci[0], C, R, R);
    }
    __syncthreads();
  }
  const T *R = m[CH];
  for (int e = threadIdx.x; e < 2 * PL; e += NT) E[b * 2 * PL + e] = R[e];
  if (Eh) {
    for (int e = threadIdx.x; e < PL; e += NT) {
      const int r = e >> 4, c = e & 15;
      Eh[b * 2 * PL + e] = R[c * 16 + r];
      Eh[b * 2 * PL + PL + e] = -R[PL + c * 16 + r];
    }
  }
}

template <typename T> bool small_expm_ok(int dp) {
  return dp == 16 || dp == 32 || (dp == 48 && sizeof(T) == 4);
}

template <typename T>
hipError_t launch_expm_small(const T *Hf, const double *u, int dp, int M, int N, const int *pn,
                             const double *sc, T *X, T *Dlev, T *Dh, hipStream_t st) {
  switch (dp) {
    case 16:
      return hipErrorInvalidValue;  // launch_expm16 (norm and pair choice fused)
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

template <typename T> unsigned expm16_blocks(int N) {
  return (unsigned)std::min<long>((N + E16_WAVES - 1) / E16_WAVES, 4096);
}

template <typename T>
hipError_t launch_expm16(const T *Hf, const double *u, int M, int N, T *X, T *Dlev, T *Dh,
                         const Norm16 &nm, hipStream_t st) {
  hipLaunchKernelGGL(k_expm16<T>, dim3(expm16_blocks<T>(N)), dim3(64 * E16_WAVES), 0, st, Hf,
                     u, M, N, X, Dlev, Dh, nm);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_blockprod_small(const T *D, int dp, int N, int L, int nb, T *E, T *Eh,
                                  const Pick16<T> *pick, hipStream_t st) {
  switch (dp) {
    case 16: {
      Pick16<T> pk{};
      if (pick) pk = *pick;
      hipLaunchKernelGGL(k_blockprod_tree16<T>, dim3(nb), dim3(64 * TreeWaves<T>::value), 0, st,
                         D, N, L, E, Eh, pk);
      break;
    }
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
template hipError_t launch_expm16<float>(const float *, const double *, int, int, float *,
                                         float *, float *, const Norm16 &, hipStream_t);
template hipError_t launch_expm16<double>(const double *, const double *, int, int, double *,
                                          double *, double *, const Norm16 &, hipStream_t);
template hipError_t launch_blockprod_small<float>(const float *, int, int, int, int, float *,
                                                  float *, const Pick16<float> *, hipStream_t);
template hipError_t launch_blockprod_small<double>(const double *, int, int, int, int, double *,
                                                   double *, const Pick16<double> *,
                                                   hipStream_t);
template unsigned expm16_blocks<float>(int);
template unsigned expm16_blocks<double>(int);

}  // namespace qoc
