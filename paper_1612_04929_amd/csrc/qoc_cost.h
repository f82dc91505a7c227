// Cost pieces as wavefront-level device functions, shared by the cost
// kernel and by the single-wavefront backward block sweep, which folds them
// into its own launch at padded d 16 (Sec. II.A and Table I: fidelity,
// per-step penalties C5, amplitude and variation terms C3, C4).
#pragma once

#include "qoc_device.h"
#include "qoc_kernels.h"

namespace qoc {

// Penalty pass of wavefront wi of W: the transitions j = wi, wi + W, ...
// (FP64: c_{j+1} = (1/S) sum_s sum_m w_m |psi_{j+1}^s[m]|^2 to out[2 + j],
// the largest | ||psi_{j+1}^s||^2 - ||psi_j^s||^2 |) and the amplitudes
// e = 64 wi + lane, ... (|u|^2 and control variations).  Results are
// wavefront totals, equal in every lane.
template <typename T>
__device__ inline void pen_wave(const SweepArgs<T> &a, long wi, long W, double &cpen, double &camp,
                                double &cvar, double &dmax) {
  const int dp = a.dp, S = a.S, N = a.N;
  const long set = 2L * S * dp;
  const int lane = threadIdx.x & 63;
  cpen = 0.0;
  dmax = 0.0;
  for (long j = wi; j < N; j += W) {
    double csum = 0.0;
    for (int s = 0; s < S; ++s) {
      const T *p0r = a.psi_buf + j * set + (long)s * dp, *p0i = p0r + (long)S * dp;
      const T *p1r = a.psi_buf + (j + 1) * set + (long)s * dp, *p1i = p1r + (long)S * dp;
      double n0 = 0.0, n1 = 0.0, pen = 0.0;
      for (int m = lane; m < dp; m += 64) {
        const double ar = p0r[m], ai = p0i[m], br = p1r[m], bi = p1i[m];
        const double q1 = br * br + bi * bi;
        n0 += ar * ar + ai * ai;
        n1 += q1;
        if (a.w64) pen += a.w64[m] * q1;
      }
      n0 = wave_sum(n0);
      n1 = wave_sum(n1);
      if (a.w64) csum += wave_sum(pen);
      dmax = fmax(dmax, fabs(n1 - n0));
    }
    const double cj = csum / S;
    if (lane == 0) a.out[2 + j] = cj;
    cpen += cj;
  }
  camp = 0.0;
  cvar = 0.0;
  const long MN = (long)a.M * N;
  for (long e = wi * 64 + lane; e < MN; e += W * 64) {
    const double x = a.u[e];
    camp += x * x;
    if (e % N >= 1) {
      const double dx = x - a.u[e - 1];
      cvar += dx * dx;
    }
  }
  camp = wave_sum(camp);
  cvar = wave_sum(cvar);
  dmax = wave_max(dmax);
}

// Fidelity and the final costate entry of state s, row m, for one
// wavefront of a single-wavefront sweep (lanes with kq == 0 own the rows):
// every state's overlap <T_q|psi_N^q> in FP64 (wavefront sums), z, F; the
// wavefront of state 0 writes F, C_fid and the overlaps; returns
// lambda_N^s[m] = -a_fid coef_s T_s[m] + pw_m psi_N^s[m] rounded to T.
template <typename T, int DP>
__device__ inline void lam_wave(const SweepArgs<T> &a, int s, int m, int kq, T &xr, T &xi) {
  const int d = a.d, S = a.S, N = a.N;
  const long set = 2L * S * DP;
  const T *psiN = a.psi_buf + (long)N * set;
  const int lane = threadIdx.x & 63;
  double zr = 0.0, zi = 0.0, Finc = 0.0, own_r = 0.0, own_i = 0.0;
  // every operand is read at a clamped row (and state) and masked afterwards
  // (a load under a lane-dependent condition gets a branch and a wait of its
  // own); the single-wavefront sweeps hold S <= 64 / DP states, so all the
  // overlaps' loads and wavefront sums are issued together
  constexpr int SMAX = 64 / DP;
  const int mc = m < d ? m : d - 1;
  const bool on = kq == 0 && m < d;
  // this state's target entry and penalty term, read with the overlaps' operands
  double tr = a.psiT64[((long)s * d + mc) * 2], ti = a.psiT64[((long)s * d + mc) * 2 + 1];
  const double wm = a.pw ? (double)a.pw[m] : 0.0;
  const double ysr = (double)psiN[s * DP + m], ysi = (double)psiN[(S + s) * DP + m];
  double pr[SMAX], pi[SMAX];
#pragma unroll
  for (int q = 0; q < SMAX; ++q) {
    const int qc = q < S ? q : S - 1;
    const double tr = a.psiT64[((long)qc * d + mc) * 2], ti = a.psiT64[((long)qc * d + mc) * 2 + 1];
    const double yr = (double)psiN[qc * DP + m], yi = (double)psiN[(S + qc) * DP + m];
    pr[q] = on && q < S ? tr * yr + ti * yi : 0.0;  // conj(T) psi
    pi[q] = on && q < S ? tr * yi - ti * yr : 0.0;
  }
#pragma unroll
  for (int q = 0; q < SMAX; ++q) {
    pr[q] = wave_sum(pr[q]);
    pi[q] = wave_sum(pi[q]);
  }
#pragma unroll
  for (int q = 0; q < SMAX; ++q) {
    if (q < S) {  // uniform
      zr += pr[q];
      zi += pi[q];
      Finc += pr[q] * pr[q] + pi[q] * pi[q];
      if (q == s) {
        own_r = pr[q];
        own_i = pi[q];
      }
      if (s == 0 && lane == 0) {
        a.zinfo[3 + 2 * q] = pr[q];
        a.zinfo[4 + 2 * q] = pi[q];
      }
    }
  }
  zr /= S;
  zi /= S;
  const double F = (a.fid_mode == 0) ? (zr * zr + zi * zi) : Finc / S;
  if (s == 0 && lane == 0) {
    a.out[1] = 1.0 - F;
    a.zinfo[0] = zr;
    a.zinfo[1] = zi;
    a.zinfo[2] = F;
  }
  const double cr = (a.fid_mode == 0 ? zr : own_r) / S, ci = (a.fid_mode == 0 ? zi : own_i) / S;
  tr = m < d ? tr : 0.0;
  ti = m < d ? ti : 0.0;
  double lr = -a.alpha_fid * (cr * tr - ci * ti);
  double li = -a.alpha_fid * (cr * ti + ci * tr);
  if (a.pw) {
    lr += wm * ysr;
    li += wm * ysi;
  }
  xr = (T)lr;
  xi = (T)li;
}

}  // namespace qoc
