// Device-side choice of the Taylor order p and squaring count n from
// theta_max (Sec. III): the least total product count p - 1 + n whose
// truncation bound meets the tolerance, as the host rule does.
#pragma once

#include "qoc_device.h"

namespace qoc {

// (p, n) from theta by the rule of qoc_taylor_select, one wavefront, one
// lane per squaring count n; returns {p, n, status} and dt / 2^n.  status:
// 0 ok, 1 no pair / pair beyond the caps (error), 2 a fixed pair that
// misses the tolerance (warning).
__device__ inline void select_pn(double theta, double dt, double tol, int n_cap, int p_cap,
                                 int fixed_p, int fixed_n, int *pn, double *sc) {
  const int lane = threadIdx.x & 63;
  long key = 0x7fffffffffffL;  // G * 64 + n, smallest wins (ties to fewer squarings)
  int my_p = 0;
  if (lane < 60 && theta >= 0.0) {
    const int n = lane;
    const double x = ldexp(theta, -n), ex = exp(x), tn = ldexp(1.0, n);
    double f = 1.0, pw = x;
    for (int p = 1; p <= 30; ++p) {
      f *= (p + 1);
      pw *= x;  // x^(p+1)
      if (p >= 2 && tn * pw / f * ex <= tol) {
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
      // a fixed pair is used as given; status 2 flags that it misses the
      // tolerance at this theta
      p = fixed_p;
      n = fixed_n;
      found = true;
      const double x = ldexp(theta, -n);
      double f = 1.0, pw = x;
      for (int q = 1; q <= p; ++q) {
        f *= (q + 1);
        pw *= x;
      }
      if (!(ldexp(1.0, n) * pw / f * exp(x) <= tol)) status = 2;
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

}  // namespace qoc
