// The total cost of one call and its norm drift, from the per-workgroup
// partials of the penalty pass (penalties, |u|^2, control variations, drift
// maxima) and the fidelity, reduced in a fixed order by one workgroup of 256
// threads: the last kernel of a call (k_total), or an extra workgroup of the
// padded-d-16 derivative kernel, which then runs it beside the steps.
#pragma once

#include "qoc_device.h"

namespace qoc {

struct TotalArgs {
  const double *part;   // 4 x npart partials
  int npart;
  const double *zinfo;  // [.., .., F, ..]
  double *out;          // out[0] receives C
  double alpha_fid, alpha_pen, alpha_amp, alpha_var;
  unsigned long long *drift_bits;
  // per-step terms of the forbidden-state / time-optimal pass (null: none):
  // ext_part[q] forbidden occupancies, ext_part[next + q] fidelities F_j
  const double *ext_part;
  int next;
  double alpha_time;
  int N;
};

__device__ inline void cost_total_block(const TotalArgs &a) {
  __shared__ double red[4];
  __shared__ double dred[4];
  double cpen = 0.0, camp = 0.0, cvar = 0.0, dmax = 0.0;
  for (int q = threadIdx.x; q < a.npart; q += blockDim.x) {
    cpen += a.part[q];
    camp += a.part[a.npart + q];
    cvar += a.part[2 * a.npart + q];
    dmax = fmax(dmax, a.part[3 * a.npart + q]);
  }
  double epen = 0.0, eF = 0.0;
  if (a.ext_part)  // block-uniform
    for (int q = threadIdx.x; q < a.next; q += blockDim.x) {
      epen += a.ext_part[q];
      eF += a.ext_part[a.next + q];
    }
  cpen = block_sum(cpen, red);
  camp = block_sum(camp, red);
  cvar = block_sum(cvar, red);
  epen = block_sum(epen, red);
  eF = block_sum(eF, red);
  dmax = wave_max(dmax);
  if ((threadIdx.x & 63) == 0) dred[threadIdx.x >> 6] = dmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double Cfid = 1.0 - a.zinfo[2];
    double C = a.alpha_fid * Cfid + a.alpha_pen * cpen + a.alpha_amp * camp + a.alpha_var * cvar;
    // C5 over forbidden states, and C_time = 1 - (1/N) sum_j F_j (C6 / C7)
    if (a.ext_part) C += a.alpha_pen * epen + a.alpha_time * (1.0 - eF / a.N);
    a.out[0] = C;
    const double m = fmax(fmax(dred[0], dred[1]), fmax(dred[2], dred[3]));
    *a.drift_bits = (unsigned long long)__double_as_longlong(m);
  }
}

}  // namespace qoc
