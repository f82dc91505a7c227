// Host-side launchers of the libqoc HIP kernels (implemented in the *.hip
// files of this directory, instantiated for float and double).
#pragma once
#include <hip/hip_runtime.h>

#include "qoc_total.h"

namespace qoc {

// Batched complex product with a fused epilogue, one matrix per step:
//   C_j  = alpha P + betaA A_j + betaB B_j + gamma I + sum_i xc[i] Xi_j
//   C2_j = c2P P + c2A A_j + c2B B_j + g2 I + sum_i xc2[i] Xi_j  (if C2)
// with P = op(A_j) B_j.  Matrices are dp x dp planar (re plane, then im
// plane), matrix j of a stack at base + j * stride (the extra addends Xi
// and C2 at base + j * strideC).  op(A) = A (opa = 0) or A^H (opa = 1).
template <typename T> struct StageArgs {
  const T *A;
  long strideA;
  const T *B;
  long strideB;
  T *C;
  long strideC;
  int nmat, dp;
  T alpha, betaA, betaB, gamma;
  int bf3;  // 1: bf16x3 split products (FP32 storage, padded d multiple of 64)
  int nx;                 // extra addends used (0..3)
  const T *xadd[3];
  T xc[3];
  T *C2;                  // optional second output (null: none)
  T c2P, c2A, c2B, g2;
  T xc2[3];
  // segments (seg > 0): matrix j = b seg + i of a stack sits at
  // base + b * seg{A,B,C} + i * stride (the per-block trees of the block
  // products); seg = 0: base + j * stride
  int seg;
  long segA, segB, segC;
};

// X_j = -i s (H_0 + sum_k u_{k,j} H_k) for all steps and, when Q is not
// null, Q_j = I + X_j / p (the innermost Horner factor).
template <typename T>
hipError_t launch_assemble(const T *Hf, const double *u, int dp, int M, int N, T s, T inv_p,
                           T *X, T *Q, hipStream_t st);

template <typename T> hipError_t launch_stage(int opa, const StageArgs<T> &a, hipStream_t st);

// Whether launch_stage runs bf16x3 split products for padded d dp (when
// StageArgs.bf3 asks for them); otherwise the chain precision's kernels run.
bool stage_bf3_ok(int dp);

// Each workgroup of the norm kernel folds its maximum into `acc` (atomic
// max on the FP64 bit pattern) and takes a number from `ticket`; the last
// one (both words zero at the first launch and cleared by that workgroup)
// writes theta_bits[0], clears theta_bits[1] (the drift word of the call)
// and, when pn is not null, chooses (p, n): pn = {p, n, status},
// sc = {dt / 2^n, theta}; status 1 when the pair exceeds n_cap / p_cap or
// none meets tol, 2 when a fixed pair (fixed_p >= 2) misses tol here.
struct SelectArgs {
  int *pn;
  double *sc;
  unsigned *ticket;
  double tol;
  int n_cap, p_cap, fixed_p, fixed_n;
  unsigned long long *acc;
};
// Structured (sparse) Hamiltonians: the union of the nonzero patterns of
// H_0 .. H_M in compressed columns, with the M + 1 FP64 values of every
// union entry (zero where a Hamiltonian has no entry there).
struct SparseU {
  const int *colptr;   // d + 1
  const int *rowidx;   // nnz_union
  const double *vals;  // nnz_union x (M + 1) x 2 (re, im), H_0 first
};
// theta_max = max_j ||dt H_j||_1 in FP64 (maximum on the bit pattern);
// with sp (not null) each column sums over its union entries only.
hipError_t launch_norm(const double *H64, const double *u, int d, int M, int N, double dt,
                       unsigned long long *theta_bits, const SelectArgs &sel, hipStream_t st,
                       const SparseU *sp = nullptr);

template <typename T> hipError_t launch_fill(T *p, long n, T v, hipStream_t st);
// dst[0:n] = src[0:n] (a kernel, so that captured graphs hold no copy nodes)
template <typename T> hipError_t launch_copy(T *dst, const T *src, long n, hipStream_t st);
// count segments of n elements: dst + b * dstride <- src + b * sstride
template <typename T>
hipError_t launch_copy_strided(T *dst, long dstride, const T *src, long sstride, long n,
                               long count, hipStream_t st);

// Small padded d (16, 32; 48 in FP32): the whole Taylor + squaring chain of
// a step in LDS, (p, n, dt/2^n) read from device memory (pn, sc).  Level
// D^(i) is stored at slot n - i (slot 0 = the final D^(n)).
template <typename T> bool small_expm_ok(int dp);
template <typename T>
hipError_t launch_expm_small(const T *Hf, const double *u, int dp, int M, int N, const int *pn,
                             const double *sc, T *X, T *Dlev, T *Dh, hipStream_t st);
// Padded d 16: the step exponentials with their FP64 norms fused in,
// computed with the pair held in sel.pn (the previous call's, recorded in
// pn[3]); each of the expm16_blocks(N) workgroups stores its largest
// ||dt H_j||_1 bit pattern in part.  The block-product kernel then chooses
// (p, n) (Pick16) and recomputes where the pair changed.
struct Norm16 {
  const double *H64;  // FP64 Hamiltonians, (M + 1) x d x d interleaved complex
  int d;
  double dt;
  unsigned long long *theta_bits;  // [0] receives theta_max
  unsigned long long *part;        // one word per workgroup of the exponential pass
  SelectArgs sel;
};
template <typename T> unsigned expm16_blocks(int N);
template <typename T>
hipError_t launch_expm16(const T *Hf, const double *u, int M, int N, T *X, T *Dlev, T *Dh,
                         const Norm16 &nm, hipStream_t st);
// Sub-blocks of the padded-d-16 in-block passes: SUB16 consecutive steps
// (a block of L = k SUB16 steps holds k of them, the last one of a call may
// be shorter); sub-block s covers steps [s SUB16, min(N, (s + 1) SUB16)).
constexpr int SUB16 = 8;
// Pair choice and recompute inputs for the padded-d-16 block products, and
// the optional sub-block products (Es, Ehs: one matrix minus identity, and
// its conjugate transpose, per sub-block; null: not written; L must then be
// a multiple of SUB16).
template <typename T> struct Pick16 {
  Norm16 nm;  // nm.part null: no choice to make
  int nparts;
  const T *Hf;
  const double *u;
  int M;
  T *X, *Dlev, *Dh;
  T *Es, *Ehs;
};
// Dh / Eh: optional conjugate transposes of the final D_j / of E_b (null: not written)
template <typename T>
hipError_t launch_blockprod_small(const T *D, int dp, int N, int L, int nb, T *E, T *Eh,
                                  const Pick16<T> *pick, hipStream_t st);

// Blocked two-level sweep.  State sets are [2][S][dp] (re plane of S
// states, then im plane).  Block b covers steps [b*L, min(N, (b+1)*L)).
template <typename T> struct SweepArgs {
  int N, L, nb, dp, d, S, M;
  const T *D;          // N x (2 dp^2): D_j = U_j - I
  const T *E;          // nb x (2 dp^2): block products minus identity
  const T *Dh, *Eh;    // D_j^H, E_b^H (single-wavefront sweeps)
  const T *Es, *Ehs;   // sub-block products and their ^H (padded d 16; null: not used)
  T *nu;               // per sub-block partial penalty costate (with Es and a penalty)
  const T *psi0;       // one state set
  T *ckpt;             // (nb+1) state sets: psi at block starts
  T *psi_buf;          // (N+1) state sets: psi_j
  T *lam_ckpt;         // (nb+1) state sets: lambda at block starts
  T *mu;               // nb state sets: block-local penalty costates
  T *lam_buf;          // N state sets: lambda_{j+1} for step j
  const double *w64;   // dp penalty weights (FP64) or null
  const T *pw;         // dp scaled weights a_pen / S * w or null
  unsigned long long *drift_bits;
  // cost
  const double *psiT64;  // S x d interleaved complex targets
  const double *u;       // M x N controls (FP64)
  double alpha_fid, alpha_pen, alpha_amp, alpha_var;
  int fid_mode;
  double *out;          // [C, C_fid, c_1..c_N]
  double *zinfo;        // [Re z, Im z, F, then Re/Im overlap of each column]
  double *part;         // 4 x npart partials (penalties, |u|^2, variations, drift max)
  int npart;            // penalty workgroups of k_cost (wavefronts when fused)
  int fuse_cost;        // single-wavefront B2 computes lambda_N and runs the penalties
  // per-step costate sources beyond the level penalty (forbidden states,
  // time-optimal term; null: none), (N + 1) state sets, src_j at set j; read
  // by the generic per-block kernels only (k_fwd_replay's mu pass, k_bwd_pairs)
  const T *src;
  int replay_mode;      // k_fwd_replay: 0 replay and mu, 1 replay only, 2 mu only
  // totals of the per-step terms of k_ext (null: none): 2 x next partials
  const double *ext_part;
  int next;
  double alpha_time;
};
template <typename T> __host__ __device__ inline TotalArgs total_args(const SweepArgs<T> &a) {
  return TotalArgs{a.part, a.npart, a.zinfo, a.out, a.alpha_fid, a.alpha_pen,
                   a.alpha_amp, a.alpha_var, a.drift_bits, a.ext_part, a.next,
                   a.alpha_time, a.N};
}

// Forbidden states and the time-optimal term (kernels_ext.hip): one
// wavefront per step j = 1..N computes, in FP64, the overlaps of psi_j with
// the forbidden states and the targets, adds (1/S) sum |<F_f|psi_j^s>|^2 to
// c_j in out, writes the costate source src_j (chain precision), adds src_N
// to lambda_N (lamN, written by the cost launch before), and leaves
// per-workgroup sums of the forbidden occupancies and of F_j in part
// (2 x nblk) for the total.
constexpr int QOC_MAX_FORBIDDEN = 16;
template <typename T> struct ExtArgs {
  const double *forb64;  // nf x d interleaved complex forbidden states
  int nf;                // 0 .. QOC_MAX_FORBIDDEN
  double alpha_time;
  T *src;                // (N + 1) state sets
  T *lamN;               // lambda_N state set
  double *part;          // 2 x nblk
  int nblk;
};
template <typename T>
hipError_t launch_ext(const SweepArgs<T> &a, const ExtArgs<T> &e, hipStream_t st);

// FP64 unitarity drift max |(D + D^H + D^H D)_{rc}| of the final step
// propagators U_j = I + D_j (true d x d block) over the steps N-1,
// N-1-stride, ..., folded into *acc as (epoch << 32 | FP32 bits) by atomic
// maximum (kernels_ext.hip).
// Adam over n FP64 amplitudes with a device-side step count t (kernels_ext.hip).
hipError_t launch_adam(long n, double *u, const double *g, double *m, double *v, double *t,
                       double lr, double b1, double b2, double eps, hipStream_t st);

template <typename T>
hipError_t launch_unitarity(const T *D, int dp, int d, int N, int stride, unsigned epoch,
                            unsigned long long *acc, hipStream_t st);
template <typename T> hipError_t launch_fwd_blocks(const SweepArgs<T> &a, hipStream_t st);
template <typename T> hipError_t launch_fwd_replay(const SweepArgs<T> &a, hipStream_t st);
template <typename T> hipError_t launch_bwd_blocks(const SweepArgs<T> &a, hipStream_t st);
template <typename T> hipError_t launch_bwd_pairs(const SweepArgs<T> &a, hipStream_t st);
// Time segments: the costate at a segment's first step (>= 1) into the
// segment's first checkpoint (arguments offset to the segment).
template <typename T> hipError_t launch_seg_lambda(const SweepArgs<T> &a, hipStream_t st);
// Small padded d (<= 64): all columns per workgroup, prefetched step matrices.
// which: 0 = F2, 1 = F3, 2 = B2, 3 = B3.
template <typename T> bool small_sweep_ok(int dp, int S);
template <typename T> hipError_t launch_small_sweep(int which, const SweepArgs<T> &a, hipStream_t st);
// One wavefront holding the whole state set (S * dp <= 64, dp = 16 or 32).
template <typename T> bool wave_sweep_ok(int dp, int S);
template <typename T> hipError_t launch_wave_sweep(int which, const SweepArgs<T> &a, hipStream_t st);
// Padded d 64 .. 128 (FP32): one workgroup of 8 d_pad threads per chain
// with a register prefetch ring of matrix slices.  which as below.
template <typename T> bool chain_sweep_ok(int dp, int S);
template <typename T> hipError_t launch_chain_sweep(int which, const SweepArgs<T> &a, hipStream_t st);
// Large padded d (>= 80): the sweeps as per-step launches spread over many
// workgroups.  which: 0 = F2, 1 = F3, 2 = B2, 3 = B3.
template <typename T> bool wide_sweep_ok(int dp, int S);
// mm: the products on the MFMA (16-row x 16-state tiles), else on the VALU.
template <typename T> hipError_t launch_wide_sweep(int which, const SweepArgs<T> &a, hipStream_t st,
                                                   bool mm = false);
// One launch: per-step penalties c_j (FP64) and norm drift partials,
// parallel over steps, beside the fidelity, C_fid and lambda_N (one
// workgroup; needs the final states only).  npart + 1 workgroups.
template <typename T> hipError_t launch_cost(const SweepArgs<T> &a, hipStream_t st);
// Total cost and norm drift from launch_cost's partials and fidelity.
template <typename T> hipError_t launch_total(const SweepArgs<T> &a, hipStream_t st);

// Exact per-step derivative of the Taylor + squaring evaluation, contracted
// with the control Hamiltonians (see kernels_adjoint.hip).
template <typename T> struct AdjointArgs {
  int N, dp, M, S, p, n, Rcap, nblocks;
  const T *X;          // N x 2 dp^2
  const T *Dlev;       // (n+1) x N x 2 dp^2: D^(i)_j, level-major
  const T *lam_buf;    // N state sets
  const T *psi_buf;    // (N+1) state sets
  const T *Hf;         // (M+1) x 2 dp^2 (index 0 = H_0)
  const double *u;     // M x N
  double s_scale;      // dt / 2^n
  const int *pn;       // if not null: p, n read from here (device-side choice),
  const double *sc;    //   dt / 2^n from sc[0], and level i at slot n - i
  double alpha_amp, alpha_var;
  T *scratch;          // nblocks x groups_per_block x scratch_elems
  long scratch_elems;
  double *grad;        // M x N
  double *part;        // batched variant: N x slices x M partial sums
  T *xbar;             // batched variant: N x 2 dp^2 work space for Xbar_j
  int bf3;             // batched variant: bf16x3 split products
  int *bf3_launched;   // host flag, may be null: set to 1 when a split product is launched
  int with_total;      // padded d 16: one extra workgroup reduces the cost (total)
  TotalArgs total;
  // batched variant with structured control Hamiltonians (rptr null:
  // dense): the union of the controls' nonzero patterns by rows (rptr: d + 1
  // offsets, rcol: columns) and, per union entry e, the controls with a
  // nonzero there (ek[eptr[e] .. eptr[e+1]]) and their values (eval: re
  // plane, then im plane, nev each); the gradient contracts Xbar_j only at
  // these entries, formed from the derivative's panels instead of storing
  // Xbar_j.  d: true dimension.
  const int *rptr, *rcol, *eptr, *ek;
  const T *eval;
  long nev;
  int d;
  // batched variant, one time segment of a longer horizon: the N steps are
  // global steps j0 .. j0 + N - 1 of ldN (u and grad are M x ldN; ldN 0: N)
  long j0;
  int ldN;
};
template <typename T> long adjoint_scratch_elems(int dp, int p, int Rcap);
// Time steps processed concurrently per workgroup (one per wave for small d).
template <typename T> int adjoint_groups_per_block(int dp);
template <typename T> hipError_t launch_adjoint(const AdjointArgs<T> &a, hipStream_t st);
// Register-resident variant for padded d = 16 (one wavefront per step, no
// scratch); p_max bounds the Taylor order it may be asked to handle.
template <typename T> bool adjoint16_ok(int dp, int p_max);
// Batched variant for padded d >= 64: one launch per stage of the reverse
// recurrence over all N steps; scratch is per step (N x per_step elements),
// `xbar` holds N matrices and `part` N x slices x M partial sums.  The
// control Hamiltonians must be exactly Hermitian (X^H = -X is used).
// (p, n) must be host-known.
template <typename T> bool adjoint_big_ok(int dp);
template <typename T> long adjoint_big_scratch_per_step(int dp, int p, int Rcap);
// Entry slices of the batched gradient contraction (partial sums per step
// and control: N x slices x M doubles in `part`).
long adjoint_big_slices(int dp);
template <typename T> hipError_t launch_adjoint_big(const AdjointArgs<T> &a, hipStream_t st);
template <typename T> hipError_t launch_adjoint16(const AdjointArgs<T> &a, hipStream_t st);
// The paper's first-order gradient (eq. 7) for any padded d: Y_j = sum_s
// lambda_{j+1}^s psi_{j+1}^{s H} into a.xbar, contracted with every H_k
// (partial sums in a.part: N x adjoint_big_slices(dp) x M), times 2 dt, plus
// the C3 / C4 gradients.
template <typename T> hipError_t launch_grad_first(const AdjointArgs<T> &a, double dt,
                                                   hipStream_t st);
// grad[k, j0 + j] = two_s sum_t part[(j tiles + t) M + k] + the C3 / C4
// gradients, for the N steps j0 .. j0 + N - 1 of a horizon of Nf steps.
hipError_t launch_grad_finish(const double *part, const double *u, double *grad, double two_s,
                              double alpha_amp, double alpha_var, int N, int M, int tiles, long j0,
                              int Nf, hipStream_t st);

// ---------------------------------------------------------------- action form
// State-mode action form (kernels_action.hip): H_j in an ELL layout over the
// union pattern of H_0 .. H_M, K slots per row.
template <typename T> struct ActValArgs {
  const double *hm;  // (M+1) x K x 2 x dp: each matrix's slot values (re plane, im plane)
  const double *u;   // M x N
  int M, N, K, dp;
  T *hv;             // N x K x 2 x dp: H_j's slot values
};
template <typename T> struct ActionArgs {
  int N, dp, S, K, p, n, P;  // P = p 2^n products per step and column
  T s;                       // dt / 2^n
  T coef[33], inv[33];       // s / k and 1 / k, k = 1 .. p (p <= 32)
  const int *ecol;           // K x dp: column of slot (kk, r)
  const T *hv;               // N x K x 2 x dp
  const T *psi0;             // state set
  T *psi_buf;                // (N+1) state sets
  T *A;                      // N x S x P x 2 x dp: product inputs (null: not kept)
  const T *lamN;             // state set: lambda_N
  T *lam_buf;                // N state sets: lambda_{j+1} at set j
  const T *pw, *src;         // per-step costate sources (null: none)
  T *Ybar;                   // N x S x P x 2 x dp: product output cotangents (null: not kept)
};
template <typename T> struct ActGradArgs {
  // product inputs a_q and output cotangents ybar_q of step j, column s:
  // base + j * (a|y)j + s * (a|y)s + q * (a|y)q, imaginary plane at +(a|y)plane
  const T *A, *Y;
  long aj, as, aq, aplane, yj, ys, yq, yplane;
  int N, S, P, dp, M;
  int nent;                   // entries of the union of the controls' patterns
  const int *erow, *ecol;     // their rows and columns
  const int *cptr, *cent;     // per control k: entries cent[cptr[k] .. cptr[k+1])
  const T *cval;              // ... and values (re plane, then im plane at +npairs)
  long npairs;
  double *part;               // N x S x M partial sums
};
template <typename T> hipError_t launch_act_values(const ActValArgs<T> &a, hipStream_t st);
// which 0: forward chain (psi, product inputs); 1: backward chain (lambda,
// product cotangents).  One workgroup per column.
template <typename T> hipError_t launch_act_chain(int which, const ActionArgs<T> &a,
                                                  hipStream_t st);
template <typename T> hipError_t launch_act_grad(const ActGradArgs<T> &a, hipStream_t st);
// Shapes the chains handle: padded d <= 1024 and K slots (4, 8, 16, 32) per
// row within the register budget; LDS bytes of the gradient kernel.
template <typename T> bool act_shape_ok(int dp, int K);
template <typename T> long act_grad_lds(int dp, long nent);

}  // namespace qoc
