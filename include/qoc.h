/*
 * qoc.h - C ABI of libqoc: cost and exact gradient of piecewise-constant
 * quantum optimal control on one AMD Instinct MI355X (gfx950).
 *
 * Method: Leung, Abdelhafez, Koch, Schuster, "Speedup for quantum optimal
 * control from automatic differentiation based on graphics processing
 * units", arXiv:1612.04929.
 *
 * The problem statement follows the paper's Sec. II and Table I:
 *   H_j   = H_0 + sum_k u_{k,j} H_k                      (eq. 1)
 *   U_j   = exp(-i H_j dt)                                (eq. 3), hbar = 1
 *   psi_{j+1}^s = U_j psi_j^s, j = 0..N-1, s = 0..S-1     (eqs. 2, 4)
 *   z     = (1/S) sum_s <T_s|psi_N^s>,  C_fid = 1 - |z|^2 (composite state
 *           infidelity, Sec. II.A; equals the gate infidelity C1 when the
 *           S = d columns of the identity are propagated)
 *   c_j   = (1/S) sum_s [sum_m w_m |psi_j^s[m]|^2 + sum_f |<F_f|psi_j^s>|^2],
 *           j = 1..N  (Table I, C5: forbidden levels with weights w and a set
 *           of forbidden states F_f, summed, Sec. II.A)
 *   C_amp = sum u^2 (C3),  C_var = sum_k sum_{j>=1} (u_{k,j}-u_{k,j-1})^2 (C4)
 *   C_time = 1 - (1/N) sum_{j=1..N} F_j, F_j the fidelity of psi_j against the
 *           targets in the mode of C_fid (Table I, C6 coherent / C7
 *           incoherent: the time-optimal term)
 *   C     = a_fid C_fid + a_pen sum_j c_j + a_amp C_amp + a_var C_var
 *           + a_time C_time
 * Each U_j is evaluated by a truncated Taylor series of order p with n
 * scaling-and-squaring steps, with one global (p, n) (Sec. III, eq. 6),
 * and the gradient dC/du_{k,j} is the exact derivative of that evaluation
 * (reverse accumulation through the Taylor and squaring recurrences, in
 * place of the first-order formula of eq. 7).
 *
 * Conventions for every entry point
 *  - Complex numbers crossing the ABI are interleaved (re, im) doubles.
 *  - Matrices are row-major d x d; H_k is stored [k][row][col].
 *  - States are stored state-major: component m of state s at [s*d + m].
 *  - Controls are stored u[k*N + j] (control k, step j); the gradient uses
 *    the same layout.
 *  - The caller owns every pointer it passes.  qoc_create copies all
 *    problem data, so the caller may free it after the call returns.
 *    Outputs are caller-allocated.  The handle owns all device memory.
 *  - Errors are reported by the returned status only; no exception or
 *    abort crosses the ABI.  On error, outputs are left untouched and
 *    qoc_last_error() describes the cause (thread-local string).
 *  - A handle is not thread-safe; distinct handles may be used from
 *    distinct threads.
 */
#ifndef QOC_H
#define QOC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qoc_handle qoc_handle;

typedef enum {
  QOC_OK = 0,
  QOC_ERR_ARG = -1,            /* null pointer or invalid scalar argument   */
  QOC_ERR_SHAPE = -2,          /* d, M, N, S out of range or inconsistent   */
  QOC_ERR_NOT_HERMITIAN = -3,  /* H_0 or some H_k fails the Hermitian check */
  QOC_ERR_NONFINITE = -4,      /* NaN/Inf in an input                       */
  QOC_ERR_NOMEM = -5,          /* device or host allocation failed          */
  QOC_ERR_DEVICE = -6,         /* HIP runtime error or no usable device     */
  QOC_ERR_UNSUPPORTED = -7     /* valid request this build does not handle  */
} qoc_status;

/* Precision of the matrix-product chains (Taylor, squaring, adjoint). */
enum { QOC_FP64 = 0, QOC_FP32 = 1, QOC_BF16X3 = 2 };

/* Fidelity mode: coherent |(1/S) sum_s <T_s|psi_N^s>|^2 (phase-sensitive,
 * equals the gate fidelity on a full basis) or incoherent
 * (1/S) sum_s |<T_s|psi_N^s>|^2 (mean of the per-state fidelity C2). */
enum { QOC_FID_COHERENT = 0, QOC_FID_INCOHERENT = 1 };

/* Bits of *flags_out. */
enum {
  QOC_WARN_DRIFT = 1,  /* norm drift of the propagated columns above drift_warn */
  QOC_WARN_TAYLOR = 2, /* a fixed (taylor_p, taylor_n) misses taylor_tol at this
                          call's theta_max (the call still uses the fixed pair) */
  QOC_WARN_PRECISION = 4, /* QOC_BF16X3: the automatic policy ran some product
                            classes in FP32 (qoc_info.bf16x3_classes) because
                            the predicted bf16x3 error exceeded its budget */
  QOC_WARN_UNITARITY = 8, /* the FP64 unitarity check (qoc_set_unitarity_check)
                             found max |(U^H U - I)_{rc}| above drift_warn */
  QOC_WARN_NO_PAIR = 16   /* device-pointer calls (reported by qoc_get_info):
                             no (p, n) within the path's capacity met
                             taylor_tol at the call's theta_max, or theta_max
                             was not finite (NaN / Inf amplitudes); the call
                             ran with a clamped pair and its results are not
                             accurate.  Host-array calls return
                             QOC_ERR_UNSUPPORTED instead. */
};

/* Product classes of the QOC_BF16X3 precision: each class runs as bf16x3
 * split products (three bf16 MFMA products of hi/lo operand halves, FP32
 * accumulation) or as FP32 products.  Sec. III: the Taylor series of
 * eq. 6 on the scaled generator, the squarings that undo the scaling; Sec.
 * II.B: the reverse pass. */
enum { QOC_PROP_MATRIX = 0, QOC_PROP_ACTION = 1 };

enum {
  QOC_BF3_TAYLOR = 1,     /* Taylor (Horner / Paterson-Stockmeyer) products   */
  QOC_BF3_SQUARING = 2,   /* the n squarings D <- 2D + D^2                    */
  QOC_BF3_BLOCKPROD = 4,  /* block products of the blocked two-level scan     */
  QOC_BF3_ADJOINT = 8,    /* products of the exact per-step derivative        */
  QOC_BF3_ALL = 15
};

typedef struct {
  int d;                    /* Hilbert-space dimension, 1 <= d <= 1024     */
  int M;                    /* number of control Hamiltonians, 0 <= M <= 64 */
  int N;                    /* number of time steps, N >= 1                 */
  int S;                    /* propagated columns, 1 <= S <= d              */
  double dt;                /* step length (> 0), same time unit as 1/H     */
  const double *H0;         /* d*d complex, Hermitian                       */
  const double *Hk;         /* M*d*d complex, each Hermitian (NULL if M=0)  */
  const double *psi0;       /* S*d complex initial states                   */
  const double *psiT;       /* S*d complex target states (zero outside the
                               target subspace: the projector P_S of the
                               composite infidelity is implicit)            */
  const double *penalty_w;  /* d real weights >= 0 of forbidden levels, or
                               NULL (no per-step penalty)                   */
  double alpha_fid, alpha_amp, alpha_var, alpha_pen;   /* cost weights      */
  int fid_mode;             /* QOC_FID_COHERENT or QOC_FID_INCOHERENT       */
  int precision;            /* QOC_FP32 (default), QOC_FP64 or QOC_BF16X3   */
  int checkpoint_every;     /* state checkpoint interval L of the blocked
                               sweeps (any L >= 1, used as given); 0 = the
                               power of two nearest sqrt(N)                 */
  double taylor_tol;        /* truncation tolerance tau of the (p, n) rule;
                               0 = 1e-10 (FP32, BF16X3) or 1e-15 (FP64)     */
  int taylor_p, taylor_n;   /* taylor_p >= 2 and taylor_n >= 0: fixed global
                               (p, n), no per-call host synchronisation;
                               taylor_p == 0: (p, n) chosen per call from
                               theta_max; anything else is QOC_ERR_ARG      */
  double drift_warn;        /* threshold of QOC_WARN_DRIFT; 0 = 1e-4        */
  int device;               /* HIP device ordinal                           */
  int n_forbidden;          /* forbidden states of C5, 0 .. 16 (weighted by
                               alpha_pen; ignored when alpha_pen == 0)      */
  const double *forbidden;  /* n_forbidden*d complex, state-major (state f at
                               [f*d + m]), or NULL when n_forbidden == 0    */
  double alpha_time;        /* weight of the time-optimal term C_time        */
  int pad_multiple;         /* d is padded with zeros (exact: exp of a zero
                               block is the identity) to a multiple of 16
                               (0 or 16: the default), 32 or 64; a multiple
                               of 64 runs every product on 64 x 64 MFMA
                               tiles (a tile-shape choice for measuring
                               tuners); anything else is QOC_ERR_ARG       */
  int segment_steps;        /* memory-lean mode (batched path, padded
                               d >= 64): 0 = one
                               segment; otherwise the horizon is cut into
                               time segments of this many steps (rounded up
                               to a multiple of the checkpoint interval L)
                               and every per-step stack (propagators, Taylor
                               and squaring levels, derivative work space)
                               holds one segment: the backward pass
                               recomputes each segment's exponentials from
                               the controls (Sec. 5.2 and App. A trade
                               memory for recomputation the same way).  The
                               states, checkpoints and costates stay whole
                               (O(N S d)).  Negative: QOC_ERR_ARG; a handle
                               on the small-d path: QOC_ERR_UNSUPPORTED    */
  int propagation;          /* QOC_PROP_MATRIX (0, default): every step
                               exponential formed as a matrix (batched
                               Taylor + squaring products); QOC_PROP_ACTION:
                               the state-mode action form of Sec. IV, the
                               approximant applied to the S columns by
                               p 2^n matrix-vector products per step with
                               H_j in a sparse (ELL) layout over the union
                               pattern of H_0 .. H_M, no U_j formed and no
                               per-step matrix stack held; (p, n) by the
                               fewest products within the same bound (and
                               theta / 2^n <= 1).  FP32 or FP64; the union
                               pattern may hold at most 32 nonzeros per row
                               (FP32, padded d <= 512; 16 in FP64 or above
                               512), else QOC_ERR_UNSUPPORTED at create    */
} qoc_problem_desc;

/* Diagnostics of the most recent forward / cost_grad call on a handle. */
typedef struct {
  int p, n;                 /* Taylor order and squaring count used          */
  double theta_max;         /* max_j ||dt H_j||_1, evaluated in FP64         */
  double norm_drift;        /* max_{j,s} | ||psi_{j+1}^s||^2 - ||psi_j^s||^2 |
                               (FP64), the unitarity drift seen by the
                               propagated columns                           */
  int block_len;            /* checkpoint interval L actually used           */
  int n_blocks;             /* ceil(N / L)                                   */
  int d_pad;                /* device padding of d (multiple of 16)          */
  int flags;                /* warning bits (QOC_WARN_*) of the last call    */
  size_t device_bytes;      /* device memory held by the handle              */
  int bf16x3_classes;       /* QOC_BF3_* classes that ran bf16x3 products in
                               the last call: the chain classes need padded
                               d a multiple of 64, and the derivative's class
                               counts only if one of its products was wide
                               enough (64 columns) or dense enough to have a
                               split kernel                                  */
  double unitarity_drift;   /* max over the checked steps of
                               max_{r,c} |(D_j + D_j^H + D_j^H D_j)_{rc}| =
                               |(U_j^H U_j - I)_{rc}|, evaluated in FP64 (kept
                               to FP32 precision); -1 when the last call ran
                               no check (qoc_set_unitarity_check)           */
  int structured;           /* 1 when the last call ran the structured
                               (sparse) norm and gradient contraction       */
  int segments;             /* time segments of the memory-lean mode (1: the
                               whole horizon at once)                       */
  int propagation;          /* QOC_PROP_* of the handle                      */
} qoc_info;

/* Create a handle: validates and copies the problem to device memory.
 * Checks: shapes; S <= d; finite inputs; dt > 0; Hermiticity of H_0 and
 * every H_k with ||H - H^dagger||_max <= 1e-12 * max(1, ||H||_max);
 * penalty weights >= 0; 0 <= n_forbidden <= 16 (QOC_ERR_SHAPE).  With
 * forbidden states (and alpha_pen != 0) or alpha_time != 0 the sweeps run on
 * the generic per-block kernels (the sweep variants of qoc_set_sweep do not
 * apply) and the per-step terms add one FP64 pass over the states.  Paper:
 * Sec. II (problem statement), Table I. */
qoc_status qoc_create(const qoc_problem_desc *desc, qoc_handle **out);

/* Forward pass only (Sec. II, eqs. 1-4; Table I).  u: M*N host doubles.
 * Outputs (host, each may be NULL): *cost_fid = C_fid; step_penalty[j-1] =
 * c_j for j = 1..N; psiN: S*d complex final states; *flags_out: warning
 * bits.  Blocks until the results are on the host. */
qoc_status qoc_forward(qoc_handle *h, const double *u, double *cost_fid,
                       double *step_penalty, double *psiN, int *flags_out);

/* Cost and exact gradient (Sec. II.B reverse accumulation; Table I costs).
 * u, grad: M*N host doubles (grad may be NULL only if M == 0).
 * *cost = C (weighted total), *cost_fid = C_fid, step_penalty[j-1] = c_j
 * (or NULL), *flags_out warning bits (or NULL).  Blocks until done. */
qoc_status qoc_cost_grad(qoc_handle *h, const double *u, double *cost,
                         double *cost_fid, double *step_penalty, double *grad,
                         int *flags_out);

/* Device-resident variant of qoc_cost_grad for callers that keep u and the
 * outputs in HBM (e.g. a torch.autograd.Function).  u_dev: M*N doubles on
 * the handle's device; out_dev: 2 + N doubles written as
 * [C, C_fid, c_1, ..., c_N]; grad_dev: M*N doubles.  Work is enqueued on
 * `stream` (a hipStream_t; NULL = the default stream).  When (p, n) is not
 * fixed in the descriptor the call synchronises `stream` once to read
 * theta_max back (padded d >= 64; smaller d choose (p, n) on the device);
 * with a fixed (p, n) it is fully asynchronous and capturable in a HIP
 * graph, the fixed pair being checked against taylor_tol on the device
 * (QOC_WARN_TAYLOR in qoc_info.flags). */
qoc_status qoc_cost_grad_device(qoc_handle *h, const double *u_dev,
                                double *out_dev, double *grad_dev, void *stream);

/* Variant of qoc_cost_grad_device that allocates nothing, for callers that
 * cannot allocate device memory during a call: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and stream semantics as qoc_cost_grad_device; the
 * per-call work space (the Taylor / squaring levels, the derivative's
 * scratch and partial sums) is carved from a static device array of 256
 * MiB that the library holds on each GPU it runs on until the process ends,
 * instead of the handle's lazily grown buffers (which are left untouched).
 * A call whose work space exceeds 256 MiB returns QOC_ERR_UNSUPPORTED
 * before its first kernel on the small-d path (padded d <= 48), and after
 * the FP64 norm kernel otherwise; so does a handle with per-phase profiling
 * enabled (events would be created).  All calls on one GPU share that
 * array: calls that overlap in time on the same GPU (other streams, other
 * threads) race and must be serialised by the caller.  The array keeps the
 * last call's contents; every value a call reads from it is written by the
 * same call first.  Sec. II.B and Sec. III as for qoc_cost_grad_device. */
qoc_status qoc_cost_grad_device_noalloc(qoc_handle *h, const double *u_dev,
                                        double *out_dev, double *grad_dev,
                                        void *stream);

/* Batched variant: B independent handles (uneven d, N, M allowed), each
 * with its own device u / out / grad pointers as in qoc_cost_grad_device,
 * enqueued on one stream. */
qoc_status qoc_cost_grad_batched(int B, qoc_handle *const *hs,
                                 const double *const *u_dev,
                                 double *const *out_dev,
                                 double *const *grad_dev, void *stream);

/* One Adam step (the optimiser of the paper's examples, Sec. IV) over n
 * FP64 amplitudes on the device, e.g. the controls of many instances packed
 * back to back:
 *   m <- beta1 m + (1 - beta1) g,  v <- beta2 v + (1 - beta2) g^2,
 *   t <- t + 1,  u <- u - lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps).
 * u_dev, m_dev, v_dev (updated in place), grad_dev: n doubles each; t_dev:
 * one double on the device holding the step count (0 before the first
 * step), advanced by the call, so replays of a captured iteration keep
 * counting.  Enqueued on `stream`, no host synchronisation; two kernel
 * launches, no allocation.  QOC_ERR_ARG for n < 0, NULL arrays, lr < 0,
 * betas outside [0, 1) or eps <= 0. */
qoc_status qoc_adam_step(long n, double *u_dev, const double *grad_dev, double *m_dev,
                         double *v_dev, double *t_dev, double lr, double beta1, double beta2,
                         double eps, void *stream);

/* Diagnostics of the last call (see qoc_info).  Synchronises the handle's
 * device to read the on-device diagnostics back. */
qoc_status qoc_get_info(const qoc_handle *h, qoc_info *info);

/* Per-kernel device timing for measurement: when enabled, every kernel
 * launch of a call is bracketed with HIP events on the stream it runs on
 * (the events are resolved lazily, so enabling this adds no host
 * synchronisation).  qoc_profile_read synchronises the outstanding events
 * and returns, per phase, the summed event time in milliseconds and the
 * number of launches timed (arrays of QOC_PHASE_COUNT); reset != 0 clears
 * the counters. */
enum {
  QOC_PHASE_NORM = 0,        /* FP64 step norms, theta_max                   */
  QOC_PHASE_ASSEMBLE = 1,    /* X_j = -i dt/2^n H_j and the first Horner term */
  QOC_PHASE_TAYLOR = 2,      /* one batched complex product of the Taylor /
                                squaring chain over all N steps (per launch) */
  QOC_PHASE_BLOCKPROD = 3,   /* one level of the block-product tree          */
  QOC_PHASE_FWD_BLOCKS = 4,  /* sequential checkpoint sweep over blocks      */
  QOC_PHASE_FWD_REPLAY = 5,  /* in-block replay, penalties, block costates   */
  QOC_PHASE_COST = 6,        /* FP64 fidelity overlap and cost terms         */
  QOC_PHASE_BWD_BLOCKS = 7,  /* sequential costate sweep over blocks         */
  QOC_PHASE_BWD_PAIRS = 8,   /* in-block costates lambda_{j+1}               */
  QOC_PHASE_ADJOINT = 9,     /* per-step exact derivative + gradient         */
  QOC_PHASE_COUNT = 10
};
qoc_status qoc_profile_enable(qoc_handle *h, int on);
qoc_status qoc_profile_read(qoc_handle *h, double *ms, long long *calls,
                            int reset);

/* The (p, n) rule on the host: fewest products G = p-1+n with
 * 2^n (theta/2^n)^(p+1)/(p+1)! e^(theta/2^n) <= tol, ties to smaller n,
 * p >= 2 (Sec. III: global conservative truncation and scaling). */
qoc_status qoc_taylor_select(double theta, double tol, int *p, int *n);

/* The (p, n) rule of each evaluation form (Sec. III's conservative global
 * choice; the bound above throughout, p >= 2):
 *   QOC_FORM_HORNER   fewest Horner products p-1+n, ties to smaller n (the
 *                     small-d chains; the same as qoc_taylor_select)
 *   QOC_FORM_BATCHED  fewest evaluated products P(p)+n, P(p) the
 *                     Paterson-Stockmeyer count min over s = 2..4 of
 *                     (s-1) + floor(p/s) - [s divides p], or p-1 when
 *                     smaller, with theta/2^n <= 1, ties to smaller p (the
 *                     batched path; the derivative runs p-1 reverse stages)
 *   QOC_FORM_ACTION   fewest matrix-vector products p 2^n, theta/2^n <= 1,
 *                     ties to smaller n (the action form, Sec. IV)
 * QOC_ERR_ARG for theta < 0 or not finite, tol <= 0, another form;
 * QOC_ERR_UNSUPPORTED when no pair with p <= 30, n < 60 meets tol. */
enum { QOC_FORM_HORNER = 0, QOC_FORM_BATCHED = 1, QOC_FORM_ACTION = 2 };
qoc_status qoc_select_pair(double theta, double tol, int form, int *p, int *n);

/* The pair the handle would choose per call for a given theta_max (its
 * form and tolerance), e.g. to fix it with qoc_set_taylor before capturing
 * a graph.  A bf16x3 handle on the batched path under the automatic class
 * policy picks, among the pairs within the bound (theta/2^n <= 1), the one
 * with the least modelled product time, a bf16x3 product counting 0.52 of
 * an FP32 one, with the classes the policy allows at that pair (ties to
 * smaller p). */
qoc_status qoc_pair_for(const qoc_handle *h, double theta, int *p, int *n);

/* Fix the global (p, n) of later calls on h (p in [2, 64], n in [0, 60]),
 * or return to the per-call choice (p = 0).  A pair beyond the capacity of
 * the handle's path (p <= 16 and n <= 16 on the small-d path, padded d <=
 * 48; p <= 30 on the batched path) is QOC_ERR_UNSUPPORTED, here and in
 * qoc_create.  A fixed pair makes the
 * device-pointer calls free of host round trips (HIP-graph capturable);
 * each call checks it against taylor_tol on the device and reports a miss
 * as QOC_WARN_TAYLOR.  Sec. III: one conservative pair for all steps. */
qoc_status qoc_set_taylor(qoc_handle *h, int p, int n);

/* Product classes (QOC_BF3_* mask, 0..QOC_BF3_ALL) that later calls of a
 * QOC_BF16X3 handle run as bf16x3 split products, the others in FP32; -1
 * (the default) chooses per call.  The automatic choice always splits the
 * per-step derivative's products (they do not feed the states) and splits
 * the chain classes (Taylor, squarings, block products) only while an
 * error index of the states stays within the budget that keeps |dF| <=
 * 1e-5 at any fidelity: the index adds, per step, 2^-17 times the product
 * of the operand norms of each split chain product times its amplification
 * by the later squarings (norms from theta_max, n and the squaring levels),
 * and grows as sqrt(N) over the steps.  Any class left in FP32 by the
 * automatic choice sets QOC_WARN_PRECISION.  With a fixed (p, n) the index
 * uses the largest theta the pair admits.  Products without a split kernel
 * at the handle's shapes (chain products at padded d not a multiple of 64;
 * thin derivative products narrower than 64 columns; the sparse gradient
 * contraction) run in FP32 and are left out of qoc_info.bf16x3_classes
 * (without QOC_WARN_PRECISION).  No effect on other precisions.
 * Returns QOC_ERR_ARG for a mask outside -1..QOC_BF3_ALL.  Sec. III
 * (truncated Taylor series with scaling and squaring), Sec. II.B. */
qoc_status qoc_set_bf16x3(qoc_handle *h, int classes);

/* Gradient of later cost + gradient calls: QOC_GRAD_EXACT (default), the
 * exact derivative of the evaluated Taylor / squaring approximant, or
 * QOC_GRAD_FIRST_ORDER, the paper's approximate gradient (Sec. III, eq. 7;
 * App. A, Algorithms 1-3), which replaces dU_j/du_{k,j} by (-i dt H_k) U_j:
 *   g_{k,j} = 2 dt Im sum_s <lambda_{j+1}^s| H_k |psi_{j+1}^s>  (+ C3 / C4)
 * from the same costates, without the derivative of the step exponential
 * (a rank-S outer product per step contracted with every H_k).  It equals
 * the exact gradient only when the step Hamiltonians commute; its error
 * grows with dt ||[H_j, H_k]||.  The cost is unaffected.  Returns
 * QOC_ERR_ARG for another mode. */
enum { QOC_GRAD_EXACT = 0, QOC_GRAD_FIRST_ORDER = 1 };
qoc_status qoc_set_gradient(qoc_handle *h, int mode);

/* Structured Hamiltonians (Sec. IV and the Conclusion: sparse matrices,
 * e.g. a diagonal drift and permutation-like controls).  On the batched
 * path (padded d >= 64) qoc_create records the union of the nonzero
 * patterns of H_0 .. H_M when it has at most d^2 / 4 entries; then the FP64
 * step norms sum each column over the union only, and (for M <= 32 and a
 * derivative panel width p R <= 512) the gradient contraction g_{k,j} =
 * 2 s Im tr(Xbar_j^H H_k) forms Xbar_j at the nonzeros of the controls
 * alone instead of storing the dense d x d Xbar_j.  The Taylor,
 * squaring and block products stay dense (the step propagators are dense).
 * mode -1 (default): structured whenever the pattern was recorded (a
 * union of at most d^2 / 4 entries); 0: dense; 1: structured (QOC_ERR_UNSUPPORTED when no pattern was
 * recorded).  Results agree with the dense kernels up to summation order. */
qoc_status qoc_set_structure(qoc_handle *h, int mode);

/* FP64 unitarity check of later calls: every stride-th step propagator
 * (steps N-1, N-1-stride, ...; stride 1 checks every step) is tested for
 * max_{r,c} |(U_j^H U_j - I)_{rc}| with U_j = I + D_j, computed in FP64 on
 * the MFMA from the stored D_j; the maximum is reported in
 * qoc_info.unitarity_drift and flagged by QOC_WARN_UNITARITY above
 * drift_warn.  stride 0 (the default) turns the check off: it is one extra
 * launch of about N / stride FP64 products, which at padded d 16 costs a few
 * percent of a call.  Returns QOC_ERR_ARG for stride < 0.  Sec. III (the
 * truncated series keeps unitarity only to its truncation error). */
qoc_status qoc_set_unitarity_check(qoc_handle *h, int stride);

/* Kernel variant of the sweeps of later calls (a tuning knob; results are
 * the same up to rounding order).  which: 0 forward block sweep, 1 forward
 * in-block replay, 2 costate block sweep, 3 costate in-block pass, -1 all.
 * variant: 0 automatic, 1 one workgroup per block (per column for padded
 * d >= 80; a single wavefront for the whole state set where it fits, and
 * for FP32 at padded d 16 with a block length of 16..64 the in-block passes
 * as one wavefront per sub-block of 8 steps),
 * 2 one launch per step spread over many workgroups (padded d >= 80),
 * 3 a four-wavefront workgroup per block with the step matrices staged in
 * LDS (padded d <= 64), 4 one workgroup of 8 d_pad threads per block with
 * a register prefetch ring of matrix slices (FP32, padded d 64 .. 128), 5
 * one launch per step with the products on the MFMA (16-row x 16-state
 * tiles; padded d >= 80).  A
 * variant that does not apply falls back to the automatic choice.  Sec. II,
 * eqs. 2-4 (the sequential product of propagators). */
qoc_status qoc_set_sweep(qoc_handle *h, int which, int variant);

void qoc_destroy(qoc_handle *h);
const char *qoc_status_string(qoc_status s);
const char *qoc_last_error(void);
const char *qoc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QOC_H */
