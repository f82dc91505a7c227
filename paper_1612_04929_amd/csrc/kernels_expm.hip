// Step exponentials by truncated Taylor series with scaling and squaring
// (Sec. III, eq. 6), all N steps independent, in the "D-form":
//   X   = -i (dt / 2^n) H_j
//   Q_p = I + X/p,  Q_k = I + (1/k) X Q_{k+1}   (k = p-1 .. 2)   Horner
//   D^(0) = X Q_2 = T_p(X) - I
//   D^(i+1) = 2 D^(i) + D^(i) D^(i)            ((I + D)^2 = I + 2D + D^2)
//   U_j = I + D^(n)
// Keeping D = U - I instead of U avoids the systematic FP32 truncation of
// adding a small update to the identity at every step.
#include "qoc_device.h"
#include "qoc_kernels.h"
#include "qoc_tile.h"

namespace qoc {

// Offset of matrix j of a stage operand: j * stride, or with segments of
// a.seg matrices (the per-block trees of the block products) the segment's
// own stride between segments: (j / seg) * segstride + (j % seg) * stride.
template <typename T>
__device__ __forceinline__ long moff(const StageArgs<T> &a, long j, long stride, long segstride) {
  if (a.seg <= 0) return j * stride;
  const long b = j / a.seg;
  return b * segstride + (j - b * a.seg) * stride;
}

// Block: 256 consecutive matrix entries (one per thread, coalesced) x
// AS_STEPS steps; each Hamiltonian entry loaded feeds AS_STEPS steps, and
// the control amplitudes are wave-uniform LDS broadcasts.
constexpr int AS_STEPS = 16, AS_KC = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_assemble(const T *__restrict__ Hf,
                                                  const double *__restrict__ u, int dp, int M,
                                                  int N, T s, T inv_p, T *__restrict__ X,
                                                  T *__restrict__ Q) {
  extern __shared__ char as_smem[];
  T *coef = (T *)as_smem;  // [AS_STEPS][M]
  const long plane = (long)dp * dp;
  const int t = threadIdx.x;
  const int j0 = blockIdx.x * AS_STEPS;
  const long rc = (long)blockIdx.y * 256 + t;
  for (int e = t; e < AS_STEPS * M; e += 256) {
    const int sj = e / M, k = e - sj * M;
    coef[e] = (j0 + sj < N) ? (T)u[(long)k * N + j0 + sj] : (T)0;
  }
  __syncthreads();
  if (rc >= plane) return;  // no barrier below
  T hr[AS_STEPS], hi[AS_STEPS];
  {
    const T a = Hf[rc], b = Hf[plane + rc];
#pragma unroll
    for (int q = 0; q < AS_STEPS; ++q) {
      hr[q] = a;
      hi[q] = b;
    }
  }
  for (int k0 = 0; k0 < M; k0 += AS_KC) {
    T kr[AS_KC], ki[AS_KC];
#pragma unroll
    for (int q = 0; q < AS_KC; ++q) {
      const bool ok = k0 + q < M;
      const T *Hk = Hf + (long)(ok ? k0 + q + 1 : 0) * 2 * plane;
      kr[q] = ok ? Hk[rc] : (T)0;
      ki[q] = ok ? Hk[plane + rc] : (T)0;
    }
#pragma unroll
    for (int q = 0; q < AS_KC; ++q) {
      if (k0 + q < M) {
#pragma unroll
        for (int sj = 0; sj < AS_STEPS; ++sj) {
          const T c = coef[sj * M + k0 + q];
          hr[sj] += c * kr[q];
          hi[sj] += c * ki[q];
        }
      }
    }
  }
  const int r = (int)(rc / dp), c = (int)(rc - (long)r * dp);
#pragma unroll
  for (int sj = 0; sj < AS_STEPS; ++sj) {
    const long j = j0 + sj;
    if (j < N) {
      // -i s (hr + i hi) = s hi - i s hr
      const T xr = s * hi[sj], xi = -s * hr[sj];
      T *Xj = X + j * 2 * plane;
      Xj[rc] = xr;
      Xj[plane + rc] = xi;
      if (Q) {
        T *Qj = Q + j * 2 * plane;
        Qj[rc] = (r == c ? (T)1 : (T)0) + xr * inv_p;
        Qj[plane + rc] = xi * inv_p;
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void stage_store(const StageArgs<T> &a, long j, int row, int col,
                                            T accr, T acci) {
  const long plane = (long)a.dp * a.dp;
  const long o = (long)row * a.dp + col;
  T vr = a.alpha * accr, vi = a.alpha * acci;
  T ar = 0, ai = 0, br = 0, bi = 0;
  const bool needA = a.betaA != (T)0 || (a.C2 && a.c2A != (T)0);
  const bool needB = a.betaB != (T)0 || (a.C2 && a.c2B != (T)0);
  if (needA) {
    const T *Aj = a.A + moff(a, j, a.strideA, a.segA);
    ar = Aj[o];
    ai = Aj[plane + o];
  }
  if (needB) {
    const T *Bj = a.B + moff(a, j, a.strideB, a.segB);
    br = Bj[o];
    bi = Bj[plane + o];
  }
  vr += a.betaA * ar + a.betaB * br;
  vi += a.betaA * ai + a.betaB * bi;
  if (row == col) vr += a.gamma;
  T xr[3] = {0, 0, 0}, xi[3] = {0, 0, 0};
  for (int q = 0; q < a.nx; ++q) {
    const T *Xq = a.xadd[q] + moff(a, j, a.strideC, a.segC);
    xr[q] = Xq[o];
    xi[q] = Xq[plane + o];
    vr += a.xc[q] * xr[q];
    vi += a.xc[q] * xi[q];
  }
  T *Cj = a.C + moff(a, j, a.strideC, a.segC);
  Cj[o] = vr;
  Cj[plane + o] = vi;
  if (a.C2) {
    T wr = a.c2P * accr + a.c2A * ar + a.c2B * br;
    T wi = a.c2P * acci + a.c2A * ai + a.c2B * bi;
    if (row == col) wr += a.g2;
    for (int q = 0; q < a.nx; ++q) {
      wr += a.xc2[q] * xr[q];
      wi += a.xc2[q] * xi[q];
    }
    T *C2j = a.C2 + moff(a, j, a.strideC, a.segC);
    C2j[o] = wr;
    C2j[plane + o] = wi;
  }
}

// Stage epilogues through LDS.  Each plane of a TR x TC output tile is
// written to LDS in the kernel's MFMA layout, then emitted by every thread
// as runs of four consecutive columns of a row (TC / 4 threads per row), so
// the addends are read and the outputs written as 16-byte vectors, whole
// row segments per wavefront, all loads of a run before its stores.  The
// coefficients are real, so the planes are independent.  Rows and columns
// at or beyond dp (a multiple of 16: a run is inside or outside) are
// skipped.  All 256 threads must call.
constexpr int EP_PAD = 4;  // LDS row padding: conflict-free writes in the MFMA layout

template <typename T>
__device__ __forceinline__ void st4(T *p, const T (&v)[4]) {
  if constexpr (sizeof(T) == 4) {
    *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    *(double2 *)p = make_double2(v[0], v[1]);
    *(double2 *)(p + 2) = make_double2(v[2], v[3]);
  }
}

template <typename T, int TR, int TC = TR>
__device__ __forceinline__ void stage_emit_plane(const StageArgs<T> &a, long j, int r0, int c0,
                                                 const T *sm, int pl) {
  constexpr int LD = TC + EP_PAD, TPR = TC / 4, RPP = 256 / TPR;
  const int t = threadIdx.x;
  const long plane = (long)a.dp * a.dp;
  const bool needA = a.betaA != (T)0 || (a.C2 && a.c2A != (T)0);
  const bool needB = a.betaB != (T)0 || (a.C2 && a.c2B != (T)0);
  const T *Aj = a.A + moff(a, j, a.strideA, a.segA), *Bj = a.B + moff(a, j, a.strideB, a.segB);
  const long oc = moff(a, j, a.strideC, a.segC);
  T *Cj = a.C + oc;
  T *C2j = a.C2 ? a.C2 + oc : nullptr;
  const int rr = t / TPR, cc = 4 * (t % TPR);
#pragma unroll
  for (int q = 0; q < TR / RPP; ++q) {
    const int row = rr + RPP * q;
    if (r0 + row >= a.dp || c0 + cc >= a.dp) continue;
    const long o = pl * plane + (long)(r0 + row) * a.dp + c0 + cc;
    T p[4], va[4] = {0, 0, 0, 0}, vb[4] = {0, 0, 0, 0}, x[3][4];
    ld4(sm + row * LD + cc, p);
    if (needA) ld4(Aj + o, va);
    if (needB) ld4(Bj + o, vb);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k < a.nx) {
        ld4(a.xadd[k] + oc + o, x[k]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) x[k][e] = 0;
      }
    }
    T c[4], c2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool diag = pl == 0 && r0 + row == c0 + cc + e;
      c[e] = a.alpha * p[e] + a.betaA * va[e] + a.betaB * vb[e] + (diag ? a.gamma : (T)0);
      c2[e] = a.c2P * p[e] + a.c2A * va[e] + a.c2B * vb[e] + (diag ? a.g2 : (T)0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k < a.nx) {
          c[e] += a.xc[k] * x[k][e];
          c2[e] += a.xc2[k] * x[k][e];
        }
      }
    }
    st4(Cj + o, c);
    if (C2j) st4(C2j + o, c2);
  }
}

// (32 MT) x (32 NT) tiles: wave w holds rows 16 MT (w >> 1) + 16 m + acc_row,
// columns 16 NT (w & 1) + 16 n + lane % 16.  sm holds 32 MT x (32 NT + 4)
// elements.
template <typename T, int MT, int NT>
__device__ __forceinline__ void stage_epilogue_t(const StageArgs<T> &a, long j, int r0, int c0,
                                                 T *sm, const v4<T> (&acc)[MT][NT][2]) {
  constexpr int LD = 32 * NT + EP_PAD;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = (w >> 1) * 16 * MT, wc = (w & 1) * 16 * NT;
#pragma unroll
  for (int pl = 0; pl < 2; ++pl) {
    __syncthreads();  // the previous use of sm is done
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int n = 0; n < NT; ++n)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          sm[(wr + 16 * m + acc_row<T>(lane, v)) * LD + wc + 16 * n + (lane & 15)] =
              acc[m][n][pl][v];
    __syncthreads();
    stage_emit_plane<T, 32 * MT, 32 * NT>(a, j, r0, c0, sm, pl);
  }
}

// dp a multiple of 16: one wavefront per 16x16 output tile, operands read
// straight from L1/L2 (small matrices: the whole matrix is a few tiles).
template <typename T, int OPA>
__global__ __launch_bounds__(256) void k_stage16(StageArgs<T> a) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t1 = a.dp >> 4;
  const long tiles = (long)t1 * t1;
  const long gt = (long)blockIdx.x * 4 + w;
  if (gt >= (long)a.nmat * tiles) return;  // wave-uniform, no barriers below
  const long j = gt / tiles;
  const int t = (int)(gt - j * tiles);
  const int r0 = (t / t1) * 16, c0 = (t % t1) * 16;
  const long plane = (long)a.dp * a.dp;
  CView<const T> A = cview<const T>(a.A + moff(a, j, a.strideA, a.segA), plane, a.dp);
  CView<const T> B = cview<const T>(a.B + moff(a, j, a.strideB, a.segB), plane, a.dp);
  v4<T> cr = vzero<T>(), ci = vzero<T>();
  wave_cgemm16<T, OPA, 0>(A, B, r0, c0, a.dp, cr, ci);
#pragma unroll
  for (int v = 0; v < 4; ++v)
    stage_store(a, j, r0 + acc_row<T>(lane, v), c0 + (lane & 15), cr[v], ci[v]);
}

// dp a multiple of 64: one workgroup per 64x64 output tile, LDS-staged,
// XCD-aware block order (all tiles of one step on one XCD's L2).
// FP64: at most 168 registers (three wavefronts per SIMD; the epilogue
// would otherwise take the kernel just past it)
template <typename T, int OPA, bool PF>
__global__ __attribute__((amdgpu_flat_work_group_size(1, 256),
                          amdgpu_waves_per_eu(sizeof(T) == 8 && !PF ? 3 : 1)))
void k_stage64(StageArgs<T> a, long padded) {
  __shared__ __align__(16) T lds[T64_LDS_ELEMS];
  const int t1 = a.dp >> 6;
  const long tiles = (long)t1 * t1;
  const long logical = xcd_logical_block(blockIdx.x, padded);
  if (logical >= (long)a.nmat * tiles) return;  // block-uniform
  const long j = logical / tiles;
  const int t = (int)(logical - j * tiles);
  const int r0 = (t / t1) * 64, c0 = (t % t1) * 64;
  const long plane = (long)a.dp * a.dp;
  CView<const T> A = cview<const T>(a.A + moff(a, j, a.strideA, a.segA), plane, a.dp);
  CView<const T> B = cview<const T>(a.B + moff(a, j, a.strideB, a.segB), plane, a.dp);
  v4<T> acc[2][2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      acc[m][n][0] = vzero<T>();
      acc[m][n][1] = vzero<T>();
    }
  wg_cgemm64<T, OPA, PF>(A, B, r0, c0, a.dp, lds, acc);
  stage_epilogue_t<T, 2, 2>(a, j, r0, c0, lds, acc);
}

// dp a multiple of 32 MT and of 32 NT: one workgroup per (32 MT) x (32 NT)
// output tile (wg_cgemm), the same LDS epilogue and XCD-aware block order.
// FP32: four wavefronts per SIMD (the compiler fits the register prefetch
// in 128 registers when asked; left alone it takes three)
template <typename T, int OPA, int MT, int NT>
__global__ __attribute__((amdgpu_flat_work_group_size(1, 256),
                          amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
void k_stage_t(StageArgs<T> a, long padded) {
  constexpr int TM = 32 * MT, TN = 32 * NT;
  constexpr int LE = tcg_lds_elems<TM, TN>(), LP = TM * (TN + EP_PAD);
  __shared__ __align__(16) T lds[LE > LP ? LE : LP];
  const int tr = a.dp / TM, tc = a.dp / TN;
  const long tiles = (long)tr * tc;
  const long logical = xcd_logical_block(blockIdx.x, padded);
  if (logical >= (long)a.nmat * tiles) return;  // block-uniform
  const long j = logical / tiles;
  const int t = (int)(logical - j * tiles);
  const int r0 = (t / tc) * TM, c0 = (t % tc) * TN;
  const long plane = (long)a.dp * a.dp;
  CView<const T> A = cview<const T>(a.A + moff(a, j, a.strideA, a.segA), plane, a.dp);
  CView<const T> B = cview<const T>(a.B + moff(a, j, a.strideB, a.segB), plane, a.dp);
  v4<T> acc[MT][NT][2];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      acc[m][n][0] = vzero<T>();
      acc[m][n][1] = vzero<T>();
    }
  wg_cgemm<T, OPA, MT, NT>(A, B, r0, c0, a.dp, lds, acc);
  stage_epilogue_t<T, MT, NT>(a, j, r0, c0, lds, acc);
}

// dp a multiple of 16 but not of 64 (80, 96, 112, ...): one workgroup per
// 32x32 output tile (4 waves, one 16x16 MFMA tile each), operand chunks of
// 16 inner indices staged in LDS; rows / columns beyond dp read as zero and
// are not stored.  Waste is at most (dp + 16)^2 / dp^2 instead of the
// (dp + 48)^2 / dp^2 of 64-wide tiles.
constexpr int T32_BK = 16, T32_LD = 32 + 16;

template <typename T, int OPA>
__global__ __launch_bounds__(256) void k_stage32(StageArgs<T> a, long padded) {
  __shared__ __align__(16) T lds[4 * T32_BK * T32_LD];
  T *Asr = lds, *Asi = Asr + T32_BK * T32_LD;
  T *Bsr = Asi + T32_BK * T32_LD, *Bsi = Bsr + T32_BK * T32_LD;
  const int t1 = (a.dp + 31) >> 5;
  const long tiles = (long)t1 * t1;
  const long logical = xcd_logical_block(blockIdx.x, padded);
  if (logical >= (long)a.nmat * tiles) return;  // block-uniform
  const long j = logical / tiles;
  const int tt = (int)(logical - j * tiles);
  const int r0 = (tt / t1) * 32, c0 = (tt % t1) * 32;
  const int dp = a.dp;
  const long plane = (long)dp * dp;
  const T *Aj = a.A + moff(a, j, a.strideA, a.segA), *Bj = a.B + moff(a, j, a.strideB, a.segB);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int wr = (w >> 1) * 16, wc = (w & 1) * 16;
  v4<T> cr = vzero<T>(), ci = vzero<T>();
  // one chunk's operands, two complex elements of op(A) and of B per
  // thread: op(A)[r0 .. r0+31][k0 .. k0+15] as As[k][r], B[k0 ..][c0 ..] as
  // Bs[k][c].  The next chunk is loaded into registers while the current
  // one is multiplied; the barriers order LDS only.
  T par[2], pai[2], pbr[2], pbi[2];
  auto load = [&](int k0) {
    if (OPA == 0) {
      const int r = t >> 3, kq = (t & 7) * 2;
      const bool ok = r0 + r < dp;
      const long o = ok ? (long)(r0 + r) * dp + k0 + kq : 0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const T vr = Aj[o + q], vi = Aj[plane + o + q];
        par[q] = ok ? vr : (T)0;
        pai[q] = ok ? vi : (T)0;
      }
    } else {
      const int k = t >> 4, rq = (t & 15) * 2;
      const bool ok = r0 + rq < dp;
      const long o = ok ? (long)(k0 + k) * dp + r0 + rq : 0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const T vr = Aj[o + q], vi = Aj[plane + o + q];
        par[q] = ok ? vr : (T)0;
        pai[q] = ok ? -vi : (T)0;
      }
    }
    const int k = t >> 4, cq = (t & 15) * 2;
    const bool ok = c0 + cq < dp;
    const long o = ok ? (long)(k0 + k) * dp + c0 + cq : 0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const T vr = Bj[o + q], vi = Bj[plane + o + q];
      pbr[q] = ok ? vr : (T)0;
      pbi[q] = ok ? vi : (T)0;
    }
  };
  auto store = [&]() {
    if (OPA == 0) {
      const int r = t >> 3, kq = (t & 7) * 2;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        Asr[(kq + q) * T32_LD + r] = par[q];
        Asi[(kq + q) * T32_LD + r] = pai[q];
      }
    } else {
      const int k = t >> 4, rq = (t & 15) * 2;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        Asr[k * T32_LD + rq + q] = par[q];
        Asi[k * T32_LD + rq + q] = pai[q];
      }
    }
    const int k = t >> 4, cq = (t & 15) * 2;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      Bsr[k * T32_LD + cq + q] = pbr[q];
      Bsi[k * T32_LD + cq + q] = pbi[q];
    }
  };
  load(0);
  for (int k0 = 0; k0 < dp; k0 += T32_BK) {
    store();
    lds_barrier();
    if (k0 + T32_BK < dp) load(k0 + T32_BK);  // block-uniform
#pragma unroll
    for (int k4 = 0; k4 < T32_BK; k4 += 4) {
      const T ar = Asr[(k4 + kk) * T32_LD + wr + i], ai = Asi[(k4 + kk) * T32_LD + wr + i];
      const T br = Bsr[(k4 + kk) * T32_LD + wc + i], bi = Bsi[(k4 + kk) * T32_LD + wc + i];
      cr = mfma4(ar, br, cr);
      cr = mfma4(-ai, bi, cr);
      ci = mfma4(ar, bi, ci);
      ci = mfma4(ai, br, ci);
    }
    lds_barrier();
  }
  // epilogue through LDS (32 x 36 elements per plane, over the operand
  // chunks: the product's last LDS reads are behind the barrier above)
  T *sm = lds;
  static_assert(4 * T32_BK * T32_LD >= 32 * (32 + EP_PAD), "LDS tile too small");
#pragma unroll
  for (int pl = 0; pl < 2; ++pl) {
    if (pl) __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v)
      sm[(wr + acc_row<T>(lane, v)) * (32 + EP_PAD) + wc + (lane & 15)] = pl ? ci[v] : cr[v];
    __syncthreads();
    stage_emit_plane<T, 32>(a, j, r0, c0, sm, pl);
  }
}

// bf16x3 variant of k_stage64 (FP32 storage; the split-product tile of
// qoc_tile.h): one workgroup per 64 x 64 output tile, 4 waves of 32 x 32,
// the same LDS epilogue and XCD-aware block order, four wavefronts per SIMD
// (each chunk loaded just before its stores: the registers of a register
// prefetch would leave three).  Tiles of 128 x 64 and 64 x 128, and a
// second chunk of operands in registers, were slower: they cost occupancy,
// and the split products need the latency hiding.
template <int OPA>
__global__ __attribute__((amdgpu_flat_work_group_size(1, 256), amdgpu_waves_per_eu(4, 4)))
void k_stage64_bf3(StageArgs<float> a, long padded) {
  __shared__ BfLds L;
  const int t1 = a.dp >> 6;
  const long tiles = (long)t1 * t1;
  const long logical = xcd_logical_block(blockIdx.x, padded);
  if (logical >= (long)a.nmat * tiles) return;  // block-uniform
  const long j = logical / tiles;
  const int t = (int)(logical - j * tiles);
  const int r0 = (t / t1) * 64, c0 = (t % t1) * 64;
  const long plane = (long)a.dp * a.dp;
  const TOp<float> A = make_top<float>(a.A + moff(a, j, a.strideA, a.segA), plane, a.dp, a.dp);
  const TOp<float> B = make_top<float>(a.B + moff(a, j, a.strideB, a.segB), plane, a.dp, a.dp);
  f32x4 acc[2][2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      acc[m][n][0] = vzero<float>();
      acc[m][n][1] = vzero<float>();
    }
  // op(A) = A: inner index along rows of A; op(A) = A^H: along columns,
  // conjugated; B as stored: inner index along columns of B.  The tiles lie
  // inside the matrices (dp a multiple of 64, d <= 1024: both planes of a
  // matrix within 2^31 bytes).
  ctile_bf3<2, 2, OPA == 0, OPA == 1, false, false, true, false>(A, B, r0, c0, a.dp, L, acc);
  stage_epilogue_t<float, 2, 2>(a, j, r0, c0, (float *)&L, acc);
}

template <typename T>
hipError_t launch_assemble(const T *Hf, const double *u, int dp, int M, int N, T s, T inv_p,
                           T *X, T *Q, hipStream_t st) {
  const long plane = (long)dp * dp;
  dim3 grid((unsigned)((N + AS_STEPS - 1) / AS_STEPS), (unsigned)((plane + 255) / 256));
  const size_t shm = sizeof(T) * AS_STEPS * M;
  hipLaunchKernelGGL(k_assemble<T>, grid, dim3(256), shm, st, Hf, u, dp, M, N, s, inv_p, X, Q);
  return hipGetLastError();
}

bool stage_bf3_ok(int dp) { return dp % 64 == 0; }

template <typename T> hipError_t launch_stage(int opa, const StageArgs<T> &a, hipStream_t st) {
  if (a.nmat <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (a.bf3 && stage_bf3_ok(a.dp)) {
      const long t1 = a.dp / 64;
      const long total = (long)a.nmat * t1 * t1;
      const long padded = (total + 7) / 8 * 8;
      if (opa)
        hipLaunchKernelGGL((k_stage64_bf3<1>), dim3((unsigned)padded), dim3(256), 0, st, a,
                           padded);
      else
        hipLaunchKernelGGL((k_stage64_bf3<0>), dim3((unsigned)padded), dim3(256), 0, st, a,
                           padded);
      return hipGetLastError();
    }
  }
  // FP32, padded d a multiple of 128 and at least 256: 64 x 128 tiles (each
  // wave 32 x 64), the same sums as the 64 x 64 tiles; the wider tile
  // halves the A-operand traffic per flop (spin chain: 8.13 -> 8.02 ms per
  // product; at d_pad 128 the 64 x 64 tiles keep more workgroups busy)
  if constexpr (sizeof(T) == 4) {
    if (a.dp % 128 == 0 && a.dp >= 256) {
      const long total = (long)a.nmat * (a.dp / 64) * (a.dp / 128);
      const long padded = (total + 7) / 8 * 8;
      if (opa)
        hipLaunchKernelGGL((k_stage_t<T, 1, 2, 4>), dim3((unsigned)padded), dim3(256), 0, st, a,
                           padded);
      else
        hipLaunchKernelGGL((k_stage_t<T, 0, 2, 4>), dim3((unsigned)padded), dim3(256), 0, st, a,
                           padded);
      return hipGetLastError();
    }
  }
  if (a.dp % 64 == 0) {
    const long t1 = a.dp / 64;
    const long total = (long)a.nmat * t1 * t1;
    const long padded = (total + 7) / 8 * 8;
    // short inner dimension (d_pad <= 128): register prefetch; longer ones:
    // the occupancy-friendly loop
    const bool pf = a.dp <= 128;
    if (opa && pf)
      hipLaunchKernelGGL((k_stage64<T, 1, true>), dim3((unsigned)padded), dim3(256), 0, st, a,
                         padded);
    else if (opa)
      hipLaunchKernelGGL((k_stage64<T, 1, false>), dim3((unsigned)padded), dim3(256), 0, st, a,
                         padded);
    else if (pf)
      hipLaunchKernelGGL((k_stage64<T, 0, true>), dim3((unsigned)padded), dim3(256), 0, st, a,
                         padded);
    else
      hipLaunchKernelGGL((k_stage64<T, 0, false>), dim3((unsigned)padded), dim3(256), 0, st, a,
                         padded);
  } else if (a.dp > 48) {
    const long t1 = (a.dp + 31) / 32;
    const long total = (long)a.nmat * t1 * t1;
    const long padded = (total + 7) / 8 * 8;
    if (opa)
      hipLaunchKernelGGL((k_stage32<T, 1>), dim3((unsigned)padded), dim3(256), 0, st, a, padded);
    else
      hipLaunchKernelGGL((k_stage32<T, 0>), dim3((unsigned)padded), dim3(256), 0, st, a, padded);
  } else {
    const long t1 = a.dp / 16;
    const long total = (long)a.nmat * t1 * t1;
    const long blocks = (total + 3) / 4;
    if (opa)
      hipLaunchKernelGGL((k_stage16<T, 1>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((k_stage16<T, 0>), dim3((unsigned)blocks), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

template <typename T> __global__ void k_fill(T *p, long n, T v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T> hipError_t launch_fill(T *p, long n, T v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

template <typename T> __global__ void k_copy(T *dst, const T *src, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <typename T> hipError_t launch_copy(T *dst, const T *src, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  long blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_copy<T>, dim3((unsigned)blocks), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

template hipError_t launch_copy<float>(float *, const float *, long, hipStream_t);
template hipError_t launch_copy<double>(double *, const double *, long, hipStream_t);

// count segments of n elements: dst + b dstride <- src + b sstride
template <typename T>
__global__ void k_copy_strided(T *dst, long dstride, const T *src, long sstride, long n, long count) {
  const long b = blockIdx.y;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    dst[b * dstride + i] = src[b * sstride + i];
}

template <typename T>
hipError_t launch_copy_strided(T *dst, long dstride, const T *src, long sstride, long n,
                               long count, hipStream_t st) {
  if (n <= 0 || count <= 0) return hipSuccess;
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  for (long b0 = 0; b0 < count; b0 += 65535) {
    const long cnt = count - b0 < 65535 ? count - b0 : 65535;
    hipLaunchKernelGGL(k_copy_strided<T>, dim3((unsigned)blocks, (unsigned)cnt), dim3(256), 0, st,
                       dst + b0 * dstride, dstride, src + b0 * sstride, sstride, n, cnt);
  }
  return hipGetLastError();
}
template hipError_t launch_copy_strided<float>(float *, long, const float *, long, long, long,
                                               hipStream_t);
template hipError_t launch_copy_strided<double>(double *, long, const double *, long, long, long,
                                                hipStream_t);
template hipError_t launch_assemble<float>(const float *, const double *, int, int, int, float,
                                           float, float *, float *, hipStream_t);
template hipError_t launch_assemble<double>(const double *, const double *, int, int, int, double,
                                            double, double *, double *, hipStream_t);
template hipError_t launch_stage<float>(int, const StageArgs<float> &, hipStream_t);
template hipError_t launch_stage<double>(int, const StageArgs<double> &, hipStream_t);
template hipError_t launch_fill<float>(float *, long, float, hipStream_t);
template hipError_t launch_fill<double>(double *, long, double, hipStream_t);
template hipError_t launch_fill<unsigned long long>(unsigned long long *, long, unsigned long long,
                                                    hipStream_t);

}  // namespace qoc
