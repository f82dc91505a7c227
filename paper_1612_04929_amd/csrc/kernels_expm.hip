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

namespace qoc {

template <typename T>
__global__ __launch_bounds__(256) void k_assemble(const T *__restrict__ Hf,
                                                  const double *__restrict__ u, int dp, int M,
                                                  int N, T s, T inv_p, T *__restrict__ X,
                                                  T *__restrict__ Q) {
  const long plane = (long)dp * dp;
  const long total = (long)N * plane;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const long j = e / plane, rc = e - j * plane;
    T hr = Hf[rc], hi = Hf[plane + rc];
    for (int k = 0; k < M; ++k) {
      const T c = (T)u[(long)k * N + j];
      hr += c * Hf[(long)(k + 1) * 2 * plane + rc];
      hi += c * Hf[(long)(k + 1) * 2 * plane + plane + rc];
    }
    // -i s (hr + i hi) = s hi - i s hr
    const T xr = s * hi, xi = -s * hr;
    T *Xj = X + j * 2 * plane;
    Xj[rc] = xr;
    Xj[plane + rc] = xi;
    if (Q) {
      const int r = (int)(rc / dp), c = (int)(rc - (long)r * dp);
      T *Qj = Q + j * 2 * plane;
      Qj[rc] = (r == c ? (T)1 : (T)0) + xr * inv_p;
      Qj[plane + rc] = xi * inv_p;
    }
  }
}

template <typename T>
__device__ __forceinline__ void stage_store(const StageArgs<T> &a, long j, int row, int col,
                                            T accr, T acci) {
  const long plane = (long)a.dp * a.dp;
  const long o = (long)row * a.dp + col;
  T vr = a.alpha * accr, vi = a.alpha * acci;
  if (a.betaA != (T)0) {
    const T *Aj = a.A + j * a.strideA;
    vr += a.betaA * Aj[o];
    vi += a.betaA * Aj[plane + o];
  }
  if (a.betaB != (T)0) {
    const T *Bj = a.B + j * a.strideB;
    vr += a.betaB * Bj[o];
    vi += a.betaB * Bj[plane + o];
  }
  if (row == col) vr += a.gamma;
  T *Cj = a.C + j * a.strideC;
  Cj[o] = vr;
  Cj[plane + o] = vi;
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
  CView<const T> A = cview<const T>(a.A + j * a.strideA, plane, a.dp);
  CView<const T> B = cview<const T>(a.B + j * a.strideB, plane, a.dp);
  v4<T> cr = vzero<T>(), ci = vzero<T>();
  wave_cgemm16<T, OPA, 0>(A, B, r0, c0, a.dp, cr, ci);
#pragma unroll
  for (int v = 0; v < 4; ++v)
    stage_store(a, j, r0 + acc_row<T>(lane, v), c0 + (lane & 15), cr[v], ci[v]);
}

// dp a multiple of 64: one workgroup per 64x64 output tile, LDS-staged,
// XCD-aware block order (all tiles of one step on one XCD's L2).
template <typename T, int OPA>
__global__ __launch_bounds__(256) void k_stage64(StageArgs<T> a, long padded) {
  __shared__ T lds[T64_LDS_ELEMS];
  const int t1 = a.dp >> 6;
  const long tiles = (long)t1 * t1;
  const long logical = xcd_logical_block(blockIdx.x, padded);
  if (logical >= (long)a.nmat * tiles) return;  // block-uniform
  const long j = logical / tiles;
  const int t = (int)(logical - j * tiles);
  const int r0 = (t / t1) * 64, c0 = (t % t1) * 64;
  const long plane = (long)a.dp * a.dp;
  CView<const T> A = cview<const T>(a.A + j * a.strideA, plane, a.dp);
  CView<const T> B = cview<const T>(a.B + j * a.strideB, plane, a.dp);
  v4<T> acc[2][2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      acc[m][n][0] = vzero<T>();
      acc[m][n][1] = vzero<T>();
    }
  wg_cgemm64<T, OPA>(A, B, r0, c0, a.dp, lds, acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        stage_store(a, j, r0 + wr + 16 * m + acc_row<T>(lane, v), c0 + wc + 16 * n + (lane & 15),
                    acc[m][n][0][v], acc[m][n][1][v]);
}

// ---------------------------------------------------------------------------
// bf16x3 split-precision variant of k_stage64 (FP32 storage, FP32
// accumulation).  Each FP32 operand x is split on its way into LDS as
// hi = RNE_bf16(x), lo = RNE_bf16(x - hi) (x - hi is exact in FP32), and
// every real product is hi*hi + hi*lo + lo*hi on the bf16 16x16x32 MFMA;
// the dropped lo*lo term and the split leave a relative error of a few
// 2^-17 per product.  The inner dimension runs in chunks of 32 (one MFMA
// K); LDS holds the chunk of op(A) as [plane][row][k] and of B as
// [plane][col][k] (k contiguous, row stride 40 halves), planes re_hi,
// re_lo, im_hi, im_lo, so each lane's operand is one 16-byte LDS read.
// The next chunk's FP32 operands are loaded into registers while the
// current one is multiplied.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int BF_BK = 32;
constexpr int BF_LDK = BF_BK + 8;

__device__ __forceinline__ f32x4 mfma_bf(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 bf_neg(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

// 8 FP32 values -> hi / lo bf16 parts.
__device__ __forceinline__ void bf_split8(const float (&x)[8], bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const __bf16 h = (__bf16)x[q];
    hi[q] = h;
    lo[q] = (__bf16)(x[q] - (float)h);
  }
}

// LDS of one 64x64 output tile: 4 planes x 64 rows x BF_LDK for each operand.
struct alignas(16) BfLds {
  __bf16 a[4][64][BF_LDK];
  __bf16 b[4][64][BF_LDK];
};

// FP32 staging registers of one thread for one chunk: 8 k of one row of
// op(A) and 8 k of one column of B, real and imaginary parts.
struct BfRegs {
  float ar[8], ai[8], br[8], bi[8];
};

template <int OPA>
__device__ __forceinline__ void bf_load(const StageArgs<float> &a, const float *Aj,
                                        const float *Bj, long plane, int r0, int c0, int k0,
                                        BfRegs &g) {
  const int t = threadIdx.x;
  const int dp = a.dp;
  if (OPA == 0) {
    // row r, k = 8 kq .. 8 kq + 7 of A (contiguous): two 16-byte loads per plane
    const int r = t >> 2, kq = t & 3;
    const long o = (long)(r0 + r) * dp + k0 + 8 * kq;
    const float4 *pr = (const float4 *)(Aj + o), *pi = (const float4 *)(Aj + plane + o);
    const float4 r0v = pr[0], r1v = pr[1], i0v = pi[0], i1v = pi[1];
    g.ar[0] = r0v.x; g.ar[1] = r0v.y; g.ar[2] = r0v.z; g.ar[3] = r0v.w;
    g.ar[4] = r1v.x; g.ar[5] = r1v.y; g.ar[6] = r1v.z; g.ar[7] = r1v.w;
    g.ai[0] = i0v.x; g.ai[1] = i0v.y; g.ai[2] = i0v.z; g.ai[3] = i0v.w;
    g.ai[4] = i1v.x; g.ai[5] = i1v.y; g.ai[6] = i1v.z; g.ai[7] = i1v.w;
  } else {
    // op(A)[r][k] = conj(A[k][r]): lanes along r are contiguous in memory
    const int r = t & 63, kq = t >> 6;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const long o = (long)(k0 + 8 * kq + q) * dp + r0 + r;
      g.ar[q] = Aj[o];
      g.ai[q] = -Aj[plane + o];
    }
  }
  {
    const int c = t & 63, kq = t >> 6;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const long o = (long)(k0 + 8 * kq + q) * dp + c0 + c;
      g.br[q] = Bj[o];
      g.bi[q] = Bj[plane + o];
    }
  }
}

template <int OPA>
__device__ __forceinline__ void bf_store(const BfRegs &g, BfLds &L) {
  const int t = threadIdx.x;
  const int ra = OPA == 0 ? (t >> 2) : (t & 63), ka = OPA == 0 ? (t & 3) : (t >> 6);
  const int cb = t & 63, kb = t >> 6;
  bf16x8 h, l;
  bf_split8(g.ar, h, l);
  *(bf16x8 *)&L.a[0][ra][8 * ka] = h;
  *(bf16x8 *)&L.a[1][ra][8 * ka] = l;
  bf_split8(g.ai, h, l);
  *(bf16x8 *)&L.a[2][ra][8 * ka] = h;
  *(bf16x8 *)&L.a[3][ra][8 * ka] = l;
  bf_split8(g.br, h, l);
  *(bf16x8 *)&L.b[0][cb][8 * kb] = h;
  *(bf16x8 *)&L.b[1][cb][8 * kb] = l;
  bf_split8(g.bi, h, l);
  *(bf16x8 *)&L.b[2][cb][8 * kb] = h;
  *(bf16x8 *)&L.b[3][cb][8 * kb] = l;
}

template <int OPA>
__global__ __launch_bounds__(256) void k_stage64_bf3(StageArgs<float> a, long padded) {
  __shared__ BfLds L;
  const int t1 = a.dp >> 6;
  const long tiles = (long)t1 * t1;
  const long logical = xcd_logical_block(blockIdx.x, padded);
  if (logical >= (long)a.nmat * tiles) return;  // block-uniform
  const long j = logical / tiles;
  const int t = (int)(logical - j * tiles);
  const int r0 = (t / t1) * 64, c0 = (t % t1) * 64;
  const long plane = (long)a.dp * a.dp;
  const float *Aj = a.A + j * a.strideA;
  const float *Bj = a.B + j * a.strideB;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, g8 = 8 * (lane >> 4);
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  f32x4 acc[2][2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      acc[m][n][0] = vzero<float>();
      acc[m][n][1] = vzero<float>();
    }
  BfRegs g;
  bf_load<OPA>(a, Aj, Bj, plane, r0, c0, 0, g);
  for (int k0 = 0; k0 < a.dp; k0 += BF_BK) {
    bf_store<OPA>(g, L);
    __syncthreads();
    if (k0 + BF_BK < a.dp) bf_load<OPA>(a, Aj, Bj, plane, r0, c0, k0 + BF_BK, g);
    bf16x8 fa[2][4], fb[2][4], na[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        fa[m][p] = *(const bf16x8 *)&L.a[p][wr + 16 * m + i][g8];
        fb[m][p] = *(const bf16x8 *)&L.b[p][wc + 16 * m + i][g8];
      }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      na[m][0] = bf_neg(fa[m][2]);
      na[m][1] = bf_neg(fa[m][3]);
    }
    // Re += Ar Br - Ai Bi ; Im += Ar Bi + Ai Br, each real product as
    // hi*hi + hi*lo + lo*hi; consecutive MFMAs go to different accumulators
#define BF3_TERM(dst, X, Y)                                                    \
  _Pragma("unroll") for (int m = 0; m < 2; ++m)                                \
  _Pragma("unroll") for (int n = 0; n < 2; ++n)                                \
    acc[m][n][dst] = mfma_bf(X, Y, acc[m][n][dst]);
    BF3_TERM(0, fa[m][0], fb[n][0])
    BF3_TERM(1, fa[m][0], fb[n][2])
    BF3_TERM(0, fa[m][0], fb[n][1])
    BF3_TERM(1, fa[m][0], fb[n][3])
    BF3_TERM(0, fa[m][1], fb[n][0])
    BF3_TERM(1, fa[m][1], fb[n][2])
    BF3_TERM(0, na[m][0], fb[n][2])
    BF3_TERM(1, fa[m][2], fb[n][0])
    BF3_TERM(0, na[m][0], fb[n][3])
    BF3_TERM(1, fa[m][2], fb[n][1])
    BF3_TERM(0, na[m][1], fb[n][2])
    BF3_TERM(1, fa[m][3], fb[n][0])
#undef BF3_TERM
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        stage_store(a, j, r0 + wr + 16 * m + acc_row<float>(lane, v),
                    c0 + wc + 16 * n + (lane & 15), acc[m][n][0][v], acc[m][n][1][v]);
}

template <typename T>
hipError_t launch_assemble(const T *Hf, const double *u, int dp, int M, int N, T s, T inv_p,
                           T *X, T *Q, hipStream_t st) {
  const long total = (long)N * dp * dp;
  long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_assemble<T>, dim3((unsigned)blocks), dim3(256), 0, st, Hf, u, dp, M, N, s,
                     inv_p, X, Q);
  return hipGetLastError();
}

template <typename T> hipError_t launch_stage(int opa, const StageArgs<T> &a, hipStream_t st) {
  if (a.nmat <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (a.bf3 && a.dp % 64 == 0) {
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
  if (a.dp % 64 == 0) {
    const long t1 = a.dp / 64;
    const long total = (long)a.nmat * t1 * t1;
    const long padded = (total + 7) / 8 * 8;
    if (opa)
      hipLaunchKernelGGL((k_stage64<T, 1>), dim3((unsigned)padded), dim3(256), 0, st, a, padded);
    else
      hipLaunchKernelGGL((k_stage64<T, 0>), dim3((unsigned)padded), dim3(256), 0, st, a, padded);
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
