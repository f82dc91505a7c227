// Device-side building blocks shared by the libqoc kernels (gfx950 / CDNA4).
//
// Complex matrices are stored planar: a real plane and an imaginary plane,
// each row-major.  A complex product is four real MFMA products
//   Re(AB) = Ar Br - Ai Bi,   Im(AB) = Ar Bi + Ai Br,
// i.e. the real block form of the paper's complex-to-real isomorphism
// (Sec. III, eq. 8) applied to one operand only, without materialising the
// redundant 2d x 2d block matrix.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qoc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct V4T;
template <> struct V4T<float> { typedef f32x4 type; };
template <> struct V4T<double> { typedef f64x4 type; };
template <typename T> using v4 = typename V4T<T>::type;

// D(16x16) += A(16x4) B(4x16).  Operand layout: lane l holds A[l%16][l/16]
// and B[l/16][l%16].  Result register v of lane l holds column l%16 and row
// acc_row<T>(l, v): 4*(l/16)+v for the FP32 instruction, 4*v+(l/16) for the
// FP64 one (checked on the device).
__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T> __device__ __forceinline__ int acc_row(int lane, int v);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int v) {
  return 4 * (lane >> 4) + v;
}
template <> __device__ __forceinline__ int acc_row<double>(int lane, int v) {
  return 4 * v + (lane >> 4);
}

template <typename T> __device__ __forceinline__ v4<T> vzero() {
  v4<T> z;
  z[0] = 0; z[1] = 0; z[2] = 0; z[3] = 0;
  return z;
}

// Planar complex matrix view: element (r, c) at re[r*ld + c], im[r*ld + c].
template <typename T> struct CView {
  T *re, *im;
  int ld;
};

template <typename T>
__device__ __forceinline__ CView<T> cview(T *base, long plane, int ld) {
  CView<T> v;
  v.re = base;
  v.im = base + plane;
  v.ld = ld;
  return v;
}

// One wavefront accumulates the 16x16 complex tile (r0, c0) of
// op(A) * op(B) over an inner dimension K (multiple of 4), reading operands
// straight from global memory (L1/L2 resident).  OPA / OPB: 0 = as stored,
// 1 = conjugate transpose.  cr, ci: real / imaginary accumulators.  The
// operands of four inner chunks are loaded before their products, so one
// memory round trip serves sixteen inner indices.
template <typename T, int OPA, int OPB>
__device__ __forceinline__ void wave_cgemm16(CView<const T> A, CView<const T> B, int r0,
                                             int c0, int K, v4<T> &cr, v4<T> &ci) {
  const int lane = threadIdx.x & 63, i = lane & 15, kk = lane >> 4;
  auto ld = [&](int k, T &ar, T &ai, T &br, T &bi) {
    if (OPA == 0) {
      const long o = (long)(r0 + i) * A.ld + (k + kk);
      ar = A.re[o]; ai = A.im[o];
    } else {
      const long o = (long)(k + kk) * A.ld + (r0 + i);
      ar = A.re[o]; ai = -A.im[o];
    }
    if (OPB == 0) {
      const long o = (long)(k + kk) * B.ld + (c0 + i);
      br = B.re[o]; bi = B.im[o];
    } else {
      const long o = (long)(c0 + i) * B.ld + (k + kk);
      br = B.re[o]; bi = -B.im[o];
    }
  };
  auto mac = [&](T ar, T ai, T br, T bi) {
    cr = mfma4(ar, br, cr);
    cr = mfma4(-ai, bi, cr);
    ci = mfma4(ar, bi, ci);
    ci = mfma4(ai, br, ci);
  };
  int k = 0;
  for (; k + 16 <= K; k += 16) {
    T ar[4], ai[4], br[4], bi[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) ld(k + 4 * u, ar[u], ai[u], br[u], bi[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) mac(ar[u], ai[u], br[u], bi[u]);
  }
  for (; k < K; k += 4) {
    T ar, ai, br, bi;
    ld(k, ar, ai, br, bi);
    mac(ar, ai, br, bi);
  }
}

// ---------------------------------------------------------------------------
// Workgroup barrier that orders LDS traffic only.  __syncthreads() also
// waits for every outstanding global-memory operation of the wave (vmcnt
// covers loads and stores on this architecture), which would drain a
// register prefetch ring at every step.  Use only where no global-memory
// visibility between the waves of the workgroup is needed.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  // s_waitcnt lgkmcnt(0), vmcnt and expcnt left at their maxima
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Workgroup (256 threads, 4 waves) LDS-tiled 64x64 complex tile of
// C = op(A) * B, with op(A) = A or A^H and B as stored.  The inner
// dimension runs in chunks of BK = 16 staged in LDS in k-major layout
// (row stride 64 + 16 elements, which keeps the 16-lane fragment reads of
// each half-wave on distinct banks); with PF the next chunk is loaded into
// registers while the current one is multiplied (short inner dimensions:
// it pays at d_pad 128, while at d_pad 512 the registers it takes cost more
// occupancy than it hides latency).  Wave w owns the 32x32 sub-tile
// (32*(w>>1), 32*(w&1)) as 2x2 MFMA tiles.
// ---------------------------------------------------------------------------
constexpr int T64_BK = 16;
constexpr int T64_LD = 64 + 16;
// LDS elements of T needed by wg_cgemm64: A and B chunks, re and im planes.
constexpr int T64_LDS_ELEMS = 4 * T64_BK * T64_LD;

template <typename T, int OPA, bool PF = true>
__device__ __forceinline__ void wg_cgemm64(CView<const T> A, CView<const T> B, int r0, int c0,
                                           int K, T *lds, v4<T> (&acc)[2][2][2]) {
  T *Asr = lds;
  T *Asi = Asr + T64_BK * T64_LD;
  T *Bsr = Asi + T64_BK * T64_LD;
  T *Bsi = Bsr + T64_BK * T64_LD;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  // this thread's slots of a chunk: op(A) as As[k][r], B as Bs[k][c]
  const int ar_ = t >> 2, akq = (t & 3) * 4;   // OPA = 0: row, inner offset
  const int ak = t >> 4, arq = (t & 15) * 4;   // OPA = 1: inner, row offset
  const int bk = t >> 4, bcq = (t & 15) * 4;
  T va[2][4], vb[2][4];  // next chunk, loaded while the current one is multiplied
  auto load = [&](int k0) {
    const long oa = OPA == 0 ? (long)(r0 + ar_) * A.ld + k0 + akq : (long)(k0 + ak) * A.ld + r0 + arq;
    const long ob = (long)(k0 + bk) * B.ld + c0 + bcq;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      va[0][q] = A.re[oa + q];
      va[1][q] = A.im[oa + q];
      vb[0][q] = B.re[ob + q];
      vb[1][q] = B.im[ob + q];
    }
  };
  if (PF) load(0);
  for (int k0 = 0; k0 < K; k0 += T64_BK) {
    if (!PF) load(k0);  // without prefetch: fewer registers, more workgroups per unit
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (OPA == 0) {
        Asr[(akq + q) * T64_LD + ar_] = va[0][q];
        Asi[(akq + q) * T64_LD + ar_] = va[1][q];
      } else {
        Asr[ak * T64_LD + arq + q] = va[0][q];
        Asi[ak * T64_LD + arq + q] = -va[1][q];
      }
      Bsr[bk * T64_LD + bcq + q] = vb[0][q];
      Bsi[bk * T64_LD + bcq + q] = vb[1][q];
    }
    __syncthreads();
    if (PF && k0 + T64_BK < K) load(k0 + T64_BK);  // uniform
#pragma unroll
    for (int k4 = 0; k4 < T64_BK; k4 += 4) {
      T ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        ar[m] = Asr[(k4 + kk) * T64_LD + wr + 16 * m + i];
        ai[m] = Asi[(k4 + kk) * T64_LD + wr + 16 * m + i];
        br[m] = Bsr[(k4 + kk) * T64_LD + wc + 16 * m + i];
        bi[m] = Bsi[(k4 + kk) * T64_LD + wc + 16 * m + i];
      }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          acc[m][n][0] = mfma4(ar[m], br[n], acc[m][n][0]);
          acc[m][n][0] = mfma4(-ai[m], bi[n], acc[m][n][0]);
          acc[m][n][1] = mfma4(ar[m], bi[n], acc[m][n][1]);
          acc[m][n][1] = mfma4(ai[m], br[n], acc[m][n][1]);
        }
    }
    if (PF)
      lds_barrier();  // the chunk's LDS reads are done; the prefetch stays in flight
    else
      __syncthreads();
  }
}

// The same product on a (32 MT) x (32 NT) tile: wave w owns the
// (16 MT) x (16 NT) sub-tile (16 MT (w >> 1), 16 NT (w & 1)) as MT x NT
// MFMA tiles; chunks of 16 inner indices, LDS row stride tile + 16.  lds
// holds 2 T64_BK (TM + TN + 32) elements.
template <int TM, int TN> constexpr int tcg_lds_elems() { return 2 * T64_BK * (TM + TN + 32); }

template <typename T, int OPA, int MT, int NT>
__device__ __forceinline__ void wg_cgemm(CView<const T> A, CView<const T> B, int r0, int c0,
                                         int K, T *lds, v4<T> (&acc)[MT][NT][2]) {
  constexpr int TM = 32 * MT, TN = 32 * NT, LDA = TM + 16, LDB = TN + 16;
  constexpr int UA = TM / 64, UB = TN / 64;  // 4-element groups per thread and plane
  T *Asr = lds;
  T *Asi = Asr + T64_BK * LDA;
  T *Bsr = Asi + T64_BK * LDA;
  T *Bsi = Bsr + T64_BK * LDB;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int wr = (w >> 1) * 16 * MT, wc = (w & 1) * 16 * NT;
  const int ar_ = t >> 2, akq = (t & 3) * 4;   // OPA = 0: row (+ 64 u), inner offset
  const int ak = t >> 4, arq = (t & 15) * 4;   // OPA = 1: inner, row offset (+ 64 u)
  const int bk = t >> 4, bcq = (t & 15) * 4;   // inner, column offset (+ 64 u)
  T va[UA][2][4], vb[UB][2][4];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const long oa = OPA == 0 ? (long)(r0 + ar_ + 64 * u) * A.ld + k0 + akq
                               : (long)(k0 + ak) * A.ld + r0 + arq + 64 * u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        va[u][0][q] = A.re[oa + q];
        va[u][1][q] = A.im[oa + q];
      }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const long ob = (long)(k0 + bk) * B.ld + c0 + bcq + 64 * u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        vb[u][0][q] = B.re[ob + q];
        vb[u][1][q] = B.im[ob + q];
      }
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += T64_BK) {
#pragma unroll
    for (int u = 0; u < UA; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (OPA == 0) {
          Asr[(akq + q) * LDA + ar_ + 64 * u] = va[u][0][q];
          Asi[(akq + q) * LDA + ar_ + 64 * u] = va[u][1][q];
        } else {
          Asr[ak * LDA + arq + 64 * u + q] = va[u][0][q];
          Asi[ak * LDA + arq + 64 * u + q] = -va[u][1][q];
        }
      }
#pragma unroll
    for (int u = 0; u < UB; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Bsr[bk * LDB + bcq + 64 * u + q] = vb[u][0][q];
        Bsi[bk * LDB + bcq + 64 * u + q] = vb[u][1][q];
      }
    lds_barrier();
    if (k0 + T64_BK < K) load(k0 + T64_BK);  // uniform
#pragma unroll
    for (int k4 = 0; k4 < T64_BK; k4 += 4) {
      T br[NT], bi[NT];
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        br[n] = Bsr[(k4 + kk) * LDB + wc + 16 * n + i];
        bi[n] = Bsi[(k4 + kk) * LDB + wc + 16 * n + i];
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const T ar = Asr[(k4 + kk) * LDA + wr + 16 * m + i];
        const T ai = Asi[(k4 + kk) * LDA + wr + 16 * m + i];
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          acc[m][n][0] = mfma4(ar, br[n], acc[m][n][0]);
          acc[m][n][0] = mfma4(-ai, bi[n], acc[m][n][0]);
          acc[m][n][1] = mfma4(ar, bi[n], acc[m][n][1]);
          acc[m][n][1] = mfma4(ai, br[n], acc[m][n][1]);
        }
      }
    }
    lds_barrier();  // the chunk's LDS reads are done; the prefetch stays in flight
  }
}

// Blocks of a 1-D launch are dispatched round-robin over the 8 XCDs of an
// MI355X.  Re-map the block index so that consecutive logical blocks (the
// tiles of one matrix, which share operand panels) land on the same XCD
// and hence the same L2.  `padded` is the launch size, a multiple of 8.
__device__ __forceinline__ long xcd_logical_block(long b, long padded) {
  const long per = padded >> 3;
  return (b & 7) * per + (b >> 3);
}

// Launch size for n workgroups whose groups of `group` consecutive logical
// indices (e.g. the states of one time block, which read the same step
// matrices) must share an XCD under xcd_logical_block: n rounded up to a
// multiple of 8 group, the extra workgroups returning at once.
inline unsigned xcd_grid(long n, int group) {
  const long m = 8L * group;
  return (unsigned)((n + m - 1) / m * m);
}


// Wave-wide sum (64 lanes) with cross-lane shuffles.
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
}

// Block-wide FP64 sum (blockDim.x a multiple of 64, at most 256 threads);
// `red` holds one double per wavefront.
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

}  // namespace qoc
