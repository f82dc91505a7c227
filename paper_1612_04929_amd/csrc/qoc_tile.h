// Operand-generic 64x64 complex tile products for the batched kernels
// (Taylor / squaring stages, the per-step derivative), in the chain
// precision (FP32 or FP64 MFMA) or as bf16x3 split products.
//
// A tile is C[i0:i0+64, j0:j0+64] += op(A)[i0:, 0:K] op(B)[0:K, j0:] where
// an operand is described by a TOp: element (i, kk) of op(X), with i the
// outer index (rows of op(A) / columns of op(B)) and kk the inner one.
//   KC = true : memory is row-major over (i, col(kk)), element at
//               i * ld + col(kk) (the inner index runs along a row)
//   KC = false: element at col(kk) * ld + i
//   CJ = true : complex conjugate
// col(kk) maps the inner index to a memory column in blocks of rr,
// col(kk) = (bmul * (kk / rr) + boff) * rr + kk % rr, so that a product can
// run over non-adjacent column blocks of a stored panel.  Outer indices at
// or beyond `rows` read as zero.
//
// Requirements (checked by the callers): ld, rr and K multiples of 16,
// rows a multiple of 16, base pointers 16-byte aligned.
#pragma once
#include "qoc_device.h"

namespace qoc {

template <typename T> struct TOp {
  const T *re, *im;
  int ld, rows;
  int rr, bmul, boff;
  __device__ __forceinline__ int col(int kk) const {
    const int b = kk / rr;
    return (bmul * b + boff) * rr + (kk - b * rr);
  }
};

template <typename T>
__host__ __device__ inline TOp<T> make_top(const T *re, long plane, int ld, int rows) {
  TOp<T> o;
  o.re = re;
  o.im = re + plane;
  o.ld = ld;
  o.rows = rows;
  o.rr = 1 << 30;
  o.bmul = 1;
  o.boff = 0;
  return o;
}

__device__ __forceinline__ void ld4(const float *p, float (&v)[4]) {
  const float4 x = *(const float4 *)p;
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ __forceinline__ void ld4(const double *p, double (&v)[4]) {
  const double2 x = *(const double2 *)p, y = *(const double2 *)(p + 2);
  v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
}

// ---------------------------------------------------------------- FP32 / FP64
// LDS: A and B chunks of 16 inner indices, k-major with row stride T64_LD
// (the layout of wg_cgemm64), T64_LDS_ELEMS elements.

// The chunk load split in two halves: global loads into registers, then the
// LDS stores, so the next chunk can be in flight while one is multiplied.
template <typename T, bool KC>
__device__ __forceinline__ void load_op16(const TOp<T> &X, int i0, int k0, T (&vr)[4], T (&vi)[4],
                                          bool &ok) {
  const int t = threadIdx.x;
  if (KC) {
    const int i = t >> 2, kq = (t & 3) * 4;
    ok = i0 + i < X.rows;
    const long o = ok ? (long)(i0 + i) * X.ld + X.col(k0 + kq) : 0;
    ld4(X.re + o, vr);
    ld4(X.im + o, vi);
  } else {
    const int k = t >> 4, iq = (t & 15) * 4;
    ok = i0 + iq < X.rows;
    const long o = ok ? (long)X.col(k0 + k) * X.ld + i0 + iq : 0;
    ld4(X.re + o, vr);
    ld4(X.im + o, vi);
  }
}
template <typename T, bool KC, bool CJ>
__device__ __forceinline__ void store_op16(const T (&vr)[4], const T (&vi)[4], bool ok, T *Sr,
                                           T *Si) {
  const int t = threadIdx.x;
  if (KC) {
    const int i = t >> 2, kq = (t & 3) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Sr[(kq + q) * T64_LD + i] = ok ? vr[q] : (T)0;
      Si[(kq + q) * T64_LD + i] = ok ? (CJ ? -vi[q] : vi[q]) : (T)0;
    }
  } else {
    const int k = t >> 4, iq = (t & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Sr[k * T64_LD + iq + q] = ok ? vr[q] : (T)0;
      Si[k * T64_LD + iq + q] = ok ? (CJ ? -vi[q] : vi[q]) : (T)0;
    }
  }
}

template <typename T, bool KC, bool CJ>
__device__ __forceinline__ void stage_op16(const TOp<T> &X, int i0, int k0, T *Sr, T *Si) {
  const int t = threadIdx.x;
  T vr[4], vi[4];
  if (KC) {
    const int i = t >> 2, kq = (t & 3) * 4;
    const bool ok = i0 + i < X.rows;
    const long o = ok ? (long)(i0 + i) * X.ld + X.col(k0 + kq) : 0;
    ld4(X.re + o, vr);
    ld4(X.im + o, vi);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Sr[(kq + q) * T64_LD + i] = ok ? vr[q] : (T)0;
      Si[(kq + q) * T64_LD + i] = ok ? (CJ ? -vi[q] : vi[q]) : (T)0;
    }
  } else {
    const int k = t >> 4, iq = (t & 15) * 4;
    const bool ok = i0 + iq < X.rows;
    const long o = ok ? (long)X.col(k0 + k) * X.ld + i0 + iq : 0;
    ld4(X.re + o, vr);
    ld4(X.im + o, vi);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Sr[k * T64_LD + iq + q] = ok ? vr[q] : (T)0;
      Si[k * T64_LD + iq + q] = ok ? (CJ ? -vi[q] : vi[q]) : (T)0;
    }
  }
}

// acc[m][n][0/1] (re / im) of the 32x32 sub-tile (32 (w >> 1), 32 (w & 1))
// of wave w, as 2 x 2 MFMA tiles.  All 256 threads must call.
template <typename T, bool AKC, bool ACJ, bool BKC, bool BCJ>
__device__ __forceinline__ void ctile64(const TOp<T> &A, const TOp<T> &B, int i0, int j0, int K,
                                        T *lds, v4<T> (&acc)[2][2][2]) {
  T *Asr = lds;
  T *Asi = Asr + T64_BK * T64_LD;
  T *Bsr = Asi + T64_BK * T64_LD;
  T *Bsi = Bsr + T64_BK * T64_LD;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  // register prefetch: chunk k0 + 16 is loaded while chunk k0 is multiplied
  T avr[4], avi[4], bvr[4], bvi[4];
  bool aok, bok;
  load_op16<T, AKC>(A, i0, 0, avr, avi, aok);
  load_op16<T, BKC>(B, j0, 0, bvr, bvi, bok);
  for (int k0 = 0; k0 < K; k0 += T64_BK) {
    store_op16<T, AKC, ACJ>(avr, avi, aok, Asr, Asi);
    store_op16<T, BKC, BCJ>(bvr, bvi, bok, Bsr, Bsi);
    __syncthreads();
    if (k0 + T64_BK < K) {  // uniform
      load_op16<T, AKC>(A, i0, k0 + T64_BK, avr, avi, aok);
      load_op16<T, BKC>(B, j0, k0 + T64_BK, bvr, bvi, bok);
    }
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
    lds_barrier();  // the chunk's LDS reads are done; the prefetch stays in flight
  }
}

// ---------------------------------------------------------------- bf16x3
// Each FP32 operand x is split on its way into LDS as hi = RNE_bf16(x),
// lo = RNE_bf16(x - hi) (x - hi is exact in FP32), and every real product
// is hi*hi + hi*lo + lo*hi on the bf16 16x16x32 MFMA with FP32
// accumulation; the dropped lo*lo term and the two roundings leave a
// relative error of a few 2^-18 per product.  The inner dimension runs in
// chunks of 32 (one MFMA K; a ragged last chunk of 16 is zero-filled).
// LDS holds each operand chunk as [plane][outer][k] (k contiguous, 64-byte
// rows of four 16-byte groups, the group index XOR-ed with bits 1-2 of the
// row), planes re_hi, re_lo, im_hi, im_lo, so each lane's MFMA operand is
// one 16-byte LDS read.  The next chunk's FP32 values are
// loaded into registers while the current chunk is multiplied (or, for the
// stage products, just before its stores, at one more wavefront per SIMD).

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BF_BK = 32;
constexpr int BF_LDK = BF_BK;

// Position (in halves) of 16-byte group q of row r.  Against a padded row
// stride of 40 halves, the swizzle keeps all three access patterns of the
// tile free of LDS bank conflicts (by the hardware's conflict counters): the
// fragment reads (16 consecutive rows, one group), the row-contiguous
// stores (four lanes per row) and the across-row stores (one group of 64
// consecutive rows); the padded stride has two-way conflicts on the first
// two.  It also takes a quarter less LDS.
__device__ __forceinline__ int bf_grp(int r, int q) { return 8 * (q ^ ((r >> 1) & 3)); }

__device__ __forceinline__ f32x4 mfma_bf(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// Pairs of values through the packed FP32 -> bf16 conversion (RNE).
__device__ __forceinline__ void bf_split8(const float (&x)[8], bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
  for (int q = 0; q < 8; q += 2) {
    const f32x2v v = {x[q], x[q + 1]};
    const bf16x2v h = __builtin_convertvector(v, bf16x2v);
    const f32x2v hf = __builtin_convertvector(h, f32x2v);
    const f32x2v r = {v[0] - hf[0], v[1] - hf[1]};
    const bf16x2v l = __builtin_convertvector(r, bf16x2v);
    hi[q] = h[0];
    hi[q + 1] = h[1];
    lo[q] = l[0];
    lo[q + 1] = l[1];
  }
}

// LDS of one TM x 32 chunk of op(A) and 32 x TN chunk of op(B), both as
// [plane][outer][k].
template <int TM, int TN> struct alignas(16) BfLdsT {
  __bf16 a[4][TM][BF_LDK];
  __bf16 b[4][TN][BF_LDK];
};
typedef BfLdsT<64, 64> BfLds;

// Slot s (0 <= s < 4 TM) of a TM x 32 chunk -> (outer index, group of 8
// inner indices).  Slots s and s + 256 belong to one thread.
// KC: four consecutive lanes cover one row's 32 inner indices (one 128-byte
// segment per plane); otherwise consecutive lanes take consecutive outer
// indices of one group.  (Lanes of one row group spread over 16 rows would
// avoid the two-way LDS bank conflict of the KC stores, but cost registers
// and measured slower.)
template <bool KC, int TM> __device__ __forceinline__ void bf_slot(int s, int &i, int &kq) {
  if (KC) {
    i = s >> 2;
    kq = s & 3;
  } else {
    i = s % TM;
    kq = s / TM;
  }
}

template <bool KC, bool CJ, int TM>
__device__ __forceinline__ void bf_load_op(const TOp<float> &X, int s, int i0, int k0, int K,
                                           float (&vr)[8], float (&vi)[8]) {
  int i, kq;
  bf_slot<KC, TM>(s, i, kq);
  const int kk = k0 + 8 * kq;
  const bool ok = (i0 + i < X.rows) && (kk < K);
  if (KC) {
    const long o = ok ? (long)(i0 + i) * X.ld + X.col(kk) : 0;
    const float4 *pr = (const float4 *)(X.re + o), *pi = (const float4 *)(X.im + o);
    const float4 r0 = pr[0], r1 = pr[1], q0 = pi[0], q1 = pi[1];
    vr[0] = r0.x; vr[1] = r0.y; vr[2] = r0.z; vr[3] = r0.w;
    vr[4] = r1.x; vr[5] = r1.y; vr[6] = r1.z; vr[7] = r1.w;
    vi[0] = q0.x; vi[1] = q0.y; vi[2] = q0.z; vi[3] = q0.w;
    vi[4] = q1.x; vi[5] = q1.y; vi[6] = q1.z; vi[7] = q1.w;
  } else {
    const int c = ok ? X.col(kk) : 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const long o = ok ? (long)(c + q) * X.ld + i0 + i : 0;
      vr[q] = X.re[o];
      vi[q] = X.im[o];
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    vr[q] = ok ? vr[q] : 0.0f;
    vi[q] = ok ? (CJ ? -vi[q] : vi[q]) : 0.0f;
  }
}

// The same chunk load for tiles that lie inside the operand (outer indices
// below rows, K a multiple of 32, no column blocks, both planes within 2^31
// bytes of re): no guards, and the per-lane part of each address is one
// 32-bit byte offset.  Inner index along memory rows: 16-byte global loads
// from the uniform plane pointers; across rows: dword buffer loads whose
// row and plane offsets are wave-uniform (scalar offsets), so no lane
// computes a 64-bit address.  The buffer's range covers both planes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t bf_rsrc(const TOp<float> &X) {
  const long bytes = ((long)(X.im - X.re) + (long)X.rows * X.ld) * 4;
  return __builtin_amdgcn_make_buffer_rsrc((void *)X.re, 0,
                                           (int)(bytes < 0x7fffffffL ? bytes : 0x7fffffffL),
                                           0x00020000);
}

template <bool KC, bool CJ, int TM>
__device__ __forceinline__ void bf_load_full(const TOp<float> &X, __amdgpu_buffer_rsrc_t rs,
                                             int s, int i0, int k0, float (&vr)[8],
                                             float (&vi)[8]) {
  int i, kq;
  bf_slot<KC, TM>(s, i, kq);
  if (KC) {
    const unsigned o = (unsigned)(((i0 + i) * X.ld + k0 + 8 * kq) * 4);
    const char *re = (const char *)X.re, *im = (const char *)X.im;
    const float4 r0 = *(const float4 *)(re + o), r1 = *(const float4 *)(re + o + 16);
    const float4 q0 = *(const float4 *)(im + o), q1 = *(const float4 *)(im + o + 16);
    vr[0] = r0.x; vr[1] = r0.y; vr[2] = r0.z; vr[3] = r0.w;
    vr[4] = r1.x; vr[5] = r1.y; vr[6] = r1.z; vr[7] = r1.w;
    vi[0] = q0.x; vi[1] = q0.y; vi[2] = q0.z; vi[3] = q0.w;
    vi[4] = q1.x; vi[5] = q1.y; vi[6] = q1.z; vi[7] = q1.w;
  } else {
    // kq = s / TM is the same on every lane of a wave (TM a multiple of 64)
    const int kw = __builtin_amdgcn_readfirstlane(kq);
    const int im = (int)(X.im - X.re) * 4;
    const int o = (i0 + i) * 4;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int row = (k0 + 8 * kw + q) * X.ld * 4;
      vr[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o, row, 0));
      vi[q] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, o, row + im, 0));
    }
  }
  if (CJ) {
#pragma unroll
    for (int q = 0; q < 8; ++q) vi[q] = -vi[q];
  }
}

template <bool KC, int TM>
__device__ __forceinline__ void bf_store_op(int s, const float (&vr)[8], const float (&vi)[8],
                                            __bf16 (&S)[4][TM][BF_LDK]) {
  int i, kq;
  bf_slot<KC, TM>(s, i, kq);
  bf16x8 h, l;
  const int g = bf_grp(i, kq);
  bf_split8(vr, h, l);
  *(bf16x8 *)&S[0][i][g] = h;
  *(bf16x8 *)&S[1][i][g] = l;
  bf_split8(vi, h, l);
  *(bf16x8 *)&S[2][i][g] = h;
  *(bf16x8 *)&S[3][i][g] = l;
}

// acc[m][n][0/1] (re / im) += the (16 MT) x (16 NT) sub-tile of wave w at
// rows 16 MT (w >> 1), columns 16 NT (w & 1) of the (32 MT) x (32 NT) tile
// at (i0, j0).  All 256 threads must call.  Every accumulator receives its
// terms in the same order whatever MT and NT, so tiles of any shape give
// the same sums.
template <int MT, int NT, bool AKC, bool ACJ, bool BKC, bool BCJ, bool FULL = false,
          bool PF = true>
__device__ __forceinline__ void ctile_bf3(const TOp<float> &A, const TOp<float> &B, int i0,
                                          int j0, int K, BfLdsT<32 * MT, 32 * NT> &L,
                                          f32x4 (&acc)[MT][NT][2]) {
  constexpr int TM = 32 * MT, TN = 32 * NT, UA = TM / 64, UB = TN / 64;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int wr = (w >> 1) * 16 * MT, wc = (w & 1) * 16 * NT;
  float ar[UA][8], ai[UA][8], br[UB][8], bi[UB][8];
  __amdgpu_buffer_rsrc_t rsa, rsb;
  if constexpr (FULL) {
    rsa = bf_rsrc(A);
    rsb = bf_rsrc(B);
  }
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      if constexpr (FULL)
        bf_load_full<AKC, ACJ, TM>(A, rsa, t + 256 * u, i0, k0, ar[u], ai[u]);
      else
        bf_load_op<AKC, ACJ, TM>(A, t + 256 * u, i0, k0, K, ar[u], ai[u]);
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      if constexpr (FULL)
        bf_load_full<BKC, BCJ, TN>(B, rsb, t + 256 * u, j0, k0, br[u], bi[u]);
      else
        bf_load_op<BKC, BCJ, TN>(B, t + 256 * u, j0, k0, K, br[u], bi[u]);
    }
  };
  // Ai Bi accumulates on its own (added with a minus sign at the end), so
  // no fragment needs a negation
  f32x4 accn[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) accn[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  // PF: the next chunk is loaded into registers while the current one is
  // multiplied; without it each chunk is loaded just before its stores
  // (fewer registers: one more wavefront per SIMD hides the latency)
  if (PF) load(0);
  for (int k0 = 0; k0 < K; k0 += BF_BK) {
    if (!PF) load(k0);
#pragma unroll
    for (int u = 0; u < UA; ++u) bf_store_op<AKC, TM>(t + 256 * u, ar[u], ai[u], L.a);
#pragma unroll
    for (int u = 0; u < UB; ++u) bf_store_op<BKC, TN>(t + 256 * u, br[u], bi[u], L.b);
    __syncthreads();
    if (PF && k0 + BF_BK < K) load(k0 + BF_BK);  // block-uniform
    bf16x8 fb[NT][4];
#pragma unroll
    for (int n = 0; n < NT; ++n)
#pragma unroll
      for (int p = 0; p < 4; ++p)
        fb[n][p] = *(const bf16x8 *)&L.b[p][wc + 16 * n + i][bf_grp(wc + 16 * n + i, q)];
    // Re += Ar Br - Ai Bi ; Im += Ar Bi + Ai Br, each real product as
    // hi*hi + hi*lo + lo*hi; consecutive MFMAs go to different accumulators.
    // MT <= 2: every fragment of op(A) up front, term by term over all
    // tiles; above, one row block of fragments at a time (register budget).
    constexpr int FA = MT <= 2 ? MT : 1;
#define QOC_BF3_TERMS(MLO, MHI, FA_)                                           \
  QOC_BF3_TERM(MLO, MHI, acc[m][n][0], FA_[0], fb[n][0])                       \
  QOC_BF3_TERM(MLO, MHI, acc[m][n][1], FA_[0], fb[n][2])                       \
  QOC_BF3_TERM(MLO, MHI, accn[m][n], FA_[2], fb[n][2])                         \
  QOC_BF3_TERM(MLO, MHI, acc[m][n][0], FA_[0], fb[n][1])                       \
  QOC_BF3_TERM(MLO, MHI, acc[m][n][1], FA_[0], fb[n][3])                       \
  QOC_BF3_TERM(MLO, MHI, accn[m][n], FA_[2], fb[n][3])                         \
  QOC_BF3_TERM(MLO, MHI, acc[m][n][0], FA_[1], fb[n][0])                       \
  QOC_BF3_TERM(MLO, MHI, acc[m][n][1], FA_[1], fb[n][2])                       \
  QOC_BF3_TERM(MLO, MHI, accn[m][n], FA_[3], fb[n][2])                         \
  QOC_BF3_TERM(MLO, MHI, acc[m][n][1], FA_[2], fb[n][0])                       \
  QOC_BF3_TERM(MLO, MHI, acc[m][n][1], FA_[2], fb[n][1])                       \
  QOC_BF3_TERM(MLO, MHI, acc[m][n][1], FA_[3], fb[n][0])
#define QOC_BF3_TERM(MLO, MHI, D, X, Y)                                        \
  _Pragma("unroll") for (int m = MLO; m < MHI; ++m)                            \
  _Pragma("unroll") for (int n = 0; n < NT; ++n) D = mfma_bf(X, Y, D);
    if constexpr (MT <= 2) {
      bf16x8 fa[FA][4];
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int p = 0; p < 4; ++p)
          fa[m][p] = *(const bf16x8 *)&L.a[p][wr + 16 * m + i][bf_grp(wr + 16 * m + i, q)];
      QOC_BF3_TERMS(0, MT, fa[m])
    } else {
#pragma unroll
      for (int mb = 0; mb < MT; ++mb) {
        bf16x8 fa[4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
          fa[p] = *(const bf16x8 *)&L.a[p][wr + 16 * mb + i][bf_grp(wr + 16 * mb + i, q)];
        QOC_BF3_TERMS(mb, mb + 1, fa)
      }
    }
#undef QOC_BF3_TERM
#undef QOC_BF3_TERMS
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[m][n][0] -= accn[m][n];
}

template <bool AKC, bool ACJ, bool BKC, bool BCJ>
__device__ __forceinline__ void ctile64_bf3(const TOp<float> &A, const TOp<float> &B, int i0,
                                            int j0, int K, BfLds &L, f32x4 (&acc)[2][2][2]) {
  ctile_bf3<2, 2, AKC, ACJ, BKC, BCJ>(A, B, i0, j0, K, L, acc);
}

// Dispatch: one 64x64 tile in the chain precision or as bf16x3 (float only).
// lds must hold max(T64_LDS_ELEMS * sizeof(T), sizeof(BfLds)) bytes.
template <typename T, bool BF3, bool AKC, bool ACJ, bool BKC, bool BCJ>
__device__ __forceinline__ void tile64(const TOp<T> &A, const TOp<T> &B, int i0, int j0, int K,
                                       void *lds, v4<T> (&acc)[2][2][2]) {
  if constexpr (BF3 && sizeof(T) == 4)
    ctile64_bf3<AKC, ACJ, BKC, BCJ>(A, B, i0, j0, K, *(BfLds *)lds, acc);
  else
    ctile64<T, AKC, ACJ, BKC, BCJ>(A, B, i0, j0, K, (T *)lds, acc);
}

constexpr int TILE64_LDS_BYTES =
    (int)sizeof(BfLds) > T64_LDS_ELEMS * 8 ? (int)sizeof(BfLds) : T64_LDS_ELEMS * 8;

// Row / column of element v of accumulator [m][n] of this lane in a 64x64 tile.
template <typename T>
__device__ __forceinline__ void tile64_pos(int m, int n, int v, int &r, int &c) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  r = (w >> 1) * 32 + 16 * m + acc_row<T>(lane, v);
  c = (w & 1) * 32 + 16 * n + (lane & 15);
}

}  // namespace qoc
