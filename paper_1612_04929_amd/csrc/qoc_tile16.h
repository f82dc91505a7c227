// 16x16 complex tiles on the FP32 / FP64 16x16x4 MFMA for padded d = 16,
// shared by the per-step exponential chain and the per-step derivative.
//
// Operand order.  Within one 16x16x4 MFMA the lanes of group g = l / 16
// supply inner index g; across the four MFMAs t of a 16-deep product the
// pair (t, g) stands for the inner index K(t, g) = acc_row(16 g, t)
// (4 g + t for FP32, 4 t + g for FP64).  With that order a result tile,
// whose lane l holds rows acc_row(l, v) of column l % 16, is already the
// right-hand operand of the next product (MFMA t takes register t), so a
// chain X Q, X (X Q), ... needs no data movement; a result used as a
// left operand (or conjugate-transposed) goes through an LDS tile.
#pragma once

#include "qoc_device.h"

namespace qoc {

constexpr int A16_LD = 20;    // LDS row stride of a staged tile (16-byte rows)

template <typename T> struct CTile {  // 16x16 complex tile, MFMA result layout
  v4<T> r, i;
};

template <typename T> __device__ __forceinline__ CTile<T> ctile_zero() {
  CTile<T> z;
  z.r = vzero<T>();
  z.i = vzero<T>();
  return z;
}

__device__ __forceinline__ void wave_lds_sync() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// operand fragments: entry t of lane l is the element at inner index
// K(t, l / 16) = acc_row(l, t)
template <typename T> struct Frag {
  T r[4], i[4];
};

template <typename T>
__device__ __forceinline__ void stage(T *tr, T *ti, const CTile<T> &c) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int o = acc_row<T>(lane, v) * A16_LD + (lane & 15);
    tr[o] = c.r[v];
    ti[o] = c.i[v];
  }
}
// left operand M (rows q = l % 16) from a staged tile
template <typename T> __device__ __forceinline__ Frag<T> fragA(const T *tr, const T *ti) {
  const int lane = threadIdx.x & 63, q = lane & 15;
  Frag<T> f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f.r[t] = tr[q * A16_LD + acc_row<T>(lane, t)];
    f.i[t] = ti[q * A16_LD + acc_row<T>(lane, t)];
  }
  return f;
}
// right operand M^H (element [k][q] = conj(M[q][k])) from a staged tile
template <typename T> __device__ __forceinline__ Frag<T> fragBH(const T *tr, const T *ti) {
  const int lane = threadIdx.x & 63, q = lane & 15;
  Frag<T> f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f.r[t] = tr[q * A16_LD + acc_row<T>(lane, t)];
    f.i[t] = -ti[q * A16_LD + acc_row<T>(lane, t)];
  }
  return f;
}
// right operand from a result tile: no data movement
template <typename T> __device__ __forceinline__ Frag<T> asB(const CTile<T> &c) {
  Frag<T> f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f.r[t] = c.r[t];
    f.i[t] = c.i[t];
  }
  return f;
}
// left operand of a global 16x16 matrix (OPH = conjugate transpose)
template <typename T, bool OPH>
__device__ __forceinline__ Frag<T> fragA_global(const T *__restrict__ g) {
  const int lane = threadIdx.x & 63, q = lane & 15;
  Frag<T> f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = acc_row<T>(lane, t);
    if (!OPH) {
      f.r[t] = g[q * 16 + k];
      f.i[t] = g[256 + q * 16 + k];
    } else {
      f.r[t] = g[k * 16 + q];
      f.i[t] = -g[256 + k * 16 + q];
    }
  }
  return f;
}

template <typename T>
__device__ __forceinline__ void cmma(const Frag<T> &a, const Frag<T> &b, CTile<T> &c) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    c.r = mfma4(a.r[t], b.r[t], c.r);
    c.r = mfma4(-a.i[t], b.i[t], c.r);
    c.i = mfma4(a.r[t], b.i[t], c.i);
    c.i = mfma4(a.i[t], b.r[t], c.i);
  }
}

template <typename T>
__device__ __forceinline__ CTile<T> axpy(T alpha, const CTile<T> &x, const CTile<T> &y) {
  CTile<T> o;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    o.r[v] = alpha * x.r[v] + y.r[v];
    o.i[v] = alpha * x.i[v] + y.i[v];
  }
  return o;
}

}  // namespace qoc
