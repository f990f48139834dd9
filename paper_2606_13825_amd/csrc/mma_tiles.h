// Matrix-core tile helpers shared by the PSD kernels (16 x 16 x 4 products,
// FP32 or FP64) and small workgroup utilities.  Internal linkage: every
// translation unit that includes this gets its own copy.
#pragma once

#include "cosmo_internal.h"

namespace cosmo {
namespace {

// 16 x 16 x 4 matrix-core products.  Both take A(i, k) from lane i + 16 k and
// B(k, j) from lane j + 16 k; they differ in where result row i of column j
// lands: f32 puts rows 4 (l/16) .. 4 (l/16) + 3 in the four accumulator
// registers of lane l, f64 interleaves them (register e of lane l holds row
// l/16 + 4 e).
template <typename T> struct Mma;
template <> struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};
template <> struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};

constexpr double RSQRT2 = 0.70710678118654752440;
constexpr double SQRT2 = 1.41421356237309504880;

// 16 x 16 tile of C = A B with A(i, k), B(k, j) given by functors that return
// 0 outside the matrices.  Lane l feeds A(I0 + l%16, k0 + l/16) and
// B(k0 + l/16, J0 + l%16); accumulator element e of lane l is
// C(I0 + Mma<T>::row(l, e), J0 + l%16).
// The k loop is unrolled by four products so the operand reads of a group
// are issued together.
template <typename T, typename FA, typename FB>
__device__ inline typename Mma<T>::v4 tile_mma(int I0, int J0, int kdim, FA fa, FB fb) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kk = lane >> 4;
  typename Mma<T>::v4 acc = {0, 0, 0, 0};
  int k0 = 0;
  for (; k0 + 16 <= kdim; k0 += 16) {
    T a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = fa(I0 + r, k0 + 4 * u + kk);
      b[u] = fb(k0 + 4 * u + kk, J0 + r);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = Mma<T>::op(a[u], b[u], acc);
  }
  for (; k0 < kdim; k0 += 4) {
    const int k = k0 + kk;
    acc = Mma<T>::op(fa(I0 + r, k), fb(k, J0 + r), acc);
  }
  return acc;
}

// Upper-triangle tile enumeration: t -> (I, J), I <= J.
__device__ inline void upper_tile(int t, int &I, int &J) {
  J = 0;
  while ((J + 1) * (J + 2) / 2 <= t) ++J;
  I = t - J * (J + 1) / 2;
}

__device__ inline int svec_col(int idx) {
  int j = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
  while (j * (j + 1) / 2 > idx) --j;
  while ((j + 1) * (j + 2) / 2 <= idx) ++j;
  return j;
}

template <typename T, int NT> __device__ inline T wg_sum(T v, T *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = 0;
  for (int w = 0; w < NT / 64; ++w) t += red[w];
  return t;
}

}  // namespace
}  // namespace cosmo
