// Cross-lane helpers for 64-lane waves shared by the CG and dense-block
// kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace cosmo {

// The value of v held by lane l, in every lane (no LDS round trip).
template <typename AT> __device__ inline AT read_lane(AT v, int l) {
  if constexpr (sizeof(AT) == 8) {
    const long long b = __double_as_longlong((double)v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return (AT)__longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  } else {
    return (AT)__int_as_float(__builtin_amdgcn_readlane(__float_as_int((float)v), l));
  }
}

// Wave sums of U = 2^k values per lane with 6 + U - 2 shuffles instead of 6 U:
// each of the first k butterfly steps halves the values a lane holds (the
// lanes with the step's bit set keep the upper half, the others the lower),
// the remaining steps sum one value; row u's total then sits in lane
// u << (6 - k), from where it is read into every lane.
template <int U, typename AT> __device__ inline void wave_sums(AT (&v)[U]) {
  static_assert(U == 1 || U == 2 || U == 4 || U == 8, "U must be a power of two <= 8");
  constexpr int K = U == 1 ? 0 : (U == 2 ? 1 : (U == 4 ? 2 : 3));
  const int lane = threadIdx.x % 64;
  AT w[U];
#pragma unroll
  for (int i = 0; i < U; ++i) w[i] = v[i];
#pragma unroll
  for (int s = 0, cnt = U; s < K; ++s) {
    const int off = 32 >> s, half = cnt / 2;
    const bool up = (lane & off) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const AT send = up ? w[i] : w[i + half];
      const AT keep = up ? w[i + half] : w[i];
      w[i] = keep + __shfl_xor(send, off, 64);
    }
    cnt = half;
  }
#pragma unroll
  for (int off = 32 >> K; off > 0; off >>= 1) w[0] += __shfl_xor(w[0], off, 64);
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = read_lane(w[0], u << (6 - K));
}

}  // namespace cosmo
