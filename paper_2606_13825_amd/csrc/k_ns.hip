// Newton-Schulz comparison rule of the PSD projection (eq:newton-schulz):
// (S + sign(S) S) / 2 with sign(S) from K steps of the scaled iteration,
// forward and reverse pass through the unrolled products, over a set of
// svec blocks; every iterate and its square are kept in a caller tape.
#include "cosmo_internal.h"
#include "mma_tiles.h"

namespace cosmo {
namespace {

constexpr int NXCD = 8;   // accelerator complex dies of the MI355X, one L2 each

// Matrices live in a caller tape, column-major p x p per block, addressed by
// slot: base + d.moff + slot p^2.

// 32 x 32 block of C = A B per wave as 2 x 2 matrix-core tiles that share
// their operand reads: per k step a lane loads two A and two B values and
// issues four products (the 16 x 16 tile_mma issues one per two loads).
// acc[2 a + b] is the tile at rows I0 + 16 a, columns J0 + 16 b, laid out as
// in tile_mma.
template <typename T, typename FA, typename FB>
__device__ inline void tile_mma22(int I0, int J0, int kdim, FA fa, FB fb, typename Mma<T>::v4 acc[4]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = typename Mma<T>::v4{0, 0, 0, 0};
  int k0 = 0;
  for (; k0 + 8 <= kdim; k0 += 8) {
    T a[2][2], b[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int k = k0 + 4 * u + kk;
      a[u][0] = fa(I0 + r, k);
      a[u][1] = fa(I0 + 16 + r, k);
      b[u][0] = fb(k, J0 + r);
      b[u][1] = fb(k, J0 + 16 + r);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = Mma<T>::op(a[u][t >> 1], b[u][t & 1], acc[t]);
  }
  for (; k0 < kdim; k0 += 4) {
    const int k = k0 + kk;
    const T a0 = fa(I0 + r, k), a1 = fa(I0 + 16 + r, k), b0 = fb(k, J0 + r), b1 = fb(k, J0 + 16 + r);
    acc[0] = Mma<T>::op(a0, b0, acc[0]);
    acc[1] = Mma<T>::op(a0, b1, acc[1]);
    acc[2] = Mma<T>::op(a1, b0, acc[2]);
    acc[3] = Mma<T>::op(a1, b1, acc[3]);
  }
}

// C = alpha op(A) op(B) + beta D over every block; one workgroup of four
// waves per TILE x TILE tile of C.  TILE = 64: the workgroup stages 64 x 32
// panels of op(A) and op(B) in LDS (each read from the tape along its
// contiguous direction, transposed operands included) and each wave
// computes a 32 x 32 block from them (tile_mma22); TILE = 32, used when the
// larger tiles would leave the chip short of workgroups: each wave one
// 16 x 16 tile read straight from the tape (tile_mma).
// op(X) = X' when the flag is set.  D may be C itself (each element is read
// and written by the lane that owns it); A and B are never C.
template <typename T, int TILE>
__global__ __launch_bounds__(256) void k_ns_gemm(const NsDesc *__restrict__ descs, int32_t nblk, T *base,
                                                 NsGemm g) {
  constexpr int W = TILE / 2;                // edge of one wave's block
  constexpr int KC = 32;                     // k extent of one staged panel
  // panel row stride: the four k rows one operand read touches (16 lanes
  // each) start 16 banks apart
  constexpr int LDP = TILE + 16;
  __shared__ T As[TILE == 64 ? KC * LDP : 1], Bs[TILE == 64 ? KC * LDP : 1];
  // Workgroups are dealt to the 8 XCDs round-robin (workgroup b to XCD
  // b mod 8), each XCD with its own L2: give XCD x a contiguous range of
  // tiles, so the tiles of one matrix, which read the same operand panels,
  // share an L2.  With N tiles, XCD x holds N/8 (+1 for x < N mod 8) of them.
  const int nwg = gridDim.x, x = blockIdx.x % NXCD, k = blockIdx.x / NXCD;
  const int q = nwg / NXCD, rem = nwg % NXCD;
  const int t = x * q + (x < rem ? x : rem) + k;
  int lo = 0, hi = nblk - 1;                 // last block with tile0 <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile0 <= t) lo = mid;
    else hi = mid - 1;
  }
  const NsDesc d = descs[lo];
  const int p = d.p, nt = (p + TILE - 1) / TILE, lt = t - d.tile0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int TI = (lt / nt) * TILE, TJ = (lt % nt) * TILE;
  const int I0 = TI + (wave >> 1) * W, J0 = TJ + (wave & 1) * W;
  const size_t pp = (size_t)p * p;
  T *blk = base + d.moff;
  const T *A = blk + g.a * pp, *B = blk + g.b * pp;
  T *C = blk + g.c * pp;
  const T *D = g.d >= 0 ? blk + g.d * pp : nullptr;
  const bool ta = g.ta, tb = g.tb;
  constexpr int NQ = TILE == 64 ? 4 : 1;
  typename Mma<T>::v4 acc[NQ];
  if constexpr (TILE == 64) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = typename Mma<T>::v4{0, 0, 0, 0};
    // panel element (k, x) holds op(A)(TI + x, k0 + k) in As and
    // op(B)(k0 + k, TJ + x) in Bs, zero outside the matrices
    for (int k0 = 0; k0 < p; k0 += KC) {
      for (int e = threadIdx.x; e < KC * TILE; e += 256) {
        // A' / B: consecutive threads walk k (contiguous in the tape);
        // A / B': consecutive threads walk the tile index
        const int ka = ta ? e % KC : e / TILE, xa = ta ? e / KC : e % TILE;
        const int ia = TI + xa, kga = k0 + ka;
        As[ka * LDP + xa] = (ia < p && kga < p) ? (ta ? A[kga + (size_t)ia * p] : A[ia + (size_t)kga * p]) : (T)0;
        const int kb = tb ? e / TILE : e % KC, xb = tb ? e % TILE : e / KC;
        const int jb = TJ + xb, kgb = k0 + kb;
        Bs[kb * LDP + xb] = (jb < p && kgb < p) ? (tb ? B[jb + (size_t)kgb * p] : B[kgb + (size_t)jb * p]) : (T)0;
      }
      __syncthreads();
      auto fa = [&](int i, int k) -> T { return As[k * LDP + (i - TI)]; };
      auto fb = [&](int k, int j) -> T { return Bs[k * LDP + (j - TJ)]; };
      typename Mma<T>::v4 part[4];
      tile_mma22<T>(I0, J0, KC, fa, fb, part);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += part[q];
      __syncthreads();
    }
    if (I0 >= p || J0 >= p) return;
  } else {
    if (I0 >= p || J0 >= p) return;
    auto fa = [&](int i, int k) -> T { return (i < p && k < p) ? (ta ? A[k + (size_t)i * p] : A[i + (size_t)k * p]) : (T)0; };
    auto fb = [&](int k, int j) -> T { return (k < p && j < p) ? (tb ? B[j + (size_t)k * p] : B[k + (size_t)j * p]) : (T)0; };
    acc[0] = tile_mma<T>(I0, J0, p, fa, fb);
  }
  const T alpha = (T)g.alpha, beta = (T)g.beta;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int col = J0 + 16 * (q & 1) + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I0 + 16 * (q >> 1) + Mma<T>::row(lane, e);
      if (row < p && col < p) {
        const size_t o = row + (size_t)col * p;
        C[o] = D ? alpha * acc[q][e] + beta * D[o] : alpha * acc[q][e];
      }
    }
  }
}

// Forward set-up, one workgroup per block: c = ||smat(v)||_F = ||v||_2,
// slot S = smat(v), slot X_0 = S / c.
template <typename T>
__global__ __launch_bounds__(256) void k_ns_init(const NsDesc *__restrict__ descs, const T *__restrict__ v,
                                                 T *base, double *cnorm, int32_t slot_x0, int32_t slot_s) {
  __shared__ double red[256 / 64];
  const NsDesc d = descs[blockIdx.x];
  const int p = d.p, nrows = p * (p + 1) / 2;
  const T *vb = v + d.row0;
  double ss = 0.0;
  for (int idx = threadIdx.x; idx < nrows; idx += 256) {
    const double x = (double)vb[idx];
    ss += x * x;
  }
  const double c = sqrt(wg_sum<double, 256>(ss, red));
  if (threadIdx.x == 0) cnorm[blockIdx.x] = c;
  const size_t pp = (size_t)p * p;
  T *S = base + d.moff + slot_s * pp, *X = base + d.moff + slot_x0 * pp;
  const T inv = (T)(1.0 / c);
  for (int idx = threadIdx.x; idx < nrows; idx += 256) {
    const int j = svec_col(idx);
    const int i = idx - j * (j + 1) / 2;
    const T val = (i == j) ? vb[idx] : vb[idx] * (T)RSQRT2;
    S[i + (size_t)j * p] = val;
    S[j + (size_t)i * p] = val;
    X[i + (size_t)j * p] = val * inv;
    X[j + (size_t)i * p] = val * inv;
  }
}

// out = svec of the symmetric part of slot W.
template <typename T>
__global__ __launch_bounds__(256) void k_ns_pack(const NsDesc *__restrict__ descs, const T *base, int32_t slot_w,
                                                 T *__restrict__ out) {
  const NsDesc d = descs[blockIdx.x];
  const int p = d.p, nrows = p * (p + 1) / 2;
  const T *W = base + d.moff + slot_w * (size_t)p * p;
  for (int idx = threadIdx.x; idx < nrows; idx += 256) {
    const int j = svec_col(idx);
    const int i = idx - j * (j + 1) / 2;
    out[d.row0 + idx] = (i == j) ? W[i + (size_t)i * p]
                                 : (W[i + (size_t)j * p] + W[j + (size_t)i * p]) * (T)(0.5 * SQRT2);
  }
}

// slot TB = smat(g).
template <typename T>
__global__ __launch_bounds__(256) void k_ns_unpack(const NsDesc *__restrict__ descs, const T *__restrict__ g,
                                                   T *base, int32_t slot_t) {
  const NsDesc d = descs[blockIdx.x];
  const int p = d.p, nrows = p * (p + 1) / 2;
  T *Tb = base + d.moff + slot_t * (size_t)p * p;
  for (int idx = threadIdx.x; idx < nrows; idx += 256) {
    const int j = svec_col(idx);
    const int i = idx - j * (j + 1) / 2;
    const T val = (i == j) ? g[d.row0 + idx] : g[d.row0 + idx] * (T)RSQRT2;
    Tb[i + (size_t)j * p] = val;
    Tb[j + (size_t)i * p] = val;
  }
}

// Reverse of S_0 = S / c and of smat: Sbar += Y / c - <Y, S> S / c^3 with
// Y = cotangent of S_0, then gin = svec of the symmetric part of Sbar.
template <typename T>
__global__ __launch_bounds__(256) void k_ns_final(const NsDesc *__restrict__ descs, const T *base,
                                                  const double *cnorm, int32_t slot_y, int32_t slot_s,
                                                  int32_t slot_sb, T *__restrict__ gin) {
  __shared__ double red[256 / 64];
  const NsDesc d = descs[blockIdx.x];
  const int p = d.p, nrows = p * (p + 1) / 2;
  const size_t pp = (size_t)p * p;
  const T *Y = base + d.moff + slot_y * pp, *S = base + d.moff + slot_s * pp, *SB = base + d.moff + slot_sb * pp;
  double dot = 0.0;
  for (size_t e = threadIdx.x; e < pp; e += 256) dot += (double)Y[e] * (double)S[e];
  dot = wg_sum<double, 256>(dot, red);
  const double c = cnorm[blockIdx.x];
  const T ic = (T)(1.0 / c), k3 = (T)(dot / (c * c * c));
  for (int idx = threadIdx.x; idx < nrows; idx += 256) {
    const int j = svec_col(idx);
    const int i = idx - j * (j + 1) / 2;
    const size_t a = i + (size_t)j * p, b = j + (size_t)i * p;
    const T ga = SB[a] + Y[a] * ic - k3 * S[a];
    if (i == j) gin[d.row0 + idx] = ga;
    else gin[d.row0 + idx] = (ga + SB[b] + Y[b] * ic - k3 * S[b]) * (T)RSQRT2;
  }
}

template <typename T>
void ns_gemm(const NsDesc *d, int32_t nblk, int32_t ntiles, int32_t tile, T *base, const NsGemm &g, hipStream_t st) {
  if (tile == 64) k_ns_gemm<T, 64><<<ntiles, 256, 0, st>>>(d, nblk, base, g);
  else k_ns_gemm<T, 32><<<ntiles, 256, 0, st>>>(d, nblk, base, g);
}

}  // namespace

// Newton-Schulz forward: K steps of eq:newton-schulz, every iterate X_k and
// square Q_k kept in the tape for the reverse pass, then
// out = svec(sym((S + X_K S) / 2)).
template <typename T>
void launch_ns_forward(const NsDesc *d, int32_t nblk, int32_t ntiles, int32_t tile, int32_t K, const T *v, T *out,
                       T *base, double *cnorm, hipStream_t st) {
  const NsSlots sl(K);
  k_ns_init<T><<<nblk, 256, 0, st>>>(d, v, base, cnorm, sl.x(0), sl.S);
  for (int k = 0; k < K; ++k) {
    ns_gemm<T>(d, nblk, ntiles, tile, base, NsGemm{sl.x(k), sl.x(k), sl.q(k), -1, 0, 0, 1.0, 0.0}, st);
    ns_gemm<T>(d, nblk, ntiles, tile, base, NsGemm{sl.x(k), sl.q(k), sl.x(k + 1), sl.x(k), 0, 0, -0.5, 1.5}, st);
  }
  ns_gemm<T>(d, nblk, ntiles, tile, base, NsGemm{sl.x(K), sl.S, sl.W, sl.S, 0, 0, 0.5, 0.5}, st);
  k_ns_pack<T><<<nblk, 256, 0, st>>>(d, base, sl.W, out);
}

// Newton-Schulz reverse pass from the tape of launch_ns_forward (same blocks
// and K): for C = A B, Abar = Cbar B' and Bbar = A' Cbar.
template <typename T>
void launch_ns_vjp(const NsDesc *d, int32_t nblk, int32_t ntiles, int32_t tile, int32_t K, const T *g, T *gin,
                   T *base, const double *cnorm, hipStream_t st) {
  const NsSlots sl(K);
  k_ns_unpack<T><<<nblk, 256, 0, st>>>(d, g, base, sl.TB);
  // Pi = S / 2 + X_K S / 2
  ns_gemm<T>(d, nblk, ntiles, tile, base, NsGemm{sl.x(K), sl.TB, sl.SB, sl.TB, 1, 0, 0.5, 0.5}, st);
  ns_gemm<T>(d, nblk, ntiles, tile, base, NsGemm{sl.TB, sl.S, sl.Y, -1, 0, 1, 0.5, 0.0}, st);
  for (int k = K - 1; k >= 0; --k) {
    // X_{k+1} = 3/2 X_k - 1/2 X_k Q_k with Q_k = X_k X_k; Y = cotangent of X_{k+1}
    ns_gemm<T>(d, nblk, ntiles, tile, base, NsGemm{sl.Y, sl.q(k), sl.Z, sl.Y, 0, 1, -0.5, 1.5}, st);
    ns_gemm<T>(d, nblk, ntiles, tile, base, NsGemm{sl.x(k), sl.Y, sl.QB, -1, 1, 0, -0.5, 0.0}, st);
    ns_gemm<T>(d, nblk, ntiles, tile, base, NsGemm{sl.QB, sl.x(k), sl.Z, sl.Z, 0, 1, 1.0, 1.0}, st);
    ns_gemm<T>(d, nblk, ntiles, tile, base, NsGemm{sl.x(k), sl.QB, sl.Y, sl.Z, 1, 0, 1.0, 1.0}, st);
  }
  k_ns_final<T><<<nblk, 256, 0, st>>>(d, base, cnorm, sl.Y, sl.S, sl.SB, gin);
}

template void launch_ns_forward<float>(const NsDesc *, int32_t, int32_t, int32_t, int32_t, const float *, float *,
                                       float *, double *, hipStream_t);
template void launch_ns_forward<double>(const NsDesc *, int32_t, int32_t, int32_t, int32_t, const double *, double *,
                                        double *, double *, hipStream_t);
template void launch_ns_vjp<float>(const NsDesc *, int32_t, int32_t, int32_t, int32_t, const float *, float *, float *,
                                   const double *, hipStream_t);
template void launch_ns_vjp<double>(const NsDesc *, int32_t, int32_t, int32_t, int32_t, const double *, double *,
                                    double *, const double *, hipStream_t);

}  // namespace cosmo
