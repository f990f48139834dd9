// PSD-cone blocks: projection by eigendecomposition (eq:psd-proj) and the
// Daleckii-Krein vector-Jacobian product (eq:psd-cotangent-dk, eq:lowner).
//
// Eigensolver: one-sided (Hestenes) cyclic Jacobi on the shifted block
// G = S + c I, c = 1.1 min(||S||_F, ||S||_inf) >= 1.1 ||S||_2, so G is
// positive definite with condition number below 21.  Column pairs of W
// (initially G) are rotated until every pair is orthogonal to the tolerance;
// then W = G V with V orthogonal and W'W diagonal, hence the normalised
// columns of W are eigenvectors of S and the column norms minus c are its
// eigenvalues.  Rotations never mix columns that are already orthogonal, so
// exactly or nearly repeated eigenvalues need no special treatment: the
// eigenvectors come out orthonormal to working precision regardless of
// gaps.  The whole p x p block stays in LDS (<= 160 KiB).
//
// One round pairs every column once (round-robin "circle" schedule, p-1
// rounds per sweep); G consecutive lanes own one pair, reduce the three dot
// products with a butterfly and rotate the two columns.  One barrier per
// round.
//
// Reconstruction Pi = U diag(max(lam, 0)) U' and the four products of the DK
// rule U (L o (U' T U)) U' run on the matrix cores (v_mfma 16x16x4, FP32 or
// FP64), on 16 x 16 output tiles, one wave per tile.
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

template <typename T> struct Unit;
template <> struct Unit<float> { static constexpr float eps = 5.96e-8f; };
template <> struct Unit<double> { static constexpr double eps = 1.11e-16; };

constexpr double RSQRT2 = 0.70710678118654752440;
constexpr double SQRT2 = 1.41421356237309504880;
constexpr int MAXP = COSMO_MAX_PSD_ORDER_F32;

// 16 x 16 tile of C = A B with A(i, k), B(k, j) given by functors that return
// 0 outside the matrices.  Lane l feeds A(I0 + l%16, k0 + l/16) and
// B(k0 + l/16, J0 + l%16); accumulator element e of lane l is
// C(I0 + Mma<T>::row(l, e), J0 + l%16).
template <typename T, typename FA, typename FB>
__device__ inline typename Mma<T>::v4 tile_mma(int I0, int J0, int kdim, FA fa, FB fb) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kk = lane >> 4;
  typename Mma<T>::v4 acc = {0, 0, 0, 0};
  for (int k0 = 0; k0 < kdim; k0 += 4) {
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

template <typename T, int NT> __device__ inline T wg_max(T v, T *red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = red[0];
  for (int w = 1; w < NT / 64; ++w) t = fmax(t, red[w]);
  return t;
}

// mode 0: COSMO step on the block (s+ and y+ rows); mode 1: projection only.
template <typename T, int NT, int G, int PMAX>
__global__ __launch_bounds__(NT) void k_psd_eig(const PsdDesc *__restrict__ descs, int32_t max_sweeps, T tol_base,
                                                int32_t mode, const T *__restrict__ rho_hat,
                                                const T *__restrict__ vin, const T *__restrict__ sh,
                                                const T *__restrict__ y, T *__restrict__ s_new,
                                                T *__restrict__ y_new, T *__restrict__ Uout,
                                                T *__restrict__ lamout, cosmo_stats *stats, int32_t refine,
                                                double *__restrict__ rscratch, const T *__restrict__ Uprev) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *W = reinterpret_cast<T *>(smem_raw);
  __shared__ T red[NT / 64];
  __shared__ double redd[2 * (NT / 64)];
  __shared__ double lamd[MAXP];
  __shared__ int pos_idx[MAXP];
  __shared__ int flags[3];
  __shared__ int npos_s;

  const PsdDesc d = descs[blockIdx.x];
  const int p = d.p;
  const int nrows = p * (p + 1) / 2;
  const T *v = vin + d.row0;
  const int tid = threadIdx.x;

  // S = smat(v) into W (column-major, full); ||S||_F^2 = ||v||^2 (svec is isometric)
  T fro2 = 0;
  for (int idx = tid; idx < nrows; idx += NT) {
    const int j = svec_col(idx);
    const int i = idx - j * (j + 1) / 2;
    T val = v[idx];
    fro2 += val * val;
    if (i != j) val *= (T)RSQRT2;
    W[i + j * p] = val;
    W[j + i * p] = val;
  }
  if (tid < 3) flags[tid] = 0;
  fro2 = wg_sum<T, NT>(fro2, red);   // contains barriers: W complete after this
  T rowmax = 0;
  for (int i = tid; i < p; i += NT) {
    T a = 0;
    for (int j = 0; j < p; ++j) a += fabs(W[i + j * p]);
    rowmax = fmax(rowmax, a);
  }
  const T inf = wg_max<T, NT>(rowmax, red);
  T c = (T)1.1 * fmin(sqrt(fro2), inf);
  if (!(c > (T)0)) c = (T)1;
  if (Uprev) {
    // Warm start: W = (S + c I) U_prev, with U_prev the eigenvectors of the same
    // block at the previous unrolled step.  One-sided Jacobi on W computes the
    // same decomposition (W = G V with V orthogonal, W'W diagonal at the end);
    // a nearly diagonalising start only shortens the sweeps.
    const T *Up = Uprev + d.uoff;
    const int nt0 = (p + 15) / 16;
    const int wave0 = tid >> 6, lane0 = tid & 63;
    for (int t = wave0; t < nt0 * nt0; t += NT / 64) {
      const int I = t / nt0, J = t % nt0;
      const typename Mma<T>::v4 acc = tile_mma<T>(
          I * 16, J * 16, p,
          [&](int i, int k) -> T {
            if (i >= p || k >= p) return (T)0;
            const int a = i < k ? i : k, b = i < k ? k : i;
            const T val = v[b * (b + 1) / 2 + a];
            return a == b ? val : val * (T)RSQRT2;
          },
          [&](int k, int j) -> T { return (k < p && j < p) ? Up[k + j * p] : (T)0; });
      const int col = J * 16 + (lane0 & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = I * 16 + Mma<T>::row(lane0, e);
        if (row < p && col < p) W[row + col * p] = acc[e] + c * Up[row + col * p];
      }
    }
  } else {
    for (int i = tid; i < p; i += NT) W[i + i * p] += c;
  }
  __syncthreads();

  const T tol = tol_base > (T)0 ? tol_base : (T)4 * Unit<T>::eps * sqrt((T)p);
  const int P = p + (p & 1);
  const int npairs = P / 2;
  const int ngroups = NT / G;
  const int grp = tid / G, gl = tid % G;
  constexpr int MAXE = (PMAX + G - 1) / G;   // column elements held per lane
  int sweep = 0;
  bool converged = (p == 1);
  for (; sweep < max_sweeps && !converged; ++sweep) {
    const int fslot = sweep % 3;
    for (int r = 0; r < P - 1; ++r) {
      for (int k = grp; k < npairs; k += ngroups) {
        int a, b;
        if (k == 0) {
          a = r;
          b = P - 1;
        } else {
          a = (r + k) % (P - 1);
          b = (r - k + P - 1) % (P - 1);
        }
        if (a >= p || b >= p) continue;   // dummy column of an odd order
        if (a > b) {
          const int tmp = a;
          a = b;
          b = tmp;
        }
        T *wa = W + a * p;
        T *wb = W + b * p;
        T xa[MAXE], xb[MAXE];
        T al = 0, be = 0, ga = 0;
#pragma unroll
        for (int e = 0; e < MAXE; ++e) {
          const int i = gl + e * G;
          xa[e] = (i < p) ? wa[i] : (T)0;
          xb[e] = (i < p) ? wb[i] : (T)0;
          al += xa[e] * xa[e];
          be += xb[e] * xb[e];
          ga += xa[e] * xb[e];
        }
        for (int off = G >> 1; off > 0; off >>= 1) {
          al += __shfl_xor(al, off, 64);
          be += __shfl_xor(be, off, 64);
          ga += __shfl_xor(ga, off, 64);
        }
        if (fabs(ga) > tol * sqrt(al * be)) {
          const T zeta = (be - al) / ((T)2 * ga);
          const T tt = (zeta >= (T)0 ? (T)1 : (T)-1) / (fabs(zeta) + sqrt((T)1 + zeta * zeta));
          const T cs = (T)1 / sqrt((T)1 + tt * tt);
          const T sn = cs * tt;
#pragma unroll
          for (int e = 0; e < MAXE; ++e) {
            const int i = gl + e * G;
            if (i < p) {
              wa[i] = cs * xa[e] - sn * xb[e];
              wb[i] = sn * xa[e] + cs * xb[e];
            }
          }
          if (gl == 0) flags[fslot] = 1;
        }
      }
      __syncthreads();
    }
    converged = (flags[fslot] == 0);
    if (tid == 0) flags[(sweep + 2) % 3] = 0;
  }
  // every thread computed `converged` from the same flag after the same barrier

  // eigenpairs: lam_i = ||w_i|| - c, u_i = w_i / ||w_i||
  for (int i = tid; i < p; i += NT) {
    const T *wi = W + i * p;
    double ss = 0;
    for (int r = 0; r < p; ++r) ss += (double)wi[r] * (double)wi[r];
    lamd[i] = sqrt(ss);
  }
  __syncthreads();
  for (int e = tid; e < p * p; e += NT) {
    const double sg = lamd[e / p];
    W[e] = sg > 0.0 ? (T)((double)W[e] / sg) : (T)0;
  }
  __syncthreads();
  for (int i = tid; i < p; i += NT) lamd[i] -= (double)c;
  __syncthreads();

  const int nt = (p + 15) / 16;
  const int wave = tid >> 6, lane = tid & 63;
  constexpr int NWv = NT / 64;
  const int pp = p * p;

  // Optional float64 refinement of the float32 eigenpairs (Ogita & Aishima,
  // "Iterative refinement for symmetric eigenvalue decomposition", 2018):
  //   R = I - X'X,  S~ = X' S X,  lam_i = S~_ii / (1 - R_ii),
  //   delta = 2 (||S~ - diag(lam)|| + ||S|| ||R||)   (Frobenius bounds),
  //   E_ij = (S~_ij + lam_j R_ij) / (lam_j - lam_i) if |lam_j - lam_i| > delta, else R_ij / 2,
  //   X <- X + X E.
  // Every product is accumulated in float64 on the matrix cores.  Pairs
  // closer than delta (and pairs whose correction would not be small) are
  // only re-orthogonalised; the projection is then formed by Rayleigh-Ritz on
  // the positive subspace, Pi = X+ (X+' S X+) X+', which depends on the split
  // between positive and non-positive eigenvalues only, not on how the
  // eigenvectors are chosen inside a cluster.
  const double *Xg = nullptr;   // refined eigenvectors in global float64 scratch
  double *bA = nullptr, *bE = nullptr, *bX = nullptr;
  if (refine > 0) {
    bA = rscratch + 3 * d.uoff;
    bE = bA + pp;
    bX = bE + pp;
    double *xdst = bX;
    const double sfro = sqrt((double)fro2);
    for (int step = 0; step < refine; ++step) {
      const double *xs = Xg;
      auto X = [&](int i, int j) -> double { return xs ? xs[i + j * p] : (double)W[i + j * p]; };
      auto Sv = [&](int i, int k) -> double {
        const int a = i < k ? i : k, b = i < k ? k : i;
        const double val = (double)v[b * (b + 1) / 2 + a];
        return a == b ? val : val * RSQRT2;
      };
      // A1 = S X
      for (int t = wave; t < nt * nt; t += NWv) {
        const int I = t / nt, J = t % nt;
        const typename Mma<double>::v4 acc = tile_mma<double>(
            I * 16, J * 16, p, [&](int i, int k) -> double { return (i < p && k < p) ? Sv(i, k) : 0.0; },
            [&](int k, int j) -> double { return (k < p && j < p) ? X(k, j) : 0.0; });
        const int col = J * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = I * 16 + Mma<double>::row(lane, e);
          if (row < p && col < p) bA[row + col * p] = acc[e];
        }
      }
      __syncthreads();
      for (int i = tid; i < p; i += NT) {
        double si = 0, gi = 0;
        for (int r = 0; r < p; ++r) {
          const double xr = X(r, i);
          si += xr * bA[r + i * p];
          gi += xr * xr;
        }
        lamd[i] = si / gi;
      }
      __syncthreads();
      // pass 1: Frobenius norms of S~ - diag(lam) and R; pass 2: E
      double nS = 0, nR = 0, delta = 0;
      for (int pass = 0; pass < 2; ++pass) {
        for (int t = wave; t < nt * nt; t += NWv) {
          const int I = t / nt, J = t % nt;
          auto fxt = [&](int i, int k) -> double { return (i < p && k < p) ? X(k, i) : 0.0; };
          const typename Mma<double>::v4 as = tile_mma<double>(
              I * 16, J * 16, p, fxt, [&](int k, int j) -> double { return (k < p && j < p) ? bA[k + j * p] : 0.0; });
          const typename Mma<double>::v4 ag = tile_mma<double>(
              I * 16, J * 16, p, fxt, [&](int k, int j) -> double { return (k < p && j < p) ? X(k, j) : 0.0; });
          const int col = J * 16 + (lane & 15);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int row = I * 16 + Mma<double>::row(lane, e);
            if (row < p && col < p) {
              const double rij = (row == col ? 1.0 : 0.0) - ag[e];
              if (pass == 0) {
                const double dv = (row == col) ? as[e] - lamd[row] : as[e];
                nS += dv * dv;
                nR += rij * rij;
              } else {
                const double li = lamd[row], lj = lamd[col];
                const double num = as[e] + lj * rij, gap = lj - li;
                // The projection and the Loewner-weighted VJP depend only on
                // the split between positive and non-positive eigenvalues, so
                // only pairs across that split are rotated, and only when the
                // correction is small (|E_ij| <= 1e-3); every other pair is
                // re-orthogonalised.  The test is symmetric in (i, j), so
                // E + E' = R entry by entry and X stays orthonormal to second
                // order.
                const double cpl = fabs(as[e]) + fmax(fabs(li), fabs(lj)) * fabs(rij);
                const bool rotate = (li * lj < 0.0) && fabs(gap) > delta && cpl <= 1e-3 * fabs(gap);
                bE[row + col * p] = rotate ? num / gap : 0.5 * rij;
              }
            }
          }
        }
        if (pass == 0) {
          for (int off = 32; off > 0; off >>= 1) {
            nS += __shfl_xor(nS, off, 64);
            nR += __shfl_xor(nR, off, 64);
          }
          __syncthreads();
          if (lane == 0) {
            redd[wave] = nS;
            redd[NWv + wave] = nR;
          }
          __syncthreads();
          double ts = 0, tr = 0;
          for (int w = 0; w < NWv; ++w) {
            ts += redd[w];
            tr += redd[NWv + w];
          }
          delta = 2.0 * (sqrt(ts) + sfro * sqrt(tr));
        }
      }
      __syncthreads();
      // X <- X + X E  (into the buffer not being read)
      for (int t = wave; t < nt * nt; t += NWv) {
        const int I = t / nt, J = t % nt;
        const typename Mma<double>::v4 acc = tile_mma<double>(
            I * 16, J * 16, p, [&](int i, int k) -> double { return (i < p && k < p) ? X(i, k) : 0.0; },
            [&](int k, int j) -> double { return (k < p && j < p) ? bE[k + j * p] : 0.0; });
        const int col = J * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = I * 16 + Mma<double>::row(lane, e);
          if (row < p && col < p) xdst[row + col * p] = X(row, col) + acc[e];
        }
      }
      __syncthreads();
      Xg = xdst;
      xdst = (xdst == bX) ? bA : bX;
    }
  }

  if (lamout)
    for (int i = tid; i < p; i += NT) lamout[d.loff + i] = (T)lamd[i];
  if (Uout)
    for (int e = tid; e < pp; e += NT) Uout[d.uoff + e] = Xg ? (T)Xg[e] : W[e];
  if (tid == 0) {
    int np = 0;
    for (int i = 0; i < p; ++i)
      if (lamd[i] > 0.0) pos_idx[np++] = i;
    npos_s = np;
    if (stats) {
      atomicMax(&stats[d.inst].eig_sweeps_max, sweep);
      if (!converged) atomicAdd(&stats[d.inst].eig_not_converged, 1);
    }
  }
  __syncthreads();
  const int npos = npos_s;

  const int ntiles = nt * (nt + 1) / 2;
  const T *yb = y + d.row0;
  const T *shb = sh + d.row0;
  const T rh = (mode == 0) ? rho_hat[d.row0] : (T)0;
  const int ntp = (npos + 15) / 16;
  double *Mrr = nullptr;   // X+' S X+  (npos x npos) for the Rayleigh-Ritz form
  double *Crr = nullptr;   // X+ (X+' S X+)  (p x npos)
  if (Xg && npos > 0) {
    double *free1 = (Xg == bA) ? bX : bA;
    double *free2 = bE;
    auto Sv = [&](int i, int k) -> double {
      const int a = i < k ? i : k, b = i < k ? k : i;
      const double val = (double)v[b * (b + 1) / 2 + a];
      return a == b ? val : val * RSQRT2;
    };
    // T1 = S X+  (p x npos) -> free1
    for (int t = wave; t < nt * ntp; t += NWv) {
      const int I = t / ntp, J = t % ntp;
      const typename Mma<double>::v4 acc = tile_mma<double>(
          I * 16, J * 16, p, [&](int i, int k) -> double { return (i < p && k < p) ? Sv(i, k) : 0.0; },
          [&](int k, int j) -> double { return (k < p && j < npos) ? Xg[k + pos_idx[j] * p] : 0.0; });
      const int col = J * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = I * 16 + Mma<double>::row(lane, e);
        if (row < p && col < npos) free1[row + col * p] = acc[e];
      }
    }
    __syncthreads();
    // M = X+' T1  (npos x npos) -> free2
    for (int t = wave; t < ntp * ntp; t += NWv) {
      const int I = t / ntp, J = t % ntp;
      const typename Mma<double>::v4 acc = tile_mma<double>(
          I * 16, J * 16, p, [&](int i, int k) -> double { return (i < npos && k < p) ? Xg[k + pos_idx[i] * p] : 0.0; },
          [&](int k, int j) -> double { return (k < p && j < npos) ? free1[k + j * p] : 0.0; });
      const int col = J * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = I * 16 + Mma<double>::row(lane, e);
        if (row < npos && col < npos) free2[row + col * npos] = acc[e];
      }
    }
    __syncthreads();
    // C = X+ M  (p x npos) -> free1
    for (int t = wave; t < nt * ntp; t += NWv) {
      const int I = t / ntp, J = t % ntp;
      const typename Mma<double>::v4 acc = tile_mma<double>(
          I * 16, J * 16, npos,
          [&](int i, int k) -> double { return (i < p && k < npos) ? Xg[i + pos_idx[k] * p] : 0.0; },
          [&](int k, int j) -> double { return (k < npos && j < npos) ? free2[k + j * npos] : 0.0; });
      const int col = J * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = I * 16 + Mma<double>::row(lane, e);
        if (row < p && col < npos) free1[row + col * p] = acc[e];
      }
    }
    __syncthreads();
    Mrr = free2;
    Crr = free1;
  }
  (void)Mrr;

  // Pi: Rayleigh-Ritz C X+' when refined, else sum_{lam_k > 0} lam_k u_k u_k'
  // (upper-triangle tiles only)
  for (int t = wave; t < ntiles; t += NWv) {
    int I, J;
    upper_tile(t, I, J);
    double accv[4];
    int rowv[4];
    if (Xg) {
      const typename Mma<double>::v4 acc = tile_mma<double>(
          I * 16, J * 16, npos,
          [&](int i, int k) -> double { return (i >= p || k >= npos) ? 0.0 : Crr[i + k * p]; },
          [&](int k, int j) -> double { return (j >= p || k >= npos) ? 0.0 : Xg[j + pos_idx[k] * p]; });
      for (int e = 0; e < 4; ++e) {
        accv[e] = acc[e];
        rowv[e] = Mma<double>::row(lane, e);
      }
    } else {
      const typename Mma<T>::v4 acc = tile_mma<T>(
          I * 16, J * 16, npos,
          [&](int i, int k) -> T {
            if (i >= p || k >= npos) return (T)0;
            const int c2 = pos_idx[k];
            return W[i + c2 * p] * (T)lamd[c2];
          },
          [&](int k, int j) -> T { return (j >= p || k >= npos) ? (T)0 : W[j + pos_idx[k] * p]; });
      for (int e = 0; e < 4; ++e) {
        accv[e] = (double)acc[e];
        rowv[e] = Mma<T>::row(lane, e);
      }
    }
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I * 16 + rowv[e];
      if (row <= col && col < p) {
        const int idx = col * (col + 1) / 2 + row;
        const T val = (T)((row == col) ? accv[e] : accv[e] * SQRT2);
        s_new[d.row0 + idx] = val;
        if (mode == 0) y_new[d.row0 + idx] = yb[idx] + rh * (shb[idx] - val);
      }
    }
  }
}

// DK VJP: out = svec(U (L o (U' smat(g) U)) U').  Buffers: B0 and B1 (p x p)
// in LDS when they fit, else B1 in global scratch; U read from LDS when a
// third buffer fits, else from global memory.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_psd_vjp(const PsdDesc *__restrict__ descs, const T *__restrict__ Ug,
                                                const T *__restrict__ lam, const T *__restrict__ g,
                                                T *__restrict__ out, T *__restrict__ scratch, int32_t lds_elems) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  __shared__ T lam_s[MAXP];
  const PsdDesc d = descs[blockIdx.x];
  const int p = d.p, pp = p * p;
  const int tid = threadIdx.x;
  T *B0 = lds;
  T *B1 = (2 * pp <= lds_elems) ? lds + pp : scratch + d.uoff;
  const T *U = Ug + d.uoff;
  if (3 * pp <= lds_elems) {
    T *Ul = lds + 2 * pp;
    for (int e = tid; e < pp; e += NT) Ul[e] = U[e];
    U = Ul;
  }
  for (int i = tid; i < p; i += NT) lam_s[i] = lam[d.loff + i];
  const T *gb = g + d.row0;
  const int nrows = p * (p + 1) / 2;
  for (int idx = tid; idx < nrows; idx += NT) {
    const int j = svec_col(idx);
    const int i = idx - j * (j + 1) / 2;
    T val = gb[idx];
    if (i != j) val *= (T)RSQRT2;
    B0[i + j * p] = val;
    B0[j + i * p] = val;
  }
  __syncthreads();
  const int nt = (p + 15) / 16;
  const int wave = tid >> 6, lane = tid & 63;
  const int NWv = NT / 64;
  // B1 = B0 U
  for (int t = wave; t < nt * nt; t += NWv) {
    const int I = t / nt, J = t % nt;
    auto fa = [&](int i, int k) -> T { return (i < p && k < p) ? B0[i + k * p] : (T)0; };
    auto fb = [&](int k, int j) -> T { return (k < p && j < p) ? U[k + j * p] : (T)0; };
    const typename Mma<T>::v4 acc = tile_mma<T>(I * 16, J * 16, p, fa, fb);
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I * 16 + Mma<T>::row(lane, e);
      if (row < p && col < p) B1[row + col * p] = acc[e];
    }
  }
  __syncthreads();
  // B0 = L o (U' B1)
  for (int t = wave; t < nt * nt; t += NWv) {
    const int I = t / nt, J = t % nt;
    auto fa = [&](int i, int k) -> T { return (i < p && k < p) ? U[k + i * p] : (T)0; };
    auto fb = [&](int k, int j) -> T { return (k < p && j < p) ? B1[k + j * p] : (T)0; };
    const typename Mma<T>::v4 acc = tile_mma<T>(I * 16, J * 16, p, fa, fb);
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I * 16 + Mma<T>::row(lane, e);
      if (row < p && col < p) {
        const T li = lam_s[row], lj = lam_s[col];
        T L;
        if (li > (T)0 && lj > (T)0) L = (T)1;
        else if (li <= (T)0 && lj <= (T)0) L = (T)0;
        else L = fmax(li, lj) / (fabs(li) + fabs(lj));
        B0[row + col * p] = L * acc[e];
      }
    }
  }
  __syncthreads();
  // B1 = U B0
  for (int t = wave; t < nt * nt; t += NWv) {
    const int I = t / nt, J = t % nt;
    auto fa = [&](int i, int k) -> T { return (i < p && k < p) ? U[i + k * p] : (T)0; };
    auto fb = [&](int k, int j) -> T { return (k < p && j < p) ? B0[k + j * p] : (T)0; };
    const typename Mma<T>::v4 acc = tile_mma<T>(I * 16, J * 16, p, fa, fb);
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I * 16 + Mma<T>::row(lane, e);
      if (row < p && col < p) B1[row + col * p] = acc[e];
    }
  }
  __syncthreads();
  // out = svec(B1 U'), upper tiles
  const int ntiles = nt * (nt + 1) / 2;
  T *ob = out + d.row0;
  for (int t = wave; t < ntiles; t += NWv) {
    int I, J;
    upper_tile(t, I, J);
    auto fa = [&](int i, int k) -> T { return (i < p && k < p) ? B1[i + k * p] : (T)0; };
    auto fb = [&](int k, int j) -> T { return (k < p && j < p) ? U[j + k * p] : (T)0; };
    const typename Mma<T>::v4 acc = tile_mma<T>(I * 16, J * 16, p, fa, fb);
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I * 16 + Mma<T>::row(lane, e);
      if (row <= col && col < p) {
        const int idx = col * (col + 1) / 2 + row;
        ob[idx] = (row == col) ? acc[e] : acc[e] * (T)SQRT2;
      }
    }
  }
}

constexpr size_t LDS_LIMIT = 163840;

// Allow a kernel the whole LDS of a workgroup minus its static allocation.
void set_dyn_lds_cap(const void *fn) {
  hipFuncAttributes a{};
  size_t stat = 4096;
  if (hipFuncGetAttributes(&a, fn) == hipSuccess) stat = a.sharedSizeBytes;
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(LDS_LIMIT - stat));
}

template <typename T, int NT, int G, int PMAX>
void run_eig(const PsdDesc *d, int32_t n, int32_t max_p, const PsdLaunchCfg &cfg, int32_t mode, const T *rho_hat,
             const T *vv, const T *sh, const T *y, T *s_new, T *y_new, T *U, T *lam, cosmo_stats *stats,
             double *rscratch, const T *Uprev, hipStream_t st) {
  const size_t dyn = (size_t)max_p * max_p * sizeof(T);
  static bool attr_set = false;
  if (!attr_set) {
    set_dyn_lds_cap(reinterpret_cast<const void *>(&k_psd_eig<T, NT, G, PMAX>));
    attr_set = true;
  }
  k_psd_eig<T, NT, G, PMAX><<<n, NT, dyn, st>>>(d, cfg.max_sweeps, (T)cfg.tol, mode, rho_hat, vv, sh, y, s_new,
                                                y_new, U, lam, stats, rscratch ? cfg.refine : 0, rscratch, Uprev);
}

}  // namespace

// Blocks arrive sorted by order class (see the plan): callers pass one class
// per call with its largest order.
template <typename T>
void launch_psd_step(const PsdDesc *d, int32_t n, const PsdLaunchCfg &cfg, const T *rho_hat, const T *vv,
                     const T *sh, const T *y, T *s_new, T *y_new, T *U, T *lam, double *rscratch,
                     const T *Uprev, cosmo_stats *stats, hipStream_t st) {
  if (n <= 0) return;
  const int mode = (y_new != nullptr) ? 0 : 1;
  const int mp = cfg.max_p;
  if (mp <= 32) run_eig<T, 64, 4, 32>(d, n, mp, cfg, mode, rho_hat, vv, sh, y, s_new, y_new, U, lam, stats, rscratch, Uprev, st);
  else if (mp <= 64) run_eig<T, 256, 8, 64>(d, n, mp, cfg, mode, rho_hat, vv, sh, y, s_new, y_new, U, lam, stats, rscratch, Uprev, st);
  else if (mp <= 128) run_eig<T, 512, 8, 128>(d, n, mp, cfg, mode, rho_hat, vv, sh, y, s_new, y_new, U, lam, stats, rscratch, Uprev, st);
  else run_eig<T, 1024, 8, 200>(d, n, mp, cfg, mode, rho_hat, vv, sh, y, s_new, y_new, U, lam, stats, rscratch, Uprev, st);
}

template <typename T>
void launch_psd_vjp(const PsdDesc *d, int32_t n, int32_t max_p, const T *U, const T *lam, const T *g, T *out,
                    T *scratch, hipStream_t st) {
  if (n <= 0) return;
  const size_t pp = (size_t)max_p * max_p;
  const size_t budget = (LDS_LIMIT - 4096) / sizeof(T);
  size_t elems = pp;
  if (3 * pp <= budget) elems = 3 * pp;
  else if (2 * pp <= budget) elems = 2 * pp;
  static bool attr_set = false;
  if (!attr_set) {
    set_dyn_lds_cap(reinterpret_cast<const void *>(&k_psd_vjp<T, 512>));
    attr_set = true;
  }
  k_psd_vjp<T, 512><<<n, 512, elems * sizeof(T), st>>>(d, U, lam, g, out, scratch, (int32_t)elems);
}

template void launch_psd_step<float>(const PsdDesc *, int32_t, const PsdLaunchCfg &, const float *, const float *,
                                     const float *, const float *, float *, float *, float *, float *, double *,
                                     const float *, cosmo_stats *, hipStream_t);
template void launch_psd_step<double>(const PsdDesc *, int32_t, const PsdLaunchCfg &, const double *,
                                      const double *, const double *, const double *, double *, double *, double *,
                                      double *, double *, const double *, cosmo_stats *, hipStream_t);
template void launch_psd_vjp<float>(const PsdDesc *, int32_t, int32_t, const float *, const float *, const float *,
                                    float *, float *, hipStream_t);
template void launch_psd_vjp<double>(const PsdDesc *, int32_t, int32_t, const double *, const double *,
                                     const double *, double *, double *, hipStream_t);

}  // namespace cosmo
