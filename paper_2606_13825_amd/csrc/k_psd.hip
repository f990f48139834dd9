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
// FP64; helpers in mma_tiles.h), on 16 x 16 output tiles, one wave per tile.
#include <type_traits>

#include "cosmo_internal.h"
#include "mma_tiles.h"

namespace cosmo {
namespace {

template <typename T> struct Unit;
template <> struct Unit<float> { static constexpr float eps = 5.96e-8f; };
template <> struct Unit<double> { static constexpr double eps = 1.11e-16; };

constexpr int MAXP = COSMO_MAX_PSD_ORDER_F32;

template <typename T, int NT> __device__ inline T wg_max(T v, T *red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  T t = red[0];
  for (int w = 1; w < NT / 64; ++w) t = fmax(t, red[w]);
  return t;
}

// Jacobi lanes move 16 bytes per LDS access in the padded classes.
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// Leading dimension of a p x p block held in LDS.  In order classes up to
// 128 the G lanes of a Jacobi pair read a column in 16-byte pieces (VE
// elements per lane, VE G rows per access of the group) without masks:
// columns are padded with zero rows to a multiple of VE G, then by 8 more
// elements, so ld is an odd multiple of 8 and the groups of a wave, which
// work on consecutive columns in the circle schedule, hit different LDS
// banks.  In the largest class a block alone nearly fills the LDS: even
// orders pad to the next odd one, lanes read single elements and reads past
// row p are clamped.  p * eig_ld(p) does not decrease with p.
template <typename T, int G, int PMAX> __host__ __device__ constexpr int eig_rows(int p) {
  return PMAX <= 128 ? (16 / (int)sizeof(T)) * G * ((p + (16 / (int)sizeof(T)) * G - 1) / ((16 / (int)sizeof(T)) * G))
                     : p;
}
template <typename T, int G, int PMAX> __host__ __device__ constexpr int eig_ld(int p) {
  return PMAX <= 128 ? eig_rows<T, G, PMAX>(p) + 8 : (p | 1);
}

// Cross-lane moves inside rows of 16 lanes (DPP): quad_perm [1,0,3,2] and
// [2,3,0,1], row_half_mirror, row_mirror.
template <int CTRL> __device__ inline float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ inline double dpp_mov(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over aligned groups of G = 4, 8 or 16 lanes, in every lane of the group.
template <int G, typename T> __device__ inline T group_sum(T x) {
  static_assert(G == 4 || G == 8 || G == 16, "group of 4, 8 or 16 lanes");
  x += dpp_mov<0xB1>(x);
  x += dpp_mov<0x4E>(x);
  if constexpr (G >= 8) x += dpp_mov<0x141>(x);
  if constexpr (G >= 16) x += dpp_mov<0x140>(x);
  return x;
}

// Jacobi rotation (cs, sn) that makes columns with squared norms al, be and
// inner product ga orthogonal (smaller angle, |tan| <= 1).  Float32 uses the
// hardware reciprocal and reciprocal square root: any rotation with
// cs^2 + sn^2 = 1 to working precision is valid, a slightly inexact angle only
// leaves a little more for the next sweep.
__device__ inline void jacobi_rot(float al, float be, float ga, float &cs, float &sn) {
  const float zeta = (be - al) * __builtin_amdgcn_rcpf(2.f * ga);
  const float tt = __builtin_amdgcn_rcpf(fabsf(zeta) + __builtin_amdgcn_sqrtf(1.f + zeta * zeta));
  cs = __builtin_amdgcn_rsqf(1.f + tt * tt);
  sn = copysignf(cs * tt, zeta);
}
__device__ inline void jacobi_rot(double al, double be, double ga, double &cs, double &sn) {
  const double zeta = (be - al) / (2.0 * ga);
  const double tt = 1.0 / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  cs = 1.0 / sqrt(1.0 + tt * tt);
  sn = copysign(cs * tt, zeta);
}

// Two 16 x 16 tiles C1 = A B1, C2 = A B2 sharing the A operand.
template <typename T, typename FA, typename FB1, typename FB2>
__device__ inline void tile_mma2(int I0, int J0, int kdim, FA fa, FB1 fb1, FB2 fb2, typename Mma<T>::v4 &c1,
                                 typename Mma<T>::v4 &c2) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kk = lane >> 4;
  c1 = typename Mma<T>::v4{0, 0, 0, 0};
  c2 = typename Mma<T>::v4{0, 0, 0, 0};
  int k0 = 0;
  for (; k0 + 16 <= kdim; k0 += 16) {
    T a[4], b1[4], b2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + kk;
      a[u] = fa(I0 + r, k);
      b1[u] = fb1(k, J0 + r);
      b2[u] = fb2(k, J0 + r);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c1 = Mma<T>::op(a[u], b1[u], c1);
      c2 = Mma<T>::op(a[u], b2[u], c2);
    }
  }
  for (; k0 < kdim; k0 += 4) {
    const int k = k0 + kk;
    const T a = fa(I0 + r, k);
    c1 = Mma<T>::op(a, fb1(k, J0 + r), c1);
    c2 = Mma<T>::op(a, fb2(k, J0 + r), c2);
  }
}

// Runs comp(t) for the tiles t = wave, wave + nw, ... below ntiles and stores
// each result with wr(t, result).  INPL: the wave keeps all its results in
// registers until every wave has finished computing (one barrier), so wr may
// overwrite what comp reads; HOLD must cover the tiles of one wave.  Ends
// with a barrier.
template <int HOLD, bool INPL, typename Fc, typename Fw>
__device__ inline void tile_pass(int ntiles, int wave, int nw, Fc comp, Fw wr) {
  if constexpr (INPL) {
    decltype(comp(0)) hold[HOLD];
#pragma unroll
    for (int h = 0; h < HOLD; ++h) {
      const int t = wave + h * nw;
      if (t < ntiles) hold[h] = comp(t);
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < HOLD; ++h) {
      const int t = wave + h * nw;
      if (t < ntiles) wr(t, hold[h]);
    }
  } else {
    for (int t = wave; t < ntiles; t += nw) wr(t, comp(t));
  }
  __syncthreads();
}

struct Acc2d {
  Mma<double>::v4 g, h;
};

// Refinement pair tag: the lowest mantissa bit of a stored E entry marks a
// pair on one side of the positive / non-positive split that was rotated.
__device__ inline float pair_tag(float e, bool rotated) {
  const unsigned int u = __float_as_uint(e);
  return __uint_as_float(rotated ? (u | 1u) : (u & ~1u));
}
__device__ inline bool pair_rotated(float e) { return (__float_as_uint(e) & 1u) != 0; }

// mode 0: COSMO step on the block (s+ and y+ rows); mode 1: projection only.
template <typename T, int NT, int G, int PMAX>
__global__ __launch_bounds__(NT) void k_psd_eig(const PsdDesc *__restrict__ descs, int32_t max_sweeps, T tol_base,
                                                int32_t mode, const T *__restrict__ rho_hat,
                                                const T *__restrict__ vin, const T *__restrict__ sh,
                                                const T *__restrict__ y, T *__restrict__ s_new,
                                                T *__restrict__ y_new, T *__restrict__ Uout,
                                                T *__restrict__ lamout, cosmo_stats *stats, int32_t refine,
                                                double *__restrict__ rscratch, const T *__restrict__ Uprev,
                                                int32_t attempt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *W = reinterpret_cast<T *>(smem_raw);
  __shared__ T red[NT / 64];
  __shared__ double redd[2 * (NT / 64)];
  __shared__ double lamd[PMAX];
  __shared__ short pos_idx[PMAX];
  __shared__ short posof[PMAX];
  __shared__ signed char cls[PMAX];
  __shared__ int flags[3];
  __shared__ int bigf[3];
  __shared__ int npos_s;
  __shared__ int redo_s;
  __shared__ int again_s;

  const PsdDesc d = descs[blockIdx.x];
  const int p = d.p;
  // Early-stopped sweeps (float32, orders up to 128, with refinement) can
  // leave a pair across the positive / non-positive split too coupled for
  // the refinement's first-order rotation; such a block writes only its
  // current eigenvectors (to the eigenvector output, when there is one), sets
  // its flag (a slot of the refinement scratch these classes do not use
  // otherwise), and a second launch (attempt 1) solves only the flagged
  // blocks, started from those eigenvectors, with the sweeps run to
  // convergence.
  constexpr bool EARLY = std::is_same<T, float>::value && PMAX <= 128;
  int *redo_g = (EARLY && refine > 0 && rscratch) ? reinterpret_cast<int *>(rscratch + 3 * (size_t)d.uoff) : nullptr;
  if (attempt == 1) {
    if (!redo_g || *redo_g == 0) return;   // the same value in every thread
  } else if (redo_g && threadIdx.x == 0) {
    *redo_g = 0;
  }
  const T *Uwarm = (attempt == 1 && Uout) ? Uout : Uprev;   // warm start of this attempt
  const int ld = eig_ld<T, G, PMAX>(p);
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
    W[i + j * ld] = val;
    W[j + i * ld] = val;
  }
  constexpr bool PADDED = PMAX <= 128;   // zero rows up to eig_rows (see eig_ld)
  const int ne = (p + G - 1) / G;         // column rows per Jacobi lane (unpadded class)
  if constexpr (PADDED) {
    const int npad = eig_rows<T, G, PMAX>(p) - p;
    for (int e = tid; e < npad * p; e += NT) {
      const int j = e / npad;
      W[p + (e - j * npad) + j * ld] = (T)0;
    }
  }
  if (tid < 3) flags[tid] = bigf[tid] = 0;
  if (tid == 0) redo_s = 0;
  fro2 = wg_sum<T, NT>(fro2, red);   // contains barriers: W complete after this
  if (!isfinite(fro2)) {
    // a non-finite block yields a non-finite projection (never a clipped one)
    for (int idx = tid; idx < nrows; idx += NT) {
      s_new[d.row0 + idx] = (T)NAN;
      if (mode == 0) y_new[d.row0 + idx] = (T)NAN;
    }
    if (lamout)
      for (int i = tid; i < p; i += NT) lamout[d.loff + i] = (T)NAN;
    if (Uout)
      for (int e = tid; e < p * p; e += NT) Uout[d.uoff + e] = (T)NAN;
    return;   // fro2 is the same in every thread: the whole workgroup leaves
  }
  T rowmax = 0;
  for (int i = tid; i < p; i += NT) {
    T a = 0;
    for (int j = 0; j < p; ++j) a += fabs(W[i + j * ld]);
    rowmax = fmax(rowmax, a);
  }
  const T inf = wg_max<T, NT>(rowmax, red);
  T c = (T)1.1 * fmin(sqrt(fro2), inf);
  if (!(c > (T)0)) c = (T)1;
  // Warm start: W = (S + c I) U_prev, with U_prev the eigenvectors of the same
  // block at the previous unrolled step.  One-sided Jacobi on W computes the
  // same decomposition (W = G V with V orthogonal, W'W diagonal at the end);
  // a nearly diagonalising start only shortens the sweeps.
  bool started = false;
  if constexpr (std::is_same<T, float>::value && PMAX <= 128) {
    if (Uwarm && refine > 0) {
      // U_prev staged in the refinement buffer (free until the refinement);
      // S is in W, so the products are held in registers until all are done
      constexpr int NWs = NT / 64;
      constexpr int NTM = (PMAX + 15) / 16;
      constexpr int HOLDS = (NTM * NTM + NWs - 1) / NWs;
      const float *Up = Uwarm + d.uoff;
      float *Ub = W + p * ld;
      for (int e = tid; e < p * p; e += NT) {
        const int j = e / p;
        Ub[(e - j * p) + j * ld] = Up[e];
      }
      __syncthreads();
      const int nt0 = (p + 15) / 16;
      const int wave0 = tid >> 6, lane0 = tid & 63;
      tile_pass<HOLDS, true>(
          nt0 * nt0, wave0, NWs,
          [&](int t) {
            const int I = t / nt0, J = t % nt0;
            return tile_mma<float>(
                I * 16, J * 16, p, [&](int i, int k) -> float { return (i < p && k < p) ? W[i + k * ld] : 0.f; },
                [&](int k, int j) -> float { return (k < p && j < p) ? Ub[k + j * ld] : 0.f; });
          },
          [&](int t, const Mma<float>::v4 &acc) {
            const int I = t / nt0, J = t % nt0;
            const int col = J * 16 + (lane0 & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int row = I * 16 + Mma<float>::row(lane0, e);
              if (row < p && col < p) W[row + col * ld] = acc[e] + c * Ub[row + col * ld];
            }
          });
      started = true;
    }
  }
  if (!started && Uwarm) {
    const T *Up = Uwarm + d.uoff;
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
        if (row < p && col < p) W[row + col * ld] = acc[e] + c * Up[row + col * p];
      }
    }
  } else if (!started) {
    for (int i = tid; i < p; i += NT) W[i + i * ld] += c;
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
  const T tol2 = tol * tol;
  // With the refinement behind them the sweeps of orders up to 128 can stop
  // once a sweep's largest column cosine is below 1e-3: the couplings left
  // are then of order 1e-6, well inside what one refinement step removes.
  // The largest class converges fully (stopping early there left 1e-4
  // errors on order-196 blocks).
  const T stop2 = (redo_g && attempt == 0) ? (T)1e-6 : (T)0;
  for (; sweep < max_sweeps && !converged; ++sweep) {
    const int fslot = sweep % 3;
    for (int r = 0; r < P - 1; ++r) {
      for (int k = grp; k < npairs; k += ngroups) {
        // circle schedule: column P-1 stays, the others rotate by one per round
        int a, b;
        if (k == 0) {
          a = r;
          b = P - 1;
        } else {
          a = r + k;
          if (a >= P - 1) a -= P - 1;
          b = r - k;
          if (b < 0) b += P - 1;
        }
        const bool live = a < p && b < p;   // else the dummy column of an odd order
        T *wa = W + (live ? a : 0) * ld;
        T *wb = W + (live ? b : 0) * ld;
        T al = 0, be = 0, ga = 0;
        bool rot = false;
        if constexpr (PADDED) {
          // Pieces past the last (c >= nc) re-read the lane's last piece, are
          // masked out of the sums, and their stores repeat that piece's.
          typedef typename Vec16<T>::type V;
          constexpr int VE = 16 / (int)sizeof(T);
          constexpr int MAXC = (PMAX + VE * G - 1) / (VE * G);
          const int nc = (p + VE * G - 1) / (VE * G);
          V xa[MAXC], xb[MAXC];
#pragma unroll
          for (int c = 0; c < MAXC; ++c) {
            const int rw = VE * (gl + (c < nc ? c : nc - 1) * G);
            xa[c] = *reinterpret_cast<const V *>(wa + rw);
            xb[c] = *reinterpret_cast<const V *>(wb + rw);
          }
#pragma unroll
          for (int c = 0; c < MAXC; ++c) {
            const T m = c < nc ? (T)1 : (T)0;
#pragma unroll
            for (int q = 0; q < VE; ++q) {
              const T u = m * xa[c][q], w = m * xb[c][q];
              al += u * u;
              be += w * w;
              ga += u * w;
            }
          }
          al = group_sum<G>(al);
          be = group_sum<G>(be);
          ga = group_sum<G>(ga);
          rot = live && ga * ga > tol2 * al * be;
          if (rot) {
            T cs, sn;
            jacobi_rot(al, be, ga, cs, sn);
#pragma unroll
            for (int c = 0; c < MAXC; ++c) {
              const int rw = VE * (gl + (c < nc ? c : nc - 1) * G);
              *reinterpret_cast<V *>(wa + rw) = cs * xa[c] - sn * xb[c];
              *reinterpret_cast<V *>(wb + rw) = sn * xa[c] + cs * xb[c];
            }
          }
        } else {
          // Rows past the lane's last one (e >= ne) re-read row p - 1 or the
          // lane's last row and are masked out of the sums; their stores
          // repeat the value stored for that row.
          auto row_of = [&](int e) {
            const int rw = gl + (e < ne ? e : ne - 1) * G;
            return rw < p ? rw : p - 1;
          };
          T xa[MAXE], xb[MAXE];
#pragma unroll
          for (int e = 0; e < MAXE; ++e) {
            xa[e] = wa[row_of(e)];
            xb[e] = wb[row_of(e)];
          }
#pragma unroll
          for (int e = 0; e < MAXE; ++e) {
            const bool in = e < ne && gl + e * G < p;
            const T u = in ? xa[e] : (T)0, w = in ? xb[e] : (T)0;
            al += u * u;
            be += w * w;
            ga += u * w;
          }
          al = group_sum<G>(al);
          be = group_sum<G>(be);
          ga = group_sum<G>(ga);
          rot = live && ga * ga > tol2 * al * be;
          if (rot) {
            T cs, sn;
            jacobi_rot(al, be, ga, cs, sn);
#pragma unroll
            for (int e = 0; e < MAXE; ++e) {
              wa[row_of(e)] = cs * xa[e] - sn * xb[e];
              wb[row_of(e)] = sn * xa[e] + cs * xb[e];
            }
          }
        }
        if (rot && gl == 0) {
          flags[fslot] = 1;
          if (ga * ga > stop2 * al * be) bigf[fslot] = 1;
        }
      }
      __syncthreads();
    }
    converged = (flags[fslot] == 0) || (stop2 > (T)0 && bigf[fslot] == 0);
    if (tid == 0) flags[(sweep + 2) % 3] = bigf[(sweep + 2) % 3] = 0;
  }
  // every thread computed `converged` from the same flag after the same barrier

  // eigenpairs: lam_i = ||w_i|| - c, u_i = w_i / ||w_i||
  for (int i = tid; i < p; i += NT) {
    const T *wi = W + i * ld;
    double ss = 0;
    for (int r = 0; r < p; ++r) ss += (double)wi[r] * (double)wi[r];
    lamd[i] = sqrt(ss);
  }
  __syncthreads();
  for (int e = tid; e < p * p; e += NT) {
    const int j = e / p, i = e - j * p;
    const double sg = lamd[j];
    W[i + j * ld] = sg > 0.0 ? (T)((double)W[i + j * ld] / sg) : (T)0;
  }
  __syncthreads();
  for (int i = tid; i < p; i += NT) lamd[i] -= (double)c;
  __syncthreads();

  const int nt = (p + 15) / 16;
  const int wave = tid >> 6, lane = tid & 63;
  constexpr int NWv = NT / 64;
  constexpr int NTMAX = (PMAX + 15) / 16;
  constexpr int HOLD = (NTMAX * NTMAX + NWv - 1) / NWv;
  constexpr int HOLDU = (NTMAX * (NTMAX + 1) / 2 + NWv - 1) / NWv;
  const int ntiles = nt * (nt + 1) / 2;
  const T *yb = y + d.row0;
  const T *shb = sh + d.row0;
  const T rh = (mode == 0) ? rho_hat[d.row0] : (T)0;
  // svec entry (row, col), row <= col, of the projection, and the y+ row
  auto put = [&](int row, int col, double val) {
    const int idx = col * (col + 1) / 2 + row;
    const T o = (T)((row == col) ? val : val * SQRT2);
    s_new[d.row0 + idx] = o;
    if (mode == 0) y_new[d.row0 + idx] = yb[idx] + rh * (shb[idx] - o);
  };
  auto count = [&]() {
    if (stats) {
      atomicMax(&stats[d.inst].eig_sweeps_max, sweep);
      atomicAdd(&stats[d.inst].eig_sweeps_total, sweep);
      atomicAdd(&stats[d.inst].eig_solves, 1);
      if (!converged) atomicAdd(&stats[d.inst].eig_not_converged, 1);
    }
  };

  if constexpr (std::is_same<T, float>::value) {
    if (refine > 0) {
      // Refinement of the float32 eigenpairs (after Ogita & Aishima,
      // "Iterative refinement for symmetric eigenvalue decomposition", 2018)
      // with float64-accumulated residual products, then the projection by
      // Rayleigh-Ritz on the positive subspace.  One step, with X the current
      // eigenvectors and lam~ the current eigenvalues:
      //   D = S X - X diag(lam~)                       (small; stored in float32)
      //   R = I - X'X,  S~ = X'S X = (X'X) diag(lam~) + X'D,  lam_i = S~_ii / (1 - R_ii)
      //   a pair (i, j) is resolvable when its gap exceeds
      //          delta = 2 (||S~ - diag(lam)||_F + ||S||_F ||R||_F) and its
      //          coupling-to-gap ratio th = cpl / gap is at most 0.1;
      //   E_ij = (S~_ij + lam_j R_ij) / (lam_j - lam_i)  for rotated pairs,
      //   E_ij = R_ij / 2 otherwise (re-orthogonalisation only)
      //   X <- X + X E.
      // Every resolvable pair is rotated, on either side of the split: the
      // projection needs only the positive subspace, but the Daleckii-Krein
      // weights of a pair across the split depend on the individual
      // eigenvalues on each side, so the taped eigenvectors must be
      // eigenvectors, not just a basis of the right subspace.  A step is the
      // last when every resolvable pair's second-order remainder
      // th^2 max|lam| is below 1e-7 ||S||_F (else another step follows: the
      // remainders shrink quadratically), at most REFINE_STEPS steps.  In the
      // last step only pairs that meet that bound rotate; the others are
      // re-orthogonalised and the projection's middle factor absorbs their
      // coupling:
      //   Pi = X+ M X+',  M = X+' S X+ to first order in E:
      //          M_ii = lam_i,  M_ij = 0 for rotated pairs,
      //          M_ij = S~_ij + (lam_i + lam_j) R_ij / 2 otherwise.
      // E + E' = R entry by entry keeps X orthonormal to second order.  Only
      // D and the products building S~ and R need float64 accumulation; the
      // correction X E is small and runs in float32.
      //
      // Storage of a pair i < j in the p x p buffer SR: slot (j, i) holds
      // E_ji.  Slot (i, j) holds E_ij when the pair rotates, else (pairs on
      // one side of the split) M_ij; for pairs on one side the lowest
      // mantissa bit of slot (j, i) says which (1: rotated, then M_ij = 0).
      // One unit in the last place of E is far below what E corrects.
      constexpr bool INPL = PMAX <= 128;   // second p x p buffer in LDS, else global scratch
      constexpr int REFINE_STEPS = 3;
      float *Db = INPL ? W + p * ld : reinterpret_cast<float *>(rscratch + 3 * (size_t)d.uoff);
      float *SR = INPL ? Db : Db + p * ld;   // S~ (upper) and R (lower), then E and M
      auto Sget = [&](int i, int k) -> double {
        if constexpr (INPL) {
          return (double)Db[i + k * ld];
        } else {
          const int a = i < k ? i : k, b = i < k ? k : i;
          const double val = (double)v[b * (b + 1) / 2 + a];
          return a == b ? val : val * RSQRT2;
        }
      };
      const double thr2 = 1e-7 * sqrt((double)fro2);
      // This block's part of the refinement scratch (3 p^2 doubles) beyond
      // the redo flag (orders up to 128) or beyond D, S~ and R (larger
      // orders): the refined eigenvalues of a step (float64), then L+ and C
      // of the projection (below).
      double *xs = rscratch + 3 * (size_t)d.uoff + (INPL ? 1 : (size_t)p * ld);
      // E_kj from the pair storage (see above)
      auto Eget = [&](int k, int j) -> float {
        if (k >= j || cls[k] * cls[j] < 0) return SR[k + j * ld];
        const float low = SR[j + k * ld];
        return pair_rotated(low) ? SR[k + j * ld] : low;
      };
      const int wave_o = wave, lane_o = lane;
      int rsteps = 0;
#pragma nounroll
      for (int rstep = 0; rstep < REFINE_STEPS; ++rstep) {
        // The wave and lane numbers are re-read opaquely in every step so
        // that the compiler does not hoist each tile's addresses out of the
        // loop (which exhausts the registers).
        int wave = wave_o, lane = lane_o;
        asm volatile("" : "+v"(wave), "+v"(lane));
        const bool last_allowed = rstep == REFINE_STEPS - 1;
        if constexpr (INPL) {   // S into the second buffer (the D pass overwrites it in place)
          for (int idx = tid; idx < nrows; idx += NT) {
            const int j = svec_col(idx);
            const int i = idx - j * (j + 1) / 2;
            float val = v[idx];
            if (i != j) val *= (float)RSQRT2;
            Db[i + j * ld] = val;
            Db[j + i * ld] = val;
          }
          __syncthreads();
        }
        // D = S X - X diag(lam~)
        tile_pass<HOLD, INPL>(
            nt * nt, wave, NWv,
            [&](int t) {
              const int I = t / nt, J = t % nt;
              return tile_mma<double>(
                  I * 16, J * 16, p, [&](int i, int k) -> double { return (i < p && k < p) ? Sget(i, k) : 0.0; },
                  [&](int k, int j) -> double { return (k < p && j < p) ? (double)W[k + j * ld] : 0.0; });
            },
            [&](int t, const Mma<double>::v4 &acc) {
              const int I = t / nt, J = t % nt;
              const int col = J * 16 + (lane & 15);
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int row = I * 16 + Mma<double>::row(lane, e);
                if (row < p && col < p) Db[row + col * ld] = (float)(acc[e] - (double)W[row + col * ld] * lamd[col]);
              }
            });
        // S~ into the upper triangle, R into the lower, lam_i on the diagonal
        double nS = 0, nR = 0;
        tile_pass<HOLDU, INPL>(
            ntiles, wave, NWv,
            [&](int t) {
              int I, J;
              upper_tile(t, I, J);
              Acc2d a;
              tile_mma2<double>(
                  I * 16, J * 16, p,
                  [&](int i, int k) -> double { return (i < p && k < p) ? (double)W[k + i * ld] : 0.0; },
                  [&](int k, int j) -> double { return (k < p && j < p) ? (double)W[k + j * ld] : 0.0; },
                  [&](int k, int j) -> double { return (k < p && j < p) ? (double)Db[k + j * ld] : 0.0; }, a.g, a.h);
              return a;
            },
            [&](int t, const Acc2d &a) {
              int I, J;
              upper_tile(t, I, J);
              const int col = J * 16 + (lane & 15);
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int row = I * 16 + Mma<double>::row(lane, e);
                if (row <= col && col < p) {
                  const double st = a.h[e] + a.g[e] * lamd[col];
                  if (row < col) {
                    const double r = -a.g[e];
                    SR[row + col * ld] = (float)st;
                    SR[col + row * ld] = (float)r;
                    nS += 2.0 * st * st;
                    nR += 2.0 * r * r;
                  } else {
                    const double lam = a.g[e] > 0.0 ? st / a.g[e] : 0.0;
                    const double r = 1.0 - a.g[e];
                    xs[row] = lam;   // kept in float64
                    nS += (st - lam) * (st - lam);
                    nR += r * r;
                  }
                }
              }
            });
        for (int off = 32; off > 0; off >>= 1) {
          nS += __shfl_xor(nS, off, 64);
          nR += __shfl_xor(nR, off, 64);
        }
        if (lane == 0) {
          redd[wave] = nS;
          redd[NWv + wave] = nR;
        }
        if (tid == 0) again_s = 0;
        // refined eigenvalues, their signs, and E_ii = R_ii / 2 on the diagonal
        for (int i = tid; i < p; i += NT) {
          const double lam = xs[i];
          double g = 0;
          for (int k = 0; k < p; ++k) {
            const double x = (double)W[k + i * ld];
            g += x * x;
          }
          lamd[i] = lam;
          cls[i] = lam > 0.0 ? 1 : (lam < 0.0 ? -1 : 0);
          SR[i + i * ld] = (float)(0.5 * (1.0 - g));
        }
        __syncthreads();
        double ts = 0, tr = 0;
        for (int w = 0; w < NWv; ++w) {
          ts += redd[w];
          tr += redd[NWv + w];
        }
        const double delta = 2.0 * (sqrt(ts) + sqrt((double)fro2) * sqrt(tr));
        // Pairs i < j: which rotate in this step if it is not the last, and
        // whether any of them leaves a remainder above the bound (then this
        // step is not the last).
        int more = 0;
        for (int e = tid; e < p * p; e += NT) {
          const int j = e / p, i = e - j * p;
          if (i >= j) continue;
          const double s = (double)SR[i + j * ld], r = (double)SR[j + i * ld];
          const double li = lamd[i], lj = lamd[j];
          const double gap = lj - li;
          const double th = (fabs(s) + fmax(fabs(li), fabs(lj)) * fabs(r)) / fabs(gap);
          if (fabs(gap) > delta && th <= 0.1 && th * th * fmax(fabs(li), fabs(lj)) > thr2) more = 1;
        }
        if (more) again_s = 1;
        __syncthreads();
        const bool last = last_allowed || again_s == 0;
        for (int e = tid; e < p * p; e += NT) {
          const int j = e / p, i = e - j * p;
          if (i >= j) continue;
          const double s = (double)SR[i + j * ld], r = (double)SR[j + i * ld];
          const double li = lamd[i], lj = lamd[j];
          const double gap = lj - li;
          const double th = (fabs(s) + fmax(fabs(li), fabs(lj)) * fabs(r)) / fabs(gap);
          const bool ok = fabs(gap) > delta && th <= 0.1;
          const bool fin = th * th * fmax(fabs(li), fabs(lj)) <= thr2;
          const bool rot = ok && (fin || !last);
          const float eij = (float)(rot ? (s + lj * r) / gap : 0.5 * r);
          const float eji = (float)(rot ? (s + li * r) / (-gap) : 0.5 * r);
          if (li * lj < 0.0) {
            if (last && ok && !fin && stop2 > (T)0) redo_s = 1;   // resolvable, but not to first order
            SR[i + j * ld] = eij;
            SR[j + i * ld] = eji;
          } else {
            SR[i + j * ld] = rot ? eij : (float)(s + 0.5 * (li + lj) * r);
            SR[j + i * ld] = pair_tag(eji, rot);
          }
        }
        __syncthreads();
        if (last && redo_s) {   // read after the barrier above: the same in every thread
          if (Uout)
            for (int e = tid; e < p * p; e += NT) {
              const int j = e / p, i = e - j * p;
              Uout[d.uoff + e] = W[i + j * ld];
            }
          if (tid == 0) *redo_g = 1;
          return;
        }
        rsteps = rstep + 1;
        if (last) break;
        // X <- X + X E, in place in W (the last step's correction is kept apart, below)
        tile_pass<HOLD, true>(
            nt * nt, wave, NWv,
            [&](int t) {
              const int I = t / nt, J = t % nt;
              return tile_mma<float>(
                  I * 16, J * 16, p, [&](int i, int k) -> float { return (i < p && k < p) ? W[i + k * ld] : 0.f; },
                  [&](int k, int j) -> float { return (k < p && j < p) ? Eget(k, j) : 0.f; });
            },
            [&](int t, const Mma<float>::v4 &acc) {
              const int I = t / nt, J = t % nt;
              const int col = J * 16 + (lane & 15);
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int row = I * 16 + Mma<float>::row(lane, e);
                if (row < p && col < p) W[row + col * ld] += acc[e];
              }
            });
      }
      if (stats && tid == 0) atomicAdd(&stats[d.inst].eig_refine_steps_total, rsteps);
      if (lamout)
        for (int i = tid; i < p; i += NT) lamout[d.loff + i] = (float)lamd[i];
      if (tid == 0) {
        int np = 0;
        for (int i = 0; i < p; ++i) {
          posof[i] = cls[i] > 0 ? (short)np : (short)-1;
          if (cls[i] > 0) pos_idx[np++] = (short)i;
        }
        npos_s = np;
        count();
      }
      __syncthreads();
      const int npos = npos_s;
      const int ntp = (npos + 15) / 16;
      // The last step's correction L = X E is not rounded into X: the
      // refined eigenvectors are X + L with both parts float32 (their sum is
      // carried to about twice the float32 precision), and the projection is
      // formed from them with float64 products,
      //   C = (X+ + L+) M,   Pi = C (X+ + L+)',
      // so its accuracy is that of the refinement, not that of float32
      // eigenvectors.  The taped eigenvectors are X + L rounded to float32.
      // L+ (p x npos, float32) and C (p x npos, float64) live in this
      // block's part of the refinement scratch (xs).
      float *Lg = reinterpret_cast<float *>(xs);
      double *Cg = xs + ((size_t)p * npos + 1) / 2;
      tile_pass<HOLD, false>(
          nt * nt, wave, NWv,
          [&](int t) {
            const int I = t / nt, J = t % nt;
            return tile_mma<float>(
                I * 16, J * 16, p, [&](int i, int k) -> float { return (i < p && k < p) ? W[i + k * ld] : 0.f; },
                [&](int k, int j) -> float { return (k < p && j < p) ? Eget(k, j) : 0.f; });
          },
          [&](int t, const Mma<float>::v4 &acc) {
            const int I = t / nt, J = t % nt;
            const int col = J * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int row = I * 16 + Mma<float>::row(lane, e);
              if (row < p && col < p) {
                if (Uout) Uout[d.uoff + row + col * p] = W[row + col * ld] + acc[e];
                const int q = posof[col];
                if (q >= 0) Lg[row + q * p] = acc[e];
              }
            }
          });
      // M on the positive pairs: lam_i (float64) on the diagonal
      auto Mget = [&](int a, int b) -> double {
        if (a == b) return lamd[a];
        const int lo = a < b ? a : b, hi = a < b ? b : a;
        return pair_rotated(SR[hi + lo * ld]) ? 0.0 : (double)SR[lo + hi * ld];
      };
      auto Xp = [&](int i, int k) -> double { return (double)W[i + pos_idx[k] * ld] + (double)Lg[i + k * p]; };
      // C = (X+ + L+) M  (p x npos)
      tile_pass<HOLD, false>(
          nt * ntp, wave, NWv,
          [&](int t) {
            const int I = t / ntp, J = t % ntp;
            return tile_mma<double>(
                I * 16, J * 16, npos, [&](int i, int k) -> double { return (i < p && k < npos) ? Xp(i, k) : 0.0; },
                [&](int k, int j) -> double { return (k < npos && j < npos) ? Mget(pos_idx[k], pos_idx[j]) : 0.0; });
          },
          [&](int t, const Mma<double>::v4 &acc) {
            const int I = t / ntp, J = t % ntp;
            const int col = J * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int row = I * 16 + Mma<double>::row(lane, e);
              if (row < p && col < npos) Cg[row + col * p] = acc[e];
            }
          });
      // Pi = C (X+ + L+)', upper-triangle tiles
      for (int t = wave; t < ntiles; t += NWv) {
        int I, J;
        upper_tile(t, I, J);
        const Mma<double>::v4 acc = tile_mma<double>(
            I * 16, J * 16, npos, [&](int i, int k) -> double { return (i < p && k < npos) ? Cg[i + k * p] : 0.0; },
            [&](int k, int j) -> double { return (j < p && k < npos) ? Xp(j, k) : 0.0; });
        const int col = J * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = I * 16 + Mma<double>::row(lane, e);
          if (row <= col && col < p) put(row, col, acc[e]);
        }
      }
      return;
    }
  }

  // Unrefined: Pi = sum_{lam_k > 0} lam_k u_k u_k' (upper-triangle tiles)
  if (lamout)
    for (int i = tid; i < p; i += NT) lamout[d.loff + i] = (T)lamd[i];
  if (Uout)
    for (int e = tid; e < p * p; e += NT) {
      const int j = e / p, i = e - j * p;
      Uout[d.uoff + e] = W[i + j * ld];
    }
  if (tid == 0) {
    int np = 0;
    for (int i = 0; i < p; ++i)
      if (lamd[i] > 0.0) pos_idx[np++] = (short)i;
    npos_s = np;
    count();
  }
  __syncthreads();
  const int npos = npos_s;
  for (int t = wave; t < ntiles; t += NWv) {
    int I, J;
    upper_tile(t, I, J);
    const typename Mma<T>::v4 acc = tile_mma<T>(
        I * 16, J * 16, npos,
        [&](int i, int k) -> T {
          if (i >= p || k >= npos) return (T)0;
          const int c2 = pos_idx[k];
          return W[i + c2 * ld] * (T)lamd[c2];
        },
        [&](int k, int j) -> T { return (j >= p || k >= npos) ? (T)0 : W[j + pos_idx[k] * ld]; });
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I * 16 + Mma<T>::row(lane, e);
      if (row <= col && col < p) put(row, col, (double)acc[e]);
    }
  }
}

// Leading dimension of the DK VJP's LDS buffers: the smallest stride >= p
// that is 4 modulo 8 words, so the 16 columns one matrix-core operand read
// touches (16 lanes, one column each, four consecutive rows per column
// group) fall on distinct banks; a stride that is a multiple of 16 would put
// all 16 on one bank.
__host__ __device__ constexpr int dk_ld(int p) { return p + ((4 - p % 8) + 8) % 8; }

// Weight of entry (i, j) of U' smat(g) U in the input cotangent.
//   rule 0 (DK, eq:lowner): divided differences of max(., 0), f' on ties,
//     f'(0) = 0.
//   rule 1 (eq:psd-cotangent as autograd evaluates it on U max(L, 0) U', then
//     symmetrised by the svec adjoint): f'(l_i) on the diagonal, else
//     f(l_j) / (l_j - l_i) + f(l_i) / (l_i - l_j) with both quotients formed,
//     so a tie gives inf - inf or 0 / 0 and close eigenvalues cancel.
//   rule 2 (Tikhonov): rule 1 at the eigenvalues of S + eps I.
template <typename T> __device__ inline T vjp_weight(int rule, T li, T lj, bool diag, T eps) {
  if (rule == 0) {
    if (li > (T)0 && lj > (T)0) return (T)1;
    if (li <= (T)0 && lj <= (T)0) return (T)0;
    return fmax(li, lj) / (fabs(li) + fabs(lj));
  }
  const T a = li + eps, b = lj + eps;
  if (diag) return a > (T)0 ? (T)1 : (T)0;
  const T fa = fmax(a, (T)0), fb = fmax(b, (T)0);
  return fb / (b - a) + fa / (a - b);
}

// PSD VJP: out = svec(U (W o (U' smat(g) U)) U'), W from vjp_weight.  Buffers:
// B0 and B1 (p x p, stride dk_ld(p)) in LDS when they fit, else B1 in global
// scratch (stride p); U read from LDS when a third buffer fits, else from
// global memory.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_psd_vjp(const PsdDesc *__restrict__ descs, const T *__restrict__ Ug,
                                                const T *__restrict__ lam, const T *__restrict__ g,
                                                T *__restrict__ out, T *__restrict__ scratch, int32_t lds_elems,
                                                int32_t rule, T eps) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  __shared__ T lam_s[MAXP];
  const PsdDesc d = descs[blockIdx.x];
  const int p = d.p, pp = p * p, lp = dk_ld(p), ppl = p * lp;
  const int tid = threadIdx.x;
  T *B0 = lds;
  // B0 keeps the padded stride when it fits, else p (the largest orders)
  const int l0 = ppl <= lds_elems ? lp : p;
  const bool b1_lds = 2 * ppl <= lds_elems;
  T *B1 = b1_lds ? lds + ppl : scratch + d.uoff;
  const int l1 = b1_lds ? lp : p;
  const T *U = Ug + d.uoff;
  int lu = p;
  if (3 * ppl <= lds_elems) {
    T *Ul = lds + 2 * ppl;
    for (int e = tid; e < pp; e += NT) {
      const int j = e / p;
      Ul[(e - j * p) + j * lp] = U[e];
    }
    U = Ul;
    lu = lp;
  }
  for (int i = tid; i < p; i += NT) lam_s[i] = lam[d.loff + i];
  const T *gb = g + d.row0;
  const int nrows = p * (p + 1) / 2;
  for (int idx = tid; idx < nrows; idx += NT) {
    const int j = svec_col(idx);
    const int i = idx - j * (j + 1) / 2;
    T val = gb[idx];
    if (i != j) val *= (T)RSQRT2;
    B0[i + j * l0] = val;
    B0[j + i * l0] = val;
  }
  __syncthreads();
  const int nt = (p + 15) / 16;
  const int wave = tid >> 6, lane = tid & 63;
  const int NWv = NT / 64;
  // B1 = B0 U
  for (int t = wave; t < nt * nt; t += NWv) {
    const int I = t / nt, J = t % nt;
    auto fa = [&](int i, int k) -> T { return (i < p && k < p) ? B0[i + k * l0] : (T)0; };
    auto fb = [&](int k, int j) -> T { return (k < p && j < p) ? U[k + j * lu] : (T)0; };
    const typename Mma<T>::v4 acc = tile_mma<T>(I * 16, J * 16, p, fa, fb);
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I * 16 + Mma<T>::row(lane, e);
      if (row < p && col < p) B1[row + col * l1] = acc[e];
    }
  }
  __syncthreads();
  // B0 = W o (U' B1): U' smat(g) U and W are symmetric, so only the upper
  // tiles are formed; entry (row, col), row <= col, is written to both
  // places by the lane that owns it (one writer per element).
  const int nup = nt * (nt + 1) / 2;
  for (int t = wave; t < nup; t += NWv) {
    int I, J;
    upper_tile(t, I, J);
    auto fa = [&](int i, int k) -> T { return (i < p && k < p) ? U[k + i * lu] : (T)0; };
    auto fb = [&](int k, int j) -> T { return (k < p && j < p) ? B1[k + j * l1] : (T)0; };
    const typename Mma<T>::v4 acc = tile_mma<T>(I * 16, J * 16, p, fa, fb);
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I * 16 + Mma<T>::row(lane, e);
      if (row <= col && col < p) {
        const T val = vjp_weight<T>(rule, lam_s[row], lam_s[col], row == col, eps) * acc[e];
        B0[row + col * l0] = val;
        B0[col + row * l0] = val;
      }
    }
  }
  __syncthreads();
  // B1 = U B0
  for (int t = wave; t < nt * nt; t += NWv) {
    const int I = t / nt, J = t % nt;
    auto fa = [&](int i, int k) -> T { return (i < p && k < p) ? U[i + k * lu] : (T)0; };
    auto fb = [&](int k, int j) -> T { return (k < p && j < p) ? B0[k + j * l0] : (T)0; };
    const typename Mma<T>::v4 acc = tile_mma<T>(I * 16, J * 16, p, fa, fb);
    const int col = J * 16 + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = I * 16 + Mma<T>::row(lane, e);
      if (row < p && col < p) B1[row + col * l1] = acc[e];
    }
  }
  __syncthreads();
  // out = svec(B1 U'), upper tiles
  const int ntiles = nt * (nt + 1) / 2;
  T *ob = out + d.row0;
  for (int t = wave; t < ntiles; t += NWv) {
    int I, J;
    upper_tile(t, I, J);
    auto fa = [&](int i, int k) -> T { return (i < p && k < p) ? B1[i + k * l1] : (T)0; };
    auto fb = [&](int k, int j) -> T { return (k < p && j < p) ? U[j + k * lu] : (T)0; };
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

// Allow a kernel the whole LDS of a workgroup minus its static allocation;
// returns the dynamic LDS bytes it may use.
size_t set_dyn_lds_cap(const void *fn) {
  hipFuncAttributes a{};
  size_t stat = 4096;
  if (hipFuncGetAttributes(&a, fn) == hipSuccess) stat = a.sharedSizeBytes;
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(LDS_LIMIT - stat));
  return LDS_LIMIT - stat;
}

template <typename T, int NT, int G, int PMAX>
void run_eig(const PsdDesc *d, int32_t n, int32_t max_p, const PsdLaunchCfg &cfg, int32_t mode, const T *rho_hat,
             const T *vv, const T *sh, const T *y, T *s_new, T *y_new, T *U, T *lam, cosmo_stats *stats,
             double *rscratch, const T *Uprev, hipStream_t st) {
  // The float32 refinement keeps a second p x ld buffer in LDS for classes up
  // to order 128, in the global scratch above.
  const int refine = (std::is_same<T, float>::value && rscratch) ? cfg.refine : 0;
  const size_t nbuf = (refine > 0 && PMAX <= 128) ? 2 : 1;
  const size_t dyn = nbuf * (size_t)max_p * (size_t)eig_ld<T, G, PMAX>(max_p) * sizeof(T);
  static bool attr_set = false;
  if (!attr_set) {
    set_dyn_lds_cap(reinterpret_cast<const void *>(&k_psd_eig<T, NT, G, PMAX>));
    attr_set = true;
  }
  k_psd_eig<T, NT, G, PMAX><<<n, NT, dyn, st>>>(d, cfg.max_sweeps, (T)cfg.tol, mode, rho_hat, vv, sh, y, s_new,
                                                y_new, U, lam, stats, refine, rscratch, Uprev, 0);
  if (std::is_same<T, float>::value && PMAX <= 128 && refine > 0 && rscratch)   // the flagged blocks again
    k_psd_eig<T, NT, G, PMAX><<<n, NT, dyn, st>>>(d, cfg.max_sweeps, (T)cfg.tol, mode, rho_hat, vv, sh, y, s_new,
                                                  y_new, U, lam, stats, refine, rscratch, Uprev, 1);
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
  const int cls = mp <= 32 ? 0 : mp <= 64 ? 1 : mp <= 128 ? 2 : 3;
  const bool alt = cfg.threads != 0 && cfg.threads == kEigThreadsAlt[cls] && cfg.threads != kEigThreads[cls];
#define COSMO_EIG(NT_, G_, PMAX_) \
  run_eig<T, NT_, G_, PMAX_>(d, n, mp, cfg, mode, rho_hat, vv, sh, y, s_new, y_new, U, lam, stats, rscratch, Uprev, st)
  static_assert(kEigThreads[0] == 64 && kEigThreads[1] == 256 && kEigThreads[2] == 512 && kEigThreads[3] == 1024,
                "class defaults");
  static_assert(kEigThreadsAlt[0] == 128 && kEigThreadsAlt[1] == 512 && kEigThreadsAlt[2] == 1024, "class alternatives");
  if (cls == 0) {
    if (alt) COSMO_EIG(128, 4, 32); else COSMO_EIG(64, 4, 32);
  } else if (cls == 1) {
    if (alt) COSMO_EIG(512, 8, 64); else COSMO_EIG(256, 8, 64);
  } else if (cls == 2) {
    if (alt) COSMO_EIG(1024, 8, 128); else COSMO_EIG(512, 8, 128);
  } else if constexpr (std::is_same<T, float>::value) {
    COSMO_EIG(1024, 8, COSMO_MAX_PSD_ORDER_F32);
  } else {
    COSMO_EIG(1024, 8, COSMO_MAX_PSD_ORDER_F64);
  }
#undef COSMO_EIG
}

// 16 waves by default: a block of order ~100 has 49 output tiles per
// product, so the longest wave runs 4 of them instead of 7 with 8 waves; the
// autotuner may pick 8 waves (two workgroups per compute unit where LDS
// allows).  Every tile is formed by one wave with the same instructions
// whichever wave it is, so both shapes give bitwise the same result.
template <typename T, int NT>
bool run_vjp(const PsdDesc *d, int32_t n, int32_t max_p, const T *U, const T *lam, const T *g, T *out, T *scratch,
             hipStream_t st, int32_t rule, double eps) {
  static size_t dyn_bytes = 0;
  if (dyn_bytes == 0) dyn_bytes = set_dyn_lds_cap(reinterpret_cast<const void *>(&k_psd_vjp<T, NT>));
  // LDS holds B0 (and B1, then U) at the padded stride while they fit; the
  // largest orders keep only B0, unpadded (order 200 in float32: 160,000
  // bytes), with B1 in the global scratch.
  const size_t ppl = (size_t)max_p * dk_ld(max_p);   // p dk_ld(p) does not decrease with p
  const size_t pp = (size_t)max_p * max_p;
  const size_t budget = dyn_bytes / sizeof(T);
  size_t elems;
  if (3 * ppl <= budget) elems = 3 * ppl;
  else if (2 * ppl <= budget) elems = 2 * ppl;
  else if (ppl <= budget) elems = ppl;
  else if (pp <= budget) elems = pp;   // every order the validation admits fits here
  else return false;
  k_psd_vjp<T, NT><<<n, NT, elems * sizeof(T), st>>>(d, U, lam, g, out, scratch, (int32_t)elems, rule, (T)eps);
  return true;
}

template <typename T>
bool launch_psd_vjp(const PsdDesc *d, int32_t n, int32_t max_p, const T *U, const T *lam, const T *g, T *out,
                    T *scratch, hipStream_t st, int32_t rule, double eps, int32_t threads) {
  if (n <= 0) return true;
  static_assert(kVjpThreads == 1024 && kVjpThreadsAlt == 512, "VJP shapes");
  if (threads == kVjpThreadsAlt) return run_vjp<T, 512>(d, n, max_p, U, lam, g, out, scratch, st, rule, eps);
  return run_vjp<T, 1024>(d, n, max_p, U, lam, g, out, scratch, st, rule, eps);
}

template void launch_psd_step<float>(const PsdDesc *, int32_t, const PsdLaunchCfg &, const float *, const float *,
                                     const float *, const float *, float *, float *, float *, float *, double *,
                                     const float *, cosmo_stats *, hipStream_t);
template void launch_psd_step<double>(const PsdDesc *, int32_t, const PsdLaunchCfg &, const double *,
                                      const double *, const double *, const double *, double *, double *, double *,
                                      double *, double *, const double *, cosmo_stats *, hipStream_t);
template bool launch_psd_vjp<float>(const PsdDesc *, int32_t, int32_t, const float *, const float *, const float *,
                                    float *, float *, hipStream_t, int32_t, double, int32_t);
template bool launch_psd_vjp<double>(const PsdDesc *, int32_t, int32_t, const double *, const double *,
                                     const double *, double *, double *, hipStream_t, int32_t, double, int32_t);
}  // namespace cosmo
