// The learned hyperparameter policy inside the unroll (App. E "Policy
// Parameterization"; widths, bounds and initial values from Table 2) and the
// log-residual loss (Sec. "Experiments"): per-instance norms of the KKT and
// ADMM residuals, the per-row penalty network on the matrix cores, the
// per-instance relaxation network, and the reverse passes of all three.  The
// residual vectors and their adjoint products come from k_vec.hip
// (launch_pol_resid, launch_pol_resid_adjoint).
//
// Per iterate z^k (rows i of instance b):
//   N_p = max(|A x|, |s|, |b|)_inf,  N_d = max(|P x|, |q|, |A' y|)_inf,
//   rbar_p = r_p / N_p,  rbar_d = r_d / N_d  (0 when N = 0),
//   xi_rho,i  = (l_i, s_i, y_i, rbar_p,i, log(|rbar_d|_inf + eps), dp_i, dd_i),
//   xi_alpha  = (l_a, log(|rbar_p|_inf + eps), log(|rbar_d|_inf + eps),
//                log(|dp|_inf + eps), log(|dd|_inf + eps)),
//   dp = s - s~ (the s~ that produced s), dd = s - s^{k-1}, both 0 at k = 0;
//   l^{k+1} = l^k + MLP(xi),  rho^k = exp(log rho_min + (log rho_max -
//   log rho_min) sigmoid(l_rho^{k+1})),  alpha^k = 2 sigmoid(l_alpha^{k+1}).
// Reverse mode: ties in an infinity norm or in the max of a normaliser
// share the cotangent evenly, |.| has derivative 0 at 0.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cosmo_internal.h"
#include "mma_tiles.h"

namespace cosmo {
namespace {

constexpr int NTP = 256;                         // per-instance kernels
constexpr int NTR = 256;                         // per-row elementwise kernels
constexpr double LOG_RHO_MIN = -6.907755278982137;   // log(1e-3)
constexpr double LOG_RHO_MAX = 6.907755278982137;    // log(1e3)
constexpr double POL_EPS = 1e-12;

// offsets inside one network's parameters (the flat layout of the header):
// W1 [n_in][32] input-major, b1 [32], W2 [32][32] input-major, b2, w3, b3
constexpr int OW1 = 0;
constexpr int OB1_R = POL_FR * POL_H, OW2_R = OB1_R + POL_H, OB2_R = OW2_R + POL_H * POL_H, OW3_R = OB2_R + POL_H,
              OB3_R = OW3_R + POL_H;
constexpr int OB1_A = POL_FA * POL_H, OW2_A = OB1_A + POL_H, OB2_A = OW2_A + POL_H * POL_H, OW3_A = OB2_A + POL_H,
              OB3_A = OW3_A + POL_H;
static_assert(OB3_R + 1 == POL_RHO_PARAMS && OB3_A + 1 == POL_ALPHA_PARAMS, "parameter layout");

// LDS of the per-row network kernels: the rho network's parameters, then per
// wave the 64 x 8 features (column 7 = 1, which folds b1 into W1 as its row
// 7), the two 64 x 32 hidden layers (stride 33) and the 64 output cotangents.
constexpr int HLD = POL_H + 1;
constexpr int PER_WAVE = 64 * 8 + 2 * 64 * HLD + 64;
template <typename T> constexpr size_t row_lds_bytes() { return (POL_RHO_PARAMS + POL_WAVES * PER_WAVE) * sizeof(T); }

__device__ inline double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }

__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
// Workgroup reductions with a fixed tree (deterministic); every thread gets the result.
template <int N> __device__ inline double blk_sum(double v, double *red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = red[0];
  for (int w = 1; w < N / 64; ++w) t += red[w];
  return t;
}

__device__ inline double norm_p(const PolRec &R) { return fmax(fmax(R.nu, R.ns), R.nb); }
__device__ inline double norm_d(const PolRec &R) { return fmax(fmax(R.np, R.nq), R.nw); }

// ---- per-instance norms ---------------------------------------------------------

// One workgroup per instance: the infinity norms, their tie counts and the
// squared residual norms of the loss; all values of a pass reduced together
// (one LDS exchange per pass).
constexpr int NTN = 512;

template <int NV> __device__ inline void wave_reduce_into(double (&a)[NV], int n_max, double (*red)[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) a[q] = q < n_max ? wave_max(a[q]) : wave_sum(a[q]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[threadIdx.x >> 6][q] = a[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = red[0][q];
    for (int w = 1; w < NTN / 64; ++w) t = q < n_max ? fmax(t, red[w][q]) : t + red[w][q];
    a[q] = t;
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(NTN) void k_pol_norms(View<T> v, const T *__restrict__ u, const T *__restrict__ rp,
                                                   const T *__restrict__ p, const T *__restrict__ w,
                                                   const T *__restrict__ rd, const T *__restrict__ s,
                                                   const T *__restrict__ s_prev, const T *__restrict__ st_prev,
                                                   PolRec *__restrict__ rec) {
  __shared__ double red1[NTN / 64][12];
  __shared__ double red2[NTN / 64][8];
  const int b = blockIdx.x;
  const int64_t r0 = v.m_off[b], r1 = v.m_off[b + 1], c0 = v.n_off[b], c1 = v.n_off[b + 1];
  // maxima: u, s, b, rp, dp, dd, p, q, w, rd; sums: rp^2, rd^2
  double a[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = r0 + threadIdx.x; i < r1; i += NTN) {
    const double si = s[i], ri = rp[i];
    a[0] = fmax(a[0], fabs((double)u[i]));
    a[1] = fmax(a[1], fabs(si));
    a[2] = fmax(a[2], fabs((double)v.b[i]));
    a[3] = fmax(a[3], fabs(ri));
    if (st_prev) a[4] = fmax(a[4], fabs(si - (double)st_prev[i]));
    if (s_prev) a[5] = fmax(a[5], fabs(si - (double)s_prev[i]));
    a[10] += ri * ri;
  }
  for (int64_t j = c0 + threadIdx.x; j < c1; j += NTN) {
    const double dj = rd[j];
    a[6] = fmax(a[6], fabs((double)p[j]));
    a[7] = fmax(a[7], fabs((double)v.q[j]));
    a[8] = fmax(a[8], fabs((double)w[j]));
    a[9] = fmax(a[9], fabs(dj));
    a[11] += dj * dj;
  }
  wave_reduce_into<12>(a, 10, red1);
  PolRec R;
  R.nu = a[0];
  R.ns = a[1];
  R.nb = a[2];
  R.mrp = a[3];
  R.mdp = a[4];
  R.mdd = a[5];
  R.np = a[6];
  R.nq = a[7];
  R.nw = a[8];
  R.mrd = a[9];
  R.ssp = a[10];
  R.ssd = a[11];
  // tie counts: u, s, rp, dp, dd, p, w, rd
  double c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = r0 + threadIdx.x; i < r1; i += NTN) {
    const double si = s[i];
    c[0] += fabs((double)u[i]) == R.nu;
    c[1] += fabs(si) == R.ns;
    c[2] += fabs((double)rp[i]) == R.mrp;
    if (st_prev) c[3] += fabs(si - (double)st_prev[i]) == R.mdp;
    if (s_prev) c[4] += fabs(si - (double)s_prev[i]) == R.mdd;
  }
  for (int64_t j = c0 + threadIdx.x; j < c1; j += NTN) {
    c[5] += fabs((double)p[j]) == R.np;
    c[6] += fabs((double)w[j]) == R.nw;
    c[7] += fabs((double)rd[j]) == R.mrd;
  }
  wave_reduce_into<8>(c, 0, red2);
  R.cu = (int32_t)c[0];
  R.cs = (int32_t)c[1];
  R.crp = (int32_t)c[2];
  R.cdp = (int32_t)c[3];
  R.cdd = (int32_t)c[4];
  R.cp = (int32_t)c[5];
  R.cw = (int32_t)c[6];
  R.crd = (int32_t)c[7];
  if (threadIdx.x == 0) rec[b] = R;
}

// ---- per-instance network and loss --------------------------------------------

// The relaxation network's features at iterate k.
template <typename T> __device__ inline void alpha_features(const PolRec &R, T l, T *xi) {
  const double Np = norm_p(R), Nd = norm_d(R);
  xi[0] = l;
  xi[1] = (T)log((Np > 0 ? R.mrp / Np : 0.0) + POL_EPS);
  xi[2] = (T)log((Nd > 0 ? R.mrd / Nd : 0.0) + POL_EPS);
  xi[3] = (T)log(R.mdp + POL_EPS);
  xi[4] = (T)log(R.mdd + POL_EPS);
}

// Hidden layers of the relaxation network, threads 0..31 one unit each.
template <typename T>
__device__ inline void alpha_hidden(const T *__restrict__ th, const T *xi, T *h1, T *h2) {
  const int t = threadIdx.x;
  if (t < POL_H) {
    T a = th[OB1_A + t];
    for (int f = 0; f < POL_FA; ++f) a += xi[f] * th[OW1 + f * POL_H + t];
    h1[t] = a > (T)0 ? a : (T)0;
  }
  __syncthreads();
  if (t < POL_H) {
    T a = th[OB2_A + t];
    for (int c = 0; c < POL_H; ++c) a += h1[c] * th[OW2_A + c * POL_H + t];
    h2[t] = a > (T)0 ? a : (T)0;
  }
  __syncthreads();
}

// One workgroup of 64 per instance.  The loss: k = 0 records the
// denominators |r_d^0|^2 and |r_p^0|^2 (1 when zero); k >= 1 adds
// log(|r_d^k|^2 / D_d + |r_p^k|^2 / D_p).  With `policy`, also the
// relaxation network: l_alpha^{k+1} and alpha^k.
template <typename T>
__global__ __launch_bounds__(64) void k_pol_inst_fwd(View<T> v, const T *__restrict__ theta,
                                                     const PolRec *__restrict__ rec, int32_t k, int32_t policy,
                                                     const T *__restrict__ la_in, T *__restrict__ la_out,
                                                     T *__restrict__ alpha_k, double *__restrict__ acc3,
                                                     T *__restrict__ loss) {
  __shared__ T h1[POL_H], h2[POL_H];
  const int b = blockIdx.x;
  const PolRec R = rec[b];
  if (threadIdx.x == 0) {
    double *a = acc3 + 3 * (size_t)b;
    if (k == 0) {
      a[0] = R.ssd > 0 ? R.ssd : 1.0;
      a[1] = R.ssp > 0 ? R.ssp : 1.0;
      a[2] = 0.0;
    } else {
      a[2] += log(R.ssd / a[0] + R.ssp / a[1]);
    }
    if (loss) loss[b] = (T)a[2];
  }
  if (!policy) return;
  const T *th = theta + POL_RHO_PARAMS;
  T xi[POL_FA];
  alpha_features<T>(R, la_in ? la_in[b] : theta[POL_L0 + 4], xi);
  alpha_hidden<T>(th, xi, h1, h2);
  if (threadIdx.x == 0) {
    T o = th[OB3_A];
    for (int c = 0; c < POL_H; ++c) o += h2[c] * th[OW3_A + c];
    const T l1 = xi[0] + o;
    la_out[b] = l1;
    alpha_k[b] = (T)(2.0 / (1.0 + exp(-(double)l1)));
  }
}

// ---- per-row penalty network ------------------------------------------------------

template <typename T> struct RowLds {
  T *W, *X, *H1, *H2, *OB;
};

template <typename T> __device__ inline RowLds<T> row_lds(T *base, int wave) {
  RowLds<T> L;
  L.W = base;
  T *wb = base + POL_RHO_PARAMS + wave * PER_WAVE;
  L.X = wb;
  L.H1 = wb + 64 * 8;
  L.H2 = L.H1 + 64 * HLD;
  L.OB = L.H2 + 64 * HLD;
  return L;
}

// Row i's features (column 7 = 1); zeros for a row past the end.
template <typename T>
__device__ inline void row_features(const View<T> &v, const T *__restrict__ theta, const PolRec *__restrict__ rec,
                                    const T *__restrict__ l_in, const T *__restrict__ s, const T *__restrict__ y,
                                    const T *__restrict__ rp, const T *__restrict__ s_prev,
                                    const T *__restrict__ st_prev, int64_t i, T *xo) {
  const PolRec R = rec[v.row_inst[i]];
  const double Np = norm_p(R), Nd = norm_d(R);
  const double si = s[i];
  xo[0] = l_in ? l_in[i] : theta[POL_L0 + v.row_kind[i]];
  xo[1] = s[i];
  xo[2] = y[i];
  xo[3] = (T)(Np > 0 ? (double)rp[i] / Np : 0.0);
  xo[4] = (T)log((Nd > 0 ? R.mrd / Nd : 0.0) + POL_EPS);
  xo[5] = st_prev ? (T)(si - (double)st_prev[i]) : (T)0;
  xo[6] = s_prev ? (T)(si - (double)s_prev[i]) : (T)0;
  xo[7] = (T)1;
}

// H1 = relu(X W1') and H2 = relu(H1 W2 + b2) for the wave's 64 rows, as
// 16 x 16 matrix-core tiles (W1' = [W1; b1], the features' column 7 = 1).
template <typename T> __device__ inline void rows_forward(const RowLds<T> &L, int lane) {
  for (int t = 0; t < 8; ++t) {
    const int I = (t >> 1) * 16, J = (t & 1) * 16;
    auto acc = tile_mma<T>(I, J, 8, [&](int r, int k) { return L.X[r * 8 + k]; },
                           [&](int k, int c) { return L.W[OW1 + k * POL_H + c]; });
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const T a = acc[e];
      L.H1[(I + Mma<T>::row(lane, e)) * HLD + J + (lane & 15)] = a > (T)0 ? a : (T)0;
    }
  }
  __syncthreads();
  for (int t = 0; t < 8; ++t) {
    const int I = (t >> 1) * 16, J = (t & 1) * 16;
    auto acc = tile_mma<T>(I, J, POL_H, [&](int r, int k) { return L.H1[r * HLD + k]; },
                           [&](int k, int c) { return L.W[OW2_R + k * POL_H + c]; });
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int col = J + (lane & 15);
      const T a = acc[e] + L.W[OB2_R + col];
      L.H2[(I + Mma<T>::row(lane, e)) * HLD + col] = a > (T)0 ? a : (T)0;
    }
  }
  __syncthreads();
}

template <typename T> __device__ inline T row_output(const RowLds<T> &L, int lane) {
  T o = L.W[OB3_R];
  for (int c = 0; c < POL_H; ++c) o += L.H2[lane * HLD + c] * L.W[OW3_R + c];
  return o;
}

template <typename T>
__device__ inline void load_rows(const View<T> &v, const T *__restrict__ theta, const PolRec *__restrict__ rec,
                                 const T *__restrict__ l_in, const T *__restrict__ s, const T *__restrict__ y,
                                 const T *__restrict__ rp, const T *__restrict__ s_prev,
                                 const T *__restrict__ st_prev, RowLds<T> &L, int64_t i, bool valid, T *xo) {
  for (int e = threadIdx.x; e < POL_RHO_PARAMS; e += 64 * POL_WAVES) L.W[e] = theta[e];
  for (int f = 0; f < 8; ++f) xo[f] = (T)0;
  if (valid) row_features<T>(v, theta, rec, l_in, s, y, rp, s_prev, st_prev, i, xo);
  const int lane = threadIdx.x & 63;
  for (int f = 0; f < 8; ++f) L.X[lane * 8 + f] = xo[f];
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(64 * POL_WAVES) void k_pol_rho_fwd(View<T> v, const T *__restrict__ theta,
                                                              const PolRec *__restrict__ rec,
                                                              const T *__restrict__ l_in, T *__restrict__ l_out,
                                                              T *__restrict__ rho_k, const T *__restrict__ s,
                                                              const T *__restrict__ y, const T *__restrict__ rp,
                                                              const T *__restrict__ s_prev,
                                                              const T *__restrict__ st_prev) {
  extern __shared__ __align__(16) unsigned char pol_lds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  RowLds<T> L = row_lds<T>(reinterpret_cast<T *>(pol_lds), wave);
  const int64_t i = ((int64_t)blockIdx.x * POL_WAVES + wave) * 64 + lane;
  const bool valid = i < v.m_tot;
  T xo[8];
  load_rows<T>(v, theta, rec, l_in, s, y, rp, s_prev, st_prev, L, i, valid, xo);
  rows_forward<T>(L, lane);
  if (valid) {
    const T l1 = xo[0] + row_output<T>(L, lane);
    l_out[i] = l1;
    const double sg = 1.0 / (1.0 + exp(-(double)l1));
    rho_k[i] = (T)exp(LOG_RHO_MIN + (LOG_RHO_MAX - LOG_RHO_MIN) * sg);
  }
}

// Reverse of the penalty network at one step.  C (in: cotangent of
// l^{k+1} from later steps; out: of l^k), grho_k: the unroll's cotangent of
// rho^k.  Writes the row features' cotangents: s and y added into gs, gy;
// rbar_p, the rbar_d-log feature, dp and dd into xb[0..3][m]; adds this
// workgroup's parameter gradient into part[blockIdx.x] (then, at k = 0, the
// cotangents of l^0 summed per cone kind).
template <typename T>
__global__ __launch_bounds__(64 * POL_WAVES) void k_pol_rho_bwd(
    View<T> v, const T *__restrict__ theta, const PolRec *__restrict__ rec, const T *__restrict__ l_in,
    const T *__restrict__ s, const T *__restrict__ y, const T *__restrict__ rp, const T *__restrict__ s_prev,
    const T *__restrict__ st_prev, const T *__restrict__ grho_k, T *__restrict__ C, T *__restrict__ gs,
    T *__restrict__ gy, T *__restrict__ xb, T *__restrict__ part) {
  extern __shared__ __align__(16) unsigned char pol_lds[];
  T *base = reinterpret_cast<T *>(pol_lds);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  RowLds<T> L = row_lds<T>(base, wave);
  const int64_t m = v.m_tot;
  const int64_t i = ((int64_t)blockIdx.x * POL_WAVES + wave) * 64 + lane;
  const bool valid = i < m;
  T xo[8];
  load_rows<T>(v, theta, rec, l_in, s, y, rp, s_prev, st_prev, L, i, valid, xo);
  rows_forward<T>(L, lane);
  T ob = 0;
  if (valid) {
    const T l1 = xo[0] + row_output<T>(L, lane);
    const double sg = 1.0 / (1.0 + exp(-(double)l1));
    const double rho = exp(LOG_RHO_MIN + (LOG_RHO_MAX - LOG_RHO_MIN) * sg);
    ob = (T)((double)C[i] + (double)grho_k[i] * rho * (LOG_RHO_MAX - LOG_RHO_MIN) * sg * (1.0 - sg));
  }
  L.OB[lane] = ob;
  __syncthreads();
  // w3-bar = OB' H2 (row 0 of the tile), b3-bar = sum OB
  typename Mma<T>::v4 g_w3[2], g_b2[2], g_w2[4], g_w1[2];
  for (int J = 0; J < 2; ++J)
    g_w3[J] = tile_mma<T>(0, 16 * J, 64, [&](int r, int k) { return r == 0 ? L.OB[k] : (T)0; },
                          [&](int k, int c) { return L.H2[k * HLD + c]; });
  const T g_b3 = (T)wave_sum((double)ob);
  // H2-bar in place
  for (int c = 0; c < POL_H; ++c) {
    const T h = L.H2[lane * HLD + c];
    L.H2[lane * HLD + c] = h > (T)0 ? ob * L.W[OW3_R + c] : (T)0;
  }
  __syncthreads();
  // W2-bar = H1' H2-bar, b2-bar = 1' H2-bar
  for (int t = 0; t < 4; ++t) {
    const int I = (t >> 1) * 16, J = (t & 1) * 16;
    g_w2[t] = tile_mma<T>(I, J, 64, [&](int r, int k) { return L.H1[k * HLD + r]; },
                          [&](int k, int c) { return L.H2[k * HLD + c]; });
  }
  for (int J = 0; J < 2; ++J)
    g_b2[J] = tile_mma<T>(0, 16 * J, 64, [&](int r, int k) { return r == 0 ? (T)1 : (T)0; },
                          [&](int k, int c) { return L.H2[k * HLD + c]; });
  __syncthreads();
  // H1-bar = (H2-bar W2') o [H1 > 0], in place: each tile reads only its own H1 entries
  for (int t = 0; t < 8; ++t) {
    const int I = (t >> 1) * 16, J = (t & 1) * 16;
    auto acc = tile_mma<T>(I, J, POL_H, [&](int r, int k) { return L.H2[r * HLD + k]; },
                           [&](int k, int c) { return L.W[OW2_R + c * POL_H + k]; });
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = (I + Mma<T>::row(lane, e)) * HLD + J + (lane & 15);
      L.H1[idx] = L.H1[idx] > (T)0 ? acc[e] : (T)0;
    }
  }
  __syncthreads();
  // W1'-bar = X' H1-bar (rows 0..6: W1, row 7: b1)
  for (int J = 0; J < 2; ++J)
    g_w1[J] = tile_mma<T>(0, 16 * J, 64, [&](int r, int k) { return r < 8 ? L.X[k * 8 + r] : (T)0; },
                          [&](int k, int c) { return L.H1[k * HLD + c]; });
  T cnew = 0;   // cotangent of l^k (at k = 0: of the per-kind initial logits)
  if (valid) {
    T xib[POL_FR];
    for (int f = 0; f < POL_FR; ++f) {
      T a = 0;
      for (int c = 0; c < POL_H; ++c) a += L.H1[lane * HLD + c] * L.W[OW1 + f * POL_H + c];
      xib[f] = a;
    }
    cnew = ob + xib[0];
    C[i] = cnew;
    gs[i] += xib[1];
    gy[i] += xib[2];
    xb[i] = xib[3];
    xb[m + i] = xib[4];
    xb[2 * m + i] = st_prev ? xib[5] : (T)0;
    xb[3 * m + i] = s_prev ? xib[6] : (T)0;
  }
  __syncthreads();
  // this wave's gradient, in the flat layout, into its H2 region (free now)
  T *stage = L.H2;
  for (int J = 0; J < 2; ++J) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = Mma<T>::row(lane, e), col = 16 * J + (lane & 15);
      if (row == 0) {
        stage[OW3_R + col] = g_w3[J][e];
        stage[OB2_R + col] = g_b2[J][e];
      }
      if (row < 8) stage[OW1 + row * POL_H + col] = g_w1[J][e];
    }
  }
  for (int t = 0; t < 4; ++t) {
    const int I = (t >> 1) * 16, J = (t & 1) * 16;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      stage[OW2_R + (I + Mma<T>::row(lane, e)) * POL_H + J + (lane & 15)] = g_w2[t][e];
  }
  if (lane == 0) stage[OB3_R] = g_b3;
  // at k = 0 (l^0 from theta) the rows' cotangents of l^0, summed per cone kind
  const int kind = valid ? (int)v.row_kind[i] : -1;
  for (int c = 0; c < 4; ++c) {
    const T ks = l_in ? (T)0 : (T)wave_sum(kind == c ? (double)cnew : 0.0);
    if (lane == 0) stage[POL_RHO_PARAMS + c] = ks;
  }
  __syncthreads();
  T *dst = part + (size_t)blockIdx.x * POL_PART_STRIDE;
  for (int e = threadIdx.x; e < POL_PART_STRIDE; e += 64 * POL_WAVES) {
    T a = 0;
    for (int w = 0; w < POL_WAVES; ++w) a += row_lds<T>(base, w).H2[e];
    dst[e] += a;
  }
}

// ---- per-instance reverse ----------------------------------------------------------

// One workgroup per instance: the relaxation network's reverse (with
// `policy`), the sums of the row features' cotangents that reach the
// instance's norms, and the coefficients with which the norms and the loss
// term (with `loss_term`) send cotangents to the residual vectors.
template <typename T>
__global__ __launch_bounds__(NTP) void k_pol_inst_bwd(View<T> v, const T *__restrict__ theta,
                                                      const PolRec *__restrict__ rec, int32_t k, int32_t policy,
                                                      int32_t loss_term, const T *__restrict__ la_in,
                                                      const T *__restrict__ galpha_k, T *__restrict__ Ca,
                                                      const T *__restrict__ xb, const T *__restrict__ rp,
                                                      const double *__restrict__ acc3, PolCoef *__restrict__ coef,
                                                      T *__restrict__ parta) {
  __shared__ double red[NTP / 64];
  __shared__ T h1[POL_H], h2[POL_H], h1b[POL_H], h2b[POL_H], xi_s[POL_FA];
  __shared__ double sc[8];
  const int b = blockIdx.x, t = threadIdx.x;
  const PolRec R = rec[b];
  const int64_t m = v.m_tot, r0 = v.m_off[b], r1 = v.m_off[b + 1];
  double s3 = 0, s4 = 0;
  if (policy && xb)
    for (int64_t i = r0 + t; i < r1; i += NTP) {
      s3 += (double)xb[i] * (double)rp[i];
      s4 += (double)xb[m + i];
    }
  const double S3 = blk_sum<NTP>(s3, red), S4 = blk_sum<NTP>(s4, red);
  if (policy) {
    const T *th = theta + POL_RHO_PARAMS;
    T xi[POL_FA];
    alpha_features<T>(R, la_in ? la_in[b] : theta[POL_L0 + 4], xi);
    if (t < POL_FA) xi_s[t] = xi[t];
    alpha_hidden<T>(th, xi, h1, h2);
    if (t == 0) {
      T o = th[OB3_A];
      for (int c = 0; c < POL_H; ++c) o += h2[c] * th[OW3_A + c];
      const double sg = 1.0 / (1.0 + exp(-(double)(xi[0] + o)));
      sc[0] = (double)Ca[b] + (double)galpha_k[b] * 2.0 * sg * (1.0 - sg);
    }
    __syncthreads();
    const T ob = (T)sc[0];
    if (t < POL_H) h2b[t] = h2[t] > (T)0 ? ob * th[OW3_A + t] : (T)0;
    __syncthreads();
    if (t < POL_H) {
      T a = 0;
      for (int c = 0; c < POL_H; ++c) a += th[OW2_A + t * POL_H + c] * h2b[c];
      h1b[t] = h1[t] > (T)0 ? a : (T)0;
    }
    __syncthreads();
    if (t < POL_FA) {
      T a = 0;
      for (int c = 0; c < POL_H; ++c) a += th[OW1 + t * POL_H + c] * h1b[c];
      sc[1 + t] = (double)a;
    }
    // parameter gradient of this instance, accumulated over the steps
    T *dst = parta + (size_t)b * POL_ALPHA_PARAMS;
    for (int e = t; e < POL_ALPHA_PARAMS; e += NTP) {
      T g;
      if (e < OB1_A) g = xi_s[e / POL_H] * h1b[e % POL_H];
      else if (e < OW2_A) g = h1b[e - OB1_A];
      else if (e < OB2_A) g = h1[(e - OW2_A) / POL_H] * h2b[(e - OW2_A) % POL_H];
      else if (e < OW3_A) g = h2b[e - OB2_A];
      else if (e < OB3_A) g = ob * h2[e - OW3_A];
      else g = ob;
      dst[e] += g;
    }
    __syncthreads();
  }
  if (t != 0) return;
  const double gpb = policy ? sc[2] : 0.0, gdb = (policy ? sc[3] : 0.0) + S4;
  const double gdpb = policy ? sc[4] : 0.0, gddb = policy ? sc[5] : 0.0;
  if (policy) Ca[b] = (T)(sc[0] + sc[1]);
  const double Np = norm_p(R), Nd = norm_d(R);
  PolCoef cf{};
  if (Np > 0) {
    const double rb = R.mrp / Np;
    cf.inv_np = 1.0 / Np;
    cf.c_rp = R.crp > 0 ? gpb / (rb + POL_EPS) / Np / R.crp : 0.0;
    const double nbar = -S3 / (Np * Np) - gpb / (rb + POL_EPS) * R.mrp / (Np * Np);
    const int nt = (R.nu == Np) + (R.ns == Np) + (R.nb == Np);
    cf.c_u = (R.nu == Np && R.cu > 0) ? nbar / nt / R.cu : 0.0;
    cf.c_s = (R.ns == Np && R.cs > 0) ? nbar / nt / R.cs : 0.0;
  }
  if (Nd > 0) {
    const double rb = R.mrd / Nd;
    cf.c_rd = R.crd > 0 ? gdb / (rb + POL_EPS) / Nd / R.crd : 0.0;
    const double nbar = -gdb / (rb + POL_EPS) * R.mrd / (Nd * Nd);
    const int nt = (R.np == Nd) + (R.nq == Nd) + (R.nw == Nd);
    cf.c_p = (R.np == Nd && R.cp > 0) ? nbar / nt / R.cp : 0.0;
    cf.c_w = (R.nw == Nd && R.cw > 0) ? nbar / nt / R.cw : 0.0;
  }
  if (policy && k >= 1) {
    cf.c_dp = R.cdp > 0 ? gdpb / (R.mdp + POL_EPS) / R.cdp : 0.0;
    cf.c_dd = R.cdd > 0 ? gddb / (R.mdd + POL_EPS) / R.cdd : 0.0;
  }
  if (loss_term) {
    const double *a = acc3 + 3 * (size_t)b;
    const double S = R.ssd / a[0] + R.ssp / a[1];
    cf.cl_d = 2.0 / (a[0] * S);
    cf.cl_p = 2.0 / (a[1] * S);
  }
  coef[b] = cf;
}

// Per row: the cotangents of r_p (features, norms, loss), u = A x (into ub)
// and s (added into gs), with dp and dd; pend_s (add_pend) is the cotangent
// of this iterate's s from the next step's dd feature; write_pend stores the
// cotangents of the previous step's s~ and of s^{k-1} for the next reverse
// step.
template <typename T>
__global__ __launch_bounds__(NTR) void k_pol_rows_bwd(View<T> v, const PolRec *__restrict__ rec,
                                                      const PolCoef *__restrict__ coef, const T *__restrict__ xb,
                                                      const T *__restrict__ rp, const T *__restrict__ u,
                                                      const T *__restrict__ s, const T *__restrict__ s_prev,
                                                      const T *__restrict__ st_prev, T *__restrict__ gs,
                                                      T *__restrict__ ub, T *__restrict__ pend_st,
                                                      T *__restrict__ pend_s, int32_t add_pend, int32_t write_pend) {
  const int64_t i = blockIdx.x * (int64_t)NTR + threadIdx.x;
  const int64_t m = v.m_tot;
  if (i >= m) return;
  const int b = v.row_inst[i];
  const PolRec R = rec[b];
  const PolCoef cf = coef[b];
  const double rpi = rp[i], ui = u[i], si = s[i];
  double cp = cf.cl_p * rpi;
  if (xb) cp += (double)xb[i] * cf.inv_np;
  if (fabs(rpi) == R.mrp) cp += cf.c_rp * sgn(rpi);
  const double cu = cp + (fabs(ui) == R.nu ? cf.c_u * sgn(ui) : 0.0);
  double cs = cp + (fabs(si) == R.ns ? cf.c_s * sgn(si) : 0.0);
  double dpb = 0, ddb = 0;
  if (st_prev) {
    const double d = si - (double)st_prev[i];
    dpb = (xb ? (double)xb[2 * m + i] : 0.0) + (fabs(d) == R.mdp ? cf.c_dp * sgn(d) : 0.0);
  }
  if (s_prev) {
    const double d = si - (double)s_prev[i];
    ddb = (xb ? (double)xb[3 * m + i] : 0.0) + (fabs(d) == R.mdd ? cf.c_dd * sgn(d) : 0.0);
  }
  cs += dpb + ddb;
  if (add_pend) cs += (double)pend_s[i];
  gs[i] = (T)((double)gs[i] + cs);
  ub[i] = (T)cu;
  if (write_pend) {
    pend_st[i] = (T)(-dpb);
    pend_s[i] = (T)(-ddb);
  }
}

// Per column: the cotangents of p = P x and w = A' y from r_d (norm and
// loss) and from the normaliser N_d.
template <typename T>
__global__ __launch_bounds__(NTR) void k_pol_cols_bwd(View<T> v, const PolRec *__restrict__ rec,
                                                      const PolCoef *__restrict__ coef, const T *__restrict__ rd,
                                                      const T *__restrict__ p, const T *__restrict__ w,
                                                      T *__restrict__ pb, T *__restrict__ wb) {
  const int64_t j = blockIdx.x * (int64_t)NTR + threadIdx.x;
  if (j >= v.n_tot) return;
  const int b = v.col_inst[j];
  const PolRec R = rec[b];
  const PolCoef cf = coef[b];
  const double dj = rd[j], pj = p[j], wj = w[j];
  const double cd = cf.cl_d * dj + (fabs(dj) == R.mrd ? cf.c_rd * sgn(dj) : 0.0);
  pb[j] = (T)(cd + (fabs(pj) == R.np ? cf.c_p * sgn(pj) : 0.0));
  wb[j] = (T)(-cd + (fabs(wj) == R.nw ? cf.c_w * sgn(wj) : 0.0));
}

// ---- gradient assembly --------------------------------------------------------------

// The parameter gradient: the penalty network's and the per-kind initial
// logits' from the workgroup partials, the relaxation network's from the
// instance partials, alpha's initial logit over the instances.  A workgroup
// takes 64 consecutive entries; its 16 waves each sum every 16th partial (a
// fixed split), then the 16 sums are added in wave order: deterministic.
constexpr int WS_E = 64, WS_G = 16;

template <typename T>
__global__ __launch_bounds__(WS_E * WS_G) void k_pol_wsum(const T *__restrict__ part, int64_t nblk,
                                                          const T *__restrict__ parta, const T *__restrict__ Ca,
                                                          int32_t B, T *__restrict__ gtheta) {
  __shared__ double red[WS_G][WS_E];
  const int el = threadIdx.x % WS_E, g = threadIdx.x / WS_E;
  const int e = blockIdx.x * WS_E + el;
  double a = 0;
  if (e < POL_PARAMS) {
    if (e < POL_RHO_PARAMS || (e >= POL_L0 && e < POL_L0 + 4)) {
      const int col = e < POL_RHO_PARAMS ? e : POL_RHO_PARAMS + (e - POL_L0);
      for (int64_t q = g; q < nblk; q += WS_G) a += (double)part[q * POL_PART_STRIDE + col];
    } else if (e < POL_L0) {
      for (int b = g; b < B; b += WS_G) a += (double)parta[(size_t)b * POL_ALPHA_PARAMS + (e - POL_RHO_PARAMS)];
    } else {
      for (int b = g; b < B; b += WS_G) a += (double)Ca[b];
    }
  }
  red[g][el] = a;
  __syncthreads();
  if (g == 0 && e < POL_PARAMS) {
    double t = 0;
    for (int w = 0; w < WS_G; ++w) t += red[w][el];
    gtheta[e] = (T)t;
  }
}

inline int grid_of(int64_t n, int nt) {
  const int64_t g = (n + nt - 1) / nt;
  return (int)(g < 1 ? 1 : g);
}

template <typename K> void allow_row_lds(K kern, size_t bytes) {
  static bool done = false;   // one attribute call per kernel instantiation
  if (!done && bytes > 65536) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
  }
  done = true;
}

}  // namespace

int64_t pol_row_blocks(int64_t m) { return (m + 64 * POL_WAVES - 1) / (64 * POL_WAVES); }

template <typename T>
void launch_pol_norms(const View<T> &v, const T *u, const T *rp, const T *p, const T *w, const T *rd, const T *s,
                      const T *s_prev, const T *st_prev, PolRec *rec, hipStream_t st) {
  k_pol_norms<T><<<v.B, NTN, 0, st>>>(v, u, rp, p, w, rd, s, s_prev, st_prev, rec);
}

template <typename T>
void launch_pol_inst_fwd(const View<T> &v, const T *theta, const PolRec *rec, int32_t k, int32_t policy,
                         const T *la_in, T *la_out, T *alpha_k, double *acc3, T *loss, hipStream_t st) {
  k_pol_inst_fwd<T><<<v.B, 64, 0, st>>>(v, theta, rec, k, policy, la_in, la_out, alpha_k, acc3, loss);
}

template <typename T>
void launch_pol_rho_fwd(const View<T> &v, const T *theta, const PolRec *rec, const T *l_in, T *l_out, T *rho_k,
                        const T *s, const T *y, const T *rp, const T *s_prev, const T *st_prev, hipStream_t st) {
  const size_t lds = row_lds_bytes<T>();
  allow_row_lds(k_pol_rho_fwd<T>, lds);
  k_pol_rho_fwd<T><<<(int)pol_row_blocks(v.m_tot), 64 * POL_WAVES, lds, st>>>(v, theta, rec, l_in, l_out, rho_k, s,
                                                                              y, rp, s_prev, st_prev);
}

template <typename T>
void launch_pol_rho_bwd(const View<T> &v, const T *theta, const PolRec *rec, const T *l_in, const T *s, const T *y,
                        const T *rp, const T *s_prev, const T *st_prev, const T *grho_k, T *C, T *gs, T *gy, T *xb,
                        T *part, hipStream_t st) {
  const size_t lds = row_lds_bytes<T>();
  allow_row_lds(k_pol_rho_bwd<T>, lds);
  k_pol_rho_bwd<T><<<(int)pol_row_blocks(v.m_tot), 64 * POL_WAVES, lds, st>>>(v, theta, rec, l_in, s, y, rp, s_prev,
                                                                              st_prev, grho_k, C, gs, gy, xb, part);
}

template <typename T>
void launch_pol_inst_bwd(const View<T> &v, const T *theta, const PolRec *rec, int32_t k, int32_t policy,
                         int32_t loss_term, const T *la_in, const T *galpha_k, T *Ca, const T *xb, const T *rp,
                         const double *acc3, PolCoef *coef, T *parta, hipStream_t st) {
  k_pol_inst_bwd<T><<<v.B, NTP, 0, st>>>(v, theta, rec, k, policy, loss_term, la_in, galpha_k, Ca, xb, rp, acc3, coef,
                                         parta);
}

template <typename T>
void launch_pol_rows_bwd(const View<T> &v, const PolRec *rec, const PolCoef *coef, const T *xb, const T *rp,
                         const T *u, const T *s, const T *s_prev, const T *st_prev, T *gs, T *ub, T *pend_st,
                         T *pend_s, int32_t add_pend, int32_t write_pend, hipStream_t st) {
  k_pol_rows_bwd<T><<<grid_of(v.m_tot, NTR), NTR, 0, st>>>(v, rec, coef, xb, rp, u, s, s_prev, st_prev, gs, ub,
                                                           pend_st, pend_s, add_pend, write_pend);
}

template <typename T>
void launch_pol_cols_bwd(const View<T> &v, const PolRec *rec, const PolCoef *coef, const T *rd, const T *p, const T *w,
                         T *pb, T *wb, hipStream_t st) {
  k_pol_cols_bwd<T><<<grid_of(v.n_tot, NTR), NTR, 0, st>>>(v, rec, coef, rd, p, w, pb, wb);
}

template <typename T>
void launch_pol_grad(const View<T> &v, const T *part, int64_t nblk, const T *parta, const T *Ca, T *gtheta,
                     hipStream_t st) {
  k_pol_wsum<T><<<grid_of(POL_PARAMS, WS_E), WS_E * WS_G, 0, st>>>(part, nblk, parta, Ca, v.B, gtheta);
}

#define POL_INST(T)                                                                                               \
  template void launch_pol_norms<T>(const View<T> &, const T *, const T *, const T *, const T *, const T *,       \
                                    const T *, const T *, const T *, PolRec *, hipStream_t);                      \
  template void launch_pol_inst_fwd<T>(const View<T> &, const T *, const PolRec *, int32_t, int32_t, const T *,  \
                                       T *, T *, double *, T *, hipStream_t);                                     \
  template void launch_pol_rho_fwd<T>(const View<T> &, const T *, const PolRec *, const T *, T *, T *, const T *, \
                                      const T *, const T *, const T *, const T *, hipStream_t);                   \
  template void launch_pol_rho_bwd<T>(const View<T> &, const T *, const PolRec *, const T *, const T *, const T *, \
                                      const T *, const T *, const T *, const T *, T *, T *, T *, T *, T *,        \
                                      hipStream_t);                                                               \
  template void launch_pol_inst_bwd<T>(const View<T> &, const T *, const PolRec *, int32_t, int32_t, int32_t,    \
                                       const T *, const T *, T *, const T *, const T *, const double *,           \
                                       PolCoef *, T *, hipStream_t);                                              \
  template void launch_pol_rows_bwd<T>(const View<T> &, const PolRec *, const PolCoef *, const T *, const T *,   \
                                       const T *, const T *, const T *, const T *, T *, T *, T *, T *, int32_t,   \
                                       int32_t, hipStream_t);                                                     \
  template void launch_pol_cols_bwd<T>(const View<T> &, const PolRec *, const PolCoef *, const T *, const T *,   \
                                       const T *, T *, T *, hipStream_t);                                         \
  template void launch_pol_grad<T>(const View<T> &, const T *, int64_t, const T *, const T *, T *, hipStream_t);

POL_INST(float)
POL_INST(double)

}  // namespace cosmo
