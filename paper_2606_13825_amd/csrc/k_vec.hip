// Row- and column-wise kernels of the unrolled COSMO step: the right-hand
// side and Jacobi diagonal of the reduced system, the slack / relaxation /
// projection-onto-separable-cones pass, the reverse of those passes, penalty
// rectification and its adjoint, per-instance reductions and the residual
// loss.  All sparse products use coalesced sub-wave CSR: L consecutive lanes
// serve one row and combine their partial sums with a fixed butterfly, so
// every result is bitwise reproducible.
#include "cosmo_internal.h"

namespace cosmo {
namespace {

constexpr int NT = 256;

template <typename T> __device__ inline T subwave_sum(T v, int L) {
  for (int off = L >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Row and column sums, and the differences they feed (s~ - s, xi, the
// gradient terms), are formed in float64 from the stored values and rounded
// once: near a fixed point these differences are small against their terms,
// and float32 accumulation would leave errors of order eps |terms| in them.
// s^ and v are evaluated by this one function in the forward and the reverse
// pass, so the nonnegative-cone mask is the same in both.
template <typename T> __device__ inline double shat_of(T al, T stl, T s) {
  return (double)al * (double)stl + (1.0 - (double)al) * (double)s;
}
template <typename T> __device__ inline double v_of(T al, T stl, T s, T y, T r) {
  return shat_of(al, stl, s) + (double)y / (double)r;
}

// Contributions of the dense sub-blocks of A (computed beforehand by the
// dense product kernels into the call's float64 scratch): row i's entry of
// the row product (times its placement's scale) and column j's entries of
// the column products.
template <typename T> __device__ inline double dense_row_term(const View<T> &v, int64_t i) {
  if (!v.drow) return 0.0;
  const int32_t r = v.drow[i];
  return r >= 0 ? v.dscale[i] * v.dn[r] : 0.0;
}
template <typename T> __device__ inline void dense_col_terms(const View<T> &v, int64_t j, double &e, double &d) {
  e = d = 0.0;
  if (!v.dcol) return;
  const int32_t c = v.dcol[j];
  if (c >= 0) {
    e = v.ec[c];
    if (v.ed) d = v.ed[c];
  }
}

// Position of this thread inside the bucketed row list: returns false when
// the sub-wave has no row.  All lanes of a sub-wave agree.
struct BucketPos {
  int64_t row;
  int lane;
  int L;
};

__device__ inline bool bucket_pos(const int32_t *rows, const int64_t *begin, const int32_t *lanes,
                                  const int32_t *blk_start, BucketPos &bp) {
  const int b = blockIdx.x;
  const int c = (b < blk_start[1]) ? 0 : ((b < blk_start[2]) ? 1 : 2);
  const int L = lanes[c];
  const int per_block = NT / L;
  const int64_t idx = begin[c] + (int64_t)(b - blk_start[c]) * per_block + threadIdx.x / L;
  bp.lane = threadIdx.x % L;
  bp.L = L;
  if (idx >= begin[c + 1]) return false;
  bp.row = rows[idx];
  return true;
}

struct BucketArgs {
  const int32_t *rows;
  int64_t begin[4];
  int32_t lanes[3];
  int32_t blk_start[4];
};

BucketArgs make_bucket_args(const RowBuckets &bk) {
  BucketArgs a;
  a.rows = bk.d_rows;
  int64_t nb = 0;
  for (int c = 0; c < 3; ++c) {
    a.begin[c] = bk.begin[c];
    a.lanes[c] = bk.lanes[c];
    a.blk_start[c] = (int32_t)nb;
    const int64_t cnt = bk.begin[c + 1] - bk.begin[c];
    const int per = NT / bk.lanes[c];
    nb += (cnt + per - 1) / per;
  }
  a.begin[3] = bk.begin[3];
  a.blk_start[3] = (int32_t)nb;
  return a;
}

#define BUCKET_PREAMBLE                                                                        \
  BucketPos bp;                                                                                \
  if (!bucket_pos(ba.rows, ba.begin, ba.lanes, ba.blk_start, bp)) return;

// ---- rectification -----------------------------------------------------------

template <typename T>
__global__ void k_copy(T *__restrict__ dst, const T *__restrict__ src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) dst[i] = src[i];
}

template <typename T> __global__ void k_fill(T *__restrict__ dst, T val, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) dst[i] = val;
}

// One workgroup per (step, block): the block mean of `src` written to every
// row of the block in `dst` (rectification and its adjoint are the same map).
// Each thread keeps four loads in flight.
template <typename T> __device__ inline T block_sum(T v, T *red);

template <typename T>
__global__ __launch_bounds__(NT) void k_block_mean(const RectDesc *__restrict__ rect, int32_t nrect,
                                                   const T *__restrict__ src, T *__restrict__ dst, int64_t stride) {
  __shared__ T red[NT / 64];
  const int k = (int)(blockIdx.x / nrect);
  const RectDesc d = rect[blockIdx.x % nrect];
  const T *sp = src + k * stride + d.row0;
  T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int i = threadIdx.x;
  for (; i + 3 * NT < d.rows; i += 4 * NT) {
    a0 += sp[i];
    a1 += sp[i + NT];
    a2 += sp[i + 2 * NT];
    a3 += sp[i + 3 * NT];
  }
  for (; i < d.rows; i += NT) a0 += sp[i];
  const T mean = block_sum((a0 + a1) + (a2 + a3), red) / (T)d.rows;
  T *o = dst + k * stride + d.row0;
  for (int j = threadIdx.x; j < d.rows; j += NT) o[j] = mean;
}

// ---- forward ----------------------------------------------------------------

// Per column j of A (row j of A'):
//   dg[j] = P_jj + sigma + sum_i rho_hat_i A_ij^2        (Jacobi preconditioner)
//   xi[j] = sigma x_j - q_j + sum_i A_ij (y_i + rho_hat_i (b_i - s_i))
// With a diagonal M (every row of A has at most one nonzero and P is
// diagonal) the Jacobi-PCG solution is x~ = xi / dg exactly; `ds` then
// carries the outputs and the solve is finished here.
template <typename T>
__global__ __launch_bounds__(NT) void k_cols_pre(View<T> v, BucketArgs ba, const T *__restrict__ rho_hat,
                                                 const T *__restrict__ x, const T *__restrict__ s,
                                                 const T *__restrict__ y, T *__restrict__ dg,
                                                 double *__restrict__ xi, DiagSolve<T> ds) {
  BUCKET_PREAMBLE
  const int64_t j = bp.row;
  double a_xi = 0, a_d = 0;
  for (int64_t k = v.At_rowptr[j] + bp.lane; k < v.At_rowptr[j + 1]; k += bp.L) {
    const int32_t i = v.At_col[k];
    const double a = v.At_val[k];
    const double r = rho_hat[i];
    a_xi += a * ((double)y[i] + r * ((double)v.b[i] - (double)s[i]));
    a_d += r * a * a;
  }
  a_xi = subwave_sum(a_xi, bp.L);
  a_d = subwave_sum(a_d, bp.L);
  if (bp.lane == 0) {
    double e_xi, e_d;
    dense_col_terms(v, j, e_xi, e_d);
    a_xi += e_xi;
    a_d += e_d;
    const T d = (T)((double)v.Pdiag[j] + (double)v.sigma + a_d);
    const double r = (double)v.sigma * (double)x[j] - (double)v.q[j] + a_xi;
    dg[j] = d;
    xi[j] = r;   // kept in float64: the solve's right-hand side is not rounded
    if (ds.xt) {
      const T xt = (T)(r / (double)d);
      const T al = ds.alpha_k[v.col_inst[j]];
      ds.xt[j] = xt;
      ds.xn[j] = al * xt + ((T)1 - al) * x[j];
    }
  }
}

// Per row i: s~ = b - A x~;  s^ = alpha s~ + (1 - alpha) s;  v = s^ + y / rho_hat.
// Zero rows: s+ = 0.  Nonneg rows: s+ = max(v, 0).  Both: y+ = y + rho_hat (s^ - s+).
// SOC / PSD rows leave s^ and v for the cone kernels.
template <typename T>
__global__ __launch_bounds__(NT) void k_rows_post(View<T> v, BucketArgs ba, const T *__restrict__ rho_hat,
                                                  const T *__restrict__ alpha_k, const T *__restrict__ xt,
                                                  const T *__restrict__ s, const T *__restrict__ y,
                                                  T *__restrict__ st_out, T *__restrict__ sh_out,
                                                  T *__restrict__ vv_out, T *__restrict__ s_new,
                                                  T *__restrict__ y_new) {
  BUCKET_PREAMBLE
  const int64_t i = bp.row;
  double ax = 0;
  for (int64_t k = v.A_rowptr[i] + bp.lane; k < v.A_rowptr[i + 1]; k += bp.L)
    ax += (double)v.A_val[k] * (double)xt[v.A_col[k]];
  ax = subwave_sum(ax, bp.L);
  if (bp.lane != 0) return;
  ax += dense_row_term(v, i);
  const T al = alpha_k[v.row_inst[i]];
  const T r = rho_hat[i];
  const T stl = (T)((double)v.b[i] - ax);   // stored; s^ and v below use the stored value
  const double shat = shat_of(al, stl, s[i]);
  const double vi = v_of(al, stl, s[i], y[i], r);
  st_out[i] = stl;
  const uint8_t kind = v.row_kind[i];
  if (kind == ROW_ZERO || kind == ROW_NONNEG) {
    const T sp = (kind == ROW_ZERO) ? (T)0 : (vi < 0.0 ? (T)0 : (T)vi);   // NaN passes through
    s_new[i] = sp;
    y_new[i] = (T)((double)y[i] + (double)r * (shat - (double)sp));
  } else {
    sh_out[i] = (T)shat;
    vv_out[i] = (T)vi;
  }
}

// ---- backward ---------------------------------------------------------------

// Per row: the cotangent reaching s+ after the y-update, gsn = gs+ - rho_hat gy+;
// separable cones apply their Jacobian (zero: 0, nonneg: mask v > 0).  gsn is
// written on SOC and PSD rows, on every row when all_rows is set.
template <typename T>
__global__ __launch_bounds__(NT) void k_bwd_rows_a(View<T> v, const T *__restrict__ rho_hat,
                                                   const T *__restrict__ alpha_k, const T *__restrict__ stl,
                                                   const T *__restrict__ s, const T *__restrict__ y,
                                                   const T *__restrict__ gs_in, const T *__restrict__ gy_in,
                                                   T *__restrict__ gsn, T *__restrict__ gv, int all_rows) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i >= v.m_tot) return;
  const T r = rho_hat[i];
  const T g = (T)((double)gs_in[i] - (double)r * (double)gy_in[i]);
  const uint8_t kind = v.row_kind[i];
  if (kind == ROW_ZERO) {
    gv[i] = 0;
  } else if (kind == ROW_NONNEG) {
    const double vi = v_of(alpha_k[v.row_inst[i]], stl[i], s[i], y[i], r);
    gv[i] = vi > 0.0 ? g : (T)0;
  }
  if (all_rows || (kind != ROW_ZERO && kind != ROW_NONNEG)) gsn[i] = g;
}

// v = s^ + y / rho_hat on every row (recomputed from the tape in the reverse pass).
template <typename T>
__global__ __launch_bounds__(NT) void k_rows_v(View<T> v, const T *__restrict__ rho_hat,
                                               const T *__restrict__ alpha_k, const T *__restrict__ stl,
                                               const T *__restrict__ s, const T *__restrict__ y,
                                               T *__restrict__ vv) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i >= v.m_tot) return;
  vv[i] = (T)v_of(alpha_k[v.row_inst[i]], stl[i], s[i], y[i], rho_hat[i]);
}

// Per row, once every cone has produced v-bar:
//   gs^ = rho_hat gy+ + gv;  gy = gy+ + gv / rho_hat;
//   grh = gy+ (s^ - s+) - gv y / rho_hat^2;  gs~ = alpha gs^ (+ gst_extra, a
//   cotangent of s~ from outside the step);  gs = (1 - alpha) gs^.
template <typename T>
__global__ __launch_bounds__(NT) void k_bwd_rows_b(View<T> v, const T *__restrict__ rho_hat,
                                                   const T *__restrict__ alpha_k, const T *__restrict__ stl,
                                                   const T *__restrict__ s, const T *__restrict__ y,
                                                   const T *__restrict__ s_new, const T *__restrict__ gy_in,
                                                   const T *__restrict__ gv, T *__restrict__ gsh,
                                                   T *__restrict__ gst, T *__restrict__ gs_out,
                                                   T *__restrict__ gy_out, T *__restrict__ grh,
                                                   const T *__restrict__ gst_extra) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i >= v.m_tot) return;
  const double r = rho_hat[i];
  const T al = alpha_k[v.row_inst[i]];
  const double shat = shat_of(al, stl[i], s[i]);
  const double gyp = gy_in[i];
  const double g_v = gv[i];
  const double g_sh = r * gyp + g_v;
  gsh[i] = (T)g_sh;
  gy_out[i] = (T)(gyp + g_v / r);
  grh[i] = (T)(gyp * (shat - (double)s_new[i]) - g_v * (double)y[i] / (r * r));
  gst[i] = (T)((double)al * g_sh + (gst_extra ? (double)gst_extra[i] : 0.0));
  gs_out[i] = (T)((1.0 - (double)al) * g_sh);
}

// Per column j: xt-bar = alpha gx+ - (A' gs~)_j ; also the Jacobi diagonal.
// With a diagonal M the adjoint solve is w = xt-bar / dg (see k_cols_pre);
// then w and gx = (1 - alpha) gx+ + sigma w are written here.
template <typename T>
__global__ __launch_bounds__(NT) void k_bwd_cols(View<T> v, BucketArgs ba, const T *__restrict__ rho_hat,
                                                 const T *__restrict__ alpha_k, const T *__restrict__ gst,
                                                 const T *__restrict__ gx_in, double *__restrict__ gxt,
                                                 T *__restrict__ dg, DiagSolve<T> ds) {
  BUCKET_PREAMBLE
  const int64_t j = bp.row;
  double acc = 0, a_d = 0;
  for (int64_t k = v.At_rowptr[j] + bp.lane; k < v.At_rowptr[j + 1]; k += bp.L) {
    const int32_t i = v.At_col[k];
    const double a = v.At_val[k];
    acc += a * (double)gst[i];
    a_d += (double)rho_hat[i] * a * a;
  }
  acc = subwave_sum(acc, bp.L);
  a_d = subwave_sum(a_d, bp.L);
  if (bp.lane == 0) {
    double e_g, e_d;
    dense_col_terms(v, j, e_g, e_d);
    acc += e_g;
    a_d += e_d;
    const T al = alpha_k[v.col_inst[j]];
    const double r = (double)al * (double)gx_in[j] - acc;
    const T d = (T)((double)v.Pdiag[j] + (double)v.sigma + a_d);
    gxt[j] = r;
    dg[j] = d;
    if (ds.xt) {
      const T w = (T)(r / (double)d);
      ds.xt[j] = w;
      ds.xn[j] = ((T)1 - al) * gx_in[j] + v.sigma * w;
    }
  }
}

// Per row, with w solving M w = xt-bar and g = A w:
//   grh += g (s~ - s)   [matrix term -(A w)(A x~) plus right-hand-side term g (b - s)]
//   gy += g ;  gs -= rho_hat g
template <typename T>
__global__ __launch_bounds__(NT) void k_bwd_rows_c(View<T> v, BucketArgs ba, const T *__restrict__ rho_hat,
                                                   const T *__restrict__ w, const T *__restrict__ stl,
                                                   const T *__restrict__ s, T *__restrict__ grh,
                                                   T *__restrict__ gs_out, T *__restrict__ gy_out) {
  BUCKET_PREAMBLE
  const int64_t i = bp.row;
  double g = 0;
  for (int64_t k = v.A_rowptr[i] + bp.lane; k < v.A_rowptr[i + 1]; k += bp.L)
    g += (double)v.A_val[k] * (double)w[v.A_col[k]];
  g = subwave_sum(g, bp.L);
  if (bp.lane != 0) return;
  g += dense_row_term(v, i);
  grh[i] = (T)((double)grh[i] + g * ((double)stl[i] - (double)s[i]));
  gy_out[i] = (T)((double)gy_out[i] + g);
  gs_out[i] = (T)((double)gs_out[i] - (double)rho_hat[i] * g);
}

// Workgroup reduction with a fixed tree: deterministic.
template <typename T> __device__ inline T block_sum(T v, T *red) {
  v = subwave_sum(v, 64);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  T tot = 0;
  for (int w = 0; w < NT / 64; ++w) tot += red[w];
  return tot;
}

// One workgroup per instance: alpha-bar = gs^'(s~ - s) + gx+'(x~ - x).
template <typename T>
__global__ __launch_bounds__(NT) void k_alpha_reduce(View<T> v, const T *__restrict__ gsh,
                                                     const T *__restrict__ stl, const T *__restrict__ s,
                                                     const T *__restrict__ gx_in, const T *__restrict__ xt,
                                                     const T *__restrict__ x, T *__restrict__ galpha_k) {
  __shared__ double red[NT / 64];
  const int b = blockIdx.x;
  double a0 = 0, a1 = 0;
  auto term = [](T g, T u, T w) { return (double)g * ((double)u - (double)w); };
  const int64_t m1 = v.m_off[b + 1], n1 = v.n_off[b + 1];
  int64_t i = v.m_off[b] + threadIdx.x;
  for (; i + NT < m1; i += 2 * NT) {
    a0 += term(gsh[i], stl[i], s[i]);
    a1 += term(gsh[i + NT], stl[i + NT], s[i + NT]);
  }
  for (; i < m1; i += NT) a0 += term(gsh[i], stl[i], s[i]);
  int64_t j = v.n_off[b] + threadIdx.x;
  for (; j + NT < n1; j += 2 * NT) {
    a0 += term(gx_in[j], xt[j], x[j]);
    a1 += term(gx_in[j + NT], xt[j + NT], x[j + NT]);
  }
  for (; j < n1; j += NT) a0 += term(gx_in[j], xt[j], x[j]);
  const double tot = block_sum(a0 + a1, red);
  if (threadIdx.x == 0) galpha_k[b] = (T)tot;
}

// ---- residual loss ------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(NT) void k_loss_rp(View<T> v, BucketArgs ba, const T *__restrict__ x,
                                                const T *__restrict__ s, T *__restrict__ rp) {
  BUCKET_PREAMBLE
  const int64_t i = bp.row;
  double ax = 0;
  for (int64_t k = v.A_rowptr[i] + bp.lane; k < v.A_rowptr[i + 1]; k += bp.L)
    ax += (double)v.A_val[k] * (double)x[v.A_col[k]];
  ax = subwave_sum(ax, bp.L);
  if (bp.lane == 0) rp[i] = (T)(ax + dense_row_term(v, i) + (double)s[i] - (double)v.b[i]);
}

// rd_j = (P x)_j + q_j - (A' y)_j
template <typename T>
__global__ __launch_bounds__(NT) void k_loss_rd(View<T> v, BucketArgs ba, const T *__restrict__ x,
                                                const T *__restrict__ y, T *__restrict__ rd) {
  BUCKET_PREAMBLE
  const int64_t j = bp.row;
  double acc = 0;
  for (int64_t k = v.At_rowptr[j] + bp.lane; k < v.At_rowptr[j + 1]; k += bp.L)
    acc -= (double)v.At_val[k] * (double)y[v.At_col[k]];
  if (v.P_rowptr)
    for (int64_t k = v.P_rowptr[j] + bp.lane; k < v.P_rowptr[j + 1]; k += bp.L)
      acc += (double)v.P_val[k] * (double)x[v.P_col[k]];
  acc = subwave_sum(acc, bp.L);
  if (bp.lane == 0) {
    double e, d;
    dense_col_terms(v, j, e, d);
    rd[j] = (T)(acc - e + (double)v.q[j]);
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_loss_reduce(View<T> v, const T *__restrict__ rp, const T *__restrict__ rd,
                                                    T *__restrict__ loss) {
  __shared__ double red[NT / 64];
  const int b = blockIdx.x;
  double acc = 0;
  for (int64_t i = v.m_off[b] + threadIdx.x; i < v.m_off[b + 1]; i += NT) acc += (double)rp[i] * (double)rp[i];
  for (int64_t j = v.n_off[b] + threadIdx.x; j < v.n_off[b + 1]; j += NT) acc += (double)rd[j] * (double)rd[j];
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) loss[b] = (T)tot;
}

// gx_j = 2 (A' rp)_j + 2 (P rd)_j
template <typename T>
__global__ __launch_bounds__(NT) void k_loss_gx(View<T> v, BucketArgs ba, const T *__restrict__ rp,
                                                const T *__restrict__ rd, T *__restrict__ gx) {
  BUCKET_PREAMBLE
  const int64_t j = bp.row;
  T acc = 0;
  for (int64_t k = v.At_rowptr[j] + bp.lane; k < v.At_rowptr[j + 1]; k += bp.L) acc += v.At_val[k] * rp[v.At_col[k]];
  if (v.P_rowptr)
    for (int64_t k = v.P_rowptr[j] + bp.lane; k < v.P_rowptr[j + 1]; k += bp.L) acc += v.P_val[k] * rd[v.P_col[k]];
  acc = subwave_sum(acc, bp.L);
  if (bp.lane == 0) {
    double e, d;
    dense_col_terms(v, j, e, d);
    gx[j] = (T)2 * (acc + (T)e);
  }
}

// gs_i = 2 rp_i ; gy_i = -2 (A rd)_i
template <typename T>
__global__ __launch_bounds__(NT) void k_loss_gsy(View<T> v, BucketArgs ba, const T *__restrict__ rp,
                                                 const T *__restrict__ rd, T *__restrict__ gs,
                                                 T *__restrict__ gy) {
  BUCKET_PREAMBLE
  const int64_t i = bp.row;
  T acc = 0;
  for (int64_t k = v.A_rowptr[i] + bp.lane; k < v.A_rowptr[i + 1]; k += bp.L) acc += v.A_val[k] * rd[v.A_col[k]];
  acc = subwave_sum(acc, bp.L);
  if (bp.lane == 0) {
    acc += (T)dense_row_term(v, i);
    if (gs) gs[i] = (T)2 * rp[i];
    if (gy) gy[i] = (T)-2 * acc;
  }
}

// ---- learned policy: KKT residual vectors and their adjoint (App. E) ---------

// u = A x and rp = u + s - b on every row.
template <typename T>
__global__ __launch_bounds__(NT) void k_pol_rows(View<T> v, BucketArgs ba, const T *__restrict__ x,
                                                 const T *__restrict__ s, T *__restrict__ u, T *__restrict__ rp) {
  BUCKET_PREAMBLE
  const int64_t i = bp.row;
  double ax = 0;
  for (int64_t k = v.A_rowptr[i] + bp.lane; k < v.A_rowptr[i + 1]; k += bp.L)
    ax += (double)v.A_val[k] * (double)x[v.A_col[k]];
  ax = subwave_sum(ax, bp.L);
  if (bp.lane == 0) {
    ax += dense_row_term(v, i);
    u[i] = (T)ax;
    rp[i] = (T)(ax + (double)s[i] - (double)v.b[i]);
  }
}

// p = P x, w = A' y and rd = p + q - w on every column.
template <typename T>
__global__ __launch_bounds__(NT) void k_pol_cols(View<T> v, BucketArgs ba, const T *__restrict__ x,
                                                 const T *__restrict__ y, T *__restrict__ p, T *__restrict__ w,
                                                 T *__restrict__ rd) {
  BUCKET_PREAMBLE
  const int64_t j = bp.row;
  double aw = 0, ap = 0;
  for (int64_t k = v.At_rowptr[j] + bp.lane; k < v.At_rowptr[j + 1]; k += bp.L)
    aw += (double)v.At_val[k] * (double)y[v.At_col[k]];
  if (v.P_rowptr)
    for (int64_t k = v.P_rowptr[j] + bp.lane; k < v.P_rowptr[j + 1]; k += bp.L)
      ap += (double)v.P_val[k] * (double)x[v.P_col[k]];
  aw = subwave_sum(aw, bp.L);
  ap = subwave_sum(ap, bp.L);
  if (bp.lane == 0) {
    double e, d;
    dense_col_terms(v, j, e, d);
    aw += e;
    p[j] = (T)ap;
    w[j] = (T)aw;
    rd[j] = (T)(ap + (double)v.q[j] - aw);
  }
}

// gx_j += (A' ub)_j + (P pb)_j  (P symmetric)
template <typename T>
__global__ __launch_bounds__(NT) void k_pol_adj_cols(View<T> v, BucketArgs ba, const T *__restrict__ ub,
                                                     const T *__restrict__ pb, T *__restrict__ gx) {
  BUCKET_PREAMBLE
  const int64_t j = bp.row;
  double acc = 0;
  for (int64_t k = v.At_rowptr[j] + bp.lane; k < v.At_rowptr[j + 1]; k += bp.L)
    acc += (double)v.At_val[k] * (double)ub[v.At_col[k]];
  if (v.P_rowptr)
    for (int64_t k = v.P_rowptr[j] + bp.lane; k < v.P_rowptr[j + 1]; k += bp.L)
      acc += (double)v.P_val[k] * (double)pb[v.P_col[k]];
  acc = subwave_sum(acc, bp.L);
  if (bp.lane == 0) {
    double e, d;
    dense_col_terms(v, j, e, d);
    gx[j] = (T)((double)gx[j] + acc + e);
  }
}

// gy_i += (A wb)_i
template <typename T>
__global__ __launch_bounds__(NT) void k_pol_adj_rows(View<T> v, BucketArgs ba, const T *__restrict__ wb,
                                                     T *__restrict__ gy) {
  BUCKET_PREAMBLE
  const int64_t i = bp.row;
  double acc = 0;
  for (int64_t k = v.A_rowptr[i] + bp.lane; k < v.A_rowptr[i + 1]; k += bp.L)
    acc += (double)v.A_val[k] * (double)wb[v.A_col[k]];
  acc = subwave_sum(acc, bp.L);
  if (bp.lane == 0) gy[i] = (T)((double)gy[i] + acc + dense_row_term(v, i));
}

// ---- vanilla solve: per-row penalties from per-instance scalars ---------------

// rho[k][i] = rho_b[instance of i] (times eq_scale on zero-cone rows), k < K.
template <typename T>
__global__ __launch_bounds__(NT) void k_solve_rho(View<T> v, const double *__restrict__ rho_b, double eq_scale,
                                                  T *__restrict__ rho, int32_t K) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i >= v.m_tot) return;
  const T r = (T)(rho_b[v.row_inst[i]] * (v.row_kind[i] == ROW_ZERO ? eq_scale : 1.0));
  for (int32_t k = 0; k < K; ++k) rho[(int64_t)k * v.m_tot + i] = r;
}

// ---- health check ---------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(NT) void k_nonfinite(View<T> v, const T *__restrict__ x, const T *__restrict__ s,
                                                  const T *__restrict__ y, cosmo_stats *stats) {
  const int b = blockIdx.x;
  int bad = 0;
  for (int64_t i = v.m_off[b] + threadIdx.x; i < v.m_off[b + 1]; i += NT)
    bad |= !(isfinite(s[i]) && isfinite(y[i]));
  for (int64_t j = v.n_off[b] + threadIdx.x; j < v.n_off[b + 1]; j += NT) bad |= !isfinite(x[j]);
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0 && bad) atomicOr(&stats[b].nonfinite, 1);
}

int64_t nblocks_bucket(const BucketArgs &a) { return a.blk_start[3]; }

inline int grid_for(int64_t n) {
  int64_t g = (n + NT - 1) / NT;
  if (g < 1) g = 1;
  if (g > 65535 * 16) g = 65535 * 16;
  return (int)g;
}

}  // namespace

template <typename T>
void launch_rectify(const View<T> &v, const RectDesc *rect, int32_t nrect, const T *rho, T *rho_hat, int32_t K,
                    hipStream_t st) {
  const int64_t tot = (int64_t)K * v.m_tot;
  k_copy<T><<<grid_for(tot), NT, 0, st>>>(rho_hat, rho, tot);
  if (nrect > 0) {
    const int64_t jobs = (int64_t)nrect * K;
    k_block_mean<T><<<(int)jobs, NT, 0, st>>>(rect, nrect, rho, rho_hat, v.m_tot);
  }
}

template <typename T>
void launch_rect_adjoint(const View<T> &v, const RectDesc *rect, int32_t nrect, const T *grh, T *grho_k,
                         hipStream_t st) {
  k_copy<T><<<grid_for(v.m_tot), NT, 0, st>>>(grho_k, grh, v.m_tot);
  if (nrect > 0) k_block_mean<T><<<nrect, NT, 0, st>>>(rect, nrect, grh, grho_k, v.m_tot);
}

template <typename T>
void launch_cols_pre(const View<T> &v, const RowBuckets &bk, const T *rho_hat, const T *x, const T *s, const T *y,
                     T *dg, double *xi, DiagSolve<T> ds, hipStream_t st) {
  BucketArgs a = make_bucket_args(bk);
  if (nblocks_bucket(a) > 0)
    k_cols_pre<T><<<(int)nblocks_bucket(a), NT, 0, st>>>(v, a, rho_hat, x, s, y, dg, xi, ds);
}

template <typename T>
void launch_rows_post(const View<T> &v, const RowBuckets &bk, const T *rho_hat, const T *alpha_k, const T *xt,
                      const T *s, const T *y, T *st_out, T *sh, T *vv, T *s_new, T *y_new, hipStream_t st) {
  BucketArgs a = make_bucket_args(bk);
  if (nblocks_bucket(a) > 0)
    k_rows_post<T><<<(int)nblocks_bucket(a), NT, 0, st>>>(v, a, rho_hat, alpha_k, xt, s, y, st_out, sh, vv, s_new,
                                                          y_new);
}

template <typename T>
void launch_bwd_rows_a(const View<T> &v, const T *rho_hat, const T *alpha_k, const T *stl, const T *s, const T *y,
                       const T *s_new, const T *gs_in, const T *gy_in, T *gsn, T *gv, bool all_rows, hipStream_t st) {
  (void)s_new;
  k_bwd_rows_a<T><<<grid_for(v.m_tot), NT, 0, st>>>(v, rho_hat, alpha_k, stl, s, y, gs_in, gy_in, gsn, gv,
                                                    all_rows ? 1 : 0);
}

template <typename T>
void launch_rows_v(const View<T> &v, const T *rho_hat, const T *alpha_k, const T *stl, const T *s, const T *y, T *vv,
                   hipStream_t st) {
  k_rows_v<T><<<grid_for(v.m_tot), NT, 0, st>>>(v, rho_hat, alpha_k, stl, s, y, vv);
}

template <typename T>
void launch_bwd_rows_b(const View<T> &v, const T *rho_hat, const T *alpha_k, const T *stl, const T *s, const T *y,
                       const T *s_new, const T *gy_in, const T *gv, T *gsh, T *gst, T *gs_out, T *gy_out, T *grh,
                       const T *gst_extra, hipStream_t st) {
  k_bwd_rows_b<T><<<grid_for(v.m_tot), NT, 0, st>>>(v, rho_hat, alpha_k, stl, s, y, s_new, gy_in, gv, gsh, gst,
                                                    gs_out, gy_out, grh, gst_extra);
}

template <typename T>
void launch_bwd_cols(const View<T> &v, const RowBuckets &bk, const T *rho_hat, const T *alpha_k, const T *gst,
                     const T *gx_in, double *gxt, T *dg, DiagSolve<T> ds, hipStream_t st) {
  BucketArgs a = make_bucket_args(bk);
  if (nblocks_bucket(a) > 0)
    k_bwd_cols<T><<<(int)nblocks_bucket(a), NT, 0, st>>>(v, a, rho_hat, alpha_k, gst, gx_in, gxt, dg, ds);
}

template <typename T>
void launch_bwd_rows_c(const View<T> &v, const RowBuckets &bk, const T *rho_hat, const T *w, const T *stl,
                       const T *s, T *grh, T *gs_out, T *gy_out, hipStream_t st) {
  BucketArgs a = make_bucket_args(bk);
  if (nblocks_bucket(a) > 0)
    k_bwd_rows_c<T><<<(int)nblocks_bucket(a), NT, 0, st>>>(v, a, rho_hat, w, stl, s, grh, gs_out, gy_out);
}

template <typename T>
void launch_alpha_reduce(const View<T> &v, const T *gsh, const T *stl, const T *s, const T *gx_in, const T *xt,
                         const T *x, T *galpha_k, hipStream_t st) {
  k_alpha_reduce<T><<<v.B, NT, 0, st>>>(v, gsh, stl, s, gx_in, xt, x, galpha_k);
}

template <typename T>
void launch_loss(const View<T> &v, const RowBuckets &bkA, const RowBuckets &bkAt, const T *x, const T *s, const T *y,
                 T *rp, T *rd, T *loss, T *gx, T *gs, T *gy, hipStream_t st) {
  BucketArgs a = make_bucket_args(bkA), at = make_bucket_args(bkAt);
  // each dense product feeds the kernel right after it (the scratch is reused)
  launch_dense_rows<T>(v, x, st);
  if (nblocks_bucket(a) > 0) k_loss_rp<T><<<(int)nblocks_bucket(a), NT, 0, st>>>(v, a, x, s, rp);
  launch_dense_cols<T>(v, DC_Y, nullptr, y, nullptr, st);
  if (nblocks_bucket(at) > 0) k_loss_rd<T><<<(int)nblocks_bucket(at), NT, 0, st>>>(v, at, x, y, rd);
  k_loss_reduce<T><<<v.B, NT, 0, st>>>(v, rp, rd, loss);
  if (gx) launch_dense_cols<T>(v, DC_RP, nullptr, rp, nullptr, st);
  if (gx && nblocks_bucket(at) > 0) k_loss_gx<T><<<(int)nblocks_bucket(at), NT, 0, st>>>(v, at, rp, rd, gx);
  if (gs || gy) launch_dense_rows<T>(v, rd, st);
  if ((gs || gy) && nblocks_bucket(a) > 0) k_loss_gsy<T><<<(int)nblocks_bucket(a), NT, 0, st>>>(v, a, rp, rd, gs, gy);
}

template <typename T>
void launch_pol_resid(const View<T> &v, const RowBuckets &bkA, const RowBuckets &bkAt, const T *x, const T *s,
                      const T *y, T *u, T *rp, T *p, T *w, T *rd, hipStream_t st) {
  BucketArgs a = make_bucket_args(bkA), at = make_bucket_args(bkAt);
  launch_dense_rows<T>(v, x, st);
  if (nblocks_bucket(a) > 0) k_pol_rows<T><<<(int)nblocks_bucket(a), NT, 0, st>>>(v, a, x, s, u, rp);
  launch_dense_cols<T>(v, DC_Y, nullptr, y, nullptr, st);
  if (nblocks_bucket(at) > 0) k_pol_cols<T><<<(int)nblocks_bucket(at), NT, 0, st>>>(v, at, x, y, p, w, rd);
}

template <typename T>
void launch_pol_resid_adjoint(const View<T> &v, const RowBuckets &bkA, const RowBuckets &bkAt, const T *ub,
                              const T *pb, const T *wb, T *gx, T *gy, hipStream_t st) {
  BucketArgs a = make_bucket_args(bkA), at = make_bucket_args(bkAt);
  launch_dense_cols<T>(v, DC_RP, nullptr, ub, nullptr, st);
  if (nblocks_bucket(at) > 0) k_pol_adj_cols<T><<<(int)nblocks_bucket(at), NT, 0, st>>>(v, at, ub, pb, gx);
  launch_dense_rows<T>(v, wb, st);
  if (nblocks_bucket(a) > 0) k_pol_adj_rows<T><<<(int)nblocks_bucket(a), NT, 0, st>>>(v, a, wb, gy);
}

template <typename T>
void launch_solve_rho(const View<T> &v, const double *rho_b, double eq_scale, T *rho, int32_t K, hipStream_t st) {
  k_solve_rho<T><<<grid_for(v.m_tot), NT, 0, st>>>(v, rho_b, eq_scale, rho, K);
}

template <typename T> void launch_copy(T *dst, const T *src, int64_t n, hipStream_t st) {
  if (n > 0) k_copy<T><<<grid_for(n), NT, 0, st>>>(dst, src, n);
}

template <typename T> void launch_fill(T *dst, T val, int64_t n, hipStream_t st) {
  if (n > 0) k_fill<T><<<grid_for(n), NT, 0, st>>>(dst, val, n);
}

template <typename T>
void launch_nonfinite_check(const View<T> &v, const T *x, const T *s, const T *y, cosmo_stats *stats,
                            hipStream_t st) {
  if (stats) k_nonfinite<T><<<v.B, NT, 0, st>>>(v, x, s, y, stats);
}

#define INST(T)                                                                                                   \
  template void launch_rectify<T>(const View<T> &, const RectDesc *, int32_t, const T *, T *, int32_t,          \
                                  hipStream_t);                                                                 \
  template void launch_rect_adjoint<T>(const View<T> &, const RectDesc *, int32_t, const T *, T *, hipStream_t); \
  template void launch_cols_pre<T>(const View<T> &, const RowBuckets &, const T *, const T *, const T *,        \
                                   const T *, T *, double *, DiagSolve<T>, hipStream_t);                        \
  template void launch_rows_post<T>(const View<T> &, const RowBuckets &, const T *, const T *, const T *,       \
                                    const T *, const T *, T *, T *, T *, T *, T *, hipStream_t);                \
  template void launch_bwd_rows_a<T>(const View<T> &, const T *, const T *, const T *, const T *, const T *,    \
                                     const T *, const T *, const T *, T *, T *, bool, hipStream_t);             \
  template void launch_rows_v<T>(const View<T> &, const T *, const T *, const T *, const T *, const T *, T *,  \
                                 hipStream_t);                                                                \
  template void launch_bwd_rows_b<T>(const View<T> &, const T *, const T *, const T *, const T *, const T *,    \
                                     const T *, const T *, const T *, T *, T *, T *, T *, T *, const T *, hipStream_t);    \
  template void launch_bwd_cols<T>(const View<T> &, const RowBuckets &, const T *, const T *, const T *,        \
                                   const T *, double *, T *, DiagSolve<T>, hipStream_t);                             \
  template void launch_bwd_rows_c<T>(const View<T> &, const RowBuckets &, const T *, const T *, const T *,      \
                                     const T *, T *, T *, T *, hipStream_t);                                    \
  template void launch_alpha_reduce<T>(const View<T> &, const T *, const T *, const T *, const T *, const T *,  \
                                       const T *, T *, hipStream_t);                                            \
  template void launch_loss<T>(const View<T> &, const RowBuckets &, const RowBuckets &, const T *, const T *,   \
                               const T *, T *, T *, T *, T *, T *, T *, hipStream_t);                           \
  template void launch_pol_resid<T>(const View<T> &, const RowBuckets &, const RowBuckets &, const T *,         \
                                    const T *, const T *, T *, T *, T *, T *, T *, hipStream_t);                \
  template void launch_pol_resid_adjoint<T>(const View<T> &, const RowBuckets &, const RowBuckets &, const T *, \
                                            const T *, const T *, T *, T *, hipStream_t);                       \
  template void launch_solve_rho<T>(const View<T> &, const double *, double, T *, int32_t, hipStream_t);    \
  template void launch_copy<T>(T *, const T *, int64_t, hipStream_t);                                           \
  template void launch_fill<T>(T *, T, int64_t, hipStream_t);                                                   \
  template void launch_nonfinite_check<T>(const View<T> &, const T *, const T *, const T *, cosmo_stats *,      \
                                          hipStream_t);

INST(float)
INST(double)

}  // namespace cosmo
