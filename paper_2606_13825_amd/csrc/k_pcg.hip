// Jacobi-preconditioned conjugate gradient for the reduced COSMO system
//   M(rho_hat) x = rhs,   M = P + sigma I + A' D(rho_hat) A
// (eq:cosmo_linear_system_reduced; CG with Jacobi preconditioner, Table 2).
// The operator is applied matrix-free: t = rho_hat o (A p) over the
// instance's rows, then (M p)_j = (P p)_j + sigma p_j + (A' t)_j over its
// columns -- M and A'A are never formed (Sec. "Matrix-Free Implicit
// Differentiation").  The same kernel solves the adjoint system of the
// backward pass (M is symmetric, so the adjoint uses the same operator and
// preconditioner, eq:grad_rho).
//
// One workgroup owns one instance and iterates to its own tolerance: no
// grid-wide synchronisation, no host round trip, per-instance scalars
// (segmented CG over the super-batch).  Stopping rule: the unpreconditioned
// residual ||rhs - M x||_2 <= tol ||rhs||_2, or max_iter iterations.
#include "cosmo_internal.h"

namespace cosmo {
namespace {

constexpr int PT = 512;   // threads per instance workgroup
constexpr int NW = PT / 64;

template <typename T> __device__ inline T sub_sum(T v, int L) {
  for (int off = L >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic workgroup sum of two values.
template <typename T> __device__ inline void block_sum2(T &a, T &b, T *red) {
  a = sub_sum(a, 64);
  b = sub_sum(b, 64);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) {
    red[w] = a;
    red[NW + w] = b;
  }
  __syncthreads();
  T ta = 0, tb = 0;
  for (int i = 0; i < NW; ++i) {
    ta += red[i];
    tb += red[NW + i];
  }
  a = ta;
  b = tb;
}

// One pass of CSR row products over the rows rows[r0..r1) of one length
// class, L lanes per row (each lane keeps two products in flight), handing
// each row's sum to emit(row, sum) on its first lane.
template <typename T, int L, typename F>
__device__ inline void csr_pass(const int32_t *__restrict__ rows, int64_t r0, int64_t r1,
                                const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                const T *__restrict__ val, const T *__restrict__ vin, F emit) {
  constexpr int per = PT / L;
  const int sub = threadIdx.x / L, lane = threadIdx.x % L;
  for (int64_t base = r0; base < r1; base += per) {
    const int64_t ri = base + sub;
    int32_t row = 0;
    T a0 = 0, a1 = 0;
    if (ri < r1) {
      row = rows[ri];
      const int64_t k1 = rowptr[row + 1];
      int64_t k = rowptr[row] + lane;
      for (; k + L < k1; k += 2 * L) {
        a0 += val[k] * vin[col[k]];
        a1 += val[k + L] * vin[col[k + L]];
      }
      if (k < k1) a0 += val[k] * vin[col[k]];
    }
    const T acc = sub_sum(a0 + a1, L);   // every lane of the row group takes part
    if (ri < r1 && lane == 0) emit(row, acc);
  }
}

// out = M p over the instance; returns (in every thread) p'Mp.  Rows of A and
// of A' are taken by length class (1, 8 or 64 lanes per row).
template <typename T>
__device__ T apply_M(const View<T> &v, const T *__restrict__ rho_hat, const T *__restrict__ p, T *__restrict__ t,
                     T *__restrict__ out, int b, T *red) {
  const int64_t B1 = v.B + 1;
  // t_i = rho_hat_i (A p)_i
  auto emit_t = [&](int32_t i, T acc) { t[i] = rho_hat[i] * acc; };
  csr_pass<T, 1>(v.rowsA, v.instA[b], v.instA[b + 1], v.A_rowptr, v.A_col, v.A_val, p, emit_t);
  csr_pass<T, 8>(v.rowsA, v.instA[B1 + b], v.instA[B1 + b + 1], v.A_rowptr, v.A_col, v.A_val, p, emit_t);
  csr_pass<T, 64>(v.rowsA, v.instA[2 * B1 + b], v.instA[2 * B1 + b + 1], v.A_rowptr, v.A_col, v.A_val, p, emit_t);
  __syncthreads();
  // (M p)_j = (A' t)_j + (P p)_j + sigma p_j
  T pMp = 0, dummy = 0;
  auto emit_m = [&](int32_t j, T acc) {
    if (v.P_rowptr)
      for (int64_t k = v.P_rowptr[j]; k < v.P_rowptr[j + 1]; ++k) acc += v.P_val[k] * p[v.P_col[k]];
    const T mp = acc + v.sigma * p[j];
    out[j] = mp;
    pMp += p[j] * mp;
  };
  csr_pass<T, 1>(v.rowsAt, v.instAt[b], v.instAt[b + 1], v.At_rowptr, v.At_col, v.At_val, t, emit_m);
  csr_pass<T, 8>(v.rowsAt, v.instAt[B1 + b], v.instAt[B1 + b + 1], v.At_rowptr, v.At_col, v.At_val, t, emit_m);
  csr_pass<T, 64>(v.rowsAt, v.instAt[2 * B1 + b], v.instAt[2 * B1 + b + 1], v.At_rowptr, v.At_col, v.At_val, t,
                  emit_m);
  block_sum2(pMp, dummy, red);
  return pMp;
}

template <typename T>
__global__ __launch_bounds__(PT) void k_pcg(View<T> v, const T *__restrict__ rho_hat, const T *__restrict__ dg,
                                            const T *__restrict__ rhs, T *__restrict__ x, T *__restrict__ r,
                                            T *__restrict__ z, T *__restrict__ p, T *__restrict__ Mp,
                                            T *__restrict__ t, T tol, int32_t max_iter,
                                            const T *__restrict__ alpha_k, const T *__restrict__ xold,
                                            T *__restrict__ xnew, const T *__restrict__ gx_in,
                                            T *__restrict__ gx_out, int32_t mode, cosmo_stats *stats) {
  __shared__ T red[2 * NW];
  const int b = blockIdx.x;
  const int64_t n0 = v.n_off[b], n1 = v.n_off[b + 1];

  // r = rhs - M x (warm start)
  apply_M(v, rho_hat, x, t, Mp, b, red);
  __syncthreads();
  T rz = 0, rr = 0, bb = 0, dummy = 0;
  for (int64_t j = n0 + threadIdx.x; j < n1; j += PT) {
    const T rj = rhs[j] - Mp[j];
    const T zj = rj / dg[j];
    r[j] = rj;
    z[j] = zj;
    p[j] = zj;
    rz += rj * zj;
    rr += rj * rj;
    bb += rhs[j] * rhs[j];
  }
  block_sum2(rz, rr, red);
  block_sum2(bb, dummy, red);
  const T thr = tol * tol * bb;
  // A non-finite right-hand side, operator or iterate ends the solve and
  // marks its solution non-finite (rather than leaving the finite warm start).
  bool fail = !(isfinite(rr) && isfinite(bb));
  int it = 0;
  while (!fail && rr > thr && it < max_iter) {
    __syncthreads();   // p complete before the operator reads it
    const T pMp = apply_M(v, rho_hat, p, t, Mp, b, red);
    if (!(pMp > (T)0)) {   // breakdown at round-off level: keep the current x
      fail = !isfinite(pMp);
      break;
    }
    const T a = rz / pMp;
    T rz_new = 0, rr_new = 0;
    for (int64_t j = n0 + threadIdx.x; j < n1; j += PT) {
      x[j] += a * p[j];
      const T rj = r[j] - a * Mp[j];
      const T zj = rj / dg[j];
      r[j] = rj;
      z[j] = zj;
      rz_new += rj * zj;
      rr_new += rj * rj;
    }
    block_sum2(rz_new, rr_new, red);
    const T beta = rz_new / rz;
    rz = rz_new;
    rr = rr_new;
    fail = !isfinite(rr);
    for (int64_t j = n0 + threadIdx.x; j < n1; j += PT) p[j] = z[j] + beta * p[j];
    ++it;
  }
  if (fail)
    for (int64_t j = n0 + threadIdx.x; j < n1; j += PT) x[j] = (T)NAN;
  // epilogue (each thread touches only the columns it owns below)
  const T al = alpha_k ? alpha_k[b] : (T)1;
  if (mode == 0) {
    if (xnew)
      for (int64_t j = n0 + threadIdx.x; j < n1; j += PT) xnew[j] = al * x[j] + ((T)1 - al) * xold[j];
  } else {
    for (int64_t j = n0 + threadIdx.x; j < n1; j += PT) gx_out[j] = ((T)1 - al) * gx_in[j] + v.sigma * x[j];
  }
  if (stats && threadIdx.x == 0) {
    atomicMax(&stats[b].cg_iters_max, it);
    atomicAdd(&stats[b].cg_iters_total, it);
    if (!(rr <= thr)) atomicAdd(&stats[b].cg_not_converged, 1);
  }
}

}  // namespace

template <typename T>
void launch_pcg(const View<T> &v, const T *rho_hat, const T *dg, const T *rhs, T *x, T *r, T *z, T *p, T *Mp, T *t,
                double tol, int32_t max_iter, const T *alpha_k, const T *xold, T *xnew, const T *gx_in, T *gx_out,
                int32_t mode, cosmo_stats *stats, hipStream_t st) {
  k_pcg<T><<<v.B, PT, 0, st>>>(v, rho_hat, dg, rhs, x, r, z, p, Mp, t, (T)tol, max_iter, alpha_k, xold, xnew, gx_in,
                               gx_out, mode, stats);
}

template void launch_pcg<float>(const View<float> &, const float *, const float *, const float *, float *, float *,
                                float *, float *, float *, float *, double, int32_t, const float *, const float *,
                                float *, const float *, float *, int32_t, cosmo_stats *, hipStream_t);
template void launch_pcg<double>(const View<double> &, const double *, const double *, const double *, double *,
                                 double *, double *, double *, double *, double *, double, int32_t, const double *,
                                 const double *, double *, const double *, double *, int32_t, cosmo_stats *,
                                 hipStream_t);

}  // namespace cosmo
