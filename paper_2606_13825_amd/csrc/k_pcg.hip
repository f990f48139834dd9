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
// Two launch forms share the stopping rule (unpreconditioned residual
// ||rhs - M x||_2 <= tol ||rhs||_2, or max_iter iterations) and the per-
// instance scalars (segmented CG over the super-batch):
//  * k_pcg: one workgroup owns one instance and iterates to its own
//    tolerance, with no grid-wide synchronisation;
//  * k_pcg_coop: one cooperative launch over the whole chip; the operator
//    passes spread every instance's rows over all workgroups, the vector
//    updates run one workgroup per instance, phases are separated by grid
//    barriers, and instances that have converged drop out of the passes.
//    The loop ends for every workgroup at the same barrier, when no
//    instance is left active (at the latest after max_iter iterations).
#include <hip/hip_cooperative_groups.h>

#include <algorithm>

#include "cosmo_internal.h"

namespace cosmo {
namespace {

constexpr int PT = 512;   // threads per instance workgroup
constexpr int CT = 256;   // threads per workgroup of the cooperative form
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
// Short rows (at most 4 nonzeros, one lane each): every thread takes four
// rows per pass and reads all their entries with clamped indices and masks,
// so the whole gather is in flight at once.
template <typename T, int NTH, typename Act, typename F>
__device__ inline void short_rows(const int32_t *__restrict__ rows, int64_t first, int64_t r1, int64_t stride,
                                  const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                  const T *__restrict__ val, const T *__restrict__ vin, Act active, F emit) {
  for (int64_t base = first; base < r1; base += 4 * stride) {
    int32_t rw[4];
    int64_t k0[4], nk[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t ri = base + u * stride;
      ok[u] = ri < r1;
      rw[u] = ok[u] ? rows[ri] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ok[u] = ok[u] && active(rw[u]);
      k0[u] = ok[u] ? rowptr[rw[u]] : 0;
      nk[u] = ok[u] ? rowptr[rw[u] + 1] - k0[u] : 0;
    }
    T acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc[u] = 0;
      if (nk[u] > 0) {
        // indices clamped to the row's last entry; surplus terms masked
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t k = k0[u] + (q < nk[u] ? q : nk[u] - 1);
          const T prod = val[k] * vin[col[k]];
          acc[u] += q < nk[u] ? prod : (T)0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ok[u]) emit(rw[u], acc[u]);
  }
}

template <typename T, int L, typename F>
__device__ inline void csr_pass(const int32_t *__restrict__ rows, int64_t r0, int64_t r1,
                                const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                const T *__restrict__ val, const T *__restrict__ vin, F emit) {
  if constexpr (L == 1) {
    short_rows<T, PT>(rows, r0 + threadIdx.x, r1, PT, rowptr, col, val, vin, [](int32_t) { return true; }, emit);
    return;
  }
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

// ---- cooperative form ------------------------------------------------------

template <int NTH, typename T> __device__ inline void wg_sum2(T &a, T &b, T *red) {
  a = sub_sum(a, 64);
  b = sub_sum(b, 64);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) {
    red[w] = a;
    red[NTH / 64 + w] = b;
  }
  __syncthreads();
  T ta = 0, tb = 0;
  for (int i = 0; i < NTH / 64; ++i) {
    ta += red[i];
    tb += red[NTH / 64 + i];
  }
  a = ta;
  b = tb;
}

// Rows rows[r0..r1) of one length class spread over the whole grid, L lanes
// per row; rows whose instance is inactive are skipped.
template <typename T, int L, typename Act, typename F>
__device__ inline void grid_csr_pass(const int32_t *__restrict__ rows, int64_t r0, int64_t r1,
                                     const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                     const T *__restrict__ val, const T *__restrict__ vin, Act active, F emit) {
  if constexpr (L == 1) {
    short_rows<T, CT>(rows, r0 + (int64_t)blockIdx.x * CT + threadIdx.x, r1, (int64_t)gridDim.x * CT, rowptr, col,
                      val, vin, active, emit);
    return;
  }
  const int64_t per = CT / L;
  const int64_t gsub = (int64_t)blockIdx.x * per + threadIdx.x / L;
  const int64_t nsub = (int64_t)gridDim.x * per;
  const int lane = threadIdx.x % L;
  for (int64_t base = r0; base < r1; base += nsub) {
    const int64_t ri = base + gsub;
    int32_t row = 0;
    bool ok = false;
    T a0 = 0, a1 = 0;
    if (ri < r1) {
      row = rows[ri];
      ok = active(row);
      if (ok) {
        const int64_t k1 = rowptr[row + 1];
        int64_t k = rowptr[row] + lane;
        for (; k + L < k1; k += 2 * L) {
          a0 += val[k] * vin[col[k]];
          a1 += val[k + L] * vin[col[k + L]];
        }
        if (k < k1) a0 += val[k] * vin[col[k]];
      }
    }
    const T acc = sub_sum(a0 + a1, L);
    if (ok && lane == 0) emit(row, acc);
  }
}

// Per-instance state of the cooperative solve (caller workspace): scalars
// rz, rr, thr [B] of type T, then int32 it, act, fail [B] and two counters.
template <typename T> struct CoopState {
  T *rz, *rr, *thr;
  int32_t *it, *act, *fail, *cnt;
};

template <typename T> __device__ inline CoopState<T> coop_state(void *ws, int B) {
  CoopState<T> c;
  T *f = static_cast<T *>(ws);
  c.rz = f;
  c.rr = f + B;
  c.thr = f + 2 * B;
  int32_t *i = reinterpret_cast<int32_t *>(f + 3 * B);
  c.it = i;
  c.act = i + B;
  c.fail = i + 2 * B;
  c.cnt = i + 3 * B;
  return c;
}

// out = M vin for the active instances (grid-wide; ends with a grid barrier).
template <typename T>
__device__ void coop_apply_M(const View<T> &v, const T *__restrict__ rho_hat, const T *__restrict__ vin,
                             T *__restrict__ t, T *__restrict__ out, const int32_t *act,
                             cooperative_groups::grid_group &grid) {
  const int64_t B1 = v.B + 1;
  auto row_act = [&](int32_t i) { return act[v.row_inst[i]] != 0; };
  auto col_act = [&](int32_t j) { return act[v.col_inst[j]] != 0; };
  auto emit_t = [&](int32_t i, T acc) { t[i] = rho_hat[i] * acc; };
  grid_csr_pass<T, 1>(v.rowsA, v.instA[0], v.instA[v.B], v.A_rowptr, v.A_col, v.A_val, vin, row_act, emit_t);
  grid_csr_pass<T, 8>(v.rowsA, v.instA[B1], v.instA[B1 + v.B], v.A_rowptr, v.A_col, v.A_val, vin, row_act, emit_t);
  grid_csr_pass<T, 64>(v.rowsA, v.instA[2 * B1], v.instA[2 * B1 + v.B], v.A_rowptr, v.A_col, v.A_val, vin, row_act,
                       emit_t);
  grid.sync();
  auto emit_m = [&](int32_t j, T acc) {
    if (v.P_rowptr)
      for (int64_t k = v.P_rowptr[j]; k < v.P_rowptr[j + 1]; ++k) acc += v.P_val[k] * vin[v.P_col[k]];
    out[j] = acc + v.sigma * vin[j];
  };
  grid_csr_pass<T, 1>(v.rowsAt, v.instAt[0], v.instAt[v.B], v.At_rowptr, v.At_col, v.At_val, t, col_act, emit_m);
  grid_csr_pass<T, 8>(v.rowsAt, v.instAt[B1], v.instAt[B1 + v.B], v.At_rowptr, v.At_col, v.At_val, t, col_act,
                      emit_m);
  grid_csr_pass<T, 64>(v.rowsAt, v.instAt[2 * B1], v.instAt[2 * B1 + v.B], v.At_rowptr, v.At_col, v.At_val, t,
                       col_act, emit_m);
  grid.sync();
}

template <typename T>
__global__ __launch_bounds__(CT) void k_pcg_coop(View<T> v, const T *__restrict__ rho_hat, const T *__restrict__ dg,
                                                 const T *__restrict__ rhs, T *__restrict__ x, T *__restrict__ r,
                                                 T *__restrict__ z, T *__restrict__ p, T *__restrict__ Mp,
                                                 T *__restrict__ t, T tol, int32_t max_iter,
                                                 const T *__restrict__ alpha_k, const T *__restrict__ xold,
                                                 T *__restrict__ xnew, const T *__restrict__ gx_in,
                                                 T *__restrict__ gx_out, int32_t mode, cosmo_stats *stats,
                                                 void *state) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  __shared__ T red[2 * (CT / 64)];
  const CoopState<T> cs = coop_state<T>(state, v.B);
  // every instance takes part in the first operator application
  for (int b = blockIdx.x * CT + threadIdx.x; b < v.B; b += gridDim.x * CT) cs.act[b] = 1;
  if (blockIdx.x == 0 && threadIdx.x < 2) cs.cnt[threadIdx.x] = 0;
  grid.sync();
  // r = rhs - M x (warm start), z = r / diag M, p = z
  coop_apply_M(v, rho_hat, x, t, Mp, cs.act, grid);
  for (int b = blockIdx.x; b < v.B; b += gridDim.x) {
    const int64_t n0 = v.n_off[b], n1 = v.n_off[b + 1];
    T rz = 0, rr = 0, bb = 0, dummy = 0;
    for (int64_t j = n0 + threadIdx.x; j < n1; j += CT) {
      const T rj = rhs[j] - Mp[j];
      const T zj = rj / dg[j];
      r[j] = rj;
      z[j] = zj;
      p[j] = zj;
      rz += rj * zj;
      rr += rj * rj;
      bb += rhs[j] * rhs[j];
    }
    wg_sum2<CT>(rz, rr, red);
    wg_sum2<CT>(bb, dummy, red);
    if (threadIdx.x == 0) {
      const T thr = tol * tol * bb;
      const bool fail = !(isfinite(rr) && isfinite(bb));
      const bool act = !fail && rr > thr && max_iter > 0;
      cs.rz[b] = rz;
      cs.rr[b] = rr;
      cs.thr[b] = thr;
      cs.it[b] = 0;
      cs.fail[b] = fail;
      cs.act[b] = act;
      if (act) atomicAdd(&cs.cnt[0], 1);
    }
  }
  grid.sync();
  for (int iter = 0;; ++iter) {
    const int par = iter & 1;
    const int nact = __hip_atomic_load(&cs.cnt[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (nact == 0) break;   // the same value in every workgroup: all leave together
    if (blockIdx.x == 0 && threadIdx.x == 0) cs.cnt[par ^ 1] = 0;
    coop_apply_M(v, rho_hat, p, t, Mp, cs.act, grid);
    for (int b = blockIdx.x; b < v.B; b += gridDim.x) {
      if (!cs.act[b]) continue;
      const int64_t n0 = v.n_off[b], n1 = v.n_off[b + 1];
      T pMp = 0, dummy = 0;
      for (int64_t j = n0 + threadIdx.x; j < n1; j += CT) pMp += p[j] * Mp[j];
      wg_sum2<CT>(pMp, dummy, red);
      bool fail = false, act = true;
      if (!(pMp > (T)0)) {   // breakdown at round-off level keeps x; a non-finite one fails
        fail = !isfinite(pMp);
        act = false;
      } else {
        const T a = cs.rz[b] / pMp;
        T rz_new = 0, rr_new = 0;
        for (int64_t j = n0 + threadIdx.x; j < n1; j += CT) {
          x[j] += a * p[j];
          const T rj = r[j] - a * Mp[j];
          const T zj = rj / dg[j];
          r[j] = rj;
          z[j] = zj;
          rz_new += rj * zj;
          rr_new += rj * rj;
        }
        wg_sum2<CT>(rz_new, rr_new, red);
        const T beta = rz_new / cs.rz[b];
        for (int64_t j = n0 + threadIdx.x; j < n1; j += CT) p[j] = z[j] + beta * p[j];
        const int it = cs.it[b] + 1;
        fail = !isfinite(rr_new);
        act = !fail && rr_new > cs.thr[b] && it < max_iter;
        __syncthreads();   // every thread has read the scalars before they change
        if (threadIdx.x == 0) {
          cs.rz[b] = rz_new;
          cs.rr[b] = rr_new;
          cs.it[b] = it;
        }
      }
      if (threadIdx.x == 0) {
        cs.fail[b] = fail;
        cs.act[b] = act;
        if (act) atomicAdd(&cs.cnt[par ^ 1], 1);
      }
    }
    grid.sync();
  }
  // epilogue, one workgroup per instance
  for (int b = blockIdx.x; b < v.B; b += gridDim.x) {
    const int64_t n0 = v.n_off[b], n1 = v.n_off[b + 1];
    if (cs.fail[b])
      for (int64_t j = n0 + threadIdx.x; j < n1; j += CT) x[j] = (T)NAN;
    __syncthreads();
    const T al = alpha_k ? alpha_k[b] : (T)1;
    if (mode == 0) {
      if (xnew)
        for (int64_t j = n0 + threadIdx.x; j < n1; j += CT) xnew[j] = al * x[j] + ((T)1 - al) * xold[j];
    } else {
      for (int64_t j = n0 + threadIdx.x; j < n1; j += CT) gx_out[j] = ((T)1 - al) * gx_in[j] + v.sigma * x[j];
    }
    if (stats && threadIdx.x == 0) {
      atomicMax(&stats[b].cg_iters_max, cs.it[b]);
      atomicAdd(&stats[b].cg_iters_total, cs.it[b]);
      if (!(cs.rr[b] <= cs.thr[b])) atomicAdd(&stats[b].cg_not_converged, 1);
    }
  }
}

}  // namespace

template <typename T>
int pcg_coop_grid(int per_cu) {
  // as many workgroups as stay resident together, at most per_cu per compute
  // unit; 0 when the device has no cooperative launch
  static int nb = -1, ncu = 0;
  if (nb < 0) {
    int dev = 0, coop = 0;
    nb = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && coop &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pcg_coop<T>, CT, 0) != hipSuccess)
      nb = 0;
    if (!coop) nb = 0;
  }
  return std::min(nb, per_cu) * ncu;
}

template <typename T>
void launch_pcg(const View<T> &v, const T *rho_hat, const T *dg, const T *rhs, T *x, T *r, T *z, T *p, T *Mp, T *t,
                double tol, int32_t max_iter, const T *alpha_k, const T *xold, T *xnew, const T *gx_in, T *gx_out,
                int32_t mode, cosmo_stats *stats, void *state, int32_t form, hipStream_t st) {
  // form 0: one workgroup per instance; form f > 0: the cooperative form
  // with at most f workgroups per compute unit (the runtime refuses a grid
  // that would not be resident at once; the per-instance form then runs)
  const int grid = (form > 0 && state) ? pcg_coop_grid<T>(form) : 0;
  if (grid > 0) {
    View<T> va = v;
    T tl = (T)tol;
    int32_t mi = max_iter, md = mode;
    void *args[] = {&va, &rho_hat, &dg, &rhs, &x, &r, &z, &p, &Mp, &t, &tl, &mi, &alpha_k, &xold, &xnew, &gx_in,
                    &gx_out, &md, &stats, &state};
    if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_pcg_coop<T>), dim3(grid), dim3(CT), args, 0,
                                   st) == hipSuccess)
      return;
    (void)hipGetLastError();
  }
  k_pcg<T><<<v.B, PT, 0, st>>>(v, rho_hat, dg, rhs, x, r, z, p, Mp, t, (T)tol, max_iter, alpha_k, xold, xnew, gx_in,
                               gx_out, mode, stats);
}

template void launch_pcg<float>(const View<float> &, const float *, const float *, const float *, float *, float *,
                                float *, float *, float *, float *, double, int32_t, const float *, const float *,
                                float *, const float *, float *, int32_t, cosmo_stats *, void *, int32_t, hipStream_t);
template void launch_pcg<double>(const View<double> &, const double *, const double *, const double *, double *,
                                 double *, double *, double *, double *, double *, double, int32_t, const double *,
                                 const double *, double *, const double *, double *, int32_t, cosmo_stats *, void *,
                                 int32_t, hipStream_t);

}  // namespace cosmo
