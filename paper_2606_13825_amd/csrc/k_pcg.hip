// Jacobi-preconditioned conjugate gradient for the reduced COSMO system
//   M(rho_hat) x = rhs,   M = P + sigma I + A' D(rho_hat) A
// (rhs is held in float64: in float32 its one rounding alone can move the
// solution by up to cond(M) eps, e.g. 4e-3 on the Lovasz systems, whose
// right-hand side is dominated by the trace row's large component)
// (eq:cosmo_linear_system_reduced; CG with Jacobi preconditioner, Table 2).
// The operator is applied matrix-free: t = rho_hat o (A p) over the
// instance's rows, then (M p)_j = (P p)_j + sigma p_j + (A' t)_j over its
// columns -- M and A'A are never formed (Sec. "Matrix-Free Implicit
// Differentiation").  The same kernels solve the adjoint system of the
// backward pass (M is symmetric, so the adjoint uses the same operator and
// preconditioner, eq:grad_rho).
//
// Stopping rule: the true residual ||rhs - M x||_2 <= tol ||rhs||_2, or
// max_iter iterations in all.  The iteration runs in the working precision
// on the recursively updated residual; when that meets the tolerance the
// true residual is recomputed with float64 accumulation, and if it does not
// the CG restarts from it (iterative refinement: each restarted round solves
// for the correction and only needs to lower its own starting residual by
// 1e-2).  Refinement ends when the true residual meets the tolerance, after
// four restarts, or when a round lowered the true residual by less than 2x
// (the working precision's floor).  On an ill-conditioned M a float32
// recursion alone leaves a solution error near cond(M) eps; each refinement
// round multiplies it by about cond(M) eps again.
//
// Two launch forms share the rule and the per-instance scalars (segmented
// CG over the super-batch):
//  * k_pcg: one workgroup owns one instance and iterates to its own
//    tolerance, with no grid-wide synchronisation;
//  * k_pcg_coop: one cooperative launch over the whole chip; the operator
//    passes spread every instance's rows over all workgroups, the vector
//    updates run one workgroup per instance, phases are separated by grid
//    barriers, and instances that are done drop out of the passes.  Every
//    workgroup leaves each loop at the same barrier, when no instance is
//    left active (bounded by max_iter and the restart count).
//
// The grid barrier is written here rather than taken from the runtime: an
// arrival counter and a generation word, with an agent-scope release fence
// before arriving and an acquire fence after leaving, costs about a quarter
// of the runtime's grid synchronisation at 256-512 workgroups.  The launch
// is cooperative, so every workgroup is resident and every wait ends; each
// wait is still bounded in time, and a wait that runs out raises an abort
// word that releases every workgroup: the solve then ends at once and marks
// its solutions non-finite instead of hanging.
#include <algorithm>

#include "cosmo_internal.h"
#include "wave_ops.h"

namespace cosmo {
namespace {

// threads per instance workgroup: 16 waves (float32) keep more rows in flight
// per CU; the float64 instantiation needs more registers and runs 8 waves
template <typename T> constexpr int PT = sizeof(T) == 4 ? 1024 : 512;
constexpr int CT = 256;      // threads per workgroup of the cooperative form
// threads of the instantiations that fuse dense sub-blocks: 8 waves, so a
// wave may hold 256 registers (its pieces of a dense row, of the vector and
// of the partial product, in float64 for the residual pass)
template <typename T, int DMP> constexpr int PTK = DMP == 0 ? PT<T> : 512;
// strides per pass of the cooperative form's per-instance vector loops (8
// keeps float32 within 128 VGPRs; float64 stays at 4)
template <typename T> constexpr int VLOOP = sizeof(T) == 4 ? 8 : 4;
// 16-byte pieces of a dense row per lane for COSMO_DENSE_MAX_COLS columns
template <typename T> constexpr int MAXPC = COSMO_DENSE_MAX_COLS / (64 * (16 / (int)sizeof(T)));
constexpr int NRESTART = 4;          // restarts from a float64 residual, at most
constexpr double ROUND_DROP2 = 1e-4;  // a restarted round lowers its residual by 1e-2 (squared here)
constexpr double STALL2 = 0.25;       // a true residual that fell by less than 2x ends the refinement

template <typename T> __device__ inline T sub_sum(T v, int L) {
  for (int off = L >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic workgroup sum of two values (red holds 2 NTH / 64 entries).
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

// ---- CSR row passes ------------------------------------------------------------
//
// Rows rows[r0..r1) of one length class, handled by row groups of L lanes:
// group g of a pass takes row r0 + g + j nsub (j = 0, 1, ...).  Sums are
// accumulated in AT; each row's sum goes to emit(row, sum) on its first lane.
// active(row) skips rows (of instances that are done).

// Short rows (at most 4 nonzeros, one lane each): four rows per lane per
// pass, all entries read with clamped indices and masks so the whole gather is
// in flight at once.
template <typename AT, typename T, typename VT, typename Act, typename F>
__device__ inline void short_rows(const int32_t *__restrict__ rows, const RowSpan *__restrict__ span, int64_t first,
                                  int64_t r1, int64_t stride, const int32_t *__restrict__ col,
                                  const T *__restrict__ val, const VT *__restrict__ vin, Act active, F emit) {
  for (int64_t base = first; base < r1; base += 4 * stride) {
    int32_t rw[4];
    int64_t k0[4], nk[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t ri = base + u * stride;
      ok[u] = ri < r1;
      rw[u] = ok[u] ? rows[ri] : 0;
      const RowSpan sp = ok[u] ? span[ri] : RowSpan{0, 0};
      k0[u] = sp.kb;
      nk[u] = sp.k1 - sp.kb;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      ok[u] = ok[u] && active(rw[u]);
      if (!ok[u]) nk[u] = 0;
    }
    AT acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc[u] = 0;
      if (nk[u] > 0) {
        // indices clamped to the row's last entry; surplus terms masked
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t k = k0[u] + (q < nk[u] ? q : nk[u] - 1);
          const AT prod = (AT)val[k] * (AT)vin[col[k]];
          acc[u] += q < nk[u] ? prod : (AT)0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ok[u]) emit(rw[u], acc[u]);
  }
}

// 16-byte pieces of a row: VE = 16 / sizeof(T) values and VE column indices.
template <typename T> struct alignas(16) ValPiece {
  T v[16 / sizeof(T)];
};
template <int N> struct alignas(4 * N) ColPiece {
  int32_t c[N];
};

// L lanes per row.  The row's entries are read in 16-byte pieces (the CSR
// arrays are 16-byte aligned): entries before its first aligned piece and
// after its last full piece one per lane, the full pieces two per lane per
// pass (the second clamped and masked), so that four 16-byte loads and 2 VE
// gathers are in flight per lane.  The next row's id and entry range are
// loaded while the current row is summed, so the index loads are off the
// critical path.  gsub / nsub: this thread's row group and the number of row
// groups of the pass.
template <int L, typename AT, typename T, typename VT, typename Act, typename F>
__device__ inline void row_pass(const int32_t *__restrict__ rows, const RowSpan *__restrict__ span, int64_t r0,
                                int64_t r1, int64_t gsub, int64_t nsub, const int32_t *__restrict__ col,
                                const T *__restrict__ val, const VT *__restrict__ vin, Act active, F emit) {
  if constexpr (L == 1) {
    short_rows<AT>(rows, span, r0 + gsub, r1, nsub, col, val, vin, active, emit);
  } else {
    constexpr int VE = 16 / sizeof(T);
    using VP = ValPiece<T>;
    using CP = ColPiece<VE>;
    const int lane = threadIdx.x % L;
    int64_t ri = r0 + gsub;
    int32_t nrow = 0;
    RowSpan nsp{0, 0};
    if (ri < r1) {
      nrow = rows[ri];
      nsp = span[ri];
    }
    for (int64_t base = r0; base < r1; base += nsub, ri += nsub) {
      const int32_t row = nrow;
      const RowSpan sp = nsp;
      const bool in = ri < r1;
      if (ri + nsub < r1) {
        nrow = rows[ri + nsub];
        nsp = span[ri + nsub];
      }
      bool ok = false;
      AT a0 = 0, a1 = 0;
      if (in) {
        ok = active(row);
        if (ok) {
          const int64_t kb = sp.kb, k1 = sp.k1;
          int64_t ka = (kb + VE - 1) / VE * VE;
          if (ka > k1) ka = k1;
          const int64_t np = (k1 - ka) / VE, kt = ka + np * VE;
          if (lane < ka - kb) a0 += (AT)val[kb + lane] * (AT)vin[col[kb + lane]];
          if (lane < k1 - kt) a1 += (AT)val[kt + lane] * (AT)vin[col[kt + lane]];
          const VP *vp = reinterpret_cast<const VP *>(val + ka);
          const CP *cp = reinterpret_cast<const CP *>(col + ka);
          constexpr int U = 2;
          for (int64_t q = lane; q < np; q += U * L) {
            VP vv[U];
            CP cc[U];
            bool has[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              has[u] = q + u * L < np;
              const int64_t qu = has[u] ? q + u * L : q;
              vv[u] = vp[qu];
              cc[u] = cp[qu];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
              for (int e = 0; e < VE; ++e) {
                const AT pr = (AT)vv[u].v[e] * (AT)vin[cc[u].c[e]];
                if (u % 2 == 0) a0 += has[u] ? pr : (AT)0;
                else a1 += has[u] ? pr : (AT)0;
              }
          }
        }
      }
      const AT acc = sub_sum(a0 + a1, L);   // every lane of the row group takes part
      if (ok && lane == 0) emit(row, acc);
    }
  }
}

// All three length classes of A (cls_off = View::instA) or A' (instAt) over
// the rows of instances [b0, b1): per-instance passes use b1 = b0 + 1, grid
// passes b0 = 0, b1 = B.
template <int NTH, bool GRID, typename AT, typename T, typename VT, typename Act, typename F>
__device__ inline void class_passes(const int32_t *rows, const RowSpan *span, const int64_t *cls_off, int64_t B1,
                                    int b0, int b1, const int32_t *col, const T *val, const VT *vin, Act active,
                                    F emit) {
  auto sub = [&](int L, int64_t &g, int64_t &n) {
    if (GRID) {
      g = (int64_t)blockIdx.x * (NTH / L) + threadIdx.x / L;
      n = (int64_t)gridDim.x * (NTH / L);
    } else {
      g = threadIdx.x / L;
      n = NTH / L;
    }
  };
  int64_t g, n;
  sub(1, g, n);
  row_pass<1, AT>(rows, span, cls_off[b0], cls_off[b1], g, n, col, val, vin, active, emit);
  sub(8, g, n);
  row_pass<8, AT>(rows, span, cls_off[B1 + b0], cls_off[B1 + b1], g, n, col, val, vin, active, emit);
  sub(64, g, n);
  row_pass<64, AT>(rows, span, cls_off[2 * B1 + b0], cls_off[2 * B1 + b1], g, n, col, val, vin, active, emit);
}

// ---- dense sub-blocks inside one instance's workgroup ----------------------------
//
// Rows of A covered by a dense placement hold only their CSR part in t after
// the row passes.  Per row r of each dense block G of instance b, one wave
// forms d = G_r . vin, turns every placement's row i = row0_p + r of t into
// rho_hat_i (t_i + scale_p d), and adds w_r G_r, w_r = sum_p scale_p t_i, to
// its partial of G'w -- so G is read once per operator application.  The
// waves' partials are added in wave order into ec (the column passes add
// ec to the CSR part of A' t).  MP: 16-byte pieces of a row per lane.
template <typename T> struct alignas(16) DPiece {
  T v[16 / sizeof(T)];
};

template <int NTH, int MP, typename AT, typename TG, typename T, typename TT>
__device__ inline void dense_block_fused(const DenseDesc &d, const T *__restrict__ rho_hat, const T *__restrict__ vin,
                                         TT *__restrict__ t, AT *__restrict__ lds, double *__restrict__ ec) {
  constexpr int VE = 16 / sizeof(TG);
  constexpr int NW = NTH / 64;
  // rows in flight per wave: four while a row spans at most two pieces per
  // lane, two for wider rows (register budget); the block read is bound by
  // the bytes each CU keeps in flight
  constexpr int U = MP <= 2 ? 4 : 2;
  static_assert(COSMO_DENSE_MAX_PLACEMENTS == 4, "one lane per (row, placement): four placements per row");
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int npieces = (d.cols + VE - 1) / VE;
  AT xv[MP][VE], acc[MP][VE];
#pragma unroll
  for (int q = 0; q < MP; ++q)
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int c = (lane + 64 * q) * VE + e;
      xv[q][e] = c < d.cols ? (AT)vin[d.col0 + c] : (AT)0;
      acc[q][e] = (AT)0;
    }
  // Lane 4u + p of a pass handles placement p of the pass's row u: it loads
  // that entry of t and rho_hat (two vector loads per pass instead of one
  // per row and placement), forms and stores the new entry, and the four
  // lanes of the row sum their scale * entry into the row's weight.  Lanes
  // of placements the block does not have take scale 0 and store nothing.
  const int lu = (lane >> 2) & (U - 1), lp = lane & 3;
  const bool lplace = lp < d.nplace;
  int64_t lrow0 = d.row0[0];
  AT lsc = (AT)d.scale[0];
#pragma unroll
  for (int q = 1; q < COSMO_DENSE_MAX_PLACEMENTS; ++q)
    if (lp == q && lplace) {
      lrow0 = d.row0[q];
      lsc = (AT)d.scale[q];
    }
  if (!lplace) lsc = (AT)0;
  const DPiece<TG> *G = static_cast<const DPiece<TG> *>(d.val);
  const int64_t ldp = d.ld / VE;
  for (int r0 = wave; r0 < d.rows; r0 += U * NW) {
    DPiece<TG> g[U][MP];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = min(r0 + u * NW, d.rows - 1);   // clamped; surplus rows change nothing
#pragma unroll
      for (int q = 0; q < MP; ++q) {
        // lanes past the row's end re-read its last piece (their terms are
        // masked below), so every load of the pass is issued unconditionally
        const int pc = min(lane + 64 * q, npieces - 1);
        g[u][q] = G[(int64_t)r * ldp + pc];
      }
    }
    const int lr = r0 + lu * NW;
    const int lrc = min(lr, d.rows - 1);
    const AT tl = (AT)t[lrow0 + lrc], rl = (AT)rho_hat[lrow0 + lrc];
    // the U rows' dot products, summed over the wave together
    AT dots[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      dots[u] = 0;
#pragma unroll
      for (int q = 0; q < MP; ++q)
#pragma unroll
        for (int e = 0; e < VE; ++e) dots[u] += (AT)g[u][q].v[e] * xv[q][e];   // xv is 0 past the row's end
    }
    wave_sums<U>(dots);
    AT dl = dots[0];
#pragma unroll
    for (int u = 1; u < U; ++u) dl = lu == u ? dots[u] : dl;
    const AT ti = rl * (tl + lsc * dl);
    if (lane < 4 * U && lplace && lr < d.rows) t[lrow0 + lr] = (TT)ti;
    AT wl = lsc * ti;
    wl += __shfl_xor(wl, 1, 64);
    wl += __shfl_xor(wl, 2, 64);   // lane 4u: row u's weight
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (r0 + u * NW < d.rows) {
        const AT w = read_lane(wl, 4 * u);
#pragma unroll
        for (int q = 0; q < MP; ++q)
#pragma unroll
          for (int e = 0; e < VE; ++e) acc[q][e] += w * (AT)g[u][q].v[e];   // entries past cols are never read
      }
    }
  }
  // partials of the waves, added in wave order
#pragma unroll
  for (int q = 0; q < MP; ++q)
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int c = (lane + 64 * q) * VE + e;
      if (c < d.cols) lds[wave * d.cols + c] = acc[q][e];
    }
  __syncthreads();
  for (int c = threadIdx.x; c < d.cols; c += NTH) {
    AT sum = 0;
    for (int w = 0; w < NW; ++w) sum += lds[w * d.cols + c];
    ec[d.coff + c] = (double)sum;
  }
  __syncthreads();   // the partials are read before the next block overwrites them
}

// DMP: pieces per lane the kernel instantiation holds (the plan's widest
// block fits in it); TG: the stored type of the blocks' values.
template <int NTH, int DMP, typename AT, typename TG, typename T, typename TT>
__device__ inline void dense_fused(const View<T> &v, int b, const T *rho_hat, const T *vin, TT *t) {
  extern __shared__ double dyn_lds[];
  AT *lds = reinterpret_cast<AT *>(dyn_lds);
  for (int k = v.dense_inst[b]; k < v.dense_inst[b + 1]; ++k)
    dense_block_fused<NTH, DMP, AT, TG>(v.dense[k], rho_hat, vin, t, lds, v.ec);
}

// t = rho_hat o (A vin), then out = A' t + P vin + sigma vin, over the
// instances [b0, b1), with sync() between and after the halves (workgroup
// barrier in the per-instance form, grid barrier in the cooperative form).
template <int NTH, bool GRID, int DMP = 0, typename TG = float, typename T, typename RowAct, typename ColAct,
          typename Sync>
__device__ inline void op_apply(const View<T> &v, const T *__restrict__ rho_hat, const T *__restrict__ vin,
                                T *__restrict__ t, T *__restrict__ out, int b0, int b1, RowAct row_act,
                                ColAct col_act, Sync sync) {
  const int64_t B1 = v.B + 1;
  class_passes<NTH, GRID, T>(v.rowsA, v.spanA, v.instA, B1, b0, b1, v.A_col, v.A_val, vin, row_act,
                             [&](int32_t i, T acc) { t[i] = (v.drow && v.drow[i] >= 0) ? acc : rho_hat[i] * acc; });
  sync();
  if constexpr (!GRID && DMP > 0) {
    if (v.dense) {
      dense_fused<NTH, DMP, T, TG>(v, b0, rho_hat, vin, t);
      sync();
    }
  }
  class_passes<NTH, GRID, T>(v.rowsAt, v.spanAt, v.instAt, B1, b0, b1, v.At_col, v.At_val, t, col_act,
                             [&](int32_t j, T acc) {
                               if (v.P_rowptr)
                                 for (int64_t k = v.P_rowptr[j]; k < v.P_rowptr[j + 1]; ++k)
                                   acc += v.P_val[k] * vin[v.P_col[k]];
                               if (v.dcol && v.dcol[j] >= 0) acc += (T)v.ec[v.dcol[j]];
                               out[j] = acc + v.sigma * vin[j];
                             });
  sync();
}

// r = rhs - M x with float64 accumulation (t64 holds rho_hat o (A x) in
// float64); r is stored in the working precision.
template <int NTH, bool GRID, int DMP = 0, typename TG = float, typename T, typename RowAct, typename ColAct,
          typename Sync>
__device__ inline void op_residual64(const View<T> &v, const T *__restrict__ rho_hat, const double *__restrict__ rhs,
                                     const T *__restrict__ x, double *__restrict__ t64, T *__restrict__ r, int b0,
                                     int b1, RowAct row_act, ColAct col_act, Sync sync) {
  const int64_t B1 = v.B + 1;
  class_passes<NTH, GRID, double>(v.rowsA, v.spanA, v.instA, B1, b0, b1, v.A_col, v.A_val, x, row_act,
                                  [&](int32_t i, double acc) {
                                    t64[i] = (v.drow && v.drow[i] >= 0) ? acc : (double)rho_hat[i] * acc;
                                  });
  sync();
  if constexpr (!GRID && DMP > 0) {
    if (v.dense) {
      dense_fused<NTH, DMP, double, TG>(v, b0, rho_hat, x, t64);
      sync();
    }
  }
  class_passes<NTH, GRID, double>(v.rowsAt, v.spanAt, v.instAt, B1, b0, b1, v.At_col, v.At_val, t64, col_act,
                                  [&](int32_t j, double acc) {
                                    if (v.P_rowptr)
                                      for (int64_t k = v.P_rowptr[j]; k < v.P_rowptr[j + 1]; ++k)
                                        acc += (double)v.P_val[k] * (double)x[v.P_col[k]];
                                    if (v.dcol && v.dcol[j] >= 0) acc += v.ec[v.dcol[j]];
                                    r[j] = (T)(rhs[j] - acc - (double)v.sigma * (double)x[j]);
                                  });
  sync();
}

// Epilogue shared by both forms, over instance b's columns.
template <int NTH, typename T>
__device__ inline void finish(const View<T> &v, int b, bool fail, int it, int passes, double rrt, double thr, T *x,
                              const T *alpha_k, const T *xold, T *xnew, const T *gx_in, T *gx_out, int32_t mode,
                              cosmo_stats *stats) {
  const int64_t n0 = v.n_off[b], n1 = v.n_off[b + 1];
  if (fail)   // a non-finite system marks its solution, never a finite warm start
    for (int64_t j = n0 + threadIdx.x; j < n1; j += NTH) x[j] = (T)NAN;
  const T al = alpha_k ? alpha_k[b] : (T)1;
  if (mode == 0) {
    if (xnew)
      for (int64_t j = n0 + threadIdx.x; j < n1; j += NTH) xnew[j] = al * x[j] + ((T)1 - al) * xold[j];
  } else {
    for (int64_t j = n0 + threadIdx.x; j < n1; j += NTH) gx_out[j] = ((T)1 - al) * gx_in[j] + v.sigma * x[j];
  }
  if (stats && threadIdx.x == 0) {
    atomicMax(&stats[b].cg_iters_max, it);
    atomicAdd(&stats[b].cg_iters_total, it);
    atomicAdd(&stats[b].cg_passes_total, passes);
    if (!(rrt <= thr)) atomicAdd(&stats[b].cg_not_converged, 1);
  }
}

// ---- per-instance form -------------------------------------------------------------

template <typename T, int DMP, typename TG = T>
__global__ __launch_bounds__((PTK<T, DMP>)) void k_pcg(View<T> v, const T *__restrict__ rho_hat, const T *__restrict__ dg,
                                            const double *__restrict__ rhs, T *__restrict__ x, T *__restrict__ r,
                                            T *__restrict__ z, T *__restrict__ p, T *__restrict__ Mp,
                                            T *__restrict__ t, double *__restrict__ t64, T tol, int32_t max_iter,
                                            const T *__restrict__ alpha_k, const T *__restrict__ xold,
                                            T *__restrict__ xnew, const T *__restrict__ gx_in,
                                            T *__restrict__ gx_out, int32_t mode, cosmo_stats *stats) {
  __shared__ T red[2 * (PTK<T, DMP> / 64)];
  __shared__ double redd[2 * (PTK<T, DMP> / 64)];
  const int b = blockIdx.x;
  const int64_t n0 = v.n_off[b], n1 = v.n_off[b + 1];
  auto all = [](int32_t) { return true; };
  auto bar = []() { __syncthreads(); };

  double bb = 0, dd = 0;
  for (int64_t j = n0 + threadIdx.x; j < n1; j += PTK<T, DMP>) bb += rhs[j] * rhs[j];
  wg_sum2<PTK<T, DMP>>(bb, dd, redd);
  const double thr = (double)tol * (double)tol * bb;
  bool fail = !isfinite(bb);
  int it = 0, passes = 0;
  double rrt = 0, rrt_prev = 0;
  for (int restart = 0;; ++restart) {
    // true residual, z = r / diag M, p = z
    op_residual64<PTK<T, DMP>, false, DMP, TG>(v, rho_hat, rhs, x, t64, r, b, b + 1, all, all, bar);
    ++passes;
    T rz = 0, rr = 0;
    rrt = 0;
    for (int64_t j = n0 + threadIdx.x; j < n1; j += PTK<T, DMP>) {
      const T rj = r[j];
      const T zj = rj / dg[j];
      z[j] = zj;
      p[j] = zj;
      rz += rj * zj;
      rr += rj * rj;
      rrt += (double)rj * (double)rj;
    }
    wg_sum2<PTK<T, DMP>>(rz, rr, red);
    wg_sum2<PTK<T, DMP>>(rrt, dd, redd);
    fail = fail || !isfinite(rrt);
    const bool stalled = restart > 0 && rrt > STALL2 * rrt_prev;
    if (fail || rrt <= thr || it >= max_iter || restart > NRESTART || stalled) break;
    rrt_prev = rrt;
    const T target = (T)(restart == 0 ? thr : fmax(thr, ROUND_DROP2 * (double)rr));
    // CG on the recursive residual
    while (rr > target && it < max_iter) {
      __syncthreads();   // p complete before the operator reads it
      op_apply<PTK<T, DMP>, false, DMP, TG>(v, rho_hat, p, t, Mp, b, b + 1, all, all, bar);
      T pMp = 0, dummy = 0;
      for (int64_t j = n0 + threadIdx.x; j < n1; j += PTK<T, DMP>) pMp += p[j] * Mp[j];
      wg_sum2<PTK<T, DMP>>(pMp, dummy, red);
      if (!(pMp > (T)0)) {   // breakdown: restart from the true residual (or fail if non-finite)
        fail = !isfinite(pMp);
        break;
      }
      const T a = rz / pMp;
      T rz_new = 0, rr_new = 0;
      for (int64_t j = n0 + threadIdx.x; j < n1; j += PTK<T, DMP>) {
        x[j] += a * p[j];
        const T rj = r[j] - a * Mp[j];
        const T zj = rj / dg[j];
        r[j] = rj;
        z[j] = zj;
        rz_new += rj * zj;
        rr_new += rj * rj;
      }
      wg_sum2<PTK<T, DMP>>(rz_new, rr_new, red);
      const T beta = rz_new / rz;
      rz = rz_new;
      rr = rr_new;
      for (int64_t j = n0 + threadIdx.x; j < n1; j += PTK<T, DMP>) p[j] = z[j] + beta * p[j];
      ++it;
      if (!isfinite(rr)) {
        fail = true;
        break;
      }
    }
    if (fail) break;
    __syncthreads();   // x complete before the residual reads it
  }
  __syncthreads();
  finish<PTK<T, DMP>>(v, b, fail, it, passes, rrt, thr, x, alpha_k, xold, xnew, gx_in, gx_out, mode, stats);
}

// ---- cooperative form ------------------------------------------------------------

constexpr uint64_t BAR_TIMEOUT_TICKS = 200000000ull;   // 2 s of the 100 MHz real-time counter

// Barrier words of one cooperative solve, each in its own 256-byte line,
// zeroed on the stream before the launch.
struct GridBar {
  uint32_t *count, *gen, *abort;
  uint32_t nblk;
};

// Returns true once any wait of this solve has run out of time.
__device__ inline bool grid_barrier(const GridBar &gb, uint32_t &gen, int32_t *shared_flag) {
  __syncthreads();   // the workgroup's stores are complete (workgroup-scope release in every wave)
  const uint32_t target = gen + 1;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (__hip_atomic_fetch_add(gb.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gb.nblk - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(gb.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(gb.gen, target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      while (__hip_atomic_load(gb.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != target) {
        if (__hip_atomic_load(gb.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if (__builtin_amdgcn_s_memrealtime() - t0 > BAR_TIMEOUT_TICKS) {
          __hip_atomic_store(gb.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    *shared_flag = __hip_atomic_load(gb.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  }
  gen = target;
  __syncthreads();
  return *shared_flag != 0;
}

// Zeroes the barrier words before a cooperative solve.
__global__ void k_bar_reset(uint32_t *words) {
  if (threadIdx.x < 3) words[64 * threadIdx.x] = 0;
}

// Per-instance state of the cooperative solve (caller workspace, 16 (B + 1)
// + 256 elements of T): the three barrier words (768 bytes), then rz, rr,
// tgt [B] in T, thr, rrt, rrt_prev [B] in float64, then int32 it, act, done,
// fail, passes [B] and two counters.
template <typename T> struct CoopState {
  T *rz, *rr, *tgt;
  double *thr, *rrt, *rrt_prev;
  int32_t *it, *act, *done, *fail, *passes, *cnt;
};

constexpr size_t BAR_BYTES = 768;

template <typename T> __device__ inline CoopState<T> coop_state(void *ws, int B) {
  CoopState<T> c;
  char *base = static_cast<char *>(ws) + BAR_BYTES;
  c.rz = reinterpret_cast<T *>(base);
  c.rr = c.rz + B;
  c.tgt = c.rr + B;
  const size_t dbl = (3 * (size_t)B * sizeof(T) + 7) / 8 * 8;   // 8-byte aligned (the workspace is 256-aligned)
  c.thr = reinterpret_cast<double *>(base + dbl);
  c.rrt = c.thr + B;
  c.rrt_prev = c.rrt + B;
  int32_t *i = reinterpret_cast<int32_t *>(c.rrt_prev + B);
  c.it = i;
  c.act = i + B;
  c.done = i + 2 * B;
  c.fail = i + 3 * B;
  c.passes = i + 4 * B;
  c.cnt = i + 5 * B;
  return c;
}

template <typename T>
__global__ __launch_bounds__(CT) void k_pcg_coop(View<T> v, const T *__restrict__ rho_hat, const T *__restrict__ dg,
                                                 const double *__restrict__ rhs, T *__restrict__ x, T *__restrict__ r,
                                                 T *__restrict__ z, T *__restrict__ p, T *__restrict__ Mp,
                                                 T *__restrict__ t, double *__restrict__ t64, T tol,
                                                 int32_t max_iter, const T *__restrict__ alpha_k,
                                                 const T *__restrict__ xold, T *__restrict__ xnew,
                                                 const T *__restrict__ gx_in, T *__restrict__ gx_out, int32_t mode,
                                                 cosmo_stats *stats, void *state) {
  __shared__ T red[2 * (CT / 64)];
  __shared__ double redd[2 * (CT / 64)];
  __shared__ int32_t bar_flag;
  constexpr int VU = VLOOP<T>;
  const CoopState<T> cs = coop_state<T>(state, v.B);
  uint32_t *words = static_cast<uint32_t *>(state);
  const GridBar gb{words, words + 64, words + 128, gridDim.x};
  uint32_t gen = 0;
  bool aborted = false;
  auto gsync = [&]() { aborted = grid_barrier(gb, gen, &bar_flag) || aborted; };
  auto row_open = [&](int32_t i) { return cs.done[v.row_inst[i]] == 0; };
  auto col_open = [&](int32_t j) { return cs.done[v.col_inst[j]] == 0; };
  auto row_act = [&](int32_t i) { return cs.act[v.row_inst[i]] != 0; };
  auto col_act = [&](int32_t j) { return cs.act[v.col_inst[j]] != 0; };
  // Decision points: producers add to cnt[cur]; after a barrier every
  // workgroup reads it, workgroup 0 clears the other slot for the next
  // producer (which comes at least one barrier later), and cur flips.
  int cur = 0;
  auto decide = [&]() {
    const int n = __hip_atomic_load(&cs.cnt[cur], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (blockIdx.x == 0 && threadIdx.x == 0) cs.cnt[cur ^ 1] = 0;
    cur ^= 1;
    return n;
  };

  for (int b = blockIdx.x * CT + threadIdx.x; b < v.B; b += gridDim.x * CT) {
    cs.done[b] = 0;
    cs.act[b] = 0;
    cs.it[b] = 0;
    cs.passes[b] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x < 2) cs.cnt[threadIdx.x] = 0;
  for (int b = blockIdx.x; b < v.B; b += gridDim.x) {
    double bb = 0, dd = 0;
    for (int64_t j = v.n_off[b] + threadIdx.x; j < v.n_off[b + 1]; j += CT) bb += rhs[j] * rhs[j];
    wg_sum2<CT>(bb, dd, redd);
    if (threadIdx.x == 0) {
      cs.thr[b] = (double)tol * (double)tol * bb;
      cs.fail[b] = !isfinite(bb);
    }
  }
  gsync();
  for (int restart = 0; !aborted; ++restart) {
    // true residual of the instances not done; z, p; which go on
    op_residual64<CT, true>(v, rho_hat, rhs, x, t64, r, 0, v.B, row_open, col_open, gsync);
    if (aborted) break;
    for (int b = blockIdx.x; b < v.B; b += gridDim.x) {
      if (cs.done[b]) continue;
      const int64_t n0 = v.n_off[b], n1 = v.n_off[b + 1];
      T rz = 0, rr = 0;
      double rrt = 0, dd = 0;
      // VU strides per pass, loads first (one workgroup streams the whole
      // instance here); each thread still adds in index order
      int64_t j = n0 + threadIdx.x;
      for (; j + (VU - 1) * CT < n1; j += VU * CT) {
        T rv[VU], dv[VU];
#pragma unroll
        for (int u = 0; u < VU; ++u) {
          rv[u] = r[j + u * CT];
          dv[u] = dg[j + u * CT];
        }
#pragma unroll
        for (int u = 0; u < VU; ++u) {
          const T rj = rv[u];
          const T zj = rj / dv[u];
          z[j + u * CT] = zj;
          p[j + u * CT] = zj;
          rz += rj * zj;
          rr += rj * rj;
          rrt += (double)rj * (double)rj;
        }
      }
      for (; j < n1; j += CT) {
        const T rj = r[j];
        const T zj = rj / dg[j];
        z[j] = zj;
        p[j] = zj;
        rz += rj * zj;
        rr += rj * rj;
        rrt += (double)rj * (double)rj;
      }
      wg_sum2<CT>(rz, rr, red);
      wg_sum2<CT>(rrt, dd, redd);
      if (threadIdx.x == 0) {
        const bool fail = cs.fail[b] || !isfinite(rrt);
        const bool stalled = restart > 0 && rrt > STALL2 * cs.rrt_prev[b];
        const bool done = fail || rrt <= cs.thr[b] || cs.it[b] >= max_iter || restart > NRESTART || stalled;
        const T tgt = (T)(restart == 0 ? cs.thr[b] : fmax(cs.thr[b], ROUND_DROP2 * (double)rr));
        cs.rz[b] = rz;
        cs.rr[b] = rr;
        cs.tgt[b] = tgt;
        cs.rrt[b] = rrt;
        cs.rrt_prev[b] = rrt;
        cs.passes[b] += 1;
        cs.fail[b] = fail;
        cs.done[b] = done;
        cs.act[b] = !done && rr > tgt;
        if (!done) atomicAdd(&cs.cnt[cur], 1);
      }
    }
    gsync();
    if (aborted || decide() == 0) break;
    // CG on the recursive residual until no instance is active
    for (;;) {
      op_apply<CT, true>(v, rho_hat, p, t, Mp, 0, v.B, row_act, col_act, gsync);
      if (aborted) break;
      for (int b = blockIdx.x; b < v.B; b += gridDim.x) {
        if (!cs.act[b]) continue;
        const int64_t n0 = v.n_off[b], n1 = v.n_off[b + 1];
        T pMp = 0, dummy = 0;
        {
          int64_t j = n0 + threadIdx.x;
          for (; j + (VU - 1) * CT < n1; j += VU * CT) {
            T pv[VU], mv[VU];
#pragma unroll
            for (int u = 0; u < VU; ++u) {
              pv[u] = p[j + u * CT];
              mv[u] = Mp[j + u * CT];
            }
#pragma unroll
            for (int u = 0; u < VU; ++u) pMp += pv[u] * mv[u];
          }
          for (; j < n1; j += CT) pMp += p[j] * Mp[j];
        }
        wg_sum2<CT>(pMp, dummy, red);
        const T rz = cs.rz[b];
        const bool step = pMp > (T)0;   // else breakdown: back to the true residual (fail if non-finite)
        bool fail = step ? false : !isfinite(pMp);
        bool act = false;
        T rz_new = 0, rr_new = 0;
        if (step) {
          const T a = rz / pMp;
          int64_t j = n0 + threadIdx.x;
          for (; j + (VU - 1) * CT < n1; j += VU * CT) {
            T pv[VU], mv[VU], xv[VU], rv[VU], dv[VU];
#pragma unroll
            for (int u = 0; u < VU; ++u) {
              pv[u] = p[j + u * CT];
              mv[u] = Mp[j + u * CT];
              xv[u] = x[j + u * CT];
              rv[u] = r[j + u * CT];
              dv[u] = dg[j + u * CT];
            }
#pragma unroll
            for (int u = 0; u < VU; ++u) {
              x[j + u * CT] = xv[u] + a * pv[u];
              const T rj = rv[u] - a * mv[u];
              const T zj = rj / dv[u];
              r[j + u * CT] = rj;
              z[j + u * CT] = zj;
              rz_new += rj * zj;
              rr_new += rj * rj;
            }
          }
          for (; j < n1; j += CT) {
            x[j] += a * p[j];
            const T rj = r[j] - a * Mp[j];
            const T zj = rj / dg[j];
            r[j] = rj;
            z[j] = zj;
            rz_new += rj * zj;
            rr_new += rj * rj;
          }
          wg_sum2<CT>(rz_new, rr_new, red);
          const T beta = rz_new / rz;
          j = n0 + threadIdx.x;
          for (; j + (VU - 1) * CT < n1; j += VU * CT) {
            T zv[VU], pv[VU];
#pragma unroll
            for (int u = 0; u < VU; ++u) {
              zv[u] = z[j + u * CT];
              pv[u] = p[j + u * CT];
            }
#pragma unroll
            for (int u = 0; u < VU; ++u) p[j + u * CT] = zv[u] + beta * pv[u];
          }
          for (; j < n1; j += CT) p[j] = z[j] + beta * p[j];
          fail = !isfinite(rr_new);
          act = !fail && rr_new > cs.tgt[b] && cs.it[b] + 1 < max_iter;
        }
        __syncthreads();   // every thread has read the scalars before they change
        if (threadIdx.x == 0) {
          if (step) {
            cs.rz[b] = rz_new;
            cs.rr[b] = rr_new;
            cs.it[b] += 1;
          }
          if (fail) {
            cs.fail[b] = 1;
            cs.done[b] = 1;
          }
          cs.act[b] = act;
          if (act) atomicAdd(&cs.cnt[cur], 1);
        }
      }
      gsync();
      if (aborted || decide() == 0) break;
    }
  }
  // after an abort the solutions are marked non-finite (the state of the
  // instances is not trusted)
  for (int b = blockIdx.x; b < v.B; b += gridDim.x)
    finish<CT>(v, b, aborted || cs.fail[b] != 0, cs.it[b], cs.passes[b], cs.rrt[b], cs.thr[b], x, alpha_k, xold, xnew, gx_in,
               gx_out, mode, stats);
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
void launch_pcg(const View<T> &v, const T *rho_hat, const T *dg, const double *rhs, T *x, T *r, T *z, T *p, T *Mp, T *t,
                double *t64, double tol, int32_t max_iter, const T *alpha_k, const T *xold, T *xnew,
                const T *gx_in, T *gx_out, int32_t mode, cosmo_stats *stats, void *state, int32_t form,
                hipStream_t st) {
  // form 0: one workgroup per instance; form f > 0: the cooperative form
  // with at most f workgroups per compute unit (the runtime refuses a grid
  // that would not be resident at once; the per-instance form then runs)
  const int grid = (form > 0 && state && v.n_dense == 0) ? pcg_coop_grid<T>(form) : 0;
  if (grid > 0) {
    View<T> va = v;
    T tl = (T)tol;
    int32_t mi = max_iter, md = mode;
    void *args[] = {&va, &rho_hat, &dg,   &rhs,  &x,     &r,      &z,  &p,     &Mp,    &t,   &t64,
                    &tl, &mi,      &alpha_k, &xold, &xnew, &gx_in, &gx_out, &md, &stats, &state};
    k_bar_reset<<<1, 64, 0, st>>>(static_cast<uint32_t *>(state));
    if (hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_pcg_coop<T>), dim3(grid), dim3(CT), args, 0,
                                   st) == hipSuccess)
      return;
    (void)hipGetLastError();
  }
  if (v.n_dense <= 0) {
    k_pcg<T, 0><<<v.B, PT<T>, 0, st>>>(v, rho_hat, dg, rhs, x, r, z, p, Mp, t, t64, (T)tol, max_iter, alpha_k, xold,
                                       xnew, gx_in, gx_out, mode, stats);
    return;
  }
  // dense sub-blocks: the instantiation for the blocks' stored type holding
  // the widest block's pieces, and LDS for the waves' partials of G'w
  // (float64 in the residual pass)
  const size_t lds = (size_t)(512 / 64) * v.dense_maxcols * sizeof(double);
  auto go = [&](auto kern) {
    static bool attr_set = false;   // more than the default 64 KiB of dynamic LDS may be needed
    if (!attr_set) {
      hipFuncAttributes a{};
      size_t stat = 4096;
      if (hipFuncGetAttributes(&a, reinterpret_cast<const void *>(kern)) == hipSuccess) stat = a.sharedSizeBytes;
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(163840 - stat));
      attr_set = true;
    }
    kern<<<v.B, 512, lds, st>>>(v, rho_hat, dg, rhs, x, r, z, p, Mp, t, t64, (T)tol, max_iter, alpha_k, xold, xnew,
                                  gx_in, gx_out, mode, stats);
  };
  auto pick = [&](auto tg) {
    using TG = decltype(tg);
    constexpr int VE = 16 / sizeof(TG);
    const int pieces = (v.dense_maxcols + 64 * VE - 1) / (64 * VE);
    if (pieces <= MAXPC<TG> / 4) go(&k_pcg<T, MAXPC<TG> / 4, TG>);
    else if (pieces <= MAXPC<TG> / 2) go(&k_pcg<T, MAXPC<TG> / 2, TG>);
    else go(&k_pcg<T, MAXPC<TG>, TG>);
  };
  if (sizeof(T) == 8 && v.dense_g32) pick(float{});
  else pick(T{});
}

template void launch_pcg<float>(const View<float> &, const float *, const float *, const double *, float *, float *,
                                float *, float *, float *, float *, double *, double, int32_t, const float *,
                                const float *, float *, const float *, float *, int32_t, cosmo_stats *, void *,
                                int32_t, hipStream_t);
template void launch_pcg<double>(const View<double> &, const double *, const double *, const double *, double *,
                                 double *, double *, double *, double *, double *, double *, double, int32_t,
                                 const double *, const double *, double *, const double *, double *, int32_t,
                                 cosmo_stats *, void *, int32_t, hipStream_t);

}  // namespace cosmo
