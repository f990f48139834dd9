// Products with the dense sub-blocks of A outside the CG (the right-hand side
// and Jacobi diagonal of the reduced system, the slack pass, the reverse
// passes and the residual loss).  A dense block G is applied as such, read
// once per product in 16-byte pieces, instead of as CSR with an index per
// entry: the method needs A only through products with vectors (Sec.
// "Matrix-Free Implicit Differentiation", O(n + nnz(A)) per application).
//
// Row products   dn[doff + r] = sum_c G_rc vin[col0 + c]
//   one wave per row, a row's pieces spread over the 64 lanes, four rows in
//   flight per wave, float64 accumulation, the four rows summed over the
//   wave together (fixed order).
// Column products ec[coff + c] = sum_r G_rc w_r  (and ed = sum_r G_rc^2 wd_r)
//   one workgroup per (block, 64-piece column strip); the workgroup first
//   forms the row weights of a tile of 2048 rows in LDS (w_r sums the
//   placements' scale times the mode's per-row value), then its four waves
//   walk a quarter of the tile each, every lane owning one piece of the
//   strip; the four waves' partial sums are added in wave order.  Sums are
//   float64 and deterministic.
#include "cosmo_internal.h"
#include "wave_ops.h"

namespace cosmo {
namespace {

constexpr int NT = 256;
constexpr int NW = NT / 64;
constexpr int ROWS_PER_WG = 64;     // row products: 16 rows per wave
constexpr int TILE = 2048;          // column products: rows per weight tile (one tile for most blocks)

template <typename T> struct alignas(16) Piece {
  T v[16 / sizeof(T)];
};


// Block of the launch's workgroup: the last descriptor whose first workgroup
// is <= blockIdx.x (descriptors are in increasing order of it).
template <bool ROWS> __device__ inline int find_block(const DenseDesc *dd, int32_t nd) {
  int lo = 0, hi = nd - 1;
  const int32_t g = (int32_t)blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int32_t w0 = ROWS ? dd[mid].wg_rows0 : dd[mid].wg_cols0;
    if (w0 <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Pieces per lane needed for up to COSMO_DENSE_MAX_COLS columns.
template <typename T> constexpr int MAXP = COSMO_DENSE_MAX_COLS / (64 * (16 / (int)sizeof(T)));

// T: the plan's arithmetic type; TG: the stored type of the blocks' values.
template <typename T, typename TG>
__global__ __launch_bounds__(NT) void k_dense_rows(const DenseDesc *__restrict__ dd, int32_t nd,
                                                   const T *__restrict__ vin, double *__restrict__ dn) {
  constexpr int VE = 16 / sizeof(TG);
  constexpr int MP = MAXP<TG>;
  const DenseDesc d = dd[find_block<true>(dd, nd)];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int npieces = (d.cols + VE - 1) / VE;
  // this lane's pieces of vin (zero beyond the block's columns)
  double xv[MP][VE];
#pragma unroll
  for (int q = 0; q < MP; ++q)
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      const int c = (lane + 64 * q) * VE + e;
      xv[q][e] = c < d.cols ? (double)vin[d.col0 + c] : 0.0;
    }
  const Piece<TG> *G = static_cast<const Piece<TG> *>(d.val);
  const int64_t ldp = d.ld / VE;   // pieces per row
  const int r_begin = (int)(blockIdx.x - d.wg_rows0) * ROWS_PER_WG + wave;
  const int r_end = min(d.rows, (int)(blockIdx.x - d.wg_rows0 + 1) * ROWS_PER_WG);
  constexpr int U = 4;
  for (int r0 = r_begin; r0 < r_end; r0 += U * NW) {
    Piece<TG> g[U][MP];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = min(r0 + u * NW, r_end - 1);   // clamped; surplus rows are not written
#pragma unroll
      for (int q = 0; q < MP; ++q)
        if (q * 64 < npieces)   // uniform over the wave: pieces the block has
          g[u][q] = G[(int64_t)r * ldp + min(lane + 64 * q, npieces - 1)];   // past the end: its last piece
    }
    // xv is zero past the block's columns, so the re-read pieces add nothing
    double dots[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      dots[u] = 0.0;
#pragma unroll
      for (int q = 0; q < MP; ++q)
        if (q * 64 < npieces)
#pragma unroll
          for (int e = 0; e < VE; ++e) dots[u] += (double)g[u][q].v[e] * xv[q][e];
    }
    wave_sums<U>(dots);
    // lane u writes row u's product: one store per pass
    double mine = dots[0];
#pragma unroll
    for (int u = 1; u < U; ++u) mine = lane == u ? dots[u] : mine;
    if (lane < U && r0 + lane * NW < r_end) dn[d.doff + r0 + lane * NW] = mine;
  }
}

struct ColArgs {
  int32_t mode;
  const void *rho_hat, *u, *s, *b;
};

template <typename T>
__device__ inline void row_weights(const DenseDesc &d, const ColArgs &a, int r, double &w, double &wd) {
  const T *rh = static_cast<const T *>(a.rho_hat);
  const T *u = static_cast<const T *>(a.u);
  w = 0.0;
  wd = 0.0;
  for (int p = 0; p < d.nplace; ++p) {
    const int64_t i = d.row0[p] + r;
    const double sc = d.scale[p];
    double ui;
    if (a.mode == DC_XI) {
      const T *s = static_cast<const T *>(a.s);
      const T *b = static_cast<const T *>(a.b);
      ui = (double)u[i] + (double)rh[i] * ((double)b[i] - (double)s[i]);
    } else {
      ui = (double)u[i];
    }
    w += sc * ui;
    if (a.mode == DC_XI || a.mode == DC_GST) wd += sc * sc * (double)rh[i];
  }
}

template <typename T, typename TG>
__global__ __launch_bounds__(NT) void k_dense_cols(const DenseDesc *__restrict__ dd, int32_t nd, ColArgs a,
                                                   double *__restrict__ ec, double *__restrict__ ed) {
  constexpr int VE = 16 / sizeof(TG);
  __shared__ double wt[TILE], wdt[TILE];
  __shared__ double part[2][NW][64 * VE];
  const DenseDesc d = dd[find_block<false>(dd, nd)];
  const bool diag = a.mode == DC_XI || a.mode == DC_GST;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int npieces = (d.cols + VE - 1) / VE;
  const int pc = (int)(blockIdx.x - d.wg_cols0) * 64 + lane;   // this lane's piece of the strip
  const bool has = pc < npieces;
  const Piece<TG> *G = static_cast<const Piece<TG> *>(d.val);
  const int64_t ldp = d.ld / VE;
  double acc[VE], accd[VE];
#pragma unroll
  for (int e = 0; e < VE; ++e) acc[e] = accd[e] = 0.0;
  for (int t0 = 0; t0 < d.rows; t0 += TILE) {
    const int nr = min(TILE, d.rows - t0);
    __syncthreads();   // the previous tile's weights are no longer read
    for (int i = threadIdx.x; i < nr; i += NT) {
      double w, wd;
      row_weights<T>(d, a, t0 + i, w, wd);
      wt[i] = w;
      wdt[i] = wd;
    }
    __syncthreads();
    const int q0 = wave * (TILE / NW);
    const int q1 = min(nr, q0 + TILE / NW);
    constexpr int U = 8;
    for (int q = q0; q < q1; q += U) {
      Piece<TG> g[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = min(q + u, q1 - 1);
        if (has) g[u] = G[(int64_t)(t0 + r) * ldp + pc];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (q + u < q1 && has) {
          const double w = wt[q + u], wd = wdt[q + u];
#pragma unroll
          for (int e = 0; e < VE; ++e) {
            const double gv = (double)g[u].v[e];
            acc[e] += gv * w;
            if (diag) accd[e] += gv * gv * wd;
          }
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < VE; ++e) {
    part[0][wave][lane * VE + e] = acc[e];
    part[1][wave][lane * VE + e] = accd[e];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 64 * VE; k += NT) {
    const int c = ((int)(blockIdx.x - d.wg_cols0) * 64) * VE + k;
    if (c >= d.cols) continue;
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < NW; ++w) {
      s0 += part[0][w][k];
      s1 += part[1][w][k];
    }
    ec[d.coff + c] = s0;
    if (diag) ed[d.coff + c] = s1;
  }
}

}  // namespace

template <typename T> void launch_dense_rows(const View<T> &v, const T *vin, hipStream_t st) {
  if (v.n_dense <= 0 || v.dense_wg_rows <= 0) return;
  if (sizeof(T) == 8 && v.dense_g32)
    k_dense_rows<T, float><<<v.dense_wg_rows, NT, 0, st>>>(v.dense, v.n_dense, vin, v.dn);
  else
    k_dense_rows<T, T><<<v.dense_wg_rows, NT, 0, st>>>(v.dense, v.n_dense, vin, v.dn);
}

template <typename T>
void launch_dense_cols(const View<T> &v, int32_t mode, const T *rho_hat, const T *u, const T *s, hipStream_t st) {
  if (v.n_dense <= 0 || v.dense_wg_cols <= 0) return;
  ColArgs a{mode, rho_hat, u, s, v.b};
  if (sizeof(T) == 8 && v.dense_g32)
    k_dense_cols<T, float><<<v.dense_wg_cols, NT, 0, st>>>(v.dense, v.n_dense, a, v.ec, v.ed);
  else
    k_dense_cols<T, T><<<v.dense_wg_cols, NT, 0, st>>>(v.dense, v.n_dense, a, v.ec, v.ed);
}

// Workgroup counts of the two launches for a block (the host lays out
// DenseDesc::wg_rows0 / wg_cols0 with these); esz: bytes per stored value.
int32_t dense_row_workgroups(int32_t rows) { return (rows + ROWS_PER_WG - 1) / ROWS_PER_WG; }
int32_t dense_col_workgroups(int32_t cols, size_t esz) {
  const int32_t strip = 64 * (int32_t)(16 / esz);
  return (cols + strip - 1) / strip;
}

template void launch_dense_rows<float>(const View<float> &, const float *, hipStream_t);
template void launch_dense_rows<double>(const View<double> &, const double *, hipStream_t);
template void launch_dense_cols<float>(const View<float> &, int32_t, const float *, const float *, const float *,
                                       hipStream_t);
template void launch_dense_cols<double>(const View<double> &, int32_t, const double *, const double *,
                                        const double *, hipStream_t);

}  // namespace cosmo
