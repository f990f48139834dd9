// Internal declarations shared by the host library and the kernel files.
// Not part of the public ABI (see include/cosmo_unroll.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "cosmo_unroll.h"

namespace cosmo {

// ---- device-side descriptors --------------------------------------------

enum RowKind : uint8_t { ROW_ZERO = 0, ROW_NONNEG = 1, ROW_SOC = 2, ROW_PSD = 3 };

struct SocDesc {      // one second-order cone block
  int64_t row0;       // first row
  int32_t dim;        // rows (t first, then w)
  int32_t inst;       // owning instance
};

struct PsdDesc {      // one PSD block in svec form
  int64_t row0;       // first row of its svec
  int64_t uoff;       // element offset of its p x p eigenvector block (column-major)
  int64_t loff;       // element offset of its p eigenvalues
  int32_t p;          // matrix order
  int32_t inst;       // owning instance
};

struct RectDesc {     // a block whose penalty is averaged (SOC or PSD)
  int64_t row0;
  int32_t rows;
  int32_t pad;
};

// One dense sub-block G of A (cosmo_dense_block) as the kernels see it: its
// placements, the instance owning it, and where its per-row and per-column
// results go in the dense scratch vectors (doff: rows, coff: columns).
struct DenseDesc {
  const void *val;    // rows x ld, row-major, the plan's dtype or float32 (View::dense_g32)
  int64_t ld;
  int64_t col0;
  int64_t doff, coff;
  int64_t row0[COSMO_DENSE_MAX_PLACEMENTS];
  double scale[COSMO_DENSE_MAX_PLACEMENTS];
  int32_t rows, cols;
  int32_t nplace, inst;
  int32_t wg_rows0;   // first workgroup of this block in a row-product launch
  int32_t wg_cols0;   // first workgroup of this block in a column-product launch
};

// Entry range [kb, k1) of one row, listed beside the bucket lists so a row's
// range is one 16-byte load rather than a load of the row id and then two of
// the row pointer.
struct alignas(16) RowSpan {
  int64_t kb, k1;
};

// Rows (or columns) of a CSR matrix grouped into three length classes so a
// sub-wave of L lanes serves one row with coalesced loads.
struct RowBuckets {
  int32_t *d_rows = nullptr;   // concatenated row ids of the three classes
  RowSpan *d_span = nullptr;   // entry range of each listed row
  int64_t begin[4] = {0, 0, 0, 0};
  int32_t lanes[3] = {1, 8, 64};
};

// ---- dtype traits ------------------------------------------------------------

template <typename T> struct Eps;
template <> struct Eps<float> { static constexpr double jacobi_tol = 2.0e-7; };
template <> struct Eps<double> { static constexpr double jacobi_tol = 1.0e-14; };

// ---- launch wrappers (defined in the .hip files) ----------------------------

struct ProblemDev;   // device-side view of a plan, passed by value to kernels

template <typename T> struct View {
  // problem (caller-owned)
  const int64_t *A_rowptr; const int32_t *A_col; const T *A_val;
  const int64_t *P_rowptr; const int32_t *P_col; const T *P_val;
  const T *q; const T *b;
  // plan-owned
  const int64_t *At_rowptr; const int32_t *At_col; const T *At_val;
  const T *Pdiag;
  const uint8_t *row_kind; const int32_t *row_inst; const int32_t *col_inst;
  const int64_t *n_off; const int64_t *m_off;
  // per instance b and row-length class c (1, 8, 64 lanes per row): its rows
  // of A (columns of A for At) are rowsA[instA[c (B+1) + b] .. instA[c (B+1) + b + 1])
  const int32_t *rowsA; const int32_t *rowsAt;
  const RowSpan *spanA; const RowSpan *spanAt;   // entry ranges, aligned with rowsA / rowsAt
  const int64_t *instA; const int64_t *instAt;
  int32_t B; int64_t n_tot, m_tot;
  T sigma;
  // dense sub-blocks (dense == nullptr: none).  dense_g32: the blocks' values
  // are stored as float32 (in a float64 View; a float32 View stores float32
  // anyway).  dense_inst[b] .. dense_inst[b + 1]
  // are instance b's blocks; drow[i] is row i's entry in dn (or -1) and
  // dscale[i] the scale of the placement covering it; dcol[j] is column j's
  // entry in ec / ed (or -1).  dn, ec, ed are float64 scratch vectors of the
  // call's workspace (block rows, block columns, block columns).
  const DenseDesc *dense; const int32_t *dense_inst;
  const int32_t *drow; const double *dscale; const int32_t *dcol;
  int32_t n_dense, dense_maxcols, dense_wg_rows, dense_wg_cols, dense_g32;
  double *dn; double *ec; double *ed;
};

// Outputs of the in-kernel diagonal solve (all null: the PCG kernel solves).
// Forward: xt = x~, xn = x+, alpha_k per instance.  Adjoint: xt = w,
// xn = the cotangent of x.
template <typename T> struct DiagSolve {
  T *xt = nullptr;
  T *xn = nullptr;
  const T *alpha_k = nullptr;
};

// vector / row-wise kernels (k_vec.hip)
template <typename T> void launch_rectify(const View<T> &v, const RectDesc *rect, int32_t nrect, const T *rho,
                                          T *rho_hat, int32_t K, hipStream_t st);
template <typename T> void launch_cols_pre(const View<T> &v, const RowBuckets &bk, const T *rho_hat, const T *x,
                                           const T *s, const T *y, T *dg, double *xi, DiagSolve<T> ds, hipStream_t st);
template <typename T> void launch_rows_post(const View<T> &v, const RowBuckets &bk, const T *rho_hat,
                                            const T *alpha_k, const T *xt, const T *s, const T *y, T *st_out,
                                            T *sh, T *vv, T *s_new, T *y_new, hipStream_t st);
template <typename T> void launch_bwd_rows_a(const View<T> &v, const T *rho_hat, const T *alpha_k, const T *stl,
                                             const T *s, const T *y, const T *s_new, const T *gs_in,
                                             const T *gy_in, T *gsn, T *gv, bool all_rows, hipStream_t st);
template <typename T> void launch_rows_v(const View<T> &v, const T *rho_hat, const T *alpha_k, const T *stl,
                                         const T *s, const T *y, T *vv, hipStream_t st);
template <typename T> void launch_bwd_rows_b(const View<T> &v, const T *rho_hat, const T *alpha_k, const T *stl,
                                             const T *s, const T *y, const T *s_new, const T *gy_in, const T *gv,
                                             T *gsh, T *gst, T *gs_out, T *gy_out, T *grh, const T *gst_extra,
                                             hipStream_t st);
template <typename T> void launch_bwd_cols(const View<T> &v, const RowBuckets &bk, const T *rho_hat,
                                           const T *alpha_k, const T *gst, const T *gx_in, double *gxt, T *dg,
                                           DiagSolve<T> ds, hipStream_t st);
template <typename T> void launch_bwd_rows_c(const View<T> &v, const RowBuckets &bk, const T *rho_hat,
                                             const T *w, const T *stl, const T *s, T *grh, T *gs_out,
                                             T *gy_out, hipStream_t st);
template <typename T> void launch_rect_adjoint(const View<T> &v, const RectDesc *rect, int32_t nrect,
                                               const T *grh, T *grho_k, hipStream_t st);
template <typename T> void launch_alpha_reduce(const View<T> &v, const T *gsh, const T *stl, const T *s,
                                               const T *gx_in, const T *xt, const T *x, T *galpha_k,
                                               hipStream_t st);
template <typename T> void launch_loss(const View<T> &v, const RowBuckets &bkA, const RowBuckets &bkAt,
                                       const T *x, const T *s, const T *y, T *rp, T *rd, T *loss, T *gx,
                                       T *gs, T *gy, hipStream_t st);
// ---- learned policy (k_policy.hip) ------------------------------------------------
// Two networks with hidden layers of POL_H: the per-row penalty network
// (POL_FR features) and the per-instance relaxation network (POL_FA); the
// flat parameter layout is the public header's (COSMO_POLICY_PARAMS).
constexpr int POL_H = 32, POL_FR = 7, POL_FA = 5;
constexpr int POL_RHO_PARAMS = POL_FR * POL_H + POL_H + POL_H * POL_H + POL_H + POL_H + 1;
constexpr int POL_ALPHA_PARAMS = POL_FA * POL_H + POL_H + POL_H * POL_H + POL_H + POL_H + 1;
constexpr int POL_L0 = POL_RHO_PARAMS + POL_ALPHA_PARAMS;   // 4 per-kind penalty logits, then alpha's
constexpr int POL_PARAMS = POL_L0 + 5;
constexpr int POL_WAVES = 2;                                 // waves per workgroup of the per-row network
constexpr int POL_PART_STRIDE = POL_RHO_PARAMS + 4;          // a workgroup's partial: the network, 4 kind sums
static_assert(POL_PARAMS == COSMO_POLICY_PARAMS, "policy parameter count");

// Per instance at one iterate: infinity norms of A x (nu), s, b, P x (np),
// q, A' y (nw), r_p, r_d, dp, dd; squared norms of r_p and r_d; how many
// entries attain each norm (ties).
struct PolRec {
  double nu, ns, nb, np, nq, nw, mrp, mrd, mdp, mdd, ssp, ssd;
  int32_t cu, cs, crp, cp, cw, crd, cdp, cdd;
};
// Per instance, the reverse step's coefficients: 1/N_p; the cotangent
// reaching each entry that attains a norm (already divided by the tie count)
// for r_p, A x, s, r_d, P x, A' y, dp, dd; and the loss term's 2/(D S).
struct PolCoef {
  double inv_np, c_rp, c_u, c_s, c_rd, c_p, c_w, c_dp, c_dd, cl_p, cl_d;
};
int64_t pol_row_blocks(int64_t m);
template <typename T> void launch_pol_norms(const View<T> &v, const T *u, const T *rp, const T *p, const T *w,
                                            const T *rd, const T *s, const T *s_prev, const T *st_prev, PolRec *rec,
                                            hipStream_t st);
template <typename T> void launch_pol_inst_fwd(const View<T> &v, const T *theta, const PolRec *rec, int32_t k,
                                               int32_t policy, const T *la_in, T *la_out, T *alpha_k, double *acc3,
                                               T *loss, hipStream_t st);
template <typename T> void launch_pol_rho_fwd(const View<T> &v, const T *theta, const PolRec *rec, const T *l_in,
                                              T *l_out, T *rho_k, const T *s, const T *y, const T *rp,
                                              const T *s_prev, const T *st_prev, hipStream_t st);
template <typename T> void launch_pol_rho_bwd(const View<T> &v, const T *theta, const PolRec *rec, const T *l_in,
                                              const T *s, const T *y, const T *rp, const T *s_prev,
                                              const T *st_prev, const T *grho_k, T *C, T *gs, T *gy, T *xb, T *part,
                                              hipStream_t st);
template <typename T> void launch_pol_inst_bwd(const View<T> &v, const T *theta, const PolRec *rec, int32_t k,
                                               int32_t policy, int32_t loss_term, const T *la_in, const T *galpha_k,
                                               T *Ca, const T *xb, const T *rp, const double *acc3, PolCoef *coef,
                                               T *parta, hipStream_t st);
template <typename T> void launch_pol_rows_bwd(const View<T> &v, const PolRec *rec, const PolCoef *coef, const T *xb,
                                               const T *rp, const T *u, const T *s, const T *s_prev,
                                               const T *st_prev, T *gs, T *ub, T *pend_st, T *pend_s,
                                               int32_t add_pend, int32_t write_pend, hipStream_t st);
template <typename T> void launch_pol_cols_bwd(const View<T> &v, const PolRec *rec, const PolCoef *coef, const T *rd,
                                               const T *p, const T *w, T *pb, T *wb, hipStream_t st);
template <typename T> void launch_pol_grad(const View<T> &v, const T *part, int64_t nblk, const T *parta, const T *Ca,
                                           T *gtheta, hipStream_t st);

// Learned policy (k_vec.hip): u = A x, rp = u + s - b, p = P x, w = A' y,
// rd = p + q - w; and the adjoint gx += A' ub + P pb, gy += A wb.
template <typename T> void launch_pol_resid(const View<T> &v, const RowBuckets &bkA, const RowBuckets &bkAt,
                                            const T *x, const T *s, const T *y, T *u, T *rp, T *p, T *w, T *rd,
                                            hipStream_t st);
template <typename T> void launch_pol_resid_adjoint(const View<T> &v, const RowBuckets &bkA, const RowBuckets &bkAt,
                                                    const T *ub, const T *pb, const T *wb, T *gx, T *gy,
                                                    hipStream_t st);
// Vanilla solve (k_vec.hip): rho[k][i] = rho_b[instance] (x eq_scale on zero rows), k < K.
template <typename T> void launch_solve_rho(const View<T> &v, const double *rho_b, double eq_scale, T *rho,
                                            int32_t K, hipStream_t st);
template <typename T> void launch_copy(T *dst, const T *src, int64_t n, hipStream_t st);
template <typename T> void launch_fill(T *dst, T val, int64_t n, hipStream_t st);
template <typename T> void launch_nonfinite_check(const View<T> &v, const T *x, const T *s, const T *y,
                                                  cosmo_stats *stats, hipStream_t st);

// Dense sub-blocks (k_dense.hip).  Row products: dn[doff + r] = G_r . vin
// over the block's columns (float64 accumulation).  Column products:
// ec[coff + c] = sum_r G_rc w_r with w_r = sum_p scale_p u(row0_p + r), and
// (with the Jacobi diagonal) ed[coff + c] = sum_r G_rc^2 sum_p scale_p^2 rho_hat(row0_p + r),
// where u depends on the mode.
enum DenseColMode : int32_t {
  DC_XI = 0,    // u = y + rho_hat (b - s), with ed
  DC_GST = 1,   // u = gst, with ed
  DC_Y = 2,     // u = y
  DC_RP = 3     // u = rp
};
template <typename T> void launch_dense_rows(const View<T> &v, const T *vin, hipStream_t st);
int32_t dense_row_workgroups(int32_t rows);
int32_t dense_col_workgroups(int32_t cols, size_t esz);
template <typename T> void launch_dense_cols(const View<T> &v, int32_t mode, const T *rho_hat, const T *u,
                                            const T *s, hipStream_t st);

// PCG (k_pcg.hip): one workgroup per instance.
//   mode 0 (forward): solves M x = rhs, warm start from x (in/out), writes
//     xt_out (may alias x) and, if xnew != nullptr, x+ = alpha x~ + (1 - alpha) xold.
//   mode 1 (adjoint): solves M w = rhs; writes w and gx_out = (1 - alpha) gx_in + sigma w.
template <typename T> void launch_pcg(const View<T> &v, const T *rho_hat, const T *dg, const double *rhs, T *x,
                                      T *r, T *z, T *p, T *Mp, T *t, double *t64, double tol, int32_t max_iter,
                                      const T *alpha_k, const T *xold, T *xnew, const T *gx_in, T *gx_out,
                                      int32_t mode, cosmo_stats *stats, void *state, int32_t form,
                                      hipStream_t st);

// SOC (k_soc.hip)
template <typename T> void launch_soc_step(const SocDesc *d, int32_t n, const T *rho_hat, const T *vv,
                                           const T *sh, const T *y, T *s_new, T *y_new, hipStream_t st);
template <typename T> void launch_soc_vjp(const SocDesc *d, int32_t n, const T *vv, const T *g, T *out,
                                          hipStream_t st);
template <typename T> void launch_soc_proj(const SocDesc *d, int32_t n, const T *in, T *out, hipStream_t st);

// PSD (k_psd.hip).  Blocks are processed by order class; `d` lists blocks
// [0, n).  Forward step: eig of smat(vv_blk), Pi, s+ and y+ rows, eigenpairs
// to (U, lam).  Standalone: the same with no y update.
struct PsdLaunchCfg {
  int32_t max_sweeps;
  double tol;
  int32_t refine;          // float64 refinement steps after the Jacobi sweeps
  int32_t max_p;           // largest order in the list
  int32_t threads = 0;     // threads per workgroup of the eigensolve; 0 = the class default
};
// Eigensolve threads per workgroup of order class c (orders <= 32, <= 64,
// <= 128, larger): the default and the one alternative the autotuner times
// (twice the threads for the three smaller classes; none for the largest).
constexpr int32_t kEigThreads[4] = {64, 256, 512, 1024};
constexpr int32_t kEigThreadsAlt[4] = {128, 512, 1024, 1024};
// Threads per workgroup of the DK VJP: 16 waves (default) or 8.
constexpr int32_t kVjpThreads = 1024, kVjpThreadsAlt = 512;
template <typename T> void launch_psd_step(const PsdDesc *d, int32_t n, const PsdLaunchCfg &cfg,
                                           const T *rho_hat, const T *vv, const T *sh, const T *y, T *s_new,
                                           T *y_new, T *U, T *lam, double *rscratch, const T *Uprev,
                                           cosmo_stats *stats, hipStream_t st);
// rule 0 = Daleckii-Krein, 1 = eigendecomposition rule as autograd forms it,
// 2 = rule 1 at the eigenvalues shifted by eps (Tikhonov).  Returns false
// (nothing launched) when a block of order max_p does not fit in LDS.
// threads: kVjpThreads or kVjpThreadsAlt (0 = the default).
template <typename T> bool launch_psd_vjp(const PsdDesc *d, int32_t n, int32_t max_p, const T *U, const T *lam,
                                          const T *g, T *out, T *scratch, hipStream_t st, int32_t rule = 0,
                                          double eps = 0.0, int32_t threads = 0);

// Newton-Schulz comparison rule.  One block of the tape:
struct NsDesc {
  int64_t row0;    // first row of its svec in the input / output vectors
  int64_t moff;    // element offset of its matrix area in the tape
  int32_t p;       // matrix order
  int32_t tile0;   // index of its first output tile in a product launch
};
// One product C = alpha op(A) op(B) + beta D over every block (slots of the
// block's matrix area; d = -1: no D term; ta / tb: transpose A / B).
struct NsGemm {
  int32_t a, b, c, d, ta, tb;
  double alpha, beta;
};
// Slots of a block's matrix area for K steps: X_0..X_K, Q_0..Q_{K-1}, then
// S, W (forward output), TB, SB, Y, Z, QB (reverse pass).
struct NsSlots {
  int32_t K, S, W, TB, SB, Y, Z, QB;
  explicit NsSlots(int32_t k)
      : K(k), S(2 * k + 1), W(2 * k + 2), TB(2 * k + 3), SB(2 * k + 4), Y(2 * k + 5), Z(2 * k + 6), QB(2 * k + 7) {}
  int32_t x(int32_t k) const { return k; }
  int32_t q(int32_t k) const { return K + 1 + k; }
  static int64_t count(int32_t k) { return 2 * (int64_t)k + 8; }
};
// tile: output tile edge of one product workgroup, 64 or 32 (ntiles tiles
// of that edge over all blocks, tile0 counted in them).
template <typename T> void launch_ns_forward(const NsDesc *d, int32_t nblk, int32_t ntiles, int32_t tile, int32_t K,
                                             const T *v, T *out, T *base, double *cnorm, hipStream_t st);
template <typename T> void launch_ns_vjp(const NsDesc *d, int32_t nblk, int32_t ntiles, int32_t tile, int32_t K,
                                         const T *g, T *gin, T *base, const double *cnorm, hipStream_t st);

// bookkeeping for profiling: kernel-family events
void set_last_error(const std::string &msg);

}  // namespace cosmo
