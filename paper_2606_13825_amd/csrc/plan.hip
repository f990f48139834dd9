// Host side of the C ABI: argument validation, plan construction (transposed
// CSR of A, cone tables, length-bucketed row lists, PSD blocks grouped by
// order class), caller-owned workspace / tape layout, and the launch
// sequences of the K-step forward and reverse passes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "cosmo_internal.h"

namespace cosmo {

static thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }

}  // namespace cosmo

using namespace cosmo;

namespace {

constexpr int32_t ABI_VERSION = 2;

#define FAIL(code, msg)            \
  do {                             \
    set_last_error(msg);           \
    return code;                   \
  } while (0)

#define HIPCHK(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) {                                                                       \
      set_last_error(std::string(#expr) + ": " + hipGetErrorString(e_));                          \
      return COSMO_EHIP;                                                                          \
    }                                                                                             \
  } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Order classes of the eigensolver launch configurations.
inline int psd_class(int p) { return p <= 32 ? 0 : (p <= 64 ? 1 : (p <= 128 ? 2 : 3)); }

struct DevBuf {
  void *ptr = nullptr;
  ~DevBuf() {
    if (ptr) (void)hipFree(ptr);
  }
};

struct ProfileSlot {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t used = 0;
};

}  // namespace

struct cosmo_plan {
  cosmo_options opt{};
  int32_t pcg_form = 0;   // CG schedule: 0 one workgroup per instance, f > 0 cooperative (f per CU)
  int32_t B = 0;
  int64_t n_tot = 0, m_tot = 0;
  std::vector<int64_t> n_off, m_off;
  size_t esz = 4;
  // caller-owned problem arrays
  const int64_t *A_rowptr = nullptr;
  const int32_t *A_col = nullptr;
  const void *A_val = nullptr;
  int64_t A_nnz = 0;
  const int64_t *P_rowptr = nullptr;
  const int32_t *P_col = nullptr;
  const void *P_val = nullptr;
  int64_t P_nnz = 0;
  const void *q = nullptr, *b = nullptr;
  // plan-owned device memory (one allocation, carved)
  DevBuf mem;
  int64_t *d_n_off = nullptr, *d_m_off = nullptr;
  int64_t *d_At_rowptr = nullptr;
  int32_t *d_At_col = nullptr;
  void *d_At_val = nullptr;
  void *d_Pdiag = nullptr;
  uint8_t *d_row_kind = nullptr;
  int32_t *d_row_inst = nullptr, *d_col_inst = nullptr;
  int64_t *d_instA = nullptr, *d_instAt = nullptr;   // per-instance ranges of the row classes
  SocDesc *d_soc = nullptr;
  int32_t n_soc = 0;
  PsdDesc *d_psd = nullptr;
  int32_t n_psd = 0;
  int32_t psd_cls_begin[5] = {0, 0, 0, 0, 0};
  int32_t psd_cls_maxp[4] = {0, 0, 0, 0};
  // launch shapes of the PSD kernels: eigensolve threads per order class, DK VJP threads
  int32_t eig_threads[4] = {kEigThreads[0], kEigThreads[1], kEigThreads[2], kEigThreads[3]};
  int32_t vjp_threads = kVjpThreads;
  double psd_tune_ms[2][5] = {{-1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1}};   // last autotune: [default|alt][class 0..3, VJP]
  RectDesc *d_rect = nullptr;
  int32_t n_rect = 0;
  RowBuckets bkA, bkAt;
  int64_t sum_p = 0, sum_p2 = 0, sum_p2_large = 0;
  // dense sub-blocks of A (descriptors ordered by instance)
  int32_t n_dense = 0, dense_maxcols = 0, dense_wg_rows = 0, dense_wg_cols = 0;
  bool dense_g32 = false;   // the blocks' values are stored as float32
  int64_t dense_rows_tot = 0, dense_cols_tot = 0;
  DenseDesc *d_dense = nullptr;
  int32_t *d_dense_inst = nullptr, *d_drow = nullptr, *d_dcol = nullptr;
  double *d_dscale = nullptr;
  // M = P + sigma I + A' D A is diagonal when every row of A has at most one
  // nonzero and P is diagonal; the linear solves are then done in the
  // column kernels (x~ = xi / diag M) and the PCG kernel is not launched.
  bool diag_M = false;
  // layouts (element offsets of T)
  struct {
    size_t rho_hat, dg, xi, r, z, p, Mp, t, t64, cg, sh, vv, itA, itB, xt, st, U, lam, rp, rd, rs, dn, ec, ed, total;
  } fw{};
  struct {
    size_t slot, step, xt, st, lam, U, total;  // per-slot / per-step sizes and offsets inside a step
  } tp{};
  struct {
    size_t rho_hat, gA, gB, gsn, gv, gsh, gst, grh, gxt, w, dg, r, z, p, Mp, t, t64, cg, vv, dk, dn, ec, ed, zero, total;
  } bw{};
  bool profiling = false;
  void *tap = nullptr;   // cosmo_plan_set_tap: per-step projection input and output cotangent
  ProfileSlot prof[8];   // kinds of cosmo_plan_profile_read
  // auxiliary streams (default priority) and events for concurrent order classes
  hipStream_t aux[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[3] = {nullptr, nullptr, nullptr};
  // Graph mode: each direction's launch sequence is recorded once per set of
  // pointer arguments (on the plan's own capture stream, so the caller may
  // pass the legacy default stream) and replayed on the caller's stream.
  struct Recorded {
    hipGraphExec_t exec = nullptr;
    std::vector<const void *> key;
  };
  bool graph = false;
  hipStream_t cap = nullptr;
  Recorded rec_fwd, rec_bwd;
  void drop_graphs() {
    for (Recorded *r : {&rec_fwd, &rec_bwd}) {
      if (r->exec) (void)hipGraphExecDestroy(r->exec);
      r->exec = nullptr;
      r->key.clear();
    }
  }
  ~cosmo_plan() {
    drop_graphs();
    if (cap) (void)hipStreamDestroy(cap);
    for (auto &s : prof)
      for (auto &e : s.ev) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
    for (int i = 0; i < 3; ++i) {
      if (aux[i]) (void)hipStreamDestroy(aux[i]);
      if (ev_join[i]) (void)hipEventDestroy(ev_join[i]);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
  }
};

namespace {

template <typename T> View<T> make_view(const cosmo_plan *pl) {
  View<T> v;
  v.A_rowptr = pl->A_rowptr;
  v.A_col = pl->A_col;
  v.A_val = static_cast<const T *>(pl->A_val);
  v.P_rowptr = pl->P_nnz > 0 ? pl->P_rowptr : nullptr;
  v.P_col = pl->P_col;
  v.P_val = static_cast<const T *>(pl->P_val);
  v.q = static_cast<const T *>(pl->q);
  v.b = static_cast<const T *>(pl->b);
  v.At_rowptr = pl->d_At_rowptr;
  v.At_col = pl->d_At_col;
  v.At_val = static_cast<const T *>(pl->d_At_val);
  v.Pdiag = static_cast<const T *>(pl->d_Pdiag);
  v.row_kind = pl->d_row_kind;
  v.row_inst = pl->d_row_inst;
  v.col_inst = pl->d_col_inst;
  v.n_off = pl->d_n_off;
  v.m_off = pl->d_m_off;
  v.rowsA = pl->bkA.d_rows;
  v.rowsAt = pl->bkAt.d_rows;
  v.spanA = pl->bkA.d_span;
  v.spanAt = pl->bkAt.d_span;
  v.instA = pl->d_instA;
  v.instAt = pl->d_instAt;
  v.B = pl->B;
  v.n_tot = pl->n_tot;
  v.m_tot = pl->m_tot;
  v.sigma = (T)pl->opt.sigma;
  v.dense = pl->n_dense > 0 ? pl->d_dense : nullptr;
  v.dense_inst = pl->d_dense_inst;
  v.drow = pl->n_dense > 0 ? pl->d_drow : nullptr;
  v.dscale = pl->d_dscale;
  v.dcol = pl->n_dense > 0 ? pl->d_dcol : nullptr;
  v.n_dense = pl->n_dense;
  v.dense_maxcols = pl->dense_maxcols;
  v.dense_wg_rows = pl->dense_wg_rows;
  v.dense_wg_cols = pl->dense_wg_cols;
  v.dense_g32 = pl->dense_g32 ? 1 : 0;
  v.dn = v.ec = v.ed = nullptr;   // set per call from the call's workspace
  return v;
}

// The dense scratch vectors of a call's workspace (float64, at element
// offsets of T).
template <typename T> void bind_dense(View<T> &v, T *ws, size_t dn, size_t ec, size_t ed) {
  v.dn = reinterpret_cast<double *>(ws + dn);
  v.ec = reinterpret_cast<double *>(ws + ec);
  v.ed = reinterpret_cast<double *>(ws + ed);
}

// Profiling: events around launches of one kernel family.
struct ProfScope {
  cosmo_plan *pl;
  int kind;
  hipStream_t st;
  hipEvent_t e1 = nullptr;
  ProfScope(cosmo_plan *p, int k, hipStream_t s) : pl(p), kind(k), st(s) {
    if (!pl->profiling) return;
    ProfileSlot &sl = pl->prof[kind];
    if (sl.used == sl.ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
      sl.ev.emplace_back(a, b);
    }
    auto &pr = sl.ev[sl.used++];
    (void)hipEventRecord(pr.first, st);
    e1 = pr.second;
  }
  ~ProfScope() {
    if (e1) (void)hipEventRecord(e1, st);
  }
};

cosmo_status validate_options(const cosmo_options *o) {
  if (!o) FAIL(COSMO_EINVAL, "options is NULL");
  if (o->dtype != COSMO_F32 && o->dtype != COSMO_F64) FAIL(COSMO_EINVAL, "dtype must be COSMO_F32 or COSMO_F64");
  if (o->K < 1) FAIL(COSMO_EINVAL, "K must be >= 1");
  if (!(o->sigma > 0.0) || !std::isfinite(o->sigma)) FAIL(COSMO_EINVAL, "sigma must be finite and > 0");
  if (!(o->cg_tol >= 0.0) || !std::isfinite(o->cg_tol)) FAIL(COSMO_EINVAL, "cg_tol must be finite and >= 0");
  if (o->cg_max_iter < 1) FAIL(COSMO_EINVAL, "cg_max_iter must be >= 1");
  if (o->eig_max_sweeps < 1) FAIL(COSMO_EINVAL, "eig_max_sweeps must be >= 1");
  if (!(o->eig_tol >= 0.0) || !std::isfinite(o->eig_tol)) FAIL(COSMO_EINVAL, "eig_tol must be finite and >= 0");
  if (o->eig_refine < 0 || o->eig_refine > 1) FAIL(COSMO_EINVAL, "eig_refine must be 0 or 1");
  if (o->eig_warm_start != 0 && o->eig_warm_start != 1) FAIL(COSMO_EINVAL, "eig_warm_start must be 0 or 1");
  return COSMO_OK;
}

// Host-only checks (no device access).
cosmo_status validate_problem_host(const cosmo_problem *p, const cosmo_options *o) {
  if (!p) FAIL(COSMO_EINVAL, "problem is NULL");
  if (p->B < 1) FAIL(COSMO_EINVAL, "B must be >= 1");
  if (!p->n_off || !p->m_off) FAIL(COSMO_EINVAL, "n_off / m_off must be non-NULL host arrays");
  if (p->n_off[0] != 0 || p->m_off[0] != 0) FAIL(COSMO_EINVAL, "n_off[0] and m_off[0] must be 0");
  for (int i = 0; i < p->B; ++i) {
    if (p->n_off[i + 1] < p->n_off[i]) FAIL(COSMO_EINVAL, "n_off must be non-decreasing");
    if (p->m_off[i + 1] <= p->m_off[i]) FAIL(COSMO_EINVAL, "every instance needs at least one row");
  }
  const int64_t n_tot = p->n_off[p->B], m_tot = p->m_off[p->B];
  if (n_tot < 1) FAIL(COSMO_EINVAL, "no variables");
  if (n_tot > INT32_MAX || m_tot > INT32_MAX) FAIL(COSMO_EUNSUPPORTED, "n_tot and m_tot must fit in int32");
  if (!p->A_rowptr || !p->A_col || !p->A_val) FAIL(COSMO_EINVAL, "A arrays must be non-NULL");
  if ((reinterpret_cast<uintptr_t>(p->A_col) | reinterpret_cast<uintptr_t>(p->A_val)) % 16 != 0)
    FAIL(COSMO_EINVAL, "A_col and A_val must be 16-byte aligned");
  if (p->A_nnz < 0) FAIL(COSMO_EINVAL, "A_nnz < 0");
  if (p->P_nnz < 0) FAIL(COSMO_EINVAL, "P_nnz < 0");
  if (p->P_nnz > 0 && (!p->P_rowptr || !p->P_col || !p->P_val)) FAIL(COSMO_EINVAL, "P arrays must be non-NULL");
  if (!p->q || !p->b) FAIL(COSMO_EINVAL, "q and b must be non-NULL");
  if (p->n_cones < 1 || !p->cone_kind || !p->cone_size) FAIL(COSMO_EINVAL, "cone list is empty or NULL");
  // cones tile the rows, none straddles an instance
  int64_t row = 0;
  int inst = 0;
  const int maxp = (o->dtype == COSMO_F32) ? COSMO_MAX_PSD_ORDER_F32 : COSMO_MAX_PSD_ORDER_F64;
  for (int c = 0; c < p->n_cones; ++c) {
    const int k = p->cone_kind[c], sz = p->cone_size[c];
    if (k < COSMO_CONE_ZERO || k > COSMO_CONE_PSD) FAIL(COSMO_EINVAL, "unknown cone kind at index " + std::to_string(c));
    if (sz < 1) FAIL(COSMO_EINVAL, "cone size must be >= 1 at index " + std::to_string(c));
    if (k == COSMO_CONE_PSD && sz > maxp)
      FAIL(COSMO_EUNSUPPORTED, "PSD order " + std::to_string(sz) + " exceeds the supported maximum " + std::to_string(maxp));
    const int64_t rows = (k == COSMO_CONE_PSD) ? (int64_t)sz * (sz + 1) / 2 : sz;
    while (inst < p->B && row >= p->m_off[inst + 1]) ++inst;
    if (row + rows > p->m_off[inst + 1]) FAIL(COSMO_EINVAL, "cone " + std::to_string(c) + " straddles an instance boundary");
    row += rows;
  }
  if (row != m_tot) FAIL(COSMO_EINVAL, "cone rows sum to " + std::to_string(row) + " but m_tot is " + std::to_string(m_tot));
  // dense sub-blocks
  if (p->n_dense < 0) FAIL(COSMO_EINVAL, "n_dense < 0");
  if (p->n_dense > 0 && !p->dense) FAIL(COSMO_EINVAL, "dense descriptors are NULL");
  const size_t esz = o->dtype == COSMO_F32 ? 4 : 8;
  std::vector<std::pair<int64_t, int64_t>> rspans, cspans;
  auto inst_of = [&](const int64_t *off, int64_t idx) {
    return (int)(std::upper_bound(off, off + p->B + 1, idx) - off) - 1;
  };
  for (int k = 0; k < p->n_dense; ++k) {
    const cosmo_dense_block &d = p->dense[k];
    const std::string at = " (dense block " + std::to_string(k) + ")";
    if (d.val_f32 != 0 && d.val_f32 != 1) FAIL(COSMO_EINVAL, "dense val_f32 must be 0 or 1" + at);
    if (d.val_f32 != p->dense[0].val_f32) FAIL(COSMO_EINVAL, "dense val_f32 differs between blocks" + at);
    const size_t gsz = d.val_f32 ? 4 : esz;   // bytes per stored value
    if (!d.val) FAIL(COSMO_EINVAL, "dense values are NULL" + at);
    if (reinterpret_cast<uintptr_t>(d.val) % 16 != 0) FAIL(COSMO_EINVAL, "dense values must be 16-byte aligned" + at);
    if (d.rows < 1 || d.cols < 1) FAIL(COSMO_EINVAL, "dense block needs rows, cols >= 1" + at);
    if (d.cols > COSMO_DENSE_MAX_COLS) FAIL(COSMO_EINVAL, "dense block wider than COSMO_DENSE_MAX_COLS" + at);
    if (d.ld < d.cols || d.ld % (int64_t)(16 / gsz) != 0)
      FAIL(COSMO_EINVAL, "dense ld must be >= cols and a multiple of 16 / (bytes per stored value)" + at);
    if (d.n_place < 1 || d.n_place > COSMO_DENSE_MAX_PLACEMENTS) FAIL(COSMO_EINVAL, "dense n_place out of range" + at);
    if (d.col0 < 0 || d.col0 + d.cols > n_tot) FAIL(COSMO_EINVAL, "dense columns outside A" + at);
    const int ci = inst_of(p->n_off, d.col0);
    if (d.col0 + d.cols > p->n_off[ci + 1]) FAIL(COSMO_EINVAL, "dense columns straddle instances" + at);
    cspans.push_back({d.col0, d.col0 + d.cols});
    for (int q = 0; q < d.n_place; ++q) {
      if (!std::isfinite(d.scale[q])) FAIL(COSMO_EINVAL, "dense scale must be finite" + at);
      if (d.row0[q] < 0 || d.row0[q] + d.rows > m_tot) FAIL(COSMO_EINVAL, "dense rows outside A" + at);
      const int ri = inst_of(p->m_off, d.row0[q]);
      if (d.row0[q] + d.rows > p->m_off[ri + 1] || ri != ci)
        FAIL(COSMO_EINVAL, "dense rows and columns must lie in one instance" + at);
      rspans.push_back({d.row0[q], d.row0[q] + d.rows});
    }
  }
  for (auto *sp : {&rspans, &cspans}) {
    std::sort(sp->begin(), sp->end());
    for (size_t i = 1; i < sp->size(); ++i)
      if ((*sp)[i].first < (*sp)[i - 1].second)
        FAIL(COSMO_EINVAL, sp == &rspans ? "a row of A lies in two dense placements"
                                         : "a column of A lies in two dense blocks");
  }
  return COSMO_OK;
}

void build_buckets(const std::vector<int64_t> &rowptr, int64_t nrows, std::vector<int32_t> &rows_out,
                   RowBuckets &bk) {
  std::vector<int32_t> cls[3];
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t len = rowptr[r + 1] - rowptr[r];
    cls[len <= 4 ? 0 : (len <= 48 ? 1 : 2)].push_back((int32_t)r);
  }
  rows_out.clear();
  for (int c = 0; c < 3; ++c) {
    bk.begin[c] = (int64_t)rows_out.size();
    rows_out.insert(rows_out.end(), cls[c].begin(), cls[c].end());
  }
  bk.begin[3] = (int64_t)rows_out.size();
  bk.lanes[0] = 1;
  bk.lanes[1] = 8;
  bk.lanes[2] = 64;
}

template <typename T>
cosmo_status build_plan(cosmo_plan *pl, const cosmo_problem *p) {
  const int64_t n = pl->n_tot, m = pl->m_tot, nnz = p->A_nnz;
  // --- copy A (and P) to the host
  std::vector<int64_t> rp(m + 1);
  HIPCHK(hipMemcpy(rp.data(), p->A_rowptr, (m + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (rp[0] != 0 || rp[m] != nnz) FAIL(COSMO_EINVAL, "A_rowptr[0] must be 0 and A_rowptr[m_tot] must equal A_nnz");
  for (int64_t i = 0; i < m; ++i)
    if (rp[i + 1] < rp[i]) FAIL(COSMO_EINVAL, "A_rowptr must be non-decreasing");
  std::vector<int32_t> col(nnz);
  std::vector<T> val(nnz);
  if (nnz > 0) {
    HIPCHK(hipMemcpy(col.data(), p->A_col, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(val.data(), p->A_val, nnz * sizeof(T), hipMemcpyDeviceToHost));
  }
  for (int b = 0; b < pl->B; ++b)
    for (int64_t i = pl->m_off[b]; i < pl->m_off[b + 1]; ++i)
      for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
        if (col[k] < pl->n_off[b] || col[k] >= pl->n_off[b + 1])
          FAIL(COSMO_EINVAL, "A has an entry outside its instance's column block (row " + std::to_string(i) + ")");
  std::vector<T> pdiag(n, (T)0);
  std::vector<int64_t> prp;
  if (p->P_nnz > 0) {
    prp.resize(n + 1);
    std::vector<int32_t> pc(p->P_nnz);
    std::vector<T> pv(p->P_nnz);
    HIPCHK(hipMemcpy(prp.data(), p->P_rowptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    if (prp[0] != 0 || prp[n] != p->P_nnz) FAIL(COSMO_EINVAL, "P_rowptr[0] must be 0 and P_rowptr[n_tot] must equal P_nnz");
    HIPCHK(hipMemcpy(pc.data(), p->P_col, p->P_nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(pv.data(), p->P_val, p->P_nnz * sizeof(T), hipMemcpyDeviceToHost));
    for (int b = 0; b < pl->B; ++b)
      for (int64_t j = pl->n_off[b]; j < pl->n_off[b + 1]; ++j) {
        if (prp[j + 1] < prp[j]) FAIL(COSMO_EINVAL, "P_rowptr must be non-decreasing");
        for (int64_t k = prp[j]; k < prp[j + 1]; ++k) {
          if (pc[k] < pl->n_off[b] || pc[k] >= pl->n_off[b + 1])
            FAIL(COSMO_EINVAL, "P has an entry outside its instance's block");
          if (pc[k] == j) pdiag[j] += pv[k];
        }
      }
  } else {
    prp.assign(n + 1, 0);
  }
  // --- transpose of A (counting sort by column; rows stay increasing)
  std::vector<int64_t> trp(n + 1, 0);
  for (int64_t k = 0; k < nnz; ++k) trp[col[k] + 1]++;
  for (int64_t j = 0; j < n; ++j) trp[j + 1] += trp[j];
  std::vector<int64_t> fill(trp.begin(), trp.end() - 1);
  std::vector<int32_t> tcol(nnz);
  std::vector<T> tval(nnz);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      const int64_t dst = fill[col[k]]++;
      tcol[dst] = (int32_t)i;
      tval[dst] = val[k];
    }
  // --- row / column metadata
  std::vector<uint8_t> rkind(m);
  std::vector<int32_t> rinst(m), cinst(n);
  for (int b = 0; b < pl->B; ++b) {
    for (int64_t i = pl->m_off[b]; i < pl->m_off[b + 1]; ++i) rinst[i] = b;
    for (int64_t j = pl->n_off[b]; j < pl->n_off[b + 1]; ++j) cinst[j] = b;
  }
  std::vector<SocDesc> socs;
  std::vector<PsdDesc> psds;
  std::vector<RectDesc> rects;
  int64_t row = 0;
  for (int c = 0; c < p->n_cones; ++c) {
    const int k = p->cone_kind[c], sz = p->cone_size[c];
    const int64_t rows = (k == COSMO_CONE_PSD) ? (int64_t)sz * (sz + 1) / 2 : sz;
    for (int64_t i = row; i < row + rows; ++i) rkind[i] = (uint8_t)k;
    if (k == COSMO_CONE_SOC) {
      socs.push_back({row, sz, rinst[row]});
      rects.push_back({row, (int32_t)rows, 0});
    } else if (k == COSMO_CONE_PSD) {
      psds.push_back({row, 0, 0, sz, rinst[row]});
      rects.push_back({row, (int32_t)rows, 0});
    }
    row += rows;
  }
  // PSD blocks: eigen storage offsets in list order, then grouped by order
  // class with the largest blocks first inside each class.
  int64_t uo = 0, lo = 0, large = 0;
  for (auto &d : psds) {
    d.uoff = uo;
    d.loff = lo;
    uo += (int64_t)d.p * d.p;
    lo += d.p;
    if ((size_t)3 * d.p * d.p * sizeof(T) > 163840 - 4096) large += (int64_t)d.p * d.p;
  }
  pl->sum_p2 = uo;
  pl->sum_p = lo;
  pl->sum_p2_large = uo;   // DK scratch indexed by uoff
  (void)large;
  std::stable_sort(psds.begin(), psds.end(), [](const PsdDesc &a, const PsdDesc &b) {
    const int ca = psd_class(a.p), cb = psd_class(b.p);
    if (ca != cb) return ca < cb;
    return a.p > b.p;
  });
  for (int c = 0; c < 5; ++c) pl->psd_cls_begin[c] = 0;
  for (int c = 0; c < 4; ++c) pl->psd_cls_maxp[c] = 0;
  {
    int idx = 0;
    for (int c = 0; c < 4; ++c) {
      pl->psd_cls_begin[c] = idx;
      while (idx < (int)psds.size() && psd_class(psds[idx].p) == c) {
        pl->psd_cls_maxp[c] = std::max(pl->psd_cls_maxp[c], psds[idx].p);
        ++idx;
      }
    }
    pl->psd_cls_begin[4] = idx;
  }
  {
    bool dm = true;
    for (int64_t i = 0; i < m && dm; ++i) dm = (rp[i + 1] - rp[i]) <= 1;
    if (dm && p->P_nnz > 0) {
      std::vector<int32_t> pc(p->P_nnz);
      HIPCHK(hipMemcpy(pc.data(), p->P_col, p->P_nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
      for (int64_t j = 0; j < n && dm; ++j)
        for (int64_t k = prp[j]; k < prp[j + 1] && dm; ++k) dm = (pc[k] == j);
    }
    pl->diag_M = dm && p->n_dense == 0;
  }
  // dense sub-blocks: descriptors ordered by instance, their scratch offsets
  // and launch layouts, and the per-row / per-column maps
  std::vector<DenseDesc> dens;
  std::vector<int32_t> dinst(pl->B + 1, 0), drow, dcolm;
  std::vector<double> dscale;
  if (p->n_dense > 0) {
    pl->dense_g32 = p->dense[0].val_f32 != 0 || sizeof(T) == 4;
    drow.assign(m, -1);
    dscale.assign(m, 0.0);
    dcolm.assign(n, -1);
    for (int k = 0; k < p->n_dense; ++k) {
      const cosmo_dense_block &b = p->dense[k];
      DenseDesc d{};
      d.val = b.val;
      d.ld = b.ld;
      d.col0 = b.col0;
      d.rows = b.rows;
      d.cols = b.cols;
      d.nplace = b.n_place;
      d.inst = cinst[b.col0];
      for (int q = 0; q < COSMO_DENSE_MAX_PLACEMENTS; ++q) {
        d.row0[q] = q < b.n_place ? b.row0[q] : 0;
        d.scale[q] = q < b.n_place ? b.scale[q] : 0.0;
      }
      dens.push_back(d);
    }
    std::stable_sort(dens.begin(), dens.end(), [](const DenseDesc &a, const DenseDesc &b) { return a.inst < b.inst; });
    int64_t doff = 0, coff = 0;
    int32_t wr = 0, wc = 0;
    for (size_t k = 0; k < dens.size(); ++k) {
      DenseDesc &d = dens[k];
      d.doff = doff;
      d.coff = coff;
      d.wg_rows0 = wr;
      d.wg_cols0 = wc;
      for (int q = 0; q < d.nplace; ++q)
        for (int r = 0; r < d.rows; ++r) {
          drow[d.row0[q] + r] = (int32_t)(doff + r);
          dscale[d.row0[q] + r] = d.scale[q];
        }
      for (int c = 0; c < d.cols; ++c) dcolm[d.col0 + c] = (int32_t)(coff + c);
      doff += d.rows;
      coff += d.cols;
      wr += dense_row_workgroups(d.rows);
      wc += dense_col_workgroups(d.cols, pl->dense_g32 ? 4 : sizeof(T));
      pl->dense_maxcols = std::max(pl->dense_maxcols, d.cols);
      dinst[d.inst + 1]++;
    }
    for (int b = 0; b < pl->B; ++b) dinst[b + 1] += dinst[b];
    pl->n_dense = (int32_t)dens.size();
    pl->dense_rows_tot = doff;
    pl->dense_cols_tot = coff;
    pl->dense_wg_rows = wr;
    pl->dense_wg_cols = wc;
  }
  pl->n_soc = (int32_t)socs.size();
  pl->n_psd = (int32_t)psds.size();
  pl->n_rect = (int32_t)rects.size();
  // row buckets and per-instance lane widths
  std::vector<int32_t> rowsA, rowsAt;
  build_buckets(rp, m, rowsA, pl->bkA);
  build_buckets(trp, n, rowsAt, pl->bkAt);
  // rows of each class are listed in increasing order, so an instance's rows
  // of a class are one contiguous range of the list
  auto inst_ranges = [&](const std::vector<int32_t> &rows, const RowBuckets &bk, const std::vector<int64_t> &off) {
    std::vector<int64_t> rng(3 * (size_t)(pl->B + 1));
    for (int c = 0; c < 3; ++c) {
      auto first = rows.begin() + bk.begin[c], last = rows.begin() + bk.begin[c + 1];
      for (int b = 0; b <= pl->B; ++b)
        rng[c * (size_t)(pl->B + 1) + b] = std::lower_bound(first, last, off[b]) - rows.begin();
    }
    return rng;
  };
  const std::vector<int64_t> instA = inst_ranges(rowsA, pl->bkA, pl->m_off);
  const std::vector<int64_t> instAt = inst_ranges(rowsAt, pl->bkAt, pl->n_off);
  // --- one device allocation for everything the plan owns
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_noff = take((pl->B + 1) * sizeof(int64_t)), o_moff = take((pl->B + 1) * sizeof(int64_t));
  const size_t o_trp = take((n + 1) * sizeof(int64_t)), o_tcol = take(std::max<int64_t>(nnz, 1) * sizeof(int32_t));
  const size_t o_tval = take(std::max<int64_t>(nnz, 1) * sizeof(T)), o_pdiag = take(n * sizeof(T));
  const size_t o_rkind = take(m), o_rinst = take(m * sizeof(int32_t)), o_cinst = take(n * sizeof(int32_t));
  const size_t o_iA = take(instA.size() * sizeof(int64_t)), o_iAt = take(instAt.size() * sizeof(int64_t));
  const size_t o_soc = take(std::max<size_t>(socs.size(), 1) * sizeof(SocDesc));
  const size_t o_psd = take(std::max<size_t>(psds.size(), 1) * sizeof(PsdDesc));
  const size_t o_rect = take(std::max<size_t>(rects.size(), 1) * sizeof(RectDesc));
  const size_t o_bA = take(std::max<size_t>(rowsA.size(), 1) * sizeof(int32_t));
  const size_t o_bAt = take(std::max<size_t>(rowsAt.size(), 1) * sizeof(int32_t));
  auto spans = [](const std::vector<int32_t> &rows, const std::vector<int64_t> &ptr) {
    std::vector<RowSpan> sp(rows.size());
    for (size_t i = 0; i < rows.size(); ++i) sp[i] = RowSpan{ptr[rows[i]], ptr[rows[i] + 1]};
    return sp;
  };
  const std::vector<RowSpan> spA = spans(rowsA, rp), spAt = spans(rowsAt, trp);
  const size_t o_sA = take(std::max<size_t>(spA.size(), 1) * sizeof(RowSpan));
  const size_t o_sAt = take(std::max<size_t>(spAt.size(), 1) * sizeof(RowSpan));
  const size_t o_dense = take(std::max<size_t>(dens.size(), 1) * sizeof(DenseDesc));
  const size_t o_dinst = take(dinst.size() * sizeof(int32_t));
  const size_t o_drow = take(std::max<size_t>(drow.size(), 1) * sizeof(int32_t));
  const size_t o_dscale = take(std::max<size_t>(dscale.size(), 1) * sizeof(double));
  const size_t o_dcol = take(std::max<size_t>(dcolm.size(), 1) * sizeof(int32_t));
  if (hipMalloc(&pl->mem.ptr, off) != hipSuccess) {
    pl->mem.ptr = nullptr;
    FAIL(COSMO_ENOMEM, "plan allocation of " + std::to_string(off) + " bytes failed");
  }
  char *base = static_cast<char *>(pl->mem.ptr);
  auto up = [&](size_t o, const void *src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice);
  };
  HIPCHK(up(o_noff, pl->n_off.data(), (pl->B + 1) * sizeof(int64_t)));
  HIPCHK(up(o_moff, pl->m_off.data(), (pl->B + 1) * sizeof(int64_t)));
  HIPCHK(up(o_trp, trp.data(), (n + 1) * sizeof(int64_t)));
  HIPCHK(up(o_tcol, tcol.data(), nnz * sizeof(int32_t)));
  HIPCHK(up(o_tval, tval.data(), nnz * sizeof(T)));
  HIPCHK(up(o_pdiag, pdiag.data(), n * sizeof(T)));
  HIPCHK(up(o_rkind, rkind.data(), m));
  HIPCHK(up(o_rinst, rinst.data(), m * sizeof(int32_t)));
  HIPCHK(up(o_cinst, cinst.data(), n * sizeof(int32_t)));
  HIPCHK(up(o_iA, instA.data(), instA.size() * sizeof(int64_t)));
  HIPCHK(up(o_iAt, instAt.data(), instAt.size() * sizeof(int64_t)));
  HIPCHK(up(o_soc, socs.data(), socs.size() * sizeof(SocDesc)));
  HIPCHK(up(o_psd, psds.data(), psds.size() * sizeof(PsdDesc)));
  HIPCHK(up(o_rect, rects.data(), rects.size() * sizeof(RectDesc)));
  HIPCHK(up(o_bA, rowsA.data(), rowsA.size() * sizeof(int32_t)));
  HIPCHK(up(o_bAt, rowsAt.data(), rowsAt.size() * sizeof(int32_t)));
  HIPCHK(up(o_sA, spA.data(), spA.size() * sizeof(RowSpan)));
  HIPCHK(up(o_sAt, spAt.data(), spAt.size() * sizeof(RowSpan)));
  HIPCHK(up(o_dense, dens.data(), dens.size() * sizeof(DenseDesc)));
  HIPCHK(up(o_dinst, dinst.data(), dinst.size() * sizeof(int32_t)));
  HIPCHK(up(o_drow, drow.data(), drow.size() * sizeof(int32_t)));
  HIPCHK(up(o_dscale, dscale.data(), dscale.size() * sizeof(double)));
  HIPCHK(up(o_dcol, dcolm.data(), dcolm.size() * sizeof(int32_t)));
  pl->d_n_off = reinterpret_cast<int64_t *>(base + o_noff);
  pl->d_m_off = reinterpret_cast<int64_t *>(base + o_moff);
  pl->d_At_rowptr = reinterpret_cast<int64_t *>(base + o_trp);
  pl->d_At_col = reinterpret_cast<int32_t *>(base + o_tcol);
  pl->d_At_val = base + o_tval;
  pl->d_Pdiag = base + o_pdiag;
  pl->d_row_kind = reinterpret_cast<uint8_t *>(base + o_rkind);
  pl->d_row_inst = reinterpret_cast<int32_t *>(base + o_rinst);
  pl->d_col_inst = reinterpret_cast<int32_t *>(base + o_cinst);
  pl->d_instA = reinterpret_cast<int64_t *>(base + o_iA);
  pl->d_instAt = reinterpret_cast<int64_t *>(base + o_iAt);
  pl->d_soc = reinterpret_cast<SocDesc *>(base + o_soc);
  pl->d_psd = reinterpret_cast<PsdDesc *>(base + o_psd);
  pl->d_rect = reinterpret_cast<RectDesc *>(base + o_rect);
  pl->bkA.d_rows = reinterpret_cast<int32_t *>(base + o_bA);
  pl->bkAt.d_rows = reinterpret_cast<int32_t *>(base + o_bAt);
  pl->bkA.d_span = reinterpret_cast<RowSpan *>(base + o_sA);
  pl->bkAt.d_span = reinterpret_cast<RowSpan *>(base + o_sAt);
  pl->d_dense = reinterpret_cast<DenseDesc *>(base + o_dense);
  pl->d_dense_inst = reinterpret_cast<int32_t *>(base + o_dinst);
  pl->d_drow = reinterpret_cast<int32_t *>(base + o_drow);
  pl->d_dscale = reinterpret_cast<double *>(base + o_dscale);
  pl->d_dcol = reinterpret_cast<int32_t *>(base + o_dcol);
  return COSMO_OK;
}

// Element-offset layouts of the caller-owned buffers.
void build_layouts(cosmo_plan *pl) {
  const size_t n = pl->n_tot, m = pl->m_tot, K = pl->opt.K;
  const size_t A = 64;   // 256-byte alignment for float, 512 for double
  size_t o = 0;
  auto take = [&](size_t elems) {
    const size_t r = o;
    o = align_up(o + std::max<size_t>(elems, 1), A);
    return r;
  };
  auto &f = pl->fw;
  f.rho_hat = take(K * m);
  f.dg = take(n);
  f.xi = take(n * 8 / pl->esz);           // right-hand side of the solve, float64
  f.r = take(n);
  f.z = take(n);
  f.p = take(n);
  f.Mp = take(n);
  f.t = take(m);
  f.t64 = take(2 * m);                     // float64 residual pass of the CG (m doubles)
  f.cg = take(16 * ((size_t)pl->B + 1) + 256);  // per-instance state of the CG (cooperative form)
  f.sh = take(m);
  f.vv = take(m);
  // (x, s, y) triples laid out like a tape slot: each part starts 64-element aligned
  const size_t triple = align_up(n, A) + 2 * align_up(m, A);
  f.itA = take(triple);
  f.itB = take(triple);
  f.xt = take(n);
  f.st = take(m);
  f.U = take(pl->sum_p2);
  f.lam = take(pl->sum_p);
  f.rp = take(m);
  f.rd = take(n);
  f.rs = take(3 * (size_t)pl->sum_p2 * 8 / pl->esz);   // eigensolver refinement scratch
  // float64 scratch of the dense sub-blocks: row products, column products, Jacobi terms
  f.dn = take((size_t)pl->dense_rows_tot * 8 / pl->esz);
  f.ec = take((size_t)pl->dense_cols_tot * 8 / pl->esz);
  f.ed = take((size_t)pl->dense_cols_tot * 8 / pl->esz);
  f.total = o;
  // tape: slot k (x, s, y) for k = 0..K, then per step (x~, s~, lam, U)
  auto &t = pl->tp;
  t.slot = align_up(n, A) + 2 * align_up(m, A);
  t.xt = 0;
  t.st = align_up(n, A);
  t.lam = t.st + align_up(m, A);
  t.U = t.lam + align_up(std::max<int64_t>(pl->sum_p, 1), A);
  t.step = t.U + align_up(std::max<int64_t>(pl->sum_p2, 1), A);
  t.total = (K + 1) * t.slot + K * t.step;
  auto &w = pl->bw;
  o = 0;
  w.rho_hat = take(K * m);
  w.gA = take(triple);
  w.gB = take(triple);
  w.gsn = take(m);
  w.gv = take(m);
  w.gsh = take(m);
  w.gst = take(m);
  w.grh = take(m);
  w.gxt = take(n * 8 / pl->esz);          // right-hand side of the adjoint solve, float64
  w.w = take(n);
  w.dg = take(n);
  w.r = take(n);
  w.z = take(n);
  w.p = take(n);
  w.Mp = take(n);
  w.t = take(m);
  w.t64 = take(2 * m);
  w.cg = take(16 * ((size_t)pl->B + 1) + 256);
  w.vv = take(m);
  w.dk = take(pl->sum_p2_large);
  w.dn = take((size_t)pl->dense_rows_tot * 8 / pl->esz);
  w.ec = take((size_t)pl->dense_cols_tot * 8 / pl->esz);
  w.ed = take((size_t)pl->dense_cols_tot * 8 / pl->esz);
  w.total = o;
}

size_t slot_x(const cosmo_plan *pl, size_t k) { return k * pl->tp.slot; }
size_t slot_s(const cosmo_plan *pl, size_t k) { return k * pl->tp.slot + align_up(pl->n_tot, 64); }
size_t slot_y(const cosmo_plan *pl, size_t k) {
  return k * pl->tp.slot + align_up(pl->n_tot, 64) + align_up(pl->m_tot, 64);
}
size_t step_base(const cosmo_plan *pl, size_t k) { return (pl->opt.K + 1) * pl->tp.slot + k * pl->tp.step; }

// The PSD order classes are independent launches over disjoint blocks: the
// first non-empty class runs on the caller's stream, the others on the plan's
// auxiliary streams, forked from and joined back into the caller's stream by
// events (a pattern stream capture also accepts).
template <typename F> void fork_classes(cosmo_plan *pl, hipStream_t st, F &&launch_class) {
  int cls[4], nc = 0;
  for (int c = 0; c < 4; ++c)
    if (pl->psd_cls_begin[c + 1] > pl->psd_cls_begin[c]) cls[nc++] = c;
  if (nc == 0) return;
  if (nc > 1) (void)hipEventRecord(pl->ev_fork, st);
  for (int i = 1; i < nc; ++i) {
    (void)hipStreamWaitEvent(pl->aux[i - 1], pl->ev_fork, 0);
    launch_class(cls[i], pl->aux[i - 1]);
    (void)hipEventRecord(pl->ev_join[i - 1], pl->aux[i - 1]);
  }
  launch_class(cls[0], st);
  for (int i = 1; i < nc; ++i) (void)hipStreamWaitEvent(st, pl->ev_join[i - 1], 0);
}

template <typename T>
void launch_psd_classes(cosmo_plan *pl, const T *rho_hat, const T *vv, const T *sh, const T *y, T *s_new, T *y_new,
                        T *U, T *lam, double *rscratch, const T *Uprev, cosmo_stats *stats, hipStream_t st) {
  ProfScope ps(pl, 0, st);
  const bool refine = pl->opt.dtype == COSMO_F32 && pl->opt.eig_refine > 0;
  fork_classes(pl, st, [&](int c, hipStream_t s) {
    const int n = pl->psd_cls_begin[c + 1] - pl->psd_cls_begin[c];
    PsdLaunchCfg cfg{pl->opt.eig_max_sweeps, pl->opt.eig_tol, refine ? pl->opt.eig_refine : 0, pl->psd_cls_maxp[c],
                     pl->eig_threads[c]};
    ProfScope pc(pl, 4 + c, s);   // this class's kernel alone, on the stream it runs on
    launch_psd_step<T>(pl->d_psd + pl->psd_cls_begin[c], n, cfg, rho_hat, vv, sh, y, s_new, y_new, U, lam,
                       refine ? rscratch : nullptr, Uprev, stats, s);
  });
}

template <typename T>
bool launch_dk_classes(cosmo_plan *pl, const T *U, const T *lam, const T *g, T *out, T *scratch, hipStream_t st) {
  ProfScope ps(pl, 1, st);
  bool ok = true;
  fork_classes(pl, st, [&](int c, hipStream_t s) {
    const int n = pl->psd_cls_begin[c + 1] - pl->psd_cls_begin[c];
    ok = launch_psd_vjp<T>(pl->d_psd + pl->psd_cls_begin[c], n, pl->psd_cls_maxp[c], U, lam, g, out, scratch, s, 0,
                           0.0, pl->vjp_threads) &&
         ok;
  });
  return ok;
}

// ---- learned policy (App. E "Policy Parameterization") -------------------------

// Byte offsets of the policy's tape (logits of every step, the loss's
// denominators and running sum) and of its scratch.
struct PolLayout {
  size_t lr, la, acc3, ptape;
  size_t u, rp, p, w, rd, rec, coef, C, Ca, xb, ub, pb, wb, pend_st, pend_s, part, parta, pws;
  int64_t nblk;
};

PolLayout policy_layout(const cosmo_plan *pl) {
  const size_t esz = pl->esz, m = (size_t)pl->m_tot, n = (size_t)pl->n_tot, B = (size_t)pl->B;
  const size_t K = (size_t)pl->opt.K;
  PolLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + std::max<size_t>(bytes, 1), 256);
    return r;
  };
  L.lr = take((K + 1) * m * esz);
  L.la = take((K + 1) * B * esz);
  L.acc3 = take(3 * B * sizeof(double));
  L.ptape = o;
  o = 0;
  L.u = take(m * esz);
  L.rp = take(m * esz);
  L.p = take(n * esz);
  L.w = take(n * esz);
  L.rd = take(n * esz);
  L.rec = take(B * sizeof(PolRec));
  L.coef = take(B * sizeof(PolCoef));
  L.C = take(m * esz);
  L.Ca = take(B * esz);
  L.xb = take(4 * m * esz);
  L.ub = take(m * esz);
  L.pb = take(n * esz);
  L.wb = take(n * esz);
  L.pend_st = take(m * esz);
  L.pend_s = take(m * esz);
  L.nblk = pol_row_blocks(pl->m_tot);
  L.part = take((size_t)L.nblk * POL_PART_STRIDE * esz);
  L.parta = take(B * POL_ALPHA_PARAMS * esz);
  L.pws = o;
  return L;
}

// One policy call's buffers.
template <typename T> struct PolRun {
  PolLayout L;
  const T *theta = nullptr;
  T *rho = nullptr, *alpha = nullptr, *loss = nullptr;   // forward outputs
  T *lr = nullptr, *la = nullptr;                        // logits l^0..l^K (slot 0 unused: theta's)
  double *acc3 = nullptr;                                // per instance D_d, D_p, loss sum
  unsigned char *pws = nullptr;
  T *gtheta = nullptr;
  template <typename U> U *at(size_t off) const { return reinterpret_cast<U *>(pws + off); }
};

template <typename T>
PolRun<T> make_pol_run(const cosmo_plan *plan, const void *theta, void *ptape, void *pws) {
  PolRun<T> P;
  P.L = policy_layout(plan);
  P.theta = static_cast<const T *>(theta);
  auto *pt = static_cast<unsigned char *>(ptape);
  P.lr = reinterpret_cast<T *>(pt + P.L.lr);
  P.la = reinterpret_cast<T *>(pt + P.L.la);
  P.acc3 = reinterpret_cast<double *>(pt + P.L.acc3);
  P.pws = static_cast<unsigned char *>(pws);
  return P;
}
// The policy at iterate k < K (features -> logits -> rho^k, alpha^k, then
// rho^k rectified into rho_hat), or at k = K only the loss term.
template <typename T>
void policy_fwd_at(cosmo_plan *pl, const View<T> &v, const PolRun<T> &P, int k, const T *x, const T *s, const T *y,
                   const T *s_prev, const T *st_prev, T *rho_hat, hipStream_t st) {
  const size_t m = (size_t)pl->m_tot, B = (size_t)pl->B;
  const bool pol = k < pl->opt.K;
  T *u = P.template at<T>(P.L.u), *rp = P.template at<T>(P.L.rp), *p = P.template at<T>(P.L.p);
  T *w = P.template at<T>(P.L.w), *rd = P.template at<T>(P.L.rd);
  PolRec *rec = P.template at<PolRec>(P.L.rec);
  launch_pol_resid<T>(v, pl->bkA, pl->bkAt, x, s, y, u, rp, p, w, rd, st);
  launch_pol_norms<T>(v, u, rp, p, w, rd, s, s_prev, st_prev, rec, st);
  launch_pol_inst_fwd<T>(v, P.theta, rec, k, pol ? 1 : 0, k > 0 ? P.la + k * B : nullptr,
                         pol ? P.la + (k + 1) * B : nullptr, pol ? P.alpha + k * B : nullptr, P.acc3, P.loss, st);
  if (!pol) return;
  launch_pol_rho_fwd<T>(v, P.theta, rec, k > 0 ? P.lr + k * m : nullptr, P.lr + (k + 1) * m, P.rho + k * m, s, y, rp,
                        s_prev, st_prev, st);
  launch_rectify<T>(v, pl->d_rect, pl->n_rect, P.rho + k * m, rho_hat + k * m, 1, st);
}

// Reverse of the policy and of the loss term at iterate k: adds their
// cotangents of z^k into (gx, gs, gy); k = K: the loss term only.
template <typename T>
void policy_bwd_at(cosmo_plan *pl, const View<T> &v, const PolRun<T> &P, int k, const T *tape, const T *grho,
                   const T *galpha, T *gx, T *gs, T *gy, hipStream_t st) {
  const size_t m = (size_t)pl->m_tot, B = (size_t)pl->B;
  const bool pol = k < pl->opt.K;
  const T *x = tape + slot_x(pl, k), *s = tape + slot_s(pl, k), *y = tape + slot_y(pl, k);
  const T *s_prev = (pol && k > 0) ? tape + slot_s(pl, k - 1) : nullptr;
  const T *st_prev = (pol && k > 0) ? tape + step_base(pl, k - 1) + pl->tp.st : nullptr;
  T *u = P.template at<T>(P.L.u), *rp = P.template at<T>(P.L.rp), *p = P.template at<T>(P.L.p);
  T *w = P.template at<T>(P.L.w), *rd = P.template at<T>(P.L.rd), *xb = P.template at<T>(P.L.xb);
  T *C = P.template at<T>(P.L.C), *Ca = P.template at<T>(P.L.Ca);
  T *ub = P.template at<T>(P.L.ub), *pb = P.template at<T>(P.L.pb), *wb = P.template at<T>(P.L.wb);
  T *pend_st = P.template at<T>(P.L.pend_st), *pend_s = P.template at<T>(P.L.pend_s);
  PolRec *rec = P.template at<PolRec>(P.L.rec);
  PolCoef *coef = P.template at<PolCoef>(P.L.coef);
  launch_pol_resid<T>(v, pl->bkA, pl->bkAt, x, s, y, u, rp, p, w, rd, st);
  launch_pol_norms<T>(v, u, rp, p, w, rd, s, s_prev, st_prev, rec, st);
  if (pol)
    launch_pol_rho_bwd<T>(v, P.theta, rec, k > 0 ? P.lr + k * m : nullptr, s, y, rp, s_prev, st_prev, grho + k * m, C,
                          gs, gy, xb, P.template at<T>(P.L.part), st);
  launch_pol_inst_bwd<T>(v, P.theta, rec, k, pol ? 1 : 0, k >= 1 ? 1 : 0, k > 0 ? P.la + k * B : nullptr,
                         pol ? galpha + k * B : nullptr, Ca, pol ? xb : nullptr, rp, P.acc3, coef,
                         P.template at<T>(P.L.parta), st);
  launch_pol_rows_bwd<T>(v, rec, coef, pol ? xb : nullptr, rp, u, s, s_prev, st_prev, gs, ub, pend_st, pend_s,
                         pol ? 1 : 0, pol ? 1 : 0, st);
  launch_pol_cols_bwd<T>(v, rec, coef, rd, p, w, pb, wb, st);
  launch_pol_resid_adjoint<T>(v, pl->bkA, pl->bkAt, ub, pb, wb, gx, gy, st);
}

template <typename T>
cosmo_status forward_impl(cosmo_plan *pl, const T *rho, const T *alpha, const T *x0, const T *s0, const T *y0, T *xK,
                          T *sK, T *yK, T *tape, T *ws, cosmo_stats *stats, hipStream_t st,
                          const PolRun<T> *pol = nullptr, bool continues = false) {
  View<T> v = make_view<T>(pl);
  const int64_t n = pl->n_tot, m = pl->m_tot;
  const int K = pl->opt.K;
  auto &f = pl->fw;
  bind_dense(v, ws, f.dn, f.ec, f.ed);
  T *rho_hat = ws + f.rho_hat;
  // with the policy, each step's penalties are chosen and rectified at its iterate
  if (!pol) launch_rectify<T>(v, pl->d_rect, pl->n_rect, rho, rho_hat, K, st);
  auto X = [&](int k) -> T * { return tape ? tape + slot_x(pl, k) : ws + ((k & 1) ? f.itB : f.itA); };
  auto S = [&](int k) -> T * {
    return tape ? tape + slot_s(pl, k) : ws + ((k & 1) ? f.itB : f.itA) + align_up(n, 64);
  };
  auto Y = [&](int k) -> T * {
    return tape ? tape + slot_y(pl, k) : ws + ((k & 1) ? f.itB : f.itA) + align_up(n, 64) + align_up(m, 64);
  };
  auto XT = [&](int k) -> T * { return tape ? tape + step_base(pl, k) + pl->tp.xt : ws + f.xt; };
  auto ST = [&](int k) -> T * { return tape ? tape + step_base(pl, k) + pl->tp.st : ws + f.st; };
  auto LAM = [&](int k) -> T * { return tape ? tape + step_base(pl, k) + pl->tp.lam : ws + f.lam; };
  auto UU = [&](int k) -> T * { return tape ? tape + step_base(pl, k) + pl->tp.U : ws + f.U; };
  if (x0) launch_copy<T>(X(0), x0, n, st); else launch_fill<T>(X(0), (T)0, n, st);
  if (s0) launch_copy<T>(S(0), s0, m, st); else launch_fill<T>(S(0), (T)0, m, st);
  if (y0) launch_copy<T>(Y(0), y0, m, st); else launch_fill<T>(Y(0), (T)0, m, st);
  for (int k = 0; k < K; ++k) {
    // s^{k-1} and the s~ that produced s^k: without a tape they are the other
    // iterate buffer and the single s~ buffer, both still intact here
    if (pol) policy_fwd_at<T>(pl, v, *pol, k, X(k), S(k), Y(k), k > 0 ? S(k - 1) : nullptr, k > 0 ? ST(k - 1) : nullptr,
                              rho_hat, st);
    const T *rh = rho_hat + (size_t)k * m;
    const T *al = (pol ? pol->alpha : alpha) + (size_t)k * pl->B;
    T *x = X(k), *s = S(k), *y = Y(k), *xn = X(k + 1), *sn = S(k + 1), *yn = Y(k + 1);
    T *xt = XT(k);
    DiagSolve<T> ds;
    if (pl->diag_M) {
      ds.xt = xt;
      ds.xn = xn;
      ds.alpha_k = al;
    } else {
      // warm start of the CG: previous x~ (first step: x^0; a call that
      // continues the previous one without a tape keeps that call's last x~)
      if (tape) launch_copy<T>(xt, k == 0 ? x : XT(k - 1), n, st);
      else if (k == 0 && !continues) launch_copy<T>(xt, x, n, st);
    }
    {
      ProfScope ps(pl, 3, st);
      launch_dense_cols<T>(v, DC_XI, rh, y, s, st);
      launch_cols_pre<T>(v, pl->bkAt, rh, x, s, y, ws + f.dg, reinterpret_cast<double *>(ws + f.xi), ds, st);
    }
    if (!pl->diag_M) {
      ProfScope ps(pl, 2, st);
      launch_pcg<T>(v, rh, ws + f.dg, reinterpret_cast<const double *>(ws + f.xi), xt, ws + f.r, ws + f.z, ws + f.p, ws + f.Mp, ws + f.t,
                    reinterpret_cast<double *>(ws + f.t64), pl->opt.cg_tol, pl->opt.cg_max_iter, al, x, xn, nullptr, nullptr, 0, stats, ws + f.cg, pl->pcg_form, st);
    }
    {
      ProfScope ps(pl, 3, st);
      launch_dense_rows<T>(v, xt, st);
      launch_rows_post<T>(v, pl->bkA, rh, al, xt, s, y, ST(k), ws + f.sh, ws + f.vv, sn, yn, st);
    }
    launch_soc_step<T>(pl->d_soc, pl->n_soc, rh, ws + f.vv, ws + f.sh, y, sn, yn, st);
    // warm start from the previous step's eigenvectors of the same blocks (the
    // tape keeps them; without a tape the single buffer is updated in place,
    // each block reading its own slot before overwriting it)
    const T *Uprev = (pl->opt.eig_warm_start && (k > 0 || (continues && !tape))) ? (tape ? UU(k - 1) : UU(k))
                                                                                  : nullptr;
    launch_psd_classes<T>(pl, rh, ws + f.vv, ws + f.sh, y, sn, yn, UU(k), LAM(k),
                          reinterpret_cast<double *>(ws + f.rs), Uprev, stats, st);
  }
  if (pol) policy_fwd_at<T>(pl, v, *pol, K, X(K), S(K), Y(K), nullptr, nullptr, rho_hat, st);
  launch_nonfinite_check<T>(v, X(K), S(K), Y(K), stats, st);
  if (xK) launch_copy<T>(xK, X(K), n, st);
  if (sK) launch_copy<T>(sK, S(K), m, st);
  if (yK) launch_copy<T>(yK, Y(K), m, st);
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

// ---- vanilla COSMO to tolerance (residual balancing) ------------------------------

struct SolveLayout {
  size_t rho, alpha, rho_b, u, rp, p, w, rd, rec, xs, ss, ys, total;
};

SolveLayout solve_layout(const cosmo_plan *pl) {
  const size_t esz = pl->esz, m = (size_t)pl->m_tot, n = (size_t)pl->n_tot, B = (size_t)pl->B;
  const size_t K = (size_t)pl->opt.K;
  SolveLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + std::max<size_t>(bytes, 1), 256);
    return r;
  };
  L.rho = take(K * m * esz);
  L.alpha = take(K * B * esz);
  L.rho_b = take(B * sizeof(double));
  L.u = take(m * esz);
  L.rp = take(m * esz);
  L.p = take(n * esz);
  L.w = take(n * esz);
  L.rd = take(n * esz);
  L.rec = take(B * sizeof(PolRec));
  L.xs = take(n * esz);   // each instance's iterate at its own count
  L.ss = take(m * esz);
  L.ys = take(m * esz);
  L.total = o;
  return L;
}

template <typename T>
cosmo_status solve_impl(cosmo_plan *pl, const cosmo_solve_options &o, T *x, T *s, T *y, int32_t *iters,
                        double *rho_out, T *ws, unsigned char *sws, cosmo_stats *stats, hipStream_t st) {
  const SolveLayout L = solve_layout(pl);
  const int K = pl->opt.K, B = pl->B;
  View<T> v = make_view<T>(pl);
  bind_dense(v, ws, pl->fw.dn, pl->fw.ec, pl->fw.ed);
  T *rho = reinterpret_cast<T *>(sws + L.rho), *alpha = reinterpret_cast<T *>(sws + L.alpha);
  double *rho_b_d = reinterpret_cast<double *>(sws + L.rho_b);
  T *u = reinterpret_cast<T *>(sws + L.u), *rp = reinterpret_cast<T *>(sws + L.rp);
  T *p = reinterpret_cast<T *>(sws + L.p), *w = reinterpret_cast<T *>(sws + L.w);
  T *rd = reinterpret_cast<T *>(sws + L.rd);
  PolRec *rec = reinterpret_cast<PolRec *>(sws + L.rec);
  std::vector<double> rho_b(B, o.rho0);
  std::vector<PolRec> hrec(B);
  std::vector<char> done(B, 0);
  for (int b = 0; b < B; ++b) iters[b] = -1;
  launch_fill<T>(alpha, (T)o.alpha, (int64_t)K * B, st);
  auto upload = [&]() -> cosmo_status {
    HIPCHK(hipMemcpyAsync(rho_b_d, rho_b.data(), B * sizeof(double), hipMemcpyHostToDevice, st));
    launch_solve_rho<T>(v, rho_b_d, o.eq_scale, rho, K, st);
    return COSMO_OK;
  };
  T *xs = reinterpret_cast<T *>(sws + L.xs), *ss = reinterpret_cast<T *>(sws + L.ss);
  T *ys = reinterpret_cast<T *>(sws + L.ys);
  // copies instance b's slices of (x, s, y) into the saved iterate or back
  auto save = [&](int b, bool out) -> cosmo_status {
    const int64_t n0 = pl->n_off[b], n1 = pl->n_off[b + 1], m0 = pl->m_off[b], m1 = pl->m_off[b + 1];
    const hipMemcpyKind kd = hipMemcpyDeviceToDevice;
    if (n1 > n0) HIPCHK(hipMemcpyAsync(out ? xs + n0 : x + n0, out ? x + n0 : xs + n0, (n1 - n0) * sizeof(T), kd, st));
    if (m1 > m0) {
      HIPCHK(hipMemcpyAsync(out ? ss + m0 : s + m0, out ? s + m0 : ss + m0, (m1 - m0) * sizeof(T), kd, st));
      HIPCHK(hipMemcpyAsync(out ? ys + m0 : y + m0, out ? y + m0 : ys + m0, (m1 - m0) * sizeof(T), kd, st));
    }
    return COSMO_OK;
  };
  cosmo_status r = upload();
  if (r != COSMO_OK) return r;
  int remaining = B;
  for (int it = K; it <= o.max_iter && remaining > 0; it += K) {
    // each call continues the previous one (CG and eigensolver warm starts kept)
    r = forward_impl<T>(pl, rho, alpha, x, s, y, x, s, y, nullptr, ws, stats, st, nullptr, it > K);
    if (r != COSMO_OK) return r;
    // the residual vectors and per-instance norms of the policy's features
    launch_pol_resid<T>(v, pl->bkA, pl->bkAt, x, s, y, u, rp, p, w, rd, st);
    launch_pol_norms<T>(v, u, rp, p, w, rd, s, nullptr, nullptr, rec, st);
    HIPCHK(hipMemcpyAsync(hrec.data(), rec, B * sizeof(PolRec), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool changed = false;
    for (int b = 0; b < B; ++b) {
      if (done[b]) continue;
      const PolRec &R = hrec[b];
      const double Np = std::max(std::max(R.nu, R.ns), R.nb), Nd = std::max(std::max(R.np, R.nq), R.nw);
      if (R.mrp <= o.eps_abs + o.eps_rel * Np && R.mrd <= o.eps_abs + o.eps_rel * Nd) {
        done[b] = 1;
        iters[b] = it;
        --remaining;
        // the batch keeps stepping for the others: keep this instance's iterate
        r = save(b, true);
        if (r != COSMO_OK) return r;
        continue;
      }
      if (o.adapt && it % o.interval == 0 && Np > 0 && Nd > 0 && R.mrd > 0) {
        const double nr = std::min(std::max(rho_b[b] * std::sqrt((R.mrp / Np) / (R.mrd / Nd)), o.rho_min),
                                   o.rho_max);
        if (nr > o.tol_factor * rho_b[b] || nr < rho_b[b] / o.tol_factor) {
          rho_b[b] = nr;
          changed = true;
        }
      }
    }
    if (changed && remaining > 0) {
      r = upload();
      if (r != COSMO_OK) return r;
    }
  }
  for (int b = 0; b < B; ++b)
    if (done[b]) {
      r = save(b, false);
      if (r != COSMO_OK) return r;
    }
  if (rho_out)
    for (int b = 0; b < B; ++b) rho_out[b] = rho_b[b];
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

template <typename T>
cosmo_status backward_impl(cosmo_plan *pl, const T *rho, const T *alpha, const T *tape, const T *gxK, const T *gsK,
                           const T *gyK, T *grho, T *galpha, T *gx0, T *gs0, T *gy0, T *ws, cosmo_stats *stats,
                           hipStream_t st, const PolRun<T> *pol = nullptr) {
  View<T> v = make_view<T>(pl);
  const int64_t n = pl->n_tot, m = pl->m_tot;
  const int K = pl->opt.K;
  auto &w = pl->bw;
  bind_dense(v, ws, w.dn, w.ec, w.ed);
  T *rho_hat = ws + w.rho_hat;
  launch_rectify<T>(v, pl->d_rect, pl->n_rect, rho, rho_hat, K, st);
  const size_t on = 0, os = align_up(n, 64), oy = align_up(n, 64) + align_up(m, 64);
  T *gA = ws + w.gA, *gB = ws + w.gB;
  if (gxK) launch_copy<T>(gA + on, gxK, n, st); else launch_fill<T>(gA + on, (T)0, n, st);
  if (gsK) launch_copy<T>(gA + os, gsK, m, st); else launch_fill<T>(gA + os, (T)0, m, st);
  if (gyK) launch_copy<T>(gA + oy, gyK, m, st); else launch_fill<T>(gA + oy, (T)0, m, st);
  T *pend_st = nullptr;
  if (pol) {
    // the policy's accumulators start at zero; the loss term at z^K seeds the reverse pass
    pend_st = pol->template at<T>(pol->L.pend_st);
    launch_fill<T>(pol->template at<T>(pol->L.C), (T)0, m, st);
    launch_fill<T>(pol->template at<T>(pol->L.Ca), (T)0, pl->B, st);
    launch_fill<T>(pend_st, (T)0, m, st);
    launch_fill<T>(pol->template at<T>(pol->L.pend_s), (T)0, m, st);
    launch_fill<T>(pol->template at<T>(pol->L.part), (T)0, pol->L.nblk * POL_PART_STRIDE, st);
    launch_fill<T>(pol->template at<T>(pol->L.parta), (T)0, (int64_t)pl->B * POL_ALPHA_PARAMS, st);
    policy_bwd_at<T>(pl, v, *pol, K, tape, grho, galpha, gA + on, gA + os, gA + oy, st);
  }
  launch_fill<T>(ws + w.w, (T)0, n, st);
  launch_fill<T>(ws + w.gsn, (T)0, m, st);
  T *scratch = ws + w.dk;
  for (int k = K - 1; k >= 0; --k) {
    const T *rh = rho_hat + (size_t)k * m;
    const T *al = alpha + (size_t)k * pl->B;
    const T *x = tape + slot_x(pl, k), *s = tape + slot_s(pl, k), *y = tape + slot_y(pl, k);
    const T *sn = tape + slot_s(pl, k + 1);
    const T *xt = tape + step_base(pl, k) + pl->tp.xt, *stl = tape + step_base(pl, k) + pl->tp.st;
    const T *lam = tape + step_base(pl, k) + pl->tp.lam, *U = tape + step_base(pl, k) + pl->tp.U;
    T *gx_in = gA + on, *gs_in = gA + os, *gy_in = gA + oy;
    T *gx_out = gB + on, *gs_out = gB + os, *gy_out = gB + oy;
    {
      ProfScope ps(pl, 3, st);
      launch_bwd_rows_a<T>(v, rh, al, stl, s, y, sn, gs_in, gy_in, ws + w.gsn, ws + w.gv, pl->tap != nullptr, st);
    }
    if (pl->n_soc > 0 || pl->n_psd > 0 || pl->tap) {
      // v = s^ + y / rho_hat on every row, recomputed from the tape
      launch_rows_v<T>(v, rh, al, stl, s, y, ws + w.vv, st);
    }
    if (pl->tap) {   // v^k and the cotangent of the projection's output
      T *tp = static_cast<T *>(pl->tap) + (size_t)k * 2 * m;
      launch_copy<T>(tp, ws + w.vv, m, st);
      launch_copy<T>(tp + m, ws + w.gsn, m, st);
    }
    launch_soc_vjp<T>(pl->d_soc, pl->n_soc, ws + w.vv, ws + w.gsn, ws + w.gv, st);
    if (!launch_dk_classes<T>(pl, U, lam, ws + w.gsn, ws + w.gv, scratch, st))
      FAIL(COSMO_EUNSUPPORTED, "a PSD block is too large for the VJP's LDS layout");
    {
      ProfScope ps(pl, 3, st);
      launch_bwd_rows_b<T>(v, rh, al, stl, s, y, sn, gy_in, ws + w.gv, ws + w.gsh, ws + w.gst, gs_out, gy_out,
                           ws + w.grh, pend_st, st);
      DiagSolve<T> ds;
      if (pl->diag_M) {
        ds.xt = ws + w.w;
        ds.xn = gx_out;
        ds.alpha_k = al;
      }
      launch_dense_cols<T>(v, DC_GST, rh, ws + w.gst, nullptr, st);
      launch_bwd_cols<T>(v, pl->bkAt, rh, al, ws + w.gst, gx_in, reinterpret_cast<double *>(ws + w.gxt), ws + w.dg, ds, st);
    }
    if (!pl->diag_M) {
      ProfScope ps(pl, 2, st);
      launch_pcg<T>(v, rh, ws + w.dg, reinterpret_cast<const double *>(ws + w.gxt), ws + w.w, ws + w.r, ws + w.z, ws + w.p, ws + w.Mp, ws + w.t,
                    reinterpret_cast<double *>(ws + w.t64), pl->opt.cg_tol, pl->opt.cg_max_iter, al, nullptr, nullptr, gx_in, gx_out, 1, stats, ws + w.cg,
                    pl->pcg_form, st);
    }
    {
      ProfScope ps(pl, 3, st);
      launch_dense_rows<T>(v, ws + w.w, st);
      launch_bwd_rows_c<T>(v, pl->bkA, rh, ws + w.w, stl, s, ws + w.grh, gs_out, gy_out, st);
    }
    if (grho) launch_rect_adjoint<T>(v, pl->d_rect, pl->n_rect, ws + w.grh, grho + (size_t)k * m, st);
    if (galpha) launch_alpha_reduce<T>(v, ws + w.gsh, stl, s, gx_in, xt, x, galpha + (size_t)k * pl->B, st);
    if (pol) policy_bwd_at<T>(pl, v, *pol, k, tape, grho, galpha, gx_out, gs_out, gy_out, st);
    std::swap(gA, gB);
  }
  if (pol)
    launch_pol_grad<T>(v, pol->template at<T>(pol->L.part), pol->L.nblk, pol->template at<T>(pol->L.parta),
                       pol->template at<T>(pol->L.Ca), pol->gtheta, st);
  if (gx0) launch_copy<T>(gx0, gA + on, n, st);
  if (gs0) launch_copy<T>(gs0, gA + os, m, st);
  if (gy0) launch_copy<T>(gy0, gA + oy, m, st);
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

// Runs `body(stream)` eagerly on `st`, or in graph mode replays the recorded
// sequence for this argument set (recording it first if the set is new).
// Profiling runs are always eager (their events are read back by the host).
template <typename F>
cosmo_status run_recorded(cosmo_plan *pl, cosmo_plan::Recorded &rec, std::vector<const void *> key, hipStream_t st,
                          F &&body) {
  if (!pl->graph || pl->profiling) return body(st);
  if (!rec.exec || rec.key != key) {
    if (rec.exec) (void)hipGraphExecDestroy(rec.exec);
    rec.exec = nullptr;
    rec.key.clear();
    HIPCHK(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeRelaxed));
    const cosmo_status s = body(pl->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(pl->cap, &g);
    if (s != COSMO_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess || !g) FAIL(COSMO_EHIP, std::string("recording the unroll failed: ") + hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&rec.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      rec.exec = nullptr;
      FAIL(COSMO_EHIP, std::string("instantiating the recorded unroll failed: ") + hipGetErrorString(ei));
    }
    rec.key = std::move(key);
  }
  HIPCHK(hipGraphLaunch(rec.exec, st));
  return COSMO_OK;
}

cosmo_status check_plan(const cosmo_plan *pl) {
  if (!pl) FAIL(COSMO_EINVAL, "plan is NULL");
  return COSMO_OK;
}

}  // namespace

// ============================ C ABI ============================================

extern "C" {

const char *cosmo_status_string(cosmo_status s) {
  switch (s) {
    case COSMO_OK: return "COSMO_OK";
    case COSMO_EINVAL: return "COSMO_EINVAL: invalid argument";
    case COSMO_ENOMEM: return "COSMO_ENOMEM: allocation failed";
    case COSMO_EHIP: return "COSMO_EHIP: HIP runtime error";
    case COSMO_EUNSUPPORTED: return "COSMO_EUNSUPPORTED: outside the implemented envelope";
  }
  return "unknown cosmo_status";
}

const char *cosmo_last_error(void) { return cosmo::g_last_error.c_str(); }

int32_t cosmo_abi_version(void) { return ABI_VERSION; }

cosmo_status cosmo_plan_create(cosmo_plan **plan, const cosmo_problem *prob, const cosmo_options *opt) {
  if (!plan) FAIL(COSMO_EINVAL, "plan out-pointer is NULL");
  *plan = nullptr;
  cosmo_status s = validate_options(opt);
  if (s != COSMO_OK) return s;
  s = validate_problem_host(prob, opt);
  if (s != COSMO_OK) return s;
  cosmo_plan *pl = new (std::nothrow) cosmo_plan();
  if (!pl) FAIL(COSMO_ENOMEM, "host allocation failed");
  pl->opt = *opt;
  pl->B = prob->B;
  pl->n_off.assign(prob->n_off, prob->n_off + prob->B + 1);
  pl->m_off.assign(prob->m_off, prob->m_off + prob->B + 1);
  pl->n_tot = pl->n_off.back();
  pl->m_tot = pl->m_off.back();
  pl->esz = opt->dtype == COSMO_F32 ? 4 : 8;
  pl->A_rowptr = prob->A_rowptr;
  pl->A_col = prob->A_col;
  pl->A_val = prob->A_val;
  pl->A_nnz = prob->A_nnz;
  pl->P_rowptr = prob->P_rowptr;
  pl->P_col = prob->P_col;
  pl->P_val = prob->P_val;
  pl->P_nnz = prob->P_nnz;
  pl->q = prob->q;
  pl->b = prob->b;
  s = (opt->dtype == COSMO_F32) ? build_plan<float>(pl, prob) : build_plan<double>(pl, prob);
  if (s != COSMO_OK) {
    delete pl;
    return s;
  }
  build_layouts(pl);
  for (int i = 0; i < 3; ++i) {
    if (hipStreamCreateWithFlags(&pl->aux[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&pl->ev_join[i], hipEventDisableTiming) != hipSuccess) {
      delete pl;
      FAIL(COSMO_EHIP, "creating auxiliary streams failed");
    }
  }
  if (hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking) != hipSuccess) {
    delete pl;
    FAIL(COSMO_EHIP, "creating events failed");
  }
  *plan = pl;
  return COSMO_OK;
}

cosmo_status cosmo_plan_destroy(cosmo_plan *plan) {
  if (!plan) return COSMO_OK;
  (void)hipDeviceSynchronize();
  delete plan;
  return COSMO_OK;
}

cosmo_status cosmo_workspace_size(const cosmo_plan *plan, size_t *fwd, size_t *tape, size_t *bwd) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (fwd) *fwd = plan->fw.total * plan->esz;
  if (tape) *tape = plan->tp.total * plan->esz;
  if (bwd) *bwd = plan->bw.total * plan->esz;
  return COSMO_OK;
}

cosmo_status cosmo_tape_offsets(const cosmo_plan *plan, int32_t k, size_t *x_off, size_t *s_off, size_t *y_off,
                                size_t *xt_off, size_t *st_off) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (k < 0 || k > plan->opt.K) FAIL(COSMO_EINVAL, "k out of range [0, K]");
  if (k == plan->opt.K && (xt_off || st_off)) FAIL(COSMO_EINVAL, "x~ and s~ exist for steps 0..K-1 only");
  const size_t e = plan->esz;
  if (x_off) *x_off = slot_x(plan, k) * e;
  if (s_off) *s_off = slot_s(plan, k) * e;
  if (y_off) *y_off = slot_y(plan, k) * e;
  if (xt_off) *xt_off = (step_base(plan, k) + plan->tp.xt) * e;
  if (st_off) *st_off = (step_base(plan, k) + plan->tp.st) * e;
  return COSMO_OK;
}

cosmo_status cosmo_unroll_forward(cosmo_plan *plan, const void *rho, const void *alpha, const void *x0,
                                  const void *s0, const void *y0, void *xK, void *sK, void *yK, void *tape, void *ws,
                                  void *stats, void *stream) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!rho || !alpha) FAIL(COSMO_EINVAL, "rho and alpha are required");
  if (!ws) FAIL(COSMO_EINVAL, "workspace is required");
  auto *stp = static_cast<cosmo_stats *>(stats);
  return run_recorded(plan, plan->rec_fwd, {rho, alpha, x0, s0, y0, xK, sK, yK, tape, ws, stats},
                      static_cast<hipStream_t>(stream), [&](hipStream_t st) {
    if (plan->opt.dtype == COSMO_F32)
      return forward_impl<float>(plan, (const float *)rho, (const float *)alpha, (const float *)x0,
                                 (const float *)s0, (const float *)y0, (float *)xK, (float *)sK, (float *)yK,
                                 (float *)tape, (float *)ws, stp, st);
    return forward_impl<double>(plan, (const double *)rho, (const double *)alpha, (const double *)x0,
                                (const double *)s0, (const double *)y0, (double *)xK, (double *)sK, (double *)yK,
                                (double *)tape, (double *)ws, stp, st);
  });
}

cosmo_status cosmo_unroll_backward(cosmo_plan *plan, const void *rho, const void *alpha, const void *tape,
                                   const void *gxK, const void *gsK, const void *gyK, void *grho, void *galpha,
                                   void *gx0, void *gs0, void *gy0, void *ws, void *stats, void *stream) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!rho || !alpha) FAIL(COSMO_EINVAL, "rho and alpha are required");
  if (!tape) FAIL(COSMO_EINVAL, "the backward pass needs the tape written by cosmo_unroll_forward");
  if (!ws) FAIL(COSMO_EINVAL, "workspace is required");
  auto *stp = static_cast<cosmo_stats *>(stats);
  return run_recorded(plan, plan->rec_bwd,
                      {rho, alpha, tape, gxK, gsK, gyK, grho, galpha, gx0, gs0, gy0, ws, stats, plan->tap},
                      static_cast<hipStream_t>(stream), [&](hipStream_t st) {
    if (plan->opt.dtype == COSMO_F32)
      return backward_impl<float>(plan, (const float *)rho, (const float *)alpha, (const float *)tape,
                                  (const float *)gxK, (const float *)gsK, (const float *)gyK, (float *)grho,
                                  (float *)galpha, (float *)gx0, (float *)gs0, (float *)gy0, (float *)ws, stp, st);
    return backward_impl<double>(plan, (const double *)rho, (const double *)alpha, (const double *)tape,
                                 (const double *)gxK, (const double *)gsK, (const double *)gyK, (double *)grho,
                                 (double *)galpha, (double *)gx0, (double *)gs0, (double *)gy0, (double *)ws, stp, st);
  });
}

cosmo_status cosmo_policy_sizes(const cosmo_plan *plan, size_t *ptape_bytes, size_t *pws_bytes) {
  cosmo_status s0 = check_plan(plan);
  if (s0 != COSMO_OK) return s0;
  const PolLayout L = policy_layout(plan);
  if (ptape_bytes) *ptape_bytes = L.ptape;
  if (pws_bytes) *pws_bytes = L.pws;
  return COSMO_OK;
}

cosmo_status cosmo_policy_forward(cosmo_plan *plan, const void *theta, const void *x0, const void *s0,
                                  const void *y0, void *rho, void *alpha, void *xK, void *sK, void *yK, void *loss,
                                  void *tape, void *ptape, void *ws, void *pws, void *stats, void *stream) {
  cosmo_status st0 = check_plan(plan);
  if (st0 != COSMO_OK) return st0;
  if (!theta || !rho || !alpha || !loss || !ptape || !ws || !pws)
    FAIL(COSMO_EINVAL, "theta, rho, alpha, loss, ptape, ws and pws are required");
  auto *stp = static_cast<cosmo_stats *>(stats);
  hipStream_t st = static_cast<hipStream_t>(stream);
  cosmo_status r;
  if (plan->opt.dtype == COSMO_F32) {
    PolRun<float> P = make_pol_run<float>(plan, theta, ptape, pws);
    P.rho = (float *)rho;
    P.alpha = (float *)alpha;
    P.loss = (float *)loss;
    r = forward_impl<float>(plan, nullptr, nullptr, (const float *)x0, (const float *)s0, (const float *)y0,
                            (float *)xK, (float *)sK, (float *)yK, (float *)tape, (float *)ws, stp, st, &P);
  } else {
    PolRun<double> P = make_pol_run<double>(plan, theta, ptape, pws);
    P.rho = (double *)rho;
    P.alpha = (double *)alpha;
    P.loss = (double *)loss;
    r = forward_impl<double>(plan, nullptr, nullptr, (const double *)x0, (const double *)s0, (const double *)y0,
                             (double *)xK, (double *)sK, (double *)yK, (double *)tape, (double *)ws, stp, st, &P);
  }
  if (r != COSMO_OK) return r;
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

cosmo_status cosmo_policy_backward(cosmo_plan *plan, const void *theta, const void *rho, const void *alpha,
                                   const void *tape, const void *ptape, void *gtheta, void *grho, void *galpha,
                                   void *gx0, void *gs0, void *gy0, void *ws, void *pws, void *stats,
                                   void *stream) {
  cosmo_status st0 = check_plan(plan);
  if (st0 != COSMO_OK) return st0;
  if (!theta || !rho || !alpha || !tape || !ptape || !gtheta || !grho || !galpha || !ws || !pws)
    FAIL(COSMO_EINVAL, "theta, rho, alpha, tape, ptape, gtheta, grho, galpha, ws and pws are required");
  auto *stp = static_cast<cosmo_stats *>(stats);
  hipStream_t st = static_cast<hipStream_t>(stream);
  cosmo_status r;
  if (plan->opt.dtype == COSMO_F32) {
    PolRun<float> P = make_pol_run<float>(plan, theta, const_cast<void *>(ptape), pws);
    P.gtheta = (float *)gtheta;
    r = backward_impl<float>(plan, (const float *)rho, (const float *)alpha, (const float *)tape, nullptr, nullptr,
                             nullptr, (float *)grho, (float *)galpha, (float *)gx0, (float *)gs0, (float *)gy0,
                             (float *)ws, stp, st, &P);
  } else {
    PolRun<double> P = make_pol_run<double>(plan, theta, const_cast<void *>(ptape), pws);
    P.gtheta = (double *)gtheta;
    r = backward_impl<double>(plan, (const double *)rho, (const double *)alpha, (const double *)tape, nullptr,
                              nullptr, nullptr, (double *)grho, (double *)galpha, (double *)gx0, (double *)gs0,
                              (double *)gy0, (double *)ws, stp, st, &P);
  }
  if (r != COSMO_OK) return r;
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

cosmo_status cosmo_solve_size(const cosmo_plan *plan, size_t *sws_bytes) {
  cosmo_status s0 = check_plan(plan);
  if (s0 != COSMO_OK) return s0;
  if (sws_bytes) *sws_bytes = solve_layout(plan).total;
  return COSMO_OK;
}

cosmo_status cosmo_solve(cosmo_plan *plan, const cosmo_solve_options *opt, void *x, void *s, void *y,
                         int32_t *iters, double *rho_out, void *ws, void *sws, void *stats, void *stream) {
  cosmo_status st0 = check_plan(plan);
  if (st0 != COSMO_OK) return st0;
  if (!opt || !x || !s || !y || !iters || !ws || !sws) FAIL(COSMO_EINVAL, "opt, x, s, y, iters, ws and sws are required");
  const cosmo_solve_options &o = *opt;
  if (!(o.rho_min > 0 && o.rho_min <= o.rho0 && o.rho0 <= o.rho_max && std::isfinite(o.rho_max)))
    FAIL(COSMO_EINVAL, "need 0 < rho_min <= rho0 <= rho_max < inf");
  if (!(o.eq_scale > 0 && std::isfinite(o.eq_scale))) FAIL(COSMO_EINVAL, "eq_scale must be positive and finite");
  if (!(o.alpha > 0 && o.alpha < 2)) FAIL(COSMO_EINVAL, "alpha must lie in (0, 2)");
  if (!(o.eps_abs >= 0 && o.eps_rel >= 0 && o.eps_abs + o.eps_rel > 0))
    FAIL(COSMO_EINVAL, "eps_abs and eps_rel must be >= 0 and not both 0");
  if (!(o.tol_factor >= 1)) FAIL(COSMO_EINVAL, "tol_factor must be >= 1");
  if (o.max_iter < 1) FAIL(COSMO_EINVAL, "max_iter must be >= 1");
  if (o.adapt != 0 && o.adapt != 1) FAIL(COSMO_EINVAL, "adapt must be 0 or 1");
  if (o.interval < 1 || o.interval % plan->opt.K != 0) FAIL(COSMO_EINVAL, "interval must be a positive multiple of K");
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto *stp = static_cast<cosmo_stats *>(stats);
  auto *sw = static_cast<unsigned char *>(sws);
  if (plan->opt.dtype == COSMO_F32)
    return solve_impl<float>(plan, o, (float *)x, (float *)s, (float *)y, iters, rho_out, (float *)ws, sw, stp, st);
  return solve_impl<double>(plan, o, (double *)x, (double *)s, (double *)y, iters, rho_out, (double *)ws, sw, stp, st);
}

cosmo_status cosmo_residual_loss(cosmo_plan *plan, const void *x, const void *s, const void *y, void *loss, void *gx,
                                 void *gs, void *gy, void *ws, void *stream) {
  cosmo_status st0 = check_plan(plan);
  if (st0 != COSMO_OK) return st0;
  if (!x || !s || !y || !loss || !ws) FAIL(COSMO_EINVAL, "x, s, y, loss and ws are required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (plan->opt.dtype == COSMO_F32) {
    View<float> v = make_view<float>(plan);
    float *w = (float *)ws;
    bind_dense(v, w, plan->fw.dn, plan->fw.ec, plan->fw.ed);
    launch_loss<float>(v, plan->bkA, plan->bkAt, (const float *)x, (const float *)s, (const float *)y, w + plan->fw.rp,
                       w + plan->fw.rd, (float *)loss, (float *)gx, (float *)gs, (float *)gy, st);
  } else {
    View<double> v = make_view<double>(plan);
    double *w = (double *)ws;
    bind_dense(v, w, plan->fw.dn, plan->fw.ec, plan->fw.ed);
    launch_loss<double>(v, plan->bkA, plan->bkAt, (const double *)x, (const double *)s, (const double *)y,
                        w + plan->fw.rp, w + plan->fw.rd, (double *)loss, (double *)gx, (double *)gs, (double *)gy, st);
  }
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

// ---- schedules -------------------------------------------------------------------

cosmo_status cosmo_plan_set_pcg_form(cosmo_plan *plan, int32_t form) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (form < 0 || form > 4) FAIL(COSMO_EINVAL, "form must be 0..4");
  if (form != 0 && plan->graph) FAIL(COSMO_EUNSUPPORTED, "the cooperative CG forms are not recorded into graphs");
  if (form != 0 && plan->n_dense > 0) FAIL(COSMO_EUNSUPPORTED, "dense sub-blocks are applied by CG form 0 only");
  plan->pcg_form = form;
  return COSMO_OK;
}

cosmo_status cosmo_plan_set_graph(cosmo_plan *plan, int32_t enable) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (enable != 0 && enable != 1) FAIL(COSMO_EINVAL, "enable must be 0 or 1");
  if (enable && plan->pcg_form != 0 && !plan->diag_M)
    FAIL(COSMO_EUNSUPPORTED, "the cooperative CG forms are not recorded into graphs");
  plan->drop_graphs();
  plan->graph = enable != 0;
  return COSMO_OK;
}

cosmo_status cosmo_plan_get_graph(const cosmo_plan *plan, int32_t *enabled) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!enabled) FAIL(COSMO_EINVAL, "enabled is NULL");
  *enabled = plan->graph ? 1 : 0;
  return COSMO_OK;
}

cosmo_status cosmo_plan_get_pcg_form(const cosmo_plan *plan, int32_t *form) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!form) FAIL(COSMO_EINVAL, "form is NULL");
  *form = plan->pcg_form;
  return COSMO_OK;
}

cosmo_status cosmo_plan_set_psd_schedule(cosmo_plan *plan, const int32_t *eig_threads, int32_t vjp_threads) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!eig_threads) FAIL(COSMO_EINVAL, "eig_threads is NULL");
  for (int c = 0; c < 4; ++c)
    if (eig_threads[c] != kEigThreads[c] && eig_threads[c] != kEigThreadsAlt[c])
      FAIL(COSMO_EINVAL, "eig_threads[" + std::to_string(c) + "] must be " + std::to_string(kEigThreads[c]) +
                             (kEigThreadsAlt[c] != kEigThreads[c] ? " or " + std::to_string(kEigThreadsAlt[c]) : ""));
  if (vjp_threads != kVjpThreads && vjp_threads != kVjpThreadsAlt) FAIL(COSMO_EINVAL, "vjp_threads must be 512 or 1024");
  plan->drop_graphs();   // recorded sequences hold the previous launch shapes
  for (int c = 0; c < 4; ++c) plan->eig_threads[c] = eig_threads[c];
  plan->vjp_threads = vjp_threads;
  return COSMO_OK;
}

cosmo_status cosmo_plan_get_psd_schedule(const cosmo_plan *plan, int32_t *eig_threads, int32_t *vjp_threads) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!eig_threads || !vjp_threads) FAIL(COSMO_EINVAL, "eig_threads and vjp_threads are required");
  for (int c = 0; c < 4; ++c) eig_threads[c] = plan->eig_threads[c];
  *vjp_threads = plan->vjp_threads;
  return COSMO_OK;
}

}  // extern "C"

namespace {

// Second phase of the autotuner: the PSD launch shapes, with the CG schedule
// already fixed.  Each order class's eigensolve is timed alone by the plan's
// per-class events over a forward run under the class defaults and one under
// the alternatives (the first run of each warms code objects and caches); a
// class keeps the shape that ran faster.  The DK VJP is then timed under both
// thread counts on the eigenpairs the last forward step left in the workspace
// (its cost does not depend on the values), with a scratch cotangent.
template <typename T>
cosmo_status tune_psd(cosmo_plan *pl, const void *rho, const void *alpha, void *ws, hipStream_t st, void *xK, void *sK,
                      void *yK, hipEvent_t e0, hipEvent_t e1) {
  cosmo_status s = COSMO_OK;
  bool has[4];
  for (int c = 0; c < 4; ++c) has[c] = pl->psd_cls_begin[c + 1] > pl->psd_cls_begin[c];
  for (int a = 0; a < 2 && s == COSMO_OK; ++a) {
    for (int c = 0; c < 4; ++c) pl->eig_threads[c] = a ? kEigThreadsAlt[c] : kEigThreads[c];
    for (int rep = 0; rep < 2 && s == COSMO_OK; ++rep) {
      pl->profiling = true;
      for (auto &sl : pl->prof) sl.used = 0;
      s = cosmo_unroll_forward(pl, rho, alpha, nullptr, nullptr, nullptr, xK, sK, yK, nullptr, ws, nullptr, st);
    }
    for (int c = 0; c < 4 && s == COSMO_OK; ++c)
      if (has[c]) s = cosmo_plan_profile_read(pl, 4 + c, nullptr, &pl->psd_tune_ms[a][c]);
  }
  pl->profiling = false;
  for (auto &sl : pl->prof) sl.used = 0;
  for (int c = 0; c < 4; ++c)
    pl->eig_threads[c] = (s == COSMO_OK && has[c] && kEigThreadsAlt[c] != kEigThreads[c] &&
                          pl->psd_tune_ms[1][c] < pl->psd_tune_ms[0][c])
                             ? kEigThreadsAlt[c]
                             : kEigThreads[c];
  if (s != COSMO_OK) return s;
  DevBuf scr;
  HIPCHK(hipMalloc(&scr.ptr, (size_t)std::max<int64_t>(pl->sum_p2_large, 1) * sizeof(T)));
  T *w = static_cast<T *>(ws);
  for (int a = 0; a < 2; ++a) {
    pl->vjp_threads = a ? kVjpThreadsAlt : kVjpThreads;
    for (int rep = 0; rep < 2; ++rep) {
      (void)hipEventRecord(e0, st);
      if (!launch_dk_classes<T>(pl, w + pl->fw.U, w + pl->fw.lam, static_cast<const T *>(yK), static_cast<T *>(sK),
                                static_cast<T *>(scr.ptr), st))
        FAIL(COSMO_EUNSUPPORTED, "a PSD block is too large for the VJP's LDS layout");
      (void)hipEventRecord(e1, st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    pl->psd_tune_ms[a][4] = ms;
  }
  pl->vjp_threads = pl->psd_tune_ms[1][4] < pl->psd_tune_ms[0][4] ? kVjpThreadsAlt : kVjpThreads;
  return COSMO_OK;
}

}  // namespace

extern "C" {

cosmo_status cosmo_plan_autotune(cosmo_plan *plan, const void *rho, const void *alpha, void *ws, void *stream,
                                 double *ms_out) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!rho || !alpha || !ws) FAIL(COSMO_EINVAL, "rho, alpha and the workspace are required");
  if (ms_out)
    for (int c = 0; c < 4; ++c) ms_out[c] = -1.0;
  hipStream_t st = static_cast<hipStream_t>(stream);
  DevBuf out;
  HIPCHK(hipMalloc(&out.ptr, (2 * plan->m_tot + plan->n_tot) * plan->esz));
  char *o = static_cast<char *>(out.ptr);
  void *xK = o, *sK = o + plan->n_tot * plan->esz, *yK = o + (plan->n_tot + plan->m_tot) * plan->esz;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    FAIL(COSMO_EHIP, "hipEventCreate failed");
  }
  // candidates: CG forms 0, 2, 4 launched eagerly, then form 0 replayed from a graph
  const int32_t cand_form[4] = {0, 2, 4, 0};
  const bool cand_graph[4] = {false, false, false, true};
  const int32_t keep_form = plan->pcg_form;
  const bool keep_graph = plan->graph, keep_prof = plan->profiling;
  plan->profiling = false;
  double best = -1.0;
  int best_c = -1;
  for (int c = 0; c < 4 && s == COSMO_OK; ++c) {
    if ((plan->diag_M || plan->n_dense > 0) && cand_form[c] != 0) continue;   // no CG to schedule, or form 0 only
    plan->drop_graphs();
    plan->pcg_form = cand_form[c];
    plan->graph = cand_graph[c];
    for (int rep = 0; rep < 2 && s == COSMO_OK; ++rep) {   // the first run warms caches, code objects, records
      (void)hipEventRecord(e0, st);
      s = cosmo_unroll_forward(plan, rho, alpha, nullptr, nullptr, nullptr, xK, sK, yK, nullptr, ws, nullptr, stream);
      (void)hipEventRecord(e1, st);
    }
    if (s != COSMO_OK) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      s = COSMO_EHIP;
      break;
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms_out) ms_out[c] = ms;
    if (best < 0 || ms < best) {
      best = ms;
      best_c = c;
    }
  }
  plan->pcg_form = (s == COSMO_OK && best_c >= 0) ? cand_form[best_c] : keep_form;
  plan->graph = (s == COSMO_OK && best_c >= 0) ? cand_graph[best_c] : keep_graph;
  for (auto &row : plan->psd_tune_ms)
    for (double &t : row) t = -1.0;
  if (s == COSMO_OK && plan->n_psd > 0) {
    int32_t keep_eig[4];
    for (int c = 0; c < 4; ++c) keep_eig[c] = plan->eig_threads[c];
    const int32_t keep_vjp = plan->vjp_threads;
    plan->drop_graphs();
    s = plan->opt.dtype == COSMO_F32 ? tune_psd<float>(plan, rho, alpha, ws, st, xK, sK, yK, e0, e1)
                                     : tune_psd<double>(plan, rho, alpha, ws, st, xK, sK, yK, e0, e1);
    if (s != COSMO_OK) {   // a failed PSD phase leaves the shapes the plan had
      for (int c = 0; c < 4; ++c) plan->eig_threads[c] = keep_eig[c];
      plan->vjp_threads = keep_vjp;
    }
  }
  (void)hipStreamSynchronize(st);   // nothing in flight reads the scratch outputs when they are freed
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  plan->drop_graphs();   // the recorded sequences point at the scratch outputs
  plan->profiling = keep_prof;
  for (auto &sl : plan->prof) sl.used = 0;
  return s;
}

cosmo_status cosmo_plan_psd_tune_ms(const cosmo_plan *plan, double *ms) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!ms) FAIL(COSMO_EINVAL, "ms is NULL");
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 5; ++c) ms[5 * a + c] = plan->psd_tune_ms[a][c];
  return COSMO_OK;
}

// ---- schedule cache ----------------------------------------------------------------

}  // extern "C"

namespace {

// FNV-1a (64 bit) over the bytes of plain values.
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  template <typename V> void add(const V &v) {
    const unsigned char *b = reinterpret_cast<const unsigned char *>(&v);
    for (size_t i = 0; i < sizeof(V); ++i) h = (h ^ b[i]) * 1099511628211ull;
  }
};

std::string schedule_line(const char *key, const cosmo_schedule &sc) {
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "{\"key\": \"%s\", \"pcg_form\": %d, \"graph\": %d, \"eig_threads\": [%d, %d, %d, %d], "
                "\"vjp_threads\": %d}",
                key, sc.pcg_form, sc.graph, sc.eig_threads[0], sc.eig_threads[1], sc.eig_threads[2],
                sc.eig_threads[3], sc.vjp_threads);
  return buf;
}

// The key of a cache line, or "" when the line is not one this library wrote.
std::string line_key(const std::string &ln) {
  const std::string pre = "{\"key\": \"";
  if (ln.compare(0, pre.size(), pre) != 0) return "";
  const size_t e = ln.find('"', pre.size());
  return e == std::string::npos ? "" : ln.substr(pre.size(), e - pre.size());
}

bool parse_schedule(const std::string &ln, cosmo_schedule &sc) {
  const size_t at = ln.find("\", \"pcg_form\": ");
  if (at == std::string::npos) return false;
  cosmo_schedule t{};
  const int n = std::sscanf(ln.c_str() + at,
                            "\", \"pcg_form\": %d, \"graph\": %d, \"eig_threads\": [%d, %d, %d, %d], "
                            "\"vjp_threads\": %d}",
                            &t.pcg_form, &t.graph, &t.eig_threads[0], &t.eig_threads[1], &t.eig_threads[2],
                            &t.eig_threads[3], &t.vjp_threads);
  if (n != 7) return false;
  sc = t;
  return true;
}

bool key_ok(const char *key) {
  if (!key || !*key) return false;
  for (const char *c = key; *c; ++c)
    if (*c == '"' || *c == '\\' || *c == '\n' || *c == '\r' || (unsigned char)*c < 0x20) return false;
  return std::strlen(key) < 256;
}

}  // namespace

extern "C" {

cosmo_status cosmo_plan_signature(const cosmo_plan *plan, char *buf, int64_t len) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!buf || len < 1) FAIL(COSMO_EINVAL, "buf is NULL or len < 1");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop{};
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  std::string arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));   // the target, without feature flags
  Fnv f;
  const cosmo_options &o = plan->opt;
  f.add((int32_t)o.dtype);
  f.add(o.K);
  f.add(o.sigma);
  f.add(o.cg_tol);
  f.add(o.cg_max_iter);
  f.add(o.eig_max_sweeps);
  f.add(o.eig_tol);
  f.add(o.eig_refine);
  f.add(o.eig_warm_start);
  f.add(plan->B);
  for (int64_t v : plan->n_off) f.add(v);
  for (int64_t v : plan->m_off) f.add(v);
  f.add(plan->A_nnz);
  f.add(plan->P_nnz);
  f.add(plan->n_soc);
  f.add(plan->n_psd);
  for (int c = 0; c < 5; ++c) f.add(plan->psd_cls_begin[c]);
  for (int c = 0; c < 4; ++c) f.add(plan->psd_cls_maxp[c]);
  f.add(plan->sum_p);
  f.add(plan->sum_p2);
  f.add(plan->n_dense);
  f.add(plan->dense_maxcols);
  f.add(plan->dense_rows_tot);
  f.add(plan->dense_cols_tot);
  f.add(plan->dense_g32);
  f.add(plan->diag_M);
  char tail[160];
  std::snprintf(tail, sizeof tail, "/cu%d/%s/K%d/B%d/n%lld/m%lld/%016llx", prop.multiProcessorCount,
                o.dtype == COSMO_F32 ? "f32" : "f64", o.K, plan->B, (long long)plan->n_tot, (long long)plan->m_tot,
                (unsigned long long)f.h);
  const std::string key = arch + tail;
  if ((int64_t)key.size() + 1 > len) FAIL(COSMO_EINVAL, "buf holds fewer than " + std::to_string(key.size() + 1) + " bytes");
  std::memcpy(buf, key.c_str(), key.size() + 1);
  return COSMO_OK;
}

cosmo_status cosmo_plan_get_schedule(const cosmo_plan *plan, cosmo_schedule *sched) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!sched) FAIL(COSMO_EINVAL, "sched is NULL");
  sched->pcg_form = plan->pcg_form;
  sched->graph = plan->graph ? 1 : 0;
  for (int c = 0; c < 4; ++c) sched->eig_threads[c] = plan->eig_threads[c];
  sched->vjp_threads = plan->vjp_threads;
  return COSMO_OK;
}

cosmo_status cosmo_plan_set_schedule(cosmo_plan *plan, const cosmo_schedule *sched) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!sched) FAIL(COSMO_EINVAL, "sched is NULL");
  if (sched->graph != 0 && sched->graph != 1) FAIL(COSMO_EINVAL, "graph must be 0 or 1");
  // validate everything before changing anything
  const int32_t keep_form = plan->pcg_form;
  const bool keep_graph = plan->graph;
  plan->graph = false;
  s = cosmo_plan_set_pcg_form(plan, sched->pcg_form);
  if (s == COSMO_OK) s = cosmo_plan_set_graph(plan, sched->graph);
  if (s == COSMO_OK) s = cosmo_plan_set_psd_schedule(plan, sched->eig_threads, sched->vjp_threads);
  if (s != COSMO_OK) {
    const std::string msg = g_last_error;
    plan->pcg_form = keep_form;
    plan->drop_graphs();
    plan->graph = keep_graph;
    FAIL(s, msg);
  }
  return COSMO_OK;
}

cosmo_status cosmo_schedule_cache_load(const char *path, const char *key, cosmo_schedule *sched, int32_t *found) {
  if (!path || !sched || !found) FAIL(COSMO_EINVAL, "path, sched and found are required");
  if (!key_ok(key)) FAIL(COSMO_EINVAL, "key must be 1..255 printable characters without quotes or backslashes");
  *found = 0;
  std::ifstream in(path);
  if (!in) return COSMO_OK;   // no cache yet: a miss
  std::string ln;
  cosmo_schedule sc{};
  while (std::getline(in, ln))   // the last line with the key wins
    if (line_key(ln) == key && parse_schedule(ln, sc)) {
      *sched = sc;
      *found = 1;
    }
  return COSMO_OK;
}

cosmo_status cosmo_schedule_cache_store(const char *path, const char *key, const cosmo_schedule *sched) {
  if (!path || !sched) FAIL(COSMO_EINVAL, "path and sched are required");
  if (!key_ok(key)) FAIL(COSMO_EINVAL, "key must be 1..255 printable characters without quotes or backslashes");
  std::vector<std::string> keep;
  {
    std::ifstream in(path);
    std::string ln;
    while (in && std::getline(in, ln))
      if (!ln.empty() && line_key(ln) != key) keep.push_back(ln);
  }
  keep.push_back(schedule_line(key, *sched));
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) FAIL(COSMO_EINVAL, std::string("cannot write ") + tmp);
    for (const auto &ln : keep) out << ln << '\n';
    out.flush();
    if (!out) FAIL(COSMO_EINVAL, std::string("cannot write ") + tmp);
  }
  if (std::rename(tmp.c_str(), path) != 0) FAIL(COSMO_EINVAL, std::string("cannot replace ") + path);
  return COSMO_OK;
}

cosmo_status cosmo_plan_autotune_cached(cosmo_plan *plan, const void *rho, const void *alpha, void *ws, void *stream,
                                        const char *path, int32_t *hit) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (!path || !hit) FAIL(COSMO_EINVAL, "path and hit are required");
  *hit = 0;
  char key[256];
  s = cosmo_plan_signature(plan, key, sizeof key);
  if (s != COSMO_OK) return s;
  cosmo_schedule sc{};
  int32_t found = 0;
  s = cosmo_schedule_cache_load(path, key, &sc, &found);
  if (s != COSMO_OK) return s;
  if (found && cosmo_plan_set_schedule(plan, &sc) == COSMO_OK) {
    *hit = 1;
    return COSMO_OK;
  }
  // a miss, or an entry this plan rejects: time the schedules and record them
  s = cosmo_plan_autotune(plan, rho, alpha, ws, stream, nullptr);
  if (s != COSMO_OK) return s;
  s = cosmo_plan_get_schedule(plan, &sc);
  if (s != COSMO_OK) return s;
  return cosmo_schedule_cache_store(path, key, &sc);
}

// ---- profiling (not part of the hot path) -------------------------------------

cosmo_status cosmo_plan_set_tap(cosmo_plan *plan, void *tap) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  plan->tap = tap;
  return COSMO_OK;
}

cosmo_status cosmo_plan_set_profiling(cosmo_plan *plan, int32_t enable) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  plan->profiling = enable != 0;
  for (auto &sl : plan->prof) sl.used = 0;
  return COSMO_OK;
}

cosmo_status cosmo_plan_profile_read(cosmo_plan *plan, int32_t kind, int64_t *launches, double *total_ms) {
  cosmo_status s = check_plan(plan);
  if (s != COSMO_OK) return s;
  if (kind < 0 || kind > 7) FAIL(COSMO_EINVAL, "kind must be 0..7");
  ProfileSlot &sl = plan->prof[kind];
  double tot = 0;
  for (size_t i = 0; i < sl.used; ++i) {
    HIPCHK(hipEventSynchronize(sl.ev[i].second));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, sl.ev[i].first, sl.ev[i].second));
    tot += ms;
  }
  if (launches) *launches = (int64_t)sl.used;
  if (total_ms) *total_ms = tot;
  return COSMO_OK;
}

// ---- standalone projections ------------------------------------------------------

size_t cosmo_proj_workspace_size(int32_t nblk, const int32_t *order_or_dim) {
  if (nblk < 0) return 0;
  size_t p2 = 0;
  if (order_or_dim)
    for (int b = 0; b < nblk; ++b) p2 += (size_t)std::max(order_or_dim[b], 0) * std::max(order_or_dim[b], 0);
  return align_up((size_t)std::max(nblk, 1) * std::max(sizeof(PsdDesc), sizeof(SocDesc)), 256) + 3 * p2 * 8;
}

}  // extern "C"

namespace {

cosmo_status psd_common(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dt, void *ws,
                        hipStream_t st, std::vector<PsdDesc> &descs, int32_t cls_begin[5], int32_t cls_maxp[4]) {
  if (nblk < 1 || !order || !offset) FAIL(COSMO_EINVAL, "need nblk >= 1 and host order / offset arrays");
  if (dt != COSMO_F32 && dt != COSMO_F64) FAIL(COSMO_EINVAL, "bad dtype");
  if (!ws) FAIL(COSMO_EINVAL, "workspace is required");
  const int maxp = dt == COSMO_F32 ? COSMO_MAX_PSD_ORDER_F32 : COSMO_MAX_PSD_ORDER_F64;
  descs.resize(nblk);
  int64_t uo = 0, lo = 0;
  std::vector<std::pair<int64_t, int64_t>> ranges;
  for (int b = 0; b < nblk; ++b) {
    if (order[b] < 1 || order[b] > maxp) FAIL(order[b] < 1 ? COSMO_EINVAL : COSMO_EUNSUPPORTED, "PSD order out of range");
    if (offset[b] < 0) FAIL(COSMO_EINVAL, "negative offset");
    descs[b] = {offset[b], uo, lo, order[b], 0};
    uo += (int64_t)order[b] * order[b];
    lo += order[b];
    ranges.push_back({offset[b], offset[b] + (int64_t)order[b] * (order[b] + 1) / 2});
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second) FAIL(COSMO_EINVAL, "PSD blocks overlap");
  std::stable_sort(descs.begin(), descs.end(), [](const PsdDesc &a, const PsdDesc &b) {
    const int ca = psd_class(a.p), cb = psd_class(b.p);
    if (ca != cb) return ca < cb;
    return a.p > b.p;
  });
  int idx = 0;
  for (int c = 0; c < 4; ++c) {
    cls_begin[c] = idx;
    cls_maxp[c] = 0;
    while (idx < nblk && psd_class(descs[idx].p) == c) cls_maxp[c] = std::max(cls_maxp[c], descs[idx++].p);
  }
  cls_begin[4] = idx;
  HIPCHK(hipMemcpyAsync(ws, descs.data(), nblk * sizeof(PsdDesc), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return COSMO_OK;
}

}  // namespace

extern "C" {

cosmo_status psd_proj(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype, const void *in,
                      void *out, void *eigvals, void *eigvecs, int32_t max_sweeps, double eig_tol, int32_t refine,
                      void *ws, void *stream) {
  if (!in || !out) FAIL(COSMO_EINVAL, "in and out are required");
  if (max_sweeps < 1) FAIL(COSMO_EINVAL, "max_sweeps must be >= 1");
  if (refine < 0 || refine > 1) FAIL(COSMO_EINVAL, "refine must be 0 or 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<PsdDesc> descs;
  int32_t cb[5], cm[4];
  cosmo_status s = psd_common(nblk, order, offset, dtype, ws, st, descs, cb, cm);
  if (s != COSMO_OK) return s;
  const PsdDesc *d = static_cast<const PsdDesc *>(ws);
  double *rs = reinterpret_cast<double *>(static_cast<char *>(ws) +
                                          align_up((size_t)nblk * std::max(sizeof(PsdDesc), sizeof(SocDesc)), 256));
  const int rf = dtype == COSMO_F32 ? refine : 0;
  for (int c = 0; c < 4; ++c) {
    const int n = cb[c + 1] - cb[c];
    if (!n) continue;
    PsdLaunchCfg cfg{max_sweeps, eig_tol, rf, cm[c]};
    if (dtype == COSMO_F32)
      launch_psd_step<float>(d + cb[c], n, cfg, nullptr, (const float *)in, nullptr, nullptr, (float *)out, nullptr,
                             (float *)eigvecs, (float *)eigvals, rf ? rs : nullptr, nullptr, nullptr, st);
    else
      launch_psd_step<double>(d + cb[c], n, cfg, nullptr, (const double *)in, nullptr, nullptr, (double *)out,
                              nullptr, (double *)eigvecs, (double *)eigvals, nullptr, nullptr, nullptr, st);
  }
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

cosmo_status psd_proj_vjp(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                          const void *eigvals, const void *eigvecs, const void *gout, void *gin, void *ws,
                          void *stream) {
  return psd_proj_vjp_rule(nblk, order, offset, dtype, COSMO_PSD_RULE_DK, 0.0, eigvals, eigvecs, gout, gin, ws,
                           stream);
}

cosmo_status psd_proj_vjp_rule(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                               int32_t rule, double eps, const void *eigvals, const void *eigvecs, const void *gout,
                               void *gin, void *ws, void *stream) {
  if (rule < COSMO_PSD_RULE_DK || rule > COSMO_PSD_RULE_TIKHONOV) FAIL(COSMO_EINVAL, "unknown PSD backward rule");
  if (!std::isfinite(eps)) FAIL(COSMO_EINVAL, "eps must be finite");
  if (rule != COSMO_PSD_RULE_TIKHONOV) eps = 0.0;
  if (!eigvals || !eigvecs || !gout || !gin) FAIL(COSMO_EINVAL, "eigvals, eigvecs, gout and gin are required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<PsdDesc> descs;
  int32_t cb[5], cm[4];
  cosmo_status s = psd_common(nblk, order, offset, dtype, ws, st, descs, cb, cm);
  if (s != COSMO_OK) return s;
  const PsdDesc *d = static_cast<const PsdDesc *>(ws);
  // a p x p buffer that does not fit next to the first one in LDS lives in the
  // workspace's scratch area (sum p^2 elements, indexed like the eigenvectors)
  void *scratch = static_cast<char *>(ws) + align_up((size_t)nblk * std::max(sizeof(PsdDesc), sizeof(SocDesc)), 256);
  for (int c = 0; c < 4; ++c) {
    const int n = cb[c + 1] - cb[c];
    if (!n) continue;
    const bool ok = dtype == COSMO_F32
        ? launch_psd_vjp<float>(d + cb[c], n, cm[c], (const float *)eigvecs, (const float *)eigvals,
                                (const float *)gout, (float *)gin, (float *)scratch, st, rule, eps)
        : launch_psd_vjp<double>(d + cb[c], n, cm[c], (const double *)eigvecs, (const double *)eigvals,
                                 (const double *)gout, (double *)gin, (double *)scratch, st, rule, eps);
    if (!ok) FAIL(COSMO_EUNSUPPORTED, "a PSD block is too large for the VJP's LDS layout");
  }
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

}  // extern "C"

namespace {

// Layout of a Newton-Schulz tape: block descriptors, the per-block norms,
// then (2K + 8) p^2 elements per block.
struct NsLayout {
  std::vector<NsDesc> d;
  int64_t ntiles = 0;
  int32_t tile = 64;
  size_t off_c = 0, off_m = 0, bytes = 0;
};

cosmo_status ns_layout(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dt, int32_t iters,
                       NsLayout &L) {
  if (nblk < 1 || !order) FAIL(COSMO_EINVAL, "need nblk >= 1 and a host order array");
  if (dt != COSMO_F32 && dt != COSMO_F64) FAIL(COSMO_EINVAL, "bad dtype");
  if (iters < 0 || iters > COSMO_NS_MAX_ITERS) FAIL(COSMO_EINVAL, "Newton-Schulz step count out of range");
  const size_t esz = dt == COSMO_F32 ? 4 : 8;
  // 64 x 64 output tiles per workgroup while they still give two workgroups
  // per CU (256 CUs), else 32 x 32 tiles; the choice depends on the orders
  // only, so the forward and the reverse call agree.
  int64_t t64 = 0;
  for (int b = 0; b < nblk; ++b) {
    const int64_t n64 = (std::max(order[b], 1) + 63) / 64;
    t64 += n64 * n64;
  }
  L.tile = t64 >= 512 ? 64 : 32;
  L.d.resize(nblk);
  int64_t mo = 0, tiles = 0;
  std::vector<std::pair<int64_t, int64_t>> ranges;
  for (int b = 0; b < nblk; ++b) {
    const int p = order[b];
    if (p < 1 || p > COSMO_NS_MAX_ORDER) FAIL(p < 1 ? COSMO_EINVAL : COSMO_EUNSUPPORTED, "PSD order out of range");
    const int64_t r0 = offset ? offset[b] : 0;
    if (offset && r0 < 0) FAIL(COSMO_EINVAL, "negative offset");
    const int nt = (p + L.tile - 1) / L.tile;
    L.d[b] = {r0, mo, p, (int32_t)tiles};
    mo += NsSlots::count(iters) * p * p;
    tiles += (int64_t)nt * nt;
    if (tiles > INT32_MAX) FAIL(COSMO_EUNSUPPORTED, "too many product tiles");
    if (offset) ranges.push_back({r0, r0 + (int64_t)p * (p + 1) / 2});
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second) FAIL(COSMO_EINVAL, "PSD blocks overlap");
  L.ntiles = tiles;
  L.off_c = align_up((size_t)nblk * sizeof(NsDesc), 256);
  L.off_m = L.off_c + align_up((size_t)nblk * sizeof(double), 256);
  L.bytes = L.off_m + (size_t)mo * esz;
  return COSMO_OK;
}

}  // namespace

extern "C" {

size_t psd_ns_tape_size(int32_t nblk, const int32_t *order, cosmo_dtype dtype, int32_t iters) {
  NsLayout L;
  if (ns_layout(nblk, order, nullptr, dtype, iters, L) != COSMO_OK) return 0;
  return L.bytes;
}

cosmo_status psd_proj_ns(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                         int32_t iters, const void *in, void *out, void *tape, void *stream) {
  if (!offset || !in || !out || !tape) FAIL(COSMO_EINVAL, "offset, in, out and tape are required");
  NsLayout L;
  cosmo_status s = ns_layout(nblk, order, offset, dtype, iters, L);
  if (s != COSMO_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *t = static_cast<char *>(tape);
  HIPCHK(hipMemcpyAsync(t, L.d.data(), (size_t)nblk * sizeof(NsDesc), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  const NsDesc *d = reinterpret_cast<const NsDesc *>(t);
  double *cn = reinterpret_cast<double *>(t + L.off_c);
  if (dtype == COSMO_F32)
    launch_ns_forward<float>(d, nblk, (int32_t)L.ntiles, L.tile, iters, (const float *)in, (float *)out,
                             reinterpret_cast<float *>(t + L.off_m), cn, st);
  else
    launch_ns_forward<double>(d, nblk, (int32_t)L.ntiles, L.tile, iters, (const double *)in, (double *)out,
                              reinterpret_cast<double *>(t + L.off_m), cn, st);
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

cosmo_status psd_proj_ns_vjp(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                             int32_t iters, const void *gout, void *gin, void *tape, void *stream) {
  if (!offset || !gout || !gin || !tape) FAIL(COSMO_EINVAL, "offset, gout, gin and tape are required");
  NsLayout L;
  cosmo_status s = ns_layout(nblk, order, offset, dtype, iters, L);
  if (s != COSMO_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *t = static_cast<char *>(tape);
  const NsDesc *d = reinterpret_cast<const NsDesc *>(t);
  const double *cn = reinterpret_cast<const double *>(t + L.off_c);
  if (dtype == COSMO_F32)
    launch_ns_vjp<float>(d, nblk, (int32_t)L.ntiles, L.tile, iters, (const float *)gout, (float *)gin,
                         reinterpret_cast<float *>(t + L.off_m), cn, st);
  else
    launch_ns_vjp<double>(d, nblk, (int32_t)L.ntiles, L.tile, iters, (const double *)gout, (double *)gin,
                          reinterpret_cast<double *>(t + L.off_m), cn, st);
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

static cosmo_status soc_common(int32_t ncones, const int32_t *dim, const int64_t *offset, cosmo_dtype dt, void *ws,
                               hipStream_t st) {
  if (ncones < 1 || !dim || !offset) FAIL(COSMO_EINVAL, "need ncones >= 1 and host dim / offset arrays");
  if (dt != COSMO_F32 && dt != COSMO_F64) FAIL(COSMO_EINVAL, "bad dtype");
  if (!ws) FAIL(COSMO_EINVAL, "workspace is required");
  std::vector<SocDesc> d(ncones);
  for (int c = 0; c < ncones; ++c) {
    if (dim[c] < 1 || offset[c] < 0) FAIL(COSMO_EINVAL, "bad SOC dim / offset");
    d[c] = {offset[c], dim[c], 0};
  }
  HIPCHK(hipMemcpyAsync(ws, d.data(), ncones * sizeof(SocDesc), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return COSMO_OK;
}

cosmo_status socp_proj(int32_t ncones, const int32_t *dim, const int64_t *offset, cosmo_dtype dtype, const void *in,
                       void *out, void *ws, void *stream) {
  if (!in || !out) FAIL(COSMO_EINVAL, "in and out are required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  cosmo_status s = soc_common(ncones, dim, offset, dtype, ws, st);
  if (s != COSMO_OK) return s;
  const SocDesc *d = static_cast<const SocDesc *>(ws);
  if (dtype == COSMO_F32) launch_soc_proj<float>(d, ncones, (const float *)in, (float *)out, st);
  else launch_soc_proj<double>(d, ncones, (const double *)in, (double *)out, st);
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}

cosmo_status socp_proj_vjp(int32_t ncones, const int32_t *dim, const int64_t *offset, cosmo_dtype dtype,
                           const void *in, const void *gout, void *gin, void *ws, void *stream) {
  if (!in || !gout || !gin) FAIL(COSMO_EINVAL, "in, gout and gin are required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  cosmo_status s = soc_common(ncones, dim, offset, dtype, ws, st);
  if (s != COSMO_OK) return s;
  const SocDesc *d = static_cast<const SocDesc *>(ws);
  if (dtype == COSMO_F32) launch_soc_vjp<float>(d, ncones, (const float *)in, (const float *)gout, (float *)gin, st);
  else launch_soc_vjp<double>(d, ncones, (const double *)in, (const double *)gout, (double *)gin, st);
  HIPCHK(hipGetLastError());
  return COSMO_OK;
}


// ---- psd_proj without allocation -------------------------------------------
//
// psd_proj_static_scratch runs psd_proj with this library's own device
// scratch instead of a caller workspace: a file-scope array, one copy per
// device, held until the process ends.  Host code must never pass the
// array's name to a kernel or a copy (it is a host-side stand-in, not a
// device address): the device address is taken once per device with
// hipGetSymbolAddress and kept below.
}  // extern "C"

static __device__ __align__(256) unsigned char scratch[COSMO_PSD_STATIC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<std::pair<int, void *>> g_scratch_dev;   // (device, address of scratch on it)

cosmo_status static_scratch(void **ptr) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  for (const auto &e : g_scratch_dev)
    if (e.first == dev) {
      *ptr = e.second;
      return COSMO_OK;
    }
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    FAIL(COSMO_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_dev.push_back({dev, p});
  *ptr = p;
  return COSMO_OK;
}
}  // namespace

extern "C" {

cosmo_status psd_proj_static_scratch(int32_t nblk, const int32_t *order, const int64_t *offset, cosmo_dtype dtype,
                                     const void *in, void *out, void *eigvals, void *eigvecs, int32_t max_sweeps,
                                     double eig_tol, int32_t refine, void *stream) {
  if (nblk < 1 || !order) FAIL(COSMO_EINVAL, "need nblk >= 1 and a host order array");
  const size_t need = cosmo_proj_workspace_size(nblk, order);
  if (need > (size_t)COSMO_PSD_STATIC_SCRATCH_BYTES)
    FAIL(COSMO_EUNSUPPORTED, "psd_proj_static_scratch: these blocks need " + std::to_string(need) +
                                 " bytes of scratch; the static scratch holds " +
                                 std::to_string((size_t)COSMO_PSD_STATIC_SCRATCH_BYTES) + " (use psd_proj)");
  void *ws = nullptr;
  const cosmo_status st = static_scratch(&ws);
  if (st != COSMO_OK) return st;
  return psd_proj(nblk, order, offset, dtype, in, out, eigvals, eigvecs, max_sweeps, eig_tol, refine, ws, stream);
}

}  // extern "C"
