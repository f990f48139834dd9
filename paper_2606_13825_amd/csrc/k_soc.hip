// Second-order cone blocks (t, w), ||w||_2 <= t: projection (closed form),
// the COSMO slack / dual update on SOC rows, and the vector-Jacobian product
// of the projection (Sec. "Stable PSD Projection": the SOC projection is
// piecewise smooth).  One thread per cone: the cones of the workloads have
// a handful of rows, and the loops below are plain strided sums.  The
// arithmetic runs in float64 from the stored values and is rounded once on
// store (a float32 pipeline's s+ and y+ = y + rho (s^ - s+) then carry no
// cancellation error beyond that rounding).
#include "cosmo_internal.h"

namespace cosmo {
namespace {

constexpr int ST = 256;

// Norm of w with one rescaling pass to avoid overflow/underflow.
template <typename T> __device__ inline double wnorm(const T *w, int d) {
  double mx = 0;
  for (int i = 0; i < d; ++i) {
    const double a = fabs((double)w[i]);
    mx = (a > mx || a != a) ? a : mx;   // a NaN entry sticks (fmax would drop it)
  }
  if (mx == 0.0) return 0;
  double acc = 0;
  for (int i = 0; i < d; ++i) {
    const double u = (double)w[i] / mx;
    acc += u * u;
  }
  return mx * sqrt(acc);
}

// out = Pi(v): identity if ||w|| <= t, zero if ||w|| <= -t, else
// ((||w|| + t)/2) (1, w/||w||).
template <typename T> __device__ inline void soc_project(const T *v, T *out, int dim) {
  const double t = v[0];
  const double nw = wnorm(v + 1, dim - 1);
  if (nw <= t) {
    for (int i = 0; i < dim; ++i) out[i] = v[i];
  } else if (nw <= -t) {
    for (int i = 0; i < dim; ++i) out[i] = 0;
  } else {
    const double a = 0.5 * (1.0 + t / nw);
    out[0] = (T)(a * nw);
    for (int i = 1; i < dim; ++i) out[i] = (T)(a * (double)v[i]);
  }
}

template <typename T>
__global__ __launch_bounds__(ST) void k_soc_step(const SocDesc *__restrict__ d, int32_t n,
                                                 const T *__restrict__ rho_hat, const T *__restrict__ vv,
                                                 const T *__restrict__ sh, const T *__restrict__ y,
                                                 T *__restrict__ s_new, T *__restrict__ y_new) {
  const int c = blockIdx.x * ST + threadIdx.x;
  if (c >= n) return;
  const SocDesc cd = d[c];
  const int64_t r0 = cd.row0;
  soc_project(vv + r0, s_new + r0, cd.dim);
  for (int i = 0; i < cd.dim; ++i) {
    const int64_t r = r0 + i;
    y_new[r] = (T)((double)y[r] + (double)rho_hat[r] * ((double)sh[r] - (double)s_new[r]));
  }
}

template <typename T>
__global__ __launch_bounds__(ST) void k_soc_proj(const SocDesc *__restrict__ d, int32_t n, const T *__restrict__ in,
                                                 T *__restrict__ out) {
  const int c = blockIdx.x * ST + threadIdx.x;
  if (c >= n) return;
  soc_project(in + d[c].row0, out + d[c].row0, d[c].dim);
}

// out = J(v) g with J = 1/2 [[1, u'], [u, (1 + t/nw) I - (t/nw) u u']] on the
// boundary piece (J symmetric, so this is also the VJP).
template <typename T>
__global__ __launch_bounds__(ST) void k_soc_vjp(const SocDesc *__restrict__ d, int32_t n, const T *__restrict__ vv,
                                                const T *__restrict__ g, T *__restrict__ out) {
  const int c = blockIdx.x * ST + threadIdx.x;
  if (c >= n) return;
  const SocDesc cd = d[c];
  const T *v = vv + cd.row0;
  const T *gg = g + cd.row0;
  T *o = out + cd.row0;
  const int dim = cd.dim;
  const double t = v[0];
  const double nw = wnorm(v + 1, dim - 1);
  if (nw <= t) {
    for (int i = 0; i < dim; ++i) o[i] = gg[i];
  } else if (nw <= -t) {
    for (int i = 0; i < dim; ++i) o[i] = 0;
  } else {
    double ug = 0;   // u'g_w
    for (int i = 1; i < dim; ++i) ug += (double)v[i] * (double)gg[i];
    ug /= nw;
    const double rr = t / nw;
    const double g0 = gg[0];
    o[0] = (T)(0.5 * (g0 + ug));
    for (int i = 1; i < dim; ++i) {
      const double ui = (double)v[i] / nw;
      o[i] = (T)(0.5 * (ui * g0 + (1.0 + rr) * (double)gg[i] - rr * ui * ug));
    }
  }
}

inline int nblk(int32_t n) { return (n + ST - 1) / ST; }

}  // namespace

template <typename T>
void launch_soc_step(const SocDesc *d, int32_t n, const T *rho_hat, const T *vv, const T *sh, const T *y, T *s_new,
                     T *y_new, hipStream_t st) {
  if (n > 0) k_soc_step<T><<<nblk(n), ST, 0, st>>>(d, n, rho_hat, vv, sh, y, s_new, y_new);
}
template <typename T> void launch_soc_vjp(const SocDesc *d, int32_t n, const T *vv, const T *g, T *out, hipStream_t st) {
  if (n > 0) k_soc_vjp<T><<<nblk(n), ST, 0, st>>>(d, n, vv, g, out);
}
template <typename T> void launch_soc_proj(const SocDesc *d, int32_t n, const T *in, T *out, hipStream_t st) {
  if (n > 0) k_soc_proj<T><<<nblk(n), ST, 0, st>>>(d, n, in, out);
}

#define INST(T)                                                                                              \
  template void launch_soc_step<T>(const SocDesc *, int32_t, const T *, const T *, const T *, const T *, T *, \
                                   T *, hipStream_t);                                                        \
  template void launch_soc_vjp<T>(const SocDesc *, int32_t, const T *, const T *, T *, hipStream_t);         \
  template void launch_soc_proj<T>(const SocDesc *, int32_t, const T *, T *, hipStream_t);
INST(float)
INST(double)

}  // namespace cosmo
