// Staggered overlap operator with the staggered Wilson kernel (the staggered
// overlap fermion the paper presents D_SW as the kernel of, Secs. 1, 2 and 4):
//   A = D_SW - rho,  V = epsilon sign(epsilon A) = A (A^dag A)^{-1/2},
//   D_ov(m) psi = (rho - m/2) (psi + V psi) + m psi,
// with (A^dag A)^{-1/2} replaced by the Chebyshev interpolant p of x^{-1/2} on
// [lo, hi] (an interval containing the spectrum of A^dag A), applied to psi by
// the three-term recurrence T_{k+1} = 2 X T_k - T_{k-1}, X = (2 A^dag A -
// (hi + lo)) / (hi - lo): one A^dag A (two FP64 stencil launches of the
// kernel, Gamma_55 from corners or on the fly) and one vector launch per
// degree.  Its error in V is at most max over [lo, hi] of |x^{1/2} p(x) - 1|.
#include <cmath>
#include <cstring>
#include <vector>

#include "engine.h"

namespace lq {

// FP64 fields of the staggered Wilson kernel are 3 planes of Vp complex
// numbers; the elementwise kernels run over all 3 * Vp elements (the plane
// padding is zero in every operand and stays zero).
__global__ void __launch_bounds__(256)
cheb_first_kernel(const double2* __restrict__ q, const double2* __restrict__ v,
                  double2* __restrict__ t, double2* __restrict__ y, double a, double b, double c0,
                  double c1, size_t n) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double2 qv = q[e], vv = v[e];
  double2 tv, yv;
  tv.x = a * qv.x + b * vv.x;
  tv.y = a * qv.y + b * vv.y;
  yv.x = c0 * vv.x + c1 * tv.x;
  yv.y = c0 * vv.y + c1 * tv.y;
  t[e] = tv;
  y[e] = yv;
}

// t_next = 2 (a q + b t) - t_prev, written over t_prev; y += c t_next
__global__ void __launch_bounds__(256)
cheb_step_kernel(const double2* __restrict__ q, const double2* __restrict__ t,
                 double2* __restrict__ tp, double2* __restrict__ y, double a, double b, double c,
                 size_t n) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double2 qv = q[e], tv = t[e], pv = tp[e];
  double2 nv, yv = y[e];
  nv.x = 2.0 * (a * qv.x + b * tv.x) - pv.x;
  nv.y = 2.0 * (a * qv.y + b * tv.y) - pv.y;
  yv.x += c * nv.x;
  yv.y += c * nv.y;
  tp[e] = nv;
  y[e] = yv;
}

// out = f (v + w) + m v
__global__ void __launch_bounds__(256)
ov_finish_kernel(const double2* __restrict__ v, const double2* __restrict__ w,
                 double2* __restrict__ out, double f, double m, size_t n) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double2 vv = v[e], wv = w[e];
  out[e] = make_double2(f * (vv.x + wv.x) + m * vv.x, f * (vv.y + wv.y) + m * vv.y);
}

std::vector<double> cheb_coeffs_invsqrt(double lo, double hi, int degree) {
  // interpolant of x^{-1/2} at the degree + 1 Chebyshev points of the first kind
  const int n = degree + 1;
  std::vector<double> f(n), th(n), c(n, 0.0);
  for (int j = 0; j < n; ++j) {
    th[j] = M_PI * (j + 0.5) / n;
    f[j] = 1.0 / std::sqrt(0.5 * (hi + lo) + 0.5 * (hi - lo) * std::cos(th[j]));
  }
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += f[j] * std::cos(k * th[j]);
    c[k] = 2.0 / n * s;
  }
  c[0] *= 0.5;
  return c;
}

size_t overlap_workspace_bytes(const Geom& g, int g55) {
  const size_t vec = (size_t)3 * g.Vp * 16;
  Carver c(nullptr);
  for (int k = 0; k < 6; ++k) c.take(vec);   // v, t_prev, t, q, tmp, y
  if (g55 == LQ_G55_ONTHEFLY) c.take(g55_bytes_per_system(g, P64));
  return c.size();
}

void overlap_apply(const lq_gauge_s* gs, const lq_overlap* ov, const void* in, void* out,
                   void* ws, size_t ws_bytes, hipStream_t s) {
  const Geom& g = gs->g;
  const size_t need = overlap_workspace_bytes(g, ov->g55_mode);
  if (!ws || ws_bytes < need)
    throw Error(LQ_ERR_WORKSPACE, "overlap workspace too small: need " + std::to_string(need));
  const int op = opkind(LQ_STAGGERED_WILSON, ov->g55_mode);
  const int nl = gs->fp64_links();
  const size_t vec = (size_t)3 * g.Vp * 16;
  const size_t n = (size_t)3 * g.Vp;
  Carver c(ws);
  double2* v = (double2*)c.take(vec);
  double2* tp = (double2*)c.take(vec);
  double2* t = (double2*)c.take(vec);
  double2* q = (double2*)c.take(vec);
  double2* tmp = (double2*)c.take(vec);
  double2* y = (double2*)c.take(vec);
  OpArgs oa;
  oa.g = g;
  oa.links = gs->links(P64, nl);
  oa.corners = op == OP_SW_CORNERS ? gs->corners(P64) : nullptr;
  oa.r = ov->r;
  oa.mass0 = -ov->rho;          // A = D_SW - rho
  oa.mass = nullptr;
  oa.mass_stride = 0;
  if (op == OP_SW_OTF) {
    oa.g55_sys = g55_bytes_per_system(g, P64);
    oa.g55w = c.take(oa.g55_sys);
  }
  launch_fill_zero(ws, c.size(), s);
  const int nbp = nbp_of(g.V);
  EpiArgs e;
  std::memset(&e, 0, sizeof(e));
  e.nbp = nbp;
  e.window = -3;
  auto AdA = [&](const double2* x, double2* res) {
    e.out = tmp;
    launch_stencil(op, P64, nl, false, EPI_STORE, oa, x, e, 1, s);
    e.out = res;
    launch_stencil(op, P64, nl, true, EPI_STORE, oa, tmp, e, 1, s);
  };
  const std::vector<double> cf = cheb_coeffs_invsqrt(ov->lo, ov->hi, ov->degree);
  const double a = 2.0 / (ov->hi - ov->lo), b = -(ov->hi + ov->lo) / (ov->hi - ov->lo);
  const dim3 grid((unsigned)((n + 255) / 256)), blk(256);
  launch_field_in(P64, 3, g, in, 1, v, nbp, 0, 1, s);
  AdA(v, q);
  hipLaunchKernelGGL(cheb_first_kernel, grid, blk, 0, s, q, v, t, y, a, b, cf[0], cf[1], n);
  // t_prev starts as v: copy it so that the recurrence may overwrite it
  LQ_HIP(hipMemcpyAsync(tp, v, vec, hipMemcpyDeviceToDevice, s));
  for (int k = 2; k <= ov->degree; ++k) {
    AdA(t, q);
    hipLaunchKernelGGL(cheb_step_kernel, grid, blk, 0, s, q, t, tp, y, a, b, cf[k], n);
    std::swap(t, tp);   // the new T_k is in tp's buffer
  }
  // w = A y (into q), out = (rho - m/2) (v + w) + m v (into tmp)
  e.out = q;
  launch_stencil(op, P64, nl, false, EPI_STORE, oa, y, e, 1, s);
  hipLaunchKernelGGL(ov_finish_kernel, grid, blk, 0, s, v, q, tmp, ov->rho - 0.5 * ov->mass,
                     ov->mass, n);
  launch_field_out(P64, 3, g, tmp, out, 1, nbp, 0, 1, s);
  check_launch();
}

}  // namespace lq
