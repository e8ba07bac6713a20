// CG vector kernels (p update, reliable updates, slot loading), the Lanczos
// vector kernels, and the stencil launch dispatcher.
//
// CG on eq. (2) per system (x0 = 0), with the low-precision vectors held in
// units of a per-system scale s (true value = s * stored value):
//   t = M p;  alpha = rho / ||t||^2  (= rho / <p, A p>);  x_lo += alpha p;
//   r_lo -= alpha M^dag t;  rho' = ||r_lo||^2;  p = r_lo + (rho'/rho) p.
// A reliable update recomputes the residual in FP64:
//   x_hi += s x_lo; x_lo = 0; r_hi = b - M^dag M x_hi; s' = ||r_hi|| / sqrt(N);
//   r_lo = r_hi / s'; p *= s / s'; rho = ||r_lo||^2.
// The system is converged when ||r_hi|| <= tol ||b||.  With FP64 storage the
// scale stays 1 and reliable updates happen only to confirm convergence.
#include <stdexcept>
#include <string>

#include "kernels.h"
#include "stencil.h"

namespace lq {

void launch_stencil_wilson(int, int, bool, int, const OpArgs&, const void*, const EpiArgs&, int,
                           hipStream_t);
void launch_stencil_sw(int, int, bool, int, const OpArgs&, const void*, const EpiArgs&, int,
                       hipStream_t);
void launch_stencil_otf(int, int, bool, int, const OpArgs&, const void*, const EpiArgs&, int,
                        hipStream_t);
void launch_stencil_wilson_eo(int, int, bool, int, const OpArgs&, const void*, const EpiArgs&, int,
                              hipStream_t);

void launch_stencil(int op, int prec, int nl, bool dag, int epi, const OpArgs& oa, const void* in,
                    const EpiArgs& ea, int nrhs, hipStream_t s) {
  switch (op) {
    case OP_WILSON: return launch_stencil_wilson(prec, nl, dag, epi, oa, in, ea, nrhs, s);
    case OP_SW_CORNERS: return launch_stencil_sw(prec, nl, dag, epi, oa, in, ea, nrhs, s);
    case OP_SW_OTF: return launch_stencil_otf(prec, nl, dag, epi, oa, in, ea, nrhs, s);
    case OP_WILSON_EO: return launch_stencil_wilson_eo(prec, nl, dag, epi, oa, in, ea, nrhs, s);
    default: throw std::runtime_error("unknown operator " + std::to_string(op));
  }
}

constexpr double kGrowth2 = 1e4;   // squared residual growth that forces a reliable update

// ------------------------------------------------------------- p update
// Closes a CG iteration: beta = ||r_new||^2 / rho, p = r + beta p, and the
// per-system state step.
template <class P, int NC>
__global__ void __launch_bounds__(256)
p_update_kernel(const Geom g, SlotState* st, int par, int pend_next, const double* __restrict__ part,
                int nbp,
                const typename P::S* __restrict__ p, typename P::S* __restrict__ pout,
                const typename P::S* __restrict__ r, int k0, int nrhs) {
  using C = typename P::C;
  using R = typename P::R;
  __shared__ double red[16];
  int sb, kl;
  map_block(nbp, nrhs, 1, sb, kl);
  const int k = k0 + kl;
  SlotState* s = st + k;
  if (s->status != SLOT_RUNNING) return;
  if (s->stop[par]) {
    // frozen: carry the state into the next parity entry
    if (sb == 0 && threadIdx.x == 0) {
      s->stop[par ^ 1] = 1;
      s->rho[par ^ 1] = s->rho[par];
    }
    return;
  }
  const double rr = sum_partials(part + (size_t)k * nbp, nbp, red);
  const double rho = s->rho[par];
  const double beta = (rho > 0.0 && isfinite(rr)) ? rr / rho : 0.0;
  const int i = sb * blockDim.x + threadIdx.x;
  if (i < g.V) {
    const size_t off = (size_t)k * field_planes<P>(NC) * g.Vp;
    const R bt = (R)beta;
    C pv[NC], rv[NC];
    ld_site<P, NC>(p + off, g.Vp, i, pv);
    ld_site<P, NC>(r + off, g.Vp, i, rv);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      pv[q].x = rv[q].x + bt * pv[q].x;
      pv[q].y = rv[q].y + bt * pv[q].y;
    }
    st_site<P, NC>(pout + off, g.Vp, i, pv);
  }
  if (sb == 0 && threadIdx.x == 0) {
    const double rmax = fmax(s->rho_max, rr);
    s->rho_max = rmax;
    s->rho[par ^ 1] = rr;
    s->iter += 1;
    s->apps += 1;
    s->iter_res2 = rr * s->scale * s->scale;
    int stop = 0;
    if (!isfinite(rr) || (s->flags & 1)) { s->flags |= 1; stop = 1; }
    if (rr <= s->thr_lo2) stop = 1;
    // reliable-update triggers of the low-precision iteration: the residual
    // has dropped by delta from its largest value since the latest update,
    // or has grown 100-fold above the value at that update (restart from the
    // FP64 true residual before rounding drift can build up)
    else if (s->delta2 > 0.0 && (rr <= s->delta2 * rmax || rr > kGrowth2 * s->rho_ru)) {
      stop = 1;
      s->want_ru = 1;
    }
    if (s->iter >= s->maxiter) { s->flags |= 2; stop = 1; }
    s->stop[par ^ 1] = stop;
    // x is advanced on the last iteration of each group; stopping after
    // iteration q of a group of G leaves pend_next = (q + 1) % G terms
    // alpha[j] * p_ring[j] for the reliable update to add
    if (stop) s->pend = pend_next;
  }
}

// ------------------------------------------------------- reliable updates
template <class P, int NC>
__global__ void __launch_bounds__(256)
ru_accumulate_kernel(const Geom g, const SlotState* st, const int* mask, double2* __restrict__ xhi,
                     typename XPol<P>::type::S* __restrict__ xlo, const PRing ring, int nbp,
                     int k0, int nrhs) {
  using XP = typename XPol<P>::type;
  using C = typename XP::C;
  int sb, kl;
  map_block(nbp, nrhs, 1, sb, kl);
  const int k = k0 + kl;
  if (!ru_selected(st, mask, k)) return;
  const double sc = st[k].scale;
  const int pend = st[k].pend;
  const int i = sb * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const size_t off = (size_t)k * NC * g.Vp;
  const size_t poff = (size_t)k * field_planes<P>(NC) * g.Vp;
  C v[NC], z[NC];
  double2 acc[NC];
  ld_site<XP, NC>(xlo + off, g.Vp, i, v);
#pragma unroll
  for (int q = 0; q < NC; ++q) acc[q] = make_double2((double)v[q].x, (double)v[q].y);
  // the steps of an unfinished group, in order
  for (int j = 0; j < pend; ++j) {
    typename P::C pv[NC];
    ld_site<P, NC>((const typename P::S*)ring.p[j] + poff, g.Vp, i, pv);
    const double aj = st[k].alpha[j];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      acc[q].x += aj * (double)pv[q].x;
      acc[q].y += aj * (double)pv[q].y;
    }
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const size_t e = off + (size_t)q * g.Vp + i;
    double2 h = xhi[e];
    h.x += sc * acc[q].x;
    h.y += sc * acc[q].y;
    xhi[e] = h;
    z[q] = czero<C>();
  }
  st_site<XP, NC>(xlo + off, g.Vp, i, z);
}

// part: ||r||^2 of the normal equations being iterated.  Even-odd (part_f
// and part_g non-null): with init, ||M^dag chi||^2 = sum f + sum g; later,
// eq. (2)'s own residual ||b - A x||^2 = d^2 sum f + sum g (f: ||r^||^2 of the
// Schur system, g: ||M_eo^dag r^||^2) decides convergence, and while it is
// not met the Schur system's target is lowered in proportion.
__global__ void ru_finish_kernel(SlotState* st, const int* mask, const double* __restrict__ part,
                                 const double* __restrict__ part_f,
                                 const double* __restrict__ part_g, int nbp, int k0, double ncomp,
                                 int rescale, int max_cand, int init, int par) {
  __shared__ double red[16];
  const int k = k0 + blockIdx.x;
  SlotState* s = st + k;
  if (!ru_selected(st, mask, k)) return;
  const double rr = sum_partials(part + (size_t)k * nbp, nbp, red);
  const bool eo = part_f != nullptr;
  double f2 = 0.0, g2 = 0.0;
  if (eo) {
    f2 = sum_partials(part_f + (size_t)k * nbp, nbp, red);
    g2 = sum_partials(part_g + (size_t)k * nbp, nbp, red);
  }
  if (threadIdx.x != 0) return;
  if (init) {
    s->bnorm2 = rr;
    s->thr2 = s->tol * s->tol * rr;
    if (eo) s->bfull2 = f2 + g2;
  } else {
    s->ru += 1;
    s->apps += 1;
  }
  s->ru_iter = s->iter;
  s->true_res2 = rr;
  if (!isfinite(rr)) { s->flags |= 1; s->status = SLOT_FAILED; return; }
  if (eo && !init) {
    const double d = s->mass + 4.0;
    const double full2 = d * d * f2 + g2;
    const double goal = s->tol * s->tol * s->bfull2;
    s->full_res2 = full2;
    if (full2 <= goal) { s->status = SLOT_DONE; return; }
    if (rr <= s->thr2 && isfinite(full2)) s->thr2 = 0.25 * rr * goal / full2;
  } else if (rr <= s->thr2) {
    s->status = SLOT_DONE;
    return;
  }
  if (s->flags) { s->status = SLOT_FAILED; return; }
  // stagnation: a tolerance below the attainable accuracy is never met, and
  // cycling on from the accuracy floor lets x drift away from it; stop (not
  // converged) once max_cand updates in a row have not halved the true
  // residual, or once it has stayed 100-fold above its best at two updates
  // in a row.  A single such update is what the growth trigger of the
  // low-precision iteration requests: it restarts the iteration from the FP64
  // residual, which recovers a solve whose drift was only rounding; growth
  // that survives the restart is not rounding drift.
  s->grown = (!init && rr > kGrowth2 * s->best2) ? s->grown + 1 : 0;
  if (init || rr < 0.25 * s->best2) {
    s->best2 = rr;
    s->stall = 0;
  } else if (++s->stall > max_cand || s->grown >= 2) {
    s->flags |= 4;
    s->status = SLOT_FAILED;
    return;
  }
  if (!init && s->stop[par] && !s->want_ru) {
    // the iterated residual met tol but the true residual did not
    s->cand += 1;
    if (s->cand > max_cand) { s->flags |= 4; s->status = SLOT_FAILED; return; }
  }
  s->want_ru = 0;
  double sn = rescale ? sqrt(rr / ncomp) : 1.0;
  if (!(sn > 0.0) || !isfinite(sn)) sn = 1.0;
  s->scale_prev = init ? sn : s->scale;
  s->scale = sn;
  s->thr_lo2 = s->thr2 / (sn * sn);
}

template <class P, int NC>
__global__ void __launch_bounds__(256)
ru_convert_kernel(const Geom g, const SlotState* st, const int* mask,
                  const double2* __restrict__ rhi, typename P::S* __restrict__ rlo,
                  const PRing ring, double* __restrict__ part, int nbp, int init, int k0,
                  int nrhs) {
  using C = typename P::C;
  using R = typename P::R;
  __shared__ double red[16];
  int sb, kl;
  map_block(nbp, nrhs, 1, sb, kl);
  const int k = k0 + kl;
  if (!ru_selected(st, mask, k)) return;
  const double inv = 1.0 / st[k].scale;
  const R pr = (R)(st[k].scale_prev / st[k].scale);
  const int i = sb * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < g.V) {
    const size_t off = (size_t)k * field_planes<P>(NC) * g.Vp;
    const size_t off64 = (size_t)k * NC * g.Vp;
    C v[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const double2 h = rhi[off64 + (size_t)q * g.Vp + i];
      v[q].x = (R)(h.x * inv);
      v[q].y = (R)(h.y * inv);
    }
    acc = st_site<P, NC>(rlo + off, g.Vp, i, v);
    typename P::S* p = (typename P::S*)ring.p[0];
    if (init) {
      C vs[NC];
      ld_site<P, NC>(rlo + off, g.Vp, i, vs);   // p starts as the stored r
      st_site<P, NC>(p + off, g.Vp, i, vs);
    } else {
      // the current search direction: ring buffer pend (where the last p
      // update wrote it); the next chunk starts in buffer 0
      C pv[NC];
      ld_site<P, NC>((const typename P::S*)ring.p[st[k].pend] + off, g.Vp, i, pv);
#pragma unroll
      for (int q = 0; q < NC; ++q) { pv[q].x *= pr; pv[q].y *= pr; }
      st_site<P, NC>(p + off, g.Vp, i, pv);
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[(size_t)k * nbp + sb] = s;
}

__global__ void ru_commit_kernel(SlotState* st, const int* mask, const double* __restrict__ part,
                                 int nbp, int k0) {
  __shared__ double red[16];
  const int k = k0 + blockIdx.x;
  SlotState* s = st + k;
  if (!ru_selected(st, mask, k)) return;
  const double rr = sum_partials(part + (size_t)k * nbp, nbp, red);
  if (threadIdx.x != 0) return;
  s->rho[0] = s->rho[1] = rr;
  s->rho_ru = rr;
  s->rho_max = rr;
  s->stop[0] = s->stop[1] = 0;
  s->pend = 0;
  s->iter_res2 = rr * s->scale * s->scale;
}

template <class P, int NC>
__global__ void __launch_bounds__(256)
load_prepare_kernel(const Geom g, double2* __restrict__ xhi,
                    typename XPol<P>::type::S* __restrict__ xlo, double2* __restrict__ rhi,
                    const double2* __restrict__ b, int nbp, int k0, int nrhs) {
  using XP = typename XPol<P>::type;
  using C = typename XP::C;
  int sb, kl;
  map_block(nbp, nrhs, 1, sb, kl);
  const int k = k0 + kl;
  const int i = sb * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const size_t off = (size_t)k * NC * g.Vp;
  C z[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const size_t e = off + (size_t)q * g.Vp + i;
    xhi[e] = make_double2(0.0, 0.0);
    z[q] = czero<C>();
    rhi[e] = b[e];
  }
  st_site<XP, NC>(xlo + off, g.Vp, i, z);
}

// ----------------------------------------------------------- dispatch
#define LQ_PREC_NC_SWITCH(prec, nc, CALL)                                            \
  do {                                                                               \
    if (prec == P64 && nc == 12) { using PP = F64; constexpr int NCC = 12; CALL; }   \
    else if (prec == P64 && nc == 3) { using PP = F64; constexpr int NCC = 3; CALL; } \
    else if (prec == P32 && nc == 12) { using PP = F32; constexpr int NCC = 12; CALL; } \
    else if (prec == P32 && nc == 3) { using PP = F32; constexpr int NCC = 3; CALL; }  \
    else if (prec == P16 && nc == 12) { using PP = Q16; constexpr int NCC = 12; CALL; } \
    else if (prec == P16 && nc == 3) { using PP = Q16; constexpr int NCC = 3; CALL; }  \
    else throw std::runtime_error("unsupported precision/components");               \
  } while (0)

void launch_p_update(int prec, int nc, const Geom& g, SlotState* st, int par, int pend_next,
                     const double* part, int nbp, const void* p, void* pout, const void* r, int k0,
                     int nrhs, hipStream_t s) {
  if (nbp * nrhs == 0) return;
  LQ_PREC_NC_SWITCH(prec, nc,
                    hipLaunchKernelGGL((p_update_kernel<PP, NCC>), dim3(nbp * nrhs), dim3(kBlock),
                                       0, s, g, st, par, pend_next, part, nbp, (const typename PP::S*)p,
                                       (typename PP::S*)pout, (const typename PP::S*)r, k0, nrhs));
}

void launch_ru_accumulate(int prec, int nc, const Geom& g, const SlotState* st, const int* mask,
                          double* xhi, void* xlo, const PRing& ring, int nbp, int k0, int nrhs,
                          hipStream_t s) {
  if (nbp * nrhs == 0) return;
  LQ_PREC_NC_SWITCH(prec, nc,
                    hipLaunchKernelGGL((ru_accumulate_kernel<PP, NCC>), dim3(nbp * nrhs),
                                       dim3(kBlock), 0, s, g, st, mask, (double2*)xhi,
                                       (typename XPol<PP>::type::S*)xlo, ring, nbp, k0, nrhs));
}

void launch_ru_finish(SlotState* st, const int* mask, const double* part, const double* part_f,
                      const double* part_g, int nbp, int k0, int nrhs, double ncomp, int rescale,
                      int max_cand, int init, int par, hipStream_t s) {
  if (nrhs == 0) return;
  hipLaunchKernelGGL(ru_finish_kernel, dim3(nrhs), dim3(64), 0, s, st, mask, part, part_f, part_g,
                     nbp, k0, ncomp, rescale, max_cand, init, par);
}

void launch_ru_convert(int prec, int nc, const Geom& g, const SlotState* st, const int* mask,
                       const double* rhi, void* rlo, const PRing& ring, double* part, int nbp,
                       int init, int k0, int nrhs, hipStream_t s) {
  if (nbp * nrhs == 0) return;
  LQ_PREC_NC_SWITCH(prec, nc,
                    hipLaunchKernelGGL((ru_convert_kernel<PP, NCC>), dim3(nbp * nrhs),
                                       dim3(kBlock), 0, s, g, st, mask, (const double2*)rhi,
                                       (typename PP::S*)rlo, ring, part, nbp, init, k0, nrhs));
}

void launch_ru_commit(SlotState* st, const int* mask, const double* part, int nbp, int k0,
                      int nrhs, hipStream_t s) {
  if (nrhs == 0) return;
  hipLaunchKernelGGL(ru_commit_kernel, dim3(nrhs), dim3(64), 0, s, st, mask, part, nbp, k0);
}

void launch_load_prepare(int prec, int nc, const Geom& g, double* xhi, void* xlo, double* rhi,
                         const double* b, int nbp, int k0, int nrhs, hipStream_t s) {
  if (nbp * nrhs == 0) return;
  LQ_PREC_NC_SWITCH(prec, nc,
                    hipLaunchKernelGGL((load_prepare_kernel<PP, NCC>), dim3(nbp * nrhs),
                                       dim3(kBlock), 0, s, g, (double2*)xhi,
                                       (typename XPol<PP>::type::S*)xlo, (double2*)rhi,
                                       (const double2*)b, nbp, k0, nrhs));
}

// ------------------------------------------------------------- Lanczos
// Basis V (nvec vectors of nc*Vp complex), work vector w.  Classical
// Gram-Schmidt: h = V^H w (lz_dots + lz_reduce), w -= V h (lz_update).
constexpr int kDotChunk = 8;

__global__ void __launch_bounds__(256)
lz_dots_kernel(const Geom g, int nc, const double2* __restrict__ V, int nvec, double2* w,
               const double* __restrict__ alpha_part, int nbp_alpha, double* alpha_out,
               double* __restrict__ part_h, int nblk) {
  __shared__ double red[16];
  const size_t n = (size_t)nc * g.Vp;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  if (alpha_part) {
    // w -= alpha v_j with alpha = Re<v_j, A v_j - beta v_{j-1}>, v_j = V[nvec-1]
    const double a = sum_partials(alpha_part, nbp_alpha, red);
    if (blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = a;
    const double2* vj = V + (size_t)(nvec - 1) * n;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
      double2 x = w[e];
      x.x -= a * vj[e].x;
      x.y -= a * vj[e].y;
      w[e] = x;
    }
    __syncthreads();
  }
  for (int k0 = 0; k0 < nvec; k0 += kDotChunk) {
    double re[kDotChunk], im[kDotChunk];
#pragma unroll
    for (int c = 0; c < kDotChunk; ++c) re[c] = im[c] = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
      const double2 x = w[e];
#pragma unroll
      for (int c = 0; c < kDotChunk; ++c) {
        if (k0 + c < nvec) {
          const double2 v = V[(size_t)(k0 + c) * n + e];
          re[c] += v.x * x.x + v.y * x.y;
          im[c] += v.x * x.y - v.y * x.x;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kDotChunk; ++c) {
      if (k0 + c < nvec) {
        const double sr = block_sum(re[c], red);
        const double si = block_sum(im[c], red);
        if (threadIdx.x == 0) {
          part_h[((size_t)(k0 + c) * nblk + blockIdx.x) * 2 + 0] = sr;
          part_h[((size_t)(k0 + c) * nblk + blockIdx.x) * 2 + 1] = si;
        }
      }
    }
  }
}

__global__ void lz_reduce_kernel(const double* __restrict__ part_h, int nvec, int nblk,
                                 double2* __restrict__ h) {
  for (int k = threadIdx.x; k < nvec; k += blockDim.x) {
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < nblk; ++b) {
      sr += part_h[((size_t)k * nblk + b) * 2 + 0];
      si += part_h[((size_t)k * nblk + b) * 2 + 1];
    }
    h[k] = make_double2(sr, si);
  }
}

__global__ void __launch_bounds__(256)
lz_update_kernel(const Geom g, int nc, const double2* __restrict__ V, int nvec,
                 const double2* __restrict__ h, double2* w, double* __restrict__ part_n,
                 int with_norm) {
  __shared__ double red[16];
  __shared__ double2 hs[1024];
  for (int k = threadIdx.x; k < nvec && k < 1024; k += blockDim.x) hs[k] = h[k];
  __syncthreads();
  const size_t n = (size_t)nc * g.Vp;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    double2 x = w[e];
    for (int k = 0; k < nvec; ++k) {
      const double2 v = V[(size_t)k * n + e];
      const double2 c = hs[k];
      x.x -= v.x * c.x - v.y * c.y;
      x.y -= v.x * c.y + v.y * c.x;
    }
    w[e] = x;
    acc += x.x * x.x + x.y * x.y;
  }
  if (with_norm) {
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part_n[blockIdx.x] = s;
  }
}

__global__ void lz_finish_kernel(const double* __restrict__ part_n, int nblk, double* beta_out) {
  __shared__ double red[16];
  const double s = sum_partials(part_n, nblk, red);
  if (threadIdx.x == 0) *beta_out = sqrt(s);
}

__global__ void __launch_bounds__(256)
lz_normalize_kernel(const Geom g, int nc, const double2* __restrict__ w,
                    const double* __restrict__ beta, double2* __restrict__ vnext) {
  const size_t n = (size_t)nc * g.Vp;
  const double bt = *beta;
  const double inv = (bt > 1e-300 && isfinite(bt)) ? 1.0 / bt : 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const double2 x = w[e];
    vnext[e] = make_double2(x.x * inv, x.y * inv);
  }
}

void launch_lz_dots(const Geom& g, int nc, const double2* V, int nvec, double2* w,
                    const double* alpha_part, int nbp_alpha, double* alpha_out, double* part_h,
                    int nblk, hipStream_t s) {
  hipLaunchKernelGGL(lz_dots_kernel, dim3(nblk), dim3(kBlock), 0, s, g, nc, V, nvec, w,
                     alpha_part, nbp_alpha, alpha_out, part_h, nblk);
}
void launch_lz_reduce(const double* part_h, int nvec, int nblk, double2* h, hipStream_t s) {
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(1), dim3(256), 0, s, part_h, nvec, nblk, h);
}
void launch_lz_update(const Geom& g, int nc, const double2* V, int nvec, const double2* h,
                      double2* w, double* part_n, int nblk, int with_norm, hipStream_t s) {
  hipLaunchKernelGGL(lz_update_kernel, dim3(nblk), dim3(kBlock), 0, s, g, nc, V, nvec, h, w,
                     part_n, with_norm);
}
void launch_lz_finish(const double* part_n, int nblk, double* beta_out, hipStream_t s) {
  hipLaunchKernelGGL(lz_finish_kernel, dim3(1), dim3(64), 0, s, part_n, nblk, beta_out);
}
void launch_lz_normalize(const Geom& g, int nc, const double2* w, const double* beta,
                         double2* vnext, hipStream_t s) {
  hipLaunchKernelGGL(lz_normalize_kernel, dim3(1024), dim3(kBlock), 0, s, g, nc, w, beta, vnext);
}

}  // namespace lq
