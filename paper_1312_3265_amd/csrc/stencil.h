// Stencil kernels: one thread per (site, right-hand side), a Dirac operator's
// site function, and a fused epilogue.  The epilogues implement the steps of
// CG on eq. (2) around the two matvecs of an iteration:
//   STORE       out = op(in)
//   STORE_NORM  out = op(in), block partials of ||out||^2          (t = M p)
//   CG_UPDATE   q = op(in) kept in registers; alpha = rho/||t||^2 from the
//               partials of the previous launch; r -= alpha q; block
//               partials of ||r||^2                                 (M^dag t)
//               x is advanced once per group of G iterations (4 for the
//               FP32 and 16-bit solves, 2 for FP64), by the G steps at
//               once: x += sum_j alpha_{k-G+1+j} p_{k-G+1+j} on the group's
//               last iteration (p rotates through G buffers), which divides
//               the traffic of x, the widest vector of a low-precision solve
//               (FP32 under Q16), by G.  The sum is formed in the
//               arithmetic precision, step after step, as the single steps
//               would be.
//   RESID       out = b - op(in), partials of ||out||^2   (FP64 true residual)
//   LANCZOS     w = op(in) - beta_prev v_prev, partials of Re<v, w>
// Partial sums are FP64, reduced in a fixed order (wavefront butterfly, then
// waves in order), so results do not depend on scheduling.
//
// Grid: nbp site-blocks (a multiple of 8) x nrhs, flattened so that each XCD
// works through one contiguous range of site blocks, all right-hand sides of a
// site block one after another (see map_block): stencil neighbours and the
// links shared by the right-hand sides are then served from that XCD's L2.
#pragma once

#include "common.h"
#include "dirac.h"
#include "lq_types.h"

namespace lq {

enum Epi { EPI_STORE = 0, EPI_STORE_NORM = 1, EPI_CG_UPDATE = 2, EPI_RESID = 3, EPI_LANCZOS = 4 };

struct EpiArgs {
  void* out;              // output fields (STORE, STORE_NORM, RESID, LANCZOS)
  double* part;           // block partials out, [k * nbp + sb]
  const double* part_in;  // CG_UPDATE: partials of ||t||^2 from the previous launch
  int nbp;                // site blocks per RHS (multiple of 8)
  int k0;                 // first RHS index handled by this launch
  SlotState* st;          // per-RHS solver state (null: no state checks)
  int par;                // iteration parity (ring index into SlotState)
  int state_mode;         // 0: none, 1: running and not frozen, 2: running and in ru_mask
  const int* ru_mask;     // per-RHS reliable-update selection (state_mode 2)
  void* x;                // CG_UPDATE: x_lo
  void* r;                // CG_UPDATE: r_lo
  const void* p;          // CG_UPDATE: p_k
  const void* pring[4];   // CG_UPDATE: the ring of search directions of the group
  int q4;                 // CG_UPDATE: iteration index within its group (alpha[q4] is stored)
  int xstep;              // CG_UPDATE: 0, or the group size G on the group's last iteration:
                          // x += sum_{j<G} alpha[j] p_ring[j] (p_ring[G-1] is p)
  const void* b;          // RESID: b (FP64)
  const double* v;        // LANCZOS: v_j
  const double* vprev;    // LANCZOS: v_{j-1}
  const double* beta_prev;// LANCZOS: device scalar beta_{j-1} (null = 0)
  int rhs_per_thread;     // systems per thread (1, 2 or 4; FP32/Q16 CG kernels)
  int window;             // block order: > 0 window width, 0 whole range, -1/-2 system-major,
                          // -3/-4 tiled (map_block, map_block_tiled)
  int stream;             // CG_UPDATE, FP32/Q16: 1 = r, p, x loaded and stored non-temporal
};

// blockIdx.x -> (site block sb, rhs k), XCD-aware.  Block b runs on XCD b % 8,
// as that XCD's (b / 8)-th block.  The site blocks are swept in windows of
// 8*win consecutive blocks; in a window, XCD x owns the win blocks
// [8*win*w + win*x, ... + win) and visits them for system 0, then system 1, ...
// So the whole GPU works on one compact window at a time (its data stays in
// the shared Infinity Cache), each XCD re-reads a window's links from its own
// L2 for every system, and a block's t neighbours -- one t-slice away, which is
// one window when 8*win*256 sites make a slice -- are visited by the same XCD
// one window earlier or later.  win = 1 gives XCD-interleaved blocks with the
// systems innermost; win = nbp/8 gives each XCD one contiguous range.
//
// win < 0: the (system, site block) pairs in system-major order, XCD x taking
// the x-th contiguous eighth.  Each XCD then sweeps whole systems t-slice by
// t-slice, so every neighbour plane is reused from its own L2 within one
// system, and the links come from the shared Infinity Cache once per system.
// win = -2 reverses the sweep of every other system, so that consecutive
// systems meet on the same site blocks.
__device__ __forceinline__ void map_block(int nbp, int nrhs, int win, int& sb, int& k) {
  const int b = blockIdx.x;
  const int xcd = b & 7, kk = b >> 3;
  if (win < 0) {
    const int p = xcd * ((nbp >> 3) * nrhs) + kk;
    k = p / nbp;
    sb = p - k * nbp;
    if (win == -2 && (k & 1)) sb = nbp - 1 - sb;
    return;
  }
  const int range = nbp >> 3;                // blocks per XCD in total
  if (win <= 0 || win > range) win = range;
  const int per_win = win * nrhs;
  const int w = kk / per_win;
  const int w0 = w * win;                    // blocks per XCD before this window
  const int width = min(win, range - w0);    // the last window may be narrower
  const int rem = kk - w * per_win;
  k = rem / width;
  sb = 8 * w0 + xcd * width + (rem - k * width);
}

// win = -3 / -4: tiled orders for lattices whose x-y planes are whole site
// blocks (L1*L2 a multiple of 256, L4 a multiple of 8, L3 even, V/256 a
// multiple of 8).  XCD x owns the t-slices [x*L4/8, (x+1)*L4/8) and sweeps
// them in chunks of two z-planes: for each chunk, t runs innermost-but-one,
// so a block's t- and z-neighbours are visited by the same XCD within a few
// dozen blocks and are still in its L2.  -3 takes the systems one after the
// other (each XCD sweeps its slab once per system); -4 visits each tile for
// all systems before moving on (links shared through L2, vectors not).
// Returns false (and leaves sb, k unset) when the lattice does not qualify.
__device__ __forceinline__ bool map_block_tiled(const Geom& g, int nbp, int nrhs, int win, int& sb,
                                                int& k) {
  const int plane = g.L[0] * g.L[1];
  if ((plane & 255) || (g.L[3] & 7) || (g.L[2] & 1) || nbp * 256 != g.V) return false;
  const int b = blockIdx.x;
  const int xcd = b & 7, kk = b >> 3;
  const int P = plane >> 8, Z = g.L[2], Tx = g.L[3] >> 3;
  const int per = P * Z * Tx;             // blocks of one system on one XCD
  if (8 * per != nbp) return false;       // fields of a sublattice (even-odd halves)
  int r;
  if (win == -3) { k = kk / per; r = kk - k * per; }
  else { k = kk % nrhs; r = kk / nrhs; }
  const int p = r % P;
  r /= P;
  const int zi = r & 1;
  r >>= 1;
  const int tl = r % Tx;
  const int zc = r / Tx;
  sb = p + P * ((2 * zc + zi) + Z * (xcd * Tx + tl));
  return true;
}

__device__ __forceinline__ bool slot_active(const SlotState* st, int k, int mode, int par,
                                            const int* mask) {
  if (mode == 0) return true;
  if (st[k].status != SLOT_RUNNING) return false;
  if (mode == 1) return st[k].stop[par] == 0;
  return mask == nullptr || mask[k] != 0;
}

// Register budget: FP64 kernels are held to 3-4 waves per SIMD so that enough
// waves are resident to cover HBM latency.
//
// K systems per thread: the block covers kBlock sites of the K systems
// k0 .. k0+K-1 (k0 = ea.k0 + K * group); links and corner matrices are loaded
// once per site for all K.  Each system keeps its own alpha, state and
// partial sums, so the result of a system does not depend on K or on the
// other systems.
template <class Op, int K>
constexpr int stencil_waves() { return (Op::NC == 12 && K >= 2) ? 3 : Op::kWaves; }

// CG_UPDATE at one site for system k (offset off into the batched fields):
// r -= alpha q with ||r||^2 returned, and on the last iteration of a group of
// G x += sum_j alpha_j p_ring[j] (alpha_{G-1} = alpha, p_ring[G-1] = p_k), one
// direction at a time.  r, p and x are each touched once per
// launch; CP = kStream marks them non-temporal so that, when the batch's
// vectors overflow the caches anyway, they do not displace the links and the
// stencil input from L2.
// kb >= 0 (the lanes stencil): the fields are addressed from the uniform base
// of system kb (off = kb's offset) plus per-lane byte offsets lo_v (vectors of
// policy Pol) and lo_x (x), system k being kb + its lane's share; FP32/16-bit
// only.
template <class Op, int CP>
__device__ __forceinline__ double cg_update_site(const EpiArgs& ea, int Vp, int k, size_t off,
                                                 int i, double alpha,
                                                 const typename Op::C q[Op::NC], int kb = -1,
                                                 uint32_t lo_v = 0, uint32_t lo_x = 0) {
  using P_C = typename Op::C;
  using R = typename Op::R;
  using S = typename Op::S;
  using Pol = typename Op::Pol;
  constexpr int NC = Op::NC;
  const int kx = kb >= 0 ? kb : k;
  S* r = (S*)ea.r + off;
  const R a = (R)alpha;
  P_C rv[NC];
  ld_site<Pol, NC, CP>(r, Vp, i, rv, lo_v);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    rv[c].x -= a * q[c].x; rv[c].y -= a * q[c].y;
  }
  const double n2 = st_site<Pol, NC, CP>(r, Vp, i, rv, lo_v);
  if (ea.xstep > 0 && Pol::id == 0) {   // wavefront-uniform
    // FP64: one component at a time, so that the 48-word records are never
    // live together (they would spill)
    double2* x = (double2*)ea.x + (size_t)k * NC * Vp;
    const int G = ea.xstep;
#pragma unroll 1
    for (int c = 0; c < NC; ++c) {
      double2 xv = ld_c64<CP>(x, Vp, i, c);
      for (int j = 0; j < G; ++j) {
        const double aj = j == G - 1 ? (double)a : ea.st[k].alpha[j];
        const double2 v = ld_c64<CP>((const double2*)ea.pring[j] + off, Vp, i, c);
        xv.x += aj * v.x; xv.y += aj * v.y;
      }
      st_c64<CP>(x, Vp, i, c, xv);
    }
  } else if (ea.xstep > 0) {   // wavefront-uniform
    using XP = typename XPol<Pol>::type;
    typename XP::S* x = (typename XP::S*)ea.x + (size_t)kx * NC * Vp;
    typename XP::C xv[NC];
    ld_site<XP, NC, CP>(x, Vp, i, xv, lo_x);
    // one direction at a time: only x and one record are live
    const int G = ea.xstep;
#pragma unroll 1
    for (int j = 0; j < G; ++j) {
      const R aj = j == G - 1 ? a : (R)ea.st[k].alpha[j];
      P_C pv[NC];
      ld_site<Pol, NC, CP>((const S*)ea.pring[j] + off, Vp, i, pv, lo_v);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        xv[c].x += aj * pv[c].x; xv[c].y += aj * pv[c].y;
      }
    }
    st_site<XP, NC, CP>(x, Vp, i, xv, lo_x);
  }
  return n2;
}

// The epilogue of one site for the K systems of a thread (see the header of
// this file), with the block partial of the site block sb.  Every thread of
// the block must call it (block_sum synchronises the block).
template <class Op, int EPI, int K, int CP>
__device__ __forceinline__ void site_epilogue(const OpArgs& oa, const EpiArgs& ea, int k0,
                                              unsigned act, int i, bool valid, int sb,
                                              const typename Op::C o[K][Op::NC],
                                              const double alpha[K], double* red) {
  using P_C = typename Op::C;
  using R = typename Op::R;
  using S = typename Op::S;
  constexpr int NC = Op::NC;
  const int Vp = oa.g.Vp;
  const size_t rstride = (size_t)field_planes<typename Op::Pol>(NC) * Vp;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    if (!((act >> kk) & 1)) continue;   // uniform over the block
    const int k = k0 + kk;
    const size_t off = (size_t)k * rstride;
    double acc = 0.0;
    if (valid) {
      if constexpr (EPI == EPI_STORE || EPI == EPI_STORE_NORM) {
        const double n2 = st_site<typename Op::Pol, NC>((S*)ea.out + off, Vp, i, o[kk]);
        if constexpr (EPI == EPI_STORE_NORM) acc = n2;
      } else if constexpr (EPI == EPI_CG_UPDATE) {
        acc = cg_update_site<Op, CP>(ea, Vp, k, off, i, alpha[kk], o[kk]);
      } else if constexpr (EPI == EPI_RESID) {
        double2* out = (double2*)ea.out + off;
        const double2* b = (const double2*)ea.b + off;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          const size_t e = (size_t)q * Vp + i;
          double2 bv = b[e];
          double2 w;
          w.x = bv.x - (double)o[kk][q].x;
          w.y = bv.y - (double)o[kk][q].y;
          out[e] = w;
          acc += w.x * w.x + w.y * w.y;
        }
      } else if constexpr (EPI == EPI_LANCZOS) {
        double2* out = (double2*)ea.out + off;
        const double2* v = (const double2*)ea.v + off;
        const double2* vp = (const double2*)ea.vprev + off;
        const double bp = ea.beta_prev ? *ea.beta_prev : 0.0;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          const size_t e = (size_t)q * Vp + i;
          double2 w;
          w.x = (double)o[kk][q].x - bp * vp[e].x;
          w.y = (double)o[kk][q].y - bp * vp[e].y;
          out[e] = w;
          acc += v[e].x * w.x + v[e].y * w.y;
        }
      }
    }
    if constexpr (EPI != EPI_STORE) {
      const double bs = block_sum(acc, red);
      if (threadIdx.x == 0) ea.part[(size_t)k * ea.nbp + sb] = bs;
    }
  }
}

template <class Op, int EPI, int K, int CP>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(stencil_waves<Op, K>(), 8)))
stencil_kernel(const OpArgs oa, const typename Op::S* __restrict__ in, const EpiArgs ea,
               int ngroups, int nrhs) {
  using P_C = typename Op::C;
  using R = typename Op::R;
  using S = typename Op::S;
  constexpr int NC = Op::NC;
  __shared__ double red[16];
  int sb, kg;
  if ((ea.window != -3 && ea.window != -4) ||
      !map_block_tiled(oa.g, ea.nbp, ngroups, ea.window, sb, kg))
    map_block(ea.nbp, ngroups, ea.window < -2 ? 0 : ea.window, sb, kg);
  const int k0 = ea.k0 + kg * K;
  unsigned act = 0;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const int k = k0 + kk;
    if (k < ea.k0 + nrhs && (!ea.st || slot_active(ea.st, k, ea.state_mode, ea.par, ea.ru_mask)))
      act |= 1u << kk;
  }
  if (act == 0) return;   // uniform over the block

  const int Vp = oa.g.Vp;
  const int i = sb * blockDim.x + threadIdx.x;
  const bool valid = i < oa.g.V;
  const size_t rstride = (size_t)field_planes<typename Op::Pol>(NC) * Vp;

  double alpha[K];
  if constexpr (EPI == EPI_CG_UPDATE) {
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      alpha[kk] = 0.0;
      if (!((act >> kk) & 1)) continue;
      const int k = k0 + kk;
      const double tt = sum_partials(ea.part_in + (size_t)k * ea.nbp, ea.nbp, red);
      const double rho = ea.st[k].rho[ea.par];
      alpha[kk] = (tt > 0.0 && isfinite(tt) && isfinite(rho)) ? rho / tt : 0.0;
      if (sb == 0 && threadIdx.x == 0) {
        if (!(tt > 0.0 && isfinite(tt))) ea.st[k].flags |= 1;
        ea.st[k].alpha[ea.q4] = alpha[kk];   // read on the group's last iteration
      }
    }
  }

  P_C o[K][NC];
  if (valid) Op::template site_multi<K>(oa, in + (size_t)k0 * rstride, rstride, i, k0, act, o);

  site_epilogue<Op, EPI, K, CP>(oa, ea, k0, act, i, valid, sb, o, alpha, red);
}

}  // namespace lq
