// FP64 Wilson stencil (r = 1) that sweeps T consecutive t-slices of one
// 256-site x-y slab per block, so that the t-direction data of a site is read
// from memory once instead of three times.
//
// The single-system FP64 stencils are bound by what they fetch from beyond L2:
// with one thread per site and 256-site slabs, the z and t neighbours of a
// block belong to other blocks, which loaded them long before (a wave's eight
// hops each wait for memory), so the re-reads miss the 4 MiB L2.  Here a block
// owns the slab (p, z) for t in [t0, t0 + T) and, for each site (thread):
//   * psi(t + 1), loaded for the +t hop of t, is kept in LDS as the diagonal
//     input of the next step (so psi(t) is never fetched for the diagonal);
//   * the -t hop of t + 1, U_t(t)^dag P psi(t), is formed at step t from
//     psi(t) (LDS) and the link U_t(t) just loaded for the +t hop, and kept in
//     LDS (so psi(t - 1) and U_t(t - 1) are never fetched again; in registers
//     it would spill the hop loop).
// Per site one spinor and one link fewer are fetched than by stencil_kernel
// (two spinors fewer counting the diagonal).  Each step then runs the x, y and
// z hops as stencil_kernel does, and the epilogue of that site block.
//
// The result differs from stencil_kernel's only in the order of the FP64
// accumulation (diagonal, -t, +t, then x, y, z): it is the same to rounding.
// The choice of kernel depends on the lattice alone (not on the number of
// systems), so a system's result does not depend on its batch.
#pragma once

#include "stencil.h"

namespace lq {

// Slices per block for lattices where the sweep applies, else 0: x-y planes
// of whole 256-site blocks and no ragged last block.  T is the largest power
// of two dividing L4 that still gives every compute unit one block of a
// system (ncu = the device's compute units; the block count must also be a
// multiple of 8).  Measured on 32^3 x 64 (FP64 M^dag): T = 4, 8, 16, 32, 64
// give 2048 ... 128 blocks and 497, 467, 445, 387, 588 us against 605 us for
// stencil_kernel -- fewer, longer sweeps keep each XCD's blocks on adjacent
// z-planes in step, so their shared planes are still in L2, until the blocks
// no longer fill the GPU.
__host__ inline int tsweep_slices(const Geom& g, int ncu) {
  const int plane = g.L[0] * g.L[1];
  if ((plane & 255) || nbp_of(g.V) * 256 != g.V) return 0;
  const int slabs = (plane >> 8) * g.L[2];
  for (int T = 64; T >= 2; T >>= 1) {
    if (g.L[3] % T) continue;
    const int blocks = slabs * (g.L[3] / T);
    if (blocks >= ncu && (blocks & 7) == 0) return T;
  }
  return 0;
}

template <int NL, bool DAG, int EPI>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(3, 8)))
wilson_tsweep_kernel(const OpArgs oa, const double2* __restrict__ in, const EpiArgs ea, int T,
                     int nrhs) {
  using Op = WilsonOpR1<F64, NL, DAG>;
  using W = WilsonOp<F64, NL, DAG, false>;
  using LP = typename LinkPol<F64, NL>::type;
  using C = double2;
  using R = double;
  constexpr int sgn = DAG ? -1 : 1;
  constexpr int TTF = -sgn, TTB = sgn;   // hop along +t, along -t
  __shared__ double red[16];
  __shared__ C nxt[12][256];             // psi at the step's slice, per site of the slab
  __shared__ C ub[6][256];               // the step's -t link product U_t(t-1)^dag P psi(t-1)
  const Geom& g = oa.g;
  const int plane = g.L[0] * g.L[1];
  const int P = plane >> 8, NT = g.L[3] / T;
  const int per = P * g.L[2] * NT;       // blocks per system (a multiple of 8)
  // block b runs on XCD b % 8 as its (b / 8)-th block; XCD x takes the x-th
  // eighth of the (system, t-chunk, z, slab) blocks, slabs innermost
  const int b = blockIdx.x, xcd = b & 7, kk = b >> 3;
  const int lin = xcd * ((per >> 3) * nrhs) + kk;
  const int kr = lin / per;
  int rem = lin - kr * per;
  const int p = rem % P;
  rem /= P;
  const int z = rem % g.L[2];
  const int tc = rem / g.L[2];
  const int k = ea.k0 + kr;
  if (ea.st && !slot_active(ea.st, k, ea.state_mode, ea.par, ea.ru_mask)) return;   // uniform
  const unsigned act = 1u;
  const int Vp = g.Vp;
  const size_t rstride = (size_t)field_planes<F64>(12) * Vp;
  const C* f = in + (size_t)k * rstride;
  const typename LP::S* links = (const typename LP::S*)oa.links;
  const int tid = threadIdx.x;
  const int t0 = tc * T;

  double alpha[1] = {0.0};
  if constexpr (EPI == EPI_CG_UPDATE) {
    const double tt = sum_partials(ea.part_in + (size_t)k * ea.nbp, ea.nbp, red);
    const double rho = ea.st[k].rho[ea.par];
    alpha[0] = (tt > 0.0 && isfinite(tt) && isfinite(rho)) ? rho / tt : 0.0;
    if (p == 0 && z == 0 && tc == 0 && tid == 0) {   // the block holding site block 0
      if (!(tt > 0.0 && isfinite(tt))) ea.st[k].flags |= 1;
      ea.st[k].alpha[ea.q4] = alpha[0];
    }
  }
  const R coef = (R)-2 * (R)(rhs_mass(oa, k) + 4.0 * oa.r);

  // prologue: psi(t0) into LDS; the -t hop of t0 from psi(t0 - 1), U_t(t0 - 1)
  int i = p * 256 + tid + plane * (z + g.L[2] * t0);
  Coord c = site_coords(g, i);
  {
    C v[12];
    R sc;
    ld_site_raw<F64, 12>(f, Vp, i, v, sc);
#pragma unroll
    for (int q = 0; q < 12; ++q) nxt[q][tid] = v[q];
  }
  R fb;
  {
    bool wrap;
    const int j = nb_bwd(g, c, i, 3, wrap);
    C lk[9];
    load_link<LP, NL, true>(links, Vp, 3, j, lk);
    C psi[12];
    R sc;
    ld_site_raw<F64, 12>(f, Vp, j, psi, sc);
    C h[2][3], uhb[2][3];
    W::template project<3, TTB>(psi, h);
    mvd(lk, h[0], uhb[0]);
    mvd(lk, h[1], uhb[1]);
#pragma unroll
    for (int q = 0; q < 6; ++q) ub[q][tid] = uhb[q / 3][q % 3];
    fb = W::template hop_factor<LP>(sc, wrap && g.bc[3] < 0);
  }

#pragma unroll 1
  for (int st = 0; st < T; ++st) {
    if (st > 0) {
      i += plane * g.L[2];
      c.x[3] += 1;
    }
    const int sb = i >> 8;
    C acc[1][12];
    {
      C v[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) v[q] = nxt[q][tid];
#pragma unroll
      for (int q = 0; q < 12; ++q) acc[0][q] = cscale(v[q], coef);
    }
    // -t hop (formed at the previous step, or in the prologue)
    {
      C uhb[2][3];
#pragma unroll
      for (int q = 0; q < 6; ++q) uhb[q / 3][q % 3] = ub[q][tid];
      W::template accumulate_uh<3, TTB>(uhb, fb, acc[0]);
    }
    // +t hop; psi(t + 1) becomes the next step's diagonal input, and
    // U_t(t)^dag P psi(t) the next step's -t hop
    {
      // scheduling barriers keep the link and the neighbour spinor from being
      // live at once with the carried values (they would spill)
      bool wrap;
      const int j = nb_fwd(g, c, i, 3, wrap);
      C lk[9];
      load_link<LP, NL, true>(links, Vp, 3, i, lk);
      if (st + 1 < T) {
        C hb[2][3];
        {
          C own[12];
#pragma unroll
          for (int q = 0; q < 12; ++q) own[q] = nxt[q][tid];
          W::template project<3, TTB>(own, hb);
        }
        C uhb[2][3];
        mvd(lk, hb[0], uhb[0]);
        mvd(lk, hb[1], uhb[1]);
#pragma unroll
        for (int q = 0; q < 6; ++q) ub[q][tid] = uhb[q / 3][q % 3];
        fb = W::template hop_factor<LP>((R)1, false);   // t + 1 < L4 inside a chunk
      }
      __builtin_amdgcn_sched_barrier(0);
      C h[2][3];
      R sc;
      {
        C psi[12];
        ld_site_raw<F64, 12>(f, Vp, j, psi, sc);
        if (st + 1 < T) {
#pragma unroll
          for (int q = 0; q < 12; ++q) nxt[q][tid] = psi[q];
        }
        W::template project<3, TTF>(psi, h);
      }
      W::template accumulate<3, TTF, false>(lk, h, W::template hop_factor<LP>(sc, wrap && g.bc[3] < 0),
                                            acc[0]);
    }
    __builtin_amdgcn_sched_barrier(0);
    // x, y and z hops, as stencil_kernel (the loop kept rolled)
#pragma unroll 1
    for (int h0 = 0; h0 < 6; ++h0) {
      int hh = h0;
      asm volatile("" : "+s"(hh));
      switch (hh) {
        case 0: W::template hop_r1<0, false, 1>(oa, f, rstride, c, i, act, acc); break;
        case 1: W::template hop_r1<0, true, 1>(oa, f, rstride, c, i, act, acc); break;
        case 2: W::template hop_r1<1, false, 1>(oa, f, rstride, c, i, act, acc); break;
        case 3: W::template hop_r1<1, true, 1>(oa, f, rstride, c, i, act, acc); break;
        case 4: W::template hop_r1<2, false, 1>(oa, f, rstride, c, i, act, acc); break;
        default: W::template hop_r1<2, true, 1>(oa, f, rstride, c, i, act, acc); break;
      }
    }
    C o[1][12];
#pragma unroll
    for (int q = 0; q < 12; ++q) o[0][q] = cscale(acc[0][q], (R)-0.5);
    site_epilogue<Op, EPI, 1, 0>(oa, ea, k, act, i, true, sb, o, alpha, red);
  }
}

// ------------------------------------------------------- 16-bit, batched
// The batched 16-bit Wilson CG stencils (r = 1, one system per thread)
// sweeping t in the same way.  The kernel is written for any storage policy,
// but runs only where four of its blocks fit on a CU (launch_tsweep_lo), which
// rules out FP32 storage (130 VGPRs, 60 KB of LDS).  A block owns the slab (p, z) of one system for
// t in [t0, t0 + T); the storage words of psi at the step's slice sit in LDS,
// so the diagonal needs no fetch, and the -t hop of t + 1 is formed at step t
// from psi(t) and the link U_t(t) of the +t hop (kept in LDS: carried in
// registers through the step loop it cost a register move per value and
// hop).  With XY (x-y planes of exactly 256 sites, i.e. the slab is
// the whole plane) the x and y neighbours are read from the LDS words as well,
// and only the z and +t neighbours are fetched.
//
// Every step does what stencil_kernel does for that site in the same order
// and with the same operations (diagonal, x+, x-, y+, y-, z+, z-, t+, t-; the
// -t link product is the same mvd of the same decoded link and projection,
// only formed one step earlier), so the result is bitwise stencil_kernel's:
// the choice between them (an autotuner candidate) never changes a solve.
//
// Blocks: XCD x owns the t-slices [x L4/8, (x+1) L4/8) (T divides L4/8) and
// takes the systems one after the other, as block order -3 does, so the links
// of its slices stay in its L2 across the systems.
// Block-order codes (EpiArgs::window) of this kernel: -11, -12, -13 sweep
// T = 2, 4, 8 slices with the x and y neighbours from LDS, -14, -15, -16 the
// same with them fetched.
__host__ __device__ inline bool tsweep_lo_code(int window, int& T, bool& xy) {
  if (window > -11 || window < -16) return false;
  const int c = -window - 10;
  T = 2 << ((c - 1) % 3);
  xy = c <= 3;
  return true;
}
__host__ inline bool tsweep_lo_ok(const Geom& g, int T, bool xy) {
  const int plane = g.L[0] * g.L[1];
  if (T < 1 || (plane & 255) || nbp_of(g.V) * 256 != g.V || g.L[3] % (8 * T)) return false;
  return !xy || plane == 256;
}

// One r = 1 hop along +-MU whose neighbour lies in the slab: as
// WilsonOp::hop_r1, with the neighbour's storage words read from LDS (rc =
// the slab's words, base = the slab's first site).
template <class W, class LP, int NL, int NW, int MU, bool BACK>
__device__ __forceinline__ void tsweep_hop_lds(const Geom& g, const typename LP::S* links,
                                               const uint32_t (*rc)[256], int base,
                                               const Coord& c, int i, typename W::C acc[12]) {
  constexpr int s = W::kDag ? -1 : 1;
  constexpr int TT = BACK ? s : -s;
  bool wrap;
  const int j = BACK ? nb_bwd(g, c, i, MU, wrap) : nb_fwd(g, c, i, MU, wrap);
  const bool flip = wrap && g.bc[MU] < 0;
  typename W::C lk[9];
  load_link<LP, NL, true>(links, g.Vp, MU, BACK ? j : i, lk);
  uint32_t w[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) w[q] = rc[q][j - base];
  typename W::C h[2][3];
  typename W::R sc;
  W::template project_words<MU, TT>(w, h, sc);
  W::template accumulate<MU, TT, BACK>(lk, h, W::template hop_factor<LP>(sc, flip), acc);
}

template <class P, int NL, bool DAG, int EPI, int CP, bool XY>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(WilsonOpR1<P, NL, DAG>::kWaves, 8)))
wilson_tsweep_lo_kernel(const OpArgs oa, const typename P::S* __restrict__ in, const EpiArgs ea,
                        int T, int nrhs) {
  using Op = WilsonOpR1<P, NL, DAG>;
  using W = WilsonOp<P, NL, DAG, false>;
  using LP = typename LinkPol<P, NL>::type;
  using C = typename P::C;
  using R = typename P::R;
  constexpr int NW = vec_rec_bytes<P>(12) / 4;
  constexpr int sgn = DAG ? -1 : 1;
  constexpr int TTF = -sgn, TTB = sgn;   // hop along +t, along -t
  // the epilogue's block sum is what orders each step's LDS writes before
  // the next step's reads
  static_assert(EPI == EPI_STORE_NORM || EPI == EPI_CG_UPDATE, "epilogues with a block sum only");
  __shared__ double red[16];
  __shared__ uint32_t rec[2][NW][256];   // psi's storage words at the step's slice / the next
  __shared__ C ubs[6][256];              // the step's -t link product (registers would shuffle)
  const Geom& g = oa.g;
  const int plane = g.L[0] * g.L[1];
  const int P_ = plane >> 8, TX = (g.L[3] >> 3) / T;
  const int per = P_ * g.L[2] * TX;      // blocks of one system on one XCD
  const int b = blockIdx.x, xcd = b & 7, kk = b >> 3;
  const int kr = kk / per;
  int rem = kk - kr * per;
  const int p = rem % P_;
  rem /= P_;
  const int z = rem % g.L[2];
  const int tc = xcd * TX + rem / g.L[2];
  const int k = ea.k0 + kr;
  if (ea.st && !slot_active(ea.st, k, ea.state_mode, ea.par, ea.ru_mask)) return;   // uniform
  const int Vp = g.Vp;
  const size_t rstride = (size_t)field_planes<P>(12) * Vp;
  const typename P::S* f = in + (size_t)k * rstride;
  const typename LP::S* links = (const typename LP::S*)oa.links;
  const int tid = threadIdx.x;
  const int t0 = tc * T;

  double alpha[1] = {0.0};
  if constexpr (EPI == EPI_CG_UPDATE) {
    const double tt = sum_partials(ea.part_in + (size_t)k * ea.nbp, ea.nbp, red);
    const double rho = ea.st[k].rho[ea.par];
    alpha[0] = (tt > 0.0 && isfinite(tt) && isfinite(rho)) ? rho / tt : 0.0;
    if (p == 0 && z == 0 && tc == 0 && tid == 0) {   // the block holding site block 0
      if (!(tt > 0.0 && isfinite(tt))) ea.st[k].flags |= 1;
      ea.st[k].alpha[ea.q4] = alpha[0];
    }
  }
  const R diag = (R)(rhs_mass(oa, k) + 4.0 * oa.r);

  // prologue: psi(t0)'s words into LDS; the -t hop of t0 from psi(t0 - 1), U_t(t0 - 1)
  int i = p * 256 + tid + plane * (z + g.L[2] * t0);
  Coord c = site_coords(g, i);
  {
    uint32_t w[NW];
    ld_rec<NW * 4>(f, Vp, i, w);
#pragma unroll
    for (int q = 0; q < NW; ++q) rec[0][q][tid] = w[q];
  }
  R fb;
  {
    bool wrap;
    const int j = nb_bwd(g, c, i, 3, wrap);
    C lk[9];
    load_link<LP, NL, true>(links, Vp, 3, j, lk);
    uint32_t w[NW];
    ld_rec<NW * 4>(f, Vp, j, w);
    C h[2][3], ub[2][3];
    R sc;
    W::template project_words<3, TTB>(w, h, sc);
    mvd(lk, h[0], ub[0]);
    mvd(lk, h[1], ub[1]);
#pragma unroll
    for (int q = 0; q < 6; ++q) ubs[q][tid] = ub[q / 3][q % 3];
    fb = W::template hop_factor<LP>(sc, wrap && g.bc[3] < 0);
  }
  if constexpr (XY) __syncthreads();   // the step reads its neighbours' words

#pragma unroll 1
  for (int st = 0; st < T; ++st) {
    const int cur = st & 1;
    if (st > 0) {
      i += plane * g.L[2];
      c.x[3] += 1;
    }
    const int sb = i >> 8;
    C acc[1][12];
    {
      uint32_t w[NW];
#pragma unroll
      for (int q = 0; q < NW; ++q) w[q] = rec[cur][q][tid];
      C v[12];
      R sc;
      dec_site_raw<P, 12>(w, v, sc);
      const R coef = (R)-2 * diag * sc;
#pragma unroll
      for (int q = 0; q < 12; ++q) acc[0][q] = cscale(v[q], coef);
    }
    // x, y and z hops, both hops of a direction per iteration (the loop kept
    // rolled: unrolled, every hop's loads are hoisted and spill)
    {
      const uint32_t(*rc)[256] = rec[cur];
      const int base = i - tid;
#pragma unroll 1
      for (int m0 = 0; m0 < 3; ++m0) {
        int mu = m0;
        asm volatile("" : "+s"(mu));
        switch (mu) {
          case 0:
            if constexpr (XY) {
              tsweep_hop_lds<W, LP, NL, NW, 0, false>(g, links, rc, base, c, i, acc[0]);
              tsweep_hop_lds<W, LP, NL, NW, 0, true>(g, links, rc, base, c, i, acc[0]);
            } else {
              W::template hop_r1<0, false, 1>(oa, f, rstride, c, i, 1u, acc);
              W::template hop_r1<0, true, 1>(oa, f, rstride, c, i, 1u, acc);
            }
            break;
          case 1:
            if constexpr (XY) {
              tsweep_hop_lds<W, LP, NL, NW, 1, false>(g, links, rc, base, c, i, acc[0]);
              tsweep_hop_lds<W, LP, NL, NW, 1, true>(g, links, rc, base, c, i, acc[0]);
            } else {
              W::template hop_r1<1, false, 1>(oa, f, rstride, c, i, 1u, acc);
              W::template hop_r1<1, true, 1>(oa, f, rstride, c, i, 1u, acc);
            }
            break;
          default:
            W::template hop_r1<2, false, 1>(oa, f, rstride, c, i, 1u, acc);
            W::template hop_r1<2, true, 1>(oa, f, rstride, c, i, 1u, acc);
            break;
        }
      }
    }
    // +t hop, then the -t hop (formed at the previous step, or in the
    // prologue); psi(t + 1)'s words become the next step's, and
    // U_t(t)^dag P psi(t) the next step's -t hop (the order of the one-site
    // stencil's accumulation: t+ before t-)
    {
      bool wrap;
      const int j = nb_fwd(g, c, i, 3, wrap);
      C lk[9];
      load_link<LP, NL, true>(links, Vp, 3, i, lk);
      {
        uint32_t w[NW];
        ld_rec<NW * 4>(f, Vp, j, w);
        if (st + 1 < T) {
#pragma unroll
          for (int q = 0; q < NW; ++q) rec[cur ^ 1][q][tid] = w[q];
        }
        C h[2][3];
        R sc;
        W::template project_words<3, TTF>(w, h, sc);
        W::template accumulate<3, TTF, false>(lk, h, W::template hop_factor<LP>(sc, wrap && g.bc[3] < 0),
                                              acc[0]);
      }
      {
        C ub[2][3];
#pragma unroll
        for (int q = 0; q < 6; ++q) ub[q / 3][q % 3] = ubs[q][tid];
        W::template accumulate_uh<3, TTB>(ub, fb, acc[0]);
      }
      if (st + 1 < T) {
        uint32_t w[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) w[q] = rec[cur][q][tid];
        C h[2][3], un[2][3];
        R sc;
        W::template project_words<3, TTB>(w, h, sc);
        mvd(lk, h[0], un[0]);
        mvd(lk, h[1], un[1]);
#pragma unroll
        for (int q = 0; q < 6; ++q) ubs[q][tid] = un[q / 3][q % 3];
        fb = W::template hop_factor<LP>(sc, false);   // t + 1 < L4 inside a chunk
      }
    }
    C o[1][12];
#pragma unroll
    for (int q = 0; q < 12; ++q) o[0][q] = cscale(acc[0][q], (R)-0.5);
    site_epilogue<Op, EPI, 1, CP>(oa, ea, k, 1u, i, true, sb, o, alpha, red);
    // the epilogue's block sum orders this step's reads of rec[cur] before
    // the next step's writes to it, and this step's writes before its reads
  }
}

}  // namespace lq
