// Batched Wilson stencil (r = 1) with four systems across the lanes of each
// site and the link products on the matrix cores.
//
// Layout of a block (1024 threads = 16 wavefronts): the 256 sites of one site
// block times four consecutive systems k0 .. k0+3.  Wavefront w holds sites
// 16w .. 16w+15 of the block, lane 4s + j being site 16w + s for system k0 + j.
// Each lane projects its own system's neighbour spinor to the two-spinor h
// (as the one-system-per-thread stencil does) and, for the link product
// uh = L h (L^dag h for a backward hop), supplies the line j of the link:
// row j of L (column j for L^dag), lane j = 3 supplying zeros.  A 16-block
// 4x4x1 FP32 MFMA then forms, for every site of the wavefront at once,
//   D[r][j] = sum over the six real steps of (line r entries) x (lane j's h),
// so that lane j receives the three rows of its own system's uh.  Real and
// imaginary parts are separate MFMA chains whose steps follow the order of
// the complex multiply-adds of mv / mvd (each MFMA step rounds like one FMA),
// so uh -- and everything after it, which is the one-system code -- is
// bitwise what the one-system-per-thread kernel computes.  Block partial sums
// are reduced through LDS in the order of block_sum over the same 256 sites,
// so partials, alpha and beta are bitwise the same too.
//
// The link entries enter raw (16-bit integers or FP32 values, as the
// one-system kernel's RAW loads give them); 18-real links only (no row
// rebuild).
#pragma once

#include "stencil.h"

namespace lq {

typedef float lq_f4 __attribute__((ext_vector_type(4)));

constexpr int kLanesBlock = 1024;   // threads per block of the lanes stencil
constexpr int kLanesK = 8;          // rhs_per_thread code that selects it

template <class P, int NL, bool DAG>
struct WilsonLanesOp {
  static_assert(NL == 18, "the lanes stencil reads 18-real links");
  using W = WilsonOp<P, NL, DAG, false>;
  using Pol = P;
  static constexpr int NC = 12;
  using C = typename P::C;
  using R = typename P::R;
  using S = typename P::S;
  using LP = typename LinkPol<P, NL>::type;

  // Entries (line, c), c = 0..2, of the 18-real link record of direction MU at
  // site `ls`: row `line` (BACK = false) or column `line` (BACK = true), as
  // raw values; line 3 gives zeros.  Entry e of the record is element e of its
  // 16-byte slabs (e < 8) or of the remainder plane (e = 8).
  template <int MU, bool BACK>
  __device__ __forceinline__ static void load_line(const OpArgs& a, int ls, int line, R lr[3],
                                                   R li[3]) {
    constexpr int EB = (int)sizeof(typename LP::S);   // 4 (16-bit pairs) or 8 (FP32 pairs)
    constexpr int PER = 16 / EB;                      // entries per slab element
    constexpr int NSLAB = (9 * EB) / 16;              // whole slabs of the record
    const uint32_t vp = (uint32_t)a.g.Vp;
    const auto rs = rsrc((const typename LP::S*)a.links + (size_t)MU * 9 * a.g.Vp);
    const int ln = line < 3 ? line : 2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int e = BACK ? 3 * c + ln : 3 * ln + c;
      const uint32_t off = e < NSLAB * PER
                               ? (uint32_t)(e / PER) * vp * 16u + (uint32_t)ls * 16u + (uint32_t)(e % PER) * EB
                               : (uint32_t)NSLAB * vp * 16u + (uint32_t)ls * EB;
      C z;
      if constexpr (EB == 4) {
        const uint32_t wd = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        z = dec_raw<LP>(&wd);
      } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
        const uint32_t wd[2] = {v[0], v[1]};
        z = dec_raw<LP>(wd);
      }
      lr[c] = line < 3 ? z.x : (R)0;
      li[c] = line < 3 ? z.y : (R)0;
    }
  }

  // uh = L h (forward) or L^dag h (BACK) for the two spins, lane j holding
  // its own system's h and line j of the link (see the file header).  The
  // steps of each chain follow mv (forward: re += Lr hr, re -= Li hi, ...;
  // im += Lr hi, im += Li hr, ...) or mvd (re += Lr hr, re += Li hi; im +=
  // Lr hi, im -= Li hr) column by column.
  template <bool BACK>
  __device__ __forceinline__ static void link_product(const R lr[3], const R li[3],
                                                      const C h[2][3], C uh[2][3]) {
    lq_f4 re0 = {0, 0, 0, 0}, im0 = {0, 0, 0, 0}, re1 = {0, 0, 0, 0}, im1 = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const R nli = -li[c];
      re0 = __builtin_amdgcn_mfma_f32_4x4x1f32(lr[c], h[0][c].x, re0, 0, 0, 0);
      im0 = __builtin_amdgcn_mfma_f32_4x4x1f32(lr[c], h[0][c].y, im0, 0, 0, 0);
      re1 = __builtin_amdgcn_mfma_f32_4x4x1f32(lr[c], h[1][c].x, re1, 0, 0, 0);
      im1 = __builtin_amdgcn_mfma_f32_4x4x1f32(lr[c], h[1][c].y, im1, 0, 0, 0);
      re0 = __builtin_amdgcn_mfma_f32_4x4x1f32(BACK ? li[c] : nli, h[0][c].y, re0, 0, 0, 0);
      im0 = __builtin_amdgcn_mfma_f32_4x4x1f32(BACK ? nli : li[c], h[0][c].x, im0, 0, 0, 0);
      re1 = __builtin_amdgcn_mfma_f32_4x4x1f32(BACK ? li[c] : nli, h[1][c].y, re1, 0, 0, 0);
      im1 = __builtin_amdgcn_mfma_f32_4x4x1f32(BACK ? nli : li[c], h[1][c].x, im1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      uh[0][r].x = re0[r]; uh[0][r].y = im0[r];
      uh[1][r].x = re1[r]; uh[1][r].y = im1[r];
    }
  }

  // One r = 1 hop along +-MU for this lane's system (if active) at site i;
  // every lane of the wavefront must call it (the MFMAs use all lanes).
  template <int MU, bool BACK>
  __device__ __forceinline__ static void hop(const OpArgs& a, const S* __restrict__ in,
                                             uint32_t lo, const Coord& c, int i, int line,
                                             bool active, C acc[12]) {
    constexpr int s = DAG ? -1 : 1;
    constexpr int TT = BACK ? s : -s;
    const Geom& g = a.g;
    bool wrap;
    const int j = BACK ? nb_bwd(g, c, i, MU, wrap) : nb_fwd(g, c, i, MU, wrap);
    const bool flip = wrap && g.bc[MU] < 0;
    R lr[3], li[3];
    load_line<MU, BACK>(a, BACK ? j : i, line, lr, li);
    // an inactive lane's h only enters its own output column, which is
    // discarded: it takes zeros (the branch also keeps the next hop's loads
    // from being hoisted into this one, which would spill)
    R sc = (R)0;
    C h[2][3];
    if (active) {
      if constexpr (P::kSiteScale) {
        W::template project_q16<MU, TT>(in, g.Vp, j, h, sc, lo);
      } else {
        C psi[12];
        ld_site_raw<P, 12>(in, g.Vp, j, psi, sc, lo);
        W::template project<MU, TT>(psi, h);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 3; ++q) { h[0][q] = czero<C>(); h[1][q] = czero<C>(); }
    }
    C uh[2][3];
    link_product<BACK>(lr, li, h, uh);
    if (active) W::template accumulate_uh<MU, TT>(uh, W::template hop_factor<LP>(sc, flip), acc);
  }

  // out = M psi (or M^dag psi) at site i for the system k of this lane, whose
  // field is `lo` bytes past the wavefront-uniform `in` (the group's first
  // system).  Called by every lane; the outputs of inactive lanes (and of
  // lanes past the last site, i clamped) are discarded by the caller.
  __device__ __forceinline__ static void site(const OpArgs& a, const S* __restrict__ in,
                                              uint32_t lo, int i, int k, int line, bool active,
                                              C out[12]) {
    const Geom& g = a.g;
    const Coord c = site_coords(g, i);
    C acc[12];
    {
      const R diag = (R)(rhs_mass(a, k) + 4.0 * a.r);
      C v[12];
      R sc = (R)0;
      if (active) ld_site_raw<P, 12>(in, g.Vp, i, v, sc, lo);
      const R coef = (R)-2 * diag * sc;
#pragma unroll
      for (int q = 0; q < 12; ++q) acc[q] = active ? cscale(v[q], coef) : czero<C>();
    }
    // straight-line hops, one at a time: the barriers keep each hop's loads
    // behind the previous hop's arithmetic (a rolled loop over the hops makes
    // the compiler shuffle the accumulators between the MFMA result tuples)
    hop<0, false>(a, in, lo, c, i, line, active, acc);
    __builtin_amdgcn_sched_barrier(0);
    hop<0, true>(a, in, lo, c, i, line, active, acc);
    __builtin_amdgcn_sched_barrier(0);
    hop<1, false>(a, in, lo, c, i, line, active, acc);
    __builtin_amdgcn_sched_barrier(0);
    hop<1, true>(a, in, lo, c, i, line, active, acc);
    __builtin_amdgcn_sched_barrier(0);
    hop<2, false>(a, in, lo, c, i, line, active, acc);
    __builtin_amdgcn_sched_barrier(0);
    hop<2, true>(a, in, lo, c, i, line, active, acc);
    __builtin_amdgcn_sched_barrier(0);
    hop<3, false>(a, in, lo, c, i, line, active, acc);
    __builtin_amdgcn_sched_barrier(0);
    hop<3, true>(a, in, lo, c, i, line, active, acc);
#pragma unroll
    for (int q = 0; q < 12; ++q) out[q] = cscale(acc[q], (R)-0.5);
  }
};

// The lanes stencil with the epilogues of the batched CG: STORE, STORE_NORM
// (t = M p, ||t||^2) and CG_UPDATE (q = M^dag t, r -= alpha q, ||r||^2, the
// grouped x update).  Grid: nbp site blocks x ceil(nrhs / 4) system groups,
// in the block orders of map_block / map_block_tiled.
template <class Op, int EPI, int CP>
__global__ void __launch_bounds__(kLanesBlock)
stencil_lanes_kernel(const OpArgs oa, const typename Op::S* __restrict__ in, const EpiArgs ea,
                     int ngroups, int nrhs) {
  using C = typename Op::C;
  using S = typename Op::S;
  using Pol = typename Op::Pol;
  constexpr int NC = 12;
  __shared__ double red[16];
  __shared__ double vals[4][256];
  __shared__ double part4[4][4];
  int sb, kg;
  if ((ea.window != -3 && ea.window != -4) ||
      !map_block_tiled(oa.g, ea.nbp, ngroups, ea.window, sb, kg))
    map_block(ea.nbp, ngroups, ea.window < -2 ? 0 : ea.window, sb, kg);
  const int k0 = ea.k0 + kg * 4;
  unsigned act = 0;
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const int k = k0 + jj;
    if (k < ea.k0 + nrhs && (!ea.st || slot_active(ea.st, k, ea.state_mode, ea.par, ea.ru_mask)))
      act |= 1u << jj;
  }
  if (act == 0) return;   // uniform over the block

  const int t = threadIdx.x, wv = t >> 6, ln = t & 63;
  const int sl = 16 * wv + (ln >> 2);           // site within the block
  const int j = ln & 3;                         // system within the group
  const int Vp = oa.g.Vp;
  const int i = sb * 256 + sl;
  const bool valid = i < oa.g.V;
  const bool active = valid && ((act >> j) & 1);
  const size_t rstride = (size_t)field_planes<Pol>(NC) * Vp;

  double alpha = 0.0;
  if constexpr (EPI == EPI_CG_UPDATE) {
    // alpha of each system from the partials of the previous launch (every
    // thread takes part in the block reductions; fixed order)
#pragma unroll 1
    for (int jj = 0; jj < 4; ++jj) {
      if (!((act >> jj) & 1)) continue;   // uniform over the block
      const int k = k0 + jj;
      const double tt = sum_partials(ea.part_in + (size_t)k * ea.nbp, ea.nbp, red);
      const double rho = ea.st[k].rho[ea.par];
      const double al = (tt > 0.0 && isfinite(tt) && isfinite(rho)) ? rho / tt : 0.0;
      if (jj == j) alpha = al;
      if (sb == 0 && t == 0) {
        if (!(tt > 0.0 && isfinite(tt))) ea.st[k].flags |= 1;
        ea.st[k].alpha[ea.q4] = al;
      }
    }
  }

  // every field access goes through the uniform base of system k0 plus the
  // lane's byte offset (a per-lane base would make the buffer descriptors
  // divergent)
  C o[NC];
  const int k = k0 + j;
  const size_t off0 = (size_t)k0 * rstride;
  const uint32_t lo = (uint32_t)((size_t)j * rstride * sizeof(S));
  // lanes past the end of the batch read the group's first system (its
  // field and its mass) instead
  const bool in_batch = k < ea.k0 + nrhs;
  Op::site(oa, in + off0, in_batch ? lo : 0u, valid ? i : 0, in_batch ? k : k0, j, active, o);

  double val = 0.0;
  if (active) {
    if constexpr (EPI == EPI_STORE || EPI == EPI_STORE_NORM) {
      const double n2 = st_site<Pol, NC>((S*)ea.out + off0, Vp, i, o, lo);
      if constexpr (EPI == EPI_STORE_NORM) val = n2;
    } else if constexpr (EPI == EPI_CG_UPDATE) {
      using XP = typename XPol<Pol>::type;
      const uint32_t lox = (uint32_t)((size_t)j * NC * Vp * sizeof(typename XP::S));
      val = cg_update_site<Op, CP>(ea, Vp, k, off0, i, alpha, o, k0, lo, lox);
    }
  }
  if constexpr (EPI != EPI_STORE) {
    // per system, the sum over the block's 256 sites in block_sum's order:
    // four chunks of 64 consecutive sites, each by the wavefront butterfly,
    // then the chunks in order
    vals[j][sl] = val;
    __syncthreads();
    const int rj = wv >> 2, ch = wv & 3;
    const double v = wave_sum(vals[rj][64 * ch + ln]);
    if (ln == 0) part4[rj][ch] = v;
    __syncthreads();
    if (t < 4 && ((act >> t) & 1)) {
      double s = 0.0;
      for (int c2 = 0; c2 < 4; ++c2) s += part4[t][c2];
      ea.part[(size_t)(k0 + t) * ea.nbp + sb] = s;
    }
  }
}

}  // namespace lq
