// Per-site Dirac operators of eq. (2): the Wilson matrix (K1), the staggered
// Wilson matrix from precomputed corner matrices (K4) and with Gamma_55 built
// on the fly from the links (K2).  Each computes the NC output components of
// one site for one right-hand side into registers; the stencil kernels add
// their epilogues (store, fused norms, CG updates) around them.
#pragma once

#include "common.h"
#include "lq_types.h"

namespace lq {

// Operator arguments shared by every stencil kernel.
struct OpArgs {
  Geom g;
  const void* links;     // SoA links in the kernel's precision
  const void* corners;   // SoA corners (staggered Wilson, corner form)
  double r;              // Wilson parameter
  double mass0;          // mass when `mass` is null
  const double* mass;    // per-RHS mass, mass[k * mass_stride]
  int mass_stride;
  // even-odd blocks (WilsonEOOp): links of the other parity, the field
  // multiplying d in the Schur form, the output parity, and the form
  const void* links_nb = nullptr;
  const void* diag_in = nullptr;
  int eo_par = 0;
  int eo_schur = 0;
  // on-the-fly Gamma_55: the intermediate fields of system k start at
  // (char*)g55w + k * g55_sys (see G55Pol, kG55Fields)
  void* g55w = nullptr;
  size_t g55_sys = 0;
};

__device__ __forceinline__ double rhs_mass(const OpArgs& a, int k) {
  return a.mass ? a.mass[(size_t)k * a.mass_stride] : a.mass0;
}

// ------------------------------------------------------------------ Wilson
// (M psi)(x) = (m + 4r) psi(x) - 1/2 sum_mu [(r - s g_mu) U_mu(x) psi(x+mu)
//                                    + (r + s g_mu) U_mu(x-mu)^dag psi(x-mu)]
// s = +1 for M, -1 for M^dag (gamma_5-hermiticity).  The gamma basis is
// g_mu = [[0, B_mu], [B_mu^dag, 0]] with B_1 = i s1, B_2 = -i s2, B_3 = i s3,
// B_4 = 1.  For r = 1 the hop uses spin projection: (1 + t g_mu) psi =
// [h; t B^dag h] with h = psi_up + t B psi_lo, so only the two-spinor h is
// multiplied by the link (the paper's "8 x 2" count, Sec. 3).
template <typename C>
__device__ __forceinline__ void bmul(int mu, const C lo0, const C lo1, C& o0, C& o1) {
  // (o0, o1) = B_mu (lo0, lo1)
  switch (mu) {
    case 0: o0 = cmuli(lo1); o1 = cmuli(lo0); break;
    case 1: o0 = cneg(lo1); o1 = lo0; break;
    case 2: o0 = cmuli(lo0); o1 = cmulmi(lo1); break;
    default: o0 = lo0; o1 = lo1; break;
  }
}
template <typename C>
__device__ __forceinline__ void bdmul(int mu, const C h0, const C h1, C& o0, C& o1) {
  // (o0, o1) = B_mu^dag (h0, h1)
  switch (mu) {
    case 0: o0 = cmulmi(h1); o1 = cmulmi(h0); break;
    case 1: o0 = h1; o1 = cneg(h0); break;
    case 2: o0 = cmulmi(h0); o1 = cmuli(h1); break;
    default: o0 = h0; o1 = h1; break;
  }
}

template <class P, int NL, bool DAG, bool GENERAL_R = false>
struct WilsonOp {
  using Pol = P;
  static constexpr int NC = 12;
  static constexpr bool kDag = DAG;
  static constexpr int kWaves = P::id == 0 ? 3 : 4;
  using C = typename P::C;
  using R = typename P::R;
  using S = typename P::S;

  // General r: acc += (r + t g_mu) L psi_nb, L = the pre-loaded link lk or
  // its adjoint (no spin projection).
  __device__ __forceinline__ static void hop(const OpArgs& a, const S* __restrict__ in, int nb,
                                             int mu, bool dagger_link, R t, R sgn, const C lk[9],
                                             C acc[12]) {
    const int Vp = a.g.Vp;
    C psi[12];
    ld_site<P, 12>(in, Vp, nb, psi);
    {
      // general r: (r + t g) L psi = r L psi + t g (L psi), all four spins
      C w[4][3];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        C v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = cscale(psi[s * 3 + c], sgn);
        if (dagger_link) mvd(lk, v, w[s]); else mv(lk, v, w[s]);
      }
      const R rr = (R)a.r;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        C gu0, gu1, gl0, gl1;
        bmul(mu, w[2][c], w[3][c], gu0, gu1);    // upper = B lower
        bdmul(mu, w[0][c], w[1][c], gl0, gl1);   // lower = B^dag upper
        acc[0 * 3 + c] = cadd(acc[0 * 3 + c], cadd(cscale(w[0][c], rr), cscale(gu0, t)));
        acc[1 * 3 + c] = cadd(acc[1 * 3 + c], cadd(cscale(w[1][c], rr), cscale(gu1, t)));
        acc[2 * 3 + c] = cadd(acc[2 * 3 + c], cadd(cscale(w[2][c], rr), cscale(gl0, t)));
        acc[3 * 3 + c] = cadd(acc[3 * 3 + c], cadd(cscale(w[3][c], rr), cscale(gl1, t)));
      }
    }
  }

  template <int K>
  static constexpr bool kHopPairs() { return P::id != 0 && K == 1; }
  template <int K>
  static constexpr bool kStraight() { return P::id != 0 && K >= 2; }

  // r = 1 hop along +-MU with the gamma structure fixed at compile time:
  // h = sgn * scale * (psi_up + TT B psi_lo) (TT = -s forward, +s backward),
  // uh = L h, then acc += [uh; TT B^dag uh].  Only the link load is shared by
  // the K systems.
  // Spin projection for a hop along MU: h = psi_up + TT B psi_lo.
  template <int MU, int TT>
  __device__ __forceinline__ static void project(const C psi[12], C h[2][3]) {
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      C b0, b1;
      bmul(MU, psi[6 + cc], psi[9 + cc], b0, b1);
      h[0][cc] = TT > 0 ? cadd(psi[cc], b0) : csub(psi[cc], b0);
      h[1][cc] = TT > 0 ? cadd(psi[3 + cc], b1) : csub(psi[3 + cc], b1);
    }
  }

  // project<MU, TT> of the 16-bit site j, on the stored integers: sums and
  // differences of two int16 are exact in int32 and convert exactly to FP32,
  // so h is bitwise what projecting the converted components gives, from 12
  // conversions instead of 24.  sc = the site's scale.  project_q16_words:
  // the same from the record's storage words.
  template <int MU, int TT>
  __device__ __forceinline__ static void project_q16_words(const uint32_t* w, C h[2][3], R& sc) {
    sc = __uint_as_float(w[12]) * (1.0f / kQ16);
    const auto i16x2 = [](uint32_t v) { return make_int2((int)(short)(v & 0xffffu), (int)v >> 16); };
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      int2 b0, b1;
      bmul(MU, i16x2(w[6 + cc]), i16x2(w[9 + cc]), b0, b1);
      const int2 u0 = i16x2(w[cc]), u1 = i16x2(w[3 + cc]);
      const int2 h0 = TT > 0 ? cadd(u0, b0) : csub(u0, b0);
      const int2 h1 = TT > 0 ? cadd(u1, b1) : csub(u1, b1);
      h[0][cc] = make_float2((float)h0.x, (float)h0.y);
      h[1][cc] = make_float2((float)h1.x, (float)h1.y);
    }
  }
  template <int MU, int TT>
  __device__ __forceinline__ static void project_q16(const S* __restrict__ f, int Vp, int j,
                                                     C h[2][3], R& sc, uint32_t lo = 0) {
    constexpr int BY = vec_rec_bytes<P>(12);
    uint32_t w[BY / 4];
    ld_rec<BY>(f, Vp, j, w, lo);
    project_q16_words<MU, TT>(w, h, sc);
  }
  // project<MU, TT> of a site from its storage words, as hop_r1 forms it
  // (the raw integers for 16-bit storage, sc = the site's scale)
  template <int MU, int TT>
  __device__ __forceinline__ static void project_words(const uint32_t* w, C h[2][3], R& sc) {
    if constexpr (P::kSiteScale) {
      project_q16_words<MU, TT>(w, h, sc);
    } else {
      C psi[12];
      dec_site_raw<P, 12>(w, psi, sc);
      project<MU, TT>(psi, h);
    }
  }

  // acc += f [uh; TT B^dag uh], uh = L h with L = lk (forward) or lk^dag (BACK):
  // the site scale, the link's storage scale and the boundary sign enter as
  // the one factor f of the accumulating multiply-adds.
  template <int MU, int TT, bool BACK>
  __device__ __forceinline__ static void accumulate(const C lk[9], const C h[2][3], R f,
                                                    C acc[12]) {
    C uh[2][3];
    if (BACK) { mvd(lk, h[0], uh[0]); mvd(lk, h[1], uh[1]); }
    else { mv(lk, h[0], uh[0]); mv(lk, h[1], uh[1]); }
    accumulate_uh<MU, TT>(uh, f, acc);
  }
  // acc += f [uh; TT B^dag uh] for the link product uh = L h already formed
  template <int MU, int TT>
  __device__ __forceinline__ static void accumulate_uh(const C uh[2][3], R f, C acc[12]) {
    const R ft = TT > 0 ? f : -f;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      C d0, d1;
      bdmul(MU, uh[0][cc], uh[1][cc], d0, d1);
      acc[cc] = cfmas(uh[0][cc], f, acc[cc]);
      acc[3 + cc] = cfmas(uh[1][cc], f, acc[3 + cc]);
      acc[6 + cc] = cfmas(d0, ft, acc[6 + cc]);
      acc[9 + cc] = cfmas(d1, ft, acc[9 + cc]);
    }
  }

  // The factor f of a hop from a neighbour with site scale sc over links of
  // policy LP, with the boundary sign when the hop wraps.
  template <class LP>
  __device__ __forceinline__ static R hop_factor(R sc, bool flip) {
    constexpr bool kScaled = P::kSiteScale || (LP::kRawScale != (typename LP::R)1);
    R f = kScaled ? sc * (R)LP::kRawScale : (R)1;
    return flip ? -f : f;
  }

  // r = 1 hop along +-MU with the gamma structure fixed at compile time:
  // TT = -s forward, +s backward.  Only the link load is shared by the K
  // systems.
  template <int MU, bool BACK, int K>
  __device__ __forceinline__ static void hop_r1(const OpArgs& a, const S* __restrict__ in0,
                                                size_t rstride, const Coord& c, int i,
                                                unsigned act, C acc[K][12]) {
    constexpr int s = DAG ? -1 : 1;
    constexpr int TT = BACK ? s : -s;
    const Geom& g = a.g;
    bool wrap;
    const int j = BACK ? nb_bwd(g, c, i, MU, wrap) : nb_fwd(g, c, i, MU, wrap);
    const bool flip = wrap && g.bc[MU] < 0;
    C lk[9];
    using LP = typename LinkPol<P, NL>::type;
    // raw link: its storage scale joins the neighbour's site scale in f
    load_link<LP, NL, true>((const typename LP::S*)a.links, g.Vp, MU, BACK ? j : i, lk);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!((act >> k) & 1)) continue;
      R sc;
      C h[2][3];
      if constexpr (P::kSiteScale) {
        project_q16<MU, TT>(in0 + k * rstride, g.Vp, j, h, sc);
      } else {
        C psi[12];
        ld_site_raw<P, 12>(in0 + k * rstride, g.Vp, j, psi, sc);
        project<MU, TT>(psi, h);
      }
      accumulate<MU, TT, BACK>(lk, h, hop_factor<LP>(sc, flip), acc[k]);
    }
  }

  // K right-hand sides of one site: input k at in0 + k * rstride, mass of
  // system k0 + k, bit k of `act` set for the systems to compute.  Each link
  // is loaded (and, for 12-real storage, completed) once for all K.
  template <int K>
  __device__ __forceinline__ static void site_multi(const OpArgs& a, const S* __restrict__ in0,
                                                    size_t rstride, int i, int k0, unsigned act,
                                                    C out[K][12]) {
    const Geom& g = a.g;
    Coord c = site_coords(g, i);
    // acc starts at -2 (m + 4r) psi(x) so that out = -acc/2 at the end and
    // psi(x) is not kept live across the hops
    C acc[K][12];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R diag = (R)(rhs_mass(a, k0 + k) + 4.0 * a.r);
      C v[12];
      R sc = (R)0;
      if ((act >> k) & 1) ld_site_raw<P, 12>(in0 + k * rstride, g.Vp, i, v, sc);
      const R coef = (R)-2 * diag * sc;
#pragma unroll
      for (int q = 0; q < 12; ++q)
        acc[k][q] = ((act >> k) & 1) ? cscale(v[q], coef) : czero<C>();
    }
    if constexpr (!GENERAL_R) {
      // Each hop's code has its gamma structure and coordinates built in.
      // Several FP32/16-bit systems per thread: the eight hops in a straight
      // line, a scheduling barrier between them so that no hop's loads are
      // hoisted into an earlier one (a rolled loop would shuffle the K
      // accumulators through its back edge, a register move per value per
      // hop).  Otherwise the loop stays rolled (its index made opaque to the
      // compiler, which would unroll it and hoist every hop's loads into
      // spills); an iteration covers one hop, or both hops of a direction
      // where the registers allow (single-system FP32/Q16).
      if constexpr (kStraight<K>()) {
        hop_r1<0, false, K>(a, in0, rstride, c, i, act, acc);
        __builtin_amdgcn_sched_barrier(0);
        hop_r1<0, true, K>(a, in0, rstride, c, i, act, acc);
        __builtin_amdgcn_sched_barrier(0);
        hop_r1<1, false, K>(a, in0, rstride, c, i, act, acc);
        __builtin_amdgcn_sched_barrier(0);
        hop_r1<1, true, K>(a, in0, rstride, c, i, act, acc);
        __builtin_amdgcn_sched_barrier(0);
        hop_r1<2, false, K>(a, in0, rstride, c, i, act, acc);
        __builtin_amdgcn_sched_barrier(0);
        hop_r1<2, true, K>(a, in0, rstride, c, i, act, acc);
        __builtin_amdgcn_sched_barrier(0);
        hop_r1<3, false, K>(a, in0, rstride, c, i, act, acc);
        __builtin_amdgcn_sched_barrier(0);
        hop_r1<3, true, K>(a, in0, rstride, c, i, act, acc);
      } else if constexpr (kHopPairs<K>()) {
#pragma unroll 1
        for (int m0 = 0; m0 < 4; ++m0) {
          int mu = m0;
          asm volatile("" : "+s"(mu));
          switch (mu) {
            case 0: hop_r1<0, false, K>(a, in0, rstride, c, i, act, acc);
                    hop_r1<0, true, K>(a, in0, rstride, c, i, act, acc); break;
            case 1: hop_r1<1, false, K>(a, in0, rstride, c, i, act, acc);
                    hop_r1<1, true, K>(a, in0, rstride, c, i, act, acc); break;
            case 2: hop_r1<2, false, K>(a, in0, rstride, c, i, act, acc);
                    hop_r1<2, true, K>(a, in0, rstride, c, i, act, acc); break;
            default: hop_r1<3, false, K>(a, in0, rstride, c, i, act, acc);
                     hop_r1<3, true, K>(a, in0, rstride, c, i, act, acc); break;
          }
        }
      } else {
#pragma unroll 1
        for (int h0 = 0; h0 < 8; ++h0) {
          int h = h0;
          asm volatile("" : "+s"(h));
          switch (h) {
            case 0: hop_r1<0, false, K>(a, in0, rstride, c, i, act, acc); break;
            case 1: hop_r1<0, true, K>(a, in0, rstride, c, i, act, acc); break;
            case 2: hop_r1<1, false, K>(a, in0, rstride, c, i, act, acc); break;
            case 3: hop_r1<1, true, K>(a, in0, rstride, c, i, act, acc); break;
            case 4: hop_r1<2, false, K>(a, in0, rstride, c, i, act, acc); break;
            case 5: hop_r1<2, true, K>(a, in0, rstride, c, i, act, acc); break;
            case 6: hop_r1<3, false, K>(a, in0, rstride, c, i, act, acc); break;
            default: hop_r1<3, true, K>(a, in0, rstride, c, i, act, acc); break;
          }
        }
      }
    } else {
      const R s = DAG ? (R)-1 : (R)1;
#pragma unroll 1
      for (int h = 0; h < 8; ++h) {
        const int mu = h >> 1;
        const bool back = h & 1;
        bool wrap;
        const int j = back ? nb_bwd(g, c, i, mu, wrap) : nb_fwd(g, c, i, mu, wrap);
        const R sg = (wrap && g.bc[mu] < 0) ? (R)-1 : (R)1;
        C lk[9];
        // forward: (r - s g) U_mu(x) psi(x+mu); backward: (r + s g) U_mu(x-mu)^dag psi(x-mu)
        using LP = typename LinkPol<P, NL>::type;
        load_link<LP, NL>((const typename LP::S*)a.links, g.Vp, mu, back ? j : i, lk);
#pragma unroll
        for (int k = 0; k < K; ++k)
          if ((act >> k) & 1) hop(a, in0 + k * rstride, j, mu, back, back ? s : -s, sg, lk, acc[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < 12; ++q) out[k][q] = cscale(acc[k][q], (R)-0.5);
  }
};

// ------------------------------------------------ Wilson, even-odd blocks
// Half-lattice Wilson blocks for the even-odd preconditioned solve (the
// preconditioning of the footnote to eq. (2), Sec. 3; r = 1).  A field holds
// the sites of one parity: half site h is whichever of the lexicographic sites
// 2h, 2h + 1 has that parity (the two share x2, x3, x4, and L1 is even).
// Output sites have parity a.eo_par and `in` holds the other parity; with
// d = m + 4 and M_W = [[d, M_eo], [M_oe, d]] in (even, odd) blocks,
//   eo_schur = 0:  out = M_{par, 1-par} in          (= -H in / 2)
//   eo_schur = 1..3: out = c y - M_{par, 1-par} in / d,  y = a.diag_in (parity par),
//                  c = d, 1, 1/d
//   eo_schur = 4:  out = d y + M_{par, 1-par} in      (the parity-par half of M_W)
// so that with in = M_oe y the first Schur form is the complement
// M^ y = (d - M_eo M_oe / d) y; the others give the preconditioned source
// chi_e - M_eo chi_o / d, the odd half (chi_o - M_oe x_e) / d, and the halves
// of M_W (M_W^dag with DAG) applied to a whole field.  Links are stored per parity and half site:
// a.links those of the output parity (forward hops, U_mu(x)), a.links_nb the
// other parity's (backward hops, U_mu(x - mu)).  The geometry's V and Vp are
// those of the half-lattice fields, its extents those of the lattice.
template <class P, int NL, bool DAG>
struct WilsonEOOp {
  using W = WilsonOp<P, NL, DAG, false>;
  using Pol = P;
  static constexpr int NC = 12;
  static constexpr int kWaves = W::kWaves;
  using C = typename P::C;
  using R = typename P::R;
  using S = typename P::S;

  // Coordinates and lexicographic index of half site h of parity par.
  __device__ __forceinline__ static Coord coords_of(const Geom& g, int h, int par, int& i) {
    Coord c = site_coords(g, 2 * h);
    const int b = (c.x[1] + c.x[2] + c.x[3] + par) & 1;
    c.x[0] += b;
    i = 2 * h + b;
    return c;
  }

  // One r = 1 hop along +-MU for K systems, as WilsonOp::hop_r1 with the
  // neighbour and its link read from their parity's half-lattice arrays and
  // the hop factor times fm[k].
  template <int MU, bool BACK, int K>
  __device__ __forceinline__ static void hop_eo(const OpArgs& a, const S* __restrict__ in0,
                                                size_t rstride, const Coord& c, int i, int h,
                                                unsigned act, const R fm[K], C acc[K][12]) {
    constexpr int s = DAG ? -1 : 1;
    constexpr int TT = BACK ? s : -s;
    const Geom& g = a.g;
    bool wrap;
    const int jh = (BACK ? nb_bwd(g, c, i, MU, wrap) : nb_fwd(g, c, i, MU, wrap)) >> 1;
    const bool flip = wrap && g.bc[MU] < 0;
    C lk[9];
    using LP = typename LinkPol<P, NL>::type;
    load_link<LP, NL, true>((const typename LP::S*)(BACK ? a.links_nb : a.links), g.Vp, MU,
                            BACK ? jh : h, lk);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!((act >> k) & 1)) continue;
      R sc;
      C hh[2][3];
      if constexpr (P::kSiteScale) {
        W::template project_q16<MU, TT>(in0 + k * rstride, g.Vp, jh, hh, sc);
      } else {
        C psi[12];
        ld_site_raw<P, 12>(in0 + k * rstride, g.Vp, jh, psi, sc);
        W::template project<MU, TT>(psi, hh);
      }
      W::template accumulate<MU, TT, BACK>(lk, hh, W::template hop_factor<LP>(sc, flip) * fm[k],
                                           acc[k]);
    }
  }

  template <int K>
  __device__ __forceinline__ static void site_multi(const OpArgs& a, const S* __restrict__ in0,
                                                    size_t rstride, int h, int k0, unsigned act,
                                                    C out[K][12]) {
    const Geom& g = a.g;
    int i;
    const Coord c = coords_of(g, h, a.eo_par, i);
    // acc = -2 out: starts at -2 c y (Schur forms) or 0, and the hops enter
    // with factor -1/d (Schur forms) or 1
    C acc[K][12];
    R fm[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double d = rhs_mass(a, k0 + k) + 4.0;
      fm[k] = (a.eo_schur >= 1 && a.eo_schur <= 3) ? (R)(-1.0 / d) : (R)1;
      C v[12];
      R sc = (R)0;
      const bool diag = a.eo_schur && ((act >> k) & 1);
      if (diag) ld_site_raw<P, 12>((const S*)a.diag_in + (size_t)(k0 + k) * rstride, g.Vp, h, v, sc);
      const double cd = (a.eo_schur == 1 || a.eo_schur == 4) ? d : a.eo_schur == 2 ? 1.0 : 1.0 / d;
      const R coef = (R)(-2.0 * cd) * sc;
#pragma unroll
      for (int q = 0; q < 12; ++q) acc[k][q] = diag ? cscale(v[q], coef) : czero<C>();
    }
    if constexpr (W::template kStraight<K>()) {
      hop_eo<0, false, K>(a, in0, rstride, c, i, h, act, fm, acc);
      __builtin_amdgcn_sched_barrier(0);
      hop_eo<0, true, K>(a, in0, rstride, c, i, h, act, fm, acc);
      __builtin_amdgcn_sched_barrier(0);
      hop_eo<1, false, K>(a, in0, rstride, c, i, h, act, fm, acc);
      __builtin_amdgcn_sched_barrier(0);
      hop_eo<1, true, K>(a, in0, rstride, c, i, h, act, fm, acc);
      __builtin_amdgcn_sched_barrier(0);
      hop_eo<2, false, K>(a, in0, rstride, c, i, h, act, fm, acc);
      __builtin_amdgcn_sched_barrier(0);
      hop_eo<2, true, K>(a, in0, rstride, c, i, h, act, fm, acc);
      __builtin_amdgcn_sched_barrier(0);
      hop_eo<3, false, K>(a, in0, rstride, c, i, h, act, fm, acc);
      __builtin_amdgcn_sched_barrier(0);
      hop_eo<3, true, K>(a, in0, rstride, c, i, h, act, fm, acc);
    } else if constexpr (W::template kHopPairs<K>()) {
#pragma unroll 1
      for (int m0 = 0; m0 < 4; ++m0) {
        int mu = m0;
        asm volatile("" : "+s"(mu));
        switch (mu) {
          case 0: hop_eo<0, false, K>(a, in0, rstride, c, i, h, act, fm, acc);
                  hop_eo<0, true, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
          case 1: hop_eo<1, false, K>(a, in0, rstride, c, i, h, act, fm, acc);
                  hop_eo<1, true, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
          case 2: hop_eo<2, false, K>(a, in0, rstride, c, i, h, act, fm, acc);
                  hop_eo<2, true, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
          default: hop_eo<3, false, K>(a, in0, rstride, c, i, h, act, fm, acc);
                   hop_eo<3, true, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
        }
      }
    } else {
#pragma unroll 1
      for (int h0 = 0; h0 < 8; ++h0) {
        int hp = h0;
        asm volatile("" : "+s"(hp));
        switch (hp) {
          case 0: hop_eo<0, false, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
          case 1: hop_eo<0, true, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
          case 2: hop_eo<1, false, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
          case 3: hop_eo<1, true, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
          case 4: hop_eo<2, false, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
          case 5: hop_eo<2, true, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
          case 6: hop_eo<3, false, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
          default: hop_eo<3, true, K>(a, in0, rstride, c, i, h, act, fm, acc); break;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < 12; ++q) out[k][q] = cscale(acc[k][q], (R)-0.5);
  }
};

// Wilson with r != 1 (no spin projection); only FP64 is instantiated.
template <class P, int NL, bool DAG>
struct WilsonOpR : WilsonOp<P, NL, DAG, true> {};
template <class P, int NL, bool DAG>
struct WilsonOpR1 : WilsonOp<P, NL, DAG, false> {};

// ------------------------------------------------------- staggered Wilson
// M = D_st + r (1 - Gamma_55) + m, M^dag = -D_st + r (1 - Gamma_55) + m.
// D_st psi(x) = 1/2 sum_mu eta_mu(x) [U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu)].
// acc[k] = sum_mu eta_mu [U_mu(x) psi_k(x+mu) - U_mu(x-mu)^dag psi_k(x-mu)] for the
// K inputs psi_k = in0 + k*rstride selected by `act`; each link loaded once.
template <class P, int NL, int K>
__device__ __forceinline__ void dst_site(const OpArgs& a, const typename P::S* __restrict__ in0,
                                         size_t rstride, const Coord& c, int i, unsigned act,
                                         typename P::C acc[K][3]) {
  using C = typename P::C;
  using R = typename P::R;
  using S = typename P::S;
  const Geom& g = a.g;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[k][q] = czero<C>();
#pragma unroll 1
  for (int h = 0; h < 8; ++h) {
    const int mu = h >> 1;
    const bool back = h & 1;
    const R eta = (R)eta_sign(c, mu);
    bool wrap;
    const int j = back ? nb_bwd(g, c, i, mu, wrap) : nb_fwd(g, c, i, mu, wrap);
    // forward hops enter with +eta, backward hops with -eta
    const R sg = ((wrap && g.bc[mu] < 0) ? (R)-1 : (R)1) * (back ? -eta : eta);
    C lk[9];
    using LP = typename LinkPol<P, NL>::type;
    load_link<LP, NL, true>((const typename LP::S*)a.links, g.Vp, mu, back ? j : i, lk);
    const R sgl = sg * (R)LP::kRawScale;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!((act >> k) & 1)) continue;
      C v[3], y[3];
      R sc;
      ld_site_raw<P, 3>(in0 + k * rstride, g.Vp, j, v, sc);
      if (back) mvd(lk, v, y); else mv(lk, v, y);
      const R f = sgl * sc;
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[k][q] = cadd(acc[k][q], cscale(y[q], f));
    }
  }
}

// Site index and boundary sign of x + s for a diagonal offset s in {+-1}^4.
__device__ __forceinline__ int diag_nb(const Geom& g, const Coord& c, const int s[4], int& sign) {
  int j = 0;
  sign = 1;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    int y = c.x[mu] + s[mu];
    if (y < 0) { y += g.L[mu]; sign *= g.bc[mu]; }
    else if (y >= g.L[mu]) { y -= g.L[mu]; sign *= g.bc[mu]; }
    j += y * g.stride[mu];
  }
  return j;
}

// Corner form (K4): Gamma_55 psi(x) = phi(x) (1/16) sum_s W_s(x) psi(x+s).
// Stored: W_s for s = (s1, s2, s3, +1), index cidx = bits (s1<0, s2<0, s3<0);
// the s4 = -1 corners are W_{-s}(x) = W_s(x - s)^dag.
template <class P, int NL, bool DAG>
struct SWCornerOp {
  using Pol = P;
  static constexpr int NC = 3;
  static constexpr int kWaves = 4;
  using C = typename P::C;
  using R = typename P::R;
  using S = typename P::S;

  template <int K>
  __device__ __forceinline__ static void site_multi(const OpArgs& a, const S* __restrict__ in0,
                                                    size_t rstride, int i, int k0, unsigned act,
                                                    C out[K][3]) {
    const Geom& g = a.g;
    Coord c = site_coords(g, i);
    C d[K][3];
    dst_site<P, NL, K>(a, in0, rstride, c, i, act, d);
    C acc[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < 3; ++q) acc[k][q] = czero<C>();
    using CP = typename CornerPol<P>::type;
    const typename CP::S* W = (const typename CP::S*)a.corners;
#pragma unroll 1
    for (int h = 0; h < 16; ++h) {
      // h = 2*cidx + reflected: forward corner W_s(x) psi(x + s), or the
      // reflected one W_{-s}(x) psi(x - s) = W_s(x - s)^dag psi(x - s)
      const int cidx = h >> 1;
      const bool refl = h & 1;
      const int sg4 = refl ? -1 : 1;
      int s[4] = {(cidx & 1) ? -sg4 : sg4, (cidx & 2) ? -sg4 : sg4, (cidx & 4) ? -sg4 : sg4, sg4};
      int sign;
      const int j = diag_nb(g, c, s, sign);
      C w[9];
      load_corner<CP, true>(W, g.Vp, cidx, refl ? j : i, w);   // raw: scale joins below
      const R sgc = (R)sign * (R)CP::kRawScale;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!((act >> k) & 1)) continue;
        C v[3], y[3];
        R sc;
        ld_site_raw<P, 3>(in0 + k * rstride, g.Vp, j, v, sc);
        if (refl) mvd(w, v, y); else mv(w, v, y);
        const R f = sgc * sc;
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[k][q] = cadd(acc[k][q], cscale(y[q], f));
      }
    }
    const R gcoef = (R)(a.r * phi_sign(c) / 16.0);
    const R dcoef = DAG ? (R)-0.5 : (R)0.5;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R mr = (R)(rhs_mass(a, k0 + k) + a.r);
      C v[3] = {czero<C>(), czero<C>(), czero<C>()};
      if ((act >> k) & 1) ld_site<P, 3>(in0 + k * rstride, g.Vp, i, v);
#pragma unroll
      for (int q = 0; q < 3; ++q)
        out[k][q] = csub(cadd(cscale(v[q], mr), cscale(d[k][q], dcoef)), cscale(acc[k][q], gcoef));
    }
  }
};

// On-the-fly form (K2): the subset recursion of the symmetrised product,
//   F_{} = psi,   F_S = sum_{mu in S} C_mu F_{S\mu},   Gamma_55 psi = phi F_{1234} / 24,
// with C_mu = (V_mu + V_mu^dag)/2 (Sec. 2; the 24 orderings of C_1 C_2 C_3 C_4
// are exactly the words that take one direction out of S at a time).  Every
// F_S is a field on the whole lattice, so the recursion costs 4 + 6*2 + 4*3 +
// 4 = 32 applications of some C_mu per site, each a nearest-neighbour hop:
// level L (|S| = L) reads level L-1 at x +- mu only (halo depth 1).  Levels 1
// to 3 are separate launches (g55_level_kernel) into intermediate fields in
// the caller's workspace; level 4 is computed inside the operator below,
// beside D_st and the diagonal.  The fields are kept unnormalised
// (V + V^dag at every level), so F_{1234} carries 2^4 and the last step
// multiplies by phi / (24 * 16).
//
// Intermediate fields: FP64 for FP64 operators, FP32 for the FP32 and 16-bit
// ones (three complex numbers per site, the staggered Wilson vector record).
// Per system 14 fields: index mu (|S| = 1), 4 + pair index (|S| = 2, pairs
// 01 02 03 12 13 23), 10 + the missing direction (|S| = 3).
template <class P> struct G55Pol { using type = F32; };
template <> struct G55Pol<F64> { using type = F64; };
constexpr int kG55Fields = 14;
__host__ __device__ constexpr int g55_field(int mask) {
  // mask: bit mu set for mu in S, 1 <= |S| <= 3
  return __builtin_popcount(mask) == 1   ? __builtin_ctz(mask)
         : __builtin_popcount(mask) == 3 ? 10 + __builtin_ctz(15 ^ mask)
         : mask == 3 ? 4 : mask == 5 ? 5 : mask == 9 ? 6 : mask == 6 ? 7 : mask == 10 ? 8 : 9;
}
template <class P>
__device__ __forceinline__ const typename G55Pol<P>::type::S* g55_in(const OpArgs& a, int k,
                                                                   int field) {
  using PC = typename G55Pol<P>::type;
  const char* base = (const char*)a.g55w + (size_t)k * a.g55_sys;
  return (const typename PC::S*)(base + (size_t)field * field_planes<PC>(3) * a.g.Vp *
                                            sizeof(typename PC::S));
}

template <class P, int NL, bool DAG>
struct SWOtfOp {
  using Pol = P;
  static constexpr int NC = 3;
  static constexpr int kWaves = P::id == 0 ? 3 : 4;
  using C = typename P::C;
  using R = typename P::R;
  using S = typename P::S;

  // acc[k] += sum_mu [U_mu(x) F_{S_mu}(x + mu) + U_mu(x - mu)^dag F_{S_mu}(x - mu)],
  // S_mu = the three directions other than mu: the last level of the
  // recursion from the third-level fields of system k0 + k
  template <int K>
  __device__ __forceinline__ static void level4(const OpArgs& a, const Coord& c, int i, int k0,
                                                unsigned act, C acc[K][3]) {
    using PC = typename G55Pol<P>::type;
    using LP = typename LinkPol<P, NL>::type;
    const Geom& g = a.g;
#pragma unroll 1
    for (int h = 0; h < 8; ++h) {
      const int mu = h >> 1;
      const bool back = h & 1;
      bool wrap;
      const int j = back ? nb_bwd(g, c, i, mu, wrap) : nb_fwd(g, c, i, mu, wrap);
      const R sg = ((wrap && g.bc[mu] < 0) ? (R)-1 : (R)1) * (R)LP::kRawScale;
      C lk[9];
      load_link<LP, NL, true>((const typename LP::S*)a.links, g.Vp, mu, back ? j : i, lk);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!((act >> k) & 1)) continue;
        C v[3], y[3];
        ld_site<PC, 3>(g55_in<P>(a, k0 + k, 10 + mu), g.Vp, j, v);
        if (back) mvd(lk, v, y); else mv(lk, v, y);
#pragma unroll
        for (int q = 0; q < 3; ++q) acc[k][q] = cfmas(y[q], sg, acc[k][q]);
      }
    }
  }

  template <int K>
  __device__ __forceinline__ static void site_multi(const OpArgs& a, const S* __restrict__ in0,
                                                    size_t rstride, int i, int k0, unsigned act,
                                                    C out[K][3]) {
    const Geom& g = a.g;
    Coord c = site_coords(g, i);
    C d[K][3], f[K][3];
    dst_site<P, NL, K>(a, in0, rstride, c, i, act, d);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < 3; ++q) f[k][q] = czero<C>();
    level4<K>(a, c, i, k0, act, f);
    // phi/24 * (1/2)^4 from the four unnormalised C_mu levels
    const R gcoef = (R)(a.r * phi_sign(c) / (24.0 * 16.0));
    const R dcoef = DAG ? (R)-0.5 : (R)0.5;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const R mr = (R)(rhs_mass(a, k0 + k) + a.r);
      C v[3] = {czero<C>(), czero<C>(), czero<C>()};
      if ((act >> k) & 1) ld_site<P, 3>(in0 + k * rstride, g.Vp, i, v);
#pragma unroll
      for (int q = 0; q < 3; ++q)
        out[k][q] = csub(cadd(cscale(v[q], mr), cscale(d[k][q], dcoef)), cscale(f[k][q], gcoef));
    }
  }
};

}  // namespace lq
