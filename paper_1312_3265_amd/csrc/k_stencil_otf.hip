// Staggered Wilson with Gamma_55 applied on the fly (K2): the first three
// levels of the subset recursion F_S = sum_{mu in S} C_mu F_{S\mu} (one
// launch per level, into the intermediate fields of OpArgs::g55w), then the
// operator's stencil kernel, which takes the last level beside D_st and the
// diagonal (SWOtfOp).  Gamma_55 is hermitian and the same in M and M^dag, so
// the levels do not depend on the dagger.
#include "stencil_dispatch.h"

namespace lq {

// One hop direction MU of level L at site i (coordinates c) for system k:
// for every output subset S of size L that contains MU,
//   acc_S += f_+ U_MU(x) F_{S\MU}(x + MU) + f_- U_MU(x - MU)^dag F_{S\MU}(x - MU)
// (unnormalised C_MU; f_+- the boundary signs times the storage scales), the
// forward half (BACK = false) and the backward half in turn.
// Level 1 reads the operator's input psi (any storage) into the single
// accumulator of F_MU; levels 2 and 3 read the intermediate fields, acc[q]
// accumulating the q-th subset of the level (bit masks below).
template <class P, int NL, int L, int MU, bool BACK>
__device__ __forceinline__ void g55_half_hop(const OpArgs& a, const typename P::S* __restrict__ in,
                                             int k, const Coord& c, int i,
                                             typename P::C acc[][3]) {
  using C = typename P::C;
  using R = typename P::R;
  using PC = typename G55Pol<P>::type;
  using LP = typename LinkPol<P, NL>::type;
  constexpr int NOUT = L == 1 ? 1 : L == 2 ? 6 : 4;
  const Geom& g = a.g;
  bool wrap;
  const int j = BACK ? nb_bwd(g, c, i, MU, wrap) : nb_fwd(g, c, i, MU, wrap);
  const R sgn = (wrap && g.bc[MU] < 0) ? (R)-1 : (R)1;
  C lk[9];
  load_link<LP, NL, true>((const typename LP::S*)a.links, g.Vp, MU, BACK ? j : i, lk);
#pragma unroll
  for (int q = 0; q < NOUT; ++q) {
    // the q-th subset of size L, as a bit mask (compile-time after unrolling)
    const int S = L == 1 ? (1 << MU)
                : L == 2 ? (q == 0 ? 3 : q == 1 ? 5 : q == 2 ? 9 : q == 3 ? 6 : q == 4 ? 10 : 12)
                         : (15 ^ (1 << q));
    if (!((S >> MU) & 1)) continue;
    C v[3], y[3];
    R f = sgn * (R)LP::kRawScale;
    if constexpr (L == 1) {
      R sc;
      ld_site_raw<P, 3>(in, g.Vp, j, v, sc);
      f *= sc;
    } else {
      ld_site<PC, 3>(g55_in<P>(a, k, g55_field(S ^ (1 << MU))), g.Vp, j, v);
    }
    if (BACK) mvd(lk, v, y); else mv(lk, v, y);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) acc[q][cc] = cfmas(y[cc], f, acc[q][cc]);
  }
}

template <class P, int NL, int L, int MU>
__device__ __forceinline__ void g55_hop(const OpArgs& a, const typename P::S* __restrict__ in,
                                        int k, const Coord& c, int i, typename P::C acc[][3]) {
  g55_half_hop<P, NL, L, MU, false>(a, in, k, c, i, acc);
  // keep the backward hop's loads behind the forward hop's arithmetic: with
  // both links and inputs in flight at once the FP64 levels spill
  __builtin_amdgcn_sched_barrier(0);
  g55_half_hop<P, NL, L, MU, true>(a, in, k, c, i, acc);
}

// Level L of the recursion for every site of the site blocks and every
// selected system (the systems the stencil launch that follows computes).
// FP64 level 2 holds six accumulators of three complex doubles (72 VGPRs):
// it runs at two waves per SIMD rather than spill.
template <class P, int L>
constexpr int g55_waves() { return P::id != 0 ? 4 : (L == 2 ? 2 : 3); }

template <class P, int NL, int L>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(g55_waves<P, L>(), 8)))
g55_level_kernel(const OpArgs oa, const typename P::S* __restrict__ in, const EpiArgs ea,
                 int nrhs) {
  using C = typename P::C;
  using PC = typename G55Pol<P>::type;
  constexpr int NOUT = L == 1 ? 1 : L == 2 ? 6 : 4;
  int sb, kl;
  map_block(ea.nbp, nrhs, 1, sb, kl);
  const int k = ea.k0 + kl;
  if (ea.st && !slot_active(ea.st, k, ea.state_mode, ea.par, ea.ru_mask)) return;
  const Geom& g = oa.g;
  const int i = sb * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const Coord c = site_coords(g, i);
  const typename P::S* psi = in + (size_t)k * field_planes<P>(3) * g.Vp;
  char* base = (char*)oa.g55w + (size_t)k * oa.g55_sys;
  const size_t fbytes = (size_t)field_planes<PC>(3) * g.Vp * sizeof(typename PC::S);
  C acc[NOUT][3];
#pragma unroll
  for (int q = 0; q < NOUT; ++q)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) acc[q][cc] = czero<C>();
  // one direction per iteration, kept rolled (only one link and one input
  // record live at a time)
#pragma unroll 1
  for (int m0 = 0; m0 < 4; ++m0) {
    int mu = m0;
    asm volatile("" : "+s"(mu));
    switch (mu) {
      case 0: g55_hop<P, NL, L, 0>(oa, psi, k, c, i, acc); break;
      case 1: g55_hop<P, NL, L, 1>(oa, psi, k, c, i, acc); break;
      case 2: g55_hop<P, NL, L, 2>(oa, psi, k, c, i, acc); break;
      default: g55_hop<P, NL, L, 3>(oa, psi, k, c, i, acc); break;
    }
    if constexpr (L == 1) {
      // F_mu is complete after direction mu: store it now and keep the
      // accumulator free (the four would otherwise stay live to the end)
      typename PC::C o[3];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        o[cc].x = acc[0][cc].x; o[cc].y = acc[0][cc].y;
        acc[0][cc] = czero<C>();
      }
      st_site<PC, 3>((typename PC::S*)(base + (size_t)mu * fbytes), g.Vp, i, o);
    }
  }
  if constexpr (L == 1) return;
#pragma unroll
  for (int q = 0; q < NOUT; ++q) {
    const int S = L == 1 ? (1 << q)
                : L == 2 ? (q == 0 ? 3 : q == 1 ? 5 : q == 2 ? 9 : q == 3 ? 6 : q == 4 ? 10 : 12)
                         : (15 ^ (1 << q));
    typename PC::C o[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) { o[cc].x = acc[q][cc].x; o[cc].y = acc[q][cc].y; }
    st_site<PC, 3>((typename PC::S*)(base + (size_t)g55_field(S) * fbytes), g.Vp, i, o);
  }
}

template <class P, int NL>
static void launch_levels(const OpArgs& oa, const void* in, const EpiArgs& ea, int nrhs,
                          hipStream_t s) {
  const int grid = ea.nbp * nrhs;
  if (grid == 0) return;
  const auto* x = (const typename P::S*)in;
  hipLaunchKernelGGL((g55_level_kernel<P, NL, 1>), dim3(grid), dim3(kBlock), 0, s, oa, x, ea, nrhs);
  hipLaunchKernelGGL((g55_level_kernel<P, NL, 2>), dim3(grid), dim3(kBlock), 0, s, oa, x, ea, nrhs);
  hipLaunchKernelGGL((g55_level_kernel<P, NL, 3>), dim3(grid), dim3(kBlock), 0, s, oa, x, ea, nrhs);
}

void launch_stencil_otf(int prec, int nl, bool dag, int epi, const OpArgs& oa, const void* in,
                        const EpiArgs& ea, int nrhs, hipStream_t s) {
  if (!oa.g55w || !oa.g55_sys)
    throw std::runtime_error("on-the-fly Gamma_55 needs its intermediate fields (g55w)");
  if (prec == P64 && nl == 18) launch_levels<F64, 18>(oa, in, ea, nrhs, s);
  else if (prec == P64 && nl == 12) launch_levels<F64, 12>(oa, in, ea, nrhs, s);
  else if (prec == P32 && nl == 18) launch_levels<F32, 18>(oa, in, ea, nrhs, s);
  else if (prec == P32 && nl == 12) launch_levels<F32, 12>(oa, in, ea, nrhs, s);
  else if (prec == P16 && nl == 12) launch_levels<Q16, 12>(oa, in, ea, nrhs, s);
  else if (prec == P16 && nl == 18) launch_levels<Q16, 18>(oa, in, ea, nrhs, s);
  else throw std::runtime_error("on-the-fly Gamma_55: unsupported precision/links");
  dispatch_prec<SWOtfOp>(prec, nl, dag, epi, oa, in, ea, nrhs, s);
}

// Bytes of the intermediate fields of one system (precision prec).
size_t g55_bytes_per_system(const Geom& g, int prec) {
  const size_t el = prec == P64 ? 16 : 8;
  return (size_t)kG55Fields * 3 * g.Vp * el;
}

}  // namespace lq
