// Stencil kernel instantiations for WilsonOp.
#include <cstdlib>

#include "stencil_dispatch.h"
#include "stencil_tsweep.h"

namespace lq {
void launch_stencil_wilson_lanes(int prec, int nl, bool dag, int epi, const OpArgs& oa,
                                 const void* in, const EpiArgs& ea, int nrhs, hipStream_t s);

template <int NL, bool DAG, int EPI>
static void launch_tsweep(const OpArgs& oa, const void* in, const EpiArgs& ea, int nrhs, int T,
                          hipStream_t s) {
  const Geom& g = oa.g;
  const int per = ((g.L[0] * g.L[1]) >> 8) * g.L[2] * (g.L[3] / T);
  hipLaunchKernelGGL((wilson_tsweep_kernel<NL, DAG, EPI>), dim3(per * nrhs), dim3(256), 0, s, oa,
                     (const double2*)in, ea, T, nrhs);
}

// FP64, r = 1, one system per thread, on lattices tsweep_slices accepts:
// the t-sweeping stencil (stencil_tsweep.h); false where it does not apply.
// LQ_TSWEEP=0 turns it off (the plain stencil_kernel runs instead).
template <int NL>
static bool try_tsweep(bool dag, int epi, const OpArgs& oa, const void* in, const EpiArgs& ea,
                       int nrhs, hipStream_t s) {
  const char* e = std::getenv("LQ_TSWEEP");
  if (e && e[0] == '0') return false;
  static const int ncu = [] {   // initialised once, thread-safe
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      n = 256;
    return n > 0 ? n : 256;
  }();
  const int T = tsweep_slices(oa.g, ncu);
  if (T == 0 || nrhs < 1) return false;
  if (!dag) {
    switch (epi) {
      case EPI_STORE: launch_tsweep<NL, false, EPI_STORE>(oa, in, ea, nrhs, T, s); return true;
      case EPI_STORE_NORM: launch_tsweep<NL, false, EPI_STORE_NORM>(oa, in, ea, nrhs, T, s); return true;
      case EPI_RESID: launch_tsweep<NL, false, EPI_RESID>(oa, in, ea, nrhs, T, s); return true;
      default: return false;
    }
  }
  switch (epi) {
    case EPI_STORE: launch_tsweep<NL, true, EPI_STORE>(oa, in, ea, nrhs, T, s); return true;
    case EPI_STORE_NORM: launch_tsweep<NL, true, EPI_STORE_NORM>(oa, in, ea, nrhs, T, s); return true;
    case EPI_CG_UPDATE: launch_tsweep<NL, true, EPI_CG_UPDATE>(oa, in, ea, nrhs, T, s); return true;
    case EPI_RESID: launch_tsweep<NL, true, EPI_RESID>(oa, in, ea, nrhs, T, s); return true;
    case EPI_LANCZOS: launch_tsweep<NL, true, EPI_LANCZOS>(oa, in, ea, nrhs, T, s); return true;
    default: return false;
  }
}

// Launches the 16-bit t-sweep; false (nothing launched) where fewer than four
// of its blocks fit on a compute unit.  Wrong results were seen in such
// launches: with FP32 storage (three blocks per CU), and with the 16-bit
// kernel's LDS padded to 49 or 60 KB (three or two blocks), in the systems
// whose blocks have indices past the first 256; padded to 33 or 38 KB (four
// blocks) it stayed bitwise exact.  The cause was not found.
template <class P, int NL, bool DAG, int EPI, int CPL, bool XY>
static bool launch_tsweep_lo(const OpArgs& oa, const void* in, const EpiArgs& ea, int nrhs, int T,
                             hipStream_t s) {
  // blocks of this kernel per CU (a function-local static: initialised once,
  // also when several host threads launch at the same time)
  static const int fits = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void*>(&wilson_tsweep_lo_kernel<P, NL, DAG, EPI, CPL, XY>),
            256, 0) != hipSuccess)
      n = 0;
    return n;
  }();
  if (fits < 4) return false;
  const Geom& g = oa.g;
  const int per = ((g.L[0] * g.L[1]) >> 8) * g.L[2] * ((g.L[3] >> 3) / T);
  hipLaunchKernelGGL((wilson_tsweep_lo_kernel<P, NL, DAG, EPI, CPL, XY>), dim3(8 * per * nrhs),
                     dim3(256), 0, s, oa, (const typename P::S*)in, ea, T, nrhs);
  return true;
}

// 16-bit, r = 1, one system per thread, a t-sweep block order
// (ea.window, tsweep_lo_code) on a lattice it applies to: the CG iteration's
// two stencils sweep t (stencil_tsweep.h), bitwise equal to stencil_kernel;
// false (stencil_kernel runs) otherwise.
template <class P, int NL>
static bool try_tsweep_lo(bool dag, int epi, const OpArgs& oa, const void* in, const EpiArgs& ea,
                          int nrhs, hipStream_t s) {
  int T = 0;
  bool xy = false;
  if (nrhs < 1 || !tsweep_lo_code(ea.window, T, xy) || !tsweep_lo_ok(oa.g, T, xy)) return false;
  if (!dag && epi == EPI_STORE_NORM)
    return xy ? launch_tsweep_lo<P, NL, false, EPI_STORE_NORM, 0, true>(oa, in, ea, nrhs, T, s)
              : launch_tsweep_lo<P, NL, false, EPI_STORE_NORM, 0, false>(oa, in, ea, nrhs, T, s);
  if (dag && epi == EPI_CG_UPDATE) {
    if (ea.stream)
      return xy ? launch_tsweep_lo<P, NL, true, EPI_CG_UPDATE, kStream, true>(oa, in, ea, nrhs, T, s)
                : launch_tsweep_lo<P, NL, true, EPI_CG_UPDATE, kStream, false>(oa, in, ea, nrhs, T, s);
    return xy ? launch_tsweep_lo<P, NL, true, EPI_CG_UPDATE, 0, true>(oa, in, ea, nrhs, T, s)
              : launch_tsweep_lo<P, NL, true, EPI_CG_UPDATE, 0, false>(oa, in, ea, nrhs, T, s);
  }
  return false;
}

void launch_stencil_wilson(int prec, int nl, bool dag, int epi, const OpArgs& oa, const void* in,
          const EpiArgs& ea, int nrhs, hipStream_t s) {
  // rhs_per_thread = 8: four systems across the lanes of a site, link
  // products on the matrix cores (k_stencil_wlanes.hip)
  if (ea.rhs_per_thread == 8)
    return launch_stencil_wilson_lanes(prec, nl, dag, epi, oa, in, ea, nrhs, s);
  if (oa.r == 1.0 && prec == P64 && ea.rhs_per_thread <= 1) {
    if (nl == 12 ? try_tsweep<12>(dag, epi, oa, in, ea, nrhs, s)
                 : try_tsweep<18>(dag, epi, oa, in, ea, nrhs, s))
      return;
  }
  // 16-bit storage only: with FP32 storage the kernel fits three blocks per
  // CU and gave wrong results (launch_tsweep_lo), so FP32 keeps stencil_kernel
  if (oa.r == 1.0 && prec == P16 && ea.rhs_per_thread <= 1 && ea.window <= -11) {
    if (nl == 12 ? try_tsweep_lo<Q16, 12>(dag, epi, oa, in, ea, nrhs, s)
                 : try_tsweep_lo<Q16, 18>(dag, epi, oa, in, ea, nrhs, s))
      return;
  }
  if (oa.r == 1.0) return dispatch_prec<WilsonOpR1>(prec, nl, dag, epi, oa, in, ea, nrhs, s);
  if (prec != P64)
    throw std::runtime_error("Wilson stencil with r != 1 is built for FP64 only");
  dispatch_epi<WilsonOpR, F64, 18>(dag, epi, oa, in, ea, nrhs, s);
}
}  // namespace lq
