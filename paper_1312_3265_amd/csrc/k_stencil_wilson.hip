// Stencil kernel instantiations for WilsonOp.
#include "stencil_dispatch.h"

namespace lq {
void launch_stencil_wilson_lanes(int prec, int nl, bool dag, int epi, const OpArgs& oa,
                                 const void* in, const EpiArgs& ea, int nrhs, hipStream_t s);

void launch_stencil_wilson(int prec, int nl, bool dag, int epi, const OpArgs& oa, const void* in,
          const EpiArgs& ea, int nrhs, hipStream_t s) {
  // rhs_per_thread = 8: four systems across the lanes of a site, link
  // products on the matrix cores (k_stencil_wlanes.hip)
  if (ea.rhs_per_thread == 8)
    return launch_stencil_wilson_lanes(prec, nl, dag, epi, oa, in, ea, nrhs, s);
  if (oa.r == 1.0) return dispatch_prec<WilsonOpR1>(prec, nl, dag, epi, oa, in, ea, nrhs, s);
  if (prec != P64)
    throw std::runtime_error("Wilson stencil with r != 1 is built for FP64 only");
  dispatch_epi<WilsonOpR, F64, 18>(dag, epi, oa, in, ea, nrhs, s);
}
}  // namespace lq
