// Stencil kernel instantiations for the even-odd Wilson blocks (WilsonEOOp).
#include "stencil_dispatch.h"

namespace lq {
void launch_stencil_wilson_eo(int prec, int nl, bool dag, int epi, const OpArgs& oa, const void* in,
                              const EpiArgs& ea, int nrhs, hipStream_t s) {
  if (oa.r != 1.0) throw std::runtime_error("even-odd Wilson blocks are built for r = 1 only");
  dispatch_prec<WilsonEOOp>(prec, nl, dag, epi, oa, in, ea, nrhs, s);
}
}  // namespace lq
