// Stencil kernel instantiations for SWCornerOp.
#include "stencil_dispatch.h"

namespace lq {
void launch_stencil_sw(int prec, int nl, bool dag, int epi, const OpArgs& oa, const void* in,
          const EpiArgs& ea, int nrhs, hipStream_t s) {
  dispatch_prec<SWCornerOp>(prec, nl, dag, epi, oa, in, ea, nrhs, s);
}
}  // namespace lq
