// Instantiations of the lanes stencil (stencil_lanes.h): the batched r = 1
// Wilson stencils of the FP32 and 16-bit CG with 18-real links, four systems
// across the lanes of each site and the link products on the matrix cores.
#include <stdexcept>
#include <string>

#include "kernels.h"
#include "stencil_lanes.h"

namespace lq {

template <class P, bool DAG, int EPI>
static void launch_lanes(const OpArgs& oa, const void* in, const EpiArgs& ea, int nrhs,
                         hipStream_t s) {
  using Op = WilsonLanesOp<P, 18, DAG>;
  const int ngroups = (nrhs + 3) / 4;
  const int grid = ea.nbp * ngroups;
  if (grid == 0) return;
  const auto* x = (const typename Op::S*)in;
  if constexpr (EPI == EPI_CG_UPDATE) {
    if (ea.stream) {
      hipLaunchKernelGGL((stencil_lanes_kernel<Op, EPI, kStream>), dim3(grid), dim3(kLanesBlock),
                         0, s, oa, x, ea, ngroups, nrhs);
      return;
    }
  }
  hipLaunchKernelGGL((stencil_lanes_kernel<Op, EPI, 0>), dim3(grid), dim3(kLanesBlock), 0, s, oa,
                     x, ea, ngroups, nrhs);
}

template <class P>
static void dispatch_lanes(bool dag, int epi, const OpArgs& oa, const void* in, const EpiArgs& ea,
                           int nrhs, hipStream_t s) {
  if (!dag && epi == EPI_STORE) return launch_lanes<P, false, EPI_STORE>(oa, in, ea, nrhs, s);
  if (!dag && epi == EPI_STORE_NORM) return launch_lanes<P, false, EPI_STORE_NORM>(oa, in, ea, nrhs, s);
  if (dag && epi == EPI_STORE) return launch_lanes<P, true, EPI_STORE>(oa, in, ea, nrhs, s);
  if (dag && epi == EPI_CG_UPDATE) return launch_lanes<P, true, EPI_CG_UPDATE>(oa, in, ea, nrhs, s);
  throw std::runtime_error("lanes stencil: unsupported epilogue " + std::to_string(epi));
}

void launch_stencil_wilson_lanes(int prec, int nl, bool dag, int epi, const OpArgs& oa,
                                 const void* in, const EpiArgs& ea, int nrhs, hipStream_t s) {
  if (oa.r != 1.0 || nl != 18)
    throw std::runtime_error("the lanes stencil is built for r = 1 with 18-real links");
  if (prec == P16) return dispatch_lanes<Q16>(dag, epi, oa, in, ea, nrhs, s);
  if (prec == P32) return dispatch_lanes<F32>(dag, epi, oa, in, ea, nrhs, s);
  throw std::runtime_error("the lanes stencil is built for FP32 and 16-bit storage");
}

}  // namespace lq
