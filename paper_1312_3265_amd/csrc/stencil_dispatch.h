// Instantiates the stencil kernels of one operator family for the supported
// (precision, link storage, dagger, epilogue) combinations and launches them.
//   FP64: 18-real links; every epilogue, both M and M^dag.
//   FP32: 18- or 12-real links; STORE, STORE_NORM (M), CG_UPDATE (M^dag).
//   Q16 (16-bit fixed point): 16-bit 12-real or FP32 18-real links; same
//   epilogues as FP32.
#pragma once

#include <stdexcept>
#include <string>

#include "kernels.h"
#include "stencil.h"

namespace lq {

// Systems per thread (K) for the low-precision CG kernels; 1 elsewhere.
// The low-precision CG_UPDATE kernels come in two cache policies (ea.stream).
template <template <class, int, bool> class OpT, class P, int NL, bool DAG, int EPI, int K>
static void launch_k(const OpArgs& oa, const void* in, const EpiArgs& ea, int nrhs,
                     hipStream_t s) {
  using Op = OpT<P, NL, DAG>;
  const int ngroups = (nrhs + K - 1) / K;
  const int grid = ea.nbp * ngroups;
  if (grid == 0) return;
  if constexpr (EPI == EPI_CG_UPDATE && P::id != 0) {
    if (ea.stream) {
      hipLaunchKernelGGL((stencil_kernel<Op, EPI, K, kStream>), dim3(grid), dim3(kBlock), 0, s,
                         oa, (const typename Op::S*)in, ea, ngroups, nrhs);
      return;
    }
  }
  hipLaunchKernelGGL((stencil_kernel<Op, EPI, K, 0>), dim3(grid), dim3(kBlock), 0, s, oa,
                     (const typename Op::S*)in, ea, ngroups, nrhs);
}

template <template <class, int, bool> class OpT, class P, int NL, bool DAG, int EPI>
static void launch_one(const OpArgs& oa, const void* in, const EpiArgs& ea, int nrhs,
                       hipStream_t s) {
  constexpr bool multi = (P::id != 0) && (EPI == EPI_STORE_NORM || EPI == EPI_CG_UPDATE ||
                                          EPI == EPI_STORE);
  const int K = multi ? ea.rhs_per_thread : 1;
  if constexpr (multi) {
    if (K == 2) return launch_k<OpT, P, NL, DAG, EPI, 2>(oa, in, ea, nrhs, s);
    if (K == 4) return launch_k<OpT, P, NL, DAG, EPI, 4>(oa, in, ea, nrhs, s);
  }
  if (K != 1 && K != 0)
    throw std::runtime_error("stencil: unsupported systems per thread " + std::to_string(K));
  launch_k<OpT, P, NL, DAG, EPI, 1>(oa, in, ea, nrhs, s);
}

template <template <class, int, bool> class OpT, class P, int NL>
static void dispatch_epi(bool dag, int epi, const OpArgs& oa, const void* in, const EpiArgs& ea,
                         int nrhs, hipStream_t s) {
  constexpr bool full = (P::id == 0);
  if (!dag) {
    switch (epi) {
      case EPI_STORE: return launch_one<OpT, P, NL, false, EPI_STORE>(oa, in, ea, nrhs, s);
      case EPI_STORE_NORM: return launch_one<OpT, P, NL, false, EPI_STORE_NORM>(oa, in, ea, nrhs, s);
      default: break;
    }
    if constexpr (full) {
      if (epi == EPI_RESID) return launch_one<OpT, P, NL, false, EPI_RESID>(oa, in, ea, nrhs, s);
    }
  } else {
    switch (epi) {
      case EPI_STORE: return launch_one<OpT, P, NL, true, EPI_STORE>(oa, in, ea, nrhs, s);
      case EPI_CG_UPDATE: return launch_one<OpT, P, NL, true, EPI_CG_UPDATE>(oa, in, ea, nrhs, s);
      default: break;
    }
    if constexpr (full) {
      switch (epi) {
        case EPI_STORE_NORM: return launch_one<OpT, P, NL, true, EPI_STORE_NORM>(oa, in, ea, nrhs, s);
        case EPI_RESID: return launch_one<OpT, P, NL, true, EPI_RESID>(oa, in, ea, nrhs, s);
        case EPI_LANCZOS: return launch_one<OpT, P, NL, true, EPI_LANCZOS>(oa, in, ea, nrhs, s);
        default: break;
      }
    }
  }
  throw std::runtime_error("stencil: unsupported epilogue " + std::to_string(epi) +
                           " for precision " + std::to_string(P::id));
}

template <template <class, int, bool> class OpT>
static void dispatch_prec(int prec, int nl, bool dag, int epi, const OpArgs& oa, const void* in,
                          const EpiArgs& ea, int nrhs, hipStream_t s) {
  if (prec == P64 && nl == 18) return dispatch_epi<OpT, F64, 18>(dag, epi, oa, in, ea, nrhs, s);
  if (prec == P64 && nl == 12) return dispatch_epi<OpT, F64, 12>(dag, epi, oa, in, ea, nrhs, s);
  if (prec == P32 && nl == 18) return dispatch_epi<OpT, F32, 18>(dag, epi, oa, in, ea, nrhs, s);
  if (prec == P32 && nl == 12) return dispatch_epi<OpT, F32, 12>(dag, epi, oa, in, ea, nrhs, s);
  if (prec == P16 && nl == 12) return dispatch_epi<OpT, Q16, 12>(dag, epi, oa, in, ea, nrhs, s);
  if (prec == P16 && nl == 18) return dispatch_epi<OpT, Q16, 18>(dag, epi, oa, in, ea, nrhs, s);
  throw std::runtime_error("stencil: unsupported precision/link storage " + std::to_string(prec) +
                           "/" + std::to_string(nl));
}

}  // namespace lq
