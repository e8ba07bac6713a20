// Pion correlator of Wilson point-source propagators (Fig. 1(a), Sec. 3):
// C(t) = sum over the spatial sites of time slice t, the propagators of the
// point sources and their 12 components of |G|^2 (the pseudoscalar
// correlator, by gamma_5-hermiticity).  Canonical fields put t outermost, so
// one propagator's time slice is a contiguous run of Vs * 12 complex numbers:
// each of B blocks per slice sums a fixed stretch of it, propagator after
// propagator, in FP64 and in a fixed order; a second kernel adds each slice's
// B partials in order.  The reduction reads every propagator once (HBM-bound).
#include "kernels.h"
#include "stencil.h"

namespace lq {

__global__ void __launch_bounds__(256)
pion_partial_kernel(const double2* __restrict__ props, int nsrc, long long V, long long slice,
                    int B, double* __restrict__ part) {
  __shared__ double red[16];
  const int t = blockIdx.x / B, b = blockIdx.x - t * B;
  const long long per = (slice + B - 1) / B;
  const long long lo = (long long)b * per;
  const long long hi = lo + per < slice ? lo + per : slice;
  double acc = 0.0;
  for (int a = 0; a < nsrc; ++a) {
    const double2* f = props + (size_t)a * V * 12 + (size_t)t * slice;
    for (long long j = lo + threadIdx.x; j < hi; j += blockDim.x) {
      const double2 z = f[j];
      acc += z.x * z.x + z.y * z.y;
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(64)
pion_finish_kernel(const double* __restrict__ part, int B, double* __restrict__ corr) {
  __shared__ double red[16];
  const double s = sum_partials(part + (size_t)blockIdx.x * B, B, red);
  if (threadIdx.x == 0) corr[blockIdx.x] = s;
}

int pion_blocks_per_slice(int L4) { return L4 >= 2048 ? 1 : 2048 / L4; }

void launch_pion_correlator(const Geom& g, int nsrc, const double2* props, double* part,
                            double* corr, hipStream_t s) {
  const int L4 = g.L[3];
  const int B = pion_blocks_per_slice(L4);
  const long long slice = (long long)(g.V / L4) * 12;
  hipLaunchKernelGGL(pion_partial_kernel, dim3(L4 * B), dim3(256), 0, s, props, nsrc,
                     (long long)g.V, slice, B, part);
  hipLaunchKernelGGL(pion_finish_kernel, dim3(L4), dim3(64), 0, s, part, B, corr);
}

}  // namespace lq
