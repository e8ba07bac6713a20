// Layout kernels: canonical <-> SoA repacking, link compression to 12 reals
// (K6), the staggered Wilson corner matrices (K3) and the mean plaquette.
#include <stdexcept>

#include "kernels.h"
#include "stencil.h"

namespace lq {

// ------------------------------------------------------------ fermions
// Canonical site of field site i: i itself, or for a half-lattice field of
// parity par (EO) the lexicographic site of that parity in the pair (2i, 2i+1).
template <bool EO>
__device__ __forceinline__ size_t canon_site(const Geom& g, int i, int par, int kl) {
  if constexpr (EO) {
    const Coord c = site_coords(g, 2 * i);
    return (size_t)kl * 2 * g.V + 2 * i + ((c.x[1] + c.x[2] + c.x[3] + par) & 1);
  } else {
    return (size_t)kl * g.V + i;
  }
}

template <class P, int NC, bool F64SRC, bool EO>
__global__ void __launch_bounds__(256)
field_in_kernel(const Geom g, const void* __restrict__ canon, typename P::S* __restrict__ soa,
                int par, int nbp, int k0, int nrhs) {
  using C = typename P::C;
  using R = typename P::R;
  int sb, kl;
  map_block(nbp, nrhs, 1, sb, kl);
  const int k = k0 + kl;
  const int i = sb * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const size_t cbase = canon_site<EO>(g, i, par, kl) * NC;
  C v[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    if constexpr (F64SRC) {
      const double2 z = ((const double2*)canon)[cbase + q];
      v[q].x = (R)z.x; v[q].y = (R)z.y;
    } else {
      const float2 z = ((const float2*)canon)[cbase + q];
      v[q].x = (R)z.x; v[q].y = (R)z.y;
    }
  }
  st_site<P, NC>(soa + (size_t)k * field_planes<P>(NC) * g.Vp, g.Vp, i, v);
}

template <class P, int NC, bool F64DST, bool EO>
__global__ void __launch_bounds__(256)
field_out_kernel(const Geom g, const typename P::S* __restrict__ soa, void* __restrict__ canon,
                 int par, int nbp, int k0, int nrhs) {
  using C = typename P::C;
  int sb, kl;
  map_block(nbp, nrhs, 1, sb, kl);
  const int k = k0 + kl;
  const int i = sb * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const size_t cbase = canon_site<EO>(g, i, par, kl) * NC;
  C v[NC];
  ld_site<P, NC>(soa + (size_t)k * field_planes<P>(NC) * g.Vp, g.Vp, i, v);
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    if constexpr (F64DST) ((double2*)canon)[cbase + q] = make_double2(v[q].x, v[q].y);
    else ((float2*)canon)[cbase + q] = make_float2((float)v[q].x, (float)v[q].y);
  }
}

#define LQ_PNC(prec, nc, CALL)                                                        \
  do {                                                                                \
    if (prec == P64 && nc == 12) { using PP = F64; constexpr int NCC = 12; CALL; }    \
    else if (prec == P64 && nc == 3) { using PP = F64; constexpr int NCC = 3; CALL; }  \
    else if (prec == P32 && nc == 12) { using PP = F32; constexpr int NCC = 12; CALL; } \
    else if (prec == P32 && nc == 3) { using PP = F32; constexpr int NCC = 3; CALL; }  \
    else if (prec == P16 && nc == 12) { using PP = Q16; constexpr int NCC = 12; CALL; } \
    else if (prec == P16 && nc == 3) { using PP = Q16; constexpr int NCC = 3; CALL; }  \
    else throw std::runtime_error("unsupported precision/components");                \
  } while (0)

#define LQ_FIELD_LAUNCH(KERNEL, F64FLAG, SRC, DST)                                          \
  do {                                                                                    \
    if (par < 0)                                                                          \
      LQ_PNC(prec, nc, hipLaunchKernelGGL((KERNEL<PP, NCC, F64FLAG, false>),              \
                                          dim3(nbp * nrhs), dim3(kBlock), 0, s, g, SRC, DST, \
                                          par, nbp, k0, nrhs));                           \
    else                                                                                  \
      LQ_PNC(prec, nc, hipLaunchKernelGGL((KERNEL<PP, NCC, F64FLAG, true>),               \
                                          dim3(nbp * nrhs), dim3(kBlock), 0, s, g, SRC, DST, \
                                          par, nbp, k0, nrhs));                           \
  } while (0)

void launch_field_in(int prec, int nc, const Geom& g, const void* canon, int canon_f64, void* soa,
                     int nbp, int k0, int nrhs, hipStream_t s, int par) {
  if (nbp * nrhs == 0) return;
  if (canon_f64) LQ_FIELD_LAUNCH(field_in_kernel, true, canon, (typename PP::S*)soa);
  else LQ_FIELD_LAUNCH(field_in_kernel, false, canon, (typename PP::S*)soa);
}

void launch_field_out(int prec, int nc, const Geom& g, const void* soa, void* canon, int canon_f64,
                      int nbp, int k0, int nrhs, hipStream_t s, int par) {
  if (nbp * nrhs == 0) return;
  if (canon_f64) LQ_FIELD_LAUNCH(field_out_kernel, true, (const typename PP::S*)soa, canon);
  else LQ_FIELD_LAUNCH(field_out_kernel, false, (const typename PP::S*)soa, canon);
}

// --------------------------------------------------------------- links
// sites [i0, i0 + n) of the canonical field; canon points at site i0
__global__ void __launch_bounds__(256)
gauge_in_kernel(const Geom g, const double2* __restrict__ canon, double2* __restrict__ u64, int i0,
                int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int i = i0 + j;
#pragma unroll 4
  for (int q = 0; q < 36; ++q) u64[(size_t)q * g.Vp + i] = canon[(size_t)j * 36 + q];
}

void launch_gauge_in(const Geom& g, const void* canon, double2* u64, int i0, int n,
                     hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gauge_in_kernel, dim3((n + 255) / 256), dim3(256), 0, s, g,
                     (const double2*)canon, u64, i0, n);
}

// FP64 18-real -> precision P with NL reals (12: rows 0 and 1 only)
template <class P, int NL>
__global__ void __launch_bounds__(256)
links_convert_kernel(const Geom g, const double2* __restrict__ u64, typename P::S* __restrict__ dst) {
  using C = typename P::C;
  using R = typename P::R;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  for (int mu = 0; mu < 4; ++mu) {
    C m[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double2 z = u64[(size_t)(mu * 9 + k) * g.Vp + i];
      m[k].x = (R)z.x; m[k].y = (R)z.y;
    }
    store_link<P, NL>(dst, g.Vp, mu, i, m);
  }
}

void launch_links_convert(int prec, int nl, const Geom& g, const double2* u64, void* dst,
                          hipStream_t s) {
  dim3 grid((g.V + 255) / 256), blk(256);
  if (prec == P32 && nl == 18)
    hipLaunchKernelGGL((links_convert_kernel<F32, 18>), grid, blk, 0, s, g, u64, (float2*)dst);
  else if (prec == P32 && nl == 12)
    hipLaunchKernelGGL((links_convert_kernel<F32, 12>), grid, blk, 0, s, g, u64, (float2*)dst);
  else if (prec == P16 && nl == 12)
    hipLaunchKernelGGL((links_convert_kernel<Q16L, 12>), grid, blk, 0, s, g, u64, (short2*)dst);
  else if (prec == P16 && nl == 18)
    hipLaunchKernelGGL((links_convert_kernel<Q16L, 18>), grid, blk, 0, s, g, u64, (short2*)dst);
  else
    throw std::runtime_error("links_convert: unsupported precision/storage");
}

// FP64 18-real links -> per-parity half-lattice records of precision P with
// NL reals (the even-odd blocks): link mu of site i goes to half site i / 2 of
// its parity's array, which starts at dst + par * 4 * NSTORE * Vhp elements.
template <class P, int NL>
__global__ void __launch_bounds__(256)
links_eo_kernel(const Geom g, int Vhp, const double2* __restrict__ u64,
                typename P::S* __restrict__ dst) {
  using C = typename P::C;
  using R = typename P::R;
  constexpr int NSTORE = P::id == 0 ? 9 : NL / 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  const Coord c = site_coords(g, i);
  const int par = (c.x[0] + c.x[1] + c.x[2] + c.x[3]) & 1;
  typename P::S* d = dst + (size_t)par * 4 * NSTORE * Vhp;
  for (int mu = 0; mu < 4; ++mu) {
    C m[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double2 z = u64[(size_t)(mu * 9 + k) * g.Vp + i];
      m[k].x = (R)z.x; m[k].y = (R)z.y;
    }
    store_link<P, P::id == 0 ? 18 : NL>(d, Vhp, mu, i >> 1, m);
  }
}

void launch_links_eo(int prec, int nl, const Geom& g, int Vhp, const double2* u64, void* dst,
                     hipStream_t s) {
  dim3 grid((g.V + 255) / 256), blk(256);
  if (prec == P64)
    hipLaunchKernelGGL((links_eo_kernel<F64, 18>), grid, blk, 0, s, g, Vhp, u64, (double2*)dst);
  else if (prec == P32 && nl == 18)
    hipLaunchKernelGGL((links_eo_kernel<F32, 18>), grid, blk, 0, s, g, Vhp, u64, (float2*)dst);
  else if (prec == P32 && nl == 12)
    hipLaunchKernelGGL((links_eo_kernel<F32, 12>), grid, blk, 0, s, g, Vhp, u64, (float2*)dst);
  else if (prec == P16 && nl == 12)
    hipLaunchKernelGGL((links_eo_kernel<Q16L, 12>), grid, blk, 0, s, g, Vhp, u64, (short2*)dst);
  else if (prec == P16 && nl == 18)
    hipLaunchKernelGGL((links_eo_kernel<Q16L, 18>), grid, blk, 0, s, g, Vhp, u64, (short2*)dst);
  else
    throw std::runtime_error("links_eo: unsupported precision/storage");
}

// ---------------------------------------------------------- corners (K3)
// W_s(x) = (1/24) sum over the 24 orderings of the path products from x to
// x + s taking one link per direction.  With pt(T) = x + sum_{nu in T} s_nu nu
// and P(T) = sum of the products along all orderings of the directions in T,
//   P(T) = sum_{mu in T} P(T \ mu) L(pt(T \ mu), s_mu mu),   P({}) = 1,
// where L(y, +mu) = U_mu(y) and L(y, -mu) = U_mu(y - mu)^dag.  Level 2 is
// rebuilt inside level 3 (40 matrix products per corner, no large live state).
struct M3 { double2 e[9]; };

__device__ __forceinline__ void m3_load(const double2* __restrict__ u, int Vp, int mu, int site,
                                        bool dag, M3& m) {
  if (!dag) {
#pragma unroll
    for (int k = 0; k < 9; ++k) m.e[k] = u[(size_t)(mu * 9 + k) * Vp + site];
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) m.e[a * 3 + b] = cconj(u[(size_t)(mu * 9 + b * 3 + a) * Vp + site]);
  }
}

__device__ __forceinline__ void m3_mul_acc(const M3& a, const M3& b, M3& acc) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = acc.e[i * 3 + j];
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cfma(a.e[i * 3 + k], b.e[k * 3 + j], s);
      acc.e[i * 3 + j] = s;
    }
}

__device__ __forceinline__ void m3_zero(M3& m) {
#pragma unroll
  for (int k = 0; k < 9; ++k) m.e[k] = make_double2(0.0, 0.0);
}

// site index of x + offset (each offset component in {-1, 0, 1}), periodic
__device__ __forceinline__ int offset_site(const Geom& g, const Coord& c, const int o[4]) {
  int j = 0;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    int y = c.x[mu] + o[mu];
    if (y < 0) y += g.L[mu];
    else if (y >= g.L[mu]) y -= g.L[mu];
    j += y * g.stride[mu];
  }
  return j;
}

// link L(pt, s_mu mu) for the point pt = x + sum_{nu in T} s_nu nu
__device__ __forceinline__ void path_link(const Geom& g, const double2* __restrict__ u,
                                          const Coord& c, const int s[4], int T, int mu, M3& m) {
  int o[4];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) o[nu] = ((T >> nu) & 1) ? s[nu] : 0;
  if (s[mu] > 0) {
    m3_load(u, g.Vp, mu, offset_site(g, c, o), false, m);
  } else {
    o[mu] -= 1;
    m3_load(u, g.Vp, mu, offset_site(g, c, o), true, m);
  }
}

__global__ void __launch_bounds__(64)
corners_kernel(const Geom g, const double2* __restrict__ u, double2* __restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int cidx = blockIdx.y;
  if (i >= g.V) return;
  const Coord c = site_coords(g, i);
  const int s[4] = {(cidx & 1) ? -1 : 1, (cidx & 2) ? -1 : 1, (cidx & 4) ? -1 : 1, 1};
  M3 p4;
  m3_zero(p4);
#pragma unroll 1
  for (int mu4 = 0; mu4 < 4; ++mu4) {
    const int T3 = 15 ^ (1 << mu4);
    M3 p3;
    m3_zero(p3);
#pragma unroll 1
    for (int mu3 = 0; mu3 < 4; ++mu3) {
      if (!((T3 >> mu3) & 1)) continue;
      const int T2 = T3 ^ (1 << mu3);
      // P(T2) for T2 = {a, b}: L(x, a) L(x + a, b) + L(x, b) L(x + b, a)
      const int a = __ffs(T2) - 1;
      const int b = __ffs(T2 ^ (1 << a)) - 1;
      M3 p2, l1, l2;
      m3_zero(p2);
      path_link(g, u, c, s, 0, a, l1);
      path_link(g, u, c, s, 1 << a, b, l2);
      m3_mul_acc(l1, l2, p2);
      path_link(g, u, c, s, 0, b, l1);
      path_link(g, u, c, s, 1 << b, a, l2);
      m3_mul_acc(l1, l2, p2);
      path_link(g, u, c, s, T2, mu3, l1);
      m3_mul_acc(p2, l1, p3);
    }
    M3 l;
    path_link(g, u, c, s, T3, mu4, l);
    m3_mul_acc(p3, l, p4);
  }
#pragma unroll
  for (int k = 0; k < 9; ++k)
    w[(size_t)(cidx * 9 + k) * g.Vp + i] = make_double2(p4.e[k].x / 24.0, p4.e[k].y / 24.0);
}

void launch_corners(const Geom& g, const double2* u64, double2* c64, hipStream_t s) {
  hipLaunchKernelGGL(corners_kernel, dim3((g.V + 63) / 64, 8), dim3(64), 0, s, g, u64, c64);
}

template <class P>
__global__ void __launch_bounds__(256)
corners_convert_kernel(const Geom g, const double2* __restrict__ c64, typename P::S* __restrict__ dst) {
  using C = typename P::C;
  using R = typename P::R;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  for (int c = 0; c < 8; ++c) {
    C m[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double2 z = c64[(size_t)(c * 9 + k) * g.Vp + i];
      m[k].x = (R)z.x; m[k].y = (R)z.y;
    }
    store_corner<P>(dst, g.Vp, c, i, m);
  }
}

void launch_corners_convert(int prec, const Geom& g, const double2* c64, void* dst, hipStream_t s) {
  dim3 grid((g.V + 255) / 256), blk(256);
  if (prec == P32)
    hipLaunchKernelGGL(corners_convert_kernel<F32>, grid, blk, 0, s, g, c64, (float2*)dst);
  else if (prec == P16)
    hipLaunchKernelGGL(corners_convert_kernel<Q16L>, grid, blk, 0, s, g, c64, (short2*)dst);
  else
    throw std::runtime_error("corners_convert: unsupported precision");
}

// ------------------------------------------------------------ plaquette
// (1/3) Re tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag summed over mu < nu.
__global__ void __launch_bounds__(256)
plaquette_kernel(const Geom g, const double2* __restrict__ u, double* __restrict__ part) {
  __shared__ double red[16];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < g.V) {
    const Coord c = site_coords(g, i);
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        bool w;
        const int xm = nb_fwd(g, c, i, mu, w);
        const int xn = nb_fwd(g, c, i, nu, w);
        M3 a, b, cc, d, ab, abc;
        m3_load(u, g.Vp, mu, i, false, a);
        m3_load(u, g.Vp, nu, xm, false, b);
        m3_load(u, g.Vp, mu, xn, true, cc);
        m3_load(u, g.Vp, nu, i, true, d);
        m3_zero(ab);
        m3_mul_acc(a, b, ab);
        m3_zero(abc);
        m3_mul_acc(ab, cc, abc);
        double tr = 0.0;
        for (int p = 0; p < 3; ++p)
          for (int k = 0; k < 3; ++k) tr += abc.e[p * 3 + k].x * d.e[k * 3 + p].x - abc.e[p * 3 + k].y * d.e[k * 3 + p].y;
        acc += tr / 3.0;
      }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void plaquette_finish_kernel(const double* __restrict__ part, int n, double V,
                                        double* out) {
  __shared__ double red[16];
  const double s = sum_partials(part, n, red);
  if (threadIdx.x == 0) *out = s / (6.0 * V);
}

void launch_plaquette(const Geom& g, const double2* u64, double* part, int nbp, double* out,
                      hipStream_t s) {
  const int nb = (g.V + 255) / 256;
  (void)nbp;
  hipLaunchKernelGGL(plaquette_kernel, dim3(nb), dim3(256), 0, s, g, u64, part);
  hipLaunchKernelGGL(plaquette_finish_kernel, dim3(1), dim3(64), 0, s, part, nb, (double)g.V, out);
}

// ------------------------------------------------------ SU(3) check
// Largest deviation, over sites and directions, of the stored row 2 from
// conj(row0 x row1): zero up to rounding for SU(3) links, which is what the
// 12-real storage relies on.
__global__ void __launch_bounds__(256)
su3_dev_kernel(const Geom g, const double2* __restrict__ u, double* __restrict__ part) {
  __shared__ double red[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double dev = 0.0;
  if (i < g.V) {
    for (int mu = 0; mu < 4; ++mu) {
      double2 m[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) m[k] = u[(size_t)(mu * 9 + k) * g.Vp + i];
      const double2 r[3] = {cconj(csub(cmul(m[1], m[5]), cmul(m[2], m[4]))),
                            cconj(csub(cmul(m[2], m[3]), cmul(m[0], m[5]))),
                            cconj(csub(cmul(m[0], m[4]), cmul(m[1], m[3])))};
#pragma unroll
      for (int k = 0; k < 3; ++k)
        dev = fmax(dev, fmax(fabs(r[k].x - m[6 + k].x), fabs(r[k].y - m[6 + k].y)));
    }
  }
  for (int off = 32; off >= 1; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dev;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ void max_finish_kernel(const double* __restrict__ part, int n, double* out) {
  double v = 0.0;
  for (int k = threadIdx.x; k < n; k += 64) v = fmax(v, part[k]);
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if (threadIdx.x == 0) *out = v;
}

void launch_su3_deviation(const Geom& g, const double2* u64, double* part, double* out,
                          hipStream_t s) {
  const int nb = (g.V + 255) / 256;
  hipLaunchKernelGGL(su3_dev_kernel, dim3(nb), dim3(256), 0, s, g, u64, part);
  hipLaunchKernelGGL(max_finish_kernel, dim3(1), dim3(64), 0, s, part, nb, out);
}

// ------------------------------------------------------------- filling
__global__ void fill_zero_kernel(uint4* __restrict__ p, size_t n16) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n16;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = make_uint4(0, 0, 0, 0);
}

void launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  // callers pass 16-byte aligned, 16-byte multiple regions
  const size_t n16 = bytes / 16;
  if (n16 == 0) return;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)p, n16);
}

// Deterministic test data for timing: every component of nrhs vector fields
// uniform in [-1, 1) from a counter-based hash of (seed, system, site,
// component) (the 32-bit finaliser of MurmurHash3), stored in the field's
// precision.
__device__ __forceinline__ uint32_t mix32(uint32_t h) {
  h ^= h >> 16; h *= 0x85ebca6bu;
  h ^= h >> 13; h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}
template <class P, int NC>
__global__ void __launch_bounds__(256)
fill_test_kernel(const Geom g, typename P::S* __restrict__ f, int nbp, int nrhs, uint32_t seed) {
  using C = typename P::C;
  using R = typename P::R;
  int sb, k;
  map_block(nbp, nrhs, 1, sb, k);
  const int i = sb * blockDim.x + threadIdx.x;
  if (i >= g.V) return;
  C v[NC];
  uint32_t h = mix32(seed ^ mix32((uint32_t)k * 0x9e3779b9u ^ mix32((uint32_t)i)));
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    h = mix32(h + 0x632be5abu);
    const uint32_t h2 = mix32(h ^ 0x5bd1e995u);
    v[q].x = (R)((int32_t)h * (1.0 / 2147483648.0));
    v[q].y = (R)((int32_t)h2 * (1.0 / 2147483648.0));
  }
  st_site<P, NC>(f + (size_t)k * field_planes<P>(NC) * g.Vp, g.Vp, i, v);
}

void launch_fill_test(int prec, int nc, const Geom& g, void* soa, int nrhs, uint32_t seed,
                      hipStream_t s) {
  const int nbp = nbp_of(g.V);
  if (nbp * nrhs == 0) return;
  LQ_PNC(prec, nc, hipLaunchKernelGGL((fill_test_kernel<PP, NCC>), dim3(nbp * nrhs), dim3(256), 0,
                                      s, g, (typename PP::S*)soa, nbp, nrhs, seed));
}

}  // namespace lq
