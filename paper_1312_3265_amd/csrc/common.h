// Shared device-side definitions: complex arithmetic, precision policies,
// lattice geometry and the structure-of-arrays (SoA) field layout.
//
// Layout in HBM.  A field is a set of "planes"; plane c holds component c of
// every site, sites in canonical order, with a padded plane stride Vp >= V so
// that the many planes of one kernel do not start on the same HBM channel.
//   fermion field (one RHS):  plane = spin*3 + colour (Wilson, 12 planes) or
//                             colour (staggered Wilson, 3 planes)
//   multi-RHS field:          RHS k occupies planes [k*nplanes, (k+1)*nplanes)
//   links, 18 reals:          plane = (mu*3 + a)*3 + b      (36 planes)
//   links, 12 reals:          plane = (mu*2 + a)*3 + b      (24 planes, rows 0,1)
//   corners (8 stored):       plane = (c*3 + a)*3 + b       (72 planes),
//                             c = bits (s1<0, s2<0, s3<0) of s = (s1,s2,s3,+1)
// Consecutive lanes of a wavefront take consecutive sites, so every load of a
// plane element is a coalesced 64-lane access.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lq {

// ------------------------------------------------------------ complex helpers
template <typename R> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };

template <typename C> __device__ __forceinline__ C cmk(double re, double im) {
  C z; z.x = re; z.y = im; return z;
}
template <typename C> __device__ __forceinline__ C czero() { C z; z.x = 0; z.y = 0; return z; }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C z; z.x = a.x + b.x; z.y = a.y + b.y; return z; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C z; z.x = a.x - b.x; z.y = a.y - b.y; return z; }
template <typename C> __device__ __forceinline__ C cconj(C a) { C z; z.x = a.x; z.y = -a.y; return z; }
// i*a and -i*a
template <typename C> __device__ __forceinline__ C cmuli(C a) { C z; z.x = -a.y; z.y = a.x; return z; }
template <typename C> __device__ __forceinline__ C cmulmi(C a) { C z; z.x = a.y; z.y = -a.x; return z; }
template <typename C, typename R> __device__ __forceinline__ C cscale(C a, R s) { C z; z.x = a.x * s; z.y = a.y * s; return z; }
// acc + a*b
template <typename C> __device__ __forceinline__ C cfma(C a, C b, C acc) {
  C z;
  z.x = acc.x + a.x * b.x - a.y * b.y;
  z.y = acc.y + a.x * b.y + a.y * b.x;
  return z;
}
// acc + conj(a)*b
template <typename C> __device__ __forceinline__ C cfmac(C a, C b, C acc) {
  C z;
  z.x = acc.x + a.x * b.x + a.y * b.y;
  z.y = acc.y + a.x * b.y - a.y * b.x;
  return z;
}
template <typename C> __device__ __forceinline__ C cmul(C a, C b) { return cfma(a, b, czero<C>()); }
template <typename C> __device__ __forceinline__ double cnorm2(C a) { return (double)a.x * a.x + (double)a.y * a.y; }

// ---------------------------------------------------------- precision policy
// Storage type S of a complex number and compute type C.
struct F64 {
  using S = double2; using C = double2; using R = double;
  static constexpr int id = 0;
  __device__ __forceinline__ static C cvt(S v) { return v; }
  __device__ __forceinline__ static C ld(const S* p) { return *p; }
  __device__ __forceinline__ static void st(S* p, C v) { *p = v; }
};
struct F32 {
  using S = float2; using C = float2; using R = float;
  static constexpr int id = 1;
  __device__ __forceinline__ static C cvt(S v) { return v; }
  __device__ __forceinline__ static C ld(const S* p) { return *p; }
  __device__ __forceinline__ static void st(S* p, C v) { *p = v; }
};
struct F16 {
  using S = __half2; using C = float2; using R = float;
  static constexpr int id = 2;
  __device__ __forceinline__ static C cvt(S v) { return __half22float2(v); }
  __device__ __forceinline__ static C ld(const S* p) { return __half22float2(*p); }
  __device__ __forceinline__ static void st(S* p, C v) { *p = __float22half2_rn(v); }
};

// Storage of the solution increment x_lo: FP32 when the Krylov vectors are
// FP16.  x_lo is amplified by the operator (errors in it grow by up to kappa),
// so FP16 rounding there would stall the outer iteration.
template <class P> struct XPol { using type = P; };
template <> struct XPol<F16> { using type = F32; };

// --------------------------------------------------------------- geometry
// Division by a runtime-invariant 32-bit divisor via multiply-high
// (Granlund & Montgomery, PLDI 1994): q = (umulhi(n, m) + n) >> l for n < 2^31.
struct FastDiv {
  uint32_t d, m, l;
  __host__ void init(uint32_t dd) {
    d = dd; l = 0;
    while ((1ull << l) < dd) ++l;
    m = (uint32_t)((((1ull << l) - dd) << 32) / dd + 1);
  }
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    return (__umulhi(n, m) + n) >> l;
  }
};

struct Geom {
  int L[4];
  int stride[4];     // 1, L1, L1*L2, L1*L2*L3
  int V;             // sites
  int Vp;            // padded plane stride (elements)
  int bc[4];         // fermion boundary sign per direction (+1 / -1)
  int has_bc;        // any bc == -1
  FastDiv dv[3];     // divisors L1, L2, L3
};

struct Coord { int x[4]; };

__device__ __forceinline__ Coord site_coords(const Geom& g, int i) {
  Coord c;
  uint32_t q0 = g.dv[0].div((uint32_t)i);
  c.x[0] = i - (int)q0 * g.L[0];
  uint32_t q1 = g.dv[1].div(q0);
  c.x[1] = (int)q0 - (int)q1 * g.L[1];
  uint32_t q2 = g.dv[2].div(q1);
  c.x[2] = (int)q1 - (int)q2 * g.L[2];
  c.x[3] = (int)q2;
  return c;
}

// neighbour x + mu (fwd) or x - mu (bwd); `wrap` is set when the hop crosses
// the lattice boundary (used for the fermion boundary sign).  Branch-free.
__device__ __forceinline__ int nb_fwd(const Geom& g, const Coord& c, int i, int mu, bool& wrap) {
  wrap = (c.x[mu] == g.L[mu] - 1);
  const int d = wrap ? (1 - g.L[mu]) * g.stride[mu] : g.stride[mu];
  return i + d;
}
__device__ __forceinline__ int nb_bwd(const Geom& g, const Coord& c, int i, int mu, bool& wrap) {
  wrap = (c.x[mu] == 0);
  const int d = wrap ? (g.L[mu] - 1) * g.stride[mu] : -g.stride[mu];
  return i + d;
}

// Element `site` of plane q of a SoA array, as a raw buffer load: the array
// base is wavefront-uniform (a buffer descriptor in scalar registers), the
// plane offset q * Vp is a scalar offset and the per-lane part a 32-bit vector
// offset, so no per-load 64-bit address arithmetic is spent.  Every SoA array
// a kernel reads this way is smaller than 4 GiB (checked at lattice creation).
constexpr int kBufferDword3 = 0x00020000;   // raw (untyped) buffer access on CDNA

template <class P>
__device__ __forceinline__ typename P::C ldq(const typename P::S* __restrict__ base, int Vp, int q,
                                             int site) {
  using S = typename P::S;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, -1, kBufferDword3);
  const uint32_t vo = (uint32_t)site * (uint32_t)sizeof(S);
  const uint32_t so = (uint32_t)q * (uint32_t)Vp * (uint32_t)sizeof(S);
  if constexpr (sizeof(S) == 16) {
    return P::cvt(__builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b128(rs, vo, so, 0)));
  } else if constexpr (sizeof(S) == 8) {
    return P::cvt(__builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0)));
  } else {
    return P::cvt(__builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0)));
  }
}

// Staggered phases as +-1: eta_mu = (-1)^(x_1+..+x_{mu-1}), phi = (-1)^(x2+x4).
__device__ __forceinline__ int eta_sign(const Coord& c, int mu) {
  int s = 0;
  for (int nu = 0; nu < mu; ++nu) s += c.x[nu];
  return (s & 1) ? -1 : 1;
}
__device__ __forceinline__ int phi_sign(const Coord& c) { return ((c.x[1] + c.x[3]) & 1) ? -1 : 1; }

// ----------------------------------------------------------------- links
// Load a 3x3 link (row-major) from the SoA link arrays; 12-real storage keeps
// rows 0 and 1 and rebuilds row 2 = conj(row0 x row1), exact for SU(3).
template <class P, int NREAL>
__device__ __forceinline__ void load_link(const typename P::S* __restrict__ u, int Vp, int mu,
                                          int site, typename P::C m[9]) {
  using C = typename P::C;
  if constexpr (NREAL == 18) {
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = ldq<P>(u, Vp, mu * 9 + k, site);
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) m[k] = ldq<P>(u, Vp, mu * 6 + k, site);
    // row2 = conj(row0 x row1)
    C a0 = m[0], a1 = m[1], a2 = m[2], b0 = m[3], b1 = m[4], b2 = m[5];
    m[6] = cconj(csub(cmul(a1, b2), cmul(a2, b1)));
    m[7] = cconj(csub(cmul(a2, b0), cmul(a0, b2)));
    m[8] = cconj(csub(cmul(a0, b1), cmul(a1, b0)));
  }
}

// y = M v and y = M^dag v for a 3x3 matrix and a colour vector
template <typename C>
__device__ __forceinline__ void mv(const C m[9], const C v[3], C y[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) y[a] = cfma(m[a * 3 + 2], v[2], cfma(m[a * 3 + 1], v[1], cmul(m[a * 3], v[0])));
}
template <typename C>
__device__ __forceinline__ void mvd(const C m[9], const C v[3], C y[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
    y[a] = cfmac(m[6 + a], v[2], cfmac(m[3 + a], v[1], cfmac(m[a], v[0], czero<C>())));
}

// ------------------------------------------------------------- reductions
// Wavefront sum (64 lanes) with a fixed butterfly: deterministic.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum of one double per thread, result valid in every thread.
// `red` is LDS of at least blockDim.x/64 doubles.  Fixed order: deterministic.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < nw; ++k) s += red[k];
  return s;
}

// Sum of n partials (one per block of an earlier launch) computed by every
// block in the same fixed order, so every block obtains the identical value.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n, double* red) {
  double v = 0.0;
  if (threadIdx.x < 64)
    for (int k = threadIdx.x; k < n; k += 64) v += part[k];
  v = (threadIdx.x < 64) ? wave_sum(v) : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) red[0] = v;
  __syncthreads();
  double s = red[0];
  __syncthreads();
  return s;
}

}  // namespace lq
