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
// Storage type S of a complex number and compute type C.  Fields of the
// vector policies are read and written a whole site at a time (ld_site /
// st_site below); links and corner matrices element by element (cvt / enc).
struct F64 {
  using S = double2; using C = double2; using R = double;
  static constexpr int id = 0;
  static constexpr bool kSiteScale = false;
  __device__ __forceinline__ static C cvt(S v) { return v; }
  __device__ __forceinline__ static S enc(C v) { return v; }
  __device__ __forceinline__ static C ld(const S* p) { return *p; }
  __device__ __forceinline__ static void st(S* p, C v) { *p = v; }
};
struct F32 {
  using S = float2; using C = float2; using R = float;
  static constexpr int id = 1;
  static constexpr bool kSiteScale = false;
  __device__ __forceinline__ static C cvt(S v) { return v; }
  __device__ __forceinline__ static S enc(C v) { return v; }
  __device__ __forceinline__ static C ld(const S* p) { return *p; }
  __device__ __forceinline__ static void st(S* p, C v) { *p = v; }
};

// 16-bit fixed point.  A complex number is a pair of int16, value = q * s / 32767.
// Vectors (Q16): s is a per-site scale, the largest |re| or |im| over the
// site's components, kept in one extra float plane after the component planes;
// the rounding error is at most 1.5e-5 of the site's largest component.
// Links and corner matrices (Q16L): s = 1, since every entry of an SU(3)
// matrix and of an average of products of SU(3) matrices is at most 1 in
// modulus.  Arithmetic is FP32.
constexpr float kQ16 = 32767.0f;
__device__ __forceinline__ short q16_round(float v) {
  return (short)max(-32767, min(32767, __float2int_rn(v)));
}
struct Q16 {
  using S = short2; using C = float2; using R = float;
  static constexpr int id = 2;
  static constexpr bool kSiteScale = true;
};
struct Q16L {
  using S = short2; using C = float2; using R = float;
  static constexpr int id = 2;
  static constexpr bool kSiteScale = false;
  __device__ __forceinline__ static C cvt(S v) {
    return make_float2((float)v.x * (1.0f / kQ16), (float)v.y * (1.0f / kQ16));
  }
  __device__ __forceinline__ static S enc(C v) {
    short2 q;
    q.x = q16_round(v.x * kQ16);
    q.y = q16_round(v.y * kQ16);
    return q;
  }
};

// Policy of the links and corner matrices used with vectors of policy P.
template <class P> struct LinkPol { using type = P; };
template <> struct LinkPol<Q16> { using type = Q16L; };

// Storage of the solution increment x_lo: FP32 when the Krylov vectors are
// 16-bit.  x_lo is amplified by the operator (errors in it grow by up to
// kappa), so 16-bit rounding there would stall the outer iteration.
template <class P> struct XPol { using type = P; };
template <> struct XPol<Q16> { using type = F32; };

// Planes of one field of NC components (plus the scale plane of Q16).
template <class P> __host__ __device__ constexpr int field_planes(int nc) {
  return nc + (P::kSiteScale ? 1 : 0);
}

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

// One raw 32-bit word of plane q (the Q16 component and scale planes).
__device__ __forceinline__ uint32_t ld_word(const void* __restrict__ base, int Vp, int q, int site) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, -1, kBufferDword3);
  return __builtin_amdgcn_raw_buffer_load_b32(rs, (uint32_t)site * 4u, (uint32_t)q * (uint32_t)Vp * 4u, 0);
}

// All NC components of site i of a vector field f (planes of Vp elements).
template <class P, int NC>
__device__ __forceinline__ void ld_site(const typename P::S* __restrict__ f, int Vp, int i,
                                        typename P::C v[NC]) {
  if constexpr (P::kSiteScale) {
    const float s = __uint_as_float(ld_word(f, Vp, NC, i)) * (1.0f / kQ16);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const short2 w = __builtin_bit_cast(short2, ld_word(f, Vp, q, i));
      v[q] = make_float2((float)w.x * s, (float)w.y * s);
    }
  } else {
#pragma unroll
    for (int q = 0; q < NC; ++q) v[q] = ldq<P>(f, Vp, q, i);
  }
}

// Store site i; returns ||stored value||^2 (the rounded value actually kept).
template <class P, int NC>
__device__ __forceinline__ double st_site(typename P::S* __restrict__ f, int Vp, int i,
                                          const typename P::C v[NC]) {
  double n2 = 0.0;
  if constexpr (P::kSiteScale) {
    float m = 0.0f;
#pragma unroll
    for (int q = 0; q < NC; ++q) m = fmaxf(m, fmaxf(fabsf(v[q].x), fabsf(v[q].y)));
    const float inv = m > 0.0f ? kQ16 / m : 0.0f;
    const float s = m * (1.0f / kQ16);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      short2 w;
      w.x = q16_round(v[q].x * inv);
      w.y = q16_round(v[q].y * inv);
      f[(size_t)q * Vp + i] = w;
      const float a = (float)w.x * s, b = (float)w.y * s;
      n2 += (double)a * a + (double)b * b;
    }
    ((float*)f)[(size_t)NC * Vp + i] = m;
  } else {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      P::st(f + (size_t)q * Vp + i, v[q]);
      n2 += cnorm2(v[q]);
    }
  }
  return n2;
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
