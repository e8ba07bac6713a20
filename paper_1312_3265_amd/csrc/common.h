// Shared device-side definitions: complex arithmetic, precision policies,
// lattice geometry and the structure-of-arrays (SoA) field layout.
//
// Layout in HBM.  Each array holds per-site records (see "site records"
// below) in slabs of 16-byte elements, sites in canonical order, with a padded
// slab stride Vp >= V elements.  Record contents:
//   fermion field (one RHS):  component spin*3 + colour (Wilson, 12) or colour
//                             (staggered Wilson, 3), then the Q16 site scale
//   multi-RHS field:          RHS k is the field at offset k * field_planes * Vp
//   links:                    one record per direction mu, entries (a*3 + b),
//                             a < 3 (18 reals) or a < 2 (12 reals)
//   corners (8 stored):       record c = bits (s1<0, s2<0, s3<0) of
//                             s = (s1,s2,s3,+1), entries (a*3 + b)
// In FP64 a complex number is one 16-byte element, so a record's slab j is
// simply its component j.  Consecutive lanes of a wavefront take consecutive
// sites, so every load is a coalesced 64-lane access.
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
template <typename C> __device__ __forceinline__ C cneg(C a) { C z; z.x = -a.x; z.y = -a.y; return z; }
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
// acc + a*s for a real scalar s
template <typename C, typename R> __device__ __forceinline__ C cfmas(C a, R s, C acc) {
  C z; z.x = acc.x + a.x * s; z.y = acc.y + a.y * s; return z;
}
template <typename C> __device__ __forceinline__ double cnorm2(C a) { return (double)a.x * a.x + (double)a.y * a.y; }

// ---------------------------------------------------------- precision policy
// Storage type S of a complex number and compute type C.  Fields of the
// vector policies are read and written a whole site at a time (ld_site /
// st_site below); links and corner matrices element by element (cvt / enc).
// cvt_raw / kRawScale: a matrix entry decoded without its storage scale, and
// that scale (1 except for the 16-bit matrices), so that a kernel can apply
// the scale once to a product instead of to every entry.
struct F64 {
  using S = double2; using C = double2; using R = double;
  static constexpr int id = 0;
  static constexpr bool kSiteScale = false;
  static constexpr double kRawScale = 1.0;
  __device__ __forceinline__ static C cvt(S v) { return v; }
  __device__ __forceinline__ static C cvt_raw(S v) { return v; }
  __device__ __forceinline__ static S enc(C v) { return v; }
};
struct F32 {
  using S = float2; using C = float2; using R = float;
  static constexpr int id = 1;
  static constexpr bool kSiteScale = false;
  static constexpr float kRawScale = 1.0f;
  __device__ __forceinline__ static C cvt(S v) { return v; }
  __device__ __forceinline__ static C cvt_raw(S v) { return v; }
  __device__ __forceinline__ static S enc(C v) { return v; }
};

// 16-bit fixed point.  A complex number is a pair of int16, value = q * s / 32767.
// Vectors (Q16): s is a per-site scale, the largest |re| or |im| over the
// site's components, kept in one extra float plane after the component planes;
// the rounding error is at most 1.5e-5 of the site's largest component.
// Links and corner matrices (Q16L): s = 1, since every entry of an SU(3)
// matrix and of an average of products of SU(3) matrices is at most 1 in
// modulus.  Arithmetic is FP32.
constexpr float kQ16 = 32767.0f;
constexpr float kQ16MinScale = 1e-30f;   // smallest site scale kept (see st_site)
__device__ __forceinline__ short q16_round(float v) {
  return (short)max(-32767, min(32767, __float2int_rn(v)));
}
// Two values rounded to the nearest integer (ties to even) and packed as an
// int16 pair, for |re|, |im| <= 32767: adding 1.5 * 2^23 leaves the rounded
// integer, in two's complement, in the low mantissa bits.  fre, fim return
// the rounded values as floats (exact).
constexpr float kRoundMagic = 12582912.0f;
__device__ __forceinline__ uint32_t q16_pack(float re, float im, float inv, float& fre,
                                             float& fim) {
  const float a = __builtin_fmaf(re, inv, kRoundMagic);
  const float b = __builtin_fmaf(im, inv, kRoundMagic);
  fre = a - kRoundMagic;
  fim = b - kRoundMagic;
  return (__float_as_uint(a) & 0xffffu) | (__float_as_uint(b) << 16);
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
  static constexpr float kRawScale = 1.0f / kQ16;
  __device__ __forceinline__ static C cvt(S v) {
    return make_float2((float)v.x * (1.0f / kQ16), (float)v.y * (1.0f / kQ16));
  }
  __device__ __forceinline__ static C cvt_raw(S v) { return make_float2((float)v.x, (float)v.y); }
  __device__ __forceinline__ static S enc(C v) {
    short2 q;
    q.x = q16_round(v.x * kQ16);
    q.y = q16_round(v.y * kQ16);
    return q;
  }
};

// Storage of the links (NL reals) and of the corner matrices used with
// vectors of policy P.  16-bit vectors take 16-bit links of 12 or 18 reals:
// the 18-real form costs 6 more conversions per hop and saves the row-2
// rebuild (24 multiply-adds per hop), for 48 more bytes per site.
template <class P, int NL> struct LinkPol { using type = P; };
template <> struct LinkPol<Q16, 12> { using type = Q16L; };
template <> struct LinkPol<Q16, 18> { using type = Q16L; };
template <class P> struct CornerPol { using type = P; };
template <> struct CornerPol<Q16> { using type = Q16L; };

// Storage of the solution increment x_lo: FP32 when the Krylov vectors are
// 16-bit.  x_lo is amplified by the operator (errors in it grow by up to
// kappa), so 16-bit rounding there would stall the outer iteration.
template <class P> struct XPol { using type = P; };
template <> struct XPol<Q16> { using type = F32; };

// Size of one field of NC components in storage elements per site (the Q16
// scale adds one element); a field spans field_planes * Vp elements.
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

// ------------------------------------------------------------ site records
// Everything a site holds in one array -- the components of a vector field
// (and the Q16 scale), one direction's link, one corner matrix -- is a record
// of BYTES bytes.  A field of records keeps them in slabs of 16-byte elements
// (record bytes [16j, 16j+16) of every site in slab j), then, for what is
// left, one plane of 8-byte and/or one plane of 4-byte elements; each slab or
// plane has Vp elements, so a field occupies exactly Vp * BYTES bytes.  A lane
// loads its record with BYTES/16 128-bit loads (plus a 64- and/or a 32-bit
// one), each a coalesced access of 64 consecutive sites: four times fewer
// load instructions than one complex component at a time in FP32, up to
// sixteen times fewer in the 16-bit format.
//
// Loads and stores are raw buffer accesses: the array base is wavefront-
// uniform (a buffer descriptor in scalar registers), the slab offset a scalar
// offset and the per-lane part a 32-bit vector offset.  Every array a kernel
// reads this way is smaller than 4 GiB (checked at lattice creation).
constexpr int kBufferDword3 = 0x00020000;   // raw (untyped) buffer access on CDNA

template <int BYTES>
struct Rec {
  static_assert(BYTES % 4 == 0, "records are whole 32-bit words");
  static constexpr int A = BYTES / 16;          // 16-byte slabs
  static constexpr int B = (BYTES % 16) / 8;    // one 8-byte plane?
  static constexpr int C = (BYTES % 8) / 4;     // one 4-byte plane?
  static constexpr int W = BYTES / 4;           // 32-bit words
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, -1, kBufferDword3);
}

// CP: cache-policy bits of the buffer access; kStream marks data touched once
// per launch (non-temporal), so that it does not push out of L2 what other
// blocks re-read (links shared by the systems of a batch, stencil neighbours).
constexpr int kStream = 2;

// lo: a per-lane byte offset added to the lane's address, so that lanes may
// address different fields of a batch (a fixed stride apart) through one
// wavefront-uniform base
template <int BYTES, int CP = 0>
__device__ __forceinline__ void ld_rec(const void* __restrict__ base, int Vp, int i,
                                       uint32_t w[Rec<BYTES>::W], uint32_t lo = 0) {
  using R = Rec<BYTES>;
  const __amdgpu_buffer_rsrc_t rs = rsrc(base);
  const uint32_t vp = (uint32_t)Vp, ui = (uint32_t)i;
#pragma unroll
  for (int j = 0; j < R::A; ++j) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, lo + ui * 16u, (uint32_t)j * vp * 16u, CP);
    w[4 * j] = v[0]; w[4 * j + 1] = v[1]; w[4 * j + 2] = v[2]; w[4 * j + 3] = v[3];
  }
  if constexpr (R::B) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, lo + ui * 8u, (uint32_t)R::A * vp * 16u, CP);
    w[4 * R::A] = v[0]; w[4 * R::A + 1] = v[1];
  }
  if constexpr (R::C) {
    w[R::W - 1] = __builtin_amdgcn_raw_buffer_load_b32(
        rs, lo + ui * 4u, (uint32_t)R::A * vp * 16u + (uint32_t)R::B * vp * 8u, CP);
  }
}

template <int BYTES, int CP = 0>
__device__ __forceinline__ void st_rec(void* __restrict__ base, int Vp, int i,
                                       const uint32_t w[Rec<BYTES>::W], uint32_t lo = 0) {
  using R = Rec<BYTES>;
  const __amdgpu_buffer_rsrc_t rs = rsrc(base);
  const uint32_t vp = (uint32_t)Vp, ui = (uint32_t)i;
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  typedef uint32_t u2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int j = 0; j < R::A; ++j) {
    u4 v = {w[4 * j], w[4 * j + 1], w[4 * j + 2], w[4 * j + 3]};
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, lo + ui * 16u, (uint32_t)j * vp * 16u, CP);
  }
  if constexpr (R::B) {
    u2 v = {w[4 * R::A], w[4 * R::A + 1]};
    __builtin_amdgcn_raw_buffer_store_b64(v, rs, lo + ui * 8u, (uint32_t)R::A * vp * 16u, CP);
  }
  if constexpr (R::C) {
    __builtin_amdgcn_raw_buffer_store_b32(w[R::W - 1], rs, lo + ui * 4u,
                                          (uint32_t)R::A * vp * 16u + (uint32_t)R::B * vp * 8u, CP);
  }
}

// Component q of site i of an FP64 field (one 16-byte plane slab), for code
// that walks a record component by component.
template <int CP = 0>
__device__ __forceinline__ double2 ld_c64(const void* __restrict__ base, int Vp, int i, int q) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc(base), (uint32_t)i * 16u,
                                                       (uint32_t)q * (uint32_t)Vp * 16u, CP);
  double2 z;
  __builtin_memcpy(&z, &v, 16);
  return z;
}
template <int CP = 0>
__device__ __forceinline__ void st_c64(void* __restrict__ base, int Vp, int i, int q, double2 z) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  u4 v;
  __builtin_memcpy(&v, &z, 16);
  __builtin_amdgcn_raw_buffer_store_b128(v, rsrc(base), (uint32_t)i * 16u,
                                         (uint32_t)q * (uint32_t)Vp * 16u, CP);
}

// Storage words <-> complex values of a policy
template <class P>
__device__ __forceinline__ typename P::C dec(const uint32_t* w) {
  using S = typename P::S;
  S v;
  __builtin_memcpy(&v, w, sizeof(S));
  return P::cvt(v);
}
template <class P>
__device__ __forceinline__ typename P::C dec_raw(const uint32_t* w) {
  using S = typename P::S;
  S v;
  __builtin_memcpy(&v, w, sizeof(S));
  return P::cvt_raw(v);
}
template <class P>
__device__ __forceinline__ void enc_to(uint32_t* w, typename P::C c) {
  const typename P::S v = P::enc(c);
  __builtin_memcpy(w, &v, sizeof(v));
}

// Bytes of the record of an NC-component vector site under policy P.
template <class P> __host__ __device__ constexpr int vec_rec_bytes(int nc) {
  return nc * (int)sizeof(typename P::S) + (P::kSiteScale ? 4 : 0);
}

// All NC components of site i of a vector field f.
template <class P, int NC, int CP = 0>
__device__ __forceinline__ void ld_site(const typename P::S* __restrict__ f, int Vp, int i,
                                        typename P::C v[NC], uint32_t lo = 0) {
  constexpr int BY = vec_rec_bytes<P>(NC);
  uint32_t w[BY / 4];
  ld_rec<BY, CP>(f, Vp, i, w, lo);
  if constexpr (P::kSiteScale) {
    const float s = __uint_as_float(w[NC]) * (1.0f / kQ16);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const short2 z = __builtin_bit_cast(short2, w[q]);
      v[q] = make_float2((float)z.x * s, (float)z.y * s);
    }
  } else {
    constexpr int WPC = sizeof(typename P::S) / 4;
#pragma unroll
    for (int q = 0; q < NC; ++q) v[q] = dec<P>(w + q * WPC);
  }
}

// Site i without applying the Q16 site scale: v = stored integers (as float)
// and `scale` = the factor that turns them into values (1 for F32 and F64), so
// that a caller can apply it after a linear step on fewer numbers.
// dec_site_raw: the same from the record's storage words.
template <class P, int NC>
__device__ __forceinline__ void dec_site_raw(const uint32_t* w, typename P::C v[NC],
                                             typename P::R& scale) {
  if constexpr (P::kSiteScale) {
    scale = __uint_as_float(w[NC]) * (1.0f / kQ16);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const short2 z = __builtin_bit_cast(short2, w[q]);
      v[q] = make_float2((float)z.x, (float)z.y);
    }
  } else {
    constexpr int WPC = sizeof(typename P::S) / 4;
    scale = (typename P::R)1;
#pragma unroll
    for (int q = 0; q < NC; ++q) v[q] = dec<P>(w + q * WPC);
  }
}
template <class P, int NC>
__device__ __forceinline__ void ld_site_raw(const typename P::S* __restrict__ f, int Vp, int i,
                                            typename P::C v[NC], typename P::R& scale,
                                            uint32_t lo = 0) {
  constexpr int BY = vec_rec_bytes<P>(NC);
  uint32_t w[BY / 4];
  ld_rec<BY>(f, Vp, i, w, lo);
  dec_site_raw<P, NC>(w, v, scale);
}

// Store site i; returns ||stored value||^2 (the rounded value actually kept).
template <class P, int NC, int CP = 0>
__device__ __forceinline__ double st_site(typename P::S* __restrict__ f, int Vp, int i,
                                          const typename P::C v[NC], uint32_t lo = 0) {
  constexpr int BY = vec_rec_bytes<P>(NC);
  uint32_t w[BY / 4];
  double n2 = 0.0;
  if constexpr (P::kSiteScale) {
    float m = 0.0f;
#pragma unroll
    for (int q = 0; q < NC; ++q) m = fmaxf(m, fmaxf(fabsf(v[q].x), fabsf(v[q].y)));
    // a site whose largest component is below kQ16MinScale (far below the
    // per-system normalisation of the Krylov vectors, e.g. the exponential
    // tail of a point source several dozen hops out) is stored as zero: its
    // reciprocal would overflow FP32 and poison the site with inf and NaN
    if (!(m >= kQ16MinScale)) m = 0.0f;
    const float inv = m > 0.0f ? kQ16 / m : 0.0f;
    const float s = m * (1.0f / kQ16);
    float sq = 0.0f;   // sum of the squared stored integers (exact up to FP32 rounding)
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      float a, b;
      w[q] = q16_pack(v[q].x, v[q].y, inv, a, b);
      sq = __builtin_fmaf(a, a, __builtin_fmaf(b, b, sq));
    }
    w[NC] = __float_as_uint(m);
    n2 = (double)sq * ((double)s * (double)s);
  } else {
    constexpr int WPC = sizeof(typename P::S) / 4;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      enc_to<P>(w + q * WPC, v[q]);
      n2 += cnorm2(v[q]);
    }
  }
  st_rec<BY, CP>(f, Vp, i, w, lo);
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
// Links: four records per site, one per direction mu (the record field of mu
// starts at u + mu * Vp * NREAL/2 storage elements), each the row-major 3x3
// matrix (18 reals) or its rows 0 and 1 (12 reals; row 2 = conj(row0 x row1),
// exact for SU(3)).  Corner matrices: eight records of 9 complex numbers.
// RAW = true: the matrix times 1 / P::kRawScale (entries decoded without the
// storage scale; the rebuilt row 2 brought to the same scale).
template <class P, int NREAL, bool RAW = false>
__device__ __forceinline__ void load_link(const typename P::S* __restrict__ u, int Vp, int mu,
                                          int site, typename P::C m[9]) {
  using C = typename P::C;
  using R = typename P::R;
  constexpr int NCX = NREAL / 2;
  // FP64 links are always stored with 18 reals (one slab per entry); the
  // 12-real FP64 variant reads only the slabs of rows 0 and 1
  constexpr int NSTORE = P::id == 0 ? 9 : NCX;
  constexpr int BY = NCX * (int)sizeof(typename P::S);
  constexpr int WPC = sizeof(typename P::S) / 4;
  uint32_t w[BY / 4];
  ld_rec<BY>(u + (size_t)mu * NSTORE * Vp, Vp, site, w);
#pragma unroll
  for (int k = 0; k < NCX; ++k) m[k] = RAW ? dec_raw<P>(w + k * WPC) : dec<P>(w + k * WPC);
  if constexpr (NREAL == 12) {
    C a0 = m[0], a1 = m[1], a2 = m[2], b0 = m[3], b1 = m[4], b2 = m[5];
    m[6] = cconj(csub(cmul(a1, b2), cmul(a2, b1)));
    m[7] = cconj(csub(cmul(a2, b0), cmul(a0, b2)));
    m[8] = cconj(csub(cmul(a0, b1), cmul(a1, b0)));
    if constexpr (RAW && P::kRawScale != (R)1) {
#pragma unroll
      for (int k = 6; k < 9; ++k) m[k] = cscale(m[k], (R)P::kRawScale);
    }
  }
}
template <class P, int NREAL>
__device__ __forceinline__ void store_link(typename P::S* __restrict__ u, int Vp, int mu, int site,
                                           const typename P::C m[9]) {
  constexpr int NCX = NREAL / 2;
  constexpr int BY = NCX * (int)sizeof(typename P::S);
  constexpr int WPC = sizeof(typename P::S) / 4;
  uint32_t w[BY / 4];
#pragma unroll
  for (int k = 0; k < NCX; ++k) enc_to<P>(w + k * WPC, m[k]);
  st_rec<BY>(u + (size_t)mu * NCX * Vp, Vp, site, w);
}
template <class P, bool RAW = false>
__device__ __forceinline__ void load_corner(const typename P::S* __restrict__ c, int Vp, int cidx,
                                            int site, typename P::C m[9]) {
  constexpr int BY = 9 * (int)sizeof(typename P::S);
  constexpr int WPC = sizeof(typename P::S) / 4;
  uint32_t w[BY / 4];
  ld_rec<BY>(c + (size_t)cidx * 9 * Vp, Vp, site, w);
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k] = RAW ? dec_raw<P>(w + k * WPC) : dec<P>(w + k * WPC);
}
template <class P>
__device__ __forceinline__ void store_corner(typename P::S* __restrict__ c, int Vp, int cidx,
                                             int site, const typename P::C m[9]) {
  constexpr int BY = 9 * (int)sizeof(typename P::S);
  constexpr int WPC = sizeof(typename P::S) / 4;
  uint32_t w[BY / 4];
#pragma unroll
  for (int k = 0; k < 9; ++k) enc_to<P>(w + k * WPC, m[k]);
  st_rec<BY>(c + (size_t)cidx * 9 * Vp, Vp, site, w);
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
