// Host-side launch interface of the kernels (one translation unit per group).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "lq_types.h"

namespace lq {

struct OpArgs;
struct EpiArgs;

// The search-direction buffers of a CG solve, used in turn: iteration q of a
// group of G reads p[q] and writes p_{k+1} into p[(q + 1) % G] (G = 4, or 2
// for FP64; x takes the group's steps on its last iteration).
struct PRing {
  void* p[4];
};

// Threads per block of every site-block kernel; partial-sum arrays hold
// nbp(V) entries per right-hand side.
constexpr int kBlock = 256;
inline int nbp_of(int V, int block = kBlock) { return (((V + block - 1) / block) + 7) / 8 * 8; }

// ---- stencils: op = OpKind, prec = Prec, nl = 18/12 link reals
void launch_stencil(int op, int prec, int nl, bool dag, int epi, const OpArgs& oa,
                    const void* in, const EpiArgs& ea, int nrhs, hipStream_t s);

// Bytes of the intermediate fields of the on-the-fly Gamma_55 for one system
// (OpArgs::g55w; 14 fields of three complex numbers, FP64 or FP32).
size_t g55_bytes_per_system(const Geom& g, int prec);

// ---- CG vector kernels (templated on precision and components)
void launch_p_update(int prec, int nc, const Geom& g, SlotState* st, int par, int pend_next,
                     const double* part, int nbp, const void* p, void* pout, const void* r, int k0,
                     int nrhs, hipStream_t s);
// Reliable-update kernels act on running slots k with mask[k] != 0 (mask may be null).
void launch_ru_accumulate(int prec, int nc, const Geom& g, const SlotState* st, const int* mask,
                          double* xhi, void* xlo, const PRing& ring, int nbp, int k0, int nrhs,
                          hipStream_t s);
// part_f, part_g: the even-odd norms (null otherwise), see ru_finish_kernel
void launch_ru_finish(SlotState* st, const int* mask, const double* part, const double* part_f,
                      const double* part_g, int nbp, int k0, int nrhs, double ncomp, int rescale,
                      int max_cand, int init, int par, hipStream_t s);
void launch_ru_convert(int prec, int nc, const Geom& g, const SlotState* st, const int* mask,
                       const double* rhi, void* rlo, const PRing& ring, double* part, int nbp,
                       int init, int k0, int nrhs, hipStream_t s);
void launch_ru_commit(SlotState* st, const int* mask, const double* part, int nbp, int k0,
                      int nrhs, hipStream_t s);
void launch_load_prepare(int prec, int nc, const Geom& g, double* xhi, void* xlo, double* rhi,
                         const double* b, int nbp, int k0, int nrhs, hipStream_t s);

// ---- layout / conversion
// canonical (V, nc) complex (c128 if src_f64 else c64) -> SoA field (prec) for rhs k0..
// par >= 0: g is a half-lattice geometry and the SoA field holds the sites of
// that parity of the canonical (2 g.V, nc) field (even-odd blocks)
void launch_field_in(int prec, int nc, const Geom& g, const void* canon, int canon_f64, void* soa,
                     int nbp, int k0, int nrhs, hipStream_t s, int par = -1);
void launch_field_out(int prec, int nc, const Geom& g, const void* soa, void* canon, int canon_f64,
                      int nbp, int k0, int nrhs, hipStream_t s, int par = -1);
// sites [i0, i0 + n) of a canonical gauge field whose site i0 is at `canon`
void launch_gauge_in(const Geom& g, const void* canon, double2* u64, int i0, int n,
                     hipStream_t s);
void launch_links_convert(int prec, int nl, const Geom& g, const double2* u64, void* dst,
                          hipStream_t s);
void launch_links_eo(int prec, int nl, const Geom& g, int Vhp, const double2* u64, void* dst,
                     hipStream_t s);
void launch_corners(const Geom& g, const double2* u64, double2* c64, hipStream_t s);
void launch_corners_convert(int prec, const Geom& g, const double2* c64, void* dst, hipStream_t s);
void launch_su3_deviation(const Geom& g, const double2* u64, double* part, double* out,
                          hipStream_t s);
void launch_plaquette(const Geom& g, const double2* u64, double* part, int nbp, double* out,
                      hipStream_t s);
void launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// nrhs vector fields of nc components in precision prec, every component
// uniform in [-1, 1) from a hash of (seed, system, site, component)
void launch_fill_test(int prec, int nc, const Geom& g, void* soa, int nrhs, uint32_t seed,
                      hipStream_t s);

// ---- pion correlator (Wilson point-source propagators, canonical complex128)
int pion_blocks_per_slice(int L4);
// part: L4 * pion_blocks_per_slice(L4) doubles; corr: L4 doubles (device)
void launch_pion_correlator(const Geom& g, int nsrc, const double2* props, double* part,
                            double* corr, hipStream_t s);

// ---- Lanczos (FP64, one vector of nc planes)
void launch_lz_dots(const Geom& g, int nc, const double2* V, int nvec, double2* w,
                    const double* alpha_part, int nbp_alpha, double* alpha_out, double* part_h,
                    int nblk, hipStream_t s);
void launch_lz_reduce(const double* part_h, int nvec, int nblk, double2* h, hipStream_t s);
void launch_lz_update(const Geom& g, int nc, const double2* V, int nvec, const double2* h,
                      double2* w, double* part_n, int nblk, int with_norm, hipStream_t s);
void launch_lz_finish(const double* part_n, int nblk, double* beta_out, hipStream_t s);
void launch_lz_normalize(const Geom& g, int nc, const double2* w, const double* beta,
                         double2* vnext, hipStream_t s);

}  // namespace lq
