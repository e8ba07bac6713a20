// Host engine: lattice/gauge handles, workspace carving, the slot-based CG
// engine and the Lanczos driver.  Everything here runs on the host and only
// enqueues kernels; device memory always belongs to the caller.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lq.h"
#include "common.h"
#include "dirac.h"
#include "kernels.h"
#include "lq_types.h"
#include "hessenberg.h"
#include "stencil.h"

namespace lq {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define LQ_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::lq::Error(LQ_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(LQ_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

// Bump allocator over a caller buffer (or a size-only dry run when base is null).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
  size_t size() const { return (off + 255) & ~(size_t)255; }
};

inline size_t store_bytes(int prec) { return prec == P64 ? 16 : (prec == P32 ? 8 : 4); }
// planes of one vector field: the 16-bit format adds a per-site scale plane
inline int field_planes_host(int prec, int nc) { return nc + (prec == P16 ? 1 : 0); }
inline size_t field_bytes(const Geom& g, int prec, int nc) {
  return (size_t)field_planes_host(prec, nc) * g.Vp * store_bytes(prec);
}
// Whether the second stencil of a low-precision CG iteration streams its
// per-system vectors (non-temporal r, the search directions and x): when an
// iteration's vectors -- counted as t, r, two directions and x -- exceed the
// last-level cache (256 MiB of Infinity Cache on MI355X) none of them
// survives to the next kernel anyway, and streaming keeps the links and the
// stencil input in L2; below it they stay cached for the kernels that
// follow.  FP64 kernels always cache.
constexpr size_t kLastLevelCache = size_t(256) << 20;
inline int stream_cg_vectors(const Geom& g, int prec, int nc, int nrhs) {
  if (prec == P64) return 0;
  const size_t x = (size_t)nc * g.Vp * store_bytes(prec == P16 ? P32 : prec);
  return (size_t)nrhs * (4 * field_bytes(g, prec, nc) + x) > kLastLevelCache;
}
// Geometry of the half-lattice fields of the even-odd blocks: the lattice's
// extents, half its sites, the same plane padding rule.
inline Geom half_geom(const Geom& g) {
  Geom h = g;
  h.V = g.V / 2;
  h.Vp = ((h.V + 63) / 64) * 64 + 64;
  return h;
}
inline int ncomp_of(int formulation) { return formulation == LQ_WILSON ? 12 : 3; }
inline int opkind(int formulation, int g55) {
  if (formulation == LQ_WILSON) return OP_WILSON;
  return g55 == LQ_G55_ONTHEFLY ? OP_SW_OTF : OP_SW_CORNERS;
}

}  // namespace lq

struct lq_lattice_s {
  lq::Geom g;
  int32_t dims[4];
  int32_t bc[4];
};

struct lq_gauge_s {
  lq::Geom g;
  uint32_t features;
  double2* u64 = nullptr;     // 18-real FP64 links
  float2* u32_18 = nullptr;
  float2* u32_12 = nullptr;
  short2* u16_12 = nullptr;     // 16-bit fixed point, 12-real
  short2* u16_18 = nullptr;     // 16-bit fixed point, 18-real
  // even-odd copies (LQ_FEAT_EO): per parity, half-lattice records
  void* eo64 = nullptr;
  void* eo32_18 = nullptr;
  void* eo32_12 = nullptr;
  void* eo16_12 = nullptr;
  void* eo16_18 = nullptr;
  double2* c64 = nullptr;     // corners
  float2* c32 = nullptr;
  short2* c16 = nullptr;
  double* scratch = nullptr;  // plaquette partials + result
  double2* stage = nullptr;   // staging area of a host upload (kStageSites canonical sites)
  int nbp = 0;
  double su3_dev = 0.0;       // max |row2 - conj(row0 x row1)| over the links

  const void* links(int prec, int nl) const;
  // links of parity par for the even-odd blocks (LQ_FEAT_EO)
  const void* links_eo(int prec, int nl, int par) const;
  // FP64 links: rows 0, 1 only (row 2 rebuilt) when the field is SU(3) to
  // rounding, which reads a third fewer link bytes, else all 18 reals
  int fp64_links() const { return su3_dev <= 1e-12 ? 12 : 18; }
  const void* corners(int prec) const;
};

namespace lq {

// Canonical sites per chunk of a host gauge upload (576 bytes each).
constexpr int kStageSites = 4096;
// Carves a gauge buffer; with base == nullptr only the size is computed.
size_t gauge_layout(const Geom& g, uint32_t features, void* base, lq_gauge_s* out);

// The slot-based CG engine (single solves, batched solves and serving).
struct Engine {
  const lq_gauge_s* gauge = nullptr;
  int formulation = 0, op = 0, nc = 0;
  double r = 1.0;
  int nslots = 0;
  int prec_lo = P64, nl_lo = 18;
  int reliable_interval = 256, poll_every = 16, use_graph = 0, max_cand = 50;
  double delta = 0.0;
  int nbp = 0;
  int rhs_per_thread = 1;     // systems per thread of the CG stencils (autotuned)
  int window = 0;             // XCD window of the CG stencils' block order (autotuned)
  // even-odd preconditioning (Wilson, r = 1): the vectors hold the even sites
  // and the operator is the Schur complement M^ (vg is the half lattice)
  bool eo = false;
  Geom vg{};                  // geometry of the solver's vectors
  double2 *wbuf = nullptr;    // eo: odd half-lattice intermediate of a Schur pair
  double2 *chio = nullptr;    // eo: odd half of each source, for the solution's odd half
  double2 *bhat = nullptr;    // eo: b^_e = chi_e - M_eo chi_o / d
  double *part_f = nullptr, *part_g = nullptr;   // eo: norms behind eq. (2)'s residual
  // device
  double2 *b = nullptr, *xhi = nullptr, *rhi = nullptr, *t64 = nullptr;
  void *xlo = nullptr, *rlo = nullptr, *t = nullptr;
  void *p = nullptr, *p1 = nullptr, *p2 = nullptr, *p3 = nullptr;  // the search directions, in turn
  PRing ring() const { return PRing{{p, p1, p2, p3}}; }
  int group = 4;   // iterations per x update (2 for FP64: its vectors stay in the last-level cache)
  double *part_t = nullptr, *part_r = nullptr, *part_u = nullptr;
  void* g55w = nullptr;       // on-the-fly Gamma_55: intermediate fields, FP64-sized per slot
  SlotState* st = nullptr;
  int* mask = nullptr;        // per-slot reliable-update selection
  // host
  SlotState* hst = nullptr;   // pinned mirror
  int* hmask = nullptr;       // pinned
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t gstream = nullptr;
  int gchunk = 0;

  static size_t workspace_bytes(const Geom& g, int formulation, int g55,
                                const lq_solve_opts* opts, int nslots);
  void init(const lq_gauge_s* g, int formulation, int g55, double r, int nslots,
            const lq_solve_opts* opts, void* ws, size_t ws_bytes, hipStream_t s);
  ~Engine();

  void load(int slot, const void* chi, double mass, double tol, int maxiter, hipStream_t s);
  // advance about `iters` iterations; returns after polling the slot states
  void step(int iters, hipStream_t s);
  void fetch(int slot, void* x, lq_solve_info* info, hipStream_t s);
  void cancel(int slot, hipStream_t s);   // discard a loaded slot and free it
  int running() const;

 private:
  OpArgs op_args(int prec, int nl) const;
  // one application of the solver's operator (M, or M^ when eo) with epilogue epi
  void stencil(int prec, int nl, bool dag, int epi, const void* in, const EpiArgs& e, int nrhs,
               hipStream_t s) const;
  // the even-odd blocks in one of their forms (see WilsonEOOp), FP64, with
  // epilogue STORE or STORE_NORM (into part) over the slots e selects
  void eo_form(int par, int form, bool dag, const void* diag, const void* in, EpiArgs e, int epi,
               int nrhs, hipStream_t s) const;
  EpiArgs epi_base() const;
  void enqueue_iterations(int n, hipStream_t s);
  void enqueue_reliable_update(hipStream_t s);
  void poll(hipStream_t s);
  bool select_updates();
  void tune(hipStream_t s);
};

// Systems-per-thread choice for a batched low-precision stencil: timed on the
// device once per (GPU, lattice, operator, precision, links, batch size) and
// remembered in memory and in a small text cache file (LQ_TUNE_CACHE, default
// $HOME/.cache/lq_tune.txt).
// The Schur complement of the even-odd blocks (Wilson, r = 1) on half-lattice
// fields of the even sites: out = M^ in = d in - M_eo M_oe in / d (M^dag with
// dag).  The odd half-lattice field w receives M_oe in; the second launch
// applies epilogue `epi` with `e` (its output, partials, solver state).
// `base` carries the masses and r; the links are the gauge field's even-odd copies.
void enqueue_schur(const lq_gauge_s* g, const OpArgs& base, int prec, int nl, bool dag, int epi,
                   const void* in, void* w, const EpiArgs& e, int nrhs, hipStream_t s);

int tuned_rhs_per_thread(const std::string& key);   // 0: not tuned; else K + 16 * (window + 3)
std::string tune_key(const Geom& g, int op, int prec, int nl, int nslots);
void remember_rhs_per_thread(const std::string& key, int k);

// Lanczos with full reorthogonalisation on A = M^dag M.
size_t lanczos_workspace_bytes(const Geom& g, int formulation, int g55, int steps);
// Eigenvalues of M (the Dirac matrix of d) nearest the real shift sigma by
// shift-invert Arnoldi; see lq_spectrum.  Returns the number found.
size_t spectrum_workspace_bytes(const Geom& g, int formulation, int g55, int steps);
int spectrum_run(const lq_gauge_s* g, const lq_dirac* d, double sigma, int steps, int restarts,
                 double tol, const void* v0, void* ws, size_t ws_bytes, std::vector<cplx>& eig,
                 std::vector<double>& resid, hipStream_t s);
int lanczos_run(const lq_gauge_s* g, const lq_dirac* d, int steps, const void* v0, void* ws,
                size_t ws_bytes, std::vector<double>& alpha, std::vector<double>& beta,
                hipStream_t s);
// The staggered overlap operator (k_overlap.hip): see lq_overlap_apply.
size_t overlap_workspace_bytes(const Geom& g, int g55);
void overlap_apply(const lq_gauge_s* g, const lq_overlap* ov, const void* in, void* out, void* ws,
                   size_t ws_bytes, hipStream_t s);
// extreme eigenvalues of the symmetric tridiagonal (alpha, beta) by Sturm bisection
void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, double& lo,
                      double& hi);

}  // namespace lq
