// extern "C" entry points of include/lq.h: argument validation, error codes,
// and thin calls into the engine.  No C++ exception crosses this file.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <mutex>
#include <map>
#include <vector>

#include "engine.h"

using namespace lq;

static thread_local std::string g_last_error;

template <class F>
static int guard(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return LQ_ERR_ARG;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return LQ_ERR_ARG;
  } catch (...) {
    g_last_error = "unknown error";
    return LQ_ERR_ARG;
  }
}

static void need(bool ok, const char* msg) {
  if (!ok) throw Error(LQ_ERR_ARG, msg);
}

static hipStream_t S(void* s) { return (hipStream_t)s; }

static void check_dirac(const lq_dirac* d) {
  need(d != nullptr, "null lq_dirac");
  need(d->formulation == LQ_WILSON || d->formulation == LQ_STAGGERED_WILSON, "bad formulation");
  need(d->g55_mode == LQ_G55_CORNERS || d->g55_mode == LQ_G55_ONTHEFLY, "bad g55_mode");
  need(std::isfinite(d->mass) && std::isfinite(d->r), "mass and r must be finite");
}

static void check_prec(int32_t prec, int32_t links) {
  need(prec == LQ_PREC_F64 || prec == LQ_PREC_F32 || prec == LQ_PREC_Q16, "bad precision");
  need(links == 0 || links == LQ_LINKS_18 || links == LQ_LINKS_12, "links must be 18 or 12");
}

static int links_for(const lq_gauge* g, int32_t prec, int32_t links) {
  if (links) return links;
  if (prec == LQ_PREC_F64) return g->fp64_links();
  return prec == LQ_PREC_Q16 ? 12 : 18;
}

extern "C" {

const char* lq_last_error(void) { return g_last_error.c_str(); }

const char* lq_version(void) { return "lq 0.1 gfx950"; }

int lq_lattice_create(const int32_t dims[4], const int32_t bc[4], lq_lattice** out) {
  return guard([&] {
    need(dims && out, "null argument");
    int64_t V = 1;
    for (int mu = 0; mu < 4; ++mu) {
      need(dims[mu] >= 4 && dims[mu] % 2 == 0, "every lattice extent must be even and >= 4");
      V *= dims[mu];
    }
    need(V < (1ll << 28), "volume must be below 2^28 sites");
    auto* l = new lq_lattice_s;
    std::memset(l, 0, sizeof(*l));
    Geom& g = l->g;
    int st = 1;
    for (int mu = 0; mu < 4; ++mu) {
      g.L[mu] = dims[mu];
      g.stride[mu] = st;
      st *= dims[mu];
      l->dims[mu] = dims[mu];
      const int b = bc ? bc[mu] : 1;
      if (b != 1 && b != -1) { delete l; throw Error(LQ_ERR_ARG, "bc entries must be +1 or -1"); }
      g.bc[mu] = b;
      l->bc[mu] = b;
      if (b < 0) g.has_bc = 1;
    }
    g.V = (int)V;
    // pad each plane by 64 elements past a 64-multiple: plane starts avoid
    // falling on the same HBM channel for power-of-two volumes
    g.Vp = (int)(((V + 63) / 64) * 64 + 64);
    for (int k = 0; k < 3; ++k) g.dv[k].init((uint32_t)dims[k]);
    *out = l;
    return LQ_OK;
  });
}

void lq_lattice_destroy(lq_lattice* lat) { delete lat; }

int64_t lq_lattice_volume(const lq_lattice* lat) { return lat ? (int64_t)lat->g.V : -1; }

size_t lq_gauge_bytes(const lq_lattice* lat, uint32_t features) {
  if (!lat) return 0;
  return gauge_layout(lat->g, features, nullptr, nullptr);
}

int lq_gauge_create(const lq_lattice* lat, const void* U, int32_t where, uint32_t features,
                    void* buf, size_t buf_bytes, void* stream, lq_gauge** out) {
  return guard([&] {
    need(lat && U && buf && out, "null argument");
    need((features & ~15u) == 0, "unknown feature bits");
    need(where == LQ_WHERE_HOST || where == LQ_WHERE_DEVICE, "where must be host or device");
    const size_t nb = gauge_layout(lat->g, features, nullptr, nullptr);
    if (buf_bytes < nb)
      throw Error(LQ_ERR_WORKSPACE, "gauge buffer too small: need " + std::to_string(nb));
    std::unique_ptr<lq_gauge_s> g(new lq_gauge_s);
    gauge_layout(lat->g, features, buf, g.get());
    hipStream_t s = S(stream);
    launch_fill_zero(buf, nb, s);
    if (where == LQ_WHERE_DEVICE) {
      launch_gauge_in(g->g, U, g->u64, 0, g->g.V, s);
    } else {
      // chunks through the staging area; the copy of a chunk is ordered after
      // the repack of the previous one on the same stream
      const size_t site_bytes = 36 * 16;
      for (int i0 = 0; i0 < g->g.V; i0 += kStageSites) {
        const int n = std::min(kStageSites, g->g.V - i0);
        LQ_HIP(hipMemcpyAsync(g->stage, (const char*)U + (size_t)i0 * site_bytes,
                              (size_t)n * site_bytes, hipMemcpyHostToDevice, s));
        launch_gauge_in(g->g, g->stage, g->u64, i0, n, s);
      }
    }
    launch_su3_deviation(g->g, g->u64, g->scratch, g->scratch + g->nbp + 1, s);
    LQ_HIP(hipMemcpyAsync(&g->su3_dev, g->scratch + g->nbp + 1, sizeof(double),
                          hipMemcpyDeviceToHost, s));
    if (features & LQ_FEAT_F32) {
      launch_links_convert(P32, 18, g->g, g->u64, g->u32_18, s);
      launch_links_convert(P32, 12, g->g, g->u64, g->u32_12, s);
    }
    if (features & LQ_FEAT_Q16) {
      launch_links_convert(P16, 12, g->g, g->u64, g->u16_12, s);
      launch_links_convert(P16, 18, g->g, g->u64, g->u16_18, s);
    }
    if (features & LQ_FEAT_EO) {
      const int Vhp = half_geom(g->g).Vp;
      launch_links_eo(P64, 18, g->g, Vhp, g->u64, g->eo64, s);
      if (features & LQ_FEAT_F32) {
        launch_links_eo(P32, 18, g->g, Vhp, g->u64, g->eo32_18, s);
        launch_links_eo(P32, 12, g->g, Vhp, g->u64, g->eo32_12, s);
      }
      if (features & LQ_FEAT_Q16) {
        launch_links_eo(P16, 12, g->g, Vhp, g->u64, g->eo16_12, s);
        launch_links_eo(P16, 18, g->g, Vhp, g->u64, g->eo16_18, s);
      }
    }
    if (features & LQ_FEAT_CORNERS) {
      launch_corners(g->g, g->u64, g->c64, s);
      if (features & LQ_FEAT_F32) launch_corners_convert(P32, g->g, g->c64, g->c32, s);
      if (features & LQ_FEAT_Q16) launch_corners_convert(P16, g->g, g->c64, g->c16, s);
    }
    check_launch();
    LQ_HIP(hipStreamSynchronize(s));   // su3_dev is read on the host
    *out = g.release();
    return LQ_OK;
  });
}

void lq_gauge_destroy(lq_gauge* g) { delete g; }

int lq_gauge_su3_deviation(const lq_gauge* g, double* dev) {
  return guard([&] {
    need(g && dev, "null argument");
    *dev = g->su3_dev;
    return LQ_OK;
  });
}

int lq_gauge_plaquette(const lq_gauge* g, double* plaquette, void* stream) {
  return guard([&] {
    need(g && plaquette, "null argument");
    hipStream_t s = S(stream);
    launch_plaquette(g->g, g->u64, g->scratch, g->nbp, g->scratch + g->nbp, s);
    check_launch();
    LQ_HIP(hipMemcpyAsync(plaquette, g->scratch + g->nbp, sizeof(double), hipMemcpyDeviceToHost, s));
    LQ_HIP(hipStreamSynchronize(s));
    return LQ_OK;
  });
}

// -------------------------------------------------------------- apply
size_t lq_apply_workspace_bytes(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                                int32_t precision) {
  if (!g || (formulation != LQ_WILSON && formulation != LQ_STAGGERED_WILSON)) return 0;
  if (precision < 0 || precision > 2) return 0;
  if (g55_mode != LQ_G55_CORNERS && g55_mode != LQ_G55_ONTHEFLY) return 0;
  const size_t v = field_bytes(g->g, precision, ncomp_of(formulation));
  Carver c(nullptr);
  c.take(v); c.take(v); c.take(v);
  c.take((size_t)nbp_of(g->g.V) * 8);
  if (opkind(formulation, g55_mode) == OP_SW_OTF) c.take(g55_bytes_per_system(g->g, precision));
  return c.size();
}

static OpArgs make_op(const lq_gauge* g, const lq_dirac* d, int prec, int nl) {
  OpArgs a;
  a.g = g->g;
  a.links = g->links(prec, nl);
  const int op = opkind(d->formulation, d->g55_mode);
  a.corners = op == OP_SW_CORNERS ? g->corners(prec) : nullptr;
  a.r = d->r;
  a.mass0 = d->mass;
  a.mass = nullptr;
  a.mass_stride = 0;
  return a;
}

int lq_apply(const lq_gauge* g, const lq_dirac* d, int32_t opsel, int32_t precision,
             int32_t links, const void* in, void* out, void* ws, size_t ws_bytes, void* stream) {
  return guard([&] {
    need(g && in && out && ws, "null argument");
    check_dirac(d);
    check_prec(precision, links);
    need(opsel == LQ_OP_M || opsel == LQ_OP_MDAG || opsel == LQ_OP_MDAGM, "bad op");
    const size_t nb = lq_apply_workspace_bytes(g, d->formulation, d->g55_mode, precision);
    if (ws_bytes < nb) throw Error(LQ_ERR_WORKSPACE, "apply workspace too small: need " + std::to_string(nb));
    const int nl = links_for(g, precision, links);
    const int nc = ncomp_of(d->formulation);
    const int op = opkind(d->formulation, d->g55_mode);
    OpArgs oa = make_op(g, d, precision, nl);
    const size_t v = field_bytes(g->g, precision, nc);
    Carver c(ws);
    void* a = c.take(v);
    void* b = c.take(v);
    void* tmp = c.take(v);
    (void)c.take((size_t)nbp_of(g->g.V) * 8);
    if (op == OP_SW_OTF) {
      oa.g55_sys = g55_bytes_per_system(g->g, precision);
      oa.g55w = c.take(oa.g55_sys);
    }
    hipStream_t s = S(stream);
    const int nbp = nbp_of(g->g.V);
    const int f64 = precision == LQ_PREC_F64;
    launch_field_in(precision, nc, g->g, in, f64, a, nbp, 0, 1, s);
    EpiArgs e;
    std::memset(&e, 0, sizeof(e));
    e.nbp = nbp;
    e.window = -3;   // tiled order where the lattice allows it
    if (opsel == LQ_OP_MDAGM) {
      e.out = tmp;
      launch_stencil(op, precision, nl, false, EPI_STORE, oa, a, e, 1, s);
      e.out = b;
      launch_stencil(op, precision, nl, true, EPI_STORE, oa, tmp, e, 1, s);
    } else {
      e.out = b;
      launch_stencil(op, precision, nl, opsel == LQ_OP_MDAG, EPI_STORE, oa, a, e, 1, s);
    }
    launch_field_out(precision, nc, g->g, b, out, f64, nbp, 0, 1, s);
    check_launch();
    return LQ_OK;
  });
}

// ------------------------------------------------- allocation-free apply
// Scratch of lq_apply_noalloc: one array per GPU, resident from module load
// until the process ends.  Its name is only a host-side stand-in for the
// device symbol; the device address is looked up once per device with
// hipGetSymbolAddress and used everywhere instead.
constexpr size_t kApplyScratchBytes = size_t(80) << 20;
static __device__ __align__(256) unsigned char scratch[kApplyScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_ptr;   // device ordinal -> device address of `scratch`

static void* apply_scratch() {
  int dev = 0;
  LQ_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    throw Error(LQ_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

size_t lq_apply_noalloc_max_bytes(void) { return kApplyScratchBytes; }

int lq_apply_noalloc(const lq_gauge* g, const lq_dirac* d, int32_t opsel, int32_t precision,
                     int32_t links, const void* in, void* out, void* stream) {
  return guard([&] {
    need(g && d && in && out, "null argument");
    check_dirac(d);
    check_prec(precision, links);
    const size_t nb = lq_apply_workspace_bytes(g, d->formulation, d->g55_mode, precision);
    if (nb == 0) throw Error(LQ_ERR_ARG, "bad formulation, Gamma_55 mode or precision");
    if (nb > kApplyScratchBytes)
      throw Error(LQ_ERR_WORKSPACE, "lq_apply_noalloc: this lattice needs " + std::to_string(nb) +
                                        " bytes of scratch, above its fixed maximum of " +
                                        std::to_string(kApplyScratchBytes));
    void* ws = apply_scratch();
    const int rc = lq_apply(g, d, opsel, precision, links, in, out, ws, kApplyScratchBytes, stream);
    if (rc != LQ_OK) throw Error(rc, g_last_error);
    return LQ_OK;
  });
}

size_t lq_schur_workspace_bytes(const lq_gauge* g, int32_t precision) {
  if (!g || precision < 0 || precision > 2) return 0;
  const size_t v = field_bytes(half_geom(g->g), precision, 12);
  Carver c(nullptr);
  c.take(v); c.take(v); c.take(v);
  return c.size();
}

int lq_schur_apply(const lq_gauge* g, const lq_dirac* d, int32_t dagger, int32_t precision,
                   int32_t links, const void* in, void* out, void* ws, size_t ws_bytes,
                   void* stream) {
  return guard([&] {
    need(g && in && out && ws, "null argument");
    check_dirac(d);
    check_prec(precision, links);
    need(d->formulation == LQ_WILSON && d->r == 1.0, "the even-odd blocks are built for Wilson, r = 1");
    const size_t nb = lq_schur_workspace_bytes(g, precision);
    if (ws_bytes < nb) throw Error(LQ_ERR_WORKSPACE, "schur workspace too small: need " + std::to_string(nb));
    const int nl = links_for(g, precision, links);
    const Geom gh = half_geom(g->g);
    const size_t v = field_bytes(gh, precision, 12);
    Carver c(ws);
    void* a = c.take(v);
    void* w = c.take(v);
    void* b = c.take(v);
    hipStream_t s = S(stream);
    const int nbp = nbp_of(gh.V);
    const int f64 = precision == LQ_PREC_F64;
    launch_field_in(precision, 12, gh, in, f64, a, nbp, 0, 1, s, 0);
    OpArgs base = make_op(g, d, precision, nl);
    EpiArgs e;
    std::memset(&e, 0, sizeof(e));
    e.nbp = nbp;
    e.out = b;
    enqueue_schur(g, base, precision, nl, dagger != 0, EPI_STORE, a, w, e, 1, s);
    launch_fill_zero(out, (size_t)g->g.V * 12 * (f64 ? 16 : 8), s);
    launch_field_out(precision, 12, gh, b, out, f64, nbp, 0, 1, s, 0);
    check_launch();
    return LQ_OK;
  });
}

size_t lq_time_dslash_workspace_bytes(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                                      int32_t precision, int32_t nrhs) {
  if (!g || nrhs < 1 || precision < 0 || precision > 2) return 0;
  if (formulation != LQ_WILSON && formulation != LQ_STAGGERED_WILSON) return 0;
  if (g55_mode != LQ_G55_CORNERS && g55_mode != LQ_G55_ONTHEFLY) return 0;
  const size_t v = (size_t)nrhs * field_bytes(g->g, precision, ncomp_of(formulation));
  const size_t np = (size_t)nrhs * nbp_of(g->g.V) * sizeof(double);
  Carver c(nullptr);
  c.take(v);
  c.take(v);
  c.take(np);
  c.take(v);
  c.take(np);
  c.take((size_t)nrhs * sizeof(SlotState));
  c.take((size_t)nrhs * ncomp_of(formulation) * g->g.Vp * store_bytes(precision == P16 ? P32 : precision));
  c.take(v);
  c.take(v);   // the odd intermediate of the even-odd pairs
  c.take(v);   // two more search directions of the CG update's group of four
  c.take(v);
  if (opkind(formulation, g55_mode) == OP_SW_OTF)
    c.take((size_t)nrhs * g55_bytes_per_system(g->g, precision));
  return c.size();
}

int lq_time_dslash(const lq_gauge* g, const lq_dirac* d, int32_t kernel, int32_t precision,
                   int32_t links, int32_t nrhs, int32_t rhs_per_thread, int32_t window,
                   int32_t reps, void* ws, size_t ws_bytes, double* avg_ms, void* stream) {
  return guard([&] {
    need(g && ws && avg_ms, "null argument");
    check_dirac(d);
    check_prec(precision, links);
    need(nrhs >= 1 && reps >= 1, "nrhs and reps must be >= 1");
    need(rhs_per_thread == 1 || rhs_per_thread == 2 || rhs_per_thread == 4 || rhs_per_thread == 8,
         "rhs_per_thread must be 1, 2, 4 or 8");
    need(rhs_per_thread == 1 || precision != LQ_PREC_F64, "FP64 stencils take one system per thread");
    need(window >= -4 || (window <= -11 && window >= -16), "window must be >= -4 or a t-sweep order -11 ... -16");
    const int nl = links_for(g, precision, links);
    const int nc = ncomp_of(d->formulation);
    const int op = opkind(d->formulation, d->g55_mode);
    need(kernel >= 0 && kernel <= 4, "kernel selector must be 0 to 4");
    const bool eo = kernel >= 3;
    if (eo) need(d->formulation == LQ_WILSON && d->r == 1.0, "the even-odd pairs are built for Wilson, r = 1");
    if (rhs_per_thread == 8)
      need(d->formulation == LQ_WILSON && d->r == 1.0 && nl == 18 && !eo,
           "rhs_per_thread 8 (the lanes stencil) is built for Wilson, r = 1, 18-real links, "
           "unpreconditioned");
    const size_t v = (size_t)nrhs * field_bytes(g->g, precision, nc);
    const size_t np = (size_t)nrhs * nbp_of(g->g.V) * sizeof(double);
    Carver c(ws);
    void* a = c.take(v);
    void* b = c.take(v);
    double* part = (double*)c.take(np);
    void* r = c.take(v);
    double* part_in = (double*)c.take(np);
    SlotState* st = (SlotState*)c.take((size_t)nrhs * sizeof(SlotState));
    void* xlo = c.take((size_t)nrhs * nc * g->g.Vp * store_bytes(precision == P16 ? P32 : precision));
    void* pprev = c.take(v);
    void* w = c.take(v);
    void* pr1 = c.take(v);
    void* pr2 = c.take(v);
    OpArgs oa = make_op(g, d, precision, nl);
    if (op == OP_SW_OTF) {
      oa.g55_sys = g55_bytes_per_system(g->g, precision);
      oa.g55w = c.take((size_t)nrhs * oa.g55_sys);
    }
    if (ws_bytes < c.size())
      throw Error(LQ_ERR_WORKSPACE, "timing workspace too small: need " + std::to_string(c.size()));
    hipStream_t s = S(stream);
    launch_fill_zero(ws, c.size(), s);
    const Geom vg = eo ? half_geom(g->g) : g->g;   // geometry of the timed fields
    // non-zero data and a live solver state: every vector field uniform in
    // [-1, 1) per component, rho = 1 and partials of ||t||^2 summing to 1
    // (alpha = 1), the group's earlier steps alpha_j = 2^-(j+1)
    {
      void* vecs[] = {a, b, r, pprev, pr1, pr2};
      for (int j = 0; j < 6; ++j) launch_fill_test(precision, nc, vg, vecs[j], nrhs, 101 + j, s);
      launch_fill_test(precision == P16 ? P32 : precision, nc, vg, xlo, nrhs, 107, s);
      std::vector<SlotState> hs(nrhs);
      std::vector<double> hp((size_t)nrhs * nbp_of(vg.V), 1.0 / nbp_of(vg.V));
      for (auto& q : hs) {
        std::memset(&q, 0, sizeof(q));
        q.status = SLOT_RUNNING;
        q.rho[0] = q.rho[1] = 1.0;
        q.scale = q.scale_prev = 1.0;
        q.mass = d->mass;
        for (int j = 0; j < 4; ++j) q.alpha[j] = std::ldexp(1.0, -(j + 1));
      }
      LQ_HIP(hipMemcpyAsync(st, hs.data(), hs.size() * sizeof(SlotState), hipMemcpyHostToDevice, s));
      LQ_HIP(hipMemcpyAsync(part_in, hp.data(), hp.size() * sizeof(double), hipMemcpyHostToDevice, s));
      LQ_HIP(hipStreamSynchronize(s));   // the host arrays go out of scope
    }
    EpiArgs e;
    std::memset(&e, 0, sizeof(e));
    e.nbp = nbp_of(vg.V);
    e.out = b;
    e.part = part;
    e.rhs_per_thread = rhs_per_thread;
    e.window = window;
    // 0: the first matvec of a CG iteration (t = M p with ||t||^2); 1: the
    // plain M^dag stencil; 2: the second (q = M^dag t, r -= alpha q, ||r||^2,
    // and on every fourth launch x += the four steps of the group, as in the
    // solver's iterations), on the live state set up above; 3 and 4: the
    // same two steps of an even-odd
    // preconditioned iteration, each a pair of half-lattice launches
    // (t = M^ p with ||t||^2; M^dag t with the CG update), timed per pair
    const int epi = (kernel == 0 || kernel == 3) ? EPI_STORE_NORM
                    : kernel == 1                ? EPI_STORE
                                                 : EPI_CG_UPDATE;
    if (kernel == 2 || kernel == 4) {
      e.stream = stream_cg_vectors(vg, precision, nc, nrhs);
      e.r = r;
      e.x = xlo;
      e.p = b;
      e.pring[0] = pprev;
      e.pring[1] = precision == P64 ? b : pr1;   // groups of 2 in FP64, else 4
      e.pring[2] = pr2;
      e.pring[3] = b;
      e.part_in = part_in;
      e.st = st;
      e.state_mode = 0;
    }
    const bool dag = kernel == 1 || kernel == 2 || kernel == 4;
    auto run = [&]() {
      if (eo) enqueue_schur(g, oa, precision, nl, dag, epi, a, w, e, nrhs, s);
      else launch_stencil(op, precision, nl, dag, epi, oa, a, e, nrhs, s);
    };
    run();   // warm-up
    hipEvent_t t0, t1;
    LQ_HIP(hipEventCreate(&t0));
    LQ_HIP(hipEventCreate(&t1));
    LQ_HIP(hipEventRecord(t0, s));
    for (int k = 0; k < reps; ++k) {
      e.par = (kernel == 2 || kernel == 4) ? (k & 1) : 0;
      if (kernel == 2 || kernel == 4) {
        const int G = precision == P64 ? 2 : 4;
        e.q4 = k % G;
        e.xstep = e.q4 == G - 1 ? G : 0;
      }
      run();
    }
    LQ_HIP(hipEventRecord(t1, s));
    LQ_HIP(hipEventSynchronize(t1));
    check_launch();
    float ms = 0.0f;
    LQ_HIP(hipEventElapsedTime(&ms, t0, t1));
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    *avg_ms = ms / reps;
    return LQ_OK;
  });
}

// -------------------------------------------------------------- solves
size_t lq_solve_workspace_bytes(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                                const lq_solve_opts* opts, int32_t nrhs) {
  if (!g || nrhs < 1) return 0;
  if (formulation != LQ_WILSON && formulation != LQ_STAGGERED_WILSON) return 0;
  if (g55_mode != LQ_G55_CORNERS && g55_mode != LQ_G55_ONTHEFLY) return 0;
  return Engine::workspace_bytes(g->g, formulation, g55_mode, opts, nrhs);
}

static void check_opts(const lq_solve_opts* o) {
  if (!o) return;
  check_prec(o->precision, o->links);
  need(o->reliable_interval >= 0 && o->poll_interval >= 0 && o->max_restarts >= 0,
       "negative option");
  need(std::isfinite(o->reliable_delta) && o->reliable_delta >= 0.0 && o->reliable_delta < 1.0,
       "reliable_delta must be in [0, 1)");
  need(o->evenodd == 0 || o->evenodd == 1, "evenodd must be 0 or 1");
}

int lq_cg_solve(const lq_gauge* g, const lq_dirac* d, const void* chi, void* x, double tol,
                int32_t maxiter, const lq_solve_opts* opts, void* ws, size_t ws_bytes,
                lq_solve_info* info, void* stream) {
  return lq_cg_solve_batch(g, d ? d->formulation : -1, d ? d->g55_mode : 0, d ? d->r : 0.0, 1,
                           d ? &d->mass : nullptr, chi, x, &tol, maxiter, opts, ws, ws_bytes, info,
                           stream);
}

int lq_cg_solve_batch(const lq_gauge* g, int32_t formulation, int32_t g55_mode, double r,
                      int32_t nrhs, const double* masses, const void* chi, void* x,
                      const double* tols, int32_t maxiter, const lq_solve_opts* opts, void* ws,
                      size_t ws_bytes, lq_solve_info* infos, void* stream) {
  return guard([&] {
    const auto t0 = std::chrono::steady_clock::now();
    need(g && masses && chi && x && tols && ws && infos, "null argument");
    lq_dirac d{formulation, g55_mode, masses[0], r};
    check_dirac(&d);
    check_opts(opts);
    need(nrhs >= 1 && maxiter >= 1, "nrhs and maxiter must be >= 1");
    hipStream_t s = S(stream);
    Engine e;
    e.init(g, formulation, g55_mode, r, nrhs, opts, ws, ws_bytes, s);
    const int nc = ncomp_of(formulation);
    const size_t field = (size_t)g->g.V * nc * 16;
    for (int k = 0; k < nrhs; ++k)
      e.load(k, (const char*)chi + k * field, masses[k], tols[k], maxiter, s);
    for (int k = 0; k < nrhs; ++k)
      if (e.hst[k].status == SLOT_FAILED && (e.hst[k].flags & 1))
        throw Error(LQ_ERR_ARG, "source " + std::to_string(k) + " gives a non-finite b = M^dag chi");
    while (e.running()) e.step(1 << 20, s);
    int worst = LQ_OK;
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < nrhs; ++k) {
      e.fetch(k, (char*)x + k * field, infos + k, s);
      infos[k].seconds = secs;
      const int st = infos[k].status;
      if (st < 0 && (worst >= 0 || st < worst)) worst = st;
      if (st > 0 && worst >= 0 && st > worst) worst = st;
    }
    if (worst != LQ_OK) g_last_error = "at least one system did not converge";
    return worst;
  });
}

// ------------------------------------------------------ pion correlator
size_t lq_pion_workspace_bytes(const lq_lattice* lat) {
  if (!lat) return 0;
  const int L4 = lat->g.L[3];
  Carver c(nullptr);
  c.take((size_t)L4 * pion_blocks_per_slice(L4) * sizeof(double));
  c.take((size_t)L4 * sizeof(double));
  return c.size();
}

int lq_pion_correlator(const lq_lattice* lat, int32_t nsrc, const void* props, double* corr,
                       double* meff, void* ws, size_t ws_bytes, void* stream) {
  return guard([&] {
    need(lat && props && corr && ws, "null argument");
    need(nsrc >= 1, "nsrc must be >= 1");
    const size_t nb = lq_pion_workspace_bytes(lat);
    if (ws_bytes < nb) throw Error(LQ_ERR_WORKSPACE, "pion workspace too small: need " + std::to_string(nb));
    const int L4 = lat->g.L[3];
    Carver c(ws);
    double* part = (double*)c.take((size_t)L4 * pion_blocks_per_slice(L4) * sizeof(double));
    double* dcorr = (double*)c.take((size_t)L4 * sizeof(double));
    hipStream_t s = S(stream);
    launch_pion_correlator(lat->g, nsrc, (const double2*)props, part, dcorr, s);
    check_launch();
    LQ_HIP(hipMemcpyAsync(corr, dcorr, (size_t)L4 * sizeof(double), hipMemcpyDeviceToHost, s));
    LQ_HIP(hipStreamSynchronize(s));
    if (meff) {
      // periodic cosh effective mass; NaN where no real solution exists
      for (int t = 0; t < L4; ++t) {
        const double q = (corr[(t + L4 - 1) % L4] + corr[(t + 1) % L4]) / (2.0 * corr[t]);
        meff[t] = q >= 1.0 ? std::acosh(q) : std::nan("");
      }
    }
    return LQ_OK;
  });
}

// -------------------------------------------------- continuous batching
struct lq_batch_s {
  Engine e;
};

int lq_batch_create(const lq_gauge* g, int32_t formulation, int32_t g55_mode, double r,
                    int32_t nslots, const lq_solve_opts* opts, void* ws, size_t ws_bytes,
                    lq_batch** out) {
  return guard([&] {
    need(g && ws && out, "null argument");
    lq_dirac d{formulation, g55_mode, 0.0, r};
    check_dirac(&d);
    check_opts(opts);
    need(nslots >= 1, "nslots must be >= 1");
    std::unique_ptr<lq_batch_s> b(new lq_batch_s);
    b->e.init(g, formulation, g55_mode, r, nslots, opts, ws, ws_bytes, nullptr);
    *out = b.release();
    return LQ_OK;
  });
}

int lq_batch_load(lq_batch* b, int32_t slot, const void* chi, double mass, double tol,
                  int32_t maxiter, void* stream) {
  return guard([&] {
    need(b != nullptr, "null batch");
    b->e.load(slot, chi, mass, tol, maxiter, S(stream));
    if (b->e.hst[slot].status == SLOT_FAILED && (b->e.hst[slot].flags & 1))
      throw Error(LQ_ERR_ARG, "source gives a non-finite b = M^dag chi");
    return LQ_OK;
  });
}

int lq_batch_step(lq_batch* b, int32_t iterations, int32_t* states, void* stream) {
  return guard([&] {
    need(b != nullptr && iterations >= 0, "bad argument");
    if (iterations > 0) b->e.step(iterations, S(stream));
    if (states)
      for (int k = 0; k < b->e.nslots; ++k) states[k] = b->e.hst[k].status;
    return LQ_OK;
  });
}

int lq_batch_fetch(lq_batch* b, int32_t slot, void* x, lq_solve_info* info, void* stream) {
  return guard([&] {
    need(b != nullptr, "null batch");
    b->e.fetch(slot, x, info, S(stream));
    return LQ_OK;
  });
}

int lq_batch_cancel(lq_batch* b, int32_t slot, void* stream) {
  return guard([&] {
    need(b != nullptr, "null batch");
    b->e.cancel(slot, S(stream));
    return LQ_OK;
  });
}

int lq_tuned_launch(const lq_gauge* g, const lq_dirac* d, int32_t precision, int32_t links,
                    int32_t nrhs, int32_t* rhs_per_thread, int32_t* window) {
  return guard([&] {
    need(g && rhs_per_thread && window, "null argument");
    check_dirac(d);
    check_prec(precision, links);
    need(nrhs >= 1, "nrhs must be >= 1");
    *rhs_per_thread = 1;
    *window = -3;   // what untuned launches use
    if (precision == LQ_PREC_F64 || nrhs < 2) return LQ_OK;
    const int nl = links_for(g, precision, links);
    const int v = tuned_rhs_per_thread(
        tune_key(g->g, opkind(d->formulation, d->g55_mode), precision, nl, nrhs));
    if (v == 0) throw Error(LQ_ERR_STATE, "no batch of this shape has been tuned");
    *rhs_per_thread = v & 15;
    *window = (v >> 4) - 3;
    return LQ_OK;
  });
}

int lq_batch_peek(lq_batch* b, int32_t slot, lq_solve_info* info, double* scale) {
  return guard([&] {
    need(b != nullptr && info != nullptr, "null argument");
    need(slot >= 0 && slot < b->e.nslots, "slot out of range");
    const SlotState& h = b->e.hst[slot];
    const double bn = h.bnorm2 > 0 ? h.bnorm2 : 1.0;
    info->status = h.status;
    info->iterations = h.iter;
    info->reliable_updates = h.ru;
    info->applications = h.apps + 1;
    info->iterated_residual = std::sqrt(h.iter_res2 / bn);
    info->true_residual = std::sqrt(h.true_res2 / bn);
    info->flags = h.flags;
    info->seconds = 0.0;
    if (scale) *scale = h.scale;
    return LQ_OK;
  });
}

void lq_batch_destroy(lq_batch* b) { delete b; }

// ---------------------------------------------------- staggered overlap
size_t lq_overlap_workspace_bytes(const lq_gauge* g, int32_t g55_mode) {
  if (!g || (g55_mode != LQ_G55_CORNERS && g55_mode != LQ_G55_ONTHEFLY)) return 0;
  return overlap_workspace_bytes(g->g, g55_mode);
}

int lq_overlap_apply(const lq_gauge* g, const lq_overlap* ov, const void* in, void* out,
                     void* ws, size_t ws_bytes, void* stream) {
  return guard([&] {
    need(g && ov && in && out && ws, "null argument");
    need(std::isfinite(ov->rho) && ov->rho > 0.0, "rho must be finite and > 0");
    need(std::isfinite(ov->mass) && std::isfinite(ov->r), "mass and r must be finite");
    need(std::isfinite(ov->lo) && std::isfinite(ov->hi) && ov->lo > 0.0 && ov->hi > ov->lo,
         "need 0 < lo < hi");
    need(ov->degree >= 1 && ov->degree <= 4096, "degree must be in [1, 4096]");
    need(ov->g55_mode == LQ_G55_CORNERS || ov->g55_mode == LQ_G55_ONTHEFLY, "bad g55_mode");
    overlap_apply(g, ov, in, out, ws, ws_bytes, S(stream));
    return LQ_OK;
  });
}

// ---------------------------------------------------- condition number
size_t lq_lanczos_workspace_bytes(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                                  int32_t steps) {
  if (!g || steps < 1 || steps > 1000) return 0;
  if (formulation != LQ_WILSON && formulation != LQ_STAGGERED_WILSON) return 0;
  if (g55_mode != LQ_G55_CORNERS && g55_mode != LQ_G55_ONTHEFLY) return 0;
  return lanczos_workspace_bytes(g->g, formulation, g55_mode, steps);
}

int lq_condition_number(const lq_gauge* g, const lq_dirac* d, int32_t steps, const void* v0,
                        void* ws, size_t ws_bytes, double* lmin, double* lmax, double* kappa,
                        double* alpha, double* beta, int32_t* steps_done, void* stream) {
  return guard([&] {
    need(g && v0 && ws && lmin && lmax && kappa, "null argument");
    check_dirac(d);
    std::vector<double> a, b;
    const int n = lanczos_run(g, d, steps, v0, ws, ws_bytes, a, b, S(stream));
    double lo, hi;
    tridiag_extremes(a, b, lo, hi);
    *lmin = lo;
    *lmax = hi;
    *kappa = hi / lo;
    if (alpha) for (int j = 0; j < n; ++j) alpha[j] = a[j];
    if (beta) for (int j = 0; j + 1 < n; ++j) beta[j] = b[j];
    if (steps_done) *steps_done = n;
    return LQ_OK;
  });
}

size_t lq_spectrum_workspace_bytes(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                                   int32_t steps) {
  if (!g || steps < 2 || steps > 500) return 0;
  if (formulation != LQ_WILSON && formulation != LQ_STAGGERED_WILSON) return 0;
  if (g55_mode != LQ_G55_CORNERS && g55_mode != LQ_G55_ONTHEFLY) return 0;
  return spectrum_workspace_bytes(g->g, formulation, g55_mode, steps);
}

int lq_spectrum(const lq_gauge* g, const lq_dirac* d, double sigma, int32_t steps,
                int32_t restarts, double tol, const void* v0, void* ws, size_t ws_bytes,
                int32_t* nev, double* eig_re, double* eig_im, double* resid, void* stream) {
  return guard([&] {
    need(g && v0 && ws && nev && eig_re && eig_im, "null argument");
    check_dirac(d);
    need(std::isfinite(sigma), "sigma must be finite");
    std::vector<cplx> eig;
    std::vector<double> res;
    const int n = spectrum_run(g, d, sigma, steps, restarts, tol, v0, ws, ws_bytes, eig, res,
                               S(stream));
    for (int k = 0; k < n; ++k) {
      eig_re[k] = eig[k].real();
      eig_im[k] = eig[k].imag();
      if (resid) resid[k] = res[k];
    }
    *nev = n;
    return LQ_OK;
  });
}

int lq_critical_mass(const lq_gauge* g, int32_t formulation, int32_t g55_mode, double r, double lo,
                     double hi, int32_t ngrid, int32_t ngolden, int32_t steps, const void* v0,
                     void* ws, size_t ws_bytes, double* m_c, double* theta_min, void* stream) {
  return guard([&] {
    need(g && v0 && ws && m_c && theta_min, "null argument");
    need(std::isfinite(lo) && std::isfinite(hi) && lo < hi, "need a finite bracket lo < hi");
    need(ngrid >= 3 && ngolden >= 0, "ngrid >= 3, ngolden >= 0");
    lq_dirac d{formulation, g55_mode, lo, r};
    check_dirac(&d);
    std::vector<std::pair<double, double>> trace;
    auto f = [&](double m) {
      d.mass = m;
      std::vector<double> a, b;
      lanczos_run(g, &d, steps, v0, ws, ws_bytes, a, b, S(stream));
      double tl, th;
      tridiag_extremes(a, b, tl, th);
      trace.emplace_back(m, tl);
      return tl;
    };
    // grid scan, then golden section on the bracket around the best grid point
    std::vector<double> grid(ngrid), val(ngrid);
    for (int k = 0; k < ngrid; ++k) {
      grid[k] = lo + (hi - lo) * k / (ngrid - 1);
      val[k] = f(grid[k]);
    }
    int kb = 0;
    for (int k = 1; k < ngrid; ++k) if (val[k] < val[kb]) kb = k;
    double a = grid[std::max(kb - 1, 0)], b = grid[std::min(kb + 1, ngrid - 1)];
    const double gr = (std::sqrt(5.0) - 1.0) / 2.0;
    double c = b - gr * (b - a), e = a + gr * (b - a);
    double fc = f(c), fe = f(e);
    for (int it = 0; it < ngolden; ++it) {
      if (fc < fe) { b = e; e = c; fe = fc; c = b - gr * (b - a); fc = f(c); }
      else { a = c; c = e; fc = fe; e = a + gr * (b - a); fe = f(e); }
    }
    size_t best = 0;
    for (size_t k = 1; k < trace.size(); ++k) if (trace[k].second < trace[best].second) best = k;
    *m_c = trace[best].first;
    *theta_min = trace[best].second;
    return LQ_OK;
  });
}

}  // extern "C"
