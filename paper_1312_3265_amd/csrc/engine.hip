// Host engine implementation: gauge layout, the slot-based CG engine and the
// Lanczos driver (see engine.h).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <cstdio>
#include <sstream>
#include <utility>
#include <vector>

#include "engine.h"
#include "stencil_tsweep.h"

const void* lq_gauge_s::links(int prec, int nl) const {
  using namespace lq;
  const void* p = nullptr;
  if (prec == P64 && (nl == 18 || nl == 12)) p = u64;   // FP64 12-real reads rows 0, 1 of the 18
  if (prec == P32 && nl == 18) p = u32_18;
  if (prec == P32 && nl == 12) p = u32_12;
  if (prec == P16 && nl == 12) p = u16_12;
  if (prec == P16 && nl == 18) p = u16_18;
  if (p && nl == 12) {
    // the third row is rebuilt as conj(row0 x row1): exact only for SU(3)
    const double lim = prec == P64 ? 1e-12 : 1e-6;
    if (!(su3_dev <= lim))
      throw Error(LQ_ERR_ARG, "12-real links need SU(3) links: row 2 differs from conj(row0 x row1) "
                              "by " + std::to_string(su3_dev));
  }
  if (!p)
    throw Error(LQ_ERR_ARG, "gauge field was not built for precision " + std::to_string(prec) +
                                " with " + std::to_string(nl) + "-real links (check features)");
  return p;
}

const void* lq_gauge_s::links_eo(int prec, int nl, int par) const {
  using namespace lq;
  if (!(features & LQ_FEAT_EO))
    throw Error(LQ_ERR_ARG, "gauge field has no even-odd link copies (LQ_FEAT_EO)");
  (void)links(prec, nl);   // the same storage checks as the lexicographic links
  const void* base = nullptr;
  int nstore = 0;
  size_t el = 0;
  if (prec == P64) { base = eo64; nstore = 9; el = 16; }
  if (prec == P32 && nl == 18) { base = eo32_18; nstore = 9; el = 8; }
  if (prec == P32 && nl == 12) { base = eo32_12; nstore = 6; el = 8; }
  if (prec == P16 && nl == 12) { base = eo16_12; nstore = 6; el = 4; }
  if (prec == P16 && nl == 18) { base = eo16_18; nstore = 9; el = 4; }
  if (!base)
    throw Error(LQ_ERR_ARG, "gauge field has no even-odd links for precision " +
                                std::to_string(prec) + " with " + std::to_string(nl) + " reals");
  const size_t half = (size_t)4 * nstore * half_geom(g).Vp * el;
  return (const char*)base + par * half;
}

const void* lq_gauge_s::corners(int prec) const {
  using namespace lq;
  const void* p = prec == P64 ? (const void*)c64 : prec == P32 ? (const void*)c32 : (const void*)c16;
  if (!p)
    throw Error(LQ_ERR_ARG, "gauge field has no corner matrices for precision " +
                                std::to_string(prec) + " (LQ_FEAT_CORNERS)");
  return p;
}

namespace lq {

size_t gauge_layout(const Geom& g, uint32_t f, void* base, lq_gauge_s* out) {
  Carver c(base);
  const size_t Vp = g.Vp;
  double2* u64 = (double2*)c.take(36 * Vp * 16);
  float2 *u32_18 = nullptr, *u32_12 = nullptr, *c32 = nullptr;
  short2 *u16_12 = nullptr, *u16_18 = nullptr, *c16 = nullptr;
  double2* c64 = nullptr;
  if (f & LQ_FEAT_F32) {
    u32_18 = (float2*)c.take(36 * Vp * 8);
    u32_12 = (float2*)c.take(24 * Vp * 8);
  }
  if (f & LQ_FEAT_Q16) {
    u16_12 = (short2*)c.take(24 * Vp * 4);
    u16_18 = (short2*)c.take(36 * Vp * 4);
  }
  void *eo64 = nullptr, *eo32_18 = nullptr, *eo32_12 = nullptr, *eo16_12 = nullptr,
       *eo16_18 = nullptr;
  if (f & LQ_FEAT_EO) {
    const size_t Vhp = half_geom(g).Vp;
    eo64 = c.take(2 * 36 * Vhp * 16);
    if (f & LQ_FEAT_F32) {
      eo32_18 = c.take(2 * 36 * Vhp * 8);
      eo32_12 = c.take(2 * 24 * Vhp * 8);
    }
    if (f & LQ_FEAT_Q16) {
      eo16_12 = c.take(2 * 24 * Vhp * 4);
      eo16_18 = c.take(2 * 36 * Vhp * 4);
    }
  }
  if (f & LQ_FEAT_CORNERS) {
    c64 = (double2*)c.take(72 * Vp * 16);
    if (f & LQ_FEAT_F32) c32 = (float2*)c.take(72 * Vp * 8);
    if (f & LQ_FEAT_Q16) c16 = (short2*)c.take(72 * Vp * 4);
  }
  const int nbp = nbp_of(g.V);
  double* scratch = (double*)c.take((nbp + 8) * sizeof(double));
  double2* stage = (double2*)c.take((size_t)std::min(g.V, kStageSites) * 36 * 16);
  if (out) {
    out->g = g;
    out->features = f;
    out->u64 = u64; out->u32_18 = u32_18; out->u32_12 = u32_12; out->u16_12 = u16_12;
    out->u16_18 = u16_18;
    out->eo64 = eo64; out->eo32_18 = eo32_18; out->eo32_12 = eo32_12;
    out->eo16_12 = eo16_12; out->eo16_18 = eo16_18;
    out->c64 = c64; out->c32 = c32; out->c16 = c16;
    out->scratch = scratch;
    out->stage = stage;
    out->nbp = nbp;
  }
  return c.size();
}

// =============================================================== autotune
static std::mutex g_tune_mu;
static std::map<std::string, int>* g_tune = nullptr;

static std::string tune_path() {
  const char* e = std::getenv("LQ_TUNE_CACHE");
  if (e && *e) return e;
  const char* h = std::getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/lq_tune.txt";
}

static void tune_load_locked() {
  if (g_tune) return;
  g_tune = new std::map<std::string, int>();
  std::ifstream f(tune_path());
  std::string k;
  int v;
  while (f >> k >> v) (*g_tune)[k] = v;
}

int tuned_rhs_per_thread(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune->find(key);
  return it == g_tune->end() ? 0 : it->second;
}

void remember_rhs_per_thread(const std::string& key, int k) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  (*g_tune)[key] = k;
  std::ofstream f(tune_path(), std::ios::app);   // best effort
  if (f) f << key << " " << k << "\n";
}

std::string tune_key(const Geom& g, int op, int prec, int nl, int nslots) {
  hipDeviceProp_t prop;
  int dev = 0;
  LQ_HIP(hipGetDevice(&dev));
  LQ_HIP(hipGetDeviceProperties(&prop, dev));
  std::ostringstream key;
  key << "v13:" << prop.gcnArchName << ":" << g.L[0] << "x" << g.L[1] << "x" << g.L[2] << "x" << g.L[3]
      << ":op" << op << ":p" << prec << ":l" << nl << ":n" << nslots;
  std::string k = key.str();
  for (auto& ch : k) if (ch == ' ') ch = '_';
  return k;
}

// Time the two stencils of a CG iteration (t = M p + ||t||^2, then the M^dag
// stencil with the x, r updates) over all slots for every systems-per-thread
// K and block order that keeps the links in L2 across systems, on the
// (zeroed) solver buffers, and keep the fastest.
void Engine::tune(hipStream_t s) {
  rhs_per_thread = 1;
  window = -3;   // tiled order where the lattice allows it (the plain order elsewhere)
  if (prec_lo == P64 || nslots < 2) return;
  // LQ_LAUNCH="K,window" forces the launch configuration (testing every
  // block order against the tuned one); it is not remembered
  // K = 8: the lanes stencil (four systems across the lanes of a site, link
  // products on the matrix cores): unpreconditioned r = 1 Wilson, 18-real
  // links, on request only (LQ_LAUNCH)
  const bool lanes_ok = op == OP_WILSON && r == 1.0 && nl_lo == 18;
  if (const char* f = std::getenv("LQ_LAUNCH")) {
    int kk = 1, w = 0;
    if (std::sscanf(f, "%d,%d", &kk, &w) == 2 && (kk == 1 || kk == 2 || kk == 4 || kk == 8) &&
        (w >= -4 || (kk == 1 && w <= -11 && w >= -16))) {
      // the lanes stencil applies to r = 1 Wilson with 18-real links only;
      // elsewhere K = 8 runs the one-system kernels
      rhs_per_thread = (kk == 8 && !lanes_ok) ? 1 : kk;
      window = w;
      return;
    }
    throw Error(LQ_ERR_ARG, std::string("LQ_LAUNCH must be \"K,window\" with K in {1,2,4,8} and "
                                        "window >= -4 (or, for K = 1, a t-sweep order -11 ... -16), "
                                        "got ") + f);
  }
  const std::string k = tune_key(gauge->g, op, prec_lo, nl_lo, nslots);
  const int cached = tuned_rhs_per_thread(k);   // encoded as K + 16 * (window + 3)
  if (cached) { rhs_per_thread = cached & 15; window = (cached >> 4) - 3; return; }
  EpiArgs e = epi_base();
  e.st = nullptr;
  e.out = t;
  e.part = part_t;
  // the iteration's second stencil on the (zeroed) solver state: alpha = 0,
  // the same traffic; slot loads rewrite every state word it touches
  EpiArgs f = epi_base();
  f.state_mode = 0;
  f.part = part_r;
  f.part_in = part_t;
  f.x = xlo; f.r = rlo;
  const PRing rg = ring();
  for (int j = 0; j < 4; ++j) f.pring[j] = rg.p[j];
  f.p = p;
  hipEvent_t t0, t1;
  LQ_HIP(hipEventCreate(&t0));
  LQ_HIP(hipEventCreate(&t1));
  // the lanes stencil (8) is not a candidate: exact, but slower than one
  // system per thread (it is selected explicitly with LQ_LAUNCH).
  // The system-major orders (-1, -2) are left out: every XCD then needs all
  // the links, which alone on the GPU the last-level cache hides, but with
  // other batches in flight they are fetched again per system (16^3x32, 36
  // Wilson systems, two batches in flight: 84 solves/s with -2, 100 with -3).
  // Every candidate is timed twice, in two passes of opposite order, and
  // keeps its faster time, so that work of other streams running meanwhile
  // (a caller's concurrent batches) is less likely to decide the choice.
  std::vector<std::pair<int, int>> cand;
  for (int kk : {1, 2, 4})
    if (kk <= nslots)
      for (int w : {1, 2, 4, 0, -3, -4}) cand.push_back({kk, w});
  // the t-sweeping Wilson stencils (16-bit, one system per thread; bitwise
  // the same results as the orders above)
  if (op == OP_WILSON && r == 1.0 && prec_lo == P16)
    for (int w = -11; w >= -16; --w) {
      int T = 0;
      bool xy = false;
      if (tsweep_lo_code(w, T, xy) && tsweep_lo_ok(gauge->g, T, xy)) cand.push_back({1, w});
    }
  std::vector<float> tbest(cand.size(), 1e30f);
  for (int pass = 0; pass < 2; ++pass) {
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      const size_t c = pass == 0 ? ci : cand.size() - 1 - ci;
      e.rhs_per_thread = f.rhs_per_thread = cand[c].first;
      e.window = f.window = cand[c].second;
      stencil(prec_lo, nl_lo, false, EPI_STORE_NORM, p, e, nslots, s);
      stencil(prec_lo, nl_lo, true, EPI_CG_UPDATE, t, f, nslots, s);
      LQ_HIP(hipEventRecord(t0, s));
      for (int r = 0; r < 4; ++r) {   // whole groups: the last iteration also advances x
        const int q = r % group;
        e.par = f.par = r & 1;
        f.q4 = q;
        f.xstep = q == group - 1 ? group : 0;
        f.p = rg.p[q];
        stencil(prec_lo, nl_lo, false, EPI_STORE_NORM, rg.p[q], e, nslots, s);
        stencil(prec_lo, nl_lo, true, EPI_CG_UPDATE, t, f, nslots, s);
      }
      e.par = f.par = 0;
      f.q4 = f.xstep = 0;
      f.p = p;
      LQ_HIP(hipEventRecord(t1, s));
      LQ_HIP(hipEventSynchronize(t1));
      check_launch();
      float ms = 0.0f;
      LQ_HIP(hipEventElapsedTime(&ms, t0, t1));
      tbest[c] = std::min(tbest[c], ms);
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  int bestk = 1, bestw = 0;
  float best = 1e30f;
  for (size_t c = 0; c < cand.size(); ++c)
    if (tbest[c] < best) { best = tbest[c]; bestk = cand[c].first; bestw = cand[c].second; }
  rhs_per_thread = bestk;
  window = bestw;
  remember_rhs_per_thread(k, bestk + 16 * (bestw + 3));
}

// ======================================================== even-odd blocks
void enqueue_schur(const lq_gauge_s* g, const OpArgs& base, int prec, int nl, bool dag, int epi,
                   const void* in, void* w, const EpiArgs& e, int nrhs, hipStream_t s) {
  OpArgs o1 = base;
  o1.g = half_geom(g->g);
  o1.links = g->links_eo(prec, nl, 1);
  o1.links_nb = g->links_eo(prec, nl, 0);
  o1.eo_par = 1;
  o1.eo_schur = 0;
  o1.diag_in = nullptr;
  EpiArgs e1 = e;
  e1.out = w;
  launch_stencil(OP_WILSON_EO, prec, nl, dag, EPI_STORE, o1, in, e1, nrhs, s);
  OpArgs o2 = o1;
  o2.links = g->links_eo(prec, nl, 0);
  o2.links_nb = g->links_eo(prec, nl, 1);
  o2.eo_par = 0;
  o2.eo_schur = 1;
  o2.diag_in = in;
  launch_stencil(OP_WILSON_EO, prec, nl, dag, epi, o2, w, e, nrhs, s);
}

// ================================================================ Engine
static int prec_of(const lq_solve_opts* o) { return o ? o->precision : LQ_PREC_F64; }

size_t Engine::workspace_bytes(const Geom& g0, int formulation, int g55,
                               const lq_solve_opts* opts, int nslots) {
  const int nc = ncomp_of(formulation);
  const int prec = prec_of(opts);
  const bool eo = opts && opts->evenodd;
  const Geom vg = eo ? half_geom(g0) : g0;
  const Geom& g = vg;
  const size_t vhi = (size_t)nslots * nc * g.Vp * 16;
  const size_t vlo = (size_t)nslots * field_bytes(g, prec, nc);
  const int nbp = nbp_of(g.V);
  Carver c(nullptr);
  c.take(vhi); c.take(vhi); c.take(vhi);      // b, x_hi, r_hi
  if (eo) {                                   // wbuf, chio, bhat, part_f, part_g
    c.take(vhi); c.take(vhi); c.take(vhi);
    c.take((size_t)nslots * nbp * sizeof(double));
    c.take((size_t)nslots * nbp * sizeof(double));
  }
  if (prec != P64) c.take(vhi);               // t64 (shares t when FP64)
  const size_t vx = (size_t)nslots * nc * g.Vp * store_bytes(prec == P16 ? P32 : prec);
  c.take(vx); c.take(vlo);                    // x_lo, r_lo
  const int ndir = prec == P64 ? 2 : 4;       // search directions, one per step of a group
  for (int k = 0; k < ndir + 1; ++k) c.take(vlo);   // ... and t
  for (int k = 0; k < 3; ++k) c.take((size_t)nslots * nbp * sizeof(double));
  c.take((size_t)nslots * sizeof(SlotState));
  c.take((size_t)nslots * sizeof(int));
  if (opkind(formulation, g55) == OP_SW_OTF) c.take((size_t)nslots * g55_bytes_per_system(g, P64));
  return c.size();
}

void Engine::init(const lq_gauge_s* g, int form, int g55, double rr, int ns,
                  const lq_solve_opts* opts, void* ws, size_t ws_bytes, hipStream_t s) {
  gauge = g;
  formulation = form;
  op = opkind(form, g55);
  nc = ncomp_of(form);
  r = rr;
  nslots = ns;
  eo = opts && opts->evenodd;
  if (eo) {
    if (form != LQ_WILSON || rr != 1.0)
      throw Error(LQ_ERR_ARG, "even-odd preconditioning is built for Wilson with r = 1");
    op = OP_WILSON_EO;
  }
  vg = eo ? half_geom(g->g) : g->g;
  prec_lo = prec_of(opts);
  nl_lo = (opts && opts->links) ? opts->links : (prec_lo == P16 ? 12 : 18);
  if (prec_lo == P64) nl_lo = (opts && opts->links) ? opts->links : g->fp64_links();
  if (opts) {
    if (opts->reliable_interval > 0) reliable_interval = opts->reliable_interval;
    if (opts->poll_interval > 0) poll_every = opts->poll_interval;
    use_graph = opts->use_graph;
    if (opts->max_restarts > 0) max_cand = opts->max_restarts;
  }
  delta = prec_lo == P16 ? 0.1 : (prec_lo == P32 ? 1e-3 : 0.0);
  if (opts && opts->reliable_delta > 0.0 && prec_lo != P64) delta = opts->reliable_delta;
  group = prec_lo == P64 ? 2 : 4;
  poll_every = (poll_every + 3) & ~3;   // whole groups of iterations
  if (poll_every < 4) poll_every = 4;
  // validate the stencil storage now (throws for a missing feature)
  (void)g->links(prec_lo, nl_lo);
  (void)g->links(P64, 18);
  if (eo) { (void)g->links_eo(prec_lo, nl_lo, 0); (void)g->links_eo(P64, g->fp64_links(), 0); }
  if (op == OP_SW_CORNERS) { (void)g->corners(prec_lo); (void)g->corners(P64); }

  const size_t need = workspace_bytes(g->g, form, g55, opts, ns);
  if (!ws || ws_bytes < need)
    throw Error(LQ_ERR_WORKSPACE, "solver workspace too small: need " + std::to_string(need) +
                                      " bytes, got " + std::to_string(ws_bytes));
  nbp = nbp_of(vg.V);
  const size_t vhi = (size_t)ns * nc * vg.Vp * 16;
  const size_t vlo = (size_t)ns * field_bytes(vg, prec_lo, nc);
  Carver c(ws);
  b = (double2*)c.take(vhi);
  xhi = (double2*)c.take(vhi);
  rhi = (double2*)c.take(vhi);
  if (eo) {
    wbuf = (double2*)c.take(vhi);
    chio = (double2*)c.take(vhi);
    bhat = (double2*)c.take(vhi);
    part_f = (double*)c.take((size_t)ns * nbp * sizeof(double));
    part_g = (double*)c.take((size_t)ns * nbp * sizeof(double));
  }
  if (prec_lo != P64) t64 = (double2*)c.take(vhi);
  xlo = c.take((size_t)ns * nc * vg.Vp * store_bytes(prec_lo == P16 ? P32 : prec_lo));
  rlo = c.take(vlo);
  p = c.take(vlo);
  p1 = c.take(vlo);
  p2 = group == 4 ? c.take(vlo) : nullptr;
  p3 = group == 4 ? c.take(vlo) : nullptr;
  t = c.take(vlo);
  if (prec_lo == P64) t64 = (double2*)t;
  part_t = (double*)c.take((size_t)ns * nbp * sizeof(double));
  part_r = (double*)c.take((size_t)ns * nbp * sizeof(double));
  part_u = (double*)c.take((size_t)ns * nbp * sizeof(double));
  st = (SlotState*)c.take((size_t)ns * sizeof(SlotState));
  mask = (int*)c.take((size_t)ns * sizeof(int));
  if (op == OP_SW_OTF) g55w = c.take((size_t)ns * g55_bytes_per_system(vg, P64));
  // zero the whole workspace once: plane padding stays zero afterwards
  launch_fill_zero(ws, c.size(), s);
  check_launch();
  LQ_HIP(hipHostMalloc((void**)&hst, sizeof(SlotState) * ns, hipHostMallocDefault));
  std::memset(hst, 0, sizeof(SlotState) * ns);
  LQ_HIP(hipHostMalloc((void**)&hmask, sizeof(int) * ns, hipHostMallocDefault));
  std::memset(hmask, 0, sizeof(int) * ns);
  tune(s);
  LQ_HIP(hipStreamSynchronize(s));
}

Engine::~Engine() {
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  if (hst) (void)hipHostFree(hst);
  if (hmask) (void)hipHostFree(hmask);
}

OpArgs Engine::op_args(int prec, int nl) const {
  OpArgs a;
  a.g = gauge->g;
  a.links = gauge->links(prec, nl);
  a.corners = op == OP_SW_CORNERS ? gauge->corners(prec) : nullptr;
  a.r = r;
  a.mass0 = 0.0;
  a.mass = &st[0].mass;
  a.mass_stride = sizeof(SlotState) / sizeof(double);
  if (op == OP_SW_OTF) {
    a.g55w = g55w;
    a.g55_sys = g55_bytes_per_system(vg, prec);
  }
  return a;
}

void Engine::stencil(int prec, int nl, bool dag, int epi, const void* in, const EpiArgs& e,
                     int n, hipStream_t s) const {
  if (eo) enqueue_schur(gauge, op_args(prec, nl), prec, nl, dag, epi, in, wbuf, e, n, s);
  else launch_stencil(op, prec, nl, dag, epi, op_args(prec, nl), in, e, n, s);
}

void Engine::eo_form(int par, int form, bool dag, const void* diag, const void* in, EpiArgs e,
                     int epi, int nrhs, hipStream_t s) const {
  const int nl = gauge->fp64_links();
  OpArgs o = op_args(P64, nl);
  o.g = vg;
  o.links = gauge->links_eo(P64, nl, par);
  o.links_nb = gauge->links_eo(P64, nl, par ^ 1);
  o.eo_par = par;
  o.eo_schur = form;
  o.diag_in = diag;
  launch_stencil(OP_WILSON_EO, P64, nl, dag, epi, o, in, e, nrhs, s);
}

EpiArgs Engine::epi_base() const {
  EpiArgs e;
  std::memset(&e, 0, sizeof(e));
  e.nbp = nbp;
  e.st = st;
  e.stream = stream_cg_vectors(vg, prec_lo, nc, nslots);
  return e;
}

int Engine::running() const {
  int n = 0;
  for (int k = 0; k < nslots; ++k) n += hst[k].status == SLOT_RUNNING;
  return n;
}

void Engine::load(int slot, const void* chi, double mass, double tol, int maxiter,
                  hipStream_t s) {
  if (slot < 0 || slot >= nslots) throw Error(LQ_ERR_ARG, "slot out of range");
  if (!chi) throw Error(LQ_ERR_ARG, "null source");
  if (!std::isfinite(mass) || !std::isfinite(tol) || tol <= 0.0 || maxiter <= 0)
    throw Error(LQ_ERR_ARG, "mass and tol must be finite, tol > 0, maxiter > 0");
  if (hst[slot].status == SLOT_RUNNING) throw Error(LQ_ERR_STATE, "slot is busy");
  SlotState init;
  std::memset(&init, 0, sizeof(init));
  init.status = SLOT_RUNNING;
  init.mass = mass;
  init.tol = tol;
  init.maxiter = maxiter;
  init.scale = init.scale_prev = 1.0;
  init.delta2 = delta * delta;
  hst[slot] = init;
  LQ_HIP(hipMemcpyAsync(st + slot, hst + slot, sizeof(SlotState), hipMemcpyHostToDevice, s));
  const Geom& g = vg;
  const int nl64 = gauge->fp64_links();
  EpiArgs e = epi_base();
  e.out = b; e.part = part_u; e.k0 = slot; e.state_mode = 2;
  if (eo) {
    // chi_e (in t64), chi_o (kept); b^_e = chi_e - M_eo chi_o / d (in r_hi);
    // b = M^dag b^_e with ||b||^2
    launch_field_in(P64, nc, g, chi, 1, t64, nbp, slot, 1, s, 0);
    launch_field_in(P64, nc, g, chi, 1, chio, nbp, slot, 1, s, 1);
    EpiArgs h = e;
    h.out = bhat;
    eo_form(0, 2, false, t64, chio, h, EPI_STORE, 1, s);
    stencil(P64, nl64, true, EPI_STORE_NORM, bhat, e, 1, s);
    // ||M^dag chi||^2 of eq. (2) from its even and odd halves
    h.out = wbuf;
    h.part = part_f;
    eo_form(0, 4, true, t64, chio, h, EPI_STORE_NORM, 1, s);
    h.part = part_g;
    eo_form(1, 4, true, chio, t64, h, EPI_STORE_NORM, 1, s);
  } else {
    // chi -> FP64 SoA (in t64), b = M^dag chi with ||b||^2
    launch_field_in(P64, nc, g, chi, 1, t64, nbp, slot, 1, s);
    stencil(P64, nl64, true, EPI_STORE_NORM, t64, e, 1, s);
  }
  launch_load_prepare(prec_lo, nc, g, (double*)xhi, xlo, (double*)rhi, (const double*)b, nbp, slot,
                      1, s);
  const double ncomp = (double)nc * g.V;
  launch_ru_finish(st, nullptr, part_u, eo ? part_f : nullptr, eo ? part_g : nullptr, nbp, slot, 1,
                   ncomp, prec_lo != P64, max_cand, 1, 0, s);
  launch_ru_convert(prec_lo, nc, g, st, nullptr, (const double*)rhi, rlo, ring(), part_u, nbp, 1, slot,
                    1, s);
  launch_ru_commit(st, nullptr, part_u, nbp, slot, 1, s);
  check_launch();
  LQ_HIP(hipMemcpyAsync(hst + slot, st + slot, sizeof(SlotState), hipMemcpyDeviceToHost, s));
  LQ_HIP(hipStreamSynchronize(s));
}

void Engine::enqueue_iterations(int n, hipStream_t s) {
  // n is a multiple of four (so of the group size): a chunk starts and ends
  // with p_k in ring buffer 0; x advances on the last iteration of each
  // group, by the group's steps
  const PRing rg = ring();
  for (int it = 0; it < n; ++it) {
    const int par = it & 1, q = it % group;
    void* pk = rg.p[q];                 // p_k
    void* pn = rg.p[(q + 1) % group];   // receives p_{k+1}; its old direction is already in x
    EpiArgs e = epi_base();
    e.par = par;
    e.state_mode = 1;
    e.out = t;
    e.part = part_t;
    e.rhs_per_thread = rhs_per_thread;
    e.window = window;
    stencil(prec_lo, nl_lo, false, EPI_STORE_NORM, pk, e, nslots, s);
    EpiArgs f = epi_base();
    f.rhs_per_thread = rhs_per_thread;
    f.window = window;
    f.par = par;
    f.q4 = q;
    f.xstep = q == group - 1 ? group : 0;
    f.state_mode = 1;
    f.part = part_r;
    f.part_in = part_t;
    f.x = xlo; f.r = rlo; f.p = pk;
    for (int j = 0; j < 4; ++j) f.pring[j] = rg.p[j];
    stencil(prec_lo, nl_lo, true, EPI_CG_UPDATE, t, f, nslots, s);
    launch_p_update(prec_lo, nc, vg, st, par, (q + 1) % group, part_r, nbp, pk, pn, rlo, 0, nslots, s);
  }
}

void Engine::enqueue_reliable_update(hipStream_t s) {
  const Geom& g = vg;
  const int nl64 = gauge->fp64_links();
  LQ_HIP(hipMemcpyAsync(mask, hmask, sizeof(int) * nslots, hipMemcpyHostToDevice, s));
  launch_ru_accumulate(prec_lo, nc, g, st, mask, (double*)xhi, xlo, ring(), nbp, 0, nslots, s);
  EpiArgs e = epi_base();
  e.state_mode = 2;
  e.ru_mask = mask;
  EpiArgs f = epi_base();
  f.state_mode = 2;
  f.ru_mask = mask;
  f.out = rhi;
  f.part = part_u;
  if (eo) {
    // r^ = b^ - M^ x_hi (in t64) with ||r^||^2, ||M_eo^dag r^||^2, and the
    // residual of the iterated normal equations r_hi = M^dag r^
    e.out = t64;
    e.b = bhat;
    e.part = part_f;
    stencil(P64, nl64, false, EPI_RESID, xhi, e, nslots, s);
    EpiArgs h = e;
    h.out = wbuf;
    h.part = part_g;
    eo_form(1, 0, true, nullptr, t64, h, EPI_STORE_NORM, nslots, s);
    stencil(P64, nl64, true, EPI_STORE_NORM, t64, f, nslots, s);
  } else {
    e.out = t64;
    stencil(P64, nl64, false, EPI_STORE, xhi, e, nslots, s);
    f.b = b;
    stencil(P64, nl64, true, EPI_RESID, t64, f, nslots, s);
  }
  launch_ru_finish(st, mask, part_u, eo ? part_f : nullptr, eo ? part_g : nullptr, nbp, 0, nslots,
                   (double)nc * g.V, prec_lo != P64, max_cand, 0, 0, s);
  launch_ru_convert(prec_lo, nc, g, st, mask, (const double*)rhi, rlo, ring(), part_u, nbp, 0, 0, nslots,
                    s);
  launch_ru_commit(st, mask, part_u, nbp, 0, nslots, s);
  check_launch();
}

void Engine::poll(hipStream_t s) {
  LQ_HIP(hipMemcpyAsync(hst, st, sizeof(SlotState) * nslots, hipMemcpyDeviceToHost, s));
  LQ_HIP(hipStreamSynchronize(s));
}

// Choose, per slot and from that slot's state alone, whether the next chunk
// boundary performs a reliable update: frozen slots (iterated residual met
// tol, breakdown or maxiter) to confirm or finalise, and in mixed precision
// every `reliable_interval` iterations.
bool Engine::select_updates() {
  bool any = false;
  for (int k = 0; k < nslots; ++k) {
    const SlotState& h = hst[k];
    int sel = 0;
    if (h.status == SLOT_RUNNING) {
      if (h.stop[0] || h.flags) sel = 1;
      if (prec_lo != P64 && h.iter - h.ru_iter >= reliable_interval) sel = 1;
    }
    hmask[k] = sel;
    any = any || sel;
  }
  return any;
}

void Engine::step(int iters, hipStream_t s) {
  int done = 0;
  while (done < iters) {
    if (!running()) return;
    if (select_updates()) {
      enqueue_reliable_update(s);
      poll(s);
      if (!running()) return;
    }
    const int n = poll_every;
    bool graphed = false;
    if (use_graph && s != nullptr) {
      if (!gexec || gchunk != n || gstream != s) {
        if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; }
        if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
        LQ_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
          enqueue_iterations(n, s);
        } catch (...) {
          hipGraph_t tmp;
          (void)hipStreamEndCapture(s, &tmp);
          if (tmp) (void)hipGraphDestroy(tmp);
          throw;
        }
        LQ_HIP(hipStreamEndCapture(s, &graph));
        LQ_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        gchunk = n;
        gstream = s;
      }
      LQ_HIP(hipGraphLaunch(gexec, s));
      graphed = true;
    }
    if (!graphed) enqueue_iterations(n, s);
    check_launch();
    done += n;
    poll(s);
  }
  if (running() && select_updates()) {
    enqueue_reliable_update(s);
    poll(s);
  }
}

void Engine::fetch(int slot, void* x, lq_solve_info* info, hipStream_t s) {
  if (slot < 0 || slot >= nslots) throw Error(LQ_ERR_ARG, "slot out of range");
  SlotState& h = hst[slot];
  if (h.status == SLOT_EMPTY) throw Error(LQ_ERR_STATE, "slot is empty");
  if (h.status == SLOT_RUNNING) throw Error(LQ_ERR_STATE, "slot is still running");
  if (x && eo) {
    // x_e, and x_o = (chi_o - M_oe x_e) / d
    EpiArgs e = epi_base();
    e.out = wbuf;
    e.k0 = slot;
    e.state_mode = 0;   // the slot's mass from its state, whatever its status
    eo_form(1, 3, false, chio, xhi, e, EPI_STORE, 1, s);
    launch_field_out(P64, nc, vg, xhi, x, 1, nbp, slot, 1, s, 0);
    launch_field_out(P64, nc, vg, wbuf, x, 1, nbp, slot, 1, s, 1);
  } else if (x) {
    launch_field_out(P64, nc, vg, xhi, x, 1, nbp, slot, 1, s);
  }
  check_launch();
  if (info) {
    const double bn = h.bnorm2 > 0 ? h.bnorm2 : 1.0;
    info->status = h.status == SLOT_DONE ? LQ_OK
                   : (h.flags & 1)       ? LQ_ERR_BREAKDOWN
                   : (h.flags & 4)       ? LQ_STAGNATION
                                         : LQ_NOT_CONVERGED;
    info->flags = h.flags;
    info->iterations = h.iter;
    info->reliable_updates = h.ru;
    info->applications = h.apps + 1;   // + b = M^dag chi
    info->iterated_residual = std::sqrt(h.iter_res2 / bn);
    // the residual of eq. (2) for the whole solution (with even-odd
    // preconditioning too; the iterated residual is then the Schur system's)
    info->true_residual = eo ? std::sqrt(h.full_res2 / (h.bfull2 > 0 ? h.bfull2 : 1.0))
                             : std::sqrt(h.true_res2 / bn);
    info->seconds = 0.0;
  }
  h.status = SLOT_EMPTY;
  LQ_HIP(hipMemcpyAsync(&st[slot].status, &h.status, sizeof(int32_t), hipMemcpyHostToDevice, s));
  LQ_HIP(hipStreamSynchronize(s));
}

// Discards slot `slot` (running or finished) without copying anything out.
// Between steps no kernel of this engine is in flight (step and fetch
// synchronise), so marking the slot empty on the device takes effect from the
// next launch on: every kernel skips slots that are not running.
void Engine::cancel(int slot, hipStream_t s) {
  if (slot < 0 || slot >= nslots) throw Error(LQ_ERR_ARG, "slot out of range");
  SlotState& h = hst[slot];
  if (h.status == SLOT_EMPTY) throw Error(LQ_ERR_STATE, "slot is empty");
  h.status = SLOT_EMPTY;
  LQ_HIP(hipMemcpyAsync(&st[slot].status, &h.status, sizeof(int32_t), hipMemcpyHostToDevice, s));
  LQ_HIP(hipStreamSynchronize(s));
}

// =============================================================== Lanczos
static constexpr int kLzBlocks = 256;

size_t lanczos_workspace_bytes(const Geom& g, int formulation, int g55, int steps) {
  const int nc = ncomp_of(formulation);
  const size_t vec = (size_t)nc * g.Vp * 16;
  Carver c(nullptr);
  c.take(vec * (steps + 1));                                // basis
  c.take(vec);                                              // w
  c.take(vec);                                              // t
  c.take((size_t)(steps + 1) * 16);                         // h
  c.take((size_t)(steps + 1) * kLzBlocks * 2 * 8);          // part_h
  c.take((size_t)nbp_of(g.V) * 8);                          // alpha partials
  c.take((size_t)kLzBlocks * 8);                            // norm partials
  c.take((size_t)(steps + 2) * 8 * 2);                      // alpha, beta
  if (opkind(formulation, g55) == OP_SW_OTF) c.take(g55_bytes_per_system(g, P64));
  return c.size();
}

int lanczos_run(const lq_gauge_s* gs, const lq_dirac* d, int steps, const void* v0, void* ws,
                size_t ws_bytes, std::vector<double>& alpha, std::vector<double>& beta,
                hipStream_t s) {
  const Geom& g = gs->g;
  const int nc = ncomp_of(d->formulation);
  const int op = opkind(d->formulation, d->g55_mode);
  if (steps < 1 || steps > 1000) throw Error(LQ_ERR_ARG, "steps must be in [1, 1000]");
  const size_t need = lanczos_workspace_bytes(g, d->formulation, d->g55_mode, steps);
  if (!ws || ws_bytes < need)
    throw Error(LQ_ERR_WORKSPACE, "Lanczos workspace too small: need " + std::to_string(need));
  const size_t n = (size_t)nc * g.Vp;
  const size_t vec = n * 16;
  Carver c(ws);
  double2* V = (double2*)c.take(vec * (steps + 1));
  double2* w = (double2*)c.take(vec);
  double2* t = (double2*)c.take(vec);
  double2* h = (double2*)c.take((size_t)(steps + 1) * 16);
  double* part_h = (double*)c.take((size_t)(steps + 1) * kLzBlocks * 2 * 8);
  const int nbp = nbp_of(g.V);
  double* part_a = (double*)c.take((size_t)nbp * 8);
  double* part_n = (double*)c.take((size_t)kLzBlocks * 8);
  double* ad = (double*)c.take((size_t)(steps + 2) * 8 * 2);
  double* bd = ad + steps + 2;
  void* g55w = op == OP_SW_OTF ? c.take(g55_bytes_per_system(g, P64)) : nullptr;
  launch_fill_zero(ws, c.size(), s);

  OpArgs oa;
  oa.g = g;
  const int nl64 = gs->fp64_links();
  oa.links = gs->links(P64, nl64);
  oa.corners = op == OP_SW_CORNERS ? gs->corners(P64) : nullptr;
  oa.r = d->r;
  oa.mass0 = d->mass;
  oa.mass = nullptr;
  oa.mass_stride = 0;
  oa.g55w = g55w;
  oa.g55_sys = g55_bytes_per_system(g, P64);

  // v_1 = v0 / ||v0||
  launch_field_in(P64, nc, g, v0, 1, w, nbp, 0, 1, s);
  launch_lz_update(g, nc, V, 0, h, w, part_n, kLzBlocks, 1, s);
  launch_lz_finish(part_n, kLzBlocks, bd + steps, s);
  launch_lz_normalize(g, nc, w, bd + steps, V, s);
  check_launch();
  for (int j = 0; j < steps; ++j) {
    double2* vj = V + (size_t)j * n;
    EpiArgs e;
    std::memset(&e, 0, sizeof(e));
    e.nbp = nbp;
    e.out = t;
    launch_stencil(op, P64, nl64, false, EPI_STORE, oa, vj, e, 1, s);
    EpiArgs f;
    std::memset(&f, 0, sizeof(f));
    f.nbp = nbp;
    f.out = w;
    f.part = part_a;
    f.v = (const double*)vj;
    f.vprev = (const double*)(j > 0 ? vj - n : vj);
    f.beta_prev = j > 0 ? bd + (j - 1) : nullptr;
    launch_stencil(op, P64, nl64, true, EPI_LANCZOS, oa, t, f, 1, s);
    // w -= alpha v_j; two classical Gram-Schmidt passes against v_1..v_j
    launch_lz_dots(g, nc, V, j + 1, w, part_a, nbp, ad + j, part_h, kLzBlocks, s);
    launch_lz_reduce(part_h, j + 1, kLzBlocks, h, s);
    launch_lz_update(g, nc, V, j + 1, h, w, part_n, kLzBlocks, 0, s);
    launch_lz_dots(g, nc, V, j + 1, w, nullptr, 0, nullptr, part_h, kLzBlocks, s);
    launch_lz_reduce(part_h, j + 1, kLzBlocks, h, s);
    launch_lz_update(g, nc, V, j + 1, h, w, part_n, kLzBlocks, 1, s);
    launch_lz_finish(part_n, kLzBlocks, bd + j, s);
    if (j + 1 < steps) launch_lz_normalize(g, nc, w, bd + j, V + (size_t)(j + 1) * n, s);
    check_launch();
  }
  std::vector<double> ha(steps), hb(steps);
  LQ_HIP(hipMemcpyAsync(ha.data(), ad, steps * 8, hipMemcpyDeviceToHost, s));
  LQ_HIP(hipMemcpyAsync(hb.data(), bd, steps * 8, hipMemcpyDeviceToHost, s));
  LQ_HIP(hipStreamSynchronize(s));
  // truncate at an invariant subspace (beta_j negligible), as the basis ends there
  alpha.clear();
  beta.clear();
  for (int j = 0; j < steps; ++j) {
    alpha.push_back(ha[j]);
    if (j == steps - 1) break;
    if (!(hb[j] > 1e-14 * std::fabs(ha[j]))) break;
    beta.push_back(hb[j]);
  }
  for (double v : alpha)
    if (!std::isfinite(v)) throw Error(LQ_ERR_BREAKDOWN, "Lanczos produced a non-finite alpha");
  return (int)alpha.size();
}

// ============================================================== Arnoldi
// Shift-invert Krylov-Schur for the eigenvalues of M nearest sigma: the
// Krylov space of (M - sigma)^{-1}, each application an FP64 CG solve of
// eq. (2) with mass m - sigma (the solver engine, one slot), orthogonalised
// by two classical Gram-Schmidt passes (the Lanczos kernels, complex
// coefficients).  After `steps` vectors the projected matrix is brought to
// Schur form, the steps/2 Ritz values of largest modulus (lambda nearest
// sigma) are moved to its front, and the basis is cut to them plus the last
// vector, whose coupling becomes one full row of the projected matrix;
// Arnoldi then extends the basis again.  The eigenvalues mu of the projected
// matrix give lambda = sigma + 1/mu.
size_t spectrum_workspace_bytes(const Geom& g, int formulation, int g55, int steps) {
  const int nc = ncomp_of(formulation);
  const size_t vec = (size_t)nc * g.Vp * 16;
  const size_t canon = (size_t)g.V * nc * 16;
  Carver c(nullptr);
  c.take(vec * (steps + 1));                                // basis
  c.take(vec * (steps / 2 + 1));                            // restart: the kept vectors
  c.take(vec);                                              // w
  c.take(canon);                                            // solver input
  c.take(canon);                                            // solver output
  c.take((size_t)(steps + 1) * 16);                         // h
  c.take((size_t)(steps + 1) * kLzBlocks * 2 * 8);          // part_h
  c.take((size_t)kLzBlocks * 8);                            // norm partials
  c.take((size_t)(steps + 2) * 8);                          // beta
  c.take(Engine::workspace_bytes(g, formulation, g55, nullptr, 1));
  return c.size();
}

int spectrum_run(const lq_gauge_s* gs, const lq_dirac* d, double sigma, int steps, int restarts,
                 double tol, const void* v0, void* ws, size_t ws_bytes, std::vector<cplx>& eig,
                 std::vector<double>& resid, hipStream_t s) {
  const Geom& g = gs->g;
  const int nc = ncomp_of(d->formulation);
  if (steps < 2 || steps > 500) throw Error(LQ_ERR_ARG, "steps must be in [2, 500]");
  if (restarts < 0 || restarts > 1000) throw Error(LQ_ERR_ARG, "restarts must be in [0, 1000]");
  if (!(tol > 0.0 && tol < 1.0)) throw Error(LQ_ERR_ARG, "tol must be in (0, 1)");
  const size_t need = spectrum_workspace_bytes(g, d->formulation, d->g55_mode, steps);
  if (!ws || ws_bytes < need)
    throw Error(LQ_ERR_WORKSPACE, "spectrum workspace too small: need " + std::to_string(need));
  const int m = steps, keep = steps / 2;
  const size_t n = (size_t)nc * g.Vp;
  const size_t vec = n * 16;
  const size_t canon = (size_t)g.V * nc * 16;
  Carver c(ws);
  double2* V = (double2*)c.take(vec * (m + 1));
  double2* K = (double2*)c.take(vec * (keep + 1));
  double2* w = (double2*)c.take(vec);
  void* cin = c.take(canon);
  void* cout = c.take(canon);
  double2* h = (double2*)c.take((size_t)(m + 1) * 16);
  double* part_h = (double*)c.take((size_t)(m + 1) * kLzBlocks * 2 * 8);
  double* part_n = (double*)c.take((size_t)kLzBlocks * 8);
  double* bd = (double*)c.take((size_t)(m + 2) * 8);
  const size_t eb = Engine::workspace_bytes(g, d->formulation, d->g55_mode, nullptr, 1);
  void* ews = c.take(eb);
  launch_fill_zero(ws, (char*)ews - (char*)ws, s);
  const int nbp = nbp_of(g.V);
  Engine e;
  e.init(gs, d->formulation, d->g55_mode, d->r, 1, nullptr, ews, eb, s);

  // v_0 = v0 / ||v0||
  launch_field_in(P64, nc, g, v0, 1, w, nbp, 0, 1, s);
  launch_lz_update(g, nc, V, 0, h, w, part_n, kLzBlocks, 1, s);
  launch_lz_finish(part_n, kLzBlocks, bd + m, s);
  launch_lz_normalize(g, nc, w, bd + m, V, s);
  check_launch();
  // projected matrix, (m + 1) x m: column j holds the coefficients of
  // (M - sigma)^{-1} v_j; below the kept block it stays Hessenberg
  std::vector<cplx> H((size_t)(m + 1) * m, cplx(0.0, 0.0));
  auto Hat = [&](int r, int col) -> cplx& { return H[(size_t)r * m + col]; };
  std::vector<double2> hh(m + 1);
  int j0 = 0, mm = m;
  double beta = 0.0;
  std::vector<cplx> T, Q;
  for (int cycle = 0;; ++cycle) {
    // extend the basis to mm vectors (mm < m only at an invariant subspace)
    for (int j = j0; j < m; ++j) {
      launch_field_out(P64, nc, g, V + (size_t)j * n, cin, 1, nbp, 0, 1, s);
      check_launch();
      e.load(0, cin, d->mass - sigma, tol, 100000, s);
      while (e.running()) e.step(1 << 20, s);
      lq_solve_info inf;
      e.fetch(0, cout, &inf, s);
      if (inf.status != LQ_OK)
        throw Error(inf.status < 0 ? inf.status : LQ_ERR_BREAKDOWN,
                    "shift-invert solve " + std::to_string(j) + " did not converge");
      launch_field_in(P64, nc, g, cout, 1, w, nbp, 0, 1, s);
      for (int pass = 0; pass < 2; ++pass) {
        launch_lz_dots(g, nc, V, j + 1, w, nullptr, 0, nullptr, part_h, kLzBlocks, s);
        launch_lz_reduce(part_h, j + 1, kLzBlocks, h, s);
        LQ_HIP(hipMemcpyAsync(hh.data(), h, (size_t)(j + 1) * 16, hipMemcpyDeviceToHost, s));
        launch_lz_update(g, nc, V, j + 1, h, w, part_n, kLzBlocks, pass == 1, s);
        LQ_HIP(hipStreamSynchronize(s));
        for (int r = 0; r <= j; ++r) Hat(r, j) += cplx(hh[r].x, hh[r].y);
      }
      launch_lz_finish(part_n, kLzBlocks, bd + j, s);
      LQ_HIP(hipMemcpyAsync(&beta, bd + j, 8, hipMemcpyDeviceToHost, s));
      LQ_HIP(hipStreamSynchronize(s));
      check_launch();
      if (!std::isfinite(beta)) throw Error(LQ_ERR_BREAKDOWN, "Arnoldi produced a non-finite norm");
      double col = 0.0;
      for (int r = 0; r <= j; ++r) col = std::fmax(col, std::abs(Hat(r, j)));
      if (!(beta > 1e-13 * col)) {   // invariant subspace: the basis ends here
        mm = j + 1;
        beta = 0.0;
        break;
      }
      Hat(j + 1, j) = beta;
      launch_lz_normalize(g, nc, w, bd + j, V + (size_t)(j + 1) * n, s);
    }
    // Schur form of the projected matrix; Ritz values and estimates
    T.assign((size_t)mm * mm, cplx(0.0, 0.0));
    for (int r = 0; r < mm; ++r)
      for (int col = 0; col < mm; ++col) T[(size_t)r * mm + col] = Hat(r, col);
    schur_decompose(T, Q, mm);
    std::vector<std::pair<double, int>> order;   // by |mu| descending
    for (int r = 0; r < mm; ++r) order.push_back({-std::abs(T[(size_t)r * mm + r]), r});
    std::sort(order.begin(), order.end());
    const int want = std::min(keep, mm);
    bool converged = true;
    for (int q = 0; q < want; ++q) {
      const int r = order[q].second;
      const cplx mu = T[(size_t)r * mm + r];
      const std::vector<cplx> y = schur_eigenvector(T, Q, mm, r);
      if (!(beta * std::abs(y[mm - 1]) <= 1e3 * tol * std::abs(mu))) converged = false;
    }
    if (mm < m || cycle >= restarts || converged) break;
    // restart: the wanted Schur vectors first, then cut the basis to them
    std::vector<char> flag(mm, 0);
    for (int q = 0; q < keep; ++q) flag[order[q].second] = 1;
    schur_reorder(T, Q, mm, flag);
    std::vector<double2> negq(m);
    for (int q = 0; q < keep; ++q) {
      // K_q = sum_j Q[j][q] v_j, through w -= sum_j h_j v_j with h = -Q[:, q]
      for (int r = 0; r < m; ++r) {
        const cplx z = Q[(size_t)r * m + q];
        negq[r] = make_double2(-z.real(), -z.imag());
      }
      LQ_HIP(hipMemcpyAsync(h, negq.data(), (size_t)m * 16, hipMemcpyHostToDevice, s));
      launch_fill_zero(K + (size_t)q * n, vec, s);
      launch_lz_update(g, nc, V, m, h, K + (size_t)q * n, part_n, kLzBlocks, 0, s);
      LQ_HIP(hipStreamSynchronize(s));   // h is rewritten next round
    }
    LQ_HIP(hipMemcpyAsync(V, K, vec * keep, hipMemcpyDeviceToDevice, s));
    LQ_HIP(hipMemcpyAsync(V + (size_t)keep * n, V + (size_t)m * n, vec, hipMemcpyDeviceToDevice,
                          s));
    check_launch();
    // the projected matrix of the kept part: T's leading block, and the
    // coupling of the carried-over vector as a full row
    std::vector<cplx> Hn((size_t)(m + 1) * m, cplx(0.0, 0.0));
    for (int r = 0; r < keep; ++r)
      for (int col = 0; col < keep; ++col) Hn[(size_t)r * m + col] = T[(size_t)r * m + col];
    for (int col = 0; col < keep; ++col) Hn[(size_t)keep * m + col] = beta * Q[(size_t)(m - 1) * m + col];
    H.swap(Hn);
    j0 = keep;
  }
  // every Ritz value of the last projected matrix, nearest sigma first
  std::vector<std::pair<double, int>> near;
  std::vector<cplx> lam;
  std::vector<double> res;
  for (int r = 0; r < mm; ++r) {
    const cplx mu = T[(size_t)r * mm + r];
    if (std::abs(mu) == 0.0) continue;   // an eigenvalue of M - sigma at infinity: none nearby
    const std::vector<cplx> y = schur_eigenvector(T, Q, mm, r);
    res.push_back(beta * std::abs(y[mm - 1]) / std::abs(mu));
    lam.push_back(sigma + 1.0 / mu);
    near.push_back({std::abs(lam.back() - sigma), (int)lam.size() - 1});
  }
  std::sort(near.begin(), near.end());
  eig.clear();
  resid.clear();
  for (const auto& o : near) {
    eig.push_back(lam[o.second]);
    resid.push_back(res[o.second]);
  }
  return (int)eig.size();
}

// number of eigenvalues of tridiag(a, b) smaller than x (Sturm sequence)
static int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double d = 1.0;
  const double tiny = 1e-300;
  for (size_t i = 0; i < a.size(); ++i) {
    const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    d = a[i] - x - (i > 0 ? bb / d : 0.0);
    if (d == 0.0) d = -tiny;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

static double kth_eigenvalue(const std::vector<double>& a, const std::vector<double>& b, int k,
                             double lo, double hi) {
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(a, b, mid) > k) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, double& lo,
                      double& hi) {
  const size_t n = a.size();
  double glo = a[0], ghi = a[0];
  for (size_t i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    glo = std::min(glo, a[i] - r);
    ghi = std::max(ghi, a[i] + r);
  }
  const double pad = 1e-12 * std::max(std::fabs(glo), std::fabs(ghi)) + 1e-300;
  lo = kth_eigenvalue(a, b, 0, glo - pad, ghi + pad);
  hi = kth_eigenvalue(a, b, (int)n - 1, glo - pad, ghi + pad);
}

}  // namespace lq
