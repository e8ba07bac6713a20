/*
 * lq.h -- C ABI of the MI355X (gfx950) library for CG inversion of the Wilson
 * and 2-flavour staggered Wilson Dirac matrices through the normal equations
 *
 *     (D + m)^dag (D + m) psi = (D + m)^dag chi                 (paper eq. (2))
 *
 * and for the Lanczos estimate of the condition number of (D+m)^dag (D+m)
 * (paper Sec. 3).  Reference: D.H. Adams, D. Nogradi, A. Petrashyk,
 * C. Zielinski, "Computational efficiency of staggered Wilson fermions: A
 * first look", PoS LATTICE2013; the staggered Wilson operator itself is the one
 * of D.H. Adams, PLB 699 (2011) 394, which the paper cites in Sec. 2.
 *
 * Conventions (all functions):
 *  - Lattice dims are (L1, L2, L3, L4) = (x, y, z, t), every L even and >= 4.
 *    Canonical site index i = x1 + L1*(x2 + L2*(x3 + L3*x4)).
 *  - Canonical fields are interleaved complex arrays, site-major:
 *      gauge field  U[i][mu][a][b]  complex128   (mu = 0..3 for x, y, z, t;
 *                                                 U_mu(x) links x -> x + mu)
 *      Wilson field psi[i][spin][colour]         (4 x 3 complex per site)
 *      staggered Wilson field psi[i][colour]     (3 complex per site)
 *    complex128 = two doubles (re, im).
 *  - Operators (r = Wilson parameter, m = bare mass):
 *      Wilson:  (M psi)(x) = (m + 4r) psi(x) - 1/2 sum_mu [(r - g_mu) U_mu(x) psi(x+mu)
 *                                   + (r + g_mu) U_mu(x-mu)^dag psi(x-mu)]
 *               in the hermitian basis g_1 = [[0, i s1], [-i s1, 0]],
 *               g_2 = [[0, -i s2], [i s2, 0]], g_3 = [[0, i s3], [-i s3, 0]],
 *               g_4 = [[0, 1], [1, 0]]  (g_5 = diag(1, 1, -1, -1));
 *      staggered Wilson:  M = D_st + r (1 - Gamma_55) + m, with
 *               D_st = sum_mu eta_mu (V_mu - V_mu^dag)/2,
 *               Gamma_55 = phi (1/24) sum_{orderings} C_1 C_2 C_3 C_4,
 *               C_mu = (V_mu + V_mu^dag)/2, (V_mu psi)(x) = U_mu(x) psi(x+mu),
 *               eta_mu = (-1)^(x_1+..+x_{mu-1}), phi = (-1)^(x2+x4);
 *               M^dag = eps M eps, eps = (-1)^(x1+x2+x3+x4)   (paper Sec. 2).
 *    A fermion hop that crosses the lattice boundary in direction mu is
 *    multiplied by bc[mu] (+1 periodic, -1 antiperiodic).
 *  - Memory: the library allocates no device memory.  Every device buffer
 *    (gauge storage, solver workspace, inputs, outputs) is owned by the caller,
 *    sized with the *_bytes queries, and must stay alive while a handle that
 *    points into it is in use.  Handles hold host metadata only.  The
 *    workspace queries take the Gamma_55 mode: with LQ_G55_ONTHEFLY (staggered
 *    Wilson) the workspace also holds the intermediate fields of the subset
 *    recursion (14 fields of three complex numbers per site and system).
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  Work is
 *    enqueued on it; lq_apply and the *_create calls are asynchronous, the
 *    solve, condition-number and timing calls return after their own
 *    synchronisation with that stream.
 *  - Errors: 0 = success; negative = error (nothing useful was produced);
 *    positive = a solve finished without meeting its target (info is filled).
 *    lq_last_error() returns a thread-local description of the last failure.
 *    No C++ exception crosses this interface.
 */
#ifndef LQ_H
#define LQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LQ_OK 0
#define LQ_NOT_CONVERGED 1     /* maxiter reached; info filled                */
#define LQ_STAGNATION 2        /* stopped at the attainable accuracy: the FP64
                                  true residual did not halve over max_restarts
                                  reliable updates in a row, or stayed 100x above
                                  its best across a restart; info filled        */
#define LQ_ERR_ARG (-1)        /* bad dims, pointer, size, enum, non-finite    */
#define LQ_ERR_WORKSPACE (-2)  /* caller buffer smaller than the query says:
                                  the footprint (memory budget) error; the
                                  library never allocates, so no other
                                  out-of-memory condition exists               */
#define LQ_ERR_OOM_BUDGET LQ_ERR_WORKSPACE
#define LQ_ERR_DEVICE (-3)     /* a HIP runtime call failed                    */
#define LQ_ERR_BREAKDOWN (-4)  /* CG/Lanczos breakdown: <p,Ap> <= 0 or NaN     */
#define LQ_ERR_STATE (-5)      /* handle used in a state that does not allow it */

/* formulations */
#define LQ_WILSON 0
#define LQ_STAGGERED_WILSON 1

/* operator selector for lq_apply */
#define LQ_OP_M 0      /* out = (D + m) in          */
#define LQ_OP_MDAG 1   /* out = (D + m)^dag in      */
#define LQ_OP_MDAGM 2  /* out = (D+m)^dag (D+m) in  */

/* how the staggered Wilson Gamma_55 is applied */
#define LQ_G55_CORNERS 0    /* from precomputed path-averaged corner matrices */
#define LQ_G55_ONTHEFLY 1   /* from the links, every application, by the subset
                               recursion F_S = sum_{mu in S} C_mu F_{S\mu}: three
                               nearest-neighbour level launches into workspace
                               fields, the fourth level in the operator's own
                               stencil; 32 C_mu applications per site          */

/* arithmetic / storage precision of the stencil and Krylov vectors */
#define LQ_PREC_F64 0
#define LQ_PREC_F32 1
#define LQ_PREC_Q16 2   /* 16-bit fixed point: int16 components; vectors carry a
                           per-site float scale (largest |re|, |im| of the site),
                           links and corners a fixed scale of 1; FP32 arithmetic */

/* link storage: 18 reals (full 3x3) or 12 reals (two rows, third row
 * rebuilt in-kernel as conj(row0 x row1), valid for SU(3) links only).
 * 0 selects the default: 18 for FP32, 12 for Q16, and for FP64 12 when the
 * field is SU(3) to 1e-12 (see lq_gauge_create), else 18.  FP64 with 12 reads
 * two of the three stored rows (a third fewer link bytes).  The solvers'
 * FP64 work (plain FP64 CG, sources, reliable updates, Lanczos) follows the
 * same FP64 default. */
#define LQ_LINKS_18 18
#define LQ_LINKS_12 12

/* gauge features: which device copies lq_gauge_create builds */
#define LQ_FEAT_CORNERS 0x1u  /* corner matrices W_s(x) in every built precision */
#define LQ_FEAT_F32 0x2u      /* FP32 links, 18-real and 12-real               */
#define LQ_FEAT_Q16 0x4u      /* 16-bit fixed-point links (12- and 18-real), corners */
#define LQ_FEAT_EO 0x8u       /* even-odd copies of the links (FP64, and F32/Q16 when
                                 those are built): per parity, half-lattice records */

/* where a caller's input array lives (lq_gauge_create) */
#define LQ_WHERE_HOST 0
#define LQ_WHERE_DEVICE 1

typedef struct lq_lattice_s lq_lattice;
typedef struct lq_gauge_s lq_gauge;
typedef struct lq_batch_s lq_batch;

/* The Dirac matrix of eq. (2): formulation, bare mass, Wilson parameter r and
 * the Gamma_55 mode (ignored for Wilson). */
typedef struct {
  int32_t formulation;
  int32_t g55_mode;
  double mass;
  double r;
} lq_dirac;

/* Solver options (zero-initialised = plain FP64 CG, default polling). */
typedef struct {
  int32_t precision;          /* LQ_PREC_*: F64 = plain FP64 CG; F32/Q16 = inner
                                 CG in that storage with FP64 reliable updates   */
  int32_t links;              /* LQ_LINKS_18 or LQ_LINKS_12; with Q16 both are
                                 16-bit (12 rebuilds row 2 per hop, 18 stores it) */
  int32_t reliable_interval;  /* iterations between FP64 reliable updates
                                 (0 = default 256: the residual triggers do most
                                 of the work; unused for F64)                    */
  int32_t poll_interval;      /* iterations between host convergence polls
                                 (0 = default 16; rounded up to a multiple of 4,
                                 the solution's update groups)                   */
  int32_t use_graph;          /* 1 = replay steady iteration chunks as hipGraphs */
  int32_t max_restarts;       /* reliable updates allowed after the iterated
                                 residual first meets tol, and in a row without
                                 halving the true residual (a tol below the
                                 attainable accuracy then ends LQ_STAGNATION
                                 instead of cycling on; so does a true residual
                                 100x above its best at two reliable updates in
                                 a row, i.e. one that a restart from the FP64
                                 residual did not bring back; 0 = default 50)  */
  double reliable_delta;      /* also update once the iterated residual has
                                 dropped by this factor since the last update
                                 (0 = default: 0.1 for Q16, 1e-3 for F32)        */
  int32_t evenodd;            /* 1 = even-odd preconditioned (Wilson, r = 1, gauge
                                 built with LQ_FEAT_EO): CG on the normal
                                 equations of the Schur complement (see
                                 lq_schur_apply), M^dag M^ x_e = M^dag b^_e with
                                 b^_e = chi_e - M_eo chi_o / d, x_o = (chi_o -
                                 M_oe x_e) / d.  The stopping rule stays that of
                                 eq. (2) for the whole x: true_residual is
                                 ||b - A x|| / ||b|| with b = M^dag chi,
                                 evaluated in FP64 at each reliable update from
                                 r^ = b^_e - M^ x_e; the Schur system's target
                                 is lowered until it holds.  iterated_residual
                                 is the Schur system's.                        */
} lq_solve_opts;

/* Per-solve report.  The residuals are relative: ||b - A x|| / ||b|| with
 * b = M^dag chi, A = M^dag M; `true_residual` is recomputed in FP64 on the GPU
 * from the returned x. */
typedef struct {
  int32_t status;             /* LQ_OK, LQ_NOT_CONVERGED, LQ_STAGNATION or
                                 LQ_ERR_BREAKDOWN (lq_batch_peek: the slot state) */
  int32_t iterations;         /* CG iterations (A-applications in the loop)      */
  int32_t reliable_updates;   /* FP64 true-residual recomputations              */
  int32_t applications;       /* all applications of A, including b and updates */
  int32_t flags;              /* LQ_FLAG_* bits of the solve's stop reasons     */
  double iterated_residual;
  double true_residual;
  double seconds;             /* wall time of the call (0 from lq_batch_fetch
                                 and lq_batch_peek)                             */
} lq_solve_info;
#define LQ_FLAG_BREAKDOWN 1u   /* <p, A p> <= 0 or a non-finite residual         */
#define LQ_FLAG_MAXITER 2u     /* the iteration limit was reached                */
#define LQ_FLAG_STAGNATION 4u  /* the accuracy floor: see LQ_STAGNATION          */

/* ---------------------------------------------------------------- errors */
const char* lq_last_error(void);
const char* lq_version(void);

/* --------------------------------------------------------------- lattice
 * dims: 4 lattice extents, each even and >= 4, volume < 2^28.
 * bc:   4 fermion boundary signs, each +1 or -1 (NULL = all +1).  */
int lq_lattice_create(const int32_t dims[4], const int32_t bc[4], lq_lattice** out);
void lq_lattice_destroy(lq_lattice* lat);
int64_t lq_lattice_volume(const lq_lattice* lat);

/* ----------------------------------------------------------------- gauge
 * The gauge field of paper Sec. 3 (there: quenched beta = 6 configurations).
 * lq_gauge_bytes: device bytes lq_gauge_create needs for `features`.
 * lq_gauge_create: repacks the canonical complex128 field `U` (V*4*9 complex,
 *   in host memory if where = LQ_WHERE_HOST, in device memory if
 *   LQ_WHERE_DEVICE; the caller keeps ownership and may free it once the call
 *   has returned) into the library's structure-of-arrays layout in `buf`,
 *   builds the FP32/16-bit copies and the staggered Wilson corner matrices
 *   W_s(x) = (1/24) sum over the 24 orderings of the one-link-per-direction
 *   path products from x to x + s, s in {+-1}^4 (8 are stored; the other 8 are
 *   W_{-s}(x+s)^dag).  A host field is uploaded in chunks through a staging
 *   area inside `buf`.  The call measures how far row 2 of every link is from
 *   conj(row0 x row1) and synchronises `stream`; 12-real links are refused
 *   (LQ_ERR_ARG) unless that deviation is <= 1e-12 (FP64) or 1e-6 (FP32,
 *   Q16), i.e. unless the links are SU(3) to that accuracy.  Errors: LQ_ERR_ARG
 *   for a null pointer, unknown feature bits or where; LQ_ERR_WORKSPACE when
 *   buf_bytes < lq_gauge_bytes; LQ_ERR_DEVICE for a failed copy or launch.  */
size_t lq_gauge_bytes(const lq_lattice* lat, uint32_t features);
/* max over sites and directions of |row2 - conj(row0 x row1)| (real and
 * imaginary parts), measured by lq_gauge_create. */
int lq_gauge_su3_deviation(const lq_gauge* g, double* dev);
int lq_gauge_create(const lq_lattice* lat, const void* U, int32_t where, uint32_t features,
                    void* buf, size_t buf_bytes, void* stream, lq_gauge** out);
void lq_gauge_destroy(lq_gauge* g);
/* Mean plaquette (1/6V) sum_x sum_{mu<nu} (1/3) Re tr U_mu U_nu U_mu^dag U_nu^dag,
 * computed in FP64 on the device; synchronises `stream`. */
int lq_gauge_plaquette(const lq_gauge* g, double* plaquette, void* stream);

/* ----------------------------------------------------------------- apply
 * out = op(in) for the Dirac matrix `d` (paper eq. (2)).  in/out: device
 * canonical fields, complex128 for LQ_PREC_F64 and complex64 for F32/Q16
 * (Q16 rounds the repacked input to 16-bit storage; arithmetic is FP32).
 * `ws` is device scratch of lq_apply_workspace_bytes.  Asynchronous. */
size_t lq_apply_workspace_bytes(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                                int32_t precision);
int lq_apply(const lq_gauge* g, const lq_dirac* d, int32_t op, int32_t precision,
             int32_t links, const void* in, void* out, void* ws, size_t ws_bytes,
             void* stream);

/* Allocation-free variant of lq_apply, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same operation, arguments and results as lq_apply,
 * with the scratch taken from a fixed array inside the library instead of a
 * caller workspace.  The array holds lq_apply_noalloc_max_bytes() = 80 MiB per
 * GPU, allocated when the library's device code is loaded and kept until the
 * process ends; a lattice whose lq_apply_workspace_bytes exceeds it is refused
 * with LQ_ERR_WORKSPACE (80 MiB covers an FP64 Wilson M^dag M up to a
 * 16^3 x 32 lattice).  No device memory is allocated or freed by the call.
 * All calls on one GPU share its array: calls that overlap in time on the
 * same GPU (other streams or host threads) race on it and must be serialised
 * by the caller.  Asynchronous, like lq_apply. */
size_t lq_apply_noalloc_max_bytes(void);
int lq_apply_noalloc(const lq_gauge* g, const lq_dirac* d, int32_t op, int32_t precision,
                     int32_t links, const void* in, void* out, void* stream);

/* ------------------------------------------------------- even-odd blocks
 * The Schur complement of the even-odd preconditioned Wilson solve (the
 * preconditioning of the footnote to eq. (2), Sec. 3; r = 1): with sites split
 * by the parity of x1+x2+x3+x4 and M = [[d, M_eo], [M_oe, d]], d = m + 4,
 *     out_e = M^ in_e = d in_e - M_eo M_oe in_e / d     (M^dag when dagger),
 * out_o = 0.  in/out: device canonical full-lattice fields as for lq_apply;
 * only the even sites of `in` are read.  Needs a Wilson d with r = 1 and a
 * gauge field built with LQ_FEAT_EO (and the precision's own feature).  `ws`
 * is device scratch of lq_schur_workspace_bytes.  Asynchronous. */
size_t lq_schur_workspace_bytes(const lq_gauge* g, int32_t precision);
int lq_schur_apply(const lq_gauge* g, const lq_dirac* d, int32_t dagger, int32_t precision,
                   int32_t links, const void* in, void* out, void* ws, size_t ws_bytes,
                   void* stream);

/* Average device time (ms) of one stencil launch on `nrhs` fields already in
 * the library layout, over `reps` back-to-back launches, measured with HIP
 * events on `stream`.  The fields hold deterministic pseudo-random data
 * (every component uniform in [-1, 1)) and the solver state is live (alpha =
 * 1, the group's earlier steps non-zero), so the CG update does its full
 * arithmetic on non-zero values.  kernel = 0 times the first stencil of a CG iteration
 * (t = M p fused with ||t||^2), 1 the plain M^dag stencil, 2 the second
 * stencil of a CG iteration (q = M^dag t fused with r -= alpha q and
 * ||r||^2, and on every fourth launch (second in FP64) with x advanced by
 * the steps of the group, the solvers' x update) --
 * the same kernels the solvers launch; `reps` should be a multiple of 4 for
 * kernels 2 and 4.  kernel = 3 and 4 time
 * the same two steps of an even-odd preconditioned iteration (Wilson, r = 1,
 * LQ_FEAT_EO), each a pair of half-lattice launches: t = M^ p with ||t||^2,
 * and M^dag t fused with the CG update; the average is per pair.  rhs_per_thread (1, 2, 4;
 * FP32/Q16 only) is the number of systems each thread serves, the choice the
 * solvers' autotuner makes per batch; 8 selects the lanes stencil (kernels 0-2,
 * Wilson, r = 1, 18-real links: four systems across the lanes of each site,
 * the link products on the matrix cores, results bitwise those of 1); window, the autotuner's other choice,
 * is the block order: w > 0 sweeps windows of w site blocks per XCD over all
 * systems before moving on, 0 gives each XCD one contiguous site range, -1
 * gives each XCD a contiguous eighth of the system-major (system, site)
 * order, -2 the same with every other system swept backwards; -3 and -4 tile
 * each XCD's eighth of the t range in chunks of two z-planes with t inner,
 * systems outermost (-3) or innermost (-4) -- on lattices with whole x-y
 * planes of 256-site blocks, L4 % 8 == 0 and even L3; elsewhere they act as 0.
 * -11, -12, -13 (16-bit Wilson, r = 1, one system per thread, kernels 0-2):
 * each block sweeps one system's 256-site slab through T = 2, 4, 8 t-slices,
 * the diagonal and the x-y neighbours from LDS (x-y planes of exactly 256
 * sites); -14, -15, -16 the same with the x-y neighbours fetched; results
 * bitwise those of the other orders; where the sweep does not apply (other
 * storage, L4 not a multiple of 8T, other plane sizes, or fewer than four
 * blocks per CU) they act as 0.  ws: device scratch of
 * lq_time_dslash_workspace_bytes (contents overwritten).  */
size_t lq_time_dslash_workspace_bytes(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                                      int32_t precision,
                                      int32_t nrhs);
int lq_time_dslash(const lq_gauge* g, const lq_dirac* d, int32_t kernel,
                   int32_t precision, int32_t links, int32_t nrhs, int32_t rhs_per_thread,
                   int32_t window, int32_t reps, void* ws, size_t ws_bytes, double* avg_ms,
                   void* stream);

/* ----------------------------------------------------------------- solve
 * CG on eq. (2) for one source chi (device canonical complex128); the
 * solution x (device canonical complex128) is returned when the FP64 true
 * residual ||b - A x||/||b|| <= tol, with x0 = 0.  Mixed precision (opts)
 * iterates in FP32/Q16 and recomputes the true residual in FP64 at every
 * reliable update; scalars alpha, beta and all reductions are FP64. */
size_t lq_solve_workspace_bytes(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                                const lq_solve_opts* opts, int32_t nrhs);
int lq_cg_solve(const lq_gauge* g, const lq_dirac* d, const void* chi, void* x,
                double tol, int32_t maxiter, const lq_solve_opts* opts, void* ws,
                size_t ws_bytes, lq_solve_info* info, void* stream);

/* Batched multi-RHS CG: nrhs independent systems on one gauge field, each with
 * its own mass (masses[k], host), source (chi + k*field) and tolerance
 * (tols[k], host).  chi and x hold nrhs canonical complex128 fields back to
 * back.  Every stencil launch serves all active systems; links are shared.
 * infos: nrhs entries.  Returns the worst status. */
int lq_cg_solve_batch(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                      double r, int32_t nrhs, const double* masses, const void* chi,
                      void* x, const double* tols, int32_t maxiter,
                      const lq_solve_opts* opts, void* ws, size_t ws_bytes,
                      lq_solve_info* infos, void* stream);

/* -------------------------------------------------- continuous batching
 * A resident multi-RHS solver with `nslots` slots (serving).  Slots are loaded
 * and harvested between steps while the other slots keep iterating.
 *   lq_batch_create: ws of lq_solve_workspace_bytes(g, formulation, g55_mode,
 *                    opts, nslots).
 *   lq_batch_load:   start slot `slot` on source chi (device canonical) with
 *                    mass, tol and an iteration limit; asynchronous.
 *   lq_batch_step:   advance every running slot by about `iterations` CG
 *                    iterations (reliable updates included); then report each
 *                    slot's state in states[nslots] (0 empty, 1 running,
 *                    2 converged, 3 failed); synchronises `stream`.
 *   lq_batch_fetch:  copy a finished slot's solution to x (device canonical)
 *                    and its report to info; frees the slot.
 *   lq_batch_cancel: discard a loaded slot, running or finished, without
 *                    copying anything out; frees the slot for lq_batch_load.
 *                    LQ_ERR_STATE if the slot is empty, LQ_ERR_ARG if out of
 *                    range; synchronises `stream`.                            */
int lq_batch_create(const lq_gauge* g, int32_t formulation, int32_t g55_mode, double r,
                    int32_t nslots, const lq_solve_opts* opts, void* ws,
                    size_t ws_bytes, lq_batch** out);
int lq_batch_load(lq_batch* b, int32_t slot, const void* chi, double mass, double tol,
                  int32_t maxiter, void* stream);
int lq_batch_step(lq_batch* b, int32_t iterations, int32_t* states, void* stream);
int lq_batch_fetch(lq_batch* b, int32_t slot, void* x, lq_solve_info* info, void* stream);
int lq_batch_cancel(lq_batch* b, int32_t slot, void* stream);
/* Progress of a slot as of the latest step (host copy, no device work): info
 * gets the slot state (0..3) in `status`, the LQ_FLAG_* bits in `flags`, the
 * iteration and update counts, the iterated residual and the FP64 residual of
 * the latest reliable update; scale (may be NULL) the storage scale of its
 * low-precision vectors. */
int lq_batch_peek(lq_batch* b, int32_t slot, lq_solve_info* info, double* scale);
void lq_batch_destroy(lq_batch* b);

/* Batched solvers tune their launch configuration once per (GPU, lattice,
 * operator, storage, batch size) and cache it in the file LQ_TUNE_CACHE
 * (default $HOME/.cache/lq_tune.txt).  The environment variable LQ_LAUNCH =
 * "K,window" (K in {1, 2, 4, 8}, window >= -4, or K = 1 and a t-sweep order
 * -11 ... -16) forces a configuration instead.
 *
 * LQ_LAUNCH = "8,window" runs the unpreconditioned r = 1 Wilson stencils of
 * FP32/16-bit batches with 18-real links as the lanes stencil (see
 * lq_time_dslash); the autotuner does not choose it.
 *
 * The launch configuration the solvers' autotuner chose for batches of
 * `nrhs` systems of this operator and storage on this lattice (in this
 * process or read back from the tuning cache): systems per thread and block
 * order, as lq_time_dslash takes them.  LQ_ERR_STATE if no batch of that
 * shape has been tuned yet; FP64 and single systems are never tuned (1, -3). */
int lq_tuned_launch(const lq_gauge* g, const lq_dirac* d, int32_t precision, int32_t links,
                    int32_t nrhs, int32_t* rhs_per_thread, int32_t* window);

/* ----------------------------------------------------- pion correlator
 * The Wilson pion correlator behind the m_pi^2 against m plot (Fig. 1(a),
 * Sec. 3), read as the pseudoscalar two-point function of the point-source
 * propagators G(x, 0) = M^{-1} chi^(alpha) (the solutions of eq. (2)): by
 * gamma_5-hermiticity C(t) = sum over x vec, the nsrc propagators and their
 * 12 components of |G(x vec, t)|^2.  props: nsrc device canonical complex128
 * Wilson fields back to back (as lq_cg_solve_batch returns them).  corr[t]
 * (host, L4 entries) receives C(t) (FP64, summed in a fixed order); meff (host,
 * may be NULL) the periodic effective mass arccosh((C(t-1) + C(t+1)) / (2 C(t))),
 * NaN where that argument is below 1.  `ws` is device scratch of
 * lq_pion_workspace_bytes.  Synchronises `stream`. */
size_t lq_pion_workspace_bytes(const lq_lattice* lat);
int lq_pion_correlator(const lq_lattice* lat, int32_t nsrc, const void* props, double* corr,
                       double* meff, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------ spectrum
 * Eigenvalues of the Dirac matrix M of `d` (eq. (2)'s matrix at d->mass;
 * d->mass = 0 gives D itself, as in the low-lying staggered Wilson spectrum
 * of Fig. 1(c), Sec. 3) nearest the real shift sigma, by shift-invert
 * Krylov-Schur: Arnoldi on (M - sigma)^{-1} from the start vector v0 (device
 * canonical complex128) to a basis of `steps` vectors, each application an
 * FP64 CG solve of eq. (2) with mass d->mass - sigma to residual tol,
 * orthogonalised by two classical Gram-Schmidt passes; then, up to `restarts`
 * times (0: plain Arnoldi), the projected matrix is brought to Schur form
 * (host, shifted complex QR), the basis is cut to the steps/2 Ritz vectors
 * nearest sigma, and Arnoldi extends it again -- stopping once those have
 * Ritz estimates below 1e3 tol.  The eigenvalues mu of the projected matrix
 * give lambda = sigma + 1/mu.  eig_re/eig_im (host, steps entries) receive
 * *nev values ordered by distance from sigma; resid (host, may be NULL) the
 * Ritz estimates ||(M - sigma)^{-1} u - mu u|| / |mu| (relative).  Stops
 * early at an invariant subspace.  `ws` is device scratch of
 * lq_spectrum_workspace_bytes.  Synchronises `stream`. */
size_t lq_spectrum_workspace_bytes(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                                   int32_t steps);
int lq_spectrum(const lq_gauge* g, const lq_dirac* d, double sigma, int32_t steps,
                int32_t restarts, double tol, const void* v0, void* ws, size_t ws_bytes,
                int32_t* nev, double* eig_re, double* eig_im, double* resid, void* stream);

/* ---------------------------------------------------- staggered overlap
 * The staggered overlap operator with the 2-flavour staggered Wilson kernel
 * (the paper presents D_SW as the kernel of a staggered overlap operator,
 * Secs. 1, 2 and 4; the usual overlap construction with the flavoured
 * gamma_5 = eps = (-1)^(x1+x2+x3+x4)):
 *     A = D_SW - rho,   V = eps sign(eps A) = A (A^dag A)^{-1/2},
 *     D_ov(m) = (rho - m/2) (1 + V) + m,
 * eps-hermitian, Ginsparg-Wilson (eps D + D eps = D eps D / rho at m = 0).
 * The library applies V psi ~ A p(A^dag A) psi with p the Chebyshev
 * interpolant of degree `degree` of x^{-1/2} on [lo, hi]: the result is exact
 * up to max over [lo, hi] of |x^{1/2} p(x) - 1| per singular direction of A,
 * provided [lo, hi] contains the spectrum of A^dag A (lq_condition_number at
 * mass -rho gives its Lanczos estimates; outside the interval the polynomial
 * is not an approximation).  Cost: degree + 1/2 applications of A^dag A (FP64
 * stencils of the kernel, Gamma_55 by `g55_mode`).  */
typedef struct {
  double rho;        /* kernel mass: A = D_SW - rho; > 0                       */
  double mass;       /* m of D_ov(m)                                           */
  double r;          /* Wilson parameter of the kernel                         */
  double lo, hi;     /* 0 < lo < hi: interval containing spec(A^dag A)          */
  int32_t degree;    /* 1..4096                                                */
  int32_t g55_mode;  /* LQ_G55_CORNERS or LQ_G55_ONTHEFLY                       */
} lq_overlap;

/* out = D_ov(m) in.  in/out: device canonical staggered Wilson fields
 * (complex128).  ws: device scratch of lq_overlap_workspace_bytes (6 FP64
 * fields, plus the on-the-fly intermediate fields).  Errors: LQ_ERR_ARG for a
 * null pointer, a non-finite or out-of-range parameter, a gauge field without
 * corners for LQ_G55_CORNERS; LQ_ERR_WORKSPACE for a short ws.
 * Asynchronous. */
size_t lq_overlap_workspace_bytes(const lq_gauge* g, int32_t g55_mode);
int lq_overlap_apply(const lq_gauge* g, const lq_overlap* ov, const void* in, void* out,
                     void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------- condition number
 * Lanczos with full reorthogonalisation (classical Gram-Schmidt, twice) on
 * A = M^dag M from the caller's start vector v0 (device canonical complex128),
 * `steps` steps; the Ritz values of the tridiagonal matrix give
 * lmin = theta_min, lmax = theta_max and kappa = lmax/lmin (paper Sec. 3,
 * kappa = lambda_max/lambda_min).  alpha[steps] and beta[steps-1] (host,
 * may be NULL) receive the tridiagonal.  Workspace holds steps+1 FP64 basis
 * vectors: lq_lanczos_workspace_bytes.  Synchronises `stream`.  */
size_t lq_lanczos_workspace_bytes(const lq_gauge* g, int32_t formulation, int32_t g55_mode,
                                  int32_t steps);
int lq_condition_number(const lq_gauge* g, const lq_dirac* d, int32_t steps,
                        const void* v0, void* ws, size_t ws_bytes, double* lmin,
                        double* lmax, double* kappa, double* alpha, double* beta,
                        int32_t* steps_done, void* stream);

/* Critical mass estimate for the synthetic workloads (the paper compares at
 * equal pion mass, Sec. 3; the stand-in uses m = m_c + delta): m_c is the mass
 * in [lo, hi] that minimises the lowest Ritz value theta_min of a `steps`-step
 * Lanczos run on A(m) = (D+m)^dag (D+m) from v0 -- an ngrid-point scan, then
 * ngolden golden-section steps on the bracket around the best grid point; the
 * best evaluated point is returned.  ws as for lq_condition_number. */
int lq_critical_mass(const lq_gauge* g, int32_t formulation, int32_t g55_mode, double r,
                     double lo, double hi, int32_t ngrid, int32_t ngolden, int32_t steps,
                     const void* v0, void* ws, size_t ws_bytes, double* m_c, double* theta_min,
                     void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LQ_H */
