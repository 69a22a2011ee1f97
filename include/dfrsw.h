/*
 * dfrsw.h -- C ABI of the MI355X (gfx950) library for the hot path of the
 * direct-flux-reconstruction (DFR) shallow-water model with exponential time
 * integration on the rotated cubed sphere (Gaudreault, Charron, Dallerit,
 * Tokman, arXiv 2101.05617).
 *
 * Conventions (all entry points):
 *   - State vectors hold 3*N values, field-major: H, H u^1, H u^2, each over
 *     the N = 6 ne^2 (p+1)^2 Gauss-Legendre nodes ordered
 *     (panel, element row, element column, node row, node column), node
 *     column (x^1 direction) fastest.  u^i are contravariant components in the
 *     equiangular panel coordinates x^i (angle per unit time).
 *   - Pointers named q, v, w, jv, dqdt, b[k] are DEVICE pointers owned by the
 *     caller (e.g. torch tensors); the library never frees them.  Pointers
 *     named host_* and the descriptor's hB are HOST pointers.
 *   - Work is enqueued on the stream given to dfr_create.  dfr_rhs and
 *     dfr_jvp_complex_step are asynchronous; kiops_phi_apply and epi_step
 *     return when all the work they issued on the stream has finished (their
 *     adaptive control and their final error check wait for small results
 *     that kernels write into mapped host memory).
 *   - Units: any consistent system.  The equations keep their form for
 *     radius = 1, omega = 1 and a rescaled gravity; the complex-FP32 form needs
 *     such a scaled state so that eps times the state stays far above the
 *     FP32 underflow threshold.
 *   - Return value 0 on success, a negative DFR_E_* code on error; the message
 *     is in dfr_last_error() (thread-local).  Errors found inside kernels
 *     (non-finite input, non-positive depth) are latched in the context and
 *     returned by the next synchronising call (dfr_sync, kiops_phi_apply,
 *     epi_step).  Outputs are unspecified after an error.
 */
#ifndef DFRSW_H
#define DFRSW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DFR_OK = 0,
  DFR_E_INVAL = -1,      /* bad argument or descriptor */
  DFR_E_NOMEM = -2,      /* device or host allocation failed */
  DFR_E_HIP = -3,        /* a HIP runtime call failed */
  DFR_E_NONFINITE = -4,  /* NaN or Inf in an input state or direction */
  DFR_E_DEPTH = -5,      /* non-positive fluid depth H */
  DFR_E_KIOPS = -6       /* the Krylov controller did not converge */
};

/* Precision of the products inside KIOPS / EPI.  DFR_FP64: complex FP64.
 * DFR_FP32_JV: the complex-step evaluations inside KIOPS in complex FP32;
 * the Krylov basis, inner products, norms, Hessenberg, exponential and
 * combination, the EPI stage combination and update stay FP64, and so do
 * the products J_n (q_{n-i} - q_n) of the EPI remainders.
 * DFR_FP32_JV_BASIS32: as DFR_FP32_JV with the Krylov basis stored in FP32
 * (its vectors rounded once when stored; inner products and norms
 * accumulate in FP64 over the stored values), and with the b-columns of the
 * augmented operator (at most four) kept in FP32 for the Krylov products;
 * KIOPS / EPI and the batched ensemble form; dfr_jvp_complex_step treats it
 * as DFR_FP32_JV. */
typedef enum { DFR_FP64 = 0, DFR_FP32_JV = 1, DFR_FP32_JV_BASIS32 = 2 } dfr_precision;

/* Smallest complex-step eps accepted with DFR_FP32_JV and DFR_FP32_JV_BASIS32
 * (dfr_jvp_complex_step, kiops_phi_apply, epi_create and the ensemble
 * creation return DFR_E_INVAL below it).  Inside KIOPS the product is applied
 * to unit-norm vectors, whose typical entry is about 1/sqrt(3N); at this eps
 * their FP32 imaginary parts stay about four orders above FP32's smallest
 * normal number (1.2e-38) up to N ~ 1e7.  An FP64 eps such as 1e-150 would
 * make them zero. */
#define DFR_FP32_EPS_MIN 1e-30

typedef struct dfr_ctx dfr_ctx;
typedef struct epi_state epi_state;

/* Grid and physical constants.  Sec. 2 and App. B: a = radius, Omega =
 * omega, g_r = gravity; (lambda0, phi0, alpha0) the rotation of panel 0
 * (the paper uses (0, pi/4, 0)).  p = DFR degree, 1 <= p <= 7 (p+1 GL points
 * per element edge); ne >= 1.  hB: NULL, or N host values of the bottom
 * orography h_B at the nodes (Eq. 2); its derivative is taken element-locally
 * on the GL points. */
typedef struct {
  int ne, p;
  double radius, omega, gravity;
  double lambda0, phi0, alpha0;
  const double *hB;
} dfr_grid_desc;

/* One attempt of the Krylov controller (Sec. 4, Eq. 29: a sub-step of the
 * phi-combination tried with one small exponential): the sub-step length tau
 * it was tried with, the Krylov dimension m of its exponential, and whether
 * the sub-step was accepted (1) or rejected (0). */
typedef struct {
  double tau;
  int m;
  int accept;
} kiops_decision;

/* Decision record and replay, an instrument for separating the arithmetic of
 * a precision form from the controller's path: record the decisions of one
 * run (or take them from another implementation of the same controller) and
 * make a second run, possibly in another precision, take exactly those
 * decisions, so that the two results differ by arithmetic alone.  Owned by
 * the caller (host memory); the fields the library advances are counters the
 * caller zeroes before the first call.
 *   rec, rec_cap: NULL / 0, or host room for rec_cap decisions; each attempt
 *     appends its decisions (tau it ran with, m = the Krylov dimension its
 *     exponential used, accept).  n_rec counts the attempts recorded,
 *     including those beyond rec_cap, which are not stored.
 *   play, n_play: NULL / 0, or decisions that successive attempts take in
 *     order, from entry pos on: the attempt runs with that tau, extends the
 *     Krylov basis to that m and is accepted or rejected as stated, whatever
 *     the controller's own error estimate says.  pos is advanced past each
 *     decision taken.  Record and play may be used together.
 * Calls that share the struct continue its counters, so one epi_step (several
 * KIOPS calls in its start-up) records and replays as one sequence.
 * Errors (DFR_E_KIOPS, the message naming the attempt): the decisions run out
 * before tau_out is reached; a decision's tau passes tau_out (by more than a
 * relative 1e-12); a decision's m is below the basis already built
 * (a sweep cannot shrink), above m_max, or below 1; a happy breakdown (an
 * invariant Krylov space) ends the basis below the decision's m.  Single-grid
 * calls only (kiops_phi_apply, epi_step): the ensemble and concurrent forms
 * return DFR_E_INVAL when opts->replay is set. */
typedef struct {
  kiops_decision *rec;
  int rec_cap;
  int n_rec;
  const kiops_decision *play;
  int n_play;
  int pos;
} kiops_replay;

/* Adaptive Krylov (KIOPS-type) controller settings; see kiops_phi_apply. */
typedef struct {
  double tol;        /* relative tolerance of the phi-combination */
  int m_init;        /* initial Krylov dimension */
  int m_min, m_max;  /* bounds of the Krylov dimension (m_max <= 64) */
  int iop;           /* incomplete orthogonalisation length: 1 or 2 */
  int max_attempts;  /* cap on sub-step attempts before DFR_E_KIOPS */
  kiops_replay *replay;  /* NULL, or the decision record / replay above */
} kiops_opts;

typedef struct {
  int n_matvec;      /* complex-step J*v products */
  int n_substeps;    /* accepted sub-steps */
  int n_rejected;    /* rejected attempts */
  int m_last;        /* Krylov dimension of the last accepted sub-step */
  int happy;         /* 1 if a happy breakdown ended a sub-step */
  int n_expm;        /* small exponentials evaluated */
} kiops_stats;

/* Create a discretisation context on the current HIP device.  hip_stream is
 * a hipStream_t (NULL = default stream).  Allocates the geometry tables and
 * all workspace.  Sec. 3 (DFR), App. B (geometry), App. C (interfaces). */
int dfr_create(const dfr_grid_desc *desc, void *hip_stream, dfr_ctx **out);
int dfr_destroy(dfr_ctx *ctx);
/* N = 6 ne^2 (p+1)^2 */
int64_t dfr_num_nodes(const dfr_ctx *ctx);

/* The stiff test problems of Sec. 5.1 on the same KIOPS / EPI path: a
 * context that holds a semi-discrete ODE system du/dt = F(u) instead of a
 * grid, with second-order finite differences and the paper's constants.
 *   DFR_ODE_ADR: u_t + alpha (u_x + u_y) = eps (u_xx + u_yy) + gamma u (u -
 *     1/2)(1 - u) on [0,1]^2 (eps 1/100, alpha -10, gamma 100), homogeneous
 *     Neumann by reflection, on an n x n vertex grid (n^2 unknowns, index
 *     j n + i with i along x; 3 <= n <= 256).
 *   DFR_ODE_BURGERS: u_t + (u^2/2)_x = eps u_xx on [0,1] (eps 1e-3), u = 0
 *     at both ends, n interior points (the flux difference as (u_{i+1}^2 -
 *     u_{i-1}^2)/(4h)).
 *   DFR_ODE_SEMILINEAR: u_t - u_xx = int_0^1 u dx + phi(x, t), u = 0 at both
 *     ends, n interior points, trapezoid integral, phi such that x(1-x) e^t
 *     solves the discrete system; unknown n is the time t (n + 1 unknowns).
 * dfr_rhs gives F(u); dfr_jvp_complex_step gives the exact J(u) v (eps is
 * ignored; DFR_FP64 only); kiops_phi_apply and the epi_* calls run as on a
 * grid, in FP64 (epi_step_concurrent too).  The grid-only calls (node
 * frames, tiles, Riemann solver, diagnostics) return DFR_E_INVAL on such a
 * context.  Vectors have dfr_num_unknowns(ctx) doubles (3N on a grid). */
typedef enum { DFR_ODE_ADR = 1, DFR_ODE_BURGERS = 2, DFR_ODE_SEMILINEAR = 3 } dfr_ode_problem;
int dfr_create_ode(int problem, int n, void *hip_stream, dfr_ctx **out);
int64_t dfr_num_unknowns(const dfr_ctx *ctx);
/* Per node: unit position P and the coordinate basis dP/dx^1, dP/dx^2 on the
 * unit sphere (3 doubles each, node order as above).  Host outputs of size 3N. */
int dfr_node_frames(const dfr_ctx *ctx, double *host_P, double *host_B1, double *host_B2);
/* Wait for the context's stream; return (and clear) any latched kernel error. */
int dfr_sync(dfr_ctx *ctx);

/* Work decomposition of the DFR kernel: a workgroup takes a tile of
 * tile_tx x tile_ty elements of one panel (both dividing ne, one thread per
 * GL node, at most 1024 nodes).  The products inside kiops_phi_apply (with
 * the fused Arnoldi steps) have a tile of their own.  dfr_create picks a
 * default for both; dfr_set_tile sets both (DFR_E_INVAL if not admissible);
 * dfr_autotune times the complex-step kernel of the given precision, plain
 * and in its Krylov form, for every admissible tile on a synthetic state and
 * keeps the fastest of each (synchronises; uses the context's Krylov
 * workspace as scratch) and returns the plain one.  dfr_get_tile returns the
 * tile of dfr_rhs / dfr_jvp_complex_step, dfr_get_krylov_tile the other.
 * Results are identical for every tile up to rounding. */
int dfr_set_tile(dfr_ctx *ctx, int tile_tx, int tile_ty);
int dfr_get_tile(const dfr_ctx *ctx, int *tile_tx, int *tile_ty);
int dfr_get_krylov_tile(const dfr_ctx *ctx, int *tile_tx, int *tile_ty);
int dfr_autotune(dfr_ctx *ctx, dfr_precision prec, int *tile_tx, int *tile_ty);

/* Common flux at element faces (the Riemann problem of Sec. 3.1).
 * DFR_RUSANOV (default): local Lax-Friedrichs with the largest wave speed of
 * Eqs. (147)-(148) of the two sides.  DFR_AUSM: the AUSM flux with double
 * Froude-number splitting of App. D, Eqs. (137)-(143), with the split
 * functions of the original AUSM (Liou and Steffen 1993; cubic pressure
 * weights) and the gravity-wave speeds of App. E.  The setting belongs to the
 * context and applies to every later call on it (F, J*v, KIOPS, EPI, the
 * concurrent ensemble form).  The batched ensemble form carries the Rusanov
 * flux only: its calls return DFR_E_INVAL, naming the member, if a member
 * context is set to another.  DFR_E_INVAL for an unknown solver. */
typedef enum { DFR_RUSANOV = 0, DFR_AUSM = 1 } dfr_riemann;
int dfr_set_riemann(dfr_ctx *ctx, int solver);
int dfr_get_riemann(const dfr_ctx *ctx, int *solver);

/* dqdt = F(q): the DFR right-hand side of the covariant shallow-water
 * equations, Eqs. (1)-(2) with the flux reconstruction of Eqs. (10)-(14),
 * the context's interface fluxes (dfr_set_riemann), panel interfaces per
 * App. C.  q, dqdt: device, 3N doubles each, may not alias. */
int dfr_rhs(dfr_ctx *ctx, const double *q, double *dqdt);

/* Diagnostics of Sec. 5.4 on the state q (device, 3N doubles):
 *   zeta: relative vorticity, Eq. (43), with element-local collocation
 *         derivatives of the covariant velocity g_jk u^k (Eqs. 64-66);
 *   fcor: Coriolis parameter f, Eq. (46);
 *   host_out3: the integrals over the sphere (GL quadrature of each element,
 *         area element sqrt(g) dx^1 dx^2) of the mass H, of the total energy
 *         (1/2)[H g_ij u^i u^j + g_r((H + h_B)^2 - h_B^2)] and of the
 *         potential enstrophy (zeta + f)^2 / (2H), in the units of the grid's
 *         constants; Eq. (44) normalises their changes in time.
 * zeta, fcor: device, N doubles each, or NULL; host_out3: host, 3 doubles.
 * Synchronises the context's stream.  DFR_E_NONFINITE / DFR_E_DEPTH for an
 * invalid state; DFR_E_INVAL for NULL q or host_out3 or aliased outputs. */
int dfr_diagnostics(dfr_ctx *ctx, const double *q, double *zeta, double *fcor, double *host_out3);

/* jv = Im F(q + i eps v) / eps (Eq. 28), one complex evaluation of the same
 * right-hand side.  prec = DFR_FP64: complex FP64.  prec = DFR_FP32_JV: the
 * complex evaluation runs in FP32 on FP32 roundings of q and v (eps must
 * keep eps*|v| far above 1e-38 on the caller's scale, and eps >=
 * DFR_FP32_EPS_MIN); jv is written in FP64.
 * Branches of the interface flux (|.|, max(.,.), the AUSM split ranges)
 * are those of the real evaluation at q.  q, v, jv: device, 3N doubles; jv may not alias q or v. */
int dfr_jvp_complex_step(dfr_ctx *ctx, const double *q, const double *v, double eps,
                         dfr_precision prec, double *jv);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * product as dfr_jvp_complex_step, with the same kernels and results, that
 * allocates nothing and creates no runtime objects.  The complex-FP32 form
 * keeps its FP32 copy of q in a device array of 16 MiB compiled into the
 * library (one per device, held until the process ends) instead of context
 * memory, so it serves grids of at most 16 MiB / 12 B = 1,398,101 nodes
 * (DFR_E_INVAL beyond, the message stating the limit; DFR_FP64 has no such
 * limit and uses no scratch).  Every call on a device shares that device's
 * array: calls that overlap on one device (several streams or threads)
 * race and give undefined results; calls ordered on one stream do not.
 * The context's kernel timing (dfr_timing_enable) does not cover these
 * calls.  Arguments and errors as for dfr_jvp_complex_step. */
int dfr_jvp_complex_step_noalloc(dfr_ctx *ctx, const double *q, const double *v, double eps,
                                 dfr_precision prec, double *jv);

/* w = sum_{k=0}^{n_phi} tau_out^k phi_k(tau_out J(q_lin)) b_k   (Eq. 29)
 * with phi_k of Eq. (26) and J(q_lin) applied by complex-step products
 * (dfr_jvp_complex_step with the given eps and prec).  b: host array of
 * n_phi+1 device pointers (3N doubles each); b[0] may be NULL (zero).
 * n_phi >= 0 (n_phi = 0 is the exponential).  Adaptive sub-stepping with
 * incomplete orthogonalisation (KIOPS); the controller is deterministic and
 * documented in the library source.  w: device, 3N doubles, may not alias
 * q_lin or any b[k].  stats may be NULL.  Returns when its work on the
 * stream has finished. */
int kiops_phi_apply(dfr_ctx *ctx, const double *q_lin, double tau_out, int n_phi,
                    const double *const *b, const kiops_opts *opts, double eps,
                    dfr_precision prec, double *w, kiops_stats *stats);

/* Multistep EPI integrator (Sec. 4): order 2 (exponential Euler, Eq. 25),
 * 3 (Eq. 30) or 4, 5, 6 (Eqs. 34-38).  The first P = order-2 steps use EPI2
 * with startup_substeps equal sub-steps.  q0: device, 3N doubles (copied).
 * The state owns the history q_{n-i}, F(q_{n-i}). */
int epi_create(dfr_ctx *ctx, int order, double dt, int startup_substeps, const double *q0,
               double eps, dfr_precision prec, epi_state **out);
/* Advance one step of size dt.  q_out (device, 3N doubles, may be NULL)
 * receives q_{n+1}.  stats (may be NULL) accumulates over the step's KIOPS
 * calls.  Returns when its work on the stream has finished. */
int epi_step(dfr_ctx *ctx, epi_state *st, const kiops_opts *opts, double *q_out, kiops_stats *stats);
/* Copy the current state q_n to a device buffer of 3N doubles. */
int epi_get_state(const epi_state *st, double *q);
/* Number of steps taken. */
int64_t epi_num_steps(const epi_state *st);
int epi_destroy(epi_state *st);
/* Checkpoint and restart of an EPI integration.  epi_save writes to a host
 * buffer everything the next steps depend on: order, dt, start-up sub-steps,
 * eps, precision, step count, the grid's shape (ne, p), q_n and the history
 * q_{n-i}, F(q_{n-i}) that later steps read (Eq. 33), all as raw FP64 in the
 * library's layout behind a versioned header.  With host_buf NULL it only
 * stores the size needed in *nbytes; otherwise *nbytes is the buffer size on
 * entry and the bytes written on return (DFR_E_INVAL if too small).
 * Synchronises the stream.  epi_load makes a new state on ctx from such a
 * buffer (DFR_E_INVAL if the header or the size is wrong or the grid's ne, p
 * differ); continuing from it gives the results of the uninterrupted run,
 * bit for bit, on the same kind of device. */
int epi_save(const epi_state *st, void *host_buf, size_t *nbytes);
int epi_load(dfr_ctx *ctx, const void *host_buf, size_t nbytes, epi_state **out);

/* Ensembles (many independent grids, e.g. an ensemble of small forecasts).
 *
 * Batched form.  dfr_ensemble_create makes one context per member (member i
 * from members[i]; up to 256 members; all on hip_stream) plus device tables
 * that let one kernel launch serve every member.  epi_ensemble_step advances
 * every member by one EPI step: each operation of the step and of the Krylov
 * iteration (Sec. 4, Eq. 29) is one launch for all members; every member
 * keeps its own KIOPS controller, and members take Arnoldi steps in lockstep
 * rounds with one read-back per round in which some member's sweep reaches
 * its exponential (dfr_ensemble_set_rounds: or with the decisions taken on
 * the device).  With host-driven rounds member results equal those of
 * epi_step on the member alone with the same tiles, bit for bit (same
 * kernels, reduction orders and EPI combinations).  All members of
 * an epi_ensemble must share order, dt, start-up sub-steps and precision
 * (DFR_E_INVAL otherwise).  q0: host array of n device pointers (3 N_i
 * doubles each, copied).  stats: NULL or n entries.  dfr_ensemble_member
 * returns member i's context (owned by the ensemble; usable with every
 * single-grid entry point, e.g. dfr_node_frames, dfr_autotune, whose tiles the
 * batched launches then use).  Errors name the member. */
typedef struct dfr_ensemble dfr_ensemble;
typedef struct epi_ensemble epi_ensemble;
int dfr_ensemble_create(int n_members, const dfr_grid_desc *members, void *hip_stream, dfr_ensemble **out);
int dfr_ensemble_destroy(dfr_ensemble *e);
int dfr_ensemble_size(const dfr_ensemble *e);
dfr_ctx *dfr_ensemble_member(dfr_ensemble *e, int i);
/* Give all members with the same p one common tile (both forms), the fastest
 * of the tiles admissible for every one of them, timed on batched launches of
 * the Krylov-form product of the given precision (synchronises; uses the
 * members' Krylov workspaces as scratch). */
int dfr_ensemble_autotune(dfr_ensemble *e, dfr_precision prec);
int epi_ensemble_create(dfr_ensemble *e, int order, double dt, int startup_substeps, const double *const *q0,
                        double eps, dfr_precision prec, epi_ensemble **out);
int epi_ensemble_step(dfr_ensemble *e, epi_ensemble *x, const kiops_opts *opts, kiops_stats *stats);
int epi_ensemble_get_state(const epi_ensemble *x, int i, double *q);
int epi_ensemble_destroy(epi_ensemble *x);
/* Who drives the ensemble's KIOPS rounds (Sec. 4, Eq. 29: in each round
 * every member whose evaluation is still running takes one Arnoldi step or
 * evaluates its small exponential; one launch per kind for all members).
 *   DFR_ROUNDS_HOST (default): the host takes the decisions from read-backs
 *     of the exponentials' results and writes each round's call tables.
 *   DFR_ROUNDS_DEVICE: a planner kernel takes each member's
 *     controller decisions (the error ratio, acceptance, next sub-step and
 *     Krylov dimension) on the device and writes the round's call tables
 *     there; the round (planner and launches) is captured once in a HIP
 *     graph and replayed, the host only watching a progress word.  A member
 *     is decided in the round after its exponential, so none waits for a
 *     read-back; each group of members with the same p runs its products
 *     and updates on a graph branch of its own.  While ensemble timing is on
 *     the rounds are launched without the graph, so that events can bracket
 *     each launch.  At most 256 members.
 * Each member takes the same operations either way; decisions agree up to
 * the last bit of the log and pow of the two sides' math libraries.
 * DFR_E_INVAL for another mode.  dfr_ensemble_round_counts returns the
 * rounds with work and the rounds launched (those plus the few launched
 * ahead that found none, at most two per KIOPS call) by the device form,
 * summed since creation. */
enum { DFR_ROUNDS_HOST = 0, DFR_ROUNDS_DEVICE = 1 };
int dfr_ensemble_set_rounds(dfr_ensemble *e, int mode);
int dfr_ensemble_round_counts(const dfr_ensemble *e, int64_t *planned, int64_t *launched);

/* Concurrent form, for members that need not share order, dt or precision:
 * n_workers host threads take the members (contexts from dfr_create, each
 * ideally on its own stream), largest first, and run epi_step on them.
 * ctxs[i], states[i]: member i's context and state (contexts distinct, else
 * DFR_E_INVAL; members sharing a stream serialise on it).  stats: NULL or n
 * entries.  The first failure is returned (the message names the member);
 * members that completed their step stay advanced. */
int epi_step_concurrent(int n, dfr_ctx *const *ctxs, epi_state *const *states, const kiops_opts *opts, int n_workers,
                        kiops_stats *stats);

/* Kernel timing with HIP events, for measurement.  While enabled, every
 * kernel the library launches on the context's stream is bracketed by a pair
 * of events, classified by kind:
 *   DFR_K_JV_ARNOLDI  complex-step DFR kernel with the fused Arnoldi epilogue
 *   DFR_K_JV          complex-step DFR kernel (plain J*v, EPI remainder terms)
 *   DFR_K_RHS         real DFR kernel F(q)
 *   DFR_K_UPDATE      Gram-Schmidt update / normalisation kernel
 *   DFR_K_EXPM        small exponential (one workgroup)
 *   DFR_K_OTHER       vector kernels (start, combine, axpby, norms, checks)
 *   DFR_K_FINALIZE    one-block reductions of per-block partial sums
 * dfr_timing_enable(ctx, 1) clears the totals; dfr_timing_read synchronises
 * and returns the summed duration (ms) and launch count of one kind. */
enum { DFR_K_JV_ARNOLDI = 0, DFR_K_JV = 1, DFR_K_RHS = 2, DFR_K_UPDATE = 3, DFR_K_EXPM = 4, DFR_K_OTHER = 5,
       DFR_K_FINALIZE = 6, DFR_K_NKINDS = 7 };
int dfr_timing_enable(dfr_ctx *ctx, int enable);
int dfr_timing_read(dfr_ctx *ctx, int kind, double *total_ms, int64_t *launches);
/* The same for the batched launches of an ensemble (epi_ensemble_step; not
 * the tuning launches of dfr_ensemble_autotune), which run on the stream
 * given to dfr_ensemble_create.  *nodes (may be NULL) receives the grid
 * nodes the DFR launches of that kind covered, summed over launches and
 * members (0 for the other kinds), so that bytes per node times nodes over
 * the summed duration is the launches' algorithmic bandwidth. */
int dfr_ensemble_timing_enable(dfr_ensemble *e, int enable);
int dfr_ensemble_timing_read(dfr_ensemble *e, int kind, double *total_ms, int64_t *launches, double *nodes);
/* The kinds the ensemble's timing brackets (bit k: kind k; all by default),
 * so that a measurement can time one kind and leave the others unbracketed.
 * DFR_E_INVAL for bits beyond DFR_K_NKINDS. */
int dfr_ensemble_timing_kinds(dfr_ensemble *e, unsigned mask);

/* Measurement helper, not part of the method: copies `bytes` from src to dst
 * (device pointers, both 16-byte aligned, bytes a multiple of 16, not
 * overlapping) on `hip_stream` (NULL = default stream) with one 16-byte load
 * and store per lane, in a grid of up to 131072 workgroups of 512 threads.
 * Timed over a large buffer it gives the streaming bandwidth a kernel
 * reaches on the device, the practical ceiling beside the published peak.
 * Asynchronous.  DFR_E_INVAL for a null pointer, misalignment or a size not
 * a multiple of 16. */
int dfr_stream_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

const char *dfr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DFRSW_H */
