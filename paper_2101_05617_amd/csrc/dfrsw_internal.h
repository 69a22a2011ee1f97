// Internal declarations of the MI355X DFR shallow-water library.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dfrsw.h"

namespace dfrsw {

constexpr int MAX_NS = 8;        // p <= 7
constexpr int MAX_M = 64;        // Krylov dimension cap
constexpr int MAX_P = 8;         // phi-functions in one combination
constexpr int BLOCK = 256;       // threads per block of the DFR and vector kernels
#ifndef DFR_EXPM_BLOCK
#define DFR_EXPM_BLOCK 1024
#endif
constexpr int EXPM_BLOCK = DFR_EXPM_BLOCK;  // one workgroup of the small exponential (a multiple of 64)
#ifndef DFR_NOALLOC_SCRATCH_BYTES
#define DFR_NOALLOC_SCRATCH_BYTES (16u << 20)   // device scratch array of dfr_jvp_complex_step_noalloc
#endif
// look up the device address of that array for `device` (current), once
int scratch_init(int device);

void set_error(const std::string &msg);

// A valid precision with an eps that the complex evaluation can carry: any
// positive eps in FP64, at least DFR_FP32_EPS_MIN in the FP32 forms.
inline bool eps_prec_ok(double eps, dfr_precision prec) {
  if (prec == DFR_FP64) return eps > 0.0;
  if (prec != DFR_FP32_JV && prec != DFR_FP32_JV_BASIS32) return false;
  return eps >= DFR_FP32_EPS_MIN;
}

#define DFR_HIP(call)                                                               \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::dfrsw::set_error(std::string(#call) + ": " + hipGetErrorString(e_));       \
      return DFR_E_HIP;                                                             \
    }                                                                               \
  } while (0)

// 1-D operators on the Gauss-Legendre points (Sec. 3.1).
struct Ops1D {
  double Dt[MAX_NS][MAX_NS + 2];   // derivative of the extended interpolant at the GL points
  double lm[MAX_NS], lp[MAX_NS];   // Lagrange basis at xi = -1, +1
};

// Collocation data of the diagnostics: GL weights and the derivative of the
// GL Lagrange basis at the GL points, Dg[m][k] = l'_k(xi_m).
struct DiagOps {
  double w[MAX_NS];
  double Dg[MAX_NS][MAX_NS];
};

// The stiff test problems of Sec. 5.1 (semi-discrete, second-order finite
// differences): kind 1 advection-diffusion-reaction on an n x n vertex grid
// with reflecting (Neumann) ends, kind 2 Burgers on n interior points with
// zero ends, kind 3 semilinear parabolic on n interior points with zero ends
// and time as unknown n.  isum: the trapezoid integral of x(1-x) (kind 3).
struct OdeArgs {
  int kind, n;
  int64_t len;   // number of unknowns
  double h, eps, alpha, gamma, isum;
};

// Per-abscissa tangent data: X = tan x, 1 + X^2, 1/(1 + X^2).
struct Tan3 {
  double x, ax, rax, pad;
};

// Everything the DFR kernel needs about the grid (passed by value).
struct GridArgs {
  int ne;
  int64_t nelem;          // 6 ne^2
  int64_t n;              // nodes
  double g_red;           // gravity / radius^2
  double omega;
  double two_over_delta;  // 2 / element width in x
  double cA[6], cB[6], cC[6];      // Coriolis factor A + X B + Y C per panel
  int nb_q[6][4], nb_e[6][4], nb_rev[6][4];   // panel-edge neighbours
  const Tan3 *tnode;      // ne*ns abscissae of GL nodes
  const double *tedge;    // ne+1 element-edge tangents
  const double *xform;    // [6][4][ne*ns][4]: own <- neighbour contravariant map at panel edges
  const double *orog;     // NULL or [2][N]: (g/a^2) (h^{i1} dhB_1 + h^{i2} dhB_2) * a^2 ... per node
  int *err_flag;          // latched kernel error (vector atomics only)
  int riemann;            // common flux at element faces: 0 Rusanov, 1 AUSM
};

// Optional Arnoldi prologue/epilogue of the J*v kernel (one KIOPS iteration).
// The prologue finalises the previous kernel's reduction (partial sums `pin`)
// in a fixed order, identically in every workgroup: the norm of the vector
// built by the previous update (or of the start vector), hence sigma_j and
// the bottom block b_j; workgroup 0 records them in KDev.
struct ArnoldiArgs {
  int on;                 // 0: plain J*v
  int j;                  // index of the basis vector being multiplied
  int p;                  // number of W columns
  int start;              // 1: v_j is the sub-step's start vector
  const double *W[MAX_P]; // scaled b-vectors, column k pairs with bottom entry k
  int wil;                // 0: W[k] separate; 1: W[0] holds the columns interleaved, 4 per value
                          //    (p <= 4), FP64 or FP32; 3: three FP32 per value (FP32 basis, p <= 3):
                          //    see wil_code.  Otherwise, for 1: FP64, or
                          //    FP32 when the basis is FP32

  const void *vprev;      // v~_{j-1} as stored (basis element type) or NULL (iop = 1)
  const double *pin;      // partial sums of the previous kernel, one per workgroup
  int np_in;
  double *pout;           // this kernel's partial inner products, two per workgroup
  struct KDev *kd;
  double tol;
  double ybot[MAX_P];     // mu y(t) of the start vector (start only)
};

// One member's part of a batched launch (several grids in one kernel
// launch).  A member owns the workgroups (or, for the DFR kernel, the
// logical blocks) [b0, b0 + nblk).
struct DfrCall {
  const GridArgs *g;      // device copy of the member's grid arguments
  const Ops1D *ops;       // device copy of its 1-D operators
  int g_ne;              // its ne
  int TX, TY;             // its tile
  int b0, ntiles;
  const void *q;          // state (double, or float in the FP32 form)
  const void *v;          // direction (double, or float for an FP32 basis)
  const double *vscale;
  double eps;
  void *out;              // result (the type of v)
  ArnoldiArgs ar;
};
// basis vectors (out, w, vj, vprev, v0, V) are double, or float for an FP32
// basis (the same for every call of a launch)
struct FirstCall {
  int b0, nblk;
  int64_t n3;
  ArnoldiArgs ar;
  void *out;
};
struct UpdateCall {
  int b0, nblk;
  int64_t n3;
  int j, p;
  void *w;
  const void *vj, *vprev;
  const double *pin;
  int np_in;
  double *pout;
  struct KDev *kd;
};
struct StartCall {
  int b0, nblk;
  int64_t n3;
  const double *x;
  void *v0;
  double *pout;
  struct KDev *kd;        // its happy-breakdown flag is cleared
};
struct CombineCall {
  int b0, nblk;
  int64_t n3;
  const void *V;
  const struct KDev *kd;
  double *x;
};
struct PreCall {          // device-controlled rounds: combination and / or start (arnoldi_pre_batch)
  int b0, nblk;
  int64_t n3;
  int comb, start;        // the accepted sub-step's combination; the next sub-step's start vector
  void *V;                // the member's basis (slot 0 is the start vector)
  struct KDev *kd;
  double *x;              // the result: written by the combination, read by the start
  double *pout;           // the start's partial squared norms, one per workgroup
};
// The interleaved layout of the b-columns W for p columns: FP32 columns (an
// FP32 Krylov basis) with at most three are stored three per value (12 bytes,
// read with one 12-byte load); otherwise four per value (padded).  Returns
// the ArnoldiArgs::wil code, 3 or 1.
inline int wil_code(bool f32, int p) { return (f32 && p <= 3) ? 3 : 1; }

struct WilCall {         // W = nu [cols] interleaved four per value (a member's b-columns)
  int b0, nblk;
  int64_t n;
  int p;
  double nu;
  const double *cols[4];
  double *out;
  int f32;                // 1: as four FP32 values (a member with an FP32 Krylov basis)
};
struct ExpmCall {        // one workgroup per member
  struct KDev *kd;
  double tau;
  struct KHost *res;
  int jfin;
  const double *pin;
  int np_in;
  double tol;
};
struct AxpbyCall {       // out = a x + b y (y may be NULL); also norms, copies, checks
  int b0, nblk;
  int64_t n;
  double a, b;
  const double *x, *y;
  double *out;
};

// Device-controlled rounds of the batched form.  A planner kernel takes each
// member's controller decisions on the device and writes the round's call
// tables and their counts into device memory; the batched kernels read the
// counts from there (DevCounts), so that a round is a fixed sequence of
// launches, captured once in a HIP graph and replayed.
struct DevCounts {
  int n_pre, nb_pre;               // calls and blocks of each launch
  int n_first, nb_first;
  int n_expm, pad0;
  int dfr[MAX_NS + 1][2];          // the products, by number of GL points: calls, logical blocks
  int upd[MAX_NS + 1][2];          // the updates, by the members' number of GL points: calls, workgroups
  int last_work;                   // the last round with any work
  int round;                       // rounds planned so far
};
// The planner's progress word, mirrored to mapped host memory in one 64-bit
// store: rounds planned (high half) and the rounds certainly still needed
// after the last one (low half; 0 once every member has ended).
__host__ __device__ inline unsigned long long dev_progress(int round, int need) {
  return ((unsigned long long)(unsigned)round << 32) | (unsigned)need;
}
// one member's constants for one KIOPS call (device copy)
struct DevMember {
  int64_t n3;
  int ns, esz;                     // GL points; bytes per basis value (4: FP32 basis)
  int nblk_vec, nblk_upd, ntiles;  // workgroups of its vector launches and update; product tiles
  int TX, TY, g_ne, wil;
  char *V;                         // basis slots of 3N values
  double *W, *w;                   // b-columns; the result
  const void *q;                   // the state the product reads (FP32 copy with FP32 products)
  double *pA, *pB;                 // partial sums: product -> update, update / start -> product
  struct KDev *kd;
  const GridArgs *g;
  const Ops1D *ops;
  double eps, tau_out, tol, nu, mu;
  int p, n_phi, b0_absent, m_min, m_max, iop, max_attempts, pad1;
};
// one member's controller state (the host KiopsMachine's fields, on the device)
enum { KC_BEGIN = 0, KC_SWEEP = 1, KC_EXPM = 2, KC_WAIT = 3, KC_DONE = 4, KC_FAILED = 5 };
constexpr int KC_E_FIRST_LATE = -100;   // planner: a first Arnoldi step after a call's first round
struct KCtl {
  int phase;                       // 0 begin, 1 sweep, 2 exponential, 3 waiting for its result, 4 done, 5 failed
  int j, m, j_sweep, skipped, ireject, old_m, attempts;
  int npA, npB, err, pad;
  double t, tau, beta0, old_tau, old_omega;
  double ybot[MAX_P];
  int n_matvec, n_substeps, n_rejected, m_last, happy, n_expm;
};

// Device-side KIOPS state (one per context).
struct KDev {
  double H[(MAX_M + 2) * (MAX_M + 2)];     // Hessenberg, row-major, ld = MAX_M + 2
  double sigma[MAX_M + 2];                 // scale of the stored (unnormalised) top vectors
  double bot[(MAX_M + 2) * MAX_P];         // bottom blocks (normalised)
  double botu[(MAX_M + 2) * MAX_P];        // bottom blocks before normalisation
  double wn2[MAX_M + 2];                   // squared norms of botu
  double beta;
  double E0[MAX_M + 2];                    // first column of the small exponential
  double err;                              // error estimate of the last exponential
  double hlast;                            // h_{J,J-1}
  double eJ;                               // E[J-1][J]
  int J;
  int happy;
  int pad[2];
};

// Result block copied to the host after each small exponential.
struct KHost {
  double err, beta, hlast, eJ;
  int J, happy, pad[2];
};

// Results the host waits for inside KIOPS, written by the kernels that
// produce them straight into mapped, coherent host memory; seq is written
// last, after a system-scope fence, and the host polls it.
struct HostMail {
  KHost kh;
  double nrm2[MAX_P + 1];
  int err;                        // the latched error flags, handed over and cleared
  unsigned seq;
};

// Per-kernel timing with HIP events: while on, each launch takes a start /
// stop event pair that the runtime stamps at the kernel's own dispatch and
// completion (hipExtLaunchKernelGGL), so no marker packets enter the stream.
// Launches are classified by kind (DFR_K_*); `units` is a per-launch count
// the caller chooses (the batched DFR launches record their nodes).
struct KTimer {
  bool on = false;
  unsigned kinds = ~0u;            // the kinds bracketed while on (bit k: kind k)
  struct EvPair {
    hipEvent_t a, b;
    int kind;
    double units;
  };
  std::vector<EvPair> pool;
  size_t used = 0;
  double t_ms[DFR_K_NKINDS] = {0};
  int64_t t_n[DFR_K_NKINDS] = {0};
  double t_units[DFR_K_NKINDS] = {0};
};
bool timing_slot(KTimer *t, int kind, double units, hipEvent_t *start, hipEvent_t *stop);
void timing_done(KTimer *t);
void timing_fold(KTimer &t);       // wait for the recorded launches and add them up
void timing_reset(KTimer &t, bool on);
void timing_free(KTimer &t);

struct Ctx {
  int ne, ns, p_deg;
  int64_t n, nelem;
  int64_t n3 = 0;                 // length of a state vector (3 N on a grid)
  // a Sec. 5.1 test problem instead of a grid (0: the shallow-water grid)
  int ode_kind = 0;
  OdeArgs ode{};
  double radius, omega, gravity;
  double lam0, phi0, alp0;
  hipStream_t stream;
  int device;
  // host geometry
  std::vector<double> xi, wgl;
  Ops1D ops;
  double ec[6][3], e1[6][3], e2[6][3];
  GridArgs ga;
  // device buffers
  Tan3 *d_tnode = nullptr;
  double *d_tedge = nullptr, *d_xform = nullptr, *d_orog = nullptr;
  double *d_hB = nullptr;         // nodal orography (N) or NULL
  DiagOps dops;
  double *d_diag = nullptr;       // diagnostics: 3 partial sums per workgroup, then the 3 totals
  int *d_err = nullptr;
  // KIOPS workspace
  int kiops_mmax = 0, kiops_p = 0;
  int max_m = MAX_M;              // Krylov cap from the LDS available to one workgroup
  int tile_tx = 1, tile_ty = 1;   // elements per workgroup of the DFR kernel (x^1, x^2)
  int ar_tx = 1, ar_ty = 1;       // the same for the J*v kernel with the Arnoldi prologue/epilogue
  size_t lds_limit = 65536;       // LDS one workgroup may use
  double *d_V = nullptr;          // (MAX_M + 1) top vectors of 3N (FP64, or FP32 when basis32)
  bool basis32 = false;           // the current KIOPS call keeps its basis in FP32
  bool w_il = false;              // the current KIOPS call keeps W interleaved (W_IL)
  void *vslot(int k) const {
    return reinterpret_cast<char *>(d_V) + (size_t)k * (size_t)n3 * (basis32 ? sizeof(float) : sizeof(double));
  }
  double *d_W = nullptr;          // MAX_P scaled b columns of 3N
  double *d_partials = nullptr;   // per-block partial sums (J*v inner products)
  double *d_partials2 = nullptr;  // per-block partial sums (norms)
  unsigned *d_counter = nullptr;
  KDev *d_kd = nullptr;
  HostMail *mail = nullptr;       // mapped host memory (host address)
  HostMail *d_mail = nullptr;     // the same memory, device address
  unsigned mail_seq = 0;          // last sequence number asked for
  double *d_qf32 = nullptr;       // FP32 copy of the linearisation state (as float*)
  double *d_tmp = nullptr;        // scratch vector 3N
  // optional per-kernel event timing
  KTimer tm;
};

// a launch on timer t's terms (timed while t is on), on stream s
template <typename... KArgs, typename... Args>
inline void timed_launch(KTimer *t, int kind, double units, hipStream_t s, void (*kernel)(KArgs...), dim3 grid,
                         dim3 block, size_t shmem, Args... args) {
  hipEvent_t e0, e1;
  if (t && timing_slot(t, kind, units, &e0, &e1)) {
    hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)shmem, s, e0, e1, 0, args...);
    timing_done(t);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
  }
}

template <typename... KArgs, typename... Args>
inline void dfr_launch(Ctx *c, int kind, void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t shmem,
                       Args... args) {
  timed_launch(&c->tm, kind, 0.0, c->stream, kernel, grid, block, shmem, args...);
}

// kernels.hip
// v, out and the basis slots are FP64, or FP32 in the Krylov form when
// c->basis32 (the product of the FP32 form with an FP32 basis)
int launch_dfr(Ctx *c, const double *q, const float *q32, const void *v, const double *vscale,
               double eps, bool complex_step, bool fp32, void *out, const ArnoldiArgs *ar);
int launch_arnoldi_first(Ctx *c, const ArnoldiArgs &ar, void *out, int *np_out);
int launch_update(Ctx *c, int j, void *w, const void *vj, const void *vprev, const double *pin, int np_in,
                  double *pout, int *np_out);
int launch_start(Ctx *c, const double *x, void *v0, double *pout, int *np_out);
int launch_combine(Ctx *c, double *x);
int launch_expm(Ctx *c, double tau, int jfin, const double *pin, int np_in, double tol, unsigned seq);   // -> d_mail
int launch_axpby(Ctx *c, int64_t n, double a, const double *x, double b, const double *y, double *out);
int launch_copy_to_f32(Ctx *c, int64_t n, const double *x, float *y);
// W interleaved: out[4 i + k] = nu * cols[k][i] for k < p (NULL: zero), 0 for p <= k < 4; FP64, or
// FP32 (f32) for a KIOPS call with an FP32 basis, whose Krylov-form product reads it so
int launch_w_interleave(Ctx *c, int64_t n, int p, double nu, const double *const *cols, double *out,
                        bool f32 = false);
int64_t diag_blocks(const Ctx *c);
int launch_diagnostics(Ctx *c, const double *q, double *zeta, double *fcor);
int launch_check_state(Ctx *c, const double *q);
int launch_ode(Ctx *c, const double *q, const double *v, const double *vscale, bool jvp, double *out,
               const ArnoldiArgs *ar);
int launch_fill(Ctx *c, double *q, double *v);
int latched_error(Ctx &c);
size_t dfr_lds_bytes(int ns, int tx, int ty, bool fp32);
int dfr_set_lds_limits(Ctx *c, size_t bytes);
// KIOPS (kiops.hip): statistics of one run and its controller as a state
// machine, shared by the single-grid driver and the batched driver.
struct KiopsRun {
  int n_matvec = 0, n_substeps = 0, n_rejected = 0, m_last = 0, happy = 0, n_expm = 0;
};
struct KiopsMachine {
  Ctx *c = nullptr;
  const double *q = nullptr;
  const float *q32 = nullptr;
  const double *b[MAX_P + 1] = {};
  double *w = nullptr;
  double tau_out = 0.0, eps = 0.0;
  bool fp32 = false;
  int n_phi = 0, p = 0;
  bool b0_absent = true;
  double nu = 1.0, mu = 1.0;
  int m = 0, m_min = 0, m_max = 0;
  double t = 0.0, tau = 0.0;
  int j = 0;
  double beta0 = -1.0;
  int ireject = 0;
  double old_tau = 0.0, old_omega = 0.0;
  int old_m = -1, attempts = 0;
  double ybot[MAX_P] = {};
  int j_sweep = 0;
  bool skipped = false, need_start = false;
  int npA = 0, npB = 0;
  enum Phase { BEGIN, SWEEP, EXPM, DONE } phase = BEGIN;
  KiopsRun st;
};
int kiops_validate(const Ctx &c, const kiops_opts &o, int n_phi, double tau_out);
bool km_init(KiopsMachine &k, const double *nrm2, const kiops_opts &o);
int km_begin_attempt(KiopsMachine &k, const kiops_opts &o);
void km_arnoldi_args(const KiopsMachine &k, const kiops_opts &o, ArnoldiArgs &ar);
int km_decide(KiopsMachine &k, const KHost &r, const kiops_opts &o, bool *accept);
int latched_error(Ctx &c);
void epi_table(int order, std::vector<std::vector<double>> &A);
void add_stats(kiops_stats *acc, const KiopsRun &r);
}  // namespace dfrsw
struct epi_state;
namespace dfrsw {
void epi_rotate(epi_state *st, double *q_new);

// Staging arena for the call tables of batched launches: a pinned host arena
// and its device mirror.  Each table is copied on the stream before its
// launch; in deferred mode the tables put since stage_defer() go to the
// device in one transfer in stage_flush(), which then issues the launches
// queued meanwhile, in their order.  The arena is reset (reset_stage) only
// after the stream has been synchronised.
struct Stage {
  KTimer *timer = nullptr;                        // times the batched launches while on
  char *h = nullptr, *d = nullptr;
  size_t cap = 0, used = 0;
  bool defer = false;
  size_t pend0 = 0;                               // start of the range not yet copied
  std::vector<std::function<int()>> pending;      // launches waiting for that copy
};
int stage_put(Stage &st, hipStream_t s, const void *src, size_t bytes, void **dev);
int stage_launch(Stage &st, std::function<int()> launch);   // now, or queued in deferred mode
inline void stage_defer(Stage &st) {
  st.defer = true;
  st.pend0 = st.used;
}
int stage_flush(Stage &st, hipStream_t s);     // copy, issue the queued launches, leave deferred mode
inline void reset_stage(Stage &st) {
  st.used = 0;
  st.pend0 = 0;
}

// batched launches: every call of one launch has the same form (and, for the
// DFR kernel, the same number of GL points ns)
int launch_dfr_batch(hipStream_t s, Stage &st, int ns, bool complex_step, bool fp32, bool arnoldi, bool basis32,
                     std::vector<DfrCall> &calls);
int launch_first_batch(hipStream_t s, Stage &st, bool basis32, std::vector<FirstCall> &calls);
int launch_update_batch(hipStream_t s, Stage &st, bool basis32, std::vector<UpdateCall> &calls);
int launch_start_batch(hipStream_t s, Stage &st, bool basis32, std::vector<StartCall> &calls);
int launch_combine_batch(hipStream_t s, Stage &st, bool basis32, std::vector<CombineCall> &calls);
int launch_expm_batch(hipStream_t s, Stage &st, std::vector<ExpmCall> &calls, size_t lds);
// the device-controlled round (devctl.hip): its launches, on stream s, with
// every table and count in device memory (capturable); grids sized for every
// member active
struct DevRound {
  int nmem;                        // members (at most 256: the planner's workgroup)
  const DevMember *mem;            // device
  KCtl *ctl;                       // device
  KHost *kh;                       // device: the exponentials' results, per member
  DevCounts *cnt;                  // device
  unsigned long long *progress;    // device address of mapped host memory (dev_progress)
  PreCall *pre;                    // device tables, nmem entries each
  FirstCall *first;
  UpdateCall *upd;                 // nmem entries, grouped like dfr
  ExpmCall *expm;
  DfrCall *dfr;                    // nmem entries, grouped by number of GL points
  int grid_vec;                    // workgroups of the combination / start and first launches (blocks in turn)
  int grp_base[MAX_NS + 1];        // first entry of each group in dfr and upd
  int grp_n[MAX_NS + 1];           // members of each group (0: no launch)
  int grp_maxlog[MAX_NS + 1];      // logical blocks of each group with every member active
  int grp_maxupd[MAX_NS + 1];      // update workgroups of each group with every member active
  int grp_threads[MAX_NS + 1];
  size_t grp_lds[MAX_NS + 1];
  size_t expm_lds;
  int fp32, basis32;
  int pmax;                        // the largest p of the members
};
// first: the first round of a KIOPS call (the only one with first Arnoldi
// steps of a zero top block).  tm: NULL, or a timer whose events bracket
// each launch.  br: NULL (every launch on s), or streams and events with
// which each group's product and update run on a branch of their own
// (forked from s after the first steps, joined before the exponentials;
// for capture into a graph)
struct DevBranches {
  hipStream_t side[MAX_NS + 1];
  hipEvent_t fork, join[MAX_NS + 1];
};
int launch_dev_round(hipStream_t s, const DevRound &r, bool first, KTimer *tm, const DevBranches *br);
enum { KD_PRE = 0, KD_FIRST = 1, KD_UPDATE = 2 };
int launch_dfr_batch_dev(hipStream_t s, int ns, bool fp32, bool basis32, const DfrCall *calls, const int *dc,
                         int grid, int threads, size_t lds, KTimer *tm);
// pmax: the largest p of the calls (the update's bottom-block loops)
int launch_krylov_dev(hipStream_t s, int kind, bool basis32, const void *calls, const int *dc, int grid, int pmax,
                      KTimer *tm);
int launch_expm_dev(hipStream_t s, const ExpmCall *calls, const int *dc, int grid, size_t lds, KTimer *tm);
enum { VB_AXPBY = 0, VB_TO_F32 = 1, VB_NORM2 = 2, VB_SUM = 3, VB_CHECK = 4 };
int launch_vec_batch(hipStream_t s, Stage &st, int kind, std::vector<AxpbyCall> &calls);
int launch_wil_batch(hipStream_t s, Stage &st, std::vector<WilCall> &calls);   // W of several members, one launch
int vec_blocks(int64_t n);   // workgroups of a vector kernel on n values (at most 1024)

int64_t dfr_grid_blocks(const Ctx *c, bool arnoldi);
int64_t dfr_num_tiles(const Ctx *c, bool arnoldi);
std::vector<std::pair<int, int>> tile_candidates(const Ctx &c);   // admissible tiles (api.hip)
int launch_norm2(Ctx *c, int64_t n, const double *x, double *partials, int nblk);
// the squared 2-norms of k <= MAX_P + 1 vectors (NULL: 0) into out[0..k)
// (device), two launches; partials: k * 1024 doubles of scratch
int launch_norms2(Ctx *c, int64_t n, int k, const double *const *x, double *partials, unsigned seq);   // -> d_mail
int launch_err_mail(Ctx *c, unsigned seq);   // d_err -> d_mail->err, d_err cleared
int mail_wait(Ctx &c, unsigned seq);          // wait for result seq in c.mail (api.hip)
// out_o = sum_i a[o][i] in_i for up to four inputs and four outputs (one pass)
struct LinComb {
  int nin, nout;
  const double *in[4];
  double *out[4];
  double a[4][4];
};
int launch_lincomb(Ctx *c, int64_t n, const LinComb &lc);
struct LinCombCall {     // one member's linear combination in a batched launch
  int b0, nblk;
  int64_t n;
  LinComb lc;
};
int launch_lincomb_batch(hipStream_t s, Stage &st, std::vector<LinCombCall> &calls);
int launch_sum(Ctx *c, int np, const double *partials, double *out);

}  // namespace dfrsw

// Multistep EPI integrator state (kiops.hip): history q_{n-i}, F(q_{n-i}),
// remainders, b-vectors.
struct epi_state {
  dfrsw::Ctx *c;
  int order, P, M;
  double dt;
  int s;
  double eps;
  dfr_precision prec;
  int64_t nsteps;
  double *q, *F, *qs, *w, *d, *jd;
  std::vector<double *> hq, hF, R, bm;
  std::vector<std::vector<double>> A;   // alpha_{m,i}
};

struct dfr_ctx {
  dfrsw::Ctx c;
};
