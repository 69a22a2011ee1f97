// KIOPS-type adaptive Krylov evaluation of phi-combinations (Eq. 29) and the
// multistep EPI integrators (Sec. 4, Eqs. 25, 30, 34-38) on the GPU.
//
// Host code here only takes control decisions (sub-step size tau, Krylov
// dimension m, accept/reject) from a few scalars that the exponential kernel
// writes into mapped host memory once per small exponential; every vector
// operation, inner product, norm, the Hessenberg matrix and its exponential
// live on the device.
//
// Controller (the paper defers KIOPS's internals to its own publication; this
// is a complete statement of the one used here):
//   augmented operator A~ = [[J, W], [0, K]], W = nu [b_p .. b_1], bottom
//     state mu y(t), y(t) = (t^{p-1}/(p-1)!, .., t, 1), nu = 2^-e, mu = 2^e,
//     e = ceil(log2 max_k ||b_k||) (k >= 1); p = 0 runs as p = 1, b_1 = 0
//   Arnoldi with incomplete orthogonalisation against the last iop (<= 2)
//     vectors, classical Gram-Schmidt; happy breakdown if ||w|| < tol
//   E = exp(tau [[H_J, e_1], [0, 0]]); x(t+tau) = beta V_J E[:J, 0];
//     err = beta h_{J+1,J} |E[J-1, J]|
//   omega = (tau_out/tau) err / (tol beta_0), accept if omega <= 1.2
//   order q = log(omega/omega_old)/log(tau/tau_old) (>= 1) after a rejection
//     with equal m, else J/4; rate k = (omega/omega_old)^(1/(m_old-m)) (>= 1.1)
//     after a rejection with equal tau, else 2
//   tau_opt = clamp(tau (0.2/omega)^(1/q), tau/5, 5 tau) <= remaining
//   m_opt = clamp(ceil(J + log(omega/0.2)/log k), max(m_min, floor(3m/4)),
//                 min(m_max, ceil(4m/3)))
//   J == m_max: reject -> tau_new = max(tau/5, tau (0.6/omega)^(1/q)), m = J;
//               accept -> tau_new = tau_opt; otherwise m_new = m_opt, tau kept
//   a rejected attempt keeps the basis (larger m continues Arnoldi)
#include "dfrsw_internal.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

namespace dfrsw {

int latched_error(Ctx &c);

// squared norms of the b-vectors: one pair of launches, the sums written to
// host memory
static int norms2(Ctx &c, int k, const double *const *x, double *host_out) {
  const unsigned seq = ++c.mail_seq;
  int rc = launch_norms2(&c, c.n3, k, x, c.d_partials, seq);
  if (rc) return rc;
  if ((rc = mail_wait(c, seq))) return rc;
  for (int i = 0; i < k; ++i) host_out[i] = c.mail->nrm2[i];
  return DFR_OK;
}

int kiops_validate(const Ctx &c, const kiops_opts &o, int n_phi, double tau_out) {
  if (!(tau_out > 0.0) || !(o.tol > 0.0) || o.m_max < 1 || o.m_max > MAX_M || o.m_min < 1 || o.iop < 1 ||
      o.iop > 2 || n_phi < 0 || n_phi > MAX_P) {
    set_error("kiops: invalid options (need tau > 0, tol > 0, 1 <= m_min, m_max <= 64, iop = 1 or 2, n_phi <= 8)");
    return DFR_E_INVAL;
  }
  if (o.m_max > c.max_m) {
    set_error("kiops: m_max exceeds the Krylov dimension this device supports (" + std::to_string(c.max_m) + ")");
    return DFR_E_INVAL;
  }
  return DFR_OK;
}

// Scaling of the augmented operator from the norms ||b_k||^2 (K1) and the
// initial controller state.  Returns false if every b_k is zero (w = 0).
bool km_init(KiopsMachine &k, const double *nrm2, const kiops_opts &o) {
  double nb = 0.0;
  for (int i = 1; i <= k.n_phi; ++i) nb = std::max(nb, std::sqrt(nrm2[i]));
  if (nb == 0.0 && nrm2[0] == 0.0) return false;
  k.nu = k.mu = 1.0;
  if (nb > 0.0) {
    const int e = (int)std::ceil(std::log2(nb));
    k.nu = std::ldexp(1.0, -e);
    k.mu = std::ldexp(1.0, e);
  }
  k.p = k.n_phi == 0 ? 1 : k.n_phi;
  k.m_max = o.m_max;
  k.m_min = std::min(o.m_min, o.m_max);
  k.m = std::max(k.m_min, std::min(o.m_init, k.m_max));
  k.t = 0.0;
  k.tau = k.tau_out;
  k.j = 0;
  k.beta0 = -1.0;
  k.ireject = 0;
  k.old_tau = k.old_omega = 0.0;
  k.old_m = -1;
  k.attempts = 0;
  k.phase = KiopsMachine::BEGIN;
  return true;
}

// Start of an attempt (a sweep continued or begun, then one exponential).
int km_begin_attempt(KiopsMachine &k, const kiops_opts &o) {
  if (++k.attempts > o.max_attempts) {
    set_error("kiops: no convergence within max_attempts");
    return DFR_E_KIOPS;
  }
  if (o.replay && o.replay->play) {
    // replay: the attempt takes the next recorded (tau, m) instead of the
    // controller's; its accept is applied by km_decide
    const kiops_replay &R = *o.replay;
    const std::string at = "kiops replay, decision " + std::to_string(R.pos) + ": ";
    if (R.pos < 0 || R.pos >= R.n_play) {
      set_error(at + "the decisions ran out before the end of the step");
      return DFR_E_KIOPS;
    }
    const kiops_decision &d = R.play[R.pos];
    if (!(d.tau > 0.0) || !std::isfinite(d.tau)) {
      set_error(at + "tau is not a positive finite number");
      return DFR_E_KIOPS;
    }
    // K7: a sub-step may not pass tau_out (the controller clips tau to the
    // remaining interval; a relative 1e-12 allows for rounding)
    if (d.tau > (k.tau_out - k.t) + 1e-12 * k.tau_out) {
      set_error(at + "tau passes the end of the interval");
      return DFR_E_KIOPS;
    }
    if (d.m < 1 || d.m > k.m_max || d.m < k.j) {
      set_error(at + "m = " + std::to_string(d.m) + " outside [max(1, " + std::to_string(k.j) +
                " basis vectors built), m_max = " + std::to_string(k.m_max) + "]");
      return DFR_E_KIOPS;
    }
    k.tau = d.tau;
    k.m = d.m;
  }
  k.j_sweep = k.j;
  k.skipped = false;
  k.need_start = (k.j == 0);
  if (k.need_start) {
    for (int i = 0; i < k.p; ++i) {
      const int pw = k.p - 1 - i;
      double f = 1.0;
      for (int r = 2; r <= pw; ++r) f *= r;
      k.ybot[i] = k.mu * std::pow(k.t, (double)pw) / f;
    }
  }
  k.phase = k.j < k.m ? KiopsMachine::SWEEP : KiopsMachine::EXPM;
  return DFR_OK;
}

// Arguments of the Krylov-form product for basis vector j.
void km_arnoldi_args(const KiopsMachine &k, const kiops_opts &o, ArnoldiArgs &ar) {
  const Ctx &c = *k.c;
  const int64_t n3 = c.n3;
  ar = ArnoldiArgs{};
  ar.on = 1;
  ar.j = k.j;
  ar.p = k.p;
  ar.start = (k.j == 0);
  for (int i = 0; i < k.p; ++i) {
    ar.W[i] = c.w_il ? c.d_W : c.d_W + i * n3;
    ar.ybot[i] = k.ybot[i];
  }
  ar.wil = c.w_il ? wil_code(c.basis32, k.p) : 0;
  ar.vprev = (k.j >= 1 && o.iop >= 2) ? c.vslot(k.j - 1) : nullptr;
  ar.pin = c.d_partials2;
  ar.np_in = k.npB;
  ar.pout = c.d_partials;
  ar.kd = c.d_kd;
  ar.tol = o.tol;
}

// The controller after one exponential (K4-K7).  Sets *accept; the caller
// forms the accepted sub-step's result (combination kernel) before the next
// attempt.
int km_decide(KiopsMachine &k, const KHost &r, const kiops_opts &o, bool *accept_out) {
  const double DELTA = 1.2, GAMMA = 0.2, GAMMA_MMAX = 0.6;
  k.st.n_expm++;
  const int J = r.J;
  k.st.n_matvec += (J - k.j_sweep) - (k.skipped ? 1 : 0);
  if (k.beta0 < 0.0) k.beta0 = r.beta;
  if (!std::isfinite(r.err) || !std::isfinite(r.beta)) {
    set_error("kiops: non-finite Krylov quantities");
    return DFR_E_NONFINITE;
  }
  const double tau = k.tau, tau_out = k.tau_out, t = k.t;
  const int m = k.m;
  bool accept;
  double omega, tau_new;
  int m_new;
  if (r.happy) {
    k.j = J;
    omega = 0.0;
    accept = true;
    m_new = m;
    tau_new = std::min(tau_out - (t + tau), tau);
    k.st.happy = 1;
  } else {
    omega = (tau_out / tau) * r.err / (o.tol * k.beta0);
    omega = std::max(omega, 1e-300);
    accept = omega <= DELTA;
    double order;
    if (k.ireject >= 1 && m == k.old_m && tau != k.old_tau)
      order = std::max(1.0, std::log(omega / k.old_omega) / std::log(tau / k.old_tau));
    else
      order = J / 4.0;
    double kest;
    if (k.ireject >= 1 && m != k.old_m && tau == k.old_tau)
      kest = std::max(1.1, std::pow(omega / k.old_omega, 1.0 / (k.old_m - m)));
    else
      kest = 2.0;
    const double remaining = accept ? tau_out - (t + tau) : tau_out - t;
    double tau_opt = tau * std::pow(GAMMA / omega, 1.0 / order);
    tau_opt = std::min(remaining, std::max(tau / 5.0, std::min(5.0 * tau, tau_opt)));
    int m_opt = (int)std::ceil(J + std::log(omega / GAMMA) / std::log(kest));
    m_opt = std::max(k.m_min, std::min(k.m_max, std::max((int)std::floor(0.75 * m),
                                                          std::min(m_opt, (int)std::ceil(4.0 * m / 3.0)))));
    if (J == k.m_max) {
      if (omega > DELTA) {
        m_new = J;
        tau_new = tau * std::pow(GAMMA_MMAX / omega, 1.0 / order);
        tau_new = std::min(remaining, std::max(tau / 5.0, tau_new));
      } else {
        m_new = m;
        tau_new = tau_opt;
      }
    } else {
      m_new = m_opt;
      tau_new = std::min(remaining, tau);
    }
  }
  const bool replaying = o.replay && o.replay->play;
  if (replaying) {
    // the recorded decision (validated when the attempt began) overrides
    // the controller's; a happy breakdown must end the basis where the
    // record's did
    kiops_replay &R = *o.replay;
    const kiops_decision &d = R.play[R.pos];
    const std::string at = "kiops replay, decision " + std::to_string(R.pos) + ": ";
    if (J != d.m) {
      set_error(at + "a happy breakdown ended the Krylov basis at " + std::to_string(J) + " vectors, below m = " +
                std::to_string(d.m));
      return DFR_E_KIOPS;
    }
    if (r.happy && !d.accept) {
      set_error(at + "a happy breakdown in an attempt the record rejects");
      return DFR_E_KIOPS;
    }
    accept = d.accept != 0;
    R.pos++;
  }
  if (o.replay) {
    kiops_replay &R = *o.replay;
    if (R.rec && R.n_rec >= 0 && R.n_rec < R.rec_cap) R.rec[R.n_rec] = kiops_decision{tau, J, accept ? 1 : 0};
    R.n_rec++;
  }
  if (accept) {
    if (tau >= tau_out - t) k.t = tau_out;
    else k.t = t + tau;
    k.st.n_substeps++;
    k.st.m_last = J;
    k.j = 0;
    k.ireject = 0;
  } else {
    k.ireject++;
    k.st.n_rejected++;
  }
  k.old_tau = tau;
  k.old_m = m;
  k.old_omega = omega;
  k.tau = tau_new;
  k.m = m_new;
  *accept_out = accept;
  k.phase = k.t < tau_out ? KiopsMachine::BEGIN : KiopsMachine::DONE;
  if (!replaying && k.t < tau_out && !(k.tau > 0.0)) {
    set_error("kiops: step size collapsed");
    return DFR_E_KIOPS;
  }
  return DFR_OK;
}

// basis32: the basis vectors are kept in FP32 (the FP32 form only); inner
// products, norms, the Hessenberg and the combination stay FP64
static int kiops_core(Ctx &c, const double *q, const float *q32, double tau_out, int n_phi, const double *const *b,
                      const kiops_opts &o, double eps, bool fp32, bool basis32, double *w, KiopsRun &st) {
  const int64_t n3 = c.n3;
  int rc = kiops_validate(c, o, n_phi, tau_out);
  if (rc) return rc;
  // layouts of this call (basis precision, interleaved W), reset on exit
  struct BasisMode {
    Ctx &c;
    BasisMode(Ctx &cc, bool b32) : c(cc) {
      c.basis32 = b32;
      c.w_il = false;
    }
    ~BasisMode() {
      c.basis32 = false;
      c.w_il = false;
    }
  } mode(c, fp32 && basis32);
  KiopsMachine k;
  k.c = &c;
  k.q = q;
  k.q32 = q32;
  k.n_phi = n_phi;
  for (int i = 0; i <= n_phi; ++i) k.b[i] = b[i];
  k.b0_absent = (b[0] == nullptr);
  k.w = w;
  k.tau_out = tau_out;
  k.eps = eps;
  k.fp32 = fp32;
  // norms of b_0..b_p
  double nrm2[MAX_P + 1];
  rc = norms2(c, n_phi + 1, b, nrm2);
  if (rc) return rc;
  if (!km_init(k, nrm2, o)) {
    DFR_HIP(hipMemsetAsync(w, 0, sizeof(double) * n3, c.stream));
    DFR_HIP(hipStreamSynchronize(c.stream));
    return DFR_OK;
  }
  // W = nu [b_p, ..., b_1] (a zero column when there is no b_1); x = b_0
  // with at most four columns (every EPI order) W is kept interleaved, so
  // that the Krylov-form product reads it with wide loads
  c.w_il = !c.ode_kind && k.p <= 4;
  if (c.w_il) {
    const double *cols[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int i = 0; i < k.p; ++i) cols[i] = n_phi == 0 ? nullptr : b[k.p - i];
    rc = launch_w_interleave(&c, n3, k.p, k.nu, cols, c.d_W, c.basis32);
    if (rc) return rc;
  } else {
    for (int i = 0; i < k.p; ++i) {
      const double *bi = n_phi == 0 ? nullptr : b[k.p - i];
      rc = launch_axpby(&c, n3, k.nu, bi, 0.0, nullptr, c.d_W + i * n3);
      if (rc) return rc;
    }
  }
  c.kiops_p = k.p;
  c.kiops_mmax = k.m_max;
  rc = launch_axpby(&c, n3, 1.0, b[0], 0.0, nullptr, w);
  if (rc) return rc;

  double *pA = c.d_partials, *pB = c.d_partials2;
  while (k.phase != KiopsMachine::DONE) {
    rc = km_begin_attempt(k, o);
    if (rc) return rc;
    if (k.need_start) {
      rc = launch_start(&c, w, c.vslot(0), pB, &k.npB);
      if (rc) return rc;
    }
    while (k.j < k.m) {
      ArnoldiArgs ar;
      km_arnoldi_args(k, o, ar);
      void *out = c.vslot(k.j + 1);
      if (k.j == 0 && k.t == 0.0 && k.b0_absent) {
        rc = launch_arnoldi_first(&c, ar, out, &k.npA);
        k.skipped = true;
      } else {
        rc = launch_dfr(&c, q, q32, c.vslot(k.j), nullptr, eps, true, fp32, out, &ar);
        k.npA = (int)dfr_num_tiles(&c, true);
      }
      if (rc) return rc;
      rc = launch_update(&c, k.j, out, c.vslot(k.j), ar.vprev, pA, k.npA, pB, &k.npB);
      if (rc) return rc;
      ++k.j;
    }
    const unsigned seq = ++c.mail_seq;
    rc = launch_expm(&c, k.tau, k.j, pB, k.npB, o.tol, seq);
    if (rc) return rc;
    if ((rc = mail_wait(c, seq))) return rc;
    const KHost kh = c.mail->kh;
    bool accept = false;
    rc = km_decide(k, kh, o, &accept);
    if (rc == DFR_E_NONFINITE) {
      const int le = latched_error(c);
      return le ? le : rc;
    }
    if (rc) return rc;
    if (accept) {
      rc = launch_combine(&c, w);
      if (rc) return rc;
    }
  }
  st = k.st;
  return latched_error(c);   // every earlier operation on the stream has finished
}

// ---------------------------------------------------------------------------
// EPI
}  // namespace dfrsw



namespace dfrsw {

// Eq. (30) and Eqs. (36)-(38): rows m = 1..M, columns i = 1..P
void epi_table(int order, std::vector<std::vector<double>> &A) {
  A.clear();
  switch (order) {
    case 3: A = {{0.0}, {2.0 / 3.0}}; break;
    case 4: A = {{0.0, 0.0}, {-3.0 / 10.0, 3.0 / 40.0}, {32.0 / 5.0, -11.0 / 10.0}}; break;
    case 5:
      A = {{0.0, 0.0, 0.0}, {-4.0 / 5.0, 2.0 / 5.0, -4.0 / 45.0}, {12.0, -9.0 / 2.0, 8.0 / 9.0}, {3.0, 0.0, -1.0 / 3.0}};
      break;
    case 6:
      A = {{0.0, 0.0, 0.0, 0.0},
           {-49.0 / 60.0, 351.0 / 560.0, -359.0 / 1260.0, 367.0 / 6720.0},
           {92.0 / 7.0, -99.0 / 14.0, 176.0 / 63.0, -1.0 / 2.0},
           {485.0 / 21.0, -151.0 / 14.0, 23.0 / 9.0, -31.0 / 168.0}};
      break;
    default: break;
  }
}

// history: (q_n, F_n) becomes entry 1; q_{n+1} (in qs) becomes current
void epi_rotate(epi_state *st, double *q_new) {
  if (st->P > 0) {
    double *oq = st->hq.back(), *oF = st->hF.back();
    for (int i = st->P - 1; i > 0; --i) {
      st->hq[i] = st->hq[i - 1];
      st->hF[i] = st->hF[i - 1];
    }
    st->hq[0] = st->q;
    st->hF[0] = st->F;
    st->q = q_new;
    st->qs = oq;
    st->F = oF;
  } else {
    std::swap(st->q, st->qs);
  }
  st->nsteps++;
}

void add_stats(kiops_stats *acc, const KiopsRun &r) {
  if (!acc) return;
  acc->n_matvec += r.n_matvec;
  acc->n_substeps += r.n_substeps;
  acc->n_rejected += r.n_rejected;
  acc->m_last = r.m_last;
  acc->happy |= r.happy;
  acc->n_expm += r.n_expm;
}

static const float *prep_q32(Ctx &c, const double *q, bool fp32, int &rc) {
  rc = DFR_OK;
  if (!fp32) return nullptr;
  rc = launch_copy_to_f32(&c, c.n3, q, (float *)c.d_qf32);
  return (const float *)c.d_qf32;
}

}  // namespace dfrsw

using namespace dfrsw;

extern "C" {

int kiops_phi_apply(dfr_ctx *h, const double *q, double tau_out, int n_phi, const double *const *b, const kiops_opts *o,
                    double eps, dfr_precision prec, double *w, kiops_stats *stats) {
  if (!h || !q || !b || !o || !w || !eps_prec_ok(eps, prec)) {
    set_error("kiops_phi_apply: invalid argument (an FP32 form needs eps >= DFR_FP32_EPS_MIN)");
    return DFR_E_INVAL;
  }
  for (int k = 0; k <= n_phi && k <= MAX_P; ++k)
    if (b[k] == w || q == w) {
      set_error("kiops_phi_apply: w aliases an input");
      return DFR_E_INVAL;
    }
  Ctx &c = h->c;
  if (c.ode_kind && prec != DFR_FP64) {
    set_error("kiops_phi_apply: test problems run in FP64");
    return DFR_E_INVAL;
  }
  int rc = launch_check_state(&c, q);
  if (rc) return rc;
  const bool fp32 = prec != DFR_FP64;
  const float *q32 = prep_q32(c, q, fp32, rc);
  if (rc) return rc;
  KiopsRun r;
  rc = kiops_core(c, q, q32, tau_out, n_phi, b, *o, eps, fp32, prec == DFR_FP32_JV_BASIS32, w, r);
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    add_stats(stats, r);
  }
  return rc;
}

int epi_create(dfr_ctx *h, int order, double dt, int startup_substeps, const double *q0, double eps, dfr_precision prec,
               epi_state **out) {
  if (!h || !q0 || !out || order < 2 || order > 6 || !(dt > 0.0) || startup_substeps < 1 ||
      !eps_prec_ok(eps, prec)) {
    set_error("epi_create: invalid argument (an FP32 form needs eps >= DFR_FP32_EPS_MIN)");
    return DFR_E_INVAL;
  }
  *out = nullptr;
  if (h->c.ode_kind && prec != DFR_FP64) {
    set_error("epi_create: test problems run in FP64");
    return DFR_E_INVAL;
  }
  epi_state *st = new (std::nothrow) epi_state();
  if (!st) return DFR_E_NOMEM;
  Ctx &c = h->c;
  st->c = &c;
  st->order = order;
  epi_table(order, st->A);
  st->M = (int)st->A.size();
  st->P = order == 2 ? 0 : (int)st->A[0].size();
  st->dt = dt;
  st->s = startup_substeps;
  st->eps = eps;
  st->prec = prec;
  st->nsteps = 0;
  const size_t bytes = sizeof(double) * c.n3;
  auto alloc = [&](double **p) { return hipMalloc(p, bytes) == hipSuccess; };
  bool ok = alloc(&st->q) && alloc(&st->F) && alloc(&st->qs) && alloc(&st->w) && alloc(&st->d) && alloc(&st->jd);
  for (int i = 0; ok && i < st->P; ++i) {
    double *a, *b2, *r;
    ok = alloc(&a) && alloc(&b2) && alloc(&r);
    if (ok) {
      st->hq.push_back(a);
      st->hF.push_back(b2);
      st->R.push_back(r);
    }
  }
  for (int m = 0; ok && m < std::max(st->M, 1); ++m) {
    double *a;
    ok = alloc(&a);
    if (ok) st->bm.push_back(a);
  }
  if (!ok) {
    set_error("epi_create: out of device memory");
    epi_destroy(st);
    return DFR_E_NOMEM;
  }
  if (hipMemcpyAsync(st->q, q0, bytes, hipMemcpyDeviceToDevice, c.stream) != hipSuccess) {
    epi_destroy(st);
    set_error("epi_create: copy failed");
    return DFR_E_HIP;
  }
  *out = st;
  return DFR_OK;
}

int epi_destroy(epi_state *st) {
  if (!st) return DFR_OK;
  (void)hipStreamSynchronize(st->c->stream);
  for (double *p : {st->q, st->F, st->qs, st->w, st->d, st->jd}) (void)hipFree(p);
  for (double *p : st->hq) (void)hipFree(p);
  for (double *p : st->hF) (void)hipFree(p);
  for (double *p : st->R) (void)hipFree(p);
  for (double *p : st->bm) (void)hipFree(p);
  delete st;
  return DFR_OK;
}

int64_t epi_num_steps(const epi_state *st) { return st ? st->nsteps : -1; }

// checkpoint layout: header, then q_n, then (q_{n-i}, F_{n-i}) for the
// history entries in use, i = 1..min(nsteps, P), each 3N doubles
namespace {
struct EpiCkptHeader {
  char magic[8];          // "DFREPI01"
  int32_t order, s, prec, ne, p, nhist;
  int64_t nsteps, n;
  double dt, eps;
};
constexpr char kCkptMagic[8] = {'D', 'F', 'R', 'E', 'P', 'I', '0', '1'};
}  // namespace

int epi_save(const epi_state *st, void *buf, size_t *nbytes) {
  if (!st || !nbytes) {
    set_error("epi_save: invalid argument");
    return DFR_E_INVAL;
  }
  Ctx &c = *st->c;
  const int nh = (int)std::min<int64_t>(st->nsteps, st->P);
  const size_t vec = sizeof(double) * c.n3;
  const size_t need = sizeof(EpiCkptHeader) + vec * (1 + 2 * (size_t)nh);
  if (!buf) {
    *nbytes = need;
    return DFR_OK;
  }
  if (*nbytes < need) {
    set_error("epi_save: buffer too small");
    return DFR_E_INVAL;
  }
  EpiCkptHeader hd{};
  std::memcpy(hd.magic, kCkptMagic, 8);
  hd.order = st->order;
  hd.s = st->s;
  hd.prec = (int32_t)st->prec;
  hd.ne = c.ne;
  hd.p = c.p_deg;
  hd.nhist = nh;
  hd.nsteps = st->nsteps;
  hd.n = c.n;
  hd.dt = st->dt;
  hd.eps = st->eps;
  char *b = static_cast<char *>(buf);
  std::memcpy(b, &hd, sizeof(hd));
  b += sizeof(hd);
  DFR_HIP(hipStreamSynchronize(c.stream));
  DFR_HIP(hipMemcpy(b, st->q, vec, hipMemcpyDeviceToHost));
  b += vec;
  for (int i = 0; i < nh; ++i) {
    DFR_HIP(hipMemcpy(b, st->hq[i], vec, hipMemcpyDeviceToHost));
    b += vec;
    DFR_HIP(hipMemcpy(b, st->hF[i], vec, hipMemcpyDeviceToHost));
    b += vec;
  }
  *nbytes = need;
  return DFR_OK;
}

int epi_load(dfr_ctx *h, const void *buf, size_t nbytes, epi_state **out) {
  if (!h || !buf || !out || nbytes < sizeof(EpiCkptHeader)) {
    set_error("epi_load: invalid argument");
    return DFR_E_INVAL;
  }
  *out = nullptr;
  Ctx &c = h->c;
  EpiCkptHeader hd;
  std::memcpy(&hd, buf, sizeof(hd));
  if (std::memcmp(hd.magic, kCkptMagic, 8) != 0) {
    set_error("epi_load: not an EPI checkpoint of this version");
    return DFR_E_INVAL;
  }
  if (hd.ne != c.ne || hd.p != c.p_deg || hd.n != c.n) {
    set_error("epi_load: the checkpoint is of another grid (ne, p)");
    return DFR_E_INVAL;
  }
  const size_t vec = sizeof(double) * c.n3;
  const int P = hd.order == 2 ? 0 : hd.order - 2;
  if (hd.nhist < 0 || hd.nhist != (int)std::min<int64_t>(hd.nsteps, P) ||
      nbytes != sizeof(hd) + vec * (1 + 2 * (size_t)hd.nhist)) {
    set_error("epi_load: inconsistent checkpoint size or history");
    return DFR_E_INVAL;
  }
  const char *b = static_cast<const char *>(buf) + sizeof(hd);
  // a state with the saved parameters (q_n copied in by epi_create)
  DFR_HIP(hipMemcpyAsync(c.d_tmp, b, vec, hipMemcpyHostToDevice, c.stream));
  epi_state *st = nullptr;
  int rc = epi_create(h, hd.order, hd.dt, hd.s, c.d_tmp, hd.eps, (dfr_precision)hd.prec, &st);
  if (rc) return rc;
  b += vec;
  for (int i = 0; i < hd.nhist; ++i) {
    if (hipMemcpyAsync(st->hq[i], b, vec, hipMemcpyHostToDevice, c.stream) != hipSuccess ||
        hipMemcpyAsync(st->hF[i], b + vec, vec, hipMemcpyHostToDevice, c.stream) != hipSuccess) {
      epi_destroy(st);
      set_error("epi_load: copy failed");
      return DFR_E_HIP;
    }
    b += 2 * vec;
  }
  st->nsteps = hd.nsteps;
  if (hipStreamSynchronize(c.stream) != hipSuccess) {
    epi_destroy(st);
    set_error("epi_load: copy failed");
    return DFR_E_HIP;
  }
  *out = st;
  return DFR_OK;
}

int epi_get_state(const epi_state *st, double *q) {
  if (!st || !q) return DFR_E_INVAL;
  Ctx &c = *st->c;
  DFR_HIP(hipMemcpyAsync(q, st->q, sizeof(double) * c.n3, hipMemcpyDeviceToDevice, c.stream));
  return DFR_OK;
}

int epi_step(dfr_ctx *h, epi_state *st, const kiops_opts *o, double *q_out, kiops_stats *stats) {
  if (!h || !st || !o || st->c != &h->c) {
    set_error("epi_step: invalid argument");
    return DFR_E_INVAL;
  }
  Ctx &c = h->c;
  const int64_t n3 = c.n3;
  const bool fp32 = st->prec != DFR_FP64;
  const bool basis32 = st->prec == DFR_FP32_JV_BASIS32;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  int rc = launch_check_state(&c, st->q);
  if (rc) return rc;
  rc = launch_dfr(&c, st->q, nullptr, nullptr, nullptr, 0.0, false, false, st->F, nullptr);
  if (rc) return rc;
  double *q_new = st->qs;
  if (st->nsteps < st->P || st->order == 2) {
    // EPI2 start-up (Eq. 25) with s sub-steps, or plain EPI2
    const int s = st->order == 2 ? 1 : st->s;
    const double hstep = st->dt / s;
    DFR_HIP(hipMemcpyAsync(st->qs, st->q, sizeof(double) * n3, hipMemcpyDeviceToDevice, c.stream));
    for (int k = 0; k < s; ++k) {
      const double *Fs = st->F;
      if (k > 0) {
        rc = launch_dfr(&c, st->qs, nullptr, nullptr, nullptr, 0.0, false, false, st->d, nullptr);
        if (rc) return rc;
        Fs = st->d;
      }
      const float *q32 = prep_q32(c, st->qs, fp32, rc);
      if (rc) return rc;
      const double *bb[2] = {nullptr, Fs};
      KiopsRun r;
      rc = kiops_core(c, st->qs, q32, hstep, 1, bb, *o, st->eps, fp32, basis32, st->w, r);
      add_stats(stats, r);
      if (rc) return rc;
      rc = launch_axpby(&c, n3, 1.0, st->qs, 1.0, st->w, st->qs);
      if (rc) return rc;
    }
  } else {
    const float *q32 = prep_q32(c, st->q, fp32, rc);
    if (rc) return rc;
    for (int i = 0; i < st->P; ++i) {
      // R_i = F(q_{n-i}) - F_n - J_n (q_{n-i} - q_n)   (Eq. 33 generalised).
      // The remainder is a small difference of large terms, so its product
      // is FP64 in every precision: a complex-FP32 product here leaves
      // rounding noise in the b-vectors that the Krylov space must resolve
      // (more products per step); the FP32 forms use FP32 inside KIOPS only.
      rc = launch_axpby(&c, n3, 1.0, st->hq[i], -1.0, st->q, st->d);
      if (!rc) rc = launch_dfr(&c, st->q, nullptr, st->d, nullptr, st->eps, true, false, st->jd, nullptr);
      if (!rc) {
        LinComb lc{};
        lc.nin = 3;
        lc.nout = 1;
        lc.in[0] = st->hF[i];
        lc.in[1] = st->F;
        lc.in[2] = st->jd;
        lc.out[0] = st->R[i];
        lc.a[0][0] = 1.0;
        lc.a[0][1] = -1.0;
        lc.a[0][2] = -1.0;
        rc = launch_lincomb(&c, n3, lc);
      }
      if (rc) return rc;
    }
    // b_1 = F_n, b_m = sum_i alpha_{m,i} R_i / dt^{m-1}
    // (one pass over the remainders for all b_m, m = 2..M; M - 1 <= 3, P <= 4)
    std::vector<const double *> bb(st->M + 1, nullptr);
    bb[1] = st->F;
    if (st->M >= 2) {
      LinComb lc{};
      lc.nin = st->P;
      lc.nout = st->M - 1;
      for (int i = 0; i < st->P; ++i) lc.in[i] = st->R[i];
      for (int m = 2; m <= st->M; ++m) {
        const double sc = 1.0 / std::pow(st->dt, (double)(m - 1));
        lc.out[m - 2] = st->bm[m - 1];
        for (int i = 0; i < st->P; ++i) lc.a[m - 2][i] = st->A[m - 1][i] * sc;
        bb[m] = st->bm[m - 1];
      }
      rc = launch_lincomb(&c, n3, lc);
      if (rc) return rc;
    }
    KiopsRun r;
    rc = kiops_core(c, st->q, q32, st->dt, st->M, bb.data(), *o, st->eps, fp32, basis32, st->w, r);
    add_stats(stats, r);
    if (rc) return rc;
    rc = launch_axpby(&c, n3, 1.0, st->q, 1.0, st->w, st->qs);
    if (rc) return rc;
  }
  epi_rotate(st, q_new);
  if (q_out) DFR_HIP(hipMemcpyAsync(q_out, st->q, sizeof(double) * n3, hipMemcpyDeviceToDevice, c.stream));
  return latched_error(c);   // every earlier operation on the stream has finished
}

int epi_step_concurrent(int n, dfr_ctx *const *ctxs, epi_state *const *states, const kiops_opts *o, int n_workers,
                        kiops_stats *stats) {
  if (n < 1 || !ctxs || !states || !o) {
    set_error("epi_step_concurrent: invalid argument");
    return DFR_E_INVAL;
  }
  if (o->replay) {
    set_error("epi_step_concurrent: decision record / replay is for single-grid calls (kiops_phi_apply, epi_step)");
    return DFR_E_INVAL;
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !states[i] || states[i]->c != &ctxs[i]->c) {
      set_error("epi_step_concurrent: member " + std::to_string(i) + " has no matching context and state");
      return DFR_E_INVAL;
    }
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == ctxs[i]) {
        set_error("epi_step_concurrent: members " + std::to_string(k) + " and " + std::to_string(i) +
                  " share a context");
        return DFR_E_INVAL;
      }
    order[i] = i;
  }
  // largest members first, taken from a shared counter by the workers
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ctxs[a]->c.n > ctxs[b]->c.n; });
  const int nw = std::max(1, std::min(n_workers, n));
  std::atomic<int> next{0};
  std::atomic<int> first_rc{0};
  std::string first_msg;
  std::atomic<bool> msg_taken{false};
  auto work = [&]() {
    int dev = ctxs[order[0]]->c.device;
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n || first_rc.load() != 0) break;
      const int i = order[k];
      if (ctxs[i]->c.device != dev) dev = ctxs[i]->c.device;
      int rc = hipSetDevice(dev) == hipSuccess ? DFR_OK : DFR_E_HIP;
      if (!rc) rc = epi_step(ctxs[i], states[i], o, nullptr, stats ? &stats[i] : nullptr);
      if (rc) {
        int zero = 0;
        if (first_rc.compare_exchange_strong(zero, rc) && !msg_taken.exchange(true))
          first_msg = "member " + std::to_string(i) + ": " + dfr_last_error();
        break;
      }
    }
  };
  if (nw == 1) {
    work();
  } else {
    std::vector<std::thread> pool;
    pool.reserve(nw);
    for (int w = 0; w < nw; ++w) pool.emplace_back(work);
    for (auto &t : pool) t.join();
  }
  if (first_rc.load() != 0) {
    set_error("epi_step_concurrent: " + first_msg);
    return first_rc.load();
  }
  return DFR_OK;
}

}  // extern "C"
