// Device-controlled rounds of the batched KIOPS evaluation (Sec. 4, Eq. 29).
// The per-member controller of kiops.hip (begin an attempt, the arguments of
// an Arnoldi step, the decision after a small exponential: the steps K4-K7
// of the adaptive Krylov method) runs in a planner kernel, one thread per
// member.  The planner writes the round's call tables and their counts into
// device memory, and the round's launches read them there.  A round is thus
// a fixed sequence of launches whose grids are sized for every member active:
// it is captured once in a HIP graph and replayed until every member's
// evaluation has ended, with no host decision in between.
//
// Round: plan -> combination of the sub-steps the plan accepted and start
// vectors of the sub-steps it began (one launch) -> [first round of a call:
// first Arnoldi steps of a zero top block] -> Krylov-form products (one
// launch per number of GL points) -> Gram-Schmidt updates -> small
// exponentials.  A member whose sweep
// reaches its exponential in one round is decided by the next round's plan,
// so no member waits a round for a read-back.  Each member's sequence of
// operations, and with it its result, is the host-controlled one: members
// share no buffers, only launches.
#include "dfrsw_internal.h"

#include <cmath>

namespace dfrsw {

// The decision after an exponential (K4-K7): error ratio omega of the
// sub-step, acceptance, the next sub-step length and Krylov dimension.  The
// same arithmetic as the host controller's, in the same order.
__device__ int kc_decide(KCtl &k, const DevMember &d, const KHost &r, bool &accept) {
  const double DELTA = 1.2, GAMMA = 0.2, GAMMA_MMAX = 0.6;
  k.n_expm++;
  const int J = r.J;
  k.n_matvec += (J - k.j_sweep) - (k.skipped ? 1 : 0);
  if (k.beta0 < 0.0) k.beta0 = r.beta;
  if (!isfinite(r.err) || !isfinite(r.beta)) return DFR_E_NONFINITE;
  const double tau = k.tau, tau_out = d.tau_out, t = k.t;
  const int m = k.m;
  double omega, tau_new;
  int m_new;
  if (r.happy) {
    k.j = J;
    omega = 0.0;
    accept = true;
    m_new = m;
    tau_new = fmin(tau_out - (t + tau), tau);
    k.happy = 1;
  } else {
    omega = (tau_out / tau) * r.err / (d.tol * k.beta0);
    omega = fmax(omega, 1e-300);
    accept = omega <= DELTA;
    double order;
    if (k.ireject >= 1 && m == k.old_m && tau != k.old_tau)
      order = fmax(1.0, log(omega / k.old_omega) / log(tau / k.old_tau));
    else
      order = J / 4.0;
    double kest;
    if (k.ireject >= 1 && m != k.old_m && tau == k.old_tau)
      kest = fmax(1.1, pow(omega / k.old_omega, 1.0 / (k.old_m - m)));
    else
      kest = 2.0;
    const double remaining = accept ? tau_out - (t + tau) : tau_out - t;
    double tau_opt = tau * pow(GAMMA / omega, 1.0 / order);
    tau_opt = fmin(remaining, fmax(tau / 5.0, fmin(5.0 * tau, tau_opt)));
    int m_opt = (int)ceil(J + log(omega / GAMMA) / log(kest));
    m_opt = max(d.m_min, min(d.m_max, max((int)floor(0.75 * m), min(m_opt, (int)ceil(4.0 * m / 3.0)))));
    if (J == d.m_max) {
      if (omega > DELTA) {
        m_new = J;
        tau_new = tau * pow(GAMMA_MMAX / omega, 1.0 / order);
        tau_new = fmin(remaining, fmax(tau / 5.0, tau_new));
      } else {
        m_new = m;
        tau_new = tau_opt;
      }
    } else {
      m_new = m_opt;
      tau_new = fmin(remaining, tau);
    }
  }
  if (accept) {
    if (tau >= tau_out - t) k.t = tau_out;
    else k.t = t + tau;
    k.n_substeps++;
    k.m_last = J;
    k.j = 0;
    k.ireject = 0;
  } else {
    k.ireject++;
    k.n_rejected++;
  }
  k.old_tau = tau;
  k.old_m = m;
  k.old_omega = omega;
  k.tau = tau_new;
  k.m = m_new;
  k.phase = k.t < tau_out ? KC_BEGIN : KC_DONE;
  if (k.t < tau_out && !(k.tau > 0.0)) return DFR_E_KIOPS;
  return DFR_OK;
}

// The start of an attempt: a sweep begun (its start vector needs the bottom
// entries mu t^(p-1-i) / (p-1-i)! of Eq. 29's augmented vector) or continued.
// (Loops over the bottom entries run to MAX_P with a predicate, so that the
// state stays in registers.)
__device__ int kc_begin(KCtl &k, const DevMember &d, bool &need_start) {
  if (++k.attempts > d.max_attempts) return DFR_E_KIOPS;
  k.j_sweep = k.j;
  k.skipped = 0;
  need_start = (k.j == 0);
  if (need_start) {
#pragma unroll
    for (int i = 0; i < MAX_P; ++i) {
      if (i < d.p) {
        const int pw = d.p - 1 - i;
        double f = 1.0;
        for (int r = 2; r <= pw; ++r) f *= r;
        k.ybot[i] = d.mu * pow(k.t, (double)pw) / f;
      }
    }
  }
  k.phase = k.j < k.m ? KC_SWEEP : KC_EXPM;
  return DFR_OK;
}

__device__ __forceinline__ void *kc_slot(const DevMember &d, int j) {
  return d.V + (size_t)j * (size_t)d.n3 * (size_t)d.esz;
}

// counters of a round, per member: calls and blocks of each launch
enum {
  CN_PRE = 0, CN_FIRST = 2, CN_EXPM = 4,
  CN_DFR = 5,                          // CN_DFR + 2 (ns - 2): the products by number of GL points
  CN_UPD = CN_DFR + 2 * (MAX_NS - 1),  // CN_UPD + 2 (ns - 2): the updates, grouped the same way
  CN_N = CN_UPD + 2 * (MAX_NS - 1)
};
constexpr int PLAN_THREADS = 256;

__global__ __launch_bounds__(PLAN_THREADS) void plan_round_kernel(const DevRound r) {
  __shared__ int scan[CN_N][PLAN_THREADS];
  __shared__ int s_need;
  const int m = threadIdx.x;
  const bool mine = m < r.nmem;
  const int round = r.cnt->round + 1;
  for (int c = 0; c < CN_N; ++c) scan[c][m] = 0;
  if (m == 0) s_need = 0;
  bool do_comb = false, do_start = false, do_first = false, do_prod = false, do_upd = false, do_expm = false;
  KCtl k{};
  DevMember d{};
  int jcur = 0;
  if (mine) {
    // every load of the member up front, in one round trip (the result of
    // an exponential is read whether or not the member waits for one)
    k = r.ctl[m];
    d = r.mem[m];
    const KHost kh = r.kh[m];
    int rc = DFR_OK;
    if (k.phase == KC_WAIT) {   // last round's exponential: decide
      bool accept = false;
      rc = kc_decide(k, d, kh, accept);
      do_comb = (rc == DFR_OK) && accept;
    }
    bool need_start = false;
    if (!rc && k.phase == KC_BEGIN) {
      rc = kc_begin(k, d, need_start);
      do_start = !rc && need_start;
      if (do_start) k.npB = d.nblk_vec;
    }
    if (!rc && k.phase == KC_SWEEP) {
      jcur = k.j;
      // top block zero (w = W b_0, no product): only at the first step of a
      // call, in its first round (a rejected attempt keeps its sweep)
      do_first = (k.j == 0 && k.t == 0.0 && d.b0_absent);
      do_prod = !do_first;
      if (do_first) k.skipped = 1;   // not a product: not counted
      do_upd = true;
      if (do_first && round != 1) rc = KC_E_FIRST_LATE;
    }
    if (rc) {
      k.phase = KC_FAILED;
      k.err = rc;
      do_comb = do_start = do_first = do_prod = do_upd = false;
    }
    if (do_comb || do_start) {
      scan[CN_PRE][m] = 1;
      scan[CN_PRE + 1][m] = d.nblk_vec;
    }
    if (do_first) {
      scan[CN_FIRST][m] = 1;
      scan[CN_FIRST + 1][m] = d.nblk_vec;
    }
    if (do_upd) {
      scan[CN_UPD + 2 * (d.ns - 2)][m] = 1;
      scan[CN_UPD + 2 * (d.ns - 2) + 1][m] = d.nblk_upd;
    }
    if (do_prod) {
      scan[CN_DFR + 2 * (d.ns - 2)][m] = 1;
      scan[CN_DFR + 2 * (d.ns - 2) + 1][m] = d.ntiles;
    }
    // after this round's Arnoldi step (if any): the exponential, when the
    // sweep reaches m
    do_expm = (k.phase == KC_SWEEP && jcur + 1 >= k.m) || k.phase == KC_EXPM;
    if (do_expm) scan[CN_EXPM][m] = 1;
  }
  __syncthreads();
  // inclusive scans of every counter over the members, in place
  // (Hillis-Steele, in member order: the tables are ordered by member)
  for (int off = 1; off < PLAN_THREADS; off <<= 1) {
    int add[CN_N];
#pragma unroll
    for (int c = 0; c < CN_N; ++c) add[c] = m >= off ? scan[c][m - off] : 0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CN_N; ++c) scan[c][m] += add[c];
    __syncthreads();
  }
  if (mine) {
    // this member's offsets: the inclusive scan of the member before it
    auto ex = [&](int c) { return m > 0 ? scan[c][m - 1] : 0; };
    if (do_comb || do_start) {
      PreCall b{};
      b.b0 = ex(CN_PRE + 1);
      b.nblk = d.nblk_vec;
      b.n3 = d.n3;
      b.comb = do_comb;
      b.start = do_start;
      b.V = d.V;
      b.kd = d.kd;
      b.x = d.w;
      b.pout = d.pB;
      r.pre[ex(CN_PRE)] = b;
    }
    if (do_upd) {   // an Arnoldi step on basis vector jcur
      ArnoldiArgs ar{};
      ar.on = 1;
      ar.j = jcur;
      ar.p = d.p;
      ar.start = (jcur == 0);
#pragma unroll
      for (int i = 0; i < MAX_P; ++i) {
        if (i < d.p) {
          ar.W[i] = d.wil ? d.W : d.W + (size_t)i * (size_t)d.n3;
          ar.ybot[i] = k.ybot[i];
        }
      }
      ar.wil = d.wil;
      ar.vprev = (jcur >= 1 && d.iop >= 2) ? kc_slot(d, jcur - 1) : nullptr;
      ar.pin = d.pB;
      ar.np_in = k.npB;
      ar.pout = d.pA;
      ar.kd = d.kd;
      ar.tol = d.tol;
      if (do_first) {
        FirstCall f{};
        f.b0 = ex(CN_FIRST + 1);
        f.nblk = d.nblk_vec;
        f.n3 = d.n3;
        f.ar = ar;
        f.out = kc_slot(d, jcur + 1);
        r.first[ex(CN_FIRST)] = f;
        k.npA = d.nblk_vec;
      } else {
        const int g = CN_DFR + 2 * (d.ns - 2);
        DfrCall c{};
        c.g = d.g;
        c.ops = d.ops;
        c.g_ne = d.g_ne;
        c.TX = d.TX;
        c.TY = d.TY;
        c.b0 = ex(g + 1);
        c.ntiles = d.ntiles;
        c.q = d.q;
        c.v = kc_slot(d, jcur);
        c.vscale = nullptr;
        c.eps = d.eps;
        c.out = kc_slot(d, jcur + 1);
        c.ar = ar;
        r.dfr[r.grp_base[d.ns] + ex(g)] = c;
        k.npA = d.ntiles;
      }
      const int gu = CN_UPD + 2 * (d.ns - 2);
      UpdateCall u{};
      u.b0 = ex(gu + 1);
      u.nblk = d.nblk_upd;
      u.n3 = d.n3;
      u.j = jcur;
      u.p = d.p;
      u.w = kc_slot(d, jcur + 1);
      u.vj = kc_slot(d, jcur);
      u.vprev = ar.vprev;
      u.pin = d.pA;
      u.np_in = k.npA;
      u.pout = d.pB;
      u.kd = d.kd;
      r.upd[r.grp_base[d.ns] + ex(gu)] = u;
      k.npB = d.nblk_upd;
      if (++k.j >= k.m) k.phase = KC_EXPM;
    }
    if (do_expm) {
      ExpmCall x{};
      x.kd = d.kd;
      x.tau = k.tau;
      x.res = r.kh + m;
      x.jfin = k.j;
      x.pin = d.pB;
      x.np_in = k.npB;
      x.tol = d.tol;
      r.expm[ex(CN_EXPM)] = x;
      k.phase = KC_WAIT;
    }
    // rounds this member certainly still needs after this one: the rest of
    // its sweep, then the round that decides its exponential
    int need = 0;
    if (k.phase == KC_WAIT) need = 1;
    else if (k.phase == KC_SWEEP) need = k.m - k.j + 1;
    if (need) atomicMax(&s_need, need);
    r.ctl[m] = k;
  }
  __syncthreads();
  if (m == 0) {
    DevCounts *c = r.cnt;
    const int last = PLAN_THREADS - 1;   // inclusive totals (members beyond nmem count 0)
    c->n_pre = scan[CN_PRE][last];
    c->nb_pre = scan[CN_PRE + 1][last];
    c->n_first = scan[CN_FIRST][last];
    c->nb_first = scan[CN_FIRST + 1][last];
    c->n_expm = scan[CN_EXPM][last];
    c->dfr[0][0] = c->dfr[0][1] = c->dfr[1][0] = c->dfr[1][1] = 0;
    c->upd[0][0] = c->upd[0][1] = c->upd[1][0] = c->upd[1][1] = 0;
    for (int ns = 2; ns <= MAX_NS; ++ns) {
      c->dfr[ns][0] = scan[CN_DFR + 2 * (ns - 2)][last];
      c->dfr[ns][1] = scan[CN_DFR + 2 * (ns - 2) + 1][last];
      c->upd[ns][0] = scan[CN_UPD + 2 * (ns - 2)][last];
      c->upd[ns][1] = scan[CN_UPD + 2 * (ns - 2) + 1][last];
    }
    c->round = round;
    bool work = c->n_pre || c->n_first || c->n_expm;
    for (int ns = 2; ns <= MAX_NS; ++ns) work = work || c->upd[ns][0];
    if (work) c->last_work = round;
    // the progress word to the host: one 64-bit system-scope store.  The
    // host reads nothing else the planner writes, so no fence orders it
    // after the tables.
    __hip_atomic_store(r.progress, dev_progress(round, s_need), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

int launch_dev_round(hipStream_t s, const DevRound &r, bool first, KTimer *tm, const DevBranches *br) {
  if (r.nmem < 1 || r.nmem > PLAN_THREADS) {
    set_error("device-controlled rounds: 1 to 256 members");
    return DFR_E_INVAL;
  }
  timed_launch(tm, DFR_K_OTHER, 0.0, s, plan_round_kernel, dim3(1), dim3(PLAN_THREADS), 0, r);
  DFR_HIP(hipGetLastError());
  const bool f32 = r.fp32 != 0, b32 = r.basis32 != 0;
  int rc = launch_krylov_dev(s, KD_PRE, b32, r.pre, &r.cnt->n_pre, r.grid_vec, r.pmax, tm);
  if (!rc && first) rc = launch_krylov_dev(s, KD_FIRST, b32, r.first, &r.cnt->n_first, r.grid_vec, r.pmax, tm);
  if (rc) return rc;
  // each group: its products, then its updates (on a branch of its own)
  bool forked = false;
  for (int ns = 2; ns <= MAX_NS && !rc; ++ns) {
    if (!r.grp_n[ns]) continue;
    hipStream_t gs = s;
    if (br && forked) {
      gs = br->side[ns];
      DFR_HIP(hipStreamWaitEvent(gs, br->fork, 0));
    } else if (br) {
      DFR_HIP(hipEventRecord(br->fork, s));
      forked = true;
    }
    const int grid = ((r.grp_maxlog[ns] + 7) / 8) * 8;
    rc = launch_dfr_batch_dev(gs, ns, f32, b32, r.dfr + r.grp_base[ns], &r.cnt->dfr[ns][0], grid,
                              r.grp_threads[ns], r.grp_lds[ns], tm);
    if (!rc) rc = launch_krylov_dev(gs, KD_UPDATE, b32, r.upd + r.grp_base[ns], &r.cnt->upd[ns][0],
                                    r.grp_maxupd[ns], r.pmax, tm);
    if (!rc && gs != s) DFR_HIP(hipEventRecord(br->join[ns], gs));
  }
  if (rc) return rc;
  if (br) {
    bool main_branch = true;
    for (int ns = 2; ns <= MAX_NS; ++ns) {
      if (!r.grp_n[ns]) continue;
      if (!main_branch) DFR_HIP(hipStreamWaitEvent(s, br->join[ns], 0));
      main_branch = false;
    }
  }
  return launch_expm_dev(s, r.expm, &r.cnt->n_expm, r.nmem, r.expm_lds, tm);
}

}  // namespace dfrsw
