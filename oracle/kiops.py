"""KIOPS-type adaptive Krylov evaluation of phi-function combinations.

Oracle, test infrastructure only.

What is computed (Eq. 29, Sec. 4):
    w = sum_{k=0}^{p} tau_out^k phi_k(tau_out A) b_k
with A available only through products A v (for the shallow-water problem,
the complex-step J v of Eq. 28).

The paper names KIOPS -- one Krylov projection of an augmented matrix, with
incomplete orthogonalisation and adaptive sub-stepping -- and defers its
details to another publication.  This module is a from-scratch statement of
that algorithm with every constant written down; the GPU library implements
the same controller (readings K1-K7):

K1  Augmented operator A~ = [[A, W], [0, K]] on vectors of length n+p, with
    W = nu [b_p, ..., b_1] and the bottom block of the state mu y(t),
    y(t) = (t^{p-1}/(p-1)!, ..., t, 1), where nu = 2^-e, mu = 2^e and
    e = ceil(log2(max_k ||b_k||_2)) (k >= 1).  Powers of two keep the scaling
    exact.  p = 0 is run as p = 1 with b_1 = 0.
K2  Sub-stepping is exact composition x(t + tau) = top(exp(tau A~) [x(t); mu y(t)]).
K3  Arnoldi with incomplete orthogonalisation: the new vector A~ v_j is
    orthogonalised against the last `iop` basis vectors only, classical
    Gram-Schmidt (all `iop` inner products against the same vector, then one
    update).  Happy breakdown when the new norm is below `tol` (absolute).
K4  With J basis vectors built, E = exp(tau H_aug) where H_aug is the
    (J+1)x(J+1) matrix [[H_J, e_1], [0, 0]] (H_J the J x J Hessenberg block);
    the sub-step result is beta V_J E[:J, 0] and the error estimate is
    err = beta * h_{J+1,J} * |E[J-1, J]| (the corrected-scheme estimate).
K5  omega = (tau_out / tau) * err / (tol * beta0), beta0 = 2-norm of the
    augmented start vector at t = 0 (a relative tolerance).  Accept when
    omega <= delta = 1.2.
K6  Step-size / dimension update (gamma = 0.2, gamma_mmax = 0.6):
      order q = log(omega/omega_old)/log(tau/tau_old) (>= 1) after a rejected
        attempt with the same m and another tau, else q = J/4;
      rate k = (omega/omega_old)^(1/(m_old - m)) (>= 1.1) after a rejected
        attempt with the same tau and another m, else k = 2;
      tau_opt = clamp(tau (gamma/omega)^(1/q), tau/5, 5 tau) <= remaining;
      m_opt = clamp(ceil(J + log(omega/gamma)/log(k)),
                    max(m_min, floor(3m/4)), min(m_max, ceil(4m/3)));
      if J == m_max: reject -> tau_new = max(tau/5, tau (gamma_mmax/omega)^(1/q)),
                     m_new = J; accept -> tau_new = tau_opt, m_new = m;
      else:          m_new = m_opt, tau_new = tau  (<= remaining).
    A rejected attempt keeps the basis: a larger m continues the Arnoldi
    process, a smaller tau only recomputes E.
K7  The sub-step that reaches tau_out ends exactly at tau_out.

Decision replay: every attempt's decisions (the tau it ran with, the Krylov
dimension J of its exponential, accepted or not) are recorded in
KiopsStats.decisions.  Given a DecisionReplay, the attempts take its
decisions in order instead of the controller's (K5-K6): each attempt runs
with the recorded tau (which may not pass tau_out), extends the basis to the
recorded m and is accepted or rejected as recorded.  The arithmetic of an attempt is unchanged, so a
run that replays another's decisions differs from it by arithmetic alone.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

DELTA = 1.2
GAMMA = 0.2
GAMMA_MMAX = 0.6


class KiopsError(RuntimeError):
    pass


class DecisionReplay:
    """Decisions (tau, m, accept) that successive KIOPS attempts take in order,
    in place of the controller's; the calls that share one object (the KIOPS
    calls of an EPI step) continue its position."""

    def __init__(self, decisions):
        self.decisions = [(float(t), int(m), bool(a)) for t, m, a in decisions]
        self.pos = 0


@dataclass
class KiopsStats:
    n_matvec: int = 0
    n_substeps: int = 0
    n_rejected: int = 0
    m_last: int = 0
    happy: int = 0
    n_expm: int = 0
    decisions: list = field(default_factory=list)   # (tau, J, accepted)


def kiops(tau_out, matvec, bs, tol=1e-10, m_init=10, m_min=10, m_max=64, iop=2,
          max_attempts=1000, replay=None):
    """w = sum_k tau_out^k phi_k(tau_out A) b_k for bs = [b_0, ..., b_p].

    b_0 may be None (zero).  replay: None or a DecisionReplay.  Returns
    (w, KiopsStats)."""
    bs = list(bs)
    n = len(next(b for b in bs if b is not None))
    b0_absent = bs[0] is None
    b0 = np.zeros(n) if b0_absent else np.asarray(bs[0], dtype=np.float64).copy()
    if len(bs) == 1:
        bs.append(np.zeros(n))
    p = len(bs) - 1
    B = [np.zeros(n) if b is None else np.asarray(b, dtype=np.float64) for b in bs[1:]]
    nb = max(float(np.linalg.norm(b)) for b in B)
    if nb > 0.0:
        e = math.ceil(math.log2(nb))
        nu, mu = 2.0 ** (-e), 2.0 ** e
    else:
        nu, mu = 1.0, 1.0
    W = [nu * B[p - 1 - k] for k in range(p)]       # column k pairs with y_k

    m_min = min(m_min, m_max)
    m = max(m_min, min(m_init, m_max))
    V = np.zeros((m_max + 1, n + p))
    H = np.zeros((m_max + 1, m_max + 1))
    st = KiopsStats()

    x = b0
    t = 0.0
    tau = float(tau_out)
    j = 0
    beta = 0.0
    beta0 = None
    ireject = 0
    old_tau = old_m = old_omega = None
    attempts = 0
    while t < tau_out:
        attempts += 1
        if attempts > max_attempts:
            raise KiopsError("KIOPS did not converge")
        if replay is not None:
            if replay.pos >= len(replay.decisions):
                raise KiopsError(f"replay: the decisions ran out at decision {replay.pos}")
            tau, m, _ = replay.decisions[replay.pos]
            # a sub-step may not pass tau_out (K7: the controller clips tau to
            # the remaining interval; a relative 1e-12 allows for rounding)
            if not (tau > 0.0 and math.isfinite(tau)) or tau > (tau_out - t) + 1e-12 * tau_out \
                    or m < max(1, j) or m > m_max:
                raise KiopsError(f"replay: decision {replay.pos} (tau {tau}, m {m}) cannot be taken "
                                 f"at t = {t} of {tau_out} with {j} basis vectors built and m_max {m_max}")
        if j == 0:
            y = np.array([mu * t ** (p - 1 - k) / math.factorial(p - 1 - k) for k in range(p)])
            u = np.concatenate([x, y])
            beta = float(np.linalg.norm(u))
            if beta0 is None:
                beta0 = beta
            if beta == 0.0:
                break
            V[0] = u / beta
            H[:] = 0.0
        happy = False
        while j < m:
            vt, vb = V[j, :n], V[j, n:]
            if j == 0 and t == 0.0 and b0_absent:
                # first vector of the first sub-step when b_0 = 0: its top block
                # is exactly zero, and so is A times it
                Av = np.zeros(n)
            else:
                Av = matvec(vt)
                st.n_matvec += 1
            wt = Av.copy()
            for k in range(p):
                wt += W[k] * vb[k]
            wb = np.concatenate([vb[1:], [0.0]])
            w = np.concatenate([wt, wb])
            lo = max(0, j - iop + 1)
            hs = [float(np.dot(V[i], w)) for i in range(lo, j + 1)]
            for i, h in zip(range(lo, j + 1), hs):
                H[i, j] = h
                w = w - h * V[i]
            nrm = float(np.linalg.norm(w))
            if nrm < tol:
                happy = True
                j += 1
                break
            H[j + 1, j] = nrm
            V[j + 1] = w / nrm
            j += 1
        J = j
        Ha = np.zeros((J + 1, J + 1))
        Ha[:J, :J] = H[:J, :J]
        Ha[0, J] = 1.0
        E = scipy.linalg.expm(tau * Ha)
        st.n_expm += 1
        if happy:
            omega = 0.0
            accept = True
            m_new = m
            tau_new = min(tau_out - (t + tau), tau)
            st.happy = 1
        else:
            err = abs(beta * H[J, J - 1] * E[J - 1, J])
            omega = (tau_out / tau) * err / (tol * beta0)
            omega = max(omega, 1e-300)
            accept = omega <= DELTA
            if ireject >= 1 and m == old_m and tau != old_tau:
                order = max(1.0, math.log(omega / old_omega) / math.log(tau / old_tau))
            else:
                order = J / 4.0
            if ireject >= 1 and m != old_m and tau == old_tau:
                kest = max(1.1, (omega / old_omega) ** (1.0 / (old_m - m)))
            else:
                kest = 2.0
            remaining = tau_out - (t + tau) if accept else tau_out - t
            tau_opt = tau * (GAMMA / omega) ** (1.0 / order)
            tau_opt = min(remaining, max(tau / 5.0, min(5.0 * tau, tau_opt)))
            m_opt = math.ceil(J + math.log(omega / GAMMA) / math.log(kest))
            m_opt = max(m_min, min(m_max, max(math.floor(0.75 * m), min(m_opt, math.ceil(4.0 * m / 3.0)))))
            if J == m_max:
                if omega > DELTA:
                    m_new = J
                    tau_new = tau * (GAMMA_MMAX / omega) ** (1.0 / order)
                    tau_new = min(remaining, max(tau / 5.0, tau_new))
                else:
                    m_new = m
                    tau_new = tau_opt
            else:
                m_new = m_opt
                tau_new = min(remaining, tau)
        if replay is not None:
            _, m_rec, accept_rec = replay.decisions[replay.pos]
            if J != m_rec:
                raise KiopsError(f"replay: decision {replay.pos}: a happy breakdown ended the basis at "
                                 f"{J} vectors, below m = {m_rec}")
            if happy and not accept_rec:
                raise KiopsError(f"replay: decision {replay.pos}: a happy breakdown in a rejected attempt")
            accept = accept_rec
            replay.pos += 1
        st.decisions.append((tau, J, bool(accept)))
        if accept:
            x = beta * (V[:J, :n].T @ E[:J, 0])
            if tau >= tau_out - t:
                t = float(tau_out)
            else:
                t = t + tau
            st.n_substeps += 1
            st.m_last = J
            j = 0
            ireject = 0
        else:
            ireject += 1
            st.n_rejected += 1
        old_tau, old_m, old_omega = tau, m, omega
        tau, m = tau_new, m_new
        if replay is None and t < tau_out and not (tau > 0.0):
            raise KiopsError("KIOPS step size collapsed")
    return x, st
