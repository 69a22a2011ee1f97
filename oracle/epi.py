"""Multistep exponential propagation iterative (EPI) integrators -- oracle,
test infrastructure only.

Sec. 4 of the paper:
  EPI2 (exponential Euler), Eq. (25):  q_{n+1} = q_n + phi_1(dt J_n) dt F(q_n).
  Multistep ansatz, Eqs. (34)-(35):
      q_{n+1} = q_n + phi_1(dt J_n) dt F_n + sum_{m=1}^{M} phi_m(dt J_n) v_m,
      v_m = sum_{i=1}^{P} alpha_{m,i} dt R(q_{n-i}),
      R(q) = F(q) - F_n - J_n (q - q_n)                       (Eq. 22, 33),
  coefficient matrices A_3 (Eq. 30), A_4, A_5, A_6 (Eqs. 36-38), with
  alpha_{m,i} = A[m-1][i-1].
  One phi-combination per step (Eq. 29):  with tau = dt,
      b_1 = F_n,  b_m = sum_i alpha_{m,i} R_i / dt^{m-1}  (m >= 2),
  so that sum_m tau^m phi_m(tau J) b_m reproduces the ansatz.
  The first P steps use EPI2 with `startup_substeps` equal sub-steps (the paper
  says only "a smaller time step"); only the coarse-step states and their
  right-hand sides enter the history.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np

from .kiops import kiops

# Eq. (30): EPI3;  Eqs. (36)-(38): EPI4, EPI5, EPI6.  Rows m = 1..M, columns i = 1..P.
COEFFS = {
    2: [],
    3: [[Fr(0)], [Fr(2, 3)]],
    4: [[Fr(0), Fr(0)],
        [Fr(-3, 10), Fr(3, 40)],
        [Fr(32, 5), Fr(-11, 10)]],
    5: [[Fr(0), Fr(0), Fr(0)],
        [Fr(-4, 5), Fr(2, 5), Fr(-4, 45)],
        [Fr(12), Fr(-9, 2), Fr(8, 9)],
        [Fr(3), Fr(0), Fr(-1, 3)]],
    6: [[Fr(0), Fr(0), Fr(0), Fr(0)],
        [Fr(-49, 60), Fr(351, 560), Fr(-359, 1260), Fr(367, 6720)],
        [Fr(92, 7), Fr(-99, 14), Fr(176, 63), Fr(-1, 2)],
        [Fr(485, 21), Fr(-151, 14), Fr(23, 9), Fr(-31, 168)]],
}


def n_previous(order: int) -> int:
    """P, the number of previous steps the method uses."""
    return 0 if order == 2 else len(COEFFS[order][0])


class EPI:
    """EPI integrator over a right-hand side F and a Jacobian-vector product.

    rhs(q) -> F(q);  jvp(q, v) -> J(q) v."""

    def __init__(self, rhs, jvp, order, dt, q0, startup_substeps=10, kiops_opts=None):
        if order not in COEFFS:
            raise ValueError("order must be 2..6")
        self.rhs, self.jvp = rhs, jvp
        self.order = order
        self.P = n_previous(order)
        self.dt = float(dt)
        self.s = int(startup_substeps)
        self.kopts = dict(kiops_opts or {})
        self.q = np.array(q0, dtype=np.float64)
        self.n = 0
        self.hist_q = []      # q_{n-1}, q_{n-2}, ... (most recent first)
        self.hist_F = []
        self.stats = []

    def _phi(self, q, tau, bs):
        w, st = kiops(tau, lambda v: self.jvp(q, v), bs, **self.kopts)
        self.stats.append(st)
        return w

    def step(self):
        q = self.q
        Fn = self.rhs(q)
        if self.n < self.P or self.order == 2:
            # EPI2 start-up (Eq. 25) with s sub-steps of dt/s, or plain EPI2
            s = self.s if self.order != 2 else 1
            h = self.dt / s
            qs, Fs = q, Fn
            for k in range(s):
                if k > 0:
                    Fs = self.rhs(qs)
                w = self._phi(qs, h, [None, Fs])
                qs = qs + w
            q_new = qs
        else:
            A = COEFFS[self.order]
            M = len(A)
            R = []
            for i in range(1, self.P + 1):
                qi, Fi = self.hist_q[i - 1], self.hist_F[i - 1]
                R.append(Fi - Fn - self.jvp(q, qi - q))
            bs = [None, Fn]
            for m in range(2, M + 1):
                bm = np.zeros_like(q)
                for i in range(1, self.P + 1):
                    a = A[m - 1][i - 1]
                    if a != 0:
                        bm = bm + float(a) * R[i - 1]
                bs.append(bm / self.dt ** (m - 1))
            w = self._phi(q, self.dt, bs)
            q_new = q + w
        self.hist_q.insert(0, q)
        self.hist_F.insert(0, Fn)
        del self.hist_q[max(self.P, 1):]
        del self.hist_F[max(self.P, 1):]
        self.q = q_new
        self.n += 1
        return q_new
