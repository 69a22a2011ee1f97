"""phi-functions (Sec. 4, Eqs. 26, 31-32) -- oracle, test infrastructure only.

phi_0(z) = e^z,  phi_k(z) = int_0^1 e^{(1-s)z} s^{k-1}/(k-1)! ds  (Eq. 26),
equivalently phi_k(z) = sum_n z^n/(n+k)!  and  phi_k(z) = (phi_{k-1}(z) - 1/(k-1)!)/z.

The linear combination of Eq. (29), sum_k tau^k phi_k(tau A) b_k, is obtained
from one exponential of an augmented matrix: for
    A~ = [[A, W], [0, K]],  W = [b_p, ..., b_1],  K = upper shift (p x p),
the top block of exp(tau A~) [b_0; e_p] equals sum_k tau^k phi_k(tau A) b_k.
(Differentiate: the bottom block is y(t) = (t^{p-1}/(p-1)!, ..., t, 1), so the
top block solves x' = A x + sum_k b_k t^{k-1}/(k-1)!, x(0) = b_0, whose solution
by variation of constants is the phi-sum.)  ``phi_combination_dense`` evaluates
it with scipy's matrix exponential; it is the brute-force reference for KIOPS.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg


def phi_scalar(k: int, z: complex) -> complex:
    """phi_k(z) for a scalar: closed form via the recurrence, series near 0."""
    z = complex(z)
    if abs(z) < 0.5:
        s, term, n = 0.0 + 0.0j, 1.0 / math.factorial(k), 0
        while True:
            s_new = s + term
            if s_new == s or n > 200:
                return s_new
            s = s_new
            n += 1
            term = term * z / (n + k)
    val = np.exp(z)
    for j in range(1, k + 1):
        val = (val - 1.0 / math.factorial(j - 1)) / z
    return val


def augmented_matrix(A: np.ndarray, bs) -> np.ndarray:
    """A~ of the identity above; bs = [b_0, b_1, ..., b_p] (b_0 unused)."""
    n = A.shape[0]
    p = len(bs) - 1
    At = np.zeros((n + p, n + p))
    At[:n, :n] = A
    for k in range(p):
        At[:n, n + k] = bs[p - k]
    for k in range(p - 1):
        At[n + k, n + k + 1] = 1.0
    return At


def phi_combination_dense(A: np.ndarray, tau: float, bs) -> np.ndarray:
    """sum_{k=0}^p tau^k phi_k(tau A) b_k by one dense exponential."""
    n = A.shape[0]
    p = len(bs) - 1
    b0 = np.zeros(n) if bs[0] is None else np.asarray(bs[0], dtype=float)
    if p == 0:
        return scipy.linalg.expm(tau * A) @ b0
    At = augmented_matrix(A, bs)
    v = np.zeros(n + p)
    v[:n] = b0
    v[-1] = 1.0
    return (scipy.linalg.expm(tau * At) @ v)[:n]
