"""The stiff ODE test problems of Sec. 5.1, plain numpy (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Each problem is the
semi-discrete system du/dt = F(u) of a PDE in second-order finite
differences, with its exact Jacobian-vector product J(u) v (Sec. 5.1 uses the
exact Jacobian).  Non-autonomous problems carry time as a last unknown so
that the EPI integrators (written for autonomous systems) apply unchanged.

Readings where the text gives no detail (the same in the GPU library):
  F1  Advection-diffusion-reaction: an N x N vertex grid on [0,1]^2 with the
      boundary (N = 40, n = 1600, h = 1/(N-1)), unknown index j*N + i with i
      along x; central differences for u_x, u_y, u_xx, u_yy; the homogeneous
      Neumann condition by reflection (u_{-1} = u_1, u_N = u_{N-2}).
  F2  Burgers: n = 1024 interior points of [0,1], h = 1/(n+1), u = 0 at both
      ends; the flux derivative (u^2/2)_x as (u_{i+1}^2 - u_{i-1}^2)/(4h).
  F3  Semilinear parabolic: n = 400 interior points, h = 1/(n+1), u = 0 at
      both ends; the integral term is the spatial integral of u, by the
      trapezoid rule (weights h on the interior points); the forcing is built
      from the discrete operators so that x(1-x) e^t solves the semi-discrete
      system exactly (the exact solution of Sec. 5.1); time is unknown n.
"""
from __future__ import annotations

import numpy as np


def _lap1(u, h, left, right):
    """(u_{i+1} - 2u_i + u_{i-1}) / h^2 with given ghost values."""
    up = np.concatenate([u[1:], [right]])
    um = np.concatenate([[left], u[:-1]])
    return (up - 2.0 * u + um) / (h * h)


# ---------------------------------------------------------------------------
# advection-diffusion-reaction (F1)

def adr(N=40, eps=1.0 / 100.0, alpha=-10.0, gamma=100.0):
    """u_t + alpha (u_x + u_y) = eps (u_xx + u_yy) + gamma u (u - 1/2)(1 - u)
    on [0,1]^2, homogeneous Neumann; u0 = 256 (x y (1-x)(1-y))^2 + 0.3."""
    h = 1.0 / (N - 1)
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x)          # X[j, i] = x_i, Y[j, i] = y_j

    def shifts(U):
        # reflected neighbours: E, W, N, S
        E = np.concatenate([U[:, 1:], U[:, -2:-1]], axis=1)
        W = np.concatenate([U[:, 1:2], U[:, :-1]], axis=1)
        Nn = np.concatenate([U[1:, :], U[-2:-1, :]], axis=0)
        S = np.concatenate([U[1:2, :], U[:-1, :]], axis=0)
        return E, W, Nn, S

    def linear(U):
        E, W, Nn, S = shifts(U)
        adv = alpha * ((E - W) / (2 * h) + (Nn - S) / (2 * h))
        dif = eps * (E + W + Nn + S - 4.0 * U) / (h * h)
        return dif - adv

    def rhs(u):
        U = u.reshape(N, N)
        return (linear(U) + gamma * U * (U - 0.5) * (1.0 - U)).reshape(-1)

    def jvp(u, v):
        U, V = u.reshape(N, N), v.reshape(N, N)
        dR = -3.0 * U * U + 3.0 * U - 0.5        # d/du of u (u - 1/2)(1 - u)
        return (linear(V) + gamma * dR * V).reshape(-1)

    u0 = (256.0 * (X * Y * (1 - X) * (1 - Y)) ** 2 + 0.3).reshape(-1)
    return rhs, jvp, u0


# ---------------------------------------------------------------------------
# Burgers (F2)

def burgers(n=1024, eps=1e-3, mu=0.3, sigma=0.05):
    """u_t + (u^2/2)_x = eps u_xx on [0,1], u = 0 at both ends;
    u0 = exp(-(x - mu)^2 / (2 sigma^2))."""
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h

    def rhs(u):
        u2 = u * u
        up = np.concatenate([u2[1:], [0.0]])
        um = np.concatenate([[0.0], u2[:-1]])
        return -(up - um) / (4.0 * h) + eps * _lap1(u, h, 0.0, 0.0)

    def jvp(u, v):
        uv = u * v
        up = np.concatenate([uv[1:], [0.0]])
        um = np.concatenate([[0.0], uv[:-1]])
        return -(up - um) / (2.0 * h) + eps * _lap1(v, h, 0.0, 0.0)

    u0 = np.exp(-((x - mu) ** 2) / (2.0 * sigma ** 2))
    return rhs, jvp, u0


# ---------------------------------------------------------------------------
# semilinear parabolic (F3)

def semilinear(n=400):
    """u_t - u_xx = int_0^1 u dx + phi(x, t) on [0,1], u = 0 at both ends,
    exact solution u = x(1-x) e^t; unknowns (u_1..u_n, t)."""
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    s = x * (1.0 - x)
    # phi = e^t (s - s_xx - int s), with the discrete s_xx (= -2 exactly for a
    # quadratic, boundary values 0) and the discrete integral
    src = s + 2.0 - h * np.sum(s)

    def rhs(q):
        u, t = q[:-1], q[-1]
        return np.concatenate([_lap1(u, h, 0.0, 0.0) + h * np.sum(u) + np.exp(t) * src, [1.0]])

    def jvp(q, v):
        w, vt = v[:-1], v[-1]
        return np.concatenate([_lap1(w, h, 0.0, 0.0) + h * np.sum(w) + vt * np.exp(q[-1]) * src, [0.0]])

    def exact(t):
        return np.concatenate([s * np.exp(t), [t]])

    return rhs, jvp, exact(0.0), exact


PROBLEMS = {"adr": adr, "burgers": burgers, "semilinear": semilinear}
