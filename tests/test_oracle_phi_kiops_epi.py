"""Pins of the oracle's phi-functions, KIOPS and EPI integrators (Sec. 4,
Eqs. 25-38; Sec. 5.1)."""
import math
from dataclasses import replace
from fractions import Fraction as Fr

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

import oracle
from oracle import epi, kiops, ode, phi
from paper_2101_05617_amd import inputs


# ----------------------------------------------------------------- phi

@pytest.mark.parametrize("k", range(0, 6))
def test_phi_scalar_matches_integral_definition(k):
    # Eq. (26) by adaptive quadrature, against the closed form / series
    for z in (-3.0, -0.3, 1e-4, 0.7, 2.0, -1.0 + 2.0j):
        if k == 0:
            ref = np.exp(z)
        else:
            f = lambda s, part: (np.exp((1 - s) * z) * s ** (k - 1) / math.factorial(k - 1)).__getattribute__(part)
            ref = scipy.integrate.quad(f, 0, 1, args=("real",), epsabs=1e-15, epsrel=1e-14)[0] \
                + 1j * scipy.integrate.quad(f, 0, 1, args=("imag",), epsabs=1e-15, epsrel=1e-14)[0]
        assert abs(phi.phi_scalar(k, z) - ref) < 1e-13 * max(1.0, abs(ref))
    assert abs(phi.phi_scalar(k, 0.0) - 1.0 / math.factorial(k)) < 1e-16


def test_augmented_identity_against_eigendecomposition():
    # sum_k tau^k phi_k(tau A) b_k via the augmented exponential equals the
    # same sum built from scalar phi-functions on the eigenvalues of A
    rng = np.random.default_rng(0)
    n, p, tau = 12, 4, 0.7
    A = rng.standard_normal((n, n)) / 2
    bs = [rng.standard_normal(n) for _ in range(p + 1)]
    lam, S = np.linalg.eig(A)
    Si = np.linalg.inv(S)
    ref = np.zeros(n, dtype=complex)
    for k in range(p + 1):
        fk = np.array([phi.phi_scalar(k, tau * l) for l in lam])
        ref += tau ** k * (S @ (fk * (Si @ bs[k])))
    got = phi.phi_combination_dense(A, tau, bs)
    assert np.allclose(got, ref.real, atol=1e-12) and np.abs(ref.imag).max() < 1e-10


# ----------------------------------------------------------------- KIOPS

def _stiff_matrix(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = -np.logspace(-2, 3, n)
    A = Q @ np.diag(d) @ Q.T + 0.3 * (rng.standard_normal((n, n)) - rng.standard_normal((n, n)).T) / np.sqrt(n)
    return A


@pytest.mark.parametrize("p", [0, 1, 3, 5])
def test_kiops_matches_dense_exponential(p):
    n, tau = 80, 0.37
    A = _stiff_matrix(n, p)
    rng = np.random.default_rng(10 + p)
    bs = [rng.standard_normal(n) for _ in range(p + 1)]
    ref = phi.phi_combination_dense(A, tau, bs)
    for tol in (1e-8, 1e-12):
        w, st = kiops.kiops(tau, lambda v: A @ v, bs, tol=tol, m_init=10, m_max=40)
        assert np.linalg.norm(w - ref) <= 50 * tol * np.linalg.norm(ref)
        assert st.n_substeps >= 1


def test_kiops_zero_b0_and_substepping():
    n, tau = 60, 2.0
    A = _stiff_matrix(n, 7) * 5
    rng = np.random.default_rng(3)
    bs = [None] + [rng.standard_normal(n) for _ in range(3)]
    ref = phi.phi_combination_dense(A, tau, [np.zeros(n)] + bs[1:])
    w, st = kiops.kiops(tau, lambda v: A @ v, bs, tol=1e-10, m_init=10, m_max=16)
    assert st.n_substeps > 1        # a small Krylov space forces sub-steps
    assert np.linalg.norm(w - ref) <= 1e-8 * np.linalg.norm(ref)


def test_kiops_full_vs_incomplete_orthogonalisation():
    n, tau = 70, 0.5
    A = _stiff_matrix(n, 4)
    rng = np.random.default_rng(5)
    bs = [rng.standard_normal(n) for _ in range(3)]
    w2, _ = kiops.kiops(tau, lambda v: A @ v, bs, tol=1e-11, iop=2, m_max=40)
    wf, _ = kiops.kiops(tau, lambda v: A @ v, bs, tol=1e-11, iop=40, m_max=40)
    assert np.linalg.norm(w2 - wf) <= 1e-8 * np.linalg.norm(wf)


def test_kiops_happy_breakdown():
    # b in a 3-dimensional invariant subspace of a diagonal matrix: exact after
    # 3 Arnoldi steps, closed form exp(tau d) b
    d = -np.arange(1.0, 21.0)
    b = np.zeros(20)
    b[[2, 7, 11]] = [1.0, -2.0, 0.5]
    w, st = kiops.kiops(0.3, lambda v: d * v, [b], tol=1e-12, m_max=20)
    assert st.happy == 1
    assert np.allclose(w, np.exp(0.3 * d) * b, atol=1e-13)


def test_kiops_on_shallow_water_jacobian_tiny_grid():
    # KIOPS with complex-step products against a dense exponential of the
    # column-wise complex-step Jacobian (ne = 1, p = 2)
    w = replace(inputs.WORKLOADS["c0_ne4_p4"], ne=1, p=2, h_lmax=2)
    G = oracle.OracleGrid(w.ne, w.ns, *w.constants())
    P, B1, B2 = G.node_frames()
    Q, _ = inputs.initial_state(w, P, B1, B2)
    n = 3 * G.N
    J = np.stack([G.jvp(Q, e) for e in np.eye(n)], axis=1)
    F = G.rhs(Q)
    rng = np.random.default_rng(2)
    bs = [None, F, 1e-3 * rng.standard_normal(n), 1e-4 * rng.standard_normal(n)]
    tau = w.dt_nd * 4
    ref = phi.phi_combination_dense(J, tau, [np.zeros(n)] + bs[1:])
    got, st = kiops.kiops(tau, lambda v: G.jvp(Q, v), bs, tol=1e-12, m_max=32)
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


# ----------------------------------------------------------------- EPI

def _order_conditions(A, order):
    """Non-stiff order conditions of the multistep ansatz (Eqs. 24, 26, 34-35):
    expanding R(q(t_n + theta dt)) = sum_{k>=2} c_k theta^k dt^k and phi_m as
    sum_j z^j/(m+j)!, accuracy through dt^order requires, for k >= 2, j >= 0,
    k + j <= order - 1:  sum_m S_{m,k}/(m+j)! = k!/(k+1+j)!,
    with S_{m,k} = sum_i alpha_{m,i} (-i)^k."""
    M, P = len(A), len(A[0])
    bad = []
    for k in range(2, order):
        for j in range(0, order - k):
            lhs = sum(sum(A[m - 1][i - 1] * Fr(-i) ** k for i in range(1, P + 1)) / math.factorial(m + j)
                      for m in range(1, M + 1))
            rhs = Fr(math.factorial(k), math.factorial(k + 1 + j))
            if lhs != rhs:
                bad.append((k, j, lhs, rhs))
    return bad


@pytest.mark.parametrize("order", [3, 4, 5, 6])
def test_epi_coefficients_satisfy_order_conditions(order):
    # exact rational arithmetic on the tables of Eqs. (30), (36)-(38)
    assert _order_conditions(epi.COEFFS[order], order) == []


def test_order_conditions_detect_a_wrong_digit():
    A = [row[:] for row in epi.COEFFS[6]]
    A[3][3] = Fr(-31, 169)
    assert _order_conditions(A, 6) != []


def test_epi_is_exact_for_affine_problems():
    # R = 0 for affine F, so every EPI step is the exact propagator
    n = 40
    A = _stiff_matrix(n, 9)
    c = np.random.default_rng(1).standard_normal(n)
    rhs = lambda q: A @ q + c
    jvp = lambda q, v: A @ v
    q0 = np.random.default_rng(2).standard_normal(n)
    dt = 0.05
    for order in (2, 4, 6):
        E = epi.EPI(rhs, jvp, order, dt, q0, startup_substeps=3, kiops_opts=dict(tol=1e-13, m_max=40))
        for _ in range(6):
            E.step()
        # exact: q(t) = e^{tA} q0 + t phi_1(tA) c
        ref = phi.phi_combination_dense(A, 6 * dt, [q0, c])
        assert np.linalg.norm(E.q - ref) < 1e-10 * np.linalg.norm(ref)


def _semilinear(n=400):
    """Sec. 5.1 semilinear parabolic problem (oracle/ode.py), u = x(1-x) e^t
    exact, with time appended as a last unknown."""
    rhs, jvp, _, exact = ode.semilinear(n)
    return rhs, jvp, exact


@pytest.mark.parametrize("order", [2, 3, 4, 5, 6])
def test_epi_observed_order_semilinear_parabolic(order):
    # Sec. 5.1 / Fig. 1: the observed order equals the design order (no order
    # reduction), with exact starting values and KIOPS tolerance 1e-14
    rhs, jvp, exact = _semilinear()
    errs = []
    for nst in (5, 10, 20):
        dt = 1.0 / nst
        E = epi.EPI(rhs, jvp, order, dt, exact(0.0), kiops_opts=dict(tol=1e-14, m_max=64))
        if E.P:
            E.hist_q = [exact(-i * dt) for i in range(1, E.P + 1)]
            E.hist_F = [rhs(exact(-i * dt)) for i in range(1, E.P + 1)]
            E.n = E.P
        for _ in range(nst):
            E.step()
        errs.append(np.linalg.norm(E.q[:-1] - exact(1.0)[:-1]))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - order) < 0.25), slopes


def test_shallow_water_epi_conserves_mass():
    w = inputs.WORKLOADS["c0_ne4_p4"]
    G = oracle.OracleGrid(w.ne, w.ns, *w.constants())
    P, B1, B2 = G.node_frames()
    Q, _ = inputs.initial_state(w, P, B1, B2)
    wq = G.mass_weights()
    m0 = wq @ Q[: G.N]
    E = epi.EPI(G.rhs, lambda q, v: G.jvp(q, v, w.eps), w.order, w.dt_nd, Q, startup_substeps=2,
                kiops_opts=dict(tol=w.tol, m_max=w.m_max))
    for _ in range(3):
        E.step()
        assert abs(wq @ E.q[: G.N] - m0) / m0 < 1e-14


def test_epi_observed_order_shallow_water_c0():
    # Sec. 4 methods on the shallow-water problem itself (ne = 4, p = 4; the
    # zonal flow with a 5% height perturbation, 4 h): exact starting values
    # from an independent reference (DOP853, rtol 1e-13, about 2e-13 from
    # itself at rtol 1e-12), then EPI4/5/6 at dt = 1800, 900, 450 s.  The
    # slopes approach the design orders from below (measured 3.68/3.85,
    # 4.57/4.89, 5.22/5.35): these dt are not yet asymptotic, and dt cannot
    # shrink much further, since the errors then meet the floor set by the
    # rounding of F, a small residual of the fluxes of a near-balanced state
    # (about 4e-12 here).  Asserted: each slope >= order - 1, and at every
    # dt the higher order is the more accurate.
    import scipy.integrate
    w = replace(inputs.WORKLOADS["c0_ne4_p4"], u_amp=1.0, h_amp=0.05)
    G = oracle.OracleGrid(w.ne, w.ns, *w.constants())
    Q, _ = inputs.initial_state(w, *G.node_frames())
    T = 14400.0 * w.dt_nd / w.dt_s
    nref = 32
    sol = scipy.integrate.solve_ivp(lambda t, y: G.rhs(y), (0.0, T), Q, method="DOP853", rtol=1e-13, atol=1e-16,
                                    t_eval=np.linspace(0.0, T, nref + 1))
    assert sol.status == 0
    R = sol.y.T
    errs = {}
    for order in (4, 5, 6):
        errs[order] = []
        for nst in (8, 16, 32):
            E = epi.EPI(G.rhs, lambda q, v: G.jvp(q, v, 1e-150), order, T / nst, Q,
                        kiops_opts=dict(tol=1e-14, m_max=64))
            k = nref // nst
            E.q = R[E.P * k].copy()
            E.hist_q = [R[(E.P - i) * k].copy() for i in range(1, E.P + 1)]
            E.hist_F = [G.rhs(x) for x in E.hist_q]
            E.n = E.P
            for _ in range(nst - E.P):
                E.step()
            errs[order].append(np.linalg.norm(E.q - R[-1]) / np.linalg.norm(R[-1]))
        slopes = np.log2(np.array(errs[order][:-1]) / np.array(errs[order][1:]))
        assert np.all(slopes >= order - 1), (order, errs[order], slopes)
    for i in range(3):
        assert errs[6][i] < errs[5][i] < errs[4][i], [errs[o][i] for o in (4, 5, 6)]
