"""Pins of the oracle's Sec. 5.1 test problems (oracle/ode.py): exact
solutions, stencils against closed-form derivatives (second-order
convergence), and the exact Jacobian-vector products against central
differences of the right-hand sides."""
import numpy as np
import pytest

from oracle import ode


def test_semilinear_exact_solution_solves_the_semidiscrete_system():
    rhs, jvp, u0, exact = ode.semilinear(400)
    n = 400
    x = np.arange(1, n + 1) / (n + 1)
    for t in (0.0, 0.37, 1.0):
        ref = np.concatenate([x * (1 - x) * np.exp(t), [1.0]])
        assert np.abs(rhs(exact(t)) - ref).max() < 1e-9
    assert np.array_equal(u0, exact(0.0))


def test_semilinear_integral_and_diffusion_terms():
    # u = 1 inside (zero boundary values): the discrete Laplacian is -1/h^2 at
    # the two end nodes and 0 elsewhere; the trapezoid integral is n h
    n = 50
    rhs, jvp, _, _ = ode.semilinear(n)
    h = 1.0 / (n + 1)
    v = np.concatenate([np.ones(n), [0.0]])
    jv = jvp(np.concatenate([np.zeros(n), [0.0]]), v)
    lap = np.zeros(n)
    lap[0] = lap[-1] = -1.0 / h ** 2
    assert np.allclose(jv[:-1], lap + n * h, rtol=1e-13, atol=1e-9) and jv[-1] == 0.0


@pytest.mark.parametrize("name", ["adr", "burgers", "semilinear"])
def test_jvp_is_the_derivative_of_rhs(name):
    p = ode.PROBLEMS[name]()
    rhs, jvp, u0 = p[0], p[1], p[2]
    rng = np.random.default_rng(3)
    v = rng.standard_normal(u0.size)
    jv = jvp(u0, v)
    errs = []
    for h in (1e-3, 1e-4):
        fd = (rhs(u0 + h * v) - rhs(u0 - h * v)) / (2 * h)
        errs.append(np.linalg.norm(fd - jv) / np.linalg.norm(jv))
    # F is at most cubic in u: the central-difference error is O(h^2)
    assert errs[1] < 1e-7 and errs[1] < errs[0] / 50 or errs[0] < 1e-10


def test_adr_constants_and_reaction():
    rhs, jvp, u0 = ode.adr(20)
    for c in (0.0, 0.3, 0.5, 0.9, 1.0):
        f = rhs(np.full(400, c))
        assert np.allclose(f, 100.0 * c * (c - 0.5) * (1 - c), rtol=1e-13, atol=1e-12)
    assert abs(u0.min() - 0.3) < 1e-15 and abs(u0.max() - 1.3) < 0.02


def test_adr_second_order_on_a_neumann_compatible_field():
    a, e, g = -10.0, 0.01, 100.0
    errs = []
    for N in (17, 33, 65):
        rhs, _, _ = ode.adr(N)
        x = np.linspace(0, 1, N)
        X, Y = np.meshgrid(x, x)
        U = np.cos(np.pi * X) * np.cos(np.pi * Y)
        ux = -np.pi * np.sin(np.pi * X) * np.cos(np.pi * Y)
        uy = -np.pi * np.cos(np.pi * X) * np.sin(np.pi * Y)
        ref = -a * (ux + uy) + e * (-2 * np.pi ** 2 * U) + g * U * (U - 0.5) * (1 - U)
        errs.append(np.abs(rhs(U.reshape(-1)) - ref.reshape(-1)).max())
    r = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(r - 2.0) < 0.15), r


def test_burgers_second_order_and_initial_state():
    errs = []
    for n in (63, 127, 255):
        rhs, _, _ = ode.burgers(n)
        x = np.arange(1, n + 1) / (n + 1)
        u = np.sin(np.pi * x)
        ref = -u * np.pi * np.cos(np.pi * x) - 1e-3 * np.pi ** 2 * u
        errs.append(np.abs(rhs(u) - ref).max())
    r = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(r - 2.0) < 0.15), r
    _, _, u0 = ode.burgers()
    x = np.arange(1, 1025) / 1025
    assert np.allclose(u0, np.exp(-((x - 0.3) ** 2) / (2 * 0.05 ** 2)))


def test_burgers_mass_changes_only_through_the_boundaries():
    # sum of the conservative flux differences telescopes: with u = 0 at both
    # ends the discrete advective tendency sums to the boundary flux terms
    rhs, _, u0 = ode.burgers(200, eps=0.0)
    u = u0.copy()
    f = rhs(u)
    h = 1.0 / 201
    assert abs(f.sum() - (u[0] ** 2 + u[1] ** 2 - u[-1] ** 2 - u[-2] ** 2) / (4 * h)) < 1e-9
