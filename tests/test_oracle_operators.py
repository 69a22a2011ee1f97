"""Pins of the oracle's 1-D DFR operators (Sec. 3.1, Eqs. 7-14)."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle


def ops(ns):
    return oracle.OracleGrid(1, ns).operators()


@pytest.mark.parametrize("ns", range(1, 11))
def test_gauss_legendre_matches_library(ns):
    xi, w, *_ = ops(ns)
    xr, wr = npleg.leggauss(ns)
    assert np.allclose(xi, xr, atol=2e-15, rtol=0)
    assert np.allclose(w, wr, atol=2e-15, rtol=0)


@pytest.mark.parametrize("ns", range(1, 11))
def test_face_extrapolation_exact_for_polynomials(ns):
    # Eq. (7): the Lagrange expansion reproduces every polynomial of degree <= ns-1
    xi, w, lm, lp, _ = ops(ns)
    for d in range(ns):
        assert abs(lm @ xi ** d - (-1.0) ** d) < 1e-12
        assert abs(lp @ xi ** d - 1.0) < 1e-12


@pytest.mark.parametrize("ns", range(1, 11))
def test_extended_derivative_matrix(ns):
    # Eqs. (11)-(13): D~ differentiates exactly every polynomial of degree <= ns+1
    # sampled on {-1, xi_1..xi_ns, +1}
    xi, w, lm, lp, Dt = ops(ns)
    ext = np.concatenate([[-1.0], xi, [1.0]])
    rng = np.random.default_rng(ns)
    for d in range(ns + 2):
        c = np.zeros(d + 1)
        c[d] = 1.0
        f = npleg.legval(ext, npleg.poly2leg(c))
        df = npleg.legval(xi, npleg.legder(npleg.poly2leg(c)))
        assert np.allclose(Dt @ f, df, atol=1e-11 * max(1.0, np.abs(df).max()))
    # constants are annihilated (rows sum to zero)
    assert np.allclose(Dt.sum(axis=1), 0.0, atol=1e-12)
    # Gauss quadrature of the derivative telescopes to the end values: the
    # discrete statement of conservation, sum_k w_k D~_kn = delta_{n,ns+1} - delta_{n,0}
    tele = w @ Dt
    ref = np.zeros(ns + 2)
    ref[0], ref[-1] = -1.0, 1.0
    assert np.allclose(tele, ref, atol=1e-12)
    # random polynomial of degree ns+1: check once more with mixed coefficients
    c = rng.standard_normal(ns + 2)
    f = np.polynomial.polynomial.polyval(ext, c)
    df = np.polynomial.polynomial.polyval(xi, np.polynomial.polynomial.polyder(c))
    assert np.allclose(Dt @ f, df, atol=1e-10)


@pytest.mark.parametrize("ns", range(1, 9))
def test_end_columns_are_radau_corrections(ns):
    # after Eq. (14): the end columns of D~ equal the derivatives of the left and
    # right Radau polynomials at the GL points, which is the DFR <-> nodal DG
    # (weak form) equivalence the paper relies on
    xi, w, lm, lp, Dt = ops(ns)
    Pn = np.zeros(ns + 1); Pn[ns] = 1.0
    Pn1 = np.zeros(ns + 2); Pn1[ns + 1] = 1.0
    gL = (-1.0) ** ns / 2.0 * npleg.legsub(Pn, Pn1)
    gR = 0.5 * npleg.legadd(Pn, Pn1)
    assert np.allclose(Dt[:, 0], npleg.legval(xi, npleg.legder(gL)), atol=1e-11)
    assert np.allclose(Dt[:, -1], npleg.legval(xi, npleg.legder(gR)), atol=1e-11)
