"""Pins of the oracle's conservation diagnostics (Sec. 5.4, Eqs. 43-46):
relative vorticity, Coriolis parameter and the integrals of mass, total
energy and potential enstrophy, against closed forms on the sphere
(radius 1, Omega = 1 in the nondimensional system):

  area 4 pi;  int sin^2(lat) dA = int z^2 dA = 4 pi / 3;  int cos^2(lat) dA = 8 pi / 3;
  f = 2 Omega sin(lat);  zeta of u = u0 cos(lat) (solid-body rotation) = 2 u0 sin(lat).

Node latitudes come from the oracle's node positions; the wind is expressed
in the node basis by the input module (pinned by g_ij u^i u^j = |V|^2)."""
import math

import numpy as np
import pytest

import oracle
from paper_2101_05617_amd import inputs

ROT = inputs.ROTATION


def rest(G, H=1.0):
    return np.concatenate([np.full(G.N, H), np.zeros(2 * G.N)])


def solid_body(G, u0, H=1.0):
    P, B1, B2 = G.node_frames()
    lon, lat = inputs.lonlat(P)
    E, _ = inputs.east_north(P)
    u1, u2 = inputs.wind_to_contravariant(P, B1, B2, (u0 * np.cos(lat))[:, None] * E)
    return np.concatenate([np.full(G.N, H), H * u1, H * u2]), lat


def test_coriolis_parameter_is_two_omega_sin_latitude():
    for rot in (ROT, (0.3, 0.5, 0.2), (0.0, 0.0, 0.0)):
        G = oracle.OracleGrid(3, 4, 1.0, 1.7, 0.5, rotation=rot)
        P, _, _ = G.node_frames()
        _, f, _ = G.diagnostics(rest(G))
        assert np.abs(f - 2 * 1.7 * P[:, 2]).max() < 1e-14


@pytest.mark.parametrize("ne,p", [(3, 5), (4, 7)])
def test_rest_state_integrals(ne, p):
    g, Om = 0.8, 1.3
    G = oracle.OracleGrid(ne, p + 1, 1.0, Om, g, rotation=ROT)
    z, f, (m, e, s) = G.diagnostics(rest(G, 1.5))
    tol = 1e-9 if p == 5 else 1e-12
    assert abs(m - 1.5 * 4 * math.pi) < tol * m
    assert abs(e - 0.5 * g * 1.5 ** 2 * 4 * math.pi) < tol * e
    assert np.abs(z).max() == 0.0
    assert abs(s - (2 * Om) ** 2 / (2 * 1.5) * 4 * math.pi / 3) < tol * s


def test_energy_orography_term():
    # H = 1 over h_B = c z^2: E = g/2 int (1 + 2 h_B) dA = g/2 (4 pi + 2 c 4 pi / 3)
    g, c = 0.6, 0.05
    G = oracle.OracleGrid(4, 8, 1.0, 1.0, g, rotation=ROT)
    P, _, _ = G.node_frames()
    hB = c * P[:, 2] ** 2
    _, _, (_, e, _) = G.diagnostics(rest(G), hB=hB)
    assert abs(e - 0.5 * g * (4 * math.pi + 2 * c * 4 * math.pi / 3)) < 1e-12 * e


def test_solid_body_rotation_vorticity_energy_enstrophy():
    u0, g, Om = 0.3, 0.9, 1.0
    errs = []
    for ne, ns in ((3, 4), (3, 6), (3, 8)):
        G = oracle.OracleGrid(ne, ns, 1.0, Om, g, rotation=ROT)
        Q, lat = solid_body(G, u0)
        z, f, (m, e, s) = G.diagnostics(Q)
        errs.append(np.abs(z - 2 * u0 * np.sin(lat)).max() / (2 * u0))
    assert errs[1] < errs[0] / 20 and errs[2] < errs[1] / 20 and errs[2] < 1e-5
    e_ref = 0.5 * u0 ** 2 * 8 * math.pi / 3 + 0.5 * g * 4 * math.pi
    s_ref = 2 * (u0 + Om) ** 2 * 4 * math.pi / 3
    assert abs(e - e_ref) < 1e-10 * e_ref
    assert abs(s - s_ref) < 1e-8 * s_ref


def test_vorticity_sign_and_linearity():
    # zeta is linear in the wind at fixed H and reverses with it
    G = oracle.OracleGrid(3, 5, 1.0, 1.0, 0.5, rotation=ROT)
    Q, lat = solid_body(G, 0.2)
    Qm = Q.copy()
    Qm[G.N:] *= -1.0
    z, _, _ = G.diagnostics(Q)
    zm, _, _ = G.diagnostics(Qm)
    assert np.allclose(zm, -z, atol=1e-15)
    assert (z[lat > 0.3] > 0).all()


def test_mass_integral_is_the_rhs_weighting():
    # the mass integral uses the same weights under which the discrete mass
    # tendency vanishes
    w = inputs.WORKLOADS["c0_ne4_p4"]
    G = oracle.OracleGrid(w.ne, w.ns, *w.constants(), rotation=ROT)
    P, B1, B2 = G.node_frames()
    Q, _ = inputs.initial_state(w, P, B1, B2)
    _, _, (m, _, _) = G.diagnostics(Q)
    assert abs(m - G.mass_weights() @ Q[: G.N]) < 1e-14 * m


def test_diagnostics_reject_invalid_state():
    G = oracle.OracleGrid(2, 3)
    Q = rest(G)
    Q[3] = 0.0
    with pytest.raises(oracle.OracleError):
        G.diagnostics(Q)
