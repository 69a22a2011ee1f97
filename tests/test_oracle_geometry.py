"""Pins of the oracle's geometry (App. B, App. C) against the paper's forward map,
Eq. (50), and geographic facts -- all written independently in the test."""
import os

import numpy as np
import pytest

import oracle
from tests import geom_ref as gr

ROT = (0.0, np.pi / 4, 0.0)
ROTATIONS = [ROT, (0.3, 0.5, 0.2), (0.0, 0.0, 0.0), (0.7, 0.0, 0.0), (np.pi, -np.pi / 4, 0.0)]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_angles():
    rows = []
    with open(os.path.join(GOLDEN, "panel_angles_rot_0_pi4_0.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([eval(t, {"pi": np.pi}) for t in line.split()[1:]])
    return np.array(rows)


def test_panel_angles_worked_example():
    lam, phi, alp = oracle.panel_angles(*ROT)
    ref = _golden_angles()
    got = np.stack([lam, phi, alp], axis=1)
    # angles are compared as directions (mod 2 pi)
    assert np.allclose(np.cos(got), np.cos(ref), atol=1e-14)
    assert np.allclose(np.sin(got), np.sin(ref), atol=1e-14)


@pytest.mark.parametrize("rot", ROTATIONS)
def test_panel_centres_form_a_cube(rot):
    lam, phi, alp = oracle.panel_angles(*rot)
    c = np.stack([np.cos(phi) * np.cos(lam), np.cos(phi) * np.sin(lam), np.sin(phi)], axis=1)
    G = c @ c.T
    # antipodal pairs (0,2), (1,3), (4,5); all other pairs orthogonal
    ref = np.eye(6)
    for a, b in [(0, 2), (1, 3), (4, 5)]:
        ref[a, b] = ref[b, a] = -1.0
    assert np.allclose(G, ref, atol=1e-14)


@pytest.mark.parametrize("rot", ROTATIONS)
def test_inverse_map_matches_paper_forward_map(rot):
    G = oracle.OracleGrid(3, 4, rotation=rot)
    P, B1, B2 = G.node_frames()
    M = G.node_metric()
    ang = G.panels()
    per_panel = G.N // 6
    for p in range(6):
        sl = slice(p * per_panel, (p + 1) * per_panel)
        X, Y = gr.forward(P[sl], ang[p])
        assert np.allclose(X, M[sl, 14], atol=1e-13)
        assert np.allclose(Y, M[sl, 15], atol=1e-13)
        # basis vectors are the coordinate derivatives: d(X,Y)/ds along B1 = (1+X^2, 0)
        h = 1e-20
        X1, Y1 = gr.forward(P[sl] + 1j * h * B1[sl], ang[p])
        X2, Y2 = gr.forward(P[sl] + 1j * h * B2[sl], ang[p])
        assert np.allclose(X1.imag / h, 1 + X ** 2, atol=1e-12)
        assert np.allclose(Y1.imag / h, 0.0, atol=1e-12)
        assert np.allclose(X2.imag / h, 0.0, atol=1e-12)
        assert np.allclose(Y2.imag / h, 1 + Y ** 2, atol=1e-12)
    assert np.allclose(np.linalg.norm(P, axis=1), 1.0, atol=1e-15)


def test_metric_terms():
    a = 2.5
    G = oracle.OracleGrid(3, 5, radius=a, rotation=ROT)
    P, B1, B2 = G.node_frames()
    M = G.node_metric()
    X, Y = M[:, 14], M[:, 15]
    g11, g12, g22 = gr.metric_cov(X, Y, a)
    # Eqs. (64)-(66) are the Cartesian Gram matrix of the coordinate basis
    assert np.allclose(g11, a * a * np.einsum("ij,ij->i", B1, B1), rtol=1e-13)
    assert np.allclose(g12, a * a * np.einsum("ij,ij->i", B1, B2), rtol=1e-12, atol=1e-14)
    assert np.allclose(g22, a * a * np.einsum("ij,ij->i", B2, B2), rtol=1e-13)
    # h^ij (oracle, Eqs. 67-69) is the inverse of g_ij; sqrt(g) = sqrt(det g) (Eq. 70)
    h11, h12, h22 = M[:, 1], M[:, 2], M[:, 3]
    assert np.allclose(h11 * g11 + h12 * g12, 1.0, atol=1e-13)
    assert np.allclose(h11 * g12 + h12 * g22, 0.0, atol=1e-13)
    assert np.allclose(h12 * g12 + h22 * g22, 1.0, atol=1e-13)
    assert np.allclose(M[:, 0], np.sqrt(g11 * g22 - g12 * g12), rtol=1e-13)


def test_sphere_area_from_quadrature():
    # sum of w_m w_n sqrt(g) (Delta/2)^2 converges spectrally to 4 pi a^2 (Eq. 42)
    errs = []
    for ns in (2, 4, 6):
        G = oracle.OracleGrid(2, ns, radius=1.0)
        errs.append(abs(G.mass_weights().sum() - 4 * np.pi))
    assert errs[2] < 1e-7 and errs[2] < errs[1] < errs[0]


def _christoffel_eq50(x1, x2, a=1.0):
    """Gamma^i_jk from Eq. (50) with g_ij of Eqs. (64)-(66), complex-step derivatives."""
    h = 1e-30

    def g(x1, x2):
        g11, g12, g22 = gr.metric_cov(np.tan(x1), np.tan(x2), a)
        return np.array([[g11, g12], [g12, g22]])

    g0 = g(x1, x2).real
    dg = [g(x1 + 1j * h, x2).imag / h, g(x1, x2 + 1j * h).imag / h]   # dg[k][i][j] = d_k g_ij
    hinv = np.linalg.inv(g0)
    Gam = np.zeros((2, 2, 2))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                Gam[i, j, k] = 0.5 * sum(hinv[i, l] * (dg[k][l, j] + dg[j][l, k] - dg[l][j, k]) for l in range(2))
    return Gam


def _coriolis_eq50(x1, x2, ang, a=1.0, omega=1.0):
    """Gamma^i_0j = 1/2 h^ik (d_j g_k0 - d_k g_0j) (Eq. 50, time-independent metric)."""
    h = 1e-30

    def g0(x1, x2):
        return np.array(gr.metric_0i(np.tan(x1), np.tan(x2), ang, a, omega))

    d = [g0(x1 + 1j * h, x2).imag / h, g0(x1, x2 + 1j * h).imag / h]   # d[j][k] = d_j g_0k
    g11, g12, g22 = gr.metric_cov(np.tan(x1), np.tan(x2), a)
    hinv = np.linalg.inv(np.array([[g11, g12], [g12, g22]]))
    out = np.zeros((2, 2))
    for i in range(2):
        for j in range(2):
            out[i, j] = 0.5 * sum(hinv[i, k] * (d[j][k] - d[k][j]) for k in range(2))
    return out


def test_christoffel_symbols_from_eq50():
    G = oracle.OracleGrid(2, 3, radius=1.0, omega=1.0, rotation=ROT)
    M = G.node_metric()
    ang = G.panels()
    per_panel = G.N // 6
    for n in range(0, G.N, 7):
        X, Y = M[n, 14], M[n, 15]
        x1, x2 = np.arctan(X), np.arctan(Y)
        Gam = _christoffel_eq50(x1, x2)
        ora = np.array([[[M[n, 8], M[n, 9]], [M[n, 9], M[n, 10]]],
                        [[M[n, 11], M[n, 12]], [M[n, 12], M[n, 13]]]])
        assert np.allclose(Gam, ora, atol=1e-13)
        # the contraction h^jk Gamma^i_jk vanishes on the cubed sphere (App. B)
        hm = np.array([[M[n, 1], M[n, 2]], [M[n, 2], M[n, 3]]])
        assert np.allclose(np.einsum("jk,ijk->i", hm, ora), 0.0, atol=1e-14)
        p = n // per_panel
        C = _coriolis_eq50(x1, x2, ang[p])
        assert np.allclose(C, [[M[n, 4], M[n, 5]], [M[n, 6], M[n, 7]]], atol=1e-13)


@pytest.mark.parametrize("rot", ROTATIONS)
def test_coriolis_parameter_is_2_omega_sin_latitude(rot):
    # Eq. (45) evaluated with the oracle's Gamma^i_0j equals 2 Omega sin(latitude)
    om = 1.3
    G = oracle.OracleGrid(3, 4, radius=1.0, omega=om, rotation=rot)
    P, B1, B2 = G.node_frames()
    M = G.node_metric()
    X, Y = M[:, 14], M[:, 15]
    g11, g12, g22 = gr.metric_cov(X, Y)
    c10, c20 = M[:, 4], M[:, 6]     # Gamma^1_01, Gamma^2_01
    c11, c21 = M[:, 5], M[:, 7]     # Gamma^1_02, Gamma^2_02
    # f = (g_2k Gamma^k_10 - g_1k Gamma^k_20) / sqrt(g)
    f = ((g12 * c10 + g22 * c20) - (g11 * c11 + g12 * c21)) / M[:, 0]
    assert np.allclose(f, 2 * om * P[:, 2], atol=1e-13)


def _edge_point(edge, s):
    return {0: (-1.0, s), 1: (1.0, s), 2: (s, -1.0), 3: (s, 1.0)}[edge]


@pytest.mark.parametrize("rot", ROTATIONS)
def test_connectivity_matches_geometry(rot):
    ang = oracle.panel_angles(*rot)
    ang = np.stack(ang, axis=1)
    ss = np.tan(np.linspace(-np.pi / 4, np.pi / 4, 9)[1:-1])
    for p in range(6):
        for e in range(4):
            q, qe, rev = oracle.connectivity(p, e)
            Xs, Ys = np.array([_edge_point(e, s) for s in ss]).T
            Pt = gr.inverse(Xs, Ys, ang[p])
            Xq, Yq = gr.forward(Pt, ang[q])
            xq, yq = np.arctan(Xq), np.arctan(Yq)
            along = np.arctan(ss) * (-1 if rev else 1)
            exp = {0: (np.full_like(along, -np.pi / 4), along), 1: (np.full_like(along, np.pi / 4), along),
                   2: (along, np.full_like(along, -np.pi / 4)), 3: (along, np.full_like(along, np.pi / 4))}[qe]
            assert np.allclose(xq, exp[0], atol=1e-13), (p, e)
            assert np.allclose(yq, exp[1], atol=1e-13), (p, e)
            # the relation is symmetric
            assert oracle.connectivity(q, qe) == (p, e, rev)


@pytest.mark.parametrize("rot", ROTATIONS)
def test_appendix_c_relations_match_cartesian_jacobians(rot):
    # A_(dst) = d x_(dst) / d x_(src) A_(src), the Jacobian taken by complex step
    # through the paper's forward map on both panels
    ang = np.stack(oracle.panel_angles(*rot), axis=1)
    h = 1e-30
    for p in range(6):
        for e in range(4):
            q, qe, rev = oracle.connectivity(p, e)
            for s in np.tan(np.array([-0.6, -0.2, 0.1, 0.5])):
                X, Y = _edge_point(e, s)
                x1, x2 = np.arctan(X), np.arctan(Y)
                Jm = np.zeros((2, 2))
                for col, (d1, d2) in enumerate([(1j * h, 0), (0, 1j * h)]):
                    # point on neighbour panel q, perturbed in q's coordinates
                    Pq = gr.inverse(np.tan(x1 + 0), np.tan(x2 + 0), ang[p])
                    Xq, Yq = gr.forward(Pq, ang[q])
                    xq1, xq2 = np.arctan(Xq) + d1, np.arctan(Yq) + d2
                    Pp = gr.inverse(np.tan(xq1), np.tan(xq2), ang[q])
                    Xp, Yp = gr.forward(Pp, ang[p])
                    Jm[0, col] = np.arctan(Xp).imag / h
                    Jm[1, col] = np.arctan(Yp).imag / h
                # the tangent named in App. C: Y for equatorial pairs, X on the
                # equatorial panel for pairs with a polar panel
                if p < 4 and q < 4:
                    param = Y
                elif p < 4:
                    param = X
                else:
                    Pq = gr.inverse(X, Y, ang[p])
                    param = gr.forward(Pq, ang[q])[0]
                M = oracle.appc_matrix(p, q, param)
                assert np.allclose(M, Jm, atol=1e-12), (p, e, q, s, M, Jm)
