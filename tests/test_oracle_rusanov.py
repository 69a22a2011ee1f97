"""Pin of the oracle's Rusanov common flux through its wave speed (App. E,
Eqs. 144-148).

The Rusanov (local Lax-Friedrichs) flux at a face with normal direction n is
    F* = (F(q_L) + F(q_R))/2 - (lambda/2) (q_R - q_L),
where F is the physical normal flux of the tensor densities (Eq. 136) and
lambda the larger of the two sides' spectral radii of the flux Jacobian J^n
of Eq. (144).  Here J^1 and J^2 are built as printed in Eq. (146), their
eigenvalues are taken with numpy (not from the closed form of Eqs. 147-148),
and lambda is recovered from the oracle's common flux, component by
component, as 2 ((F_L + F_R)/2 - F*) / (q_R - q_L).

The states cover both signs of u^n, supersonic and subsonic sides, either
side carrying the larger speed, and off-diagonal metrics (h^12 != 0, as at
face points away from the panel centre lines).  The last test shows that
the plausible mistakes -- |u^n| dropped, h^nn dropped, or one side's speed
only -- each move lambda far outside the tolerance on these states."""
import numpy as np
import pytest

import oracle
from paper_2101_05617_amd import inputs

C0 = inputs.WORKLOADS["c0_ne4_p4"]
GRAV = C0.gravity_nd


def flux_jacobian(q, sg, h, n, g):
    """J^{n+1} of Eq. (146) at the tensor densities q = sqrt(g) (H, H u^1, H u^2)."""
    H = q[0] / sg
    u1, u2 = q[1] / q[0], q[2] / q[0]
    if n == 0:
        return np.array([[0.0, 1.0, 0.0],
                         [g * h[0, 0] * H - u1 * u1, 2.0 * u1, 0.0],
                         [g * h[0, 1] * H - u1 * u2, u2, u1]])
    return np.array([[0.0, 0.0, 1.0],
                     [g * h[0, 1] * H - u1 * u2, u2, u1],
                     [g * h[1, 1] * H - u2 * u2, 0.0, 2.0 * u2]])


def physical_flux(q, sg, h, n, g):
    """sqrt(g) T^{mu n} of Eq. (136), mu = 0, 1, 2 (q^0 in the mu = 0 slot)."""
    return np.array([q[1 + n]] + [q[1 + i] * q[1 + n] / q[0] + g * h[i, n] * q[0] ** 2 / (2.0 * sg)
                                  for i in range(2)])


def spectral_radius(q, sg, h, n, g):
    return float(np.max(np.abs(np.linalg.eigvals(flux_jacobian(q, sg, h, n, g)))))


def random_faces(seed, count=200):
    """(qL, qR, sg, h, n): random face states, metrics and directions."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        sg = rng.uniform(0.5, 2.0)
        a = rng.uniform(0.6, 1.6, size=2)
        c = rng.uniform(-0.45, 0.45) * np.sqrt(a[0] * a[1])
        h = np.array([[a[0], c], [c, a[1]]])      # symmetric positive definite, h^12 != 0
        n = k % 2
        qs = []
        for _ in range(2):
            H = rng.uniform(0.3, 2.0)
            speed = np.sqrt(h[n, n] * GRAV * H)
            un = rng.choice([-1.0, 1.0]) * rng.uniform(0.05, 3.0) * speed   # sub- and supersonic
            ut = rng.uniform(-1.0, 1.0) * speed
            u = np.zeros(2)
            u[n], u[1 - n] = un, ut
            qs.append(sg * H * np.array([1.0, u[0], u[1]]))
        out.append((qs[0], qs[1], sg, h, n))
    return out


def recovered_lambdas(G, qL, qR, sg, h, n):
    Fs = G.common_flux(qL, qR, sg, h, n)
    avg = 0.5 * (physical_flux(qL, sg, h, n, GRAV) + physical_flux(qR, sg, h, n, GRAV))
    dq = qR - qL
    return 2.0 * (avg - Fs) / dq


@pytest.mark.parametrize("seed", [0, 1])
def test_rusanov_speed_is_the_larger_spectral_radius_of_the_printed_jacobians(seed):
    G = oracle.OracleGrid(2, 3, 1.0, 1.0, GRAV, riemann="rusanov")
    left_larger = right_larger = 0
    for qL, qR, sg, h, n in random_faces(seed):
        rL, rR = spectral_radius(qL, sg, h, n, GRAV), spectral_radius(qR, sg, h, n, GRAV)
        lam = max(rL, rR)
        left_larger += rL > rR
        right_larger += rR > rL
        lr = recovered_lambdas(G, qL, qR, sg, h, n)
        # every component whose jump is not tiny gives the same lambda
        ok = np.abs(qR - qL) > 1e-6 * np.max(np.abs(np.concatenate([qL, qR])))
        assert ok.sum() >= 2
        assert np.all(np.abs(lr[ok] - lam) <= 1e-11 * lam), (lr, lam, n, h)
    assert left_larger > 20 and right_larger > 20


def test_rusanov_flux_is_consistent_and_linear_in_the_jump():
    # F*(q, q) = F(q); at fixed sides the dissipation is lambda/2 times the jump
    G = oracle.OracleGrid(2, 3, 1.0, 1.0, GRAV, riemann="rusanov")
    for qL, qR, sg, h, n in random_faces(7, 50):
        assert np.allclose(G.common_flux(qL, qL, sg, h, n), physical_flux(qL, sg, h, n, GRAV),
                           rtol=1e-14, atol=1e-15 * np.max(np.abs(qL)))


def test_the_pin_separates_plausible_mistakes():
    # wave speeds a mistaken oracle would use, against the eigenvalue speed:
    # each differs by far more than the 1e-11 tolerance on many faces
    faces = random_faces(3)
    wrong = {"|u^n| dropped": 0, "h^nn dropped": 0, "left side only": 0, "right side only": 0}
    for qL, qR, sg, h, n in faces:
        lam = max(spectral_radius(qL, sg, h, n, GRAV), spectral_radius(qR, sg, h, n, GRAV))

        def side(q, drop_u=False, drop_h=False):
            H, un = q[0] / sg, q[1 + n] / q[0]
            return (0.0 if drop_u else abs(un)) + np.sqrt((1.0 if drop_h else h[n, n]) * GRAV * H)

        cands = {"|u^n| dropped": max(side(qL, drop_u=True), side(qR, drop_u=True)),
                 "h^nn dropped": max(side(qL, drop_h=True), side(qR, drop_h=True)),
                 "left side only": side(qL), "right side only": side(qR)}
        for k, v in cands.items():
            wrong[k] += abs(v - lam) > 1e-6 * lam
    assert all(v > 40 for v in wrong.values()), wrong
