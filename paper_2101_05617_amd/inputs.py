"""Seeded synthetic inputs for the shallow-water workloads.

This module holds none of the numerical method's arithmetic.  Given, for
every node, its unit position vector P and the two coordinate basis vectors
dP/dx^1, dP/dx^2 on the unit sphere (computed by the caller's own geometry),
it evaluates analytic geographic fields (balanced zonal flow, jet, bumps,
mountain, random spherical-harmonic perturbations) and expresses the wind in
that basis.  Both the GPU library's tests and the oracle's tests take their
initial states from here; nothing here depends on either of them.

Unit system.  States are returned nondimensional: length a (Earth radius),
time 1/Omega, depth h_s (the reference depth of the workload).  The shallow-
water equations keep their form with radius = 1, omega = 1 and
gravity' = g h_s / (a^2 Omega^2); the library and the oracle are both called
with these constants.  Time steps scale as dt' = dt Omega.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

EARTH_RADIUS = 6.37122e6      # m
EARTH_OMEGA = 7.292e-5        # 1/s
GRAVITY = 9.80616             # m/s^2
ROTATION = (0.0, math.pi / 4.0, 0.0)   # (lambda0, phi0, alpha0) of panel 0


@dataclass(frozen=True)
class Workload:
    name: str
    ne: int
    p: int                       # DFR degree; ns = p + 1
    order: int                   # EPI order
    dt_s: float                  # time step, seconds
    steps: int
    tol: float
    m_max: int
    eps: float                   # complex-step epsilon (on the scaled state)
    seed: int
    kind: str                    # "zonal" | "jet" | "mountain"
    gh0: float = 2.94e4          # g h0, m^2/s^2
    u0: float = 2.0 * math.pi * EARTH_RADIUS / (12.0 * 86400.0)
    h_amp: float = 0.0           # perturbation amplitude of h, as a fraction of h0
    h_lmax: int = 0
    u_amp: float = 0.0           # perturbation amplitude of the wind, m/s
    precision: str = "fp64"      # "fp64" | "fp32_jv"
    startup_substeps: int = 10
    extra: dict = field(default_factory=dict)

    @property
    def ns(self) -> int:
        return self.p + 1

    @property
    def n_nodes(self) -> int:
        return 6 * self.ne * self.ne * self.ns * self.ns

    @property
    def h_scale(self) -> float:
        return self.gh0 / GRAVITY

    @property
    def gravity_nd(self) -> float:
        return self.gh0 / (EARTH_RADIUS ** 2 * EARTH_OMEGA ** 2)

    @property
    def dt_nd(self) -> float:
        return self.dt_s * EARTH_OMEGA

    def constants(self):
        """(radius, omega, gravity) of the nondimensional system."""
        return 1.0, 1.0, self.gravity_nd


WORKLOADS = {
    # ne=4, p=4, EPI4, dt 900 s, 4 steps, tol 1e-12, m <= 32, eps 1e-150
    "c0_ne4_p4": Workload("c0_ne4_p4", ne=4, p=4, order=4, dt_s=900.0, steps=4, tol=1e-12,
                          m_max=32, eps=1e-150, seed=0, kind="zonal", h_amp=1e-3, h_lmax=4),
    # ne=30, p=5, EPI5, dt 1800 s, 48 steps (1 day), tol 1e-10, m <= 64
    "c1_ne30_p5": Workload("c1_ne30_p5", ne=30, p=5, order=5, dt_s=1800.0, steps=48, tol=1e-10,
                           m_max=64, eps=1e-150, seed=1, kind="zonal", h_amp=1e-2, h_lmax=16,
                           u_amp=1.0),
    # ne=60, p=6, EPI6, dt 1200 s, 72 steps; complex-FP32 J*v with eps 1e-20
    "c2_ne60_p6_jet": Workload("c2_ne60_p6_jet", ne=60, p=6, order=6, dt_s=1200.0, steps=72,
                               tol=1e-10, m_max=64, eps=1e-20, seed=2, kind="jet",
                               precision="fp32_jv"),
    # ne=120, p=6, EPI6, dt 600 s, 144 steps; Gaussian mountain
    "c4_ne120_p6_mountain": Workload("c4_ne120_p6_mountain", ne=120, p=6, order=6, dt_s=600.0,
                                     steps=144, tol=1e-10, m_max=64, eps=1e-150, seed=4,
                                     kind="mountain", gh0=5960.0 * GRAVITY, u0=20.0),
    # the large-time-step regime: the mountain flow on a grid of 86,400 nodes
    # (ne=20, p=5) with dt = 4 h (Courant numbers 40-80 at this resolution)
    "f2_ne20_p5_mountain_dt4h": Workload("f2_ne20_p5_mountain_dt4h", ne=20, p=5, order=6, dt_s=14400.0,
                                         steps=90, tol=1e-10, m_max=64, eps=1e-150, seed=4,
                                         kind="mountain", gh0=5960.0 * GRAVITY, u0=20.0),
}


def ensemble_members(n_members=64, seed=3):
    """The batched-ensemble workload: members with ne ~ U{8,12,16,24,32,40},
    p ~ U{4,5,6}, u0 ~ U[10, 40] m/s drawn in that order from seed 3, and
    per-member perturbation seeds spawned from the same seed."""
    rng = np.random.default_rng(seed)
    nes = rng.choice(np.array([8, 12, 16, 24, 32, 40]), size=n_members)
    ps = rng.choice(np.array([4, 5, 6]), size=n_members)
    u0s = rng.uniform(10.0, 40.0, size=n_members)
    seeds = np.random.SeedSequence(seed).spawn(n_members)
    out = []
    for k in range(n_members):
        member_seed = int(seeds[k].generate_state(1)[0])
        out.append(Workload(f"c3_member{k}", ne=int(nes[k]), p=int(ps[k]), order=4, dt_s=900.0,
                            steps=96, tol=1e-10, m_max=32, eps=1e-20, seed=member_seed,
                            kind="zonal", u0=float(u0s[k]), h_amp=5e-3, h_lmax=12,
                            precision="fp32_jv"))
    return out


def small_variant(w: Workload, ne: int, p: int | None = None) -> Workload:
    """Same physics and recipe on a smaller grid (for parity tests)."""
    return replace(w, name=f"{w.name}_ne{ne}", ne=ne, p=w.p if p is None else p)


# ---------------------------------------------------------------------------
# geographic helpers

def lonlat(P):
    P = np.asarray(P)
    lon = np.arctan2(P[:, 1], P[:, 0])
    lat = np.arcsin(np.clip(P[:, 2], -1.0, 1.0))
    return lon, lat


def east_north(P):
    lon, lat = lonlat(P)
    E = np.stack([-np.sin(lon), np.cos(lon), np.zeros_like(lon)], axis=1)
    Nn = np.stack([-np.sin(lat) * np.cos(lon), -np.sin(lat) * np.sin(lon), np.cos(lat)], axis=1)
    return E, Nn


def great_circle(P, lon_c, lat_c):
    c = np.array([math.cos(lat_c) * math.cos(lon_c), math.cos(lat_c) * math.sin(lon_c), math.sin(lat_c)])
    return np.arccos(np.clip(P @ c, -1.0, 1.0))


def _sph_harm_rows(lmax, P):
    """Yield the real orthonormal spherical harmonics Y_lm, 1 <= l <= lmax,
    m = -l..l, in (l, m) order, evaluated at unit vectors P (one row at a time)."""
    P = np.asarray(P)
    ct = np.clip(P[:, 2], -1.0, 1.0)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = np.arctan2(P[:, 1], P[:, 0])
    # fully normalised associated Legendre functions, column by column in m
    Pb = {}
    pmm = np.full_like(ct, math.sqrt(1.0 / (4.0 * math.pi)))
    for m in range(0, lmax + 1):
        if m > 0:
            pmm = -math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * st * pmm
        Pb[(m, m)] = pmm
        if m + 1 <= lmax:
            Pb[(m + 1, m)] = math.sqrt(2.0 * m + 3.0) * ct * pmm
        for l in range(m + 2, lmax + 1):
            a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            Pb[(l, m)] = a * (ct * Pb[(l - 1, m)] - b * Pb[(l - 2, m)])
    cs = {m: (np.cos(m * ph), np.sin(m * ph)) for m in range(1, lmax + 1)}
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            if m < 0:
                yield math.sqrt(2.0) * Pb[(l, -m)] * cs[-m][1]
            elif m == 0:
                yield Pb[(l, 0)]
            else:
                yield math.sqrt(2.0) * Pb[(l, m)] * cs[m][0]


def n_sph_harm(lmax):
    return (lmax + 1) ** 2 - 1


def real_sph_harm(lmax, P):
    """All Y_lm (1 <= l <= lmax) at P as an array (n_lm, n_points)."""
    return np.array(list(_sph_harm_rows(lmax, P)))


def sph_harm_sum(coef, lmax, P):
    """sum_lm coef_lm Y_lm(P), accumulated row by row."""
    out = np.zeros(np.asarray(P).shape[0])
    for c, row in zip(coef, _sph_harm_rows(lmax, P)):
        out += c * row
    return out


def random_field(rng, lmax, P):
    """sum of Y_lm with N(0,1) coefficients drawn in (l, m) order, scaled to
    max |field| = 1 over the given points."""
    c = rng.standard_normal(n_sph_harm(lmax))
    f = sph_harm_sum(c, lmax, P)
    return f / np.max(np.abs(f))


def _stream_wind(rng, lmax, P):
    """Non-divergent wind r x grad(psi) of a random stream function, scaled to
    max |V| = 1.  The tangential gradient is the 3-D gradient of the
    zero-homogeneous extension psi(x/|x|), by central differences."""
    coef = rng.standard_normal(n_sph_harm(lmax))

    def psi(X):
        Xn = X / np.linalg.norm(X, axis=1, keepdims=True)
        return sph_harm_sum(coef, lmax, Xn)

    h = 1e-5
    grad = np.zeros_like(P)
    for c in range(3):
        d = np.zeros(3)
        d[c] = h
        grad[:, c] = (psi(P + d) - psi(P - d)) / (2.0 * h)
    V = np.cross(P, grad)
    return V / np.max(np.linalg.norm(V, axis=1))


def wind_to_contravariant(P, B1, B2, V):
    """Contravariant components (u^1, u^2) of the tangent vector V (given per
    unit radius, i.e. in rad per unit time) in the basis (B1, B2):
    V = u^1 B1 + u^2 B2, solved by the 2x2 normal equations."""
    g11 = np.einsum("ij,ij->i", B1, B1)
    g12 = np.einsum("ij,ij->i", B1, B2)
    g22 = np.einsum("ij,ij->i", B2, B2)
    r1 = np.einsum("ij,ij->i", B1, V)
    r2 = np.einsum("ij,ij->i", B2, V)
    det = g11 * g22 - g12 * g12
    u1 = (g22 * r1 - g12 * r2) / det
    u2 = (g11 * r2 - g12 * r1) / det
    return u1, u2


def _balanced_gh(lat, u0, gh0):
    """Free-surface geopotential of the steady zonal flow u = u0 cos(lat):
    g h = g h0 - (a Omega u0 + u0^2/2) sin^2(lat)."""
    return gh0 - (EARTH_RADIUS * EARTH_OMEGA * u0 + 0.5 * u0 * u0) * np.sin(lat) ** 2


def _jet_u(lat):
    return 80.0 * np.exp(-((lat - math.pi / 4.0) / 0.1) ** 2)


def _jet_gh(lat, gh_south):
    """g h(lat) from g dh/dlat = -a u (2 Omega sin(lat) + u tan(lat)/a),
    integrated from the south pole by composite 8-point Gauss-Legendre."""
    def dgh(phi):
        u = _jet_u(phi)
        return -EARTH_RADIUS * u * (2.0 * EARTH_OMEGA * np.sin(phi) + u * np.tan(phi) / EARTH_RADIUS)

    xg, wg = np.polynomial.legendre.leggauss(8)
    nb = 4000
    edges = np.linspace(-math.pi / 2, math.pi / 2, nb + 1)
    lo, hi = edges[:-1], edges[1:]
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    seg = (dgh(mid[:, None] + half[:, None] * xg[None, :]) * wg[None, :]).sum(axis=1) * half
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    k = np.clip(np.searchsorted(edges, lat, side="right") - 1, 0, nb - 1)
    a0 = edges[k]
    m2, h2 = 0.5 * (a0 + lat), 0.5 * (lat - a0)
    part = (dgh(m2[:, None] + h2[:, None] * xg[None, :]) * wg[None, :]).sum(axis=1) * h2
    return gh_south + cum[k] + part


def initial_state(w: Workload, P, B1, B2):
    """Nondimensional Q = (H, H u^1, H u^2) (field-major, length 3N) and the
    nondimensional orography h_B (or None) for workload `w` at the nodes
    described by P, B1, B2 (each N x 3, unit sphere)."""
    P = np.asarray(P, dtype=np.float64)
    a, Om = EARTH_RADIUS, EARTH_OMEGA
    rng = np.random.default_rng(w.seed)
    lon, lat = lonlat(P)
    E, Nn = east_north(P)
    hB = None
    if w.kind == "zonal":
        gh = _balanced_gh(lat, w.u0, w.gh0)
        ul = w.u0 * np.cos(lat)
        V = ul[:, None] * E
        H = gh / GRAVITY
    elif w.kind == "jet":
        lon_c = rng.uniform(0.0, 2.0 * math.pi)
        gh = _jet_gh(lat, w.gh0)
        V = _jet_u(lat)[:, None] * E
        d = great_circle(P, lon_c, math.pi / 4.0) * a
        H = gh / GRAVITY + 120.0 * np.exp(-(d / (a / 10.0)) ** 2)
    elif w.kind == "mountain":
        gh = _balanced_gh(lat, w.u0, w.gh0)
        ul = w.u0 * np.cos(lat)
        V = ul[:, None] * E
        d = great_circle(P, 1.5 * math.pi, math.pi / 6.0) * a
        hb = 2000.0 * np.exp(-(d / 1.5e6) ** 2)
        H = gh / GRAVITY - hb
        hB = hb / w.h_scale
    else:
        raise ValueError(w.kind)
    # seeded perturbations (drawn after the kind-specific draws)
    if w.h_amp > 0.0:
        H = H + w.h_amp * w.h_scale * random_field(rng, w.h_lmax, P)
    if w.u_amp > 0.0:
        V = V + w.u_amp * _stream_wind(rng, max(w.h_lmax, 1), P)
    # V in m/s -> rad/s on the unit sphere -> nondimensional (time unit 1/Omega)
    u1, u2 = wind_to_contravariant(P, B1, B2, V / a)
    Hn = H / w.h_scale
    u1n, u2n = u1 / Om, u2 / Om
    Q = np.concatenate([Hn, Hn * u1n, Hn * u2n])
    return Q, hB


def random_direction(n3, seed):
    """A seeded unit-scale direction vector for J*v tests (N(0,1) entries)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n3)


def ode_initial_state(name: str, n: int) -> np.ndarray:
    """Initial states of the Sec. 5.1 test problems in the library's unknown
    order: "adr" on the n x n vertex grid of [0,1]^2 (index j n + i, i along
    x), 256 (x y (1-x)(1-y))^2 + 0.3; "burgers" on the n interior points of
    [0,1], exp(-(x - 0.3)^2 / (2 0.05^2)); "semilinear" on the n interior
    points, x(1-x), followed by the time 0."""
    if name == "adr":
        x = np.arange(n) / (n - 1)
        X, Y = np.meshgrid(x, x)
        return (256.0 * (X * Y * (1 - X) * (1 - Y)) ** 2 + 0.3).reshape(-1)
    x = np.arange(1, n + 1) / (n + 1)
    if name == "burgers":
        return np.exp(-((x - 0.3) ** 2) / (2 * 0.05 ** 2))
    if name == "semilinear":
        return np.concatenate([x * (1 - x), [0.0]])
    raise KeyError(name)

