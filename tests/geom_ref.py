"""Test-only reference geometry written directly from the paper's forward map.

Eqs. (59)-(60) multiplied through by cos(lat) give X and Y as ratios of linear
forms in the Cartesian unit vector P = (cos lat cos lon, cos lat sin lon, sin lat):
    C = Px cos lp + Py sin lp,   S = Py cos lp - Px sin lp,
    den = cos fp C + Pz sin fp,
    X = (S cos ap + sin fp C sin ap - Pz cos fp sin ap) / den,
    Y = (S sin ap - sin fp C cos ap + Pz cos fp cos ap) / den.
Because X and Y are ratios of linear forms, the inverse is a cross product:
P is orthogonal to X*den_vec - numX_vec and to Y*den_vec - numY_vec.
All functions accept complex arguments (used for complex-step derivatives).
"""
import numpy as np


def _forms(lp, fp, ap):
    cl, sl, cf, sf, ca, sa = np.cos(lp), np.sin(lp), np.cos(fp), np.sin(fp), np.cos(ap), np.sin(ap)
    Cv = np.array([cl, sl, 0.0])
    Sv = np.array([-sl, cl, 0.0])
    Zv = np.array([0.0, 0.0, 1.0])
    den = cf * Cv + sf * Zv
    nx = ca * Sv + sf * sa * Cv - cf * sa * Zv
    ny = sa * Sv - sf * ca * Cv + cf * ca * Zv
    return den, nx, ny


def forward(P, angles):
    """(X, Y) of points P (..., 3) on the panel with angles (lp, fp, ap)."""
    den, nx, ny = _forms(*angles)
    d = P @ den
    return (P @ nx) / d, (P @ ny) / d


def inverse(X, Y, angles):
    """Unit-direction P (not normalised; any positive multiple) with forward(P) = (X, Y)."""
    den, nx, ny = _forms(*angles)
    X = np.asarray(X)[..., None]
    Y = np.asarray(Y)[..., None]
    a = X * den - nx
    b = Y * den - ny
    P = np.cross(a, b)
    s = np.sign(np.real(P @ den))
    return P * s[..., None]


def normalise(P):
    return P / np.sqrt(np.sum(P * P, axis=-1, keepdims=True))


def metric_cov(X, Y, a=1.0):
    """g_11, g_12, g_22 of Eqs. (64)-(66)."""
    d2 = 1.0 + X * X + Y * Y
    g11 = a * a / d2 ** 2 * (1 + X * X) ** 2 * (1 + Y * Y)
    g12 = -a * a / d2 ** 2 * X * Y * (1 + X * X) * (1 + Y * Y)
    g22 = a * a / d2 ** 2 * (1 + X * X) * (1 + Y * Y) ** 2
    return g11, g12, g22


def metric_0i(X, Y, angles, a=1.0, omega=1.0):
    """g_01, g_02 of Eqs. (62)-(63)."""
    lp, fp, ap = angles
    d2 = 1.0 + X * X + Y * Y
    g01 = a * a / d2 * omega * (1 + X * X) * (np.cos(fp) * np.cos(ap) - Y * np.sin(fp))
    g02 = a * a / d2 * omega * (1 + Y * Y) * (np.cos(fp) * np.sin(ap) + X * np.sin(fp))
    return g01, g02
