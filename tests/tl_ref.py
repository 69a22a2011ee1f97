"""An independent tangent-linear (forward-mode) evaluation of the DFR
right-hand side, for pinning the oracle's complex-step J v (Eq. 28).

Every quantity is carried as a pair (value, derivative along V) and
differentiated by hand, rule by rule: products, quotients and square roots
by the chain rule; |.| and max(., .) take the branch of the values (reading
R3).  The assembly is vectorised over the whole grid and follows the method,
not the oracle's code:
  - densities q = sqrt(g) Q (App. B), nodal fluxes sqrt(g) T^{mu n} of
    Eq. 136 in both directions;
  - states extrapolated to the four faces of every element (Eq. 7);
  - at each face point the neighbour's trace, through the panel connectivity
    and the App. C maps at panel edges, and the Rusanov common flux with the
    wave speed |u^n| + sqrt(h^nn g H) (Eqs. 147-148);
  - the extended-point derivative of Eqs. 12 and 14 in both directions,
    Coriolis and metric sources (Eq. 2 with Eqs. 71-80), division by sqrt(g).
Taken from the oracle: its 1-D operators, the nodal metric and Christoffel
tables, the panel connectivity and the App. C matrices (each pinned in the
geometry and operator tests).  Face-point metric terms (Eqs. 67-70) are
computed here.  Rusanov flux only, no orography.

Test infrastructure only."""
import numpy as np

import oracle


class Dual:
    """value v and derivative d (numpy arrays of one shape)."""

    __slots__ = ("v", "d")
    __array_ufunc__ = None     # numpy arrays on the left defer to the reflected operators

    def __init__(self, v, d):
        self.v, self.d = v, d

    @staticmethod
    def _pair(x):
        return (x.v, x.d) if isinstance(x, Dual) else (x, 0.0)

    def __add__(self, o):
        ov, od = Dual._pair(o)
        return Dual(self.v + ov, self.d + od)

    __radd__ = __add__

    def __sub__(self, o):
        ov, od = Dual._pair(o)
        return Dual(self.v - ov, self.d - od)

    def __rsub__(self, o):
        ov, od = Dual._pair(o)
        return Dual(ov - self.v, od - self.d)

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __mul__(self, o):
        ov, od = Dual._pair(o)
        return Dual(self.v * ov, self.d * ov + self.v * od)

    __rmul__ = __mul__

    def __truediv__(self, o):
        ov, od = Dual._pair(o)
        return Dual(self.v / ov, (self.d * ov - self.v * od) / (ov * ov))

    def sqrt(self):
        r = np.sqrt(self.v)
        return Dual(r, self.d / (2.0 * r))


def d_abs(z):
    s = np.where(z.v >= 0.0, 1.0, -1.0)
    return Dual(s * z.v, s * z.d)


def d_max(a, b):
    m = a.v >= b.v
    return Dual(np.where(m, a.v, b.v), np.where(m, a.d, b.d))


def lin(op, z):
    """a linear operation applied to both parts."""
    return Dual(op(z.v), op(z.d))


def metric(X, Y, a):
    """sqrt(g), h^11, h^12, h^22 at the points (X, Y) (Eqs. 67-70)."""
    d2 = 1.0 + X * X + Y * Y
    sg = a * a * (1.0 + X * X) * (1.0 + Y * Y) / (d2 * np.sqrt(d2))
    h11 = d2 / (a * a * (1.0 + X * X))
    h22 = d2 / (a * a * (1.0 + Y * Y))
    h12 = X * Y * d2 / (a * a * (1.0 + X * X) * (1.0 + Y * Y))
    return sg, h11, h12, h22


def normal_flux(q, sg, h, n, g):
    """sqrt(g) T^{mu n} of Eq. 136 from densities q = (q0, q1, q2); h[i][j]."""
    return [q[1 + n],
            q[1] * q[1 + n] / q[0] + (g * h[0][n] / (2.0 * sg)) * (q[0] * q[0]),
            q[2] * q[1 + n] / q[0] + (g * h[1][n] / (2.0 * sg)) * (q[0] * q[0])]


def rusanov(qL, qR, sg, h, n, g, aL, aR):
    """The common flux, and where its derivative is ambiguous: a branch of
    |u^n| or of the max of the wave speeds decided within rounding, where
    either one-sided derivative is correct, at a face point whose jump
    q_R - q_L (which multiplies the derivative of the wave speed) is above
    rounding.  aL, aR: the sums of the magnitudes of the terms of each side's
    normal-momentum trace, so that a sign of u^n within 16 ulps of them is
    decided within rounding."""
    FL, FR = normal_flux(qL, sg, h, n, g), normal_flux(qR, sg, h, n, g)
    uL, uR = qL[1 + n] / qL[0], qR[1 + n] / qR[0]
    gL, gR = ((h[n][n] * g / sg) * qL[0]).sqrt(), ((h[n][n] * g / sg) * qR[0]).sqrt()
    cL, cR = d_abs(uL) + gL, d_abs(uR) + gR
    lam = d_max(cL, cR)
    tol = 1e-13 * np.maximum(cL.v, cR.v)
    eps16 = 16.0 * np.finfo(np.float64).eps
    branch = (np.abs(qL[1 + n].v) <= eps16 * aL) | (np.abs(qR[1 + n].v) <= eps16 * aR) | \
        (np.abs(cL.v - cR.v) <= tol)
    jump = np.maximum.reduce([np.abs(qR[m].v - qL[m].v) for m in range(3)]) / (qL[0].v + qR[0].v)
    tie = branch & (jump > 1e-12)
    return [0.5 * (FL[m] + FR[m]) - 0.5 * lam * (qR[m] - qL[m]) for m in range(3)], tie


W_, E_, S_, N_ = 0, 1, 2, 3


def rhs_tangent(G, Q, V):
    """(F(Q), J(Q) V, ambiguous) by forward-mode differentiation; G an
    oracle.OracleGrid (Rusanov flux, no orography).  ambiguous marks the
    unknowns of elements with a face point where the Rusanov flux is not
    differentiable up to rounding (see rusanov): there J V is one of several
    correct one-sided derivatives."""
    ne, ns, g, a = G.ne, G.ns, G.gravity, G.radius
    xi, _, lm, lp, Dt = G.operators()
    Mt = G.node_metric().reshape(6, ne, ne, ns, ns, 16)
    shape = (6, ne, ne, ns, ns)      # panel, element row, element column, node row, node column
    Z = [Dual(np.asarray(Q, dtype=np.float64).reshape(3, *shape)[f],
              np.asarray(V, dtype=np.float64).reshape(3, *shape)[f]) for f in range(3)]
    sg = Mt[..., 0]
    h = [[Mt[..., 1], Mt[..., 2]], [Mt[..., 2], Mt[..., 3]]]
    q = [sg * z for z in Z]
    F = [normal_flux(q, sg, h, n, g) for n in (0, 1)]      # F[n][f]

    # traces of Q on the four faces of every element: T[edge][f], indexed
    # (panel, ej, ei, t)
    T = [[lin(lambda x: x @ lm, z) for z in Z],                         # W: along the node row
         [lin(lambda x: x @ lp, z) for z in Z],                         # E
         [lin(lambda x: np.einsum("...kt,k->...t", x, lm), z) for z in Z],   # S: along the column
         [lin(lambda x: np.einsum("...kt,k->...t", x, lp), z) for z in Z]]   # N

    # the same traces of |Q| with the weights' magnitudes: the scale of their
    # rounding errors
    A = [[np.abs(z.v) @ np.abs(lm) for z in Z], [np.abs(z.v) @ np.abs(lp) for z in Z],
         [np.einsum("...kt,k->...t", np.abs(z.v), np.abs(lm)) for z in Z],
         [np.einsum("...kt,k->...t", np.abs(z.v), np.abs(lp)) for z in Z]]

    delta = 0.5 * np.pi / ne
    edge_x = -0.25 * np.pi + delta * np.arange(ne + 1)
    node_x = -0.25 * np.pi + delta * (np.arange(ne)[:, None] + 0.5 * (1.0 + xi)[None, :])   # (element, node)

    def neighbour_traces(edge):
        """the neighbour's trace on face `edge` of every element, in this
        element's panel basis: [f] of (panel, ej, ei, t); and the same for the
        traces of magnitudes (App. C through the magnitudes of its entries)."""
        opp = {W_: E_, E_: W_, S_: N_, N_: S_}[edge]
        out = [Dual(np.empty((6, ne, ne, ns)), np.empty((6, ne, ne, ns))) for _ in range(3)]
        oab = [np.empty((6, ne, ne, ns)) for _ in range(3)]
        src = T[opp]
        for f in range(3):
            if edge == W_:
                oab[f][:, :, 1:] = A[opp][f][:, :, :-1]
            elif edge == E_:
                oab[f][:, :, :-1] = A[opp][f][:, :, 1:]
            elif edge == S_:
                oab[f][:, 1:] = A[opp][f][:, :-1]
            else:
                oab[f][:, :-1] = A[opp][f][:, 1:]
            if edge == W_:
                out[f].v[:, :, 1:], out[f].d[:, :, 1:] = src[f].v[:, :, :-1], src[f].d[:, :, :-1]
            elif edge == E_:
                out[f].v[:, :, :-1], out[f].d[:, :, :-1] = src[f].v[:, :, 1:], src[f].d[:, :, 1:]
            elif edge == S_:
                out[f].v[:, 1:], out[f].d[:, 1:] = src[f].v[:, :-1], src[f].d[:, :-1]
            else:
                out[f].v[:, :-1], out[f].d[:, :-1] = src[f].v[:, 1:], src[f].d[:, 1:]
        # panel edges: connectivity and App. C
        for p in range(6):
            qp, qedge, rev = oracle.connectivity(p, edge)
            for al in range(ne):           # element index along the edge on panel p
                ae = ne - 1 - al if rev else al
                qej, qei = {W_: (ae, 0), E_: (ae, ne - 1), S_: (0, ae), N_: (ne - 1, ae)}[qedge]
                ej, ei = {W_: (al, 0), E_: (al, ne - 1), S_: (0, al), N_: (ne - 1, al)}[edge]
                for t in range(ns):
                    qt = ns - 1 - t if rev else t
                    val = [T[qedge][f].v[qp, qej, qei, qt] for f in range(3)]
                    der = [T[qedge][f].d[qp, qej, qei, qt] for f in range(3)]
                    mag = [A[qedge][f][qp, qej, qei, qt] for f in range(3)]
                    # the along-edge tangent the App. C relation is written in
                    if p < 4 and qp < 4:
                        s = np.tan(node_x[ej, t])
                    elif p < 4:
                        s = np.tan(node_x[ei, t])
                    else:
                        s = np.tan(node_x[qei, qt])
                    M = oracle.appc_matrix(p, qp, s)
                    out[0].v[p, ej, ei, t], out[0].d[p, ej, ei, t] = val[0], der[0]
                    oab[0][p, ej, ei, t] = mag[0]
                    for i in range(2):
                        out[1 + i].v[p, ej, ei, t] = M[i, 0] * val[1] + M[i, 1] * val[2]
                        out[1 + i].d[p, ej, ei, t] = M[i, 0] * der[1] + M[i, 1] * der[2]
                        oab[1 + i][p, ej, ei, t] = abs(M[i, 0]) * mag[1] + abs(M[i, 1]) * mag[2]
        return out, oab

    # common fluxes on the four faces: C[edge][f] of (panel, ej, ei, t);
    # elements with a face point of ambiguous derivative
    C = []
    ties = np.zeros((6, ne, ne), dtype=bool)
    for edge in (W_, E_, S_, N_):
        if edge in (W_, E_):
            xe = edge_x[np.arange(ne) + (1 if edge == E_ else 0)]
            X = np.tan(xe)[None, None, :, None] * np.ones((6, ne, ne, ns))
            Y = np.tan(node_x)[None, :, None, :] * np.ones((6, ne, ne, ns))
            n = 0
        else:
            ye = edge_x[np.arange(ne) + (1 if edge == N_ else 0)]
            X = np.tan(node_x)[None, None, :, :] * np.ones((6, ne, ne, ns))
            Y = np.tan(ye)[None, :, None, None] * np.ones((6, ne, ne, ns))
            n = 1
        fsg, f11, f12, f22 = metric(X, Y, a)
        fh = [[f11, f12], [f12, f22]]
        own = [fsg * z for z in T[edge]]
        nbt, nba = neighbour_traces(edge)
        nb = [fsg * z for z in nbt]
        ao, an = fsg * A[edge][1 + n], fsg * nba[1 + n]
        if edge in (W_, S_):
            c, tie = rusanov(nb, own, fsg, fh, n, g, an, ao)
        else:
            c, tie = rusanov(own, nb, fsg, fh, n, g, ao, an)
        C.append(c)
        ties |= tie.any(axis=-1)

    # extended-point derivative (Eqs. 12, 14), sources, division by sqrt(g)
    Dw, De, Di = Dt[:, 0], Dt[:, ns + 1], Dt[:, 1:ns + 1]
    c0 = [[Mt[..., 4], Mt[..., 5]], [Mt[..., 6], Mt[..., 7]]]
    cs = [[[Mt[..., 8], Mt[..., 9]], [Mt[..., 9], Mt[..., 10]]],
          [[Mt[..., 11], Mt[..., 12]], [Mt[..., 12], Mt[..., 13]]]]
    out_v, out_d = np.empty((3, *shape)), np.empty((3, *shape))
    for f in range(3):
        # x^1: along the node row (last axis); faces W, E indexed by node row
        d1 = lin(lambda x: np.einsum("ik,...k->...i", Di, x), F[0][f])
        d1 = d1 + lin(lambda x: x[..., :, None] * Dw[None, :], C[W_][f]) \
                + lin(lambda x: x[..., :, None] * De[None, :], C[E_][f])
        # x^2: along the node column; faces S, N indexed by node column
        d2 = lin(lambda x: np.einsum("jk,...kn->...jn", Di, x), F[1][f])
        d2 = d2 + lin(lambda x: Dw[:, None] * x[..., None, :], C[S_][f]) \
                + lin(lambda x: De[:, None] * x[..., None, :], C[N_][f])
        r = (-2.0 / delta) * (d1 + d2)
        if f > 0:
            i = f - 1
            for j in range(2):
                r = r + (-2.0 * c0[i][j]) * q[1 + j]
                for k in range(2):
                    r = r - cs[i][j][k] * (q[1 + j] * q[1 + k] / q[0] + (0.5 * g * h[j][k] / sg) * (q[0] * q[0]))
        r = r / sg
        out_v[f], out_d[f] = r.v, r.d
    ambiguous = np.broadcast_to(ties[None, :, :, :, None, None], (3, *shape)).reshape(-1)
    return out_v.reshape(-1), out_d.reshape(-1), ambiguous
