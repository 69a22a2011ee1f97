"""FP64 CPU oracle for the DFR shallow-water J*v / KIOPS / EPI hot path.

TEST INFRASTRUCTURE ONLY.  This package is the reference the GPU library is
checked against.  It may be imported only by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``.
It shares no code with ``paper_2101_05617_amd`` (no kernels, headers, tables or
helpers); the only thing both sides consume is the seeded input generator
module, which holds none of the method's arithmetic.

Layout of the package:
  dfr_oracle.c  geometry, DFR right-hand side, complex-step J*v (plain C, FP64)
  phi.py        scalar phi-functions and the dense augmented-matrix reference
  kiops.py      adaptive Krylov phi-combination with incomplete orthogonalisation
  epi.py        multistep EPI2..EPI6 integrators with the EPI2 start-up
  ode.py        the stiff ODE test problems of Sec. 5.1 (numpy)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dfr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# plain build: no FMA contraction, no fast-math, so every operation is the one written;
# OpenMP only splits the element loop of the right-hand side (OMP_NUM_THREADS)
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (CPU only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        d = ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, d, d, d, d, d, d, vp]
        L.orc_destroy.argtypes = [vp]
        L.orc_num_nodes.restype = ctypes.c_int64
        L.orc_num_nodes.argtypes = [vp]
        for name in ("orc_rhs",):
            getattr(L, name).argtypes = [vp, vp, vp]
            getattr(L, name).restype = ctypes.c_int
        L.orc_jvp.argtypes = [vp, vp, vp, d, vp]
        L.orc_jvp.restype = ctypes.c_int
        L.orc_rhs_split.argtypes = [vp, vp, vp, vp, vp]
        L.orc_rhs_split.restype = ctypes.c_int
        L.orc_node_frames.argtypes = [vp, vp, vp, vp]
        L.orc_node_metric.argtypes = [vp, vp]
        L.orc_mass_weights.argtypes = [vp, vp]
        L.orc_get_operators.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_get_panels.argtypes = [vp, vp]
        L.orc_panel_angles.argtypes = [d, d, d, vp, vp, vp]
        L.orc_appc_matrix.argtypes = [ctypes.c_int, ctypes.c_int, d, vp]
        L.orc_connectivity.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.orc_ausm_split.argtypes = [d, vp, vp, vp, vp]
        L.orc_common_flux.argtypes = [vp, vp, vp, d, vp, ctypes.c_int, vp]
        L.orc_set_riemann.argtypes = [vp, ctypes.c_int]
        L.orc_diagnostics.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_diagnostics.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


_ERR = {-1: "invalid argument", -2: "out of memory", -4: "non-finite input", -5: "non-positive depth H"}


def _check(rc):
    if rc != 0:
        raise OracleError(_ERR.get(rc, f"error {rc}"))


class OracleGrid:
    """One rotated cubed-sphere DFR discretisation (ne elements per panel edge,
    ns = p+1 Gauss-Legendre points per element edge).  riemann: "rusanov"
    (Sec. 3.1) or "ausm" (App. D) for the common flux at element faces."""

    RIEMANN = {"rusanov": 0, "ausm": 1}

    def __init__(self, ne, ns, radius=1.0, omega=1.0, gravity=1.0,
                 rotation=(0.0, np.pi / 4, 0.0), hB=None, riemann="rusanov"):
        self.ne, self.ns = int(ne), int(ns)
        self.radius, self.omega, self.gravity = float(radius), float(omega), float(gravity)
        self.rotation = tuple(float(r) for r in rotation)
        L = lib()
        hb = None
        if hB is not None:
            hb = np.ascontiguousarray(hB, dtype=np.float64)
        self._hb = hb
        h = L.orc_create(self.ne, self.ns, self.radius, self.omega, self.gravity,
                         *self.rotation, _ptr(hb) if hb is not None else None)
        if not h:
            raise OracleError("orc_create failed")
        self._h = h
        self.N = int(L.orc_num_nodes(h))
        self.riemann = riemann
        L.orc_set_riemann(h, self.RIEMANN[riemann])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    # -- the method ------------------------------------------------------
    def rhs(self, Q):
        Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(-1)
        out = np.empty_like(Q)
        _check(lib().orc_rhs(self._h, _ptr(Q), _ptr(out)))
        return out

    def jvp(self, Q, V, eps=1e-150):
        Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(-1)
        V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1)
        out = np.empty_like(Q)
        _check(lib().orc_jvp(self._h, _ptr(Q), _ptr(V), float(eps), _ptr(out)))
        return out

    def rhs_complex(self, Z):
        Z = np.asarray(Z, dtype=np.complex128).reshape(-1)
        re = np.ascontiguousarray(Z.real)
        im = np.ascontiguousarray(Z.imag)
        ore, oim = np.empty_like(re), np.empty_like(im)
        _check(lib().orc_rhs_split(self._h, _ptr(re), _ptr(im), _ptr(ore), _ptr(oim)))
        return ore + 1j * oim

    def diagnostics(self, Q, hB=None):
        """Sec. 5.4: (zeta, f, (mass, energy, potential enstrophy)) -- nodal
        relative vorticity (Eq. 43), Coriolis parameter (Eq. 46) and the
        integrals over the sphere of H, the total energy and the potential
        enstrophy.  hB: the nodal orography (energy term), or None."""
        Q = np.ascontiguousarray(Q, dtype=np.float64).reshape(-1)
        hb = None if hB is None else np.ascontiguousarray(hB, dtype=np.float64)
        z, f, out = np.empty(self.N), np.empty(self.N), np.empty(3)
        _check(lib().orc_diagnostics(self._h, _ptr(Q), None if hb is None else _ptr(hb), _ptr(z), _ptr(f),
                                     _ptr(out)))
        return z, f, tuple(out)

    # -- geometry accessors (for pins and for building inputs) ------------
    def node_frames(self):
        P = np.empty((self.N, 3)); B1 = np.empty((self.N, 3)); B2 = np.empty((self.N, 3))
        lib().orc_node_frames(self._h, _ptr(P), _ptr(B1), _ptr(B2))
        return P, B1, B2

    def node_metric(self):
        out = np.empty((self.N, 16))
        lib().orc_node_metric(self._h, _ptr(out))
        return out

    def mass_weights(self):
        w = np.empty(self.N)
        lib().orc_mass_weights(self._h, _ptr(w))
        return w

    def operators(self):
        ns = self.ns
        xi, w, lm, lp = (np.empty(ns) for _ in range(4))
        Dt = np.empty((ns, ns + 2))
        lib().orc_get_operators(self._h, _ptr(xi), _ptr(w), _ptr(lm), _ptr(lp), _ptr(Dt))
        return xi, w, lm, lp, Dt

    def common_flux(self, qL, qR, sg, h, n):
        """The grid's common flux sqrt(g) T^{mu n} at one face point from real
        tensor densities qL (low side) and qR (high side); h: 2x2 h^{ij}."""
        qL = np.ascontiguousarray(qL, dtype=np.float64)
        qR = np.ascontiguousarray(qR, dtype=np.float64)
        h4 = np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(4))
        F = np.empty(3)
        lib().orc_common_flux(self._h, _ptr(qL), _ptr(qR), float(sg), _ptr(h4), int(n), _ptr(F))
        return F

    def panels(self):
        out = np.empty(18)
        lib().orc_get_panels(self._h, _ptr(out))
        return out.reshape(6, 3)


def panel_angles(l0, f0, a0):
    lam, phi, alp = np.empty(6), np.empty(6), np.empty(6)
    lib().orc_panel_angles(l0, f0, a0, _ptr(lam), _ptr(phi), _ptr(alp))
    return lam, phi, alp


def ausm_split(M):
    """AUSM split functions at a real Froude number M: (M+, M-, P+/P, P-/P)."""
    out = [ctypes.c_double() for _ in range(4)]
    lib().orc_ausm_split(float(M), *[ctypes.byref(o) for o in out])
    return tuple(o.value for o in out)


def appc_matrix(dst, src, s):
    M = np.empty(4)
    lib().orc_appc_matrix(int(dst), int(src), float(s), _ptr(M))
    return M.reshape(2, 2)


def connectivity(p, edge):
    q, e, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib().orc_connectivity(int(p), int(edge), ctypes.byref(q), ctypes.byref(e), ctypes.byref(r))
    return q.value, e.value, r.value
