"""Python binding of the MI355X library ``libdfrsw.so`` (C ABI in include/dfrsw.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device vectors are torch tensors (float64, contiguous, on the
current HIP device); the library's work is enqueued on torch's current stream.
If the shared library is missing or cannot be loaded, every entry point raises
-- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfrsw.so")

DFR_FP64 = 0
DFR_FP32_JV = 1
DFR_FP32_JV_BASIS32 = 2
DFR_FP32_EPS_MIN = 1e-30   # smallest complex-step eps of the FP32 forms (as in the header)
_PREC = {"fp64": DFR_FP64, "fp32_jv": DFR_FP32_JV, "fp32_jv_basis32": DFR_FP32_JV_BASIS32,
         DFR_FP64: DFR_FP64, DFR_FP32_JV: DFR_FP32_JV, DFR_FP32_JV_BASIS32: DFR_FP32_JV_BASIS32}

ERRORS = {-1: "DFR_E_INVAL", -2: "DFR_E_NOMEM", -3: "DFR_E_HIP", -4: "DFR_E_NONFINITE", -5: "DFR_E_DEPTH",
          -6: "DFR_E_KIOPS"}


class DfrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _GridDesc(ctypes.Structure):
    _fields_ = [("ne", ctypes.c_int), ("p", ctypes.c_int), ("radius", ctypes.c_double),
                ("omega", ctypes.c_double), ("gravity", ctypes.c_double), ("lambda0", ctypes.c_double),
                ("phi0", ctypes.c_double), ("alpha0", ctypes.c_double), ("hB", ctypes.c_void_p)]


class KiopsDecision(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("m", ctypes.c_int), ("accept", ctypes.c_int)]


class _KiopsReplay(ctypes.Structure):
    _fields_ = [("rec", ctypes.POINTER(KiopsDecision)), ("rec_cap", ctypes.c_int), ("n_rec", ctypes.c_int),
                ("play", ctypes.POINTER(KiopsDecision)), ("n_play", ctypes.c_int), ("pos", ctypes.c_int)]


class DecisionReplay:
    """A kiops_replay: record the controller's decisions (tau, m, accept) of
    the attempts of one or more calls, and/or make the attempts take given
    decisions in order.  Pass it as kiops_opts(..., replay=...)."""

    def __init__(self, play=None, rec_cap=4096):
        self._rec = (KiopsDecision * rec_cap)() if rec_cap else None
        self._play = None
        self.struct = _KiopsReplay()
        if self._rec is not None:
            self.struct.rec = ctypes.cast(self._rec, ctypes.POINTER(KiopsDecision))
            self.struct.rec_cap = rec_cap
        if play is not None:
            play = list(play)
            self._play = (KiopsDecision * max(len(play), 1))(*[KiopsDecision(float(t), int(m), int(bool(a)))
                                                               for t, m, a in play])
            self.struct.play = ctypes.cast(self._play, ctypes.POINTER(KiopsDecision))
            self.struct.n_play = len(play)

    @property
    def pos(self):
        """Decisions of the replay list taken so far."""
        return self.struct.pos

    def recorded(self):
        """The recorded decisions, a list of (tau, m, accept)."""
        n = self.struct.n_rec
        if self._rec is None or n > len(self._rec):
            raise ValueError(f"{n} decisions recorded, room for {0 if self._rec is None else len(self._rec)}")
        return [(d.tau, d.m, bool(d.accept)) for d in self._rec[:n]]


class KiopsOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("m_init", ctypes.c_int), ("m_min", ctypes.c_int),
                ("m_max", ctypes.c_int), ("iop", ctypes.c_int), ("max_attempts", ctypes.c_int),
                ("replay", ctypes.POINTER(_KiopsReplay))]


class KiopsStats(ctypes.Structure):
    _fields_ = [("n_matvec", ctypes.c_int), ("n_substeps", ctypes.c_int), ("n_rejected", ctypes.c_int),
                ("m_last", ctypes.c_int), ("happy", ctypes.c_int), ("n_expm", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def kiops_opts(tol=1e-10, m_init=10, m_min=10, m_max=64, iop=2, max_attempts=1000, replay=None):
    """kiops_opts; replay: None or a DecisionReplay (kept alive by the returned object)."""
    o = KiopsOpts(tol, m_init, m_min, m_max, iop, max_attempts)
    if replay is not None:
        o.replay = ctypes.pointer(replay.struct)
        o._keep = replay
    return o


_lib = None


def lib():
    """Load the HIP library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
        sig = {
            "dfr_create": (i, [ctypes.POINTER(_GridDesc), vp, ctypes.POINTER(vp)]),
            "dfr_destroy": (i, [vp]),
            "dfr_num_nodes": (i64, [vp]),
            "dfr_create_ode": (i, [i, i, vp, ctypes.POINTER(vp)]),
            "dfr_num_unknowns": (i64, [vp]),
            "dfr_node_frames": (i, [vp, vp, vp, vp]),
            "dfr_sync": (i, [vp]),
            "dfr_stream_copy": (i, [vp, vp, ctypes.c_size_t, vp]),
            "dfr_rhs": (i, [vp, vp, vp]),
            "dfr_jvp_complex_step": (i, [vp, vp, vp, d, i, vp]),
            "dfr_jvp_complex_step_noalloc": (i, [vp, vp, vp, d, i, vp]),
            "kiops_phi_apply": (i, [vp, vp, d, i, ctypes.POINTER(vp), ctypes.POINTER(KiopsOpts), d, i, vp,
                                    ctypes.POINTER(KiopsStats)]),
            "epi_create": (i, [vp, i, d, i, vp, d, i, ctypes.POINTER(vp)]),
            "epi_step": (i, [vp, vp, ctypes.POINTER(KiopsOpts), vp, ctypes.POINTER(KiopsStats)]),
            "epi_get_state": (i, [vp, vp]),
            "epi_num_steps": (i64, [vp]),
            "epi_destroy": (i, [vp]),
            "epi_save": (i, [vp, vp, ctypes.POINTER(ctypes.c_size_t)]),
            "epi_load": (i, [vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]),
            "epi_step_concurrent": (i, [i, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(KiopsOpts), i,
                                        ctypes.POINTER(KiopsStats)]),
            "dfr_ensemble_create": (i, [i, ctypes.POINTER(_GridDesc), vp, ctypes.POINTER(vp)]),
            "dfr_ensemble_destroy": (i, [vp]),
            "dfr_ensemble_size": (i, [vp]),
            "dfr_ensemble_member": (vp, [vp, i]),
            "dfr_ensemble_autotune": (i, [vp, i]),
            "epi_ensemble_create": (i, [vp, i, d, i, ctypes.POINTER(vp), d, i, ctypes.POINTER(vp)]),
            "epi_ensemble_step": (i, [vp, vp, ctypes.POINTER(KiopsOpts), ctypes.POINTER(KiopsStats)]),
            "epi_ensemble_get_state": (i, [vp, i, vp]),
            "epi_ensemble_destroy": (i, [vp]),
            "dfr_set_tile": (i, [vp, i, i]),
            "dfr_set_riemann": (i, [vp, i]),
            "dfr_diagnostics": (i, [vp, vp, vp, vp, ctypes.POINTER(d)]),
            "dfr_get_riemann": (i, [vp, ctypes.POINTER(i)]),
            "dfr_get_tile": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i)]),
            "dfr_get_krylov_tile": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i)]),
            "dfr_autotune": (i, [vp, i, ctypes.POINTER(i), ctypes.POINTER(i)]),
            "dfr_timing_enable": (i, [vp, i]),
            "dfr_timing_read": (i, [vp, i, ctypes.POINTER(d), ctypes.POINTER(i64)]),
            "dfr_ensemble_set_rounds": (i, [vp, i]),
            "dfr_ensemble_round_counts": (i, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
            "dfr_ensemble_timing_enable": (i, [vp, i]),
            "dfr_ensemble_timing_kinds": (i, [vp, ctypes.c_uint]),
            "dfr_ensemble_timing_read": (i, [vp, i, ctypes.POINTER(d), ctypes.POINTER(i64), ctypes.POINTER(d)]),
            "dfr_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return ["dfr_create", "dfr_destroy", "dfr_num_nodes", "dfr_create_ode", "dfr_num_unknowns", "dfr_node_frames", "dfr_sync", "dfr_rhs",
            "dfr_jvp_complex_step", "dfr_jvp_complex_step_noalloc", "kiops_phi_apply", "epi_create", "epi_step", "epi_get_state",
            "epi_num_steps", "epi_destroy", "epi_save", "epi_load", "epi_step_concurrent", "dfr_ensemble_create", "dfr_ensemble_destroy",
            "dfr_ensemble_size", "dfr_ensemble_member", "dfr_ensemble_autotune", "epi_ensemble_create", "epi_ensemble_step",
            "epi_ensemble_get_state", "epi_ensemble_destroy", "dfr_set_riemann", "dfr_get_riemann", "dfr_diagnostics", "dfr_set_tile", "dfr_get_tile", "dfr_get_krylov_tile", "dfr_autotune", "dfr_timing_enable",
            "dfr_timing_read", "dfr_ensemble_set_rounds", "dfr_ensemble_round_counts", "dfr_ensemble_timing_enable",
            "dfr_ensemble_timing_read", "dfr_ensemble_timing_kinds", "dfr_stream_copy", "dfr_last_error"]


def dfr_stream_copy(src, dst, stream=None):
    """Copy the bytes of device tensor src into dst (same size) with the
    library's streaming copy (a measurement helper)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dfr_stream_copy: sizes differ")
    _check(lib().dfr_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                                 None if stream is None else ctypes.c_void_p(stream)))


def _check(rc):
    if rc != 0:
        raise DfrError(rc, lib().dfr_last_error().decode())


def _dev(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Grid:
    """A dfr_ctx: one rotated cubed-sphere DFR discretisation on the GPU."""

    def __init__(self, ne, p, radius=1.0, omega=1.0, gravity=1.0, rotation=(0.0, np.pi / 4, 0.0), hB=None):
        self.ne, self.p, self.ns = int(ne), int(p), int(p) + 1
        self._hb = None if hB is None else np.ascontiguousarray(hB, dtype=np.float64)
        desc = _GridDesc(self.ne, self.p, float(radius), float(omega), float(gravity), *map(float, rotation),
                         None if self._hb is None else self._hb.ctypes.data_as(ctypes.c_void_p))
        h = ctypes.c_void_p()
        _check(lib().dfr_create(ctypes.byref(desc), _stream(), ctypes.byref(h)))
        self._h = h
        self.N = int(lib().dfr_num_nodes(h))

    def close(self):
        if getattr(self, "_h", None):
            lib().dfr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def node_frames(self):
        P, B1, B2 = (np.empty((self.N, 3)) for _ in range(3))
        _check(lib().dfr_node_frames(self._h, *(a.ctypes.data_as(ctypes.c_void_p) for a in (P, B1, B2))))
        return P, B1, B2

    @property
    def length(self):
        """Doubles per state vector (3N on a grid)."""
        return 3 * self.N

    def empty(self):
        import torch
        return torch.empty(self.length, dtype=torch.float64, device="cuda")


ODE_PROBLEMS = {"adr": 1, "burgers": 2, "semilinear": 3}


class OdeProblem(Grid):
    """A context holding one of the Sec. 5.1 test problems ("adr", "burgers",
    "semilinear") of size n instead of a grid; used with dfr_rhs,
    dfr_jvp_complex_step (exact J v), kiops_phi_apply and the epi_* calls."""

    def __init__(self, problem, n):
        self.problem, self.n = problem, int(n)
        self._hb = None
        h = ctypes.c_void_p()
        _check(lib().dfr_create_ode(ODE_PROBLEMS[problem], self.n, _stream(), ctypes.byref(h)))
        self._h = h
        self.N = int(lib().dfr_num_unknowns(h))

    @property
    def length(self):
        return self.N


# ---- entry points with the names of the C ABI ---------------------------------

def dfr_sync(g: Grid):
    _check(lib().dfr_sync(g.handle))


def dfr_rhs(g: Grid, q, dqdt=None):
    dqdt = g.empty() if dqdt is None else dqdt
    _check(lib().dfr_rhs(g.handle, _dev(q), _dev(dqdt)))
    return dqdt


def dfr_jvp_complex_step(g: Grid, q, v, eps=1e-150, prec="fp64", jv=None):
    jv = g.empty() if jv is None else jv
    _check(lib().dfr_jvp_complex_step(g.handle, _dev(q), _dev(v), float(eps), _PREC[prec], _dev(jv)))
    return jv


def dfr_jvp_complex_step_noalloc(g: Grid, q, v, jv, eps=1e-150, prec="fp64"):
    """The allocation-free form: jv must be given (the call allocates nothing)."""
    _check(lib().dfr_jvp_complex_step_noalloc(g.handle, _dev(q), _dev(v), float(eps), _PREC[prec], _dev(jv)))
    return jv


def kiops_phi_apply(g: Grid, q_lin, tau_out, bs, opts=None, eps=1e-150, prec="fp64", w=None):
    """w = sum_k tau^k phi_k(tau J(q_lin)) b_k for bs = [b_0 (or None), b_1, ...]."""
    opts = opts or kiops_opts()
    w = g.empty() if w is None else w
    arr = (ctypes.c_void_p * len(bs))(*[None if b is None else _dev(b).value for b in bs])
    st = KiopsStats()
    _check(lib().kiops_phi_apply(g.handle, _dev(q_lin), float(tau_out), len(bs) - 1, arr, ctypes.byref(opts),
                                 float(eps), _PREC[prec], _dev(w), ctypes.byref(st)))
    return w, st.as_dict()


class EpiState:
    """An epi_state: multistep EPI integrator with its history on the GPU."""

    def __init__(self, g: Grid, order, dt, q0, startup_substeps=10, eps=1e-150, prec="fp64", _handle=None):
        self.g = g
        if _handle is not None:
            self._h = _handle
            return
        h = ctypes.c_void_p()
        _check(lib().epi_create(g.handle, int(order), float(dt), int(startup_substeps), _dev(q0), float(eps),
                                _PREC[prec], ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().epi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def epi_save(st: EpiState) -> bytes:
    """Checkpoint of an EPI integration (host bytes)."""
    n = ctypes.c_size_t(0)
    _check(lib().epi_save(st.handle, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().epi_save(st.handle, buf, ctypes.byref(n)))
    return buf.raw[: n.value]


def epi_load(g: Grid, data: bytes) -> EpiState:
    """A new EPI state on grid g from a checkpoint made by epi_save."""
    buf = ctypes.create_string_buffer(bytes(data), len(data))
    h = ctypes.c_void_p()
    _check(lib().epi_load(g.handle, buf, len(data), ctypes.byref(h)))
    return EpiState(g, 0, 0.0, None, _handle=h)


KERNEL_KINDS = {"jv_arnoldi": 0, "jv": 1, "rhs": 2, "update": 3, "expm": 4, "other": 5, "finalize": 6}


RIEMANN = {"rusanov": 0, "ausm": 1}


def dfr_set_riemann(g, solver):
    """Common flux at element faces of the grid (or ensemble member):
    "rusanov" or "ausm"."""
    _check(lib().dfr_set_riemann(g.handle, RIEMANN[solver]))


def dfr_get_riemann(g):
    r = ctypes.c_int()
    _check(lib().dfr_get_riemann(g.handle, ctypes.byref(r)))
    return {v: k for k, v in RIEMANN.items()}[r.value]


def dfr_diagnostics(g, q, zeta=True, fcor=False):
    """Sec. 5.4 diagnostics of the device state q: (zeta or None, f or None,
    (mass, total energy, potential enstrophy))."""
    import torch
    z = torch.empty(g.N, dtype=torch.float64, device="cuda") if zeta else None
    f = torch.empty(g.N, dtype=torch.float64, device="cuda") if fcor else None
    out = (ctypes.c_double * 3)()
    _check(lib().dfr_diagnostics(g.handle, _dev(q), None if z is None else _dev(z),
                                 None if f is None else _dev(f), out))
    return z, f, (out[0], out[1], out[2])


def dfr_set_tile(g: Grid, tx, ty):
    _check(lib().dfr_set_tile(g.handle, int(tx), int(ty)))


def dfr_get_tile(g: Grid):
    tx, ty = ctypes.c_int(), ctypes.c_int()
    _check(lib().dfr_get_tile(g.handle, ctypes.byref(tx), ctypes.byref(ty)))
    return tx.value, ty.value


def dfr_get_krylov_tile(g: Grid):
    tx, ty = ctypes.c_int(), ctypes.c_int()
    _check(lib().dfr_get_krylov_tile(g.handle, ctypes.byref(tx), ctypes.byref(ty)))
    return tx.value, ty.value


def dfr_autotune(g: Grid, prec="fp64"):
    tx, ty = ctypes.c_int(), ctypes.c_int()
    _check(lib().dfr_autotune(g.handle, _PREC[prec], ctypes.byref(tx), ctypes.byref(ty)))
    return tx.value, ty.value


def dfr_timing_enable(g: Grid, enable=True):
    _check(lib().dfr_timing_enable(g.handle, int(bool(enable))))


def dfr_timing_read(g: Grid, kind):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().dfr_timing_read(g.handle, KERNEL_KINDS.get(kind, kind), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def epi_create(g: Grid, order, dt, q0, startup_substeps=10, eps=1e-150, prec="fp64"):
    return EpiState(g, order, dt, q0, startup_substeps, eps, prec)


def epi_step(g: Grid, st: EpiState, opts=None, q_out=None):
    opts = opts or kiops_opts()
    s = KiopsStats()
    _check(lib().epi_step(g.handle, st.handle, ctypes.byref(opts), None if q_out is None else _dev(q_out),
                          ctypes.byref(s)))
    return s.as_dict()


def epi_step_concurrent(grids, states, opts=None, n_workers=8):
    """One step of every member (grids[i], states[i]), several host threads;
    returns per-member stats."""
    opts = opts or kiops_opts()
    n = len(grids)
    if n != len(states) or n == 0:
        raise ValueError("need one state per grid")
    ca = (ctypes.c_void_p * n)(*[g.handle for g in grids])
    sa = (ctypes.c_void_p * n)(*[s.handle for s in states])
    st = (KiopsStats * n)()
    _check(lib().epi_step_concurrent(n, ca, sa, ctypes.byref(opts), int(n_workers), st))
    return [x.as_dict() for x in st]


class _Member(Grid):
    """A member context owned by an ensemble (not destroyed on its own)."""

    def __init__(self, handle, ne, p):
        self.ne, self.p, self.ns = int(ne), int(p), int(p) + 1
        self._hb = None
        self._h = ctypes.c_void_p(handle)
        self.N = int(lib().dfr_num_nodes(self._h))

    def close(self):
        self._h = None


class EnsembleGrid:
    """A dfr_ensemble: members (ne_i, p_i) built from a list of dicts with the
    keys of Grid (ne, p, radius, omega, gravity, rotation, hB=None)."""

    def __init__(self, members):
        n = len(members)
        self._keep = []
        descs = (_GridDesc * n)()
        for k, m in enumerate(members):
            hb = m.get("hB")
            if hb is not None:
                hb = np.ascontiguousarray(hb, dtype=np.float64)
                self._keep.append(hb)
            rot = m.get("rotation", (0.0, np.pi / 4, 0.0))
            descs[k] = _GridDesc(int(m["ne"]), int(m["p"]), float(m.get("radius", 1.0)), float(m.get("omega", 1.0)),
                                 float(m.get("gravity", 1.0)), *map(float, rot),
                                 None if hb is None else hb.ctypes.data_as(ctypes.c_void_p))
        h = ctypes.c_void_p()
        _check(lib().dfr_ensemble_create(n, descs, _stream(), ctypes.byref(h)))
        self._h = h
        self.members = [_Member(lib().dfr_ensemble_member(h, k), m["ne"], m["p"]) for k, m in enumerate(members)]

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            for m in self.members:
                m.close()
            lib().dfr_ensemble_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EpiEnsemble:
    def __init__(self, eg: EnsembleGrid, order, dt, q0s, startup_substeps=10, eps=1e-150, prec="fp64"):
        self.eg = eg
        n = len(eg.members)
        arr = (ctypes.c_void_p * n)(*[_dev(q).value for q in q0s])
        h = ctypes.c_void_p()
        _check(lib().epi_ensemble_create(eg.handle, int(order), float(dt), int(startup_substeps), arr, float(eps),
                                         _PREC[prec], ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().epi_ensemble_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dfr_ensemble_create(members):
    return EnsembleGrid(members)


def dfr_ensemble_autotune(eg: EnsembleGrid, prec="fp64"):
    _check(lib().dfr_ensemble_autotune(eg.handle, _PREC[prec]))
    return [dfr_get_krylov_tile(m) for m in eg.members]


ROUNDS = {"host": 0, "device": 1}


def dfr_ensemble_set_rounds(eg: EnsembleGrid, mode="host"):
    """Who drives the KIOPS rounds of epi_ensemble_step: "host" (the default)
    or "device" (a planner kernel, the round replayed from a HIP graph)."""
    _check(lib().dfr_ensemble_set_rounds(eg.handle, ROUNDS.get(mode, mode)))


def dfr_ensemble_round_counts(eg: EnsembleGrid):
    """(rounds with work, rounds launched) of the device-driven form so far."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().dfr_ensemble_round_counts(eg.handle, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def dfr_ensemble_timing_enable(eg: EnsembleGrid, enable=True):
    _check(lib().dfr_ensemble_timing_enable(eg.handle, int(bool(enable))))


def dfr_ensemble_timing_kinds(eg: EnsembleGrid, kinds=None):
    """Bracket only the given kinds (names or codes; None: all) with events."""
    mask = (1 << len(KERNEL_KINDS)) - 1 if kinds is None else sum(1 << KERNEL_KINDS.get(k, k) for k in kinds)
    _check(lib().dfr_ensemble_timing_kinds(eg.handle, mask))


def dfr_ensemble_timing_read(eg: EnsembleGrid, kind):
    """(summed ms, launches, nodes covered) of the batched launches of one kind."""
    ms, n, nodes = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(lib().dfr_ensemble_timing_read(eg.handle, KERNEL_KINDS.get(kind, kind), ctypes.byref(ms), ctypes.byref(n),
                                          ctypes.byref(nodes)))
    return ms.value, n.value, nodes.value


def epi_ensemble_create(eg, order, dt, q0s, startup_substeps=10, eps=1e-150, prec="fp64"):
    return EpiEnsemble(eg, order, dt, q0s, startup_substeps, eps, prec)


def epi_ensemble_step(eg: EnsembleGrid, x: EpiEnsemble, opts=None):
    """One batched EPI step of every member; returns per-member stats."""
    opts = opts or kiops_opts()
    n = len(eg.members)
    st = (KiopsStats * n)()
    _check(lib().epi_ensemble_step(eg.handle, x.handle, ctypes.byref(opts), st))
    return [v.as_dict() for v in st]


def epi_ensemble_get_state(x: EpiEnsemble, i, q=None):
    q = x.eg.members[i].empty() if q is None else q
    _check(lib().epi_ensemble_get_state(x.handle, int(i), _dev(q)))
    return q


def epi_get_state(st: EpiState, q=None):
    q = st.g.empty() if q is None else q
    _check(lib().epi_get_state(st.handle, _dev(q)))
    return q


def epi_num_steps(st: EpiState):
    return int(lib().epi_num_steps(st.handle))


@dataclass
class Loaded:
    path: str


def loaded_library():
    lib()
    return Loaded(LIB_PATH)
