"""Ensembles of independent shallow-water integrations on one GPU.

Each member is a separate grid (its own ne, p and state).  Small members are
bound by kernel-launch and read-back latency: one member's Krylov iterations
leave most of the GPU idle.  Three ways to run an ensemble:

  "batched"     the library's batched form (dfr_ensemble_create /
                epi_ensemble_step): one kernel launch per operation for all
                members, each member with its own Krylov controller;
  "concurrent"  one context per member on its own stream, members advanced by
                host threads inside the library (epi_step_concurrent);
  "sequential"  one member after another (epi_step).

Argument marshalling only; every computation runs in the HIP library.
"""
from __future__ import annotations

from . import dfrsw, inputs


class Ensemble:
    """Members built from `inputs.Workload`s (same order, dt and start-up for
    the batched form); `prec` is "fp64", "fp32_jv" or "fp32_jv_basis32".  autotune: pick each
    member's tiles by timing (dfr_autotune).  frames: optional per-member
    (P, B1, B2) node frames for the initial states (default: the library's).
    rounds: who drives the batched form's KIOPS rounds, "device" or "host"
    (dfr_ensemble_set_rounds)."""

    def __init__(self, workloads, prec="fp32_jv", form="batched", autotune=True, frames=None, rounds="host"):
        import torch
        self.prec, self.form = prec, form
        self.workloads = list(workloads)
        self.grids, self.streams = [], []
        self.eg = None
        if form == "batched":
            self.eg = dfrsw.dfr_ensemble_create([dict(ne=w.ne, p=w.p, radius=c[0], omega=c[1], gravity=c[2])
                                                 for w in self.workloads for c in [w.constants()]])
            self.grids = self.eg.members
            dfrsw.dfr_ensemble_set_rounds(self.eg, rounds)
        else:
            for w in self.workloads:
                s = torch.cuda.Stream() if form == "concurrent" else torch.cuda.current_stream()
                with torch.cuda.stream(s):
                    self.grids.append(dfrsw.Grid(w.ne, w.p, *w.constants()))
                self.streams.append(s)
        if autotune and form == "batched":
            dfrsw.dfr_ensemble_autotune(self.eg, prec)
        q0s = []
        for k, (w, g) in enumerate(zip(self.workloads, self.grids)):
            if autotune and form != "batched":
                dfrsw.dfr_autotune(g, prec)
            P, B1, B2 = frames[k] if frames is not None else g.node_frames()
            Q, hB = inputs.initial_state(w, P, B1, B2)
            if hB is not None:
                raise ValueError("ensemble members without orography only")
            q0s.append(torch.from_numpy(Q).cuda())
        torch.cuda.synchronize()
        self.eps = [w.eps if prec != "fp64" else 1e-150 for w in self.workloads]
        if form == "batched":
            w0 = self.workloads[0]
            self.x = dfrsw.epi_ensemble_create(self.eg, w0.order, w0.dt_nd, q0s, startup_substeps=w0.startup_substeps,
                                               eps=self.eps[0], prec=prec)
            self.states = None
        else:
            self.states = []
            for k, (w, g) in enumerate(zip(self.workloads, self.grids)):
                with torch.cuda.stream(self.streams[k]):
                    self.states.append(dfrsw.epi_create(g, w.order, w.dt_nd, q0s[k],
                                                        startup_substeps=w.startup_substeps, eps=self.eps[k],
                                                        prec=prec))
        torch.cuda.synchronize()
        del q0s

    def step(self, opts, n_workers=8):
        """One step of every member; per-member KIOPS statistics."""
        if self.form == "batched":
            return dfrsw.epi_ensemble_step(self.eg, self.x, opts)
        if self.form == "concurrent":
            return dfrsw.epi_step_concurrent(self.grids, self.states, opts, n_workers)
        return [dfrsw.epi_step(g, st, opts) for g, st in zip(self.grids, self.states)]

    def state(self, k):
        import torch
        torch.cuda.synchronize()
        if self.form == "batched":
            q = dfrsw.epi_ensemble_get_state(self.x, k)
        else:
            with torch.cuda.stream(self.streams[k]):
                q = dfrsw.epi_get_state(self.states[k])
        torch.cuda.synchronize()
        return q.cpu().numpy()

    def close(self):
        import torch
        torch.cuda.synchronize()
        if self.form == "batched":
            self.x.close()
            self.eg.close()
        else:
            for st in self.states:
                st.close()
            for g in self.grids:
                g.close()
        self.grids, self.states = [], []
