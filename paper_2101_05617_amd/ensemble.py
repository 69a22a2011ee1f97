"""Ensembles of independent shallow-water integrations on one GPU.

Each member is a separate grid (its own ne, p and state).  Small members are
bound by kernel-launch and read-back latency: one member's Krylov iterations
leave most of the GPU idle.  The batched form gives every member a context
on a stream of its own and advances all of them together with the library's
`epi_ensemble_step`: host worker threads (native, inside the library) drive
different members at once, so their kernels and read-backs overlap.

Argument marshalling only; every computation runs in the HIP library.
"""
from __future__ import annotations

from . import dfrsw, inputs


class Ensemble:
    """Members built from `inputs.Workload`s; `prec` is "fp64" or "fp32_jv".

    own_streams: give every member its own stream (the batched form); with
    False all members use the current stream (the one-after-another form).
    autotune: pick each member's tiles by timing (dfr_autotune)."""

    def __init__(self, workloads, prec="fp32_jv", own_streams=True, autotune=True, frames=None):
        import torch
        self.prec = prec
        self.members = []
        for k, w in enumerate(workloads):
            s = torch.cuda.Stream() if own_streams else torch.cuda.current_stream()
            with torch.cuda.stream(s):
                g = dfrsw.Grid(w.ne, w.p, *w.constants())
                if autotune:
                    dfrsw.dfr_autotune(g, prec)
                P, B1, B2 = frames[k] if frames is not None else g.node_frames()
                Q, hB = inputs.initial_state(w, P, B1, B2)
                if hB is not None:
                    raise ValueError("ensemble members without orography only")
                q0 = torch.from_numpy(Q).cuda()
                eps = w.eps if prec == "fp32_jv" else 1e-150
                st = dfrsw.epi_create(g, w.order, w.dt_nd, q0, startup_substeps=w.startup_substeps, eps=eps,
                                      prec=prec)
            self.members.append((w, s, g, st))
        torch.cuda.synchronize()

    @property
    def grids(self):
        return [m[2] for m in self.members]

    @property
    def states(self):
        return [m[3] for m in self.members]

    def step(self, opts, n_workers=8):
        """One step of every member at once (the batched form)."""
        return dfrsw.epi_ensemble_step(self.grids, self.states, opts, n_workers)

    def step_sequential(self, opts):
        """One step of every member, one member after another."""
        return [dfrsw.epi_step(g, st, opts) for _, _, g, st in self.members]

    def state(self, k):
        import torch
        w, s, g, st = self.members[k]
        with torch.cuda.stream(s):
            q = dfrsw.epi_get_state(st)
        torch.cuda.synchronize()
        return q.cpu().numpy()

    def close(self):
        import torch
        torch.cuda.synchronize()
        for _, _, g, st in self.members:
            st.close()
            g.close()
        self.members = []
