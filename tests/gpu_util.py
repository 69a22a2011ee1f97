"""Helpers shared by the GPU tests: paired oracle / library grids on the same
seeded inputs.  Inputs are built with the oracle's geometry, never the
library's, so no expected value depends on the code under test."""
from dataclasses import replace

import numpy as np

import oracle
from paper_2101_05617_amd import inputs


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch


def pair(w, hB=None, rotation=inputs.ROTATION, riemann="rusanov"):
    """(oracle grid, library grid, Q as numpy) for workload w, both with the
    given interface flux."""
    from paper_2101_05617_amd import dfrsw
    G = oracle.OracleGrid(w.ne, w.ns, *w.constants(), rotation=rotation, riemann=riemann)
    P, B1, B2 = G.node_frames()
    Q, hb = inputs.initial_state(w, P, B1, B2)
    if hB is None:
        hB = hb
    if hB is not None:
        G = oracle.OracleGrid(w.ne, w.ns, *w.constants(), rotation=rotation, hB=hB, riemann=riemann)
    D = dfrsw.Grid(w.ne, w.p, *w.constants(), rotation=rotation, hB=hB)
    if riemann != "rusanov":
        dfrsw.dfr_set_riemann(D, riemann)
    return G, D, Q


def to_dev(x):
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def to_host(t):
    torch = torch_dev()
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_fields(a, b, N):
    """max over the three fields of ||a_f - b_f||_2 / ||b_f||_2."""
    out = 0.0
    for f in range(3):
        sl = slice(f * N, (f + 1) * N)
        den = np.linalg.norm(b[sl])
        num = np.linalg.norm(a[sl] - b[sl])
        out = max(out, num / den if den > 0 else num)
    return out


def small(w, ne, p=None, **kw):
    return replace(w, ne=ne, p=w.p if p is None else p, **kw)


def rhs_rounding_floor(G, Q):
    """Relative change of the oracle's F (max over fields) when the input is
    perturbed by one unit roundoff at random: the condition of F at Q.  For a
    near-balanced state F is a small residual of much larger flux terms, and
    any two correct FP64 evaluations differ by about this much."""
    rng = np.random.default_rng(12345)
    Qp = Q * (1.0 + 2.0 ** -52 * rng.standard_normal(Q.shape))
    return rel_fields(G.rhs(Qp), G.rhs(Q), G.N)


def rhs_bar(G, Q):
    return max(1e-11, 4.0 * rhs_rounding_floor(G, Q))


METRICS = {}


def record(name, value):
    METRICS[name] = float(value)


def dump_metrics(path):
    import json
    import os
    if os.path.isdir(os.path.dirname(path) or "."):
        with open(path, "w") as f:
            json.dump(METRICS, f, indent=1, sort_keys=True)
