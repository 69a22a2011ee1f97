"""Accuracy of the full-size workloads against the FP64 oracle: the errors the
benchmark states for the mixed-precision forms rest on these.

  * Ensemble: the two smallest members of the 64-member workload (ne = 8,
    p = 4 and p = 5) over one simulated day (96 EPI4 steps of 900 s), run
    as a batched ensemble in plain FP64 (KIOPS tol 1e-10) and in the mixed
    form (complex-FP32 products, FP32 Krylov basis, tol 1e-6), against the
    oracle's FP64 run at tol 1e-10.  Bars: plain FP64 1e-11 per field (L2;
    element-wise a decade above, check_krylov); the mixed form 1e-6 relative
    L2 in h (the stated error) and 1e-6 element-wise in h against max h.
  * ne = 120, p = 6 mountain (4,233,600 nodes, 12.7 M unknowns): the first
    two EPI6 steps (EPI2 start-up with two sub-steps each), the oracle with
    the host's threads, against plain FP64 (tol 1e-10: 1e-11 per field) and
    the mixed form with an FP32 basis at tol 1e-10 and at tol 1e-6 (1e-6 in
    h, L2 and element-wise).
The measured errors are recorded in the metrics file of the GPU tests."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from oracle import epi as oepi
from paper_2101_05617_amd import inputs
from tests.gpu_util import check_krylov, record, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    from paper_2101_05617_amd import dfrsw
    dfrsw.lib()


def _h_errors(got, ref, N):
    return (np.linalg.norm(got[:N] - ref[:N]) / np.linalg.norm(ref[:N]),
            np.max(np.abs(got[:N] - ref[:N])) / np.max(np.abs(ref[:N])))


def test_smallest_ensemble_members_over_one_day_against_the_oracle():
    import torch
    from paper_2101_05617_amd import dfrsw
    from paper_2101_05617_amd.ensemble import Ensemble
    members = inputs.ensemble_members(64)
    order = sorted(range(len(members)), key=lambda k: (members[k].n_nodes, k))
    pick = [order[0]] + [k for k in order if members[k].p != members[order[0]].p][:1]
    ws = [members[k] for k in pick]
    day = int(round(86400.0 / ws[0].dt_s))
    grids = [oracle.OracleGrid(w.ne, w.ns, *w.constants()) for w in ws]
    frames = [G.node_frames() for G in grids]
    refs = []
    for w, G, fr in zip(ws, grids, frames):
        Q, _ = inputs.initial_state(w, *fr)
        E = oepi.EPI(G.rhs, lambda a, b, G=G: G.jvp(a, b), w.order, w.dt_nd, Q,
                     startup_substeps=w.startup_substeps, kiops_opts=dict(tol=w.tol, m_max=w.m_max))
        for _ in range(day):
            E.step()
        refs.append(E.q.copy())
    runs = {}
    for name, prec, tol in (("fp64", "fp64", 1e-10), ("mixed", "fp32_jv_basis32", 1e-6)):
        ens = Ensemble(ws, prec=prec, form="batched", autotune=False, frames=frames)
        opts = dfrsw.kiops_opts(tol=tol, m_max=ws[0].m_max)
        for _ in range(day):
            ens.step(opts)
        runs[name] = [ens.state(k) for k in range(len(ws))]
        ens.close()
        torch.cuda.synchronize()
    for k, (w, G) in enumerate(zip(ws, grids)):
        tag = f"day_member{pick[k]}_ne{w.ne}_p{w.p}"
        check_krylov(runs["fp64"][k], refs[k], G, 1e-11, f"{tag}_fp64")
        eh, ehm = _h_errors(runs["mixed"][k], refs[k], G.N)
        record(f"{tag}_mixed_h", eh)
        record(f"{tag}_mixed_h_max", ehm)
        assert eh < 1e-6 and ehm < 1e-6, (tag, eh, ehm)


def test_c4_two_step_subset_against_the_oracle():
    import torch
    from paper_2101_05617_amd import dfrsw
    w = replace(inputs.WORKLOADS["c4_ne120_p6_mountain"], startup_substeps=2)
    G0 = oracle.OracleGrid(w.ne, w.ns, *w.constants())
    P, B1, B2 = G0.node_frames()
    del G0
    Q, hB = inputs.initial_state(w, P, B1, B2)
    del P, B1, B2
    G = oracle.OracleGrid(w.ne, w.ns, *w.constants(), hB=hB)
    E = oepi.EPI(G.rhs, lambda a, b: G.jvp(a, b), w.order, w.dt_nd, Q, startup_substeps=w.startup_substeps,
                 kiops_opts=dict(tol=w.tol, m_max=w.m_max))
    for _ in range(2):
        E.step()
    ref = E.q.copy()
    del E
    D = dfrsw.Grid(w.ne, w.p, *w.constants(), hB=hB)
    for name, prec, eps, tol in (("fp64", "fp64", 1e-150, 1e-10), ("mixed", "fp32_jv_basis32", 1e-20, 1e-10),
                                 ("mixed_tol1e-6", "fp32_jv_basis32", 1e-20, 1e-6)):
        dfrsw.dfr_autotune(D, prec)
        st = dfrsw.epi_create(D, w.order, w.dt_nd, to_dev(Q), startup_substeps=w.startup_substeps, eps=eps, prec=prec)
        for _ in range(2):
            dfrsw.epi_step(D, st, dfrsw.kiops_opts(tol=tol, m_max=w.m_max))
        got = to_host(dfrsw.epi_get_state(st))
        st.close()
        if name == "fp64":
            check_krylov(got, ref, G, 1e-11, "c4_two_steps_fp64")
        else:
            eh, ehm = _h_errors(got, ref, G.N)
            record(f"c4_two_steps_{name}_h", eh)
            record(f"c4_two_steps_{name}_h_max", ehm)
            assert eh < 1e-6 and ehm < 1e-6, (name, eh, ehm)
        del got
    D.close()
    torch.cuda.synchronize()
