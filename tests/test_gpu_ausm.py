"""GPU parity of the AUSM interface flux (App. D, Eqs. 137-143): the HIP
library with dfr_set_riemann(DFR_AUSM) against the oracle's AUSM
discretisation on identical seeded inputs, through the C ABI.

The bars are those of the Rusanov parity tests and for the same reasons
(same formulas in FP64 on both sides, different operation order, FMA
contraction and division / square-root sequences): FP64 J v 1e-12, F(q)
max(1e-11, 4 x the oracle's own 1-ulp condition floor), complex-FP32 J v
2e-5, KIOPS and EPI 1e-11 with identical controller decisions, each
applied per field to the relative L2 and the element-wise difference, over
all nodes and over the panel-edge elements (tests/gpu_util.check_fields).
The seeded
states keep every Froude number far from the split-function breakpoints
|M| = 1 and the split Froude number far from zero, so both sides take the
same branches."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import epi as oepi
from oracle import kiops as okiops
from paper_2101_05617_amd import inputs
from tests.gpu_util import check_fields, check_krylov, check_rhs, pair, rel_fields, small, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

C0 = inputs.WORKLOADS["c0_ne4_p4"]
C1 = inputs.WORKLOADS["c1_ne30_p5"]

GRIDS = [(1, 1), (2, 2), (3, 4), (4, 4), (2, 5), (3, 6), (2, 7)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    from paper_2101_05617_amd import dfrsw
    dfrsw.lib()


@pytest.mark.parametrize("ne,p", GRIDS)
def test_ausm_rhs_and_jvp_parity(ne, p):
    w = small(C0, ne, p, u_amp=2.0)
    G, D, Q = pair(w, riemann="ausm")
    from paper_2101_05617_amd import dfrsw
    assert dfrsw.dfr_get_riemann(D) == "ausm"
    got = to_host(dfrsw.dfr_rhs(D, to_dev(Q)))
    check_rhs(got, G, Q, f"ausm_rhs_fp64_ne{ne}_p{p}")
    V = inputs.random_direction(3 * G.N, 300 + ne * 10 + p)
    got = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-150, "fp64"))
    check_fields(got, G.jvp(Q, V, 1e-150), G, 1e-12, f"ausm_jvp_fp64_ne{ne}_p{p}")


@pytest.mark.parametrize("ne,p", [(4, 4), (3, 6)])
def test_ausm_jvp_fp32_parity(ne, p):
    w = small(C0, ne, p, u_amp=2.0)
    G, D, Q = pair(w, riemann="ausm")
    from paper_2101_05617_amd import dfrsw
    V = inputs.random_direction(3 * G.N, 5)
    got = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-20, "fp32_jv"))
    check_fields(got, G.jvp(Q, V, 1e-150), G, 2e-5, f"ausm_jvp_fp32_ne{ne}_p{p}")


def test_ausm_switch_is_per_context_and_reversible():
    G, D, Q = pair(small(C0, 3, 4, u_amp=2.0))
    from paper_2101_05617_amd import dfrsw
    q = to_dev(Q)
    a = to_host(dfrsw.dfr_rhs(D, q))
    dfrsw.dfr_set_riemann(D, "ausm")
    b = to_host(dfrsw.dfr_rhs(D, q))
    dfrsw.dfr_set_riemann(D, "rusanov")
    c = to_host(dfrsw.dfr_rhs(D, q))
    assert np.array_equal(a, c)
    assert rel_fields(b, a, G.N) > 1e-8
    assert dfrsw.lib().dfr_set_riemann(D.handle, 7) == -1   # DFR_E_INVAL, setting unchanged
    assert dfrsw.dfr_get_riemann(D) == "rusanov"


def test_ausm_mass_conservation_on_gpu():
    G, D, Q = pair(small(C0, 3, 5, u_amp=3.0, h_amp=0.05), riemann="ausm")
    from paper_2101_05617_amd import dfrsw
    wq = G.mass_weights()
    F = to_host(dfrsw.dfr_rhs(D, to_dev(Q)))
    V = inputs.random_direction(3 * G.N, 9)
    J = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V)))
    assert abs(wq @ F[: G.N]) < 1e-14 * (wq @ Q[: G.N])
    assert abs(wq @ J[: G.N]) < 1e-14 * (wq @ np.abs(J[: G.N]))


def test_ausm_kiops_parity():
    w = small(C0, 3, 4, u_amp=1.0)
    G, D, Q = pair(w, riemann="ausm")
    from paper_2101_05617_amd import dfrsw
    F = G.rhs(Q)
    rng = np.random.default_rng(3)
    bs = [None, F, 1e-3 * rng.standard_normal(3 * G.N)]
    tau = 4 * w.dt_nd
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v, 1e-150), bs, tol=1e-12, m_max=32)
    got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None if b is None else to_dev(b) for b in bs],
                                     dfrsw.kiops_opts(tol=1e-12, m_max=32), 1e-150, "fp64")
    assert (gst["n_substeps"], gst["n_rejected"], gst["m_last"], gst["n_matvec"]) == \
        (rst.n_substeps, rst.n_rejected, rst.m_last, rst.n_matvec)
    check_krylov(to_host(got), ref, G, 1e-11, "ausm_kiops")


@pytest.mark.parametrize("w,steps,s", [(C0, 4, 3), (replace(small(C0, 3, 5), order=5), 5, 2)])
def test_ausm_epi_parity_every_step(w, steps, s):
    G, D, Q = pair(w, riemann="ausm")
    from paper_2101_05617_amd import dfrsw
    E = oepi.EPI(G.rhs, lambda q, v: G.jvp(q, v, 1e-150), w.order, w.dt_nd, Q, startup_substeps=s,
                 kiops_opts=dict(tol=w.tol, m_max=w.m_max))
    st = dfrsw.epi_create(D, w.order, w.dt_nd, to_dev(Q), startup_substeps=s)
    for k in range(steps):
        E.step()
        dfrsw.epi_step(D, st, dfrsw.kiops_opts(tol=w.tol, m_max=w.m_max))
        check_krylov(to_host(dfrsw.epi_get_state(st)), E.q, G, 1e-11, f"ausm_epi{w.order}_ne{w.ne}_p{w.p}_step{k + 1}")


def test_ausm_c1_full_size_rhs_jvp_parity():
    # ne = 30, p = 5 (194,400 nodes): every element of F and J v with AUSM
    G, D, Q = pair(C1, riemann="ausm")
    from paper_2101_05617_amd import dfrsw
    check_rhs(to_host(dfrsw.dfr_rhs(D, to_dev(Q))), G, Q, "ausm_c1_rhs_fp64")
    V = inputs.random_direction(3 * G.N, 32)
    check_fields(to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V))), G.jvp(Q, V), G, 1e-12,
                 "ausm_c1_jvp_fp64")


def test_batched_ensemble_rejects_ausm_members():
    from paper_2101_05617_amd import dfrsw
    torch = torch_dev()
    ms = inputs.ensemble_members(2)
    eg = dfrsw.EnsembleGrid([dict(ne=2, p=m.p, radius=c[0], omega=c[1], gravity=c[2])
                             for m in ms for c in [m.constants()]])
    try:
        dfrsw.dfr_set_riemann(eg.members[1], "ausm")
        q0 = []
        for mb in eg.members:   # fluid at rest, H = 1
            q = torch.zeros(3 * mb.N, dtype=torch.float64, device="cuda")
            q[: mb.N] = 1.0
            q0.append(q)
        with pytest.raises(dfrsw.DfrError) as e:
            x = dfrsw.epi_ensemble_create(eg, 4, ms[0].dt_nd, q0, startup_substeps=2)
            try:
                dfrsw.epi_ensemble_step(eg, x, dfrsw.kiops_opts(tol=1e-10, m_max=16))
            finally:
                x.close()
        assert e.value.code == -1 and "member 1" in str(e.value)
    finally:
        torch.cuda.synchronize()
        eg.close()
