"""The mixed form with an FP32 Krylov basis (DFR_FP32_JV_BASIS32): complex-
FP32 products and basis vectors stored in FP32, with inner products, norms,
the Hessenberg, the small exponential, the combination and the EPI update in
FP64 -- against the FP64 oracle on the jet and mountain workloads.

Bars: the mixed form's accuracy target, 1e-6 relative L2 in h after every
EPI step and 1e-4 on every field; one phi-combination within 1e-5 of the
FP64 result (FP32 storage rounds each basis vector by 6e-8 relative, and the
combination of up to 64 of them stays within the Krylov tolerance's reach)."""
import numpy as np
import pytest

from oracle import epi as oepi
from oracle import kiops as okiops
from paper_2101_05617_amd import inputs
from tests.gpu_util import pair, record, rel_fields, small, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

C2 = inputs.WORKLOADS["c2_ne60_p6_jet"]
C4 = inputs.WORKLOADS["c4_ne120_p6_mountain"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    from paper_2101_05617_amd import dfrsw
    dfrsw.lib()


def _h_error(got, ref, N):
    return np.linalg.norm(got[:N] - ref[:N]) / np.linalg.norm(ref[:N])


def test_basis32_kiops_against_fp64():
    w = small(C2, 3)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    F = G.rhs(Q)
    tau = w.dt_nd
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F], tol=1e-10, m_max=64)
    got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)], dfrsw.kiops_opts(tol=1e-10, m_max=64),
                                     w.eps, "fp32_jv_basis32")
    err = np.linalg.norm(to_host(got) - ref) / np.linalg.norm(ref)
    record("basis32_kiops_jet_ne3", err)
    record("basis32_kiops_jet_ne3_matvec", gst["n_matvec"])
    assert err < 1e-5


@pytest.mark.parametrize("w", [small(C2, 4), small(C4, 4)], ids=["jet", "mountain"])
def test_basis32_epi6_against_fp64_oracle(w):
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    dfrsw.dfr_autotune(D, "fp32_jv_basis32")
    kopt = dict(tol=w.tol, m_max=w.m_max)
    E = oepi.EPI(G.rhs, lambda q, v: G.jvp(q, v, 1e-150), w.order, w.dt_nd, Q, startup_substeps=2,
                 kiops_opts=kopt)
    st = dfrsw.epi_create(D, w.order, w.dt_nd, to_dev(Q), startup_substeps=2, eps=1e-20, prec="fp32_jv_basis32")
    for k in range(7):
        E.step()
        dfrsw.epi_step(D, st, dfrsw.kiops_opts(**kopt))
        got = to_host(dfrsw.epi_get_state(st))
        eh, ea = _h_error(got, E.q, G.N), rel_fields(got, E.q, G.N)
        record(f"basis32_epi6_{w.kind}_ne4_step{k + 1}_h", eh)
        assert eh < 1e-6 and ea < 1e-4, (k, eh, ea)


def test_basis32_product_alone_equals_fp32_form():
    # outside KIOPS the basis precision does not enter: dfr_jvp_complex_step
    # gives the FP32 form's result bit for bit
    G, D, Q = pair(small(C2, 3))
    from paper_2101_05617_amd import dfrsw
    V = inputs.random_direction(3 * G.N, 77)
    a = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-20, "fp32_jv"))
    b = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-20, "fp32_jv_basis32"))
    assert np.array_equal(a, b)


def test_batched_ensemble_rejects_fp32_basis():
    from paper_2101_05617_amd import dfrsw
    torch = torch_dev()
    ms = inputs.ensemble_members(2)
    eg = dfrsw.EnsembleGrid([dict(ne=2, p=m.p, radius=c[0], omega=c[1], gravity=c[2])
                             for m in ms for c in [m.constants()]])
    try:
        q0 = []
        for mb in eg.members:
            q = torch.zeros(3 * mb.N, dtype=torch.float64, device="cuda")
            q[: mb.N] = 1.0
            q0.append(q)
        with pytest.raises(dfrsw.DfrError) as e:
            dfrsw.epi_ensemble_create(eg, 4, ms[0].dt_nd, q0, startup_substeps=2, eps=1e-20, prec="fp32_jv_basis32")
        assert e.value.code == -1
    finally:
        torch.cuda.synchronize()
        eg.close()
