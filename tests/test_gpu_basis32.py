"""The mixed form with an FP32 Krylov basis (DFR_FP32_JV_BASIS32): complex-
FP32 products and basis vectors stored in FP32, with inner products, norms,
the Hessenberg, the small exponential, the combination and the EPI update in
FP64 -- against the FP64 oracle on the jet and mountain workloads.

Bars: the mixed form's accuracy target, 1e-6 relative L2 in h after every
EPI step (and 1e-6 element-wise in h, against max h) and 1e-4 on every
field in every measure of tests/gpu_util.check_fields; one phi-combination
within 1e-5 of the FP64 result (1e-4 element-wise, check_krylov) (FP32 storage rounds each basis vector by 6e-8 relative, and the
combination of up to 64 of them stays within the Krylov tolerance's reach)."""
import numpy as np
import pytest

from oracle import epi as oepi
from oracle import kiops as okiops
from paper_2101_05617_amd import inputs
from tests.gpu_util import check_fields, check_krylov, pair, record, small, to_dev, to_host, torch_dev

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


def _h_max_error(got, ref, N):
    return np.max(np.abs(got[:N] - ref[:N])) / np.max(np.abs(ref[:N]))


def test_basis32_kiops_against_fp64():
    w = small(C2, 3)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    F = G.rhs(Q)
    tau = w.dt_nd
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F], tol=1e-10, m_max=64)
    got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)], dfrsw.kiops_opts(tol=1e-10, m_max=64),
                                     w.eps, "fp32_jv_basis32")
    record("basis32_kiops_jet_ne3_matvec", gst["n_matvec"])
    check_krylov(to_host(got), ref, G, 1e-5, "basis32_kiops_jet_ne3")


def test_c4_full_size_kiops_fp64_and_basis32():
    # ne = 120, p = 6 mountain (12,700,800 unknowns): one phi_1 product in the
    # autotuned tiles of each form, FP64 (identical decisions, 1e-11) and
    # with FP32 products and an FP32 basis (1e-5); tau = dt/4 bounds the
    # oracle's run
    G, D, Q = pair(C4)
    from paper_2101_05617_amd import dfrsw
    F = G.rhs(Q)
    tau = C4.dt_nd / 4
    opts = dfrsw.kiops_opts(tol=C4.tol, m_max=C4.m_max)
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F], tol=C4.tol, m_max=C4.m_max)
    dfrsw.dfr_autotune(D, "fp64")
    got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)], opts)
    assert (gst["n_substeps"], gst["n_rejected"], gst["n_matvec"]) == (rst.n_substeps, rst.n_rejected, rst.n_matvec)
    check_krylov(to_host(got), ref, G, 1e-11, "kiops_c4_full_fp64")
    dfrsw.dfr_autotune(D, "fp32_jv_basis32")
    got32, _ = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)], opts, 1e-20, "fp32_jv_basis32")
    check_krylov(to_host(got32), ref, G, 1e-5, "kiops_c4_full_basis32")


def test_fp32_forms_reject_an_eps_that_underflows():
    # an FP64 step (1e-150) would zero the FP32 imaginary parts of unit-norm
    # Krylov vectors: every FP32 entry point refuses eps < DFR_FP32_EPS_MIN
    from paper_2101_05617_amd import dfrsw
    G, D, Q = pair(small(C2, 2, 3))
    q, F = to_dev(Q), to_dev(G.rhs(Q))
    opts = dfrsw.kiops_opts(tol=1e-8, m_max=16)
    for prec in ("fp32_jv", "fp32_jv_basis32"):
        with pytest.raises(dfrsw.DfrError) as e:
            dfrsw.dfr_jvp_complex_step(D, q, F, 1e-150, prec)
        assert e.value.code == -1 and "DFR_FP32_EPS_MIN" in str(e.value)
        with pytest.raises(dfrsw.DfrError) as e:
            dfrsw.kiops_phi_apply(D, q, 0.01, [None, F], opts, 1e-31, prec)
        assert e.value.code == -1
        with pytest.raises(dfrsw.DfrError) as e:
            dfrsw.epi_create(D, 4, 0.01, q, startup_substeps=1, eps=1e-150, prec=prec)
        assert e.value.code == -1
        # the bound itself is accepted, and FP64 takes any positive eps
        dfrsw.dfr_jvp_complex_step(D, q, F, 1e-30, prec)
    dfrsw.dfr_jvp_complex_step(D, q, F, 1e-300, "fp64")
    dfrsw.dfr_sync(D)


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
        eh, ehm = _h_error(got, E.q, G.N), _h_max_error(got, E.q, G.N)
        record(f"basis32_epi6_{w.kind}_ne4_step{k + 1}_h", eh)
        record(f"basis32_epi6_{w.kind}_ne4_step{k + 1}_h_max", ehm)
        assert eh < 1e-6 and ehm < 1e-6, (k, eh, ehm)
        check_fields(got, E.q, G, 1e-4, f"basis32_epi6_{w.kind}_ne4_step{k + 1}_all")


def test_basis32_product_alone_equals_fp32_form():
    # outside KIOPS the basis precision does not enter: dfr_jvp_complex_step
    # gives the FP32 form's result bit for bit
    G, D, Q = pair(small(C2, 3))
    from paper_2101_05617_amd import dfrsw
    V = inputs.random_direction(3 * G.N, 77)
    a = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-20, "fp32_jv"))
    b = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-20, "fp32_jv_basis32"))
    assert np.array_equal(a, b)


def test_batched_ensemble_fp32_basis_matches_members_run_alone():
    # the batched form with FP32 products and FP32 bases against the same
    # precision member by member (same tiles, same decisions), and against
    # plain FP64 member by member
    import torch
    from dataclasses import replace
    from paper_2101_05617_amd.ensemble import Ensemble
    ws = [small(C2, 2, 4), small(C2, 3, 5), small(C2, 2, 6)]
    ws = [replace(w, order=4, dt_s=900.0, m_max=32) for w in ws]
    from paper_2101_05617_amd import dfrsw
    opts = dfrsw.kiops_opts(tol=1e-10, m_max=32)
    ref64 = Ensemble(ws, prec="fp64", form="sequential", autotune=False)
    seq = Ensemble(ws, prec="fp32_jv_basis32", form="sequential", autotune=False)
    bat = Ensemble(ws, prec="fp32_jv_basis32", form="batched", autotune=False, rounds="host")
    try:
        for _ in range(5):
            ref64.step(opts)
            ss = seq.step(opts)
            sb = bat.step(opts)
            assert [x["n_matvec"] for x in sb] == [x["n_matvec"] for x in ss]
        for k in range(len(ws)):
            a, b, c = seq.state(k), bat.state(k), ref64.state(k)
            N = len(a) // 3
            e_seq = np.linalg.norm(b[:N] - a[:N]) / np.linalg.norm(a[:N])
            e_64 = np.linalg.norm(b[:N] - c[:N]) / np.linalg.norm(c[:N])
            record(f"ensemble_basis32_member{k}_vs_alone_h", e_seq)
            record(f"ensemble_basis32_member{k}_vs_fp64_h", e_64)
            assert np.array_equal(a, b) and e_64 < 1e-6, (k, e_seq, e_64)
    finally:
        for z in (ref64, seq, bat):
            z.close()
        torch.cuda.synchronize()
