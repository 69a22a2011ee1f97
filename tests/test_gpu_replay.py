"""GPU: decision record and replay of the Krylov controller (Sec. 4, Eq. 29;
kiops_replay in the C ABI), through the C ABI against the FP64 oracle.

The library's FP64 path records the same decisions as the oracle (Krylov
dimension and accept exactly, tau to rounding).  Replaying the oracle's
decisions, the complex-FP32 forms take the FP64 path exactly (the same
products, sub-steps and rejections), so their difference from the oracle is
the arithmetic of their products alone.

Tolerances:
  FP64, own or replayed decisions: 1e-11 (relative L2 per field, element-wise
      a decade above: tests/gpu_util.check_krylov), the plain-FP64 target.
  recorded decisions against the oracle's: the same number of attempts and,
      attempt by attempt, the same Krylov dimension and accept.  tau is
      recorded, not compared: a new tau is the old one times
      (gamma / omega)^(1/q), with omega the error estimate of the attempt's
      small exponential (a Taylor series here, Pade in the oracle), so tau
      differences start at ~1e-11 and compound over the accepted sub-steps
      (to ~1e-5 after thirty), and the last two sub-steps may split the
      remaining interval differently.  The phi-combination does not depend
      on the path of sub-steps, which is why the results still agree.
  FP32 forms on the FP64 path: 1e-5 (check_krylov), the bar of one FP32
      phi-combination elsewhere in the tests: a complex-FP32 product carries
      ~1e-6 relative error (unit roundoff 6e-8 times the flux cancellation),
      and the Krylov combination of products of one sweep does not amplify
      it beyond a decade (measured: 2.9e-6).  EPI steps on the replayed path:
      1e-8 in h in relative L2 and 1e-7 node by node against max h.  Only the
      Krylov products are FP32 (the remainders stay FP64), so a step carries
      the ~3e-6 relative error of its phi-combination times the size of the
      update against the state (~1e-4), about 3e-10, over eight steps a few
      1e-9 at most (measured: 5e-11 after one step, 1.7e-10 after eight).
      Left to their own controller the FP32 forms may take other decisions,
      and are held to 1e-6 in h, the accuracy the mixed form is held to
      (the mixed-precision tests).
"""

import numpy as np
import pytest

from oracle import epi as oepi
from oracle import kiops as okiops
from paper_2101_05617_amd import inputs
from tests.gpu_util import check_krylov, field_metrics, pair, record, small, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

C0 = inputs.WORKLOADS["c0_ne4_p4"]
C2 = inputs.WORKLOADS["c2_ne60_p6_jet"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    from paper_2101_05617_amd import dfrsw
    dfrsw.lib()
    yield


def _same_decisions(got, ref, key):
    assert len(got) == len(ref), (key, len(got), len(ref))
    worst = 0.0
    for k, (a, b) in enumerate(zip(got, ref)):
        assert a[1:] == (b[1], bool(b[2])), (key, k, a, b)
        worst = max(worst, abs(a[0] - b[0]) / abs(b[0]))
    record(f"{key}_tau_rel", worst)


def _substep_case():
    # a small Krylov cap forces sub-steps and rejections (as the KIOPS
    # sub-stepping parity test)
    w = small(C0, 3, 4, u_amp=1.0)
    G, D, Q = pair(w)
    return w, G, D, Q, G.rhs(Q), 40 * w.dt_nd


def test_fp64_records_the_oracle_decisions_and_replays_them():
    from paper_2101_05617_amd import dfrsw
    w, G, D, Q, F, tau = _substep_case()
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F], tol=1e-10, m_init=8, m_min=4, m_max=12)
    assert rst.n_substeps > 1 and rst.n_rejected > 0
    # record the library's own decisions
    rec = dfrsw.DecisionReplay(rec_cap=256)
    got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)],
                                     dfrsw.kiops_opts(tol=1e-10, m_init=8, m_min=4, m_max=12, replay=rec))
    _same_decisions(rec.recorded(), rst.decisions, "fp64_record")
    check_krylov(to_host(got), ref, G, 1e-11, "replay_fp64_own")
    # replay the oracle's decisions, recording at the same time
    rp = dfrsw.DecisionReplay(play=rst.decisions, rec_cap=256)
    got2, gst2 = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)],
                                       dfrsw.kiops_opts(tol=1e-10, m_init=8, m_min=4, m_max=12, replay=rp))
    assert rp.pos == len(rst.decisions)
    assert [d[1:] for d in rp.recorded()] == [(d[1], bool(d[2])) for d in rst.decisions]
    assert (gst2["n_matvec"], gst2["n_substeps"], gst2["n_rejected"]) == (rst.n_matvec, rst.n_substeps,
                                                                           rst.n_rejected)
    check_krylov(to_host(got2), ref, G, 1e-11, "replay_fp64_oracle_path")


@pytest.mark.parametrize("prec", ["fp32_jv", "fp32_jv_basis32"])
def test_fp32_forms_on_the_fp64_path(prec):
    # a tolerance of 1e-12 lies below the noise of a complex-FP32 product:
    # left to its own controller the FP32 form may take another path (its
    # attempts are recorded, not asserted); on the oracle's path its
    # difference from the FP64 result is that of its products' arithmetic
    from paper_2101_05617_amd import dfrsw
    w = small(C2, 3)
    G, D, Q = pair(w)
    F = G.rhs(Q)
    tau = w.dt_nd
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F], tol=1e-12, m_max=32)
    own = dfrsw.DecisionReplay(rec_cap=4096)
    try:
        dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)],
                              dfrsw.kiops_opts(tol=1e-12, m_max=32, max_attempts=200, replay=own), w.eps, prec)
        record(f"replay_{prec}_own_attempts", float(own.struct.n_rec))
    except dfrsw.DfrError as e:
        record(f"replay_{prec}_own_attempts", float(own.struct.n_rec))
        assert e.code == -6
    record("replay_fp64_attempts", float(len(rst.decisions)))
    rp = dfrsw.DecisionReplay(play=rst.decisions, rec_cap=0)
    got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)],
                                     dfrsw.kiops_opts(tol=1e-12, m_max=32, replay=rp), w.eps, prec)
    assert rp.pos == len(rst.decisions)
    assert (gst["n_matvec"], gst["n_substeps"], gst["n_rejected"]) == (rst.n_matvec, rst.n_substeps,
                                                                           rst.n_rejected)
    check_krylov(to_host(got), ref, G, 1e-5, f"replay_{prec}_oracle_path")


@pytest.mark.parametrize("prec", ["fp32_jv", "fp32_jv_basis32"])
def test_mixed_epi_steps_on_the_oracle_path(prec):
    # the jet (ne = 4, p = 6), EPI6: two start-up steps of two sub-steps, then
    # EPI6 steps; one replay object spans the KIOPS calls of all the steps
    from paper_2101_05617_amd import dfrsw
    w = small(C2, 4)
    G, D, Q = pair(w)
    kopt = dict(tol=w.tol, m_max=w.m_max)
    E = oepi.EPI(G.rhs, lambda q, v: G.jvp(q, v, 1e-150), w.order, w.dt_nd, Q, startup_substeps=2,
                 kiops_opts=kopt)
    steps = 8
    states = [E.step().copy() for _ in range(steps)]
    decisions = [d for st in E.stats for d in st.decisions]
    # the FP64 library records the same decisions over the same steps
    st64 = dfrsw.epi_create(D, w.order, w.dt_nd, to_dev(Q), startup_substeps=2)
    rec = dfrsw.DecisionReplay(rec_cap=4096)
    o64 = dfrsw.kiops_opts(tol=w.tol, m_max=w.m_max, replay=rec)
    for _ in range(steps):
        dfrsw.epi_step(D, st64, o64)
    _same_decisions(rec.recorded(), decisions, "epi6_fp64_record")
    # recorded only: the FP64 EPI bars belong to the parity tests (on this
    # near-balanced jet with EPI6 remainders the difference is ~1e-10)
    record("replay_epi6_fp64_l2", field_metrics(to_host(dfrsw.epi_get_state(st64)), E.q, G.ne, G.ns)["l2"])
    st64.close()
    # the FP32 form replays them, step by step against the oracle's states
    st = dfrsw.epi_create(D, w.order, w.dt_nd, to_dev(Q), startup_substeps=2, eps=w.eps, prec=prec)
    rp = dfrsw.DecisionReplay(play=decisions, rec_cap=0)
    o = dfrsw.kiops_opts(tol=w.tol, m_max=w.m_max, replay=rp)
    N = G.N
    for k in range(steps):
        dfrsw.epi_step(D, st, o)
        got = to_host(dfrsw.epi_get_state(st))
        ref = states[k]
        eh = np.linalg.norm(got[:N] - ref[:N]) / np.linalg.norm(ref[:N])
        ehm = np.max(np.abs(got[:N] - ref[:N])) / np.max(np.abs(ref[:N]))
        record(f"replay_epi6_{prec}_step{k + 1}_h", eh)
        record(f"replay_epi6_{prec}_step{k + 1}_h_max", ehm)
        assert eh < 1e-8 and ehm < 1e-7, (k, eh, ehm)
    assert rp.pos == len(decisions)
    st.close()


def test_decisions_that_cannot_be_taken_are_errors():
    from paper_2101_05617_amd import dfrsw
    w, G, D, Q, F, tau = _substep_case()

    def run(play):
        return dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)],
                                     dfrsw.kiops_opts(tol=1e-10, m_init=8, m_min=4, m_max=12,
                                                      replay=dfrsw.DecisionReplay(play=play, rec_cap=0)))
    cases = [([(tau / 4, 12, True)], "ran out"),
             ([(tau / 4, 13, True)], "outside"),
             ([(tau / 4, 12, False), (tau / 4, 8, True)], "outside"),
             ([(0.6 * tau, 12, True), (0.6 * tau, 12, True)], "passes the end"),
             ([(-tau, 12, True)], "positive")]
    for play, msg in cases:
        with pytest.raises(dfrsw.DfrError) as e:
            run(play)
        assert e.value.code == -6 and msg in str(e.value), (play, str(e.value))
    # the context still gives the oracle's result afterwards
    ref, _ = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F], tol=1e-10, m_init=8, m_min=4, m_max=12)
    got, _ = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)],
                                   dfrsw.kiops_opts(tol=1e-10, m_init=8, m_min=4, m_max=12))
    check_krylov(to_host(got), ref, G, 1e-11, "replay_errors_then_plain")


def test_ensemble_forms_refuse_replay():
    import torch
    from paper_2101_05617_amd import dfrsw
    from paper_2101_05617_amd.ensemble import Ensemble
    ws = [small(C0, 2, 3), small(C0, 2, 4)]
    opts = dfrsw.kiops_opts(tol=1e-10, m_max=24, replay=dfrsw.DecisionReplay(rec_cap=16))
    for form in ("batched", "concurrent"):
        ens = Ensemble(ws, prec="fp64", form=form, autotune=False)
        with pytest.raises(dfrsw.DfrError) as e:
            ens.step(opts)
        assert e.value.code == -1 and "single-grid" in str(e.value)
        ens.close()
    torch.cuda.synchronize()


def _clipped(tau_out, steps):
    """accepted (tau, m) sub-steps whose last one is clipped to end at tau_out,
    as the controller clips it."""
    out, t = [], 0.0
    for h, m, acc in steps:
        if t == tau_out:
            break
        tau = min(h, tau_out - t)
        out.append((tau, m, acc))
        if acc:
            t = tau_out if tau >= tau_out - t else t + tau
    assert t == tau_out
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32_jv", "fp32_jv_basis32"])
def test_paths_the_controller_does_not_take(prec):
    # both sides replay the same hand-made paths: uneven sub-steps; a
    # rejection continued at a larger m; a rejection followed by a smaller tau
    # on the same basis (an attempt that only recomputes the exponential); many
    # short sub-steps.  The library follows each path exactly and agrees with
    # the oracle at the FP64 bar, or at the FP32 bar for the FP32 forms.
    from paper_2101_05617_amd import dfrsw
    w = small(C0, 3, 4, u_amp=1.0)
    G, D, Q = pair(w)
    F = G.rhs(Q)
    rng = np.random.default_rng(7)
    b2 = 1e-3 * rng.standard_normal(3 * G.N)
    tau = 8 * w.dt_nd
    paths = {
        "uneven": _clipped(tau, [(0.5 * tau, 16, True), (0.125 * tau, 8, False), (0.125 * tau, 20, True),
                                 (tau, 16, True)]),
        "same_basis": _clipped(tau, [(tau, 20, False), (0.5 * tau, 20, True), (tau, 24, True)]),
        "many": _clipped(tau, [(tau / 6, 10, True)] * 7),
    }
    eps = 1e-150 if prec == "fp64" else C2.eps
    bar = 1e-11 if prec == "fp64" else 1e-5
    for name, path in paths.items():
        ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F, b2], tol=1e-10, m_max=32,
                                replay=okiops.DecisionReplay(path))
        rp = dfrsw.DecisionReplay(play=path, rec_cap=64)
        got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F), to_dev(b2)],
                                         dfrsw.kiops_opts(tol=1e-10, m_max=32, replay=rp), eps, prec)
        assert rp.pos == len(path), name
        assert [d[1:] for d in rp.recorded()] == [(m, bool(a)) for _, m, a in path], name
        assert (gst["n_matvec"], gst["n_substeps"], gst["n_rejected"], gst["n_expm"]) == \
            (rst.n_matvec, rst.n_substeps, rst.n_rejected, rst.n_expm), name
        check_krylov(to_host(got), ref, G, bar, f"replay_path_{name}_{prec}")
