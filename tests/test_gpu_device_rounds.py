"""The batched ensemble's KIOPS rounds driven from the device (a planner
kernel takes every member's controller decisions, K4-K7 of the Krylov
evaluation of Eq. 29, and writes the round's call tables; the round is
replayed from a HIP graph) against the same rounds driven from the host.

Each member takes the same operations in both forms, so the controller's
decisions (sub-steps, rejections, Krylov size, products, exponentials, happy
flag) must be identical, member by member and step by step.  The decisions
use log and pow, which the device computes with its own math library: a
last-bit difference there can move a sub-step length by an ulp, so the
states are held to 1e-13 relative per field, element-wise (a decade of
rounding above the 1e-16 of such a move, three decades below the 1e-10 of a
wrong decision or a wrong operand), and whether they came out bit-identical
is recorded.  Against the oracle the device form meets the Krylov bars of the
other ensemble tests (1e-11 L2, 1e-10 element-wise).

Covered: FP64 and the mixed form (complex-FP32 products, FP32 basis),
members of four different p (four product launches per round), rejections
and Krylov-size changes (a tolerance the first Krylov size misses), happy
breakdowns in the start-up, non-convergence naming the member, event timing
(the rounds launched without the graph), a change of options between calls
(a new capture), the round counts, and timing restricted to chosen kernel
kinds."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from oracle import epi as oepi
from paper_2101_05617_amd import inputs
from tests.gpu_util import check_fields, check_krylov, pair, record, small, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

C0 = inputs.WORKLOADS["c0_ne4_p4"]
C2 = inputs.WORKLOADS["c2_ne60_p6_jet"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    from paper_2101_05617_amd import dfrsw
    dfrsw.lib()


def _decisions(st):
    return (st["n_substeps"], st["n_rejected"], st["m_last"], st["n_matvec"], st["happy"], st["n_expm"])


def _same_states(dev, host, G, key):
    """dev against host: bit-identical, or within 1e-13 element-wise."""
    same = bool(np.array_equal(dev, host))
    record(f"{key}_bitwise", float(same))
    if not same:
        check_fields(dev, host, G, 1e-13, key)


def _run_pair(ws, prec, opts_list, frames=None):
    """The same ensemble with host- and device-driven rounds; per step the
    decisions of both, then the final states."""
    from paper_2101_05617_amd.ensemble import Ensemble
    host = Ensemble(ws, prec=prec, form="batched", autotune=False, frames=frames, rounds="host")
    dev = Ensemble(ws, prec=prec, form="batched", autotune=False, frames=frames, rounds="device")
    try:
        for k, opts in enumerate(opts_list):
            sh = host.step(opts)
            sd = dev.step(opts)
            assert [_decisions(x) for x in sd] == [_decisions(x) for x in sh], k
        return [host.state(k) for k in range(len(ws))], [dev.state(k) for k in range(len(ws))], dev
    finally:
        host.close()


def test_device_rounds_match_host_rounds_and_the_oracle_fp64():
    import torch
    from paper_2101_05617_amd import dfrsw
    ws = [small(C0, 2, 3), small(C0, 3, 4, u_amp=1.0), small(C0, 2, 2), small(C0, 4, 4), small(C0, 1, 5)]
    frames = [oracle.OracleGrid(w.ne, w.ns, *w.constants()).node_frames() for w in ws]
    opts = dfrsw.kiops_opts(tol=1e-10, m_max=24)
    hs, ds, dev = _run_pair(ws, "fp64", [opts] * 4, frames)
    planned, launched = dfrsw.dfr_ensemble_round_counts(dev.eg)
    dev.close()
    # EPI4: two start-up steps of s EPI2 sub-steps (one KIOPS call each),
    # then one call per step; a call launches at most two rounds beyond its
    # last with work
    calls = 2 * ws[0].startup_substeps + 2
    assert 0 < planned <= launched <= planned + 2 * calls, (planned, launched, calls)
    for k, w in enumerate(ws):
        G = oracle.OracleGrid(w.ne, w.ns, *w.constants())
        _same_states(ds[k], hs[k], G, f"devrounds_fp64_member{k}")
        Q, _ = inputs.initial_state(w, *frames[k])
        E = oepi.EPI(G.rhs, lambda q, v, G=G: G.jvp(q, v), w.order, w.dt_nd, Q,
                     startup_substeps=w.startup_substeps, kiops_opts=dict(tol=1e-10, m_max=24))
        for _ in range(4):
            E.step()
        check_krylov(ds[k], E.q, G, 1e-11, f"devrounds_fp64_member{k}_vs_oracle")
    torch.cuda.synchronize()


def test_device_rounds_mixed_precision_match_host_rounds():
    import torch
    from paper_2101_05617_amd import dfrsw
    ws = [small(C2, 2, 4), small(C2, 3, 5), small(C2, 2, 6), small(C2, 2, 3)]
    ws = [replace(w, order=4, dt_s=900.0, m_max=32) for w in ws]
    opts = dfrsw.kiops_opts(tol=1e-6, m_max=32)
    hs, ds, dev = _run_pair(ws, "fp32_jv_basis32", [opts] * 5)
    dev.close()
    for k, w in enumerate(ws):
        _same_states(ds[k], hs[k], oracle.OracleGrid(w.ne, w.ns, *w.constants()), f"devrounds_basis32_member{k}")
    torch.cuda.synchronize()


def test_device_rounds_rejections_and_krylov_size_changes():
    # a tolerance the initial Krylov size misses: rejected attempts, changes
    # of m and tau from the error ratios (the log/pow branches of K6/K7)
    import torch
    from paper_2101_05617_amd import dfrsw
    ws = [small(C2, 2, 4), small(C2, 3, 3), small(C2, 2, 5)]
    ws = [replace(w, order=4, dt_s=3600.0, m_max=16) for w in ws]
    opts = dfrsw.kiops_opts(tol=1e-12, m_init=6, m_min=4, m_max=16)
    from paper_2101_05617_amd.ensemble import Ensemble
    host = Ensemble(ws, prec="fp64", form="batched", autotune=False, rounds="host")
    dev = Ensemble(ws, prec="fp64", form="batched", autotune=False, rounds="device")
    rejected = 0
    try:
        for k in range(4):
            sh = host.step(opts)
            sd = dev.step(opts)
            assert [_decisions(x) for x in sd] == [_decisions(x) for x in sh], k
            rejected += sum(x["n_rejected"] for x in sh)
        assert rejected > 0
        for k, w in enumerate(ws):
            _same_states(dev.state(k), host.state(k), oracle.OracleGrid(w.ne, w.ns, *w.constants()),
                         f"devrounds_rejections_member{k}")
    finally:
        host.close()
        dev.close()
        torch.cuda.synchronize()


def test_device_rounds_happy_breakdowns_and_non_convergence():
    import torch
    from paper_2101_05617_amd import dfrsw
    from tests.test_gpu_kiops_edges import _oracle_epi_with_happy, _symmetric_rest
    G, _, Qs = _symmetric_rest(False)
    wa = small(C0, 2, 3)
    Ga, Da, Qa = pair(wa)
    g = C0.gravity_nd
    descs = [dict(ne=wa.ne, p=wa.p, radius=1.0, omega=1.0, gravity=g), dict(ne=1, p=1, radius=1.0, omega=0.0, gravity=g)]
    kopt = dict(tol=1e-10, m_max=24)
    opts = dfrsw.kiops_opts(**kopt)
    ref = _oracle_epi_with_happy(G, Qs, 4, kopt)
    eg = dfrsw.dfr_ensemble_create(descs)
    dfrsw.dfr_ensemble_set_rounds(eg, "device")
    x = dfrsw.epi_ensemble_create(eg, 4, C0.dt_nd, [to_dev(Qa), to_dev(Qs)], startup_substeps=2)
    try:
        for k in range(4):
            sb = dfrsw.epi_ensemble_step(eg, x, opts)
            assert (sb[1]["n_matvec"], sb[1]["happy"]) == ref[k][1:], (k, sb[1])
            check_krylov(to_host(dfrsw.epi_ensemble_get_state(x, 1)), ref[k][0], G, 1e-11,
                         f"devrounds_happy_sym_step{k + 1}")
        # an attempt cap no member can meet: DFR_E_KIOPS naming a member
        with pytest.raises(dfrsw.DfrError) as e:
            dfrsw.epi_ensemble_step(eg, x, dfrsw.kiops_opts(tol=1e-30, m_init=4, m_min=4, m_max=4, max_attempts=3))
        assert e.value.code == -6 and "member" in str(e.value)
    finally:
        x.close()
        eg.close()
        torch.cuda.synchronize()


def test_device_rounds_timed_and_recaptured():
    # with event timing on the rounds are launched without the graph: the
    # same decisions and states; the product launches' nodes are the
    # products counted by the controller times the member sizes.  A change
    # of m_max (another exponential workspace) makes a new capture.
    import torch
    from paper_2101_05617_amd import dfrsw
    from paper_2101_05617_amd.ensemble import Ensemble
    ws = [small(C0, 2, 3), small(C0, 3, 4, u_amp=1.0), small(C0, 2, 5)]
    host = Ensemble(ws, prec="fp64", form="batched", autotune=False, rounds="host")
    dev = Ensemble(ws, prec="fp64", form="batched", autotune=False, rounds="device")
    try:
        o24, o32 = dfrsw.kiops_opts(tol=1e-10, m_max=24), dfrsw.kiops_opts(tol=1e-10, m_max=32)
        for opts in (o24, o32):
            assert [_decisions(x) for x in dev.step(opts)] == [_decisions(x) for x in host.step(opts)]
        dfrsw.dfr_ensemble_timing_enable(dev.eg, True)
        sh = host.step(o32)
        sd = dev.step(o32)
        assert [_decisions(x) for x in sd] == [_decisions(x) for x in sh]
        ms, n, nodes = dfrsw.dfr_ensemble_timing_read(dev.eg, "jv_arnoldi")
        expect = sum(s["n_matvec"] * 6 * w.ne ** 2 * w.ns ** 2 for s, w in zip(sd, ws))
        assert ms > 0 and n > 0 and nodes == expect, (ms, n, nodes, expect)
        dfrsw.dfr_ensemble_timing_enable(dev.eg, False)
        assert [_decisions(x) for x in dev.step(o24)] == [_decisions(x) for x in host.step(o24)]
        for k, w in enumerate(ws):
            _same_states(dev.state(k), host.state(k), oracle.OracleGrid(w.ne, w.ns, *w.constants()),
                         f"devrounds_timed_member{k}")
    finally:
        host.close()
        dev.close()
        torch.cuda.synchronize()


def test_ensemble_timing_brackets_only_the_chosen_kinds():
    # dfr_ensemble_timing_kinds: with only the Krylov-form product chosen, the
    # other kinds record no launch; a mask beyond the kinds is refused
    import torch
    from paper_2101_05617_amd import dfrsw
    from paper_2101_05617_amd.ensemble import Ensemble
    ws = [small(C0, 2, 3), small(C0, 2, 4)]
    ens = Ensemble(ws, prec="fp64", form="batched", autotune=False, rounds="host")
    try:
        opts = dfrsw.kiops_opts(tol=1e-10, m_max=24)
        dfrsw.dfr_ensemble_timing_kinds(ens.eg, ["jv_arnoldi"])
        dfrsw.dfr_ensemble_timing_enable(ens.eg, True)
        st = ens.step(opts)
        ms, n, nodes = dfrsw.dfr_ensemble_timing_read(ens.eg, "jv_arnoldi")
        assert ms > 0 and n > 0 and nodes == sum(s["n_matvec"] * 6 * w.ne ** 2 * w.ns ** 2 for s, w in zip(st, ws))
        for kind in ("update", "expm", "other", "rhs"):
            assert dfrsw.dfr_ensemble_timing_read(ens.eg, kind)[1] == 0, kind
        dfrsw.dfr_ensemble_timing_kinds(ens.eg, None)
        dfrsw.dfr_ensemble_timing_enable(ens.eg, True)
        ens.step(opts)
        assert dfrsw.dfr_ensemble_timing_read(ens.eg, "update")[1] > 0
        with pytest.raises(dfrsw.DfrError):
            dfrsw._check(dfrsw.lib().dfr_ensemble_timing_kinds(ens.eg.handle, 1 << 12))
    finally:
        dfrsw.dfr_ensemble_timing_enable(ens.eg, False)
        ens.close()
        torch.cuda.synchronize()
