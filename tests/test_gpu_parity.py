"""GPU parity: the HIP library against the FP64 oracle on identical seeded
inputs, element by element, through the C ABI.

Every comparison of a state-sized result applies its bar to four measures
per field (tests/gpu_util.check_fields): the relative L2 difference, the
element-wise maximum difference against the field's largest value, and both
over the nodes of the elements that touch a panel edge, where the App. C
maps act; a failure names the worst node (field, panel, element, node).

Tolerances (each measure per field, maximum over the three fields):
  FP64 J v            1e-12.  Both sides evaluate the same formulas in FP64;
      they differ only in operation order, FMA contraction and the division /
      square-root sequences, i.e. O(1e-16) per operation; J v of a random
      direction is well conditioned (a 1-ulp input perturbation moves it by
      ~5e-16), so 1e-12 leaves three orders of margin.
  FP64 F(q)           max(1e-11, 4 x floor), floor = the oracle's own relative
      change under a random 1-ulp perturbation of q (in the same measure).
      The tendency of a near-balanced state is a residual of flux terms
      1e3-1e5 times larger:
      its condition makes any two correct FP64 evaluations differ by ~floor
      (2.6e-11 at ne = 30, p = 5; 6e-11 at ne = 4, p = 4).
  FP32 J v            2e-5.  Complex FP32 evaluation (unit roundoff 6e-8)
      with the same cancellation factor (~1e2-1e3).
  KIOPS, EPI          1e-11 after every step (the plain-FP64 target), with
      identical controller decisions (sub-steps, rejections, Krylov size);
      the element-wise measures a decade above (check_krylov: rounding of
      Krylov results gathers at a few nodes).
"""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from oracle import epi as oepi
from oracle import kiops as okiops
from paper_2101_05617_amd import inputs
from tests.gpu_util import (check_fields, check_krylov, check_rhs, field_metrics, pair, record, small, to_dev,
                            to_host, torch_dev)

pytestmark = pytest.mark.gpu

C0 = inputs.WORKLOADS["c0_ne4_p4"]
C1 = inputs.WORKLOADS["c1_ne30_p5"]
C2 = inputs.WORKLOADS["c2_ne60_p6_jet"]
C4 = inputs.WORKLOADS["c4_ne120_p6_mountain"]

# (ne, p): single-element panels, every supported degree, ragged last blocks
GRIDS = [(1, 1), (2, 2), (3, 4), (4, 4), (2, 5), (3, 6), (5, 6), (2, 7), (3, 3)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    from paper_2101_05617_amd import dfrsw
    dfrsw.lib()
    yield


@pytest.mark.parametrize("ne,p", GRIDS)
def test_rhs_parity(ne, p):
    w = small(C0, ne, p, u_amp=2.0)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    got = to_host(dfrsw.dfr_rhs(D, to_dev(Q)))
    dfrsw.dfr_sync(D)
    check_rhs(got, G, Q, f"rhs_fp64_ne{ne}_p{p}")


@pytest.mark.parametrize("ne,p", GRIDS)
def test_jvp_parity_fp64(ne, p):
    w = small(C0, ne, p, u_amp=2.0)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    V = inputs.random_direction(3 * G.N, 100 + ne * 10 + p)
    ref = G.jvp(Q, V, 1e-150)
    got = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-150, "fp64"))
    dfrsw.dfr_sync(D)
    check_fields(got, ref, G, 1e-12, f"jvp_fp64_ne{ne}_p{p}")


def test_jvp_eps_independence_and_linearity():
    G, D, Q = pair(C0)
    from paper_2101_05617_amd import dfrsw
    V = inputs.random_direction(3 * G.N, 7)
    q, v = to_dev(Q), to_dev(V)
    a = to_host(dfrsw.dfr_jvp_complex_step(D, q, v, 1e-100))
    b = to_host(dfrsw.dfr_jvp_complex_step(D, q, v, 1e-200))
    c = to_host(dfrsw.dfr_jvp_complex_step(D, q, to_dev(2.0 * V), 1e-150))
    assert np.linalg.norm(a - b) <= 1e-14 * np.linalg.norm(a)
    assert np.linalg.norm(c - 2 * a) <= 1e-14 * np.linalg.norm(c)


@pytest.mark.parametrize("ne,p", [(4, 4), (3, 6), (2, 5)])
def test_jvp_parity_fp32(ne, p):
    w = small(C0, ne, p, u_amp=2.0)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    V = inputs.random_direction(3 * G.N, 5)
    ref = G.jvp(Q, V, 1e-150)
    got = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-20, "fp32_jv"))
    dfrsw.dfr_sync(D)
    check_fields(got, ref, G, 2e-5, f"jvp_fp32_ne{ne}_p{p}")


def test_mass_conservation_on_gpu():
    G, D, Q = pair(small(C0, 3, 5, u_amp=3.0, h_amp=0.05))
    from paper_2101_05617_amd import dfrsw
    wq = G.mass_weights()
    F = to_host(dfrsw.dfr_rhs(D, to_dev(Q)))
    V = inputs.random_direction(3 * G.N, 9)
    J = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V)))
    assert abs(wq @ F[: G.N]) < 1e-15 * (wq @ Q[: G.N]) * 10
    assert abs(wq @ J[: G.N]) < 1e-14 * (wq @ np.abs(J[: G.N]))


def test_orography_parity():
    # perturbed flow over the mountain: the standard bar
    w = replace(inputs.WORKLOADS["c4_ne120_p6_mountain"], ne=3, h_amp=0.01, h_lmax=6, u_amp=2.0)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    got = to_host(dfrsw.dfr_rhs(D, to_dev(Q)))
    check_rhs(got, G, Q, "rhs_mountain_perturbed")
    # the unperturbed state is nearly in balance: its tendency (~1e-6) is a
    # cancellation of gravity and orography terms ~4e5 times larger
    w0 = replace(inputs.WORKLOADS["c4_ne120_p6_mountain"], ne=3)
    G0, D0, Q0 = pair(w0)
    got0 = to_host(dfrsw.dfr_rhs(D0, to_dev(Q0)))
    check_rhs(got0, G0, Q0, "rhs_mountain_balanced")
    V = inputs.random_direction(3 * G.N, 4)
    check_fields(to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V))), G.jvp(Q, V), G, 1e-12,
                 "jvp_mountain")


@pytest.mark.parametrize("rot", [(0.0, 0.0, 0.0), (0.3, 0.5, 0.2)])
def test_other_rotations(rot):
    w = small(C0, 3, 4, u_amp=1.0)
    G, D, Q = pair(w, rotation=rot)
    from paper_2101_05617_amd import dfrsw
    check_rhs(to_host(dfrsw.dfr_rhs(D, to_dev(Q))), G, Q, f"rhs_rotation_{rot[0]}_{rot[1]}_{rot[2]}")


def test_invalid_depth_is_reported():
    G, D, Q = pair(small(C0, 2, 3))
    from paper_2101_05617_amd import dfrsw
    Qb = Q.copy()
    Qb[3] = -0.5
    dfrsw.dfr_rhs(D, to_dev(Qb))
    with pytest.raises(dfrsw.DfrError) as e:
        dfrsw.dfr_sync(D)
    assert e.value.code == -5
    dfrsw.dfr_sync(D)   # the latch is cleared
    Qn = Q.copy()
    Qn[2 * G.N + 1] = np.nan
    with pytest.raises(dfrsw.DfrError) as e:
        dfrsw.kiops_phi_apply(D, to_dev(Qn), 0.01, [None, to_dev(Q)])
    assert e.value.code == -4


# ---------------------------------------------------------------------------
# KIOPS and EPI

def _kopts(tol, m_max, **kw):
    from paper_2101_05617_amd import dfrsw
    return dfrsw.kiops_opts(tol=tol, m_max=m_max, **kw)


@pytest.mark.parametrize("nphi,with_b0", [(1, False), (3, False), (0, True), (2, True), (4, True), (6, False)])
def test_kiops_parity(nphi, with_b0):
    w = small(C0, 3, 4, u_amp=1.0)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    rng = np.random.default_rng(nphi)
    F = G.rhs(Q)
    bs = [Q.copy() if with_b0 else None] + [F] + [1e-3 * rng.standard_normal(3 * G.N) for _ in range(nphi - 1)]
    bs = bs[: nphi + 1]
    tau = 4 * w.dt_nd
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v, 1e-150), bs, tol=1e-12, m_max=32)
    got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None if b is None else to_dev(b) for b in bs],
                                     _kopts(1e-12, 32), 1e-150, "fp64")
    got = to_host(got)
    assert (gst["n_substeps"], gst["n_rejected"], gst["m_last"]) == (rst.n_substeps, rst.n_rejected, rst.m_last)
    assert gst["n_matvec"] == rst.n_matvec
    check_krylov(got, ref, G, 1e-11, f"kiops_nphi{nphi}_b0{int(with_b0)}")


def test_kiops_substepping_parity():
    # a small Krylov cap forces sub-steps and rejections
    w = small(C0, 3, 4, u_amp=1.0)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    F = G.rhs(Q)
    tau = 40 * w.dt_nd
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F], tol=1e-10, m_init=8, m_min=4, m_max=12)
    got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)], _kopts(1e-10, 12, m_init=8, m_min=4))
    assert rst.n_substeps > 1
    assert (gst["n_substeps"], gst["n_rejected"]) == (rst.n_substeps, rst.n_rejected)
    check_krylov(to_host(got), ref, G, 1e-11, "kiops_substepping")


def test_kiops_iop1_parity_and_invalid_iop():
    # orthogonalisation against the last vector only; iop > 2 is rejected
    w = small(C0, 3, 4, u_amp=1.0)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    F = G.rhs(Q)
    tau = 4 * w.dt_nd
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F], tol=1e-12, m_max=32, iop=1)
    got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)], _kopts(1e-12, 32, iop=1))
    assert (gst["n_substeps"], gst["n_rejected"], gst["n_matvec"]) == (rst.n_substeps, rst.n_rejected, rst.n_matvec)
    check_krylov(to_host(got), ref, G, 1e-11, "kiops_iop1")
    with pytest.raises(dfrsw.DfrError) as e:
        dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)], _kopts(1e-12, 32, iop=3))
    assert e.value.code == -1


def _epi_compare(w, steps, s, tol_rel=1e-11, prec="fp64", eps=1e-150, check_every=True):
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    kopt = dict(tol=w.tol, m_max=w.m_max)
    E = oepi.EPI(G.rhs, lambda q, v: G.jvp(q, v, eps), w.order, w.dt_nd, Q, startup_substeps=s, kiops_opts=kopt)
    st = dfrsw.epi_create(D, w.order, w.dt_nd, to_dev(Q), startup_substeps=s, eps=eps, prec=prec)
    errs = []
    for k in range(steps):
        E.step()
        stats = dfrsw.epi_step(D, st, _kopts(w.tol, w.m_max))
        got = to_host(dfrsw.epi_get_state(st))
        key = f"epi{w.order}_{w.name}_ne{w.ne}_p{w.p}_step{k + 1}"
        if check_every:
            errs.append(check_krylov(got, E.q, G, tol_rel, key)["l2"])
        else:
            errs.append(field_metrics(got, E.q, G.ne, G.ns)["l2"])
            record(key, errs[-1])
    return errs


def test_epi4_parity_c0_every_step():
    # the smallest configuration: ne = 4, p = 4, EPI4, dt 900 s, 4 steps
    errs = _epi_compare(C0, C0.steps, C0.startup_substeps)
    assert max(errs) < 1e-11


@pytest.mark.parametrize("order", [2, 3, 5, 6])
def test_epi_orders_parity(order):
    w = replace(small(C0, 3, 4), order=order)
    errs = _epi_compare(w, 6 if order > 2 else 3, 2)
    assert max(errs) < 1e-11


def test_c1_full_size_rhs_jvp_parity():
    # ne = 30, p = 5 (194,400 nodes): every element of F and J v
    G, D, Q = pair(C1)
    from paper_2101_05617_amd import dfrsw
    check_rhs(to_host(dfrsw.dfr_rhs(D, to_dev(Q))), G, Q, "c1_rhs_fp64")
    V = inputs.random_direction(3 * G.N, 31)
    ref = G.jvp(Q, V)
    got = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V)))
    check_fields(got, ref, G, 1e-12, "c1_jvp_fp64")
    got32 = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-20, "fp32_jv"))
    check_fields(got32, ref, G, 2e-5, "c1_jvp_fp32")


def test_c2_full_size_rhs_jvp_parity():
    # ne = 60, p = 6 (1,058,400 nodes), mid-latitude jet: every element of F
    # and J v, FP64 and complex-FP32, in the autotuned tiles of the J v timing
    G, D, Q = pair(C2)
    from paper_2101_05617_amd import dfrsw
    dfrsw.dfr_autotune(D, "fp64")
    check_rhs(to_host(dfrsw.dfr_rhs(D, to_dev(Q))), G, Q, "c2_rhs_fp64")
    V = inputs.random_direction(3 * G.N, 21)
    ref = G.jvp(Q, V)
    got = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V)))
    check_fields(got, ref, G, 1e-12, "c2_jvp_fp64")
    dfrsw.dfr_autotune(D, "fp32_jv")
    got32 = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-20, "fp32_jv"))
    check_fields(got32, ref, G, 2e-5, "c2_jvp_fp32")


def test_c4_full_size_rhs_jvp_parity():
    # ne = 120, p = 6 (4,233,600 nodes), Gaussian mountain (orography): every
    # element of F and J v, FP64 and complex-FP32, in the autotuned tiles
    G, D, Q = pair(C4)
    from paper_2101_05617_amd import dfrsw
    dfrsw.dfr_autotune(D, "fp64")
    check_rhs(to_host(dfrsw.dfr_rhs(D, to_dev(Q))), G, Q, "c4_rhs_fp64")
    V = inputs.random_direction(3 * G.N, 41)
    ref = G.jvp(Q, V)
    got = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V)))
    check_fields(got, ref, G, 1e-12, "c4_jvp_fp64")
    dfrsw.dfr_autotune(D, "fp32_jv")
    got32 = to_host(dfrsw.dfr_jvp_complex_step(D, to_dev(Q), to_dev(V), 1e-20, "fp32_jv"))
    check_fields(got32, ref, G, 2e-5, "c4_jvp_fp32")


def test_c1_full_size_epi5_parity():
    # ne = 30, p = 5, EPI5, dt 1800 s: three start-up steps and the first EPI5
    # step in the launch configuration the benchmark times (start-up with 2
    # sub-steps to bound the oracle's run time)
    errs = _epi_compare(C1, 4, 2)
    assert max(errs) < 1e-11


@pytest.mark.parametrize("ne,p", [(6, 3), (4, 6), (2, 2)])
def test_every_tile_shape_gives_the_same_result(ne, p):
    # the workgroup tile (TX x TY elements) changes only the decomposition
    w = small(C0, ne, p, u_amp=2.0)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    V = inputs.random_direction(3 * G.N, 77)
    ref_j = G.jvp(Q, V)
    q, v = to_dev(Q), to_dev(V)
    nn = (p + 1) ** 2
    tried = 0
    for tx in range(1, ne + 1):
        for ty in range(1, ne + 1):
            if ne % tx or ne % ty or tx * ty * nn > 1024:
                continue
            dfrsw.dfr_set_tile(D, tx, ty)
            assert dfrsw.dfr_get_tile(D) == (tx, ty)
            check_rhs(to_host(dfrsw.dfr_rhs(D, q)), G, Q, f"tile_rhs_ne{ne}_p{p}_{tx}x{ty}")
            check_fields(to_host(dfrsw.dfr_jvp_complex_step(D, q, v)), ref_j, G, 1e-12,
                         f"tile_jvp_ne{ne}_p{p}_{tx}x{ty}")
            tried += 1
    assert tried >= 3
    with pytest.raises(dfrsw.DfrError):
        dfrsw.dfr_set_tile(D, ne + 1, 1)
    tx, ty = dfrsw.dfr_autotune(D, "fp64")
    assert ne % tx == 0 and ne % ty == 0
    check_fields(to_host(dfrsw.dfr_jvp_complex_step(D, q, v)), ref_j, G, 1e-12)


def test_krylov_form_tiles_give_the_same_result():
    # the Krylov-form product (fused Arnoldi steps) under several tiles
    w = small(C0, 4, 4, u_amp=1.0)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    F = G.rhs(Q)
    tau = 4 * w.dt_nd
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F, 1e-2 * F], tol=1e-12, m_max=32)
    for tx, ty in [(1, 1), (2, 1), (4, 4), (1, 4)]:
        dfrsw.dfr_set_tile(D, tx, ty)
        assert dfrsw.dfr_get_krylov_tile(D) == (tx, ty)
        got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F), to_dev(1e-2 * F)],
                                         _kopts(1e-12, 32))
        assert (gst["n_substeps"], gst["n_rejected"], gst["n_matvec"]) == (rst.n_substeps, rst.n_rejected,
                                                                           rst.n_matvec)
        check_krylov(to_host(got), ref, G, 1e-11, f"kiops_tile_{tx}x{ty}")


def _h_error(got, ref, N):
    return np.linalg.norm(got[:N] - ref[:N]) / np.linalg.norm(ref[:N])


def _h_max_error(got, ref, N):
    return np.max(np.abs(got[:N] - ref[:N])) / np.max(np.abs(ref[:N]))


def test_mixed_precision_epi6_jet_against_fp64_oracle():
    # complex-FP32 J v inside the FP64 Krylov / EPI6 machinery on the jet
    # workload (ne = 4, p = 6): four start-up steps and four EPI6 steps against
    # the FP64 oracle.  Bar: 1e-6 relative L2 in h (the accuracy the mixed
    # form is held to) and 1e-6 element-wise in h (against max h); 1e-4 on
    # every field in every measure.
    w = small(C2, 4)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    kopt = dict(tol=w.tol, m_max=w.m_max)
    E = oepi.EPI(G.rhs, lambda q, v: G.jvp(q, v, 1e-150), w.order, w.dt_nd, Q, startup_substeps=2,
                 kiops_opts=kopt)
    st = dfrsw.epi_create(D, w.order, w.dt_nd, to_dev(Q), startup_substeps=2, eps=w.eps, prec="fp32_jv")
    for k in range(8):
        E.step()
        dfrsw.epi_step(D, st, _kopts(w.tol, w.m_max))
        got = to_host(dfrsw.epi_get_state(st))
        eh, ehm = _h_error(got, E.q, G.N), _h_max_error(got, E.q, G.N)
        record(f"mixed_epi6_jet_ne4_step{k + 1}_h", eh)
        record(f"mixed_epi6_jet_ne4_step{k + 1}_h_max", ehm)
        assert eh < 1e-6 and ehm < 1e-6, (k, eh, ehm)
        check_fields(got, E.q, G, 1e-4, f"mixed_epi6_jet_ne4_step{k + 1}_all")


def test_mixed_precision_kiops_against_fp64():
    # one phi-combination with the FP32 product: within the FP32 rounding
    # level of the FP64 oracle's result
    w = small(C2, 3)
    G, D, Q = pair(w)
    from paper_2101_05617_amd import dfrsw
    F = G.rhs(Q)
    tau = w.dt_nd
    ref, _ = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F], tol=1e-10, m_max=64)
    got, _ = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)], _kopts(1e-10, 64), w.eps, "fp32_jv")
    check_krylov(to_host(got), ref, G, 1e-5, "mixed_kiops_jet_ne3")


def test_c2_full_size_kiops_parity():
    # ne = 60, p = 6 jet (3,175,200 unknowns): one phi_1 product in the
    # autotuned Krylov-form tiles, FP64 (identical decisions, the plain-FP64
    # bar) and with the complex-FP32 product (FP32 bar).  tau = dt/8 keeps
    # the oracle's run to about 20 J v (one sub-step after two rejections).
    G, D, Q = pair(C2)
    from paper_2101_05617_amd import dfrsw
    dfrsw.dfr_autotune(D, "fp64")
    F = G.rhs(Q)
    tau = C2.dt_nd / 8
    ref, rst = okiops.kiops(tau, lambda v: G.jvp(Q, v), [None, F], tol=C2.tol, m_max=C2.m_max)
    assert rst.n_rejected > 0
    got, gst = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)], _kopts(C2.tol, C2.m_max))
    assert (gst["n_substeps"], gst["n_rejected"], gst["n_matvec"]) == (rst.n_substeps, rst.n_rejected, rst.n_matvec)
    check_krylov(to_host(got), ref, G, 1e-11, "kiops_c2_full_fp64")
    dfrsw.dfr_autotune(D, "fp32_jv")
    got32, _ = dfrsw.kiops_phi_apply(D, to_dev(Q), tau, [None, to_dev(F)], _kopts(C2.tol, C2.m_max), C2.eps,
                                     "fp32_jv")
    check_krylov(to_host(got32), ref, G, 1e-5, "kiops_c2_full_fp32_jv")


def test_ensemble_forms_match_members_run_alone():
    # the batched form (one launch per operation for all members) and the
    # concurrent form give what epi_step gives member by member, and the
    # members agree with the oracle
    import torch
    from paper_2101_05617_amd import dfrsw
    from paper_2101_05617_amd.ensemble import Ensemble
    ws = [small(C0, 2, 3), small(C0, 3, 4, u_amp=1.0), small(C0, 2, 2), small(C0, 4, 4), small(C0, 1, 5)]
    frames = [oracle.OracleGrid(w.ne, w.ns, *w.constants()).node_frames() for w in ws]
    opts = _kopts(1e-10, 24)
    ref = Ensemble(ws, prec="fp64", form="sequential", autotune=False, frames=frames)
    # host-driven rounds: bit for bit (the device-driven form is held to the
    # host-driven one in test_gpu_device_rounds)
    bat = Ensemble(ws, prec="fp64", form="batched", autotune=False, frames=frames, rounds="host")
    con = Ensemble(ws, prec="fp64", form="concurrent", autotune=False, frames=frames)
    for _ in range(4):
        sr = ref.step(opts)
        sb = bat.step(opts)
        sc = con.step(opts, n_workers=3)
        assert [x["n_matvec"] for x in sb] == [x["n_matvec"] for x in sr]
        assert [x["n_matvec"] for x in sc] == [x["n_matvec"] for x in sr]
    for k, w in enumerate(ws):
        a, b, c = ref.state(k), bat.state(k), con.state(k)
        assert np.array_equal(a, c), (k, np.abs(a - c).max())
        # same kernels, tiles, reduction orders and EPI combinations
        assert np.array_equal(a, b), (k, np.abs(a - b).max())
        G = oracle.OracleGrid(w.ne, w.ns, *w.constants())
        Q, _ = inputs.initial_state(w, *frames[k])
        E = oepi.EPI(G.rhs, lambda q, v: G.jvp(q, v), w.order, w.dt_nd, Q, startup_substeps=w.startup_substeps,
                     kiops_opts=dict(tol=1e-10, m_max=24))
        for _ in range(4):
            E.step()
        check_krylov(b, E.q, G, 1e-11, f"ensemble_member{k}_vs_oracle")
    with pytest.raises(dfrsw.DfrError):
        dfrsw.epi_step_concurrent([con.grids[0], con.grids[0]], [con.states[0], con.states[0]], opts, 2)
    for e in (ref, bat, con):
        e.close()
    torch.cuda.synchronize()


def test_batched_ensemble_mixed_precision_and_errors():
    # FP32 products in the batched form against FP64 member by member; a bad
    # member state is reported with the member's index
    import torch
    from paper_2101_05617_amd import dfrsw
    from paper_2101_05617_amd.ensemble import Ensemble
    ws = [small(C2, 2, 4), small(C2, 3, 5), small(C2, 2, 6)]
    ws = [replace(w, order=4, dt_s=900.0, m_max=32) for w in ws]
    opts = _kopts(1e-10, 32)
    ref = Ensemble(ws, prec="fp64", form="sequential", autotune=False)
    bat = Ensemble(ws, prec="fp32_jv", form="batched", autotune=True)
    for _ in range(5):
        ref.step(opts)
        bat.step(opts)
    for k in range(len(ws)):
        a, b = ref.state(k), bat.state(k)
        N = len(a) // 3
        eh = np.linalg.norm(b[:N] - a[:N]) / np.linalg.norm(a[:N])
        record(f"ensemble_fp32_member{k}_h", eh)
        assert eh < 1e-6, (k, eh)
    # a non-positive depth in member 1
    eg = dfrsw.dfr_ensemble_create([dict(ne=w.ne, p=w.p, radius=w.constants()[0], omega=w.constants()[1],
                                         gravity=w.constants()[2]) for w in ws])
    qs = [torch.from_numpy(ref.state(k)).cuda() for k in range(len(ws))]
    qs[1][5] = -1.0
    x = dfrsw.epi_ensemble_create(eg, ws[0].order, ws[0].dt_nd, qs, prec="fp64")
    with pytest.raises(dfrsw.DfrError) as e:
        dfrsw.epi_ensemble_step(eg, x, opts)
    assert e.value.code == -5 and "member 1" in str(e.value)
    x.close()
    eg.close()
    for z in (ref, bat):
        z.close()
    torch.cuda.synchronize()
