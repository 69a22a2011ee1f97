"""Pins of the oracle's decision record and replay (oracle/kiops.py,
DecisionReplay): the KIOPS controller of Sec. 4 (Eq. 29) with its attempts'
decisions taken from a list instead of from its error estimate.

What fixes the result independently of the replay code:
  - replaying a run's own decisions repeats that run exactly (same arithmetic,
    same path);
  - any admissible path of sub-steps still computes the phi-combination of
    Eq. 29, checked against the dense augmented exponential;
  - a rejected attempt keeps its Krylov basis (K4), so rejecting at m and then
    accepting at m' > m gives the same result, bit for bit, as accepting at m'
    directly;
  - decisions that cannot be taken are errors;
  - (property test) any admissible path of resolved sub-steps, with rejected
    attempts anywhere in it, gives the dense result, and its rejections
    change nothing."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as hst

from oracle import epi, kiops, ode, phi


def _stiff_matrix(n, seed, scale):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = -np.logspace(-2, 3, n)
    A = Q @ np.diag(d) @ Q.T + 0.3 * (rng.standard_normal((n, n)) - rng.standard_normal((n, n)).T) / np.sqrt(n)
    return A * scale


def _path(tau_out, steps, m):
    """Accepted sub-steps of the given lengths, the last clipped to end at
    tau_out as the controller clips it (K7): (tau, m, True) each."""
    out, t = [], 0.0
    for h in steps:
        tau = min(h, tau_out - t)
        out.append((tau, m, True))
        t = tau_out if tau >= tau_out - t else t + tau
    assert t == tau_out
    return out


def _problem():
    n = 60
    A = _stiff_matrix(n, 7, 5.0)
    rng = np.random.default_rng(3)
    bs = [None] + [rng.standard_normal(n) for _ in range(3)]
    return A, bs, 1e-2


def test_replay_of_own_decisions_repeats_the_run():
    A, bs, tau = _problem()
    w, st = kiops.kiops(tau, lambda v: A @ v, bs, tol=1e-10, m_init=10, m_max=16)
    # a path with sub-steps and rejections, so that the replay has work to do
    assert st.n_substeps >= 2 and st.n_rejected >= 1
    r = kiops.DecisionReplay(st.decisions)
    w2, st2 = kiops.kiops(tau, lambda v: A @ v, bs, tol=1e-10, m_init=10, m_max=16, replay=r)
    assert np.array_equal(w, w2)
    assert st2.decisions == st.decisions
    assert (st2.n_matvec, st2.n_substeps, st2.n_rejected, st2.n_expm) == \
        (st.n_matvec, st.n_substeps, st.n_rejected, st.n_expm)
    assert r.pos == len(st.decisions)


def test_replayed_foreign_path_computes_the_phi_combination():
    # four sub-steps the controller would not choose (the last one clipped to
    # end exactly at tau_out, K7), one rejected attempt in between
    A, bs, tau = _problem()
    ref = phi.phi_combination_dense(A, tau, [np.zeros(A.shape[0])] + bs[1:])
    path = _path(tau, [0.3 * tau] * 4, 24)
    path.insert(1, (path[1][0], 12, False))
    r = kiops.DecisionReplay(path)
    w, st = kiops.kiops(tau, lambda v: A @ v, bs, tol=1e-10, m_init=10, m_max=32, replay=r)
    assert st.n_substeps == 4 and st.n_rejected == 1
    assert [d[1:] for d in st.decisions] == [d[1:] for d in path]
    assert np.linalg.norm(w - ref) <= 1e-9 * np.linalg.norm(ref)


def test_rejected_attempt_keeps_its_basis():
    A, bs, tau = _problem()
    direct = _path(tau, [0.25 * tau] * 4, 20)
    w1, st1 = kiops.kiops(tau, lambda v: A @ v, bs, tol=1e-10, m_max=32, replay=kiops.DecisionReplay(direct))
    path = []
    for d in direct:
        path += [(d[0], 8, False), d]
    w2, st2 = kiops.kiops(tau, lambda v: A @ v, bs, tol=1e-10, m_max=32, replay=kiops.DecisionReplay(path))
    assert np.array_equal(w1, w2)
    assert st1.n_matvec == st2.n_matvec
    assert (st1.n_expm, st2.n_expm) == (4, 8)


def test_decisions_that_cannot_be_taken_are_errors():
    A, bs, tau = _problem()
    mv = lambda v: A @ v
    with pytest.raises(kiops.KiopsError, match="ran out"):
        kiops.kiops(tau, mv, bs, m_max=32, replay=kiops.DecisionReplay([(0.5 * tau, 20, True)]))
    with pytest.raises(kiops.KiopsError, match="cannot be taken"):
        # a sweep cannot shrink: 16 vectors are built when the second attempt asks for 8
        kiops.kiops(tau, mv, bs, m_max=32, replay=kiops.DecisionReplay([(tau, 16, False), (tau, 8, True)]))
    with pytest.raises(kiops.KiopsError, match="cannot be taken"):
        kiops.kiops(tau, mv, bs, m_max=32, replay=kiops.DecisionReplay([(tau, 40, True)]))
    with pytest.raises(kiops.KiopsError, match="cannot be taken"):
        # a sub-step past tau_out
        kiops.kiops(tau, mv, bs, m_max=32, replay=kiops.DecisionReplay([(0.6 * tau, 20, True), (0.6 * tau, 20, True)]))
    # an invariant Krylov space of dimension 3 (b in three eigenvectors of a
    # diagonal operator): a happy breakdown ends the basis below m = 10
    d = -np.arange(1.0, 21.0)
    b = np.zeros(20)
    b[[2, 7, 11]] = 1.0
    with pytest.raises(kiops.KiopsError, match="happy breakdown"):
        kiops.kiops(0.3, lambda v: d * v, [b], tol=1e-12, m_max=20, replay=kiops.DecisionReplay([(0.3, 10, True)]))


def test_epi_steps_replay_across_their_kiops_calls():
    # an EPI4 run (two EPI2 start-up steps of four sub-steps, then EPI4 steps):
    # one replay object carries its position across the step's KIOPS calls
    rhs, jvp, u0, _ = ode.semilinear(60)
    ref = epi.EPI(rhs, jvp, 4, 0.05, u0, startup_substeps=4, kiops_opts=dict(tol=1e-10, m_max=24))
    for _ in range(4):
        ref.step()
    decisions = [d for st in ref.stats for d in st.decisions]
    r = kiops.DecisionReplay(decisions)
    rep = epi.EPI(rhs, jvp, 4, 0.05, u0, startup_substeps=4, kiops_opts=dict(tol=1e-10, m_max=24, replay=r))
    for _ in range(4):
        rep.step()
    assert np.array_equal(ref.q, rep.q)
    assert r.pos == len(decisions) == sum(len(st.decisions) for st in rep.stats)


def _mild_problem():
    # a non-normal operator with ||A|| ~ 2, so that any sub-step of at most the
    # whole interval is resolved by 24 Krylov vectors (||tau A||^24 / 24! ~ 3e-17)
    rng = np.random.default_rng(11)
    n = 40
    A = -np.diag(np.linspace(0.1, 2.0, n)) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n)
    bs = [rng.standard_normal(n)] + [rng.standard_normal(n) for _ in range(2)]
    return A, bs, 1.0


def _random_path(fracs, rejects, m):
    """Accepted sub-steps in proportion to fracs (clipped to end at tau_out),
    each preceded by a rejected attempt at m' = rejects[k] < m if nonzero."""
    tau_out = 1.0
    total = sum(fracs)
    acc = _path(tau_out, [tau_out * f / total for f in fracs[:-1]] + [tau_out], m)
    full, plain = [], []
    for d, r in zip(acc, rejects):
        if r:
            full.append((d[0], r, False))
        full.append(d)
        plain.append(d)
    return full, plain


@settings(max_examples=25, deadline=None, derandomize=True)
@given(fracs=hst.lists(hst.floats(0.05, 1.0), min_size=1, max_size=5),
       rejects=hst.lists(hst.integers(0, 20), min_size=5, max_size=5))
def test_any_admissible_path_gives_the_phi_combination(fracs, rejects):
    # property: whatever sub-steps a path takes (each resolved), with rejected
    # attempts anywhere in it, the result is the dense phi-combination (K2:
    # sub-steps compose exactly); a rejected attempt followed by the accepted
    # one leaves the result unchanged bit for bit (K4: the basis is kept)
    A, bs, tau = _mild_problem()
    ref = phi.phi_combination_dense(A, tau, bs)
    full, plain = _random_path(fracs, rejects[:len(fracs)], 24)
    w1, st1 = kiops.kiops(tau, lambda v: A @ v, bs, tol=1e-12, m_max=24, replay=kiops.DecisionReplay(full))
    w2, st2 = kiops.kiops(tau, lambda v: A @ v, bs, tol=1e-12, m_max=24, replay=kiops.DecisionReplay(plain))
    assert np.array_equal(w1, w2)
    assert st1.n_substeps == st2.n_substeps == len(plain)
    assert st1.n_rejected == sum(1 for r in rejects[:len(fracs)] if r)
    assert np.linalg.norm(w1 - ref) <= 1e-10 * np.linalg.norm(ref)
