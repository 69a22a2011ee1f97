"""The large-time-step regime (Sec. 5.5): the mountain flow with dt = 4 h,
where KIOPS needs several sub-steps, rejections and large Krylov spaces, with
EPI2 (Eq. 25), EPI3 (Eq. 30) and EPI6 (Eqs. 34-38) -- the GPU path against
the oracle after every step, with the same controller decisions.

Bar: 1e-11 per field (the plain-FP64 target) in relative L2 and 1e-10
element by element (check_krylov), over all nodes and over the panel-edge
elements; both sides take
the same sub-steps and Krylov sizes, so they differ only by rounding."""
from dataclasses import replace

import pytest

from oracle import epi as oepi
from paper_2101_05617_amd import inputs
from tests.gpu_util import check_krylov, pair, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

F2 = inputs.WORKLOADS["f2_ne20_p5_mountain_dt4h"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    from paper_2101_05617_amd import dfrsw
    dfrsw.lib()


@pytest.mark.parametrize("order,steps", [(2, 3), (3, 4), (6, 6)])
def test_large_dt_epi_parity_and_adaptivity(order, steps):
    from paper_2101_05617_amd import dfrsw
    w = replace(F2, ne=4, order=order)
    G, D, Q = pair(w)
    kopt = dict(tol=w.tol, m_max=w.m_max)
    E = oepi.EPI(G.rhs, lambda q, v: G.jvp(q, v, 1e-150), order, w.dt_nd, Q, startup_substeps=2, kiops_opts=kopt)
    st = dfrsw.epi_create(D, order, w.dt_nd, to_dev(Q), startup_substeps=2)
    sub = rej = calls = 0
    for k in range(steps):
        n0 = len(E.stats)
        E.step()
        ost = E.stats[n0:]
        gst = dfrsw.epi_step(D, st, dfrsw.kiops_opts(**kopt))
        assert gst["n_substeps"] == sum(s.n_substeps for s in ost)
        assert gst["n_rejected"] == sum(s.n_rejected for s in ost)
        sub += gst["n_substeps"]
        rej += gst["n_rejected"]
        calls += len(ost)
        check_krylov(to_host(dfrsw.epi_get_state(st)), E.q, G, 1e-11, f"large_dt_epi{order}_step{k + 1}")
    # the controller was exercised: sub-stepping or rejections
    assert sub > calls or rej > 0
