"""GPU parity of the Sec. 5.4 diagnostics (dfr_diagnostics: relative
vorticity, Coriolis parameter, integrals of mass, total energy and potential
enstrophy) against the oracle on identical seeded states, through the C ABI.

Bars: zeta 1e-12 relative L2 (a collocation derivative of smooth products:
both sides add the same few terms in a different order, O(1e-16) each, with
cancellation of at most ~1e2); f 1e-14 (a closed form per node); the three
integrals 1e-13 relative (sums of positive terms, different summation
trees)."""
import numpy as np
import pytest

from paper_2101_05617_amd import inputs
from tests.gpu_util import pair, record, small, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

C0 = inputs.WORKLOADS["c0_ne4_p4"]
C1 = inputs.WORKLOADS["c1_ne30_p5"]
C2 = inputs.WORKLOADS["c2_ne60_p6_jet"]
C4 = inputs.WORKLOADS["c4_ne120_p6_mountain"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    from paper_2101_05617_amd import dfrsw
    dfrsw.lib()


def _check(w, tag):
    from paper_2101_05617_amd import dfrsw
    G, D, Q = pair(w)
    P, B1, B2 = G.node_frames()
    _, hB = inputs.initial_state(w, P, B1, B2)
    zr, fr, ir = G.diagnostics(Q, hB=hB)
    z, f, it = dfrsw.dfr_diagnostics(D, to_dev(Q), zeta=True, fcor=True)
    z, f = to_host(z), to_host(f)
    ez = np.linalg.norm(z - zr) / np.linalg.norm(zr)
    ef = np.abs(f - fr).max() / np.abs(fr).max()
    ei = max(abs(a - b) / abs(b) for a, b in zip(it, ir))
    record(f"diag_{tag}_zeta", ez)
    record(f"diag_{tag}_integrals", ei)
    assert ez < 1e-12 and ef < 1e-14 and ei < 1e-13, (ez, ef, ei)
    return it


@pytest.mark.parametrize("ne,p", [(1, 1), (2, 2), (3, 4), (4, 4), (2, 5), (3, 6), (2, 7)])
def test_diagnostics_parity_zonal(ne, p):
    _check(small(C0, ne, p, u_amp=2.0), f"zonal_ne{ne}_p{p}")


def test_diagnostics_parity_jet_and_mountain():
    _check(small(C2, 5, 6), "jet_ne5_p6")
    _check(small(C4, 4, 6), "mountain_ne4_p6")


def test_diagnostics_parity_c1_full_size():
    _check(C1, "c1")


def test_diagnostics_invalid_state_and_null_outputs():
    from paper_2101_05617_amd import dfrsw
    G, D, Q = pair(small(C0, 2, 3))
    z, f, it = dfrsw.dfr_diagnostics(D, to_dev(Q), zeta=False, fcor=False)
    assert z is None and f is None and it[0] > 0
    Q[7] = -1.0
    with pytest.raises(dfrsw.DfrError) as e:
        dfrsw.dfr_diagnostics(D, to_dev(Q))
    assert e.value.code == -5
    Q[7] = np.nan
    with pytest.raises(dfrsw.DfrError) as e:
        dfrsw.dfr_diagnostics(D, to_dev(Q))
    assert e.value.code == -4


def test_mass_conserved_over_epi_steps_on_gpu():
    # Sec. 5.4: the normalised mass change (Eq. 44) stays at round-off over
    # EPI steps; energy and enstrophy change by far more but stay small
    from paper_2101_05617_amd import dfrsw
    w = small(C1, 8)
    G, D, Q = pair(w)
    st = dfrsw.epi_create(D, w.order, w.dt_nd, to_dev(Q), startup_substeps=2)
    _, _, i0 = dfrsw.dfr_diagnostics(D, to_dev(Q), zeta=False)
    for _ in range(6):
        dfrsw.epi_step(D, st, dfrsw.kiops_opts(tol=w.tol, m_max=w.m_max))
    _, _, i1 = dfrsw.dfr_diagnostics(D, dfrsw.epi_get_state(st), zeta=False)
    dm = abs(i1[0] - i0[0]) / i0[0]
    de = abs(i1[1] - i0[1]) / i0[1]
    record("diag_epi_mass_change", dm)
    record("diag_epi_energy_change", de)
    assert dm < 1e-13 and de < 1e-4
