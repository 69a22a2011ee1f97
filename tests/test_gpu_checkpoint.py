"""Checkpoint and restart of an EPI integration (epi_save / epi_load): a run
restarted from a checkpoint continues bit for bit like the uninterrupted run
(the same kernels and reduction orders on the same context), during the
EPI2 start-up and after it, in FP64 and in the mixed form; malformed
checkpoints and checkpoints of another grid are rejected."""
import numpy as np
import pytest

from paper_2101_05617_amd import inputs
from tests.gpu_util import pair, small, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

C1 = inputs.WORKLOADS["c1_ne30_p5"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch_dev()
    from paper_2101_05617_amd import dfrsw
    dfrsw.lib()


@pytest.mark.parametrize("save_after,prec", [(2, "fp64"), (5, "fp64"), (4, "fp32_jv")])
def test_restart_is_bitwise(save_after, prec):
    from paper_2101_05617_amd import dfrsw
    w = small(C1, 4)
    G, D, Q = pair(w)
    opts = dfrsw.kiops_opts(tol=w.tol, m_max=w.m_max)
    eps = 1e-150 if prec == "fp64" else 1e-20
    st = dfrsw.epi_create(D, w.order, w.dt_nd, to_dev(Q), startup_substeps=2, eps=eps, prec=prec)
    for _ in range(save_after):
        dfrsw.epi_step(D, st, opts)
    ck = dfrsw.epi_save(st)
    for _ in range(4):
        dfrsw.epi_step(D, st, opts)
    a = to_host(dfrsw.epi_get_state(st))
    r = dfrsw.epi_load(D, ck)
    assert dfrsw.lib().epi_num_steps(r.handle) == save_after
    for _ in range(4):
        dfrsw.epi_step(D, r, opts)
    b = to_host(dfrsw.epi_get_state(r))
    assert np.array_equal(a, b)
    assert dfrsw.lib().epi_num_steps(r.handle) == save_after + 4
    st.close()
    r.close()


def test_checkpoint_errors():
    from paper_2101_05617_amd import dfrsw
    w = small(C1, 3)
    G, D, Q = pair(w)
    st = dfrsw.epi_create(D, 4, w.dt_nd, to_dev(Q), startup_substeps=2)
    dfrsw.epi_step(D, st, dfrsw.kiops_opts(tol=w.tol, m_max=w.m_max))
    ck = dfrsw.epi_save(st)
    # another grid
    _, D2, _ = pair(small(C1, 2))
    with pytest.raises(dfrsw.DfrError) as e:
        dfrsw.epi_load(D2, ck)
    assert e.value.code == -1
    # truncated, corrupted
    for bad in (ck[:-8], b"XXXXXXXX" + ck[8:], ck[:16]):
        with pytest.raises(dfrsw.DfrError) as e:
            dfrsw.epi_load(D, bad)
        assert e.value.code == -1
    # a buffer that is too small for epi_save
    import ctypes
    n = ctypes.c_size_t(len(ck) - 1)
    buf = ctypes.create_string_buffer(len(ck))
    assert dfrsw.lib().epi_save(st.handle, buf, ctypes.byref(n)) == -1
    st.close()
