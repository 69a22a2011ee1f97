"""The allocation-free complex-step product (dfr_jvp_complex_step_noalloc),
through the C ABI, against dfr_jvp_complex_step on the same inputs: two calls
in a row on two grids, the second smaller, in complex FP32 (its FP32 copy of
q in the library's device scratch array) and FP64.  Both entry points run
the same kernels on the same values, so the results must agree bit for bit
(well inside the bars of the product's parity tests); the FP32 results are
also held to the product's FP32 bar against the oracle.  A grid beyond the
array's size is refused with DFR_E_INVAL, and the refusal leaves the
array's last contents in use by nobody: a following call is still exact."""
import numpy as np
import pytest

from paper_2101_05617_amd import inputs
from tests.gpu_util import check_fields, pair, small, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

C0 = inputs.WORKLOADS["c0_ne4_p4"]
C1 = inputs.WORKLOADS["c1_ne30_p5"]


def _one(w, seed):
    import torch
    from paper_2101_05617_amd import dfrsw
    G, D, Q = pair(w)
    V = inputs.random_direction(3 * G.N, seed)
    q, v = to_dev(Q), to_dev(V)
    ref_o = G.jvp(Q, V)
    for prec, eps in (("fp32_jv", 1e-20), ("fp64", 1e-150)):
        a = to_host(dfrsw.dfr_jvp_complex_step(D, q, v, eps, prec))
        out = torch.full((3 * G.N,), float("nan"), dtype=torch.float64, device="cuda")
        b = to_host(dfrsw.dfr_jvp_complex_step_noalloc(D, q, v, out, eps, prec))
        dfrsw.dfr_sync(D)
        assert np.array_equal(a, b), (w.name, w.ne, prec, np.abs(a - b).max())
        check_fields(b, ref_o, G, 2e-5 if prec == "fp32_jv" else 1e-12)
    D.close()


def test_noalloc_product_matches_the_allocating_entry_point():
    torch_dev()
    # ne = 30, p = 5 (194,400 nodes), then ne = 4, p = 4 (2,400 nodes)
    _one(C1, 11)
    _one(small(C0, 4, 4, u_amp=2.0), 12)


def test_noalloc_product_refuses_grids_beyond_its_scratch():
    torch_dev()
    import torch
    from paper_2101_05617_amd import dfrsw
    # ne = 80, p = 6: 1,881,600 nodes, 22.6 MB of FP32 state > 16 MiB
    D = dfrsw.Grid(80, 6, *C0.constants())
    n3 = 3 * D.N
    q = torch.ones(n3, dtype=torch.float64, device="cuda")
    v = torch.zeros(n3, dtype=torch.float64, device="cuda")
    out = torch.empty(n3, dtype=torch.float64, device="cuda")
    with pytest.raises(dfrsw.DfrError) as e:
        dfrsw.dfr_jvp_complex_step_noalloc(D, q, v, out, 1e-20, "fp32_jv")
    assert e.value.code == -1 and "1398101 nodes" in str(e.value)
    D.close()
    del q, v, out
    torch.cuda.synchronize()
    _one(small(C0, 3, 6, u_amp=1.0), 13)
