"""GPU: the library's streaming-copy measurement helper (dfr_stream_copy)
copies exactly, refuses misaligned or ragged sizes, and reaches a plausible
fraction of the published HBM peak over 2 GiB."""
import ctypes

import pytest

from tests.gpu_util import torch_dev

pytestmark = pytest.mark.gpu


def test_stream_copy_exact_and_argument_checks():
    import torch
    from paper_2101_05617_amd import dfrsw
    torch_dev()
    for n in (1, 2, 3, 511, 512, 513, 1 << 20, (1 << 20) + 7):
        a = torch.randn(2 * n, dtype=torch.float64, device="cuda")    # 16 * n bytes
        b = torch.zeros_like(a)
        dfrsw.dfr_stream_copy(a, b)
        torch.cuda.synchronize()
        assert torch.equal(a, b), n
    a = torch.zeros(64, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    L = dfrsw.lib()
    for src, dst, nb in ((a.data_ptr() + 8, b.data_ptr(), 256), (a.data_ptr(), b.data_ptr() + 8, 256),
                         (a.data_ptr(), b.data_ptr(), 100), (0, b.data_ptr(), 256)):
        rc = L.dfr_stream_copy(ctypes.c_void_p(src), ctypes.c_void_p(dst), nb, None)
        assert rc == -1, (src, dst, nb)
    assert L.dfr_stream_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), 0, None) == 0


def test_stream_copy_bandwidth_is_plausible():
    import bench
    gbs = bench.measured_copy_gbs()
    print(f"dfr_stream_copy over 2 GiB: {gbs:.0f} GB/s")
    assert 0.3 * bench.HBM_PEAK_GBS < gbs < bench.HBM_PEAK_GBS
