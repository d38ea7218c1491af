"""The allocation-free entry point (svd_values_noalloc) against svd_values_ex.

svd_values_noalloc runs the same kernels on a fixed device array owned by the
library instead of an allocated workspace; its values must equal those of
svd_values_ex with the same configuration bitwise.  Two calls in a row, the
second on a smaller matrix (the array keeps the first call's contents), and a
size beyond the array's capacity that must be rejected without GPU work.
"""
import ctypes

import numpy as np
import pytest

import workloads
from gpu_util import banner, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _svdv():
    import paper_2608_21227_amd as svdv
    return svdv


def _call_noalloc(svdv, torch, a_dev, cfg):
    a2, m, n, lda = svdv._as_colmajor(a_dev)
    s = torch.empty(min(m, n), dtype=a_dev.dtype, device=a_dev.device)
    rc = svdv.lib().svd_values_noalloc(ctypes.c_void_p(a2.data_ptr()), m, n, lda, svdv._dtype_code(a_dev),
                                       ctypes.c_void_p(s.data_ptr()), svdv._stream(a_dev.device), svdv._cfg_ptr(cfg))
    return rc, s


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_noalloc_matches_allocating_entry_point(dtype):
    torch = torch_cuda()
    svdv = _svdv()
    cfg = svdv.default_config(1024, 1024, dtype)
    for (m, n) in [(1024, 1024), (300, 257)]:  # second call smaller than the first
        a = workloads.as_dtype(workloads.gaussian(m, n, cfg_id=75, dtype=dtype), dtype)
        dev = to_dev(a, torch, fortran=True)
        banner(f"noalloc {dtype} m={m} n={n} {cfg}")
        want = svdv.svd_values(dev, config=cfg)
        torch.cuda.synchronize()
        rc, got = _call_noalloc(svdv, torch, dev, cfg)
        assert rc == 0, svdv.lib().svdv_last_error().decode()
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want.cpu().numpy())


def test_noalloc_rejects_sizes_beyond_its_array():
    torch = torch_cuda()
    svdv = _svdv()
    cap = svdv.lib().svdv_noalloc_capacity()
    assert cap == 64 << 20
    n = 4200  # float64 workspace of a 4200 x 4200 matrix exceeds the array
    a = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    banner("noalloc oversize rejection")
    rc, _ = _call_noalloc(svdv, torch, a, None)
    assert rc == -2  # SVDV_ERR_UNSUPPORTED
    assert b"exceeds" in svdv.lib().svdv_last_error()
