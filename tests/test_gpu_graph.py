"""The allocation-free entry point under graph capture: one call captured after an
eager warm-up (which takes the fixed array's address), then replayed several times
with new data written into the captured input between replays and eager library
work in between; every replay must equal the allocating call on the same matrix
bitwise (same kernels, same configuration)."""
import numpy as np
import pytest

import workloads
from gpu_util import banner, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_noalloc_call_captured_in_a_graph_replays_correctly(dtype):
    torch = torch_cuda()
    import paper_2608_21227_amd as svdv
    n = 700
    mats = [workloads.as_dtype(workloads.gaussian(n, n, cfg_id=97, dtype=dtype, idx=i), dtype) for i in range(3)]
    banner(f"graph capture of svd_values_noalloc n={n} {dtype}: eager references")
    eager = [svdv.svd_values(to_dev(a, torch, fortran=True)).cpu().numpy() for a in mats]
    x = to_dev(mats[0], torch, fortran=True)  # the captured input (column-major view)
    out = torch.empty(n, dtype=x.dtype, device="cuda")
    side = torch.cuda.Stream()  # default priority
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        svdv.svd_values_noalloc(x, out)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    banner("capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        svdv.svd_values_noalloc(x, out)
    for r in range(6):
        i = (r + 1) % 3
        x.copy_(to_dev(mats[i], torch, fortran=True))
        torch.cuda.synchronize()
        banner(f"replay {r} (matrix {i})")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager[i]), f"replay {r}"
        svdv.svd_values(to_dev(mats[(i + 1) % 3], torch, fortran=True))  # eager work between replays
        torch.cuda.synchronize()
