"""Calls on different streams of one GPU overlap: each stream has its own workspace
(progress and ticket counters included), and a bulge chase waits only for sweep
groups that already hold a ticket in its own launch, so two persistent chases in
flight at once cannot block each other.  Overlapped calls must return bitwise the
values of the same calls made one after another."""
import numpy as np
import pytest

import workloads
from gpu_util import banner, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def test_calls_on_two_streams_overlap_and_match_sequential_calls():
    torch = torch_cuda()
    import paper_2608_21227_amd as svdv
    a = workloads.as_dtype(workloads.gaussian(1000, 1000, cfg_id=95, dtype="float32"), "float32")
    b = workloads.gaussian(700, 900, cfg_id=96, dtype="float64")
    da, db = to_dev(a, torch, fortran=True), to_dev(b, torch, fortran=True)
    banner("sequential reference calls (default stream)")
    ref_a = svdv.svd_values(da).cpu().numpy()
    ref_b = svdv.svd_values(db).cpu().numpy()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()  # default priority
    torch.cuda.synchronize()
    banner("overlapped calls on two streams, three rounds")
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            oa = svdv.svd_values(da)
        with torch.cuda.stream(s2):
            ob = svdv.svd_values(db)
        outs.append((oa, ob))
    torch.cuda.synchronize()
    for oa, ob in outs:
        assert np.array_equal(oa.cpu().numpy(), ref_a)
        assert np.array_equal(ob.cpu().numpy(), ref_b)
