"""GPU parity of the configurations the headline number is measured with.

Dense N(0, 1) matrices of n = 1024, 2048 and 4096 (float32 and float64, the
dense square workload of the evaluation) through the C-ABI, against the float64
oracle's singular values stored in ``tests/golden/`` (written by
``tests/golden/make_golden.py``, which calls only the oracle).  At n = 2048 and
4096 the float32 tile-16 path runs its multi-chunk panel tree (more than 2048
rows per panel) and the 1024-thread register strip of the trailing update on
panels of 513 to 2048 rows; the library default and the tuned table's
configurations are both checked.
"""
import os

import numpy as np
import pytest

import workloads
from gpu_util import banner, gate, to_dev, torch_cuda, valid_config

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _svdv():
    import paper_2608_21227_amd as svdv
    return svdv


def _golden(n, dtype):
    path = os.path.join(GOLDEN, f"cfg1_n{n}_{dtype}.npy")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written")
    return np.load(path)


def _run(n, dtype, cfg, label):
    torch = torch_cuda()
    svdv = _svdv()
    ref = _golden(n, dtype)
    a = workloads.cfg1_matrix(n, dtype)
    banner(f"headline-path {dtype} n={n} {label} {cfg}")
    s = svdv.svd_values(to_dev(a, torch, fortran=True), config=cfg)
    torch.cuda.synchronize()
    got = s.cpu().numpy()
    assert got.shape == (n,)
    assert np.all(np.isfinite(got))
    assert np.all(np.diff(got.astype(np.float64)) <= 0), "values must be descending"
    nw, rel = gate(dtype, got, ref)
    print(f"[gpu-case] {dtype} n={n} {label}: normwise {nw:.3e}, max relative {rel:.3e}", flush=True)
    return got


# the library's own default (what svd_values() runs without a configuration)
@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("n", [1024, 2048, 4096])
def test_default_config_matches_golden(n, dtype):
    _run(n, dtype, None, "library default")


# the tuned configurations the bench times (tile 16 at the measured thread counts)
TUNED = {"float32": dict(tile=16, threads=1024, inner_block=1, sweep_width=4),
         "float64": dict(tile=16, threads=512, inner_block=1, sweep_width=6)}


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("n", [2048, 4096])
def test_tuned_config_matches_golden(n, dtype):
    svdv = _svdv()
    cfg = svdv.Config(**TUNED[dtype])
    assert svdv.check_config(n, n, dtype, cfg), f"tuned configuration {cfg} rejected"
    _run(n, dtype, cfg, "tuned")


def test_tuned_table_config_matches_golden():
    """Whatever the committed tuned table holds for the headline cell."""
    svdv = _svdv()
    from paper_2608_21227_amd import tuner
    cfg = tuner.lookup(tuner.load_table(), 4096, "float32")
    if cfg is None:
        pytest.skip("no tuned entry for n=4096 float32")
    _run(4096, "float32", cfg, "tuned table")


# every other tile of the space at n = 1024, with a configuration the library accepts
@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("tile", [32, 64, 128])
def test_other_tiles_match_golden(tile, dtype):
    svdv = _svdv()
    cfg = valid_config(svdv, 1024, 1024, dtype, tile, sweep_width=2)
    if cfg is None:
        pytest.skip(f"no {dtype} configuration is built for tile {tile}")
    _run(1024, dtype, cfg, f"tile {tile}")


def test_default_and_tuned_agree_bitwise_across_calls():
    """The same configuration twice on the same input gives bitwise the same values."""
    torch = torch_cuda()
    svdv = _svdv()
    a = to_dev(workloads.cfg1_matrix(2048, "float32"), torch, fortran=True)
    cfg = svdv.Config(**TUNED["float32"])
    banner("headline-path float32 n=2048 repeatability")
    s1 = svdv.svd_values(a, config=cfg).cpu().numpy()
    s2 = svdv.svd_values(a, config=cfg).cpu().numpy()
    assert np.array_equal(s1, s2)
