"""Batched singular values: every stage runs once for the whole batch (per-matrix
argument tables), captured in a hipGraph and replayed; each matrix checked
against the float64 oracle with the single-matrix gates."""
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import banner, gate, torch_cuda

pytestmark = pytest.mark.gpu


def _svdv():
    import paper_2608_21227_amd as svdv
    return svdv


def _batch(count, lo, hi, dtype, seed):
    """Uneven shapes, some rectangular both ways, with known log-uniform spectra."""
    rng = np.random.default_rng(seed)
    mats = []
    for i in range(count):
        n = int(rng.integers(lo, hi + 1))
        m = n if i % 3 else int(rng.integers(lo, hi + 1))
        k = min(m, n)
        s = np.sort(10.0 ** rng.uniform(-4, 0, k))[::-1]
        mats.append(workloads.as_dtype(workloads.known_spectrum(m, n, s, cfg_id=2, dtype=dtype, idx=seed * 1000 + i),
                                       dtype))
    return mats


def _check(mats, packed, offs, dtype):
    got = packed.cpu().numpy().astype(np.float64)
    for a, off in zip(mats, offs):
        k = min(a.shape)
        ref = oracle.svd_values(a)
        gate(dtype, got[off:off + k], ref)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_batched_uneven_sizes_and_replays(dtype):
    torch = torch_cuda()
    svdv = _svdv()
    mats = _batch(24, 1, 160, dtype, seed=5)
    mats[3] = mats[3][:1, :1].copy()   # a 1 x 1 matrix
    mats[7] = mats[7][:2, :].copy()    # a 2-row matrix (wide)
    devs = [torch.from_numpy(np.ascontiguousarray(a.T)).t().cuda() for a in mats]
    banner(f"batched {dtype} count={len(mats)} (capture)")
    packed, offs = svdv.svd_values_batched(devs)
    torch.cuda.synchronize()
    _check(mats, packed, offs, dtype)
    # replays of the captured graph, with other GPU work in between, each checked
    out = packed
    for r in range(3):
        banner(f"batched {dtype} replay {r}")
        junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
        out.fill_(-1)
        packed2, _ = svdv.svd_values_batched(devs, out=out)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        _check(mats, packed2, offs, dtype)
    # same shapes, new data (the pointer table is refreshed)
    mats2 = [np.ascontiguousarray(0.5 * a[::-1, :]) for a in mats]  # other values and layout, same shapes
    devs2 = [torch.from_numpy(np.ascontiguousarray(a.T)).t().cuda() for a in mats2]
    banner(f"batched {dtype} new data")
    packed3, offs3 = svdv.svd_values_batched(devs2)
    torch.cuda.synchronize()
    _check(mats2, packed3, offs3, dtype)


def test_batched_matches_single_calls_bitwise():
    torch = torch_cuda()
    svdv = _svdv()
    mats = _batch(10, 16, 96, "float32", seed=9)
    devs = [torch.from_numpy(np.ascontiguousarray(a.T)).t().cuda() for a in mats]
    cfg = svdv.Config(tile=16, threads=1024, inner_block=1, sweep_width=2)
    banner("batched vs single, float32")
    packed, offs = svdv.svd_values_batched(devs, config=cfg)
    singles = [svdv.svd_values(d, config=cfg) for d in devs]
    torch.cuda.synchronize()
    got = packed.cpu().numpy()
    for s1, off in zip(singles, offs):
        s1 = s1.cpu().numpy()
        assert np.array_equal(got[off:off + s1.size], s1)  # same kernels, same arithmetic


def test_batched_fallback_configuration():
    torch = torch_cuda()
    svdv = _svdv()
    mats = _batch(6, 8, 64, "float32", seed=11)
    devs = [torch.from_numpy(np.ascontiguousarray(a.T)).t().cuda() for a in mats]
    cfg = svdv.Config(tile=16, threads=256, inner_block=2, sweep_width=2)  # streaming update: one by one
    banner("batched fallback, float32")
    packed, offs = svdv.svd_values_batched(devs, config=cfg)
    torch.cuda.synchronize()
    _check(mats, packed, offs, "float32")


def test_batched_default_uses_each_matrix_tuned_configuration_bitwise():
    """Without a configuration the batch is grouped by the tuned configuration of
    each matrix's size; every matrix then equals a single call with its default."""
    torch = torch_cuda()
    svdv = _svdv()
    mats = _batch(12, 8, 300, "float32", seed=13)
    devs = [torch.from_numpy(np.ascontiguousarray(a.T)).t().cuda() for a in mats]
    banner("batched default configurations vs single calls, float32")
    packed, offs = svdv.svd_values_batched(devs)
    singles = [svdv.svd_values(d) for d in devs]
    torch.cuda.synchronize()
    got = packed.cpu().numpy()
    for s1, off in zip(singles, offs):
        s1 = s1.cpu().numpy()
        assert np.array_equal(got[off:off + s1.size], s1)


GOLDEN_CFG2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg2_b512_float32.npy")


def test_batched_workload_against_oracle_values():
    """The batched workload: 512 float32 matrices, n uniform in [32, 512], log-uniform
    spectra in [1e-4, 1]; every matrix against the stored float64 oracle values of
    exactly its rounded matrix (tests/golden/cfg2_b512_float32.npy), with the
    single-matrix gates."""
    if not os.path.exists(GOLDEN_CFG2):
        pytest.skip("cfg2 golden values not written")
    torch = torch_cuda()
    svdv = _svdv()
    mats, _ = workloads.cfg2_batch(512, 32, 512, "float32")
    ref_all = np.load(GOLDEN_CFG2)
    devs = [torch.from_numpy(np.ascontiguousarray(a.T)).t().cuda() for a in mats]
    banner("batched workload 512 x float32 n in [32, 512] vs oracle")
    packed, offs = svdv.svd_values_batched(devs)
    torch.cuda.synchronize()
    got = packed.cpu().numpy().astype(np.float64)
    assert ref_all.size == sum(min(a.shape) for a in mats)
    worst = 0.0
    pos = 0
    for a, off in zip(mats, offs):
        k = min(a.shape)
        ref = ref_all[pos:pos + k]
        pos += k
        nw, _ = gate("float32", got[off:off + k], ref)
        worst = max(worst, nw)
    print(f"[batched] 512 matrices: worst normwise error vs oracle {worst:.3e}", flush=True)
