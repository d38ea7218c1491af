"""Helpers shared by the GPU tests (device tensors, error metrics, case banners)."""
import sys

import numpy as np
import pytest

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def banner(msg: str):
    """Print what the next GPU step runs (flushed, so a crash still names the case)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def valid_config(svdv, m, n, dtype, tile, sweep_width=1):
    """A runnable configuration for this tile: the first (threads, inner_block) pair
    in a fixed preference order that the library accepts."""
    for threads, ib in [(256, 2), (256, 1), (128, 2), (128, 1), (64, 1), (512, 1)]:
        for sw in (sweep_width, 2, 1):
            cfg = svdv.Config(tile=tile, threads=threads, inner_block=ib, sweep_width=sw)
            if svdv.check_config(m, n, dtype, cfg):
                return cfg
    return None


def to_dev(a: np.ndarray, torch, fortran: bool = False):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if fortran:
        t = torch.from_numpy(np.ascontiguousarray(a.T)).t()
    return t.cuda()


def sigma_errors(got: np.ndarray, ref: np.ndarray):
    """(normwise max|d|/sigma1, max relative per value over nonzero ref)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    s1 = ref[0] if ref.size and ref[0] > 0 else 1.0
    diff = np.abs(got - ref)
    nz = ref > 0
    rel = np.max(diff[nz] / ref[nz]) if np.any(nz) else 0.0
    return float(np.max(diff) / s1) if diff.size else 0.0, float(rel)


def gate(dtype: str, got, ref):
    """Parity gate: float64 normwise <= 1e-12; float32 per-value relative <= 1e-5 * cond."""
    nw, rel = sigma_errors(got, ref)
    if dtype == "float64":
        assert nw <= 1e-12, f"float64 normwise error {nw:.3e} > 1e-12"
    else:
        cond = ref[0] / ref[-1] if ref[-1] > 0 else np.inf
        assert rel <= 1e-5 * cond, f"float32 relative error {rel:.3e} > 1e-5 * cond ({cond:.3e})"
        assert nw <= 1e-5, f"float32 normwise error {nw:.3e} > 1e-5"
    return nw, rel
