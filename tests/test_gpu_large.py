"""GPU checks at n = 16384, the largest size the tuner measures, with the library's
default (tuned) configuration for that size.

The float64 oracle does not finish at this size, so the checks use what holds at
any size: a matrix built with known singular values (a diagonal between products
of Householder reflectors, formed in float64 on the host), and for a dense
N(0, 1) matrix the Frobenius identity sum(sigma^2) = ||A||_F^2 together with the
order, sign and finiteness of the values.
"""
import numpy as np
import pytest

import workloads
from gpu_util import banner, sigma_errors, torch_cuda

pytestmark = pytest.mark.gpu

N = 16384


def _svdv():
    import paper_2608_21227_amd as svdv
    return svdv


def _known(n: int, dtype: str):
    """(A, s): A = H1 H2 diag(s) H3 H4 with s geometric from 1 to 1e-3 and H_i = I - 2 v v^T / v^T v
    for N(0, 1) vectors v (seeded); the singular values of A are s."""
    rng = np.random.default_rng(2026_16384)
    s = np.geomspace(1.0, 1e-3, n)
    a = np.diag(s)
    for side in ("left", "left", "right", "right"):
        v = rng.standard_normal(n)
        v /= np.linalg.norm(v)
        if side == "left":
            a -= 2.0 * np.outer(v, v @ a)
        else:
            a -= 2.0 * np.outer(a @ v, v)
    return workloads.as_dtype(a, dtype), s


def _run(torch, svdv, a):
    dev = torch.from_numpy(np.ascontiguousarray(a.T)).t().cuda()
    s = svdv.svd_values(dev).cpu().numpy().astype(np.float64)
    del dev
    torch.cuda.empty_cache()
    return s


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_known_spectrum_n16384(dtype):
    torch = torch_cuda()
    svdv = _svdv()
    a, want = _known(N, dtype)
    banner(f"n={N} {dtype} known spectrum, default configuration {svdv.default_config(N, N, dtype)}")
    got = _run(torch, svdv, a)
    assert np.all(np.isfinite(got)) and np.all(got >= 0) and np.all(np.diff(got) <= 0)
    nw, _ = sigma_errors(got, want)
    # float32: the input's own rounding moves the values by about u32 ||A||_2 times a
    # small factor; float64: the Z14 gate
    assert nw <= (1e-5 if dtype == "float32" else 1e-12), f"normwise {nw:.3e}"


def test_frobenius_identity_dense_n16384_float32():
    torch = torch_cuda()
    svdv = _svdv()
    a = workloads.cfg1_matrix(N, "float32")
    fro2 = float(np.sum(np.square(a, dtype=np.float64)))
    banner(f"n={N} float32 dense N(0,1), default configuration {svdv.default_config(N, N, 'float32')}")
    got = _run(torch, svdv, a)
    assert np.all(np.isfinite(got)) and np.all(got >= 0) and np.all(np.diff(got) <= 0)
    assert abs(np.sum(got ** 2) - fro2) <= 1e-5 * fro2
    # the largest value of a square N(0, 1) matrix is close to 2 sqrt(n)
    assert abs(got[0] / np.sqrt(N) - 2.0) < 0.05
