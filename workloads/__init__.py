"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws matrices; it contains none of the singular-value
arithmetic.  Every matrix is generated in float64 and, for float32 workloads,
rounded once with ``astype(float32)`` (round to nearest even).  Whoever checks a
float32 result must compare against the singular values of that *rounded*
matrix, which is what :func:`as_dtype` returns.

Workload families (sizes and spectra follow the evaluation section of the paper
for the dense square case and the project's own forms for the rest):

* ``known_spectrum``  A = U diag(s) V^T with Haar-distributed U, V.
* ``gaussian``        i.i.d. N(0, 1) entries.
* ``batch``           many square matrices with log-uniform known spectra.

Seeds: ``np.random.SeedSequence(ROOT_SEED, spawn_key=(cfg_id, n, dtype_code, idx))``
with independent children for G (Gaussian draws), U and V.
"""
from __future__ import annotations

import numpy as np

ROOT_SEED = 260821227
DTYPE_CODES = {"float32": 0, "float64": 1}


def _seq(cfg_id: int, n: int, dtype: str, idx: int = 0) -> np.random.SeedSequence:
    return np.random.SeedSequence(ROOT_SEED, spawn_key=(int(cfg_id), int(n), DTYPE_CODES[dtype], int(idx)))


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: Q of QR(G) with the signs of diag(R) folded in."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    sgn = np.sign(np.diag(r))
    sgn[sgn == 0] = 1.0
    return q * sgn[None, :]


def known_spectrum(m: int, n: int, s: np.ndarray, cfg_id: int, dtype: str, idx: int = 0) -> np.ndarray:
    """float64 matrix U[:, :k] diag(s) V[:, :k]^T with k = min(m, n) = len(s)."""
    k = min(m, n)
    s = np.asarray(s, dtype=np.float64)
    assert s.shape == (k,)
    children = _seq(cfg_id, max(m, n), dtype, idx).spawn(3)
    u = haar_orthogonal(m, np.random.default_rng(children[1]))[:, :k]
    v = haar_orthogonal(n, np.random.default_rng(children[2]))[:, :k]
    return (u * s[None, :]) @ v.T


def geometric_spectrum(k: int, lo: float) -> np.ndarray:
    """s_i = lo^(i/(k-1)), i = 0..k-1: from 1 down to lo (descending)."""
    if k == 1:
        return np.ones(1)
    return lo ** (np.arange(k, dtype=np.float64) / (k - 1))


def gaussian(m: int, n: int, cfg_id: int, dtype: str, idx: int = 0) -> np.ndarray:
    children = _seq(cfg_id, max(m, n), dtype, idx).spawn(3)
    return np.random.default_rng(children[0]).standard_normal((m, n))


def as_dtype(a: np.ndarray, dtype: str) -> np.ndarray:
    """Round to the working dtype (the matrix every checker must use)."""
    return np.ascontiguousarray(a.astype(np.float32 if dtype == "float32" else np.float64))


# --------------------------------------------------------------------------
# The workload configurations used by the tests and the bench.
# --------------------------------------------------------------------------

def cfg0_matrix() -> np.ndarray:
    """256x256 float64, A = U diag(s) V^T, s geometric from 1 to 1e-3."""
    n = 256
    return known_spectrum(n, n, geometric_spectrum(n, 1e-3), cfg_id=0, dtype="float64")


def cfg0_spectrum() -> np.ndarray:
    return geometric_spectrum(256, 1e-3)


def cfg1_matrix(n: int, dtype: str) -> np.ndarray:
    """Square dense n x n, i.i.d. N(0,1), rounded to dtype."""
    return as_dtype(gaussian(n, n, cfg_id=1, dtype=dtype), dtype)


def cfg2_batch(count: int = 512, lo: int = 32, hi: int = 512, dtype: str = "float32"):
    """Uneven batch: sizes uniform in [lo, hi], spectra log-uniform in [1e-4, 1].

    Returns (list of matrices rounded to dtype, list of float64 spectra)."""
    root = np.random.default_rng(_seq(2, count, dtype, 0))
    sizes = root.integers(lo, hi + 1, size=count)
    mats, spectra = [], []
    for i, n in enumerate(sizes):
        rng = np.random.default_rng(_seq(2, int(n), dtype, i + 1).spawn(1)[0])
        s = np.sort(10.0 ** rng.uniform(-4.0, 0.0, size=int(n)))[::-1].copy()
        mats.append(as_dtype(known_spectrum(int(n), int(n), s, cfg_id=2, dtype=dtype, idx=i + 1), dtype))
        spectra.append(s)
    return mats, spectra


def cfg3_matrix(n: int = 8192, dtype: str = "float32") -> np.ndarray:
    """n x n, A = U diag(s) V^T with s geometric from 1 to 1e-4 (cond 1e4)."""
    return as_dtype(known_spectrum(n, n, geometric_spectrum(n, 1e-4), cfg_id=3, dtype=dtype), dtype)


def cfg3_spectrum(n: int = 8192) -> np.ndarray:
    return geometric_spectrum(n, 1e-4)
