"""CPU oracle for the two-stage singular-value method -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU path
(``paper_2608_21227_amd``) and imports nothing from it.

Everything here is float64 and deliberately plain: reflectors are applied one
at a time, with no blocking, tiling or reordering beyond what the steps below
state.

* :func:`svd_values`   -- the result the whole method reaches: the singular
  values of A (the transforms of the two-stage method are orthogonal, so they
  leave the singular values unchanged -- evaluation section, "Algorithm").
  One-sided Jacobi in C (``jacobi.c``).
* :func:`band_reduce`  -- stage 1, Algorithm 1: for each diagonal tile k, a QR
  sweep on the tile column and an LQ sweep on the tile row, each followed by
  the trailing update; the result is upper banded with bandwidth = tile size.
* :func:`bulge_chase`  -- stage 2, band -> bidiagonal.  The paper only names
  this step; the reading taken is Householder bulge chasing, one sweep per row,
  each sweep a chain of (right reflector, left reflector) pairs.
* :func:`bidiag_values` -- stage 3, bidiagonal -> singular values (Jacobi on
  the dense bidiagonal).
* :func:`golub_kahan`  -- one-stage Householder bidiagonalisation, used only as
  a cross-check of stage 2 (uniqueness of the Golub-Kahan bidiagonal).
* :func:`householder`  -- the reflector convention (LAPACK ``dlarfg``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``jacobi.c`` into ``liboracle.so`` with gcc + OpenMP."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
               os.path.join(_HERE, "jacobi.c"), "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_svd_values.restype = ctypes.c_int
        lib.oracle_svd_values.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
            ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def svd_values(a, threads: int = 0, max_sweeps: int = 60, info: dict | None = None) -> np.ndarray:
    """Singular values of ``a`` (any real dtype, promoted exactly to float64), descending."""
    a = np.asarray(a)
    if a.ndim != 2:
        raise ValueError("expected a matrix")
    a64 = np.asfortranarray(a.astype(np.float64))
    m, n = a64.shape
    k = min(m, n)
    out = np.zeros(k, dtype=np.float64)
    if k == 0:
        return out
    sweeps = ctypes.c_int(0)
    off = ctypes.c_double(0.0)
    rc = _load().oracle_svd_values(a64.ctypes.data, m, n, max(1, m), out.ctypes.data,
                                   max_sweeps, threads, ctypes.byref(sweeps), ctypes.byref(off))
    if info is not None:
        info.update(sweeps=sweeps.value, offmax=off.value, rc=rc)
    if rc == -2:
        raise OracleError("non-finite input")
    if rc == -3:
        raise OracleError(f"Jacobi did not converge in {max_sweeps} sweeps (max rel. off {off.value:.3e})")
    if rc != 0:
        raise OracleError(f"oracle failed with code {rc}")
    return out


# ---------------------------------------------------------------------------
# Householder reflector (dlarfg convention)
# ---------------------------------------------------------------------------

def householder(x: np.ndarray):
    """Reflector H = I - tau v v^T with H x = beta e_1 and v[0] = 1.

    beta = -sign(alpha) * ||x|| (sign(0) = +1), tau = (beta - alpha) / beta,
    v[1:] = x[1:] / (alpha - beta).  A zero tail gives tau = 0 (H = I) and
    beta = alpha.
    """
    x = np.asarray(x, dtype=np.float64)
    alpha = x[0]
    v = np.zeros_like(x)
    v[0] = 1.0
    tail = x[1:]
    xnorm = np.sqrt(np.dot(tail, tail)) if tail.size else 0.0
    if xnorm == 0.0:
        return v, 0.0, alpha
    beta = -np.copysign(np.hypot(alpha, xnorm), alpha if alpha != 0.0 else 1.0)
    tau = (beta - alpha) / beta
    v[1:] = tail / (alpha - beta)
    return v, tau, beta


# ---------------------------------------------------------------------------
# Stage 1: Algorithm 1, reduction to band form (bandwidth = tile size)
# ---------------------------------------------------------------------------

def band_reduce(a, tile: int, return_uv: bool = False):
    """Reduce ``a`` (m x n; transposed first if m < n) to upper band form.

    For each diagonal tile k (Algorithm 1):
      QR sweep -- Householder QR of the tile column W[k*TS:, k*TS:(k+1)*TS],
                  each reflector applied to the trailing matrix from the left;
      LQ sweep -- Householder LQ of the tile row W[k*TS:(k+1)*TS, (k+1)*TS:],
                  each reflector applied to the trailing matrix from the right.
    Returns the n x n band matrix B (B_ij = 0 unless 0 <= j - i <= tile),
    and with ``return_uv`` also U (m x m), V (n x n) with U^T W V = [B; 0].
    """
    w = np.array(a, dtype=np.float64, copy=True)
    if w.shape[0] < w.shape[1]:
        w = w.T.copy()
    m, n = w.shape
    u = np.eye(m) if return_uv else None
    vv = np.eye(n) if return_uv else None
    ntiles = (n + tile - 1) // tile
    for k in range(ntiles):
        r0 = c0 = k * tile
        bw = min(tile, n - c0)
        # QR sweep on the tile column (GEQRT/TSQRT) + trailing update (UNMQR/TSMQR).
        for j in range(bw):
            row, col = r0 + j, c0 + j
            if row >= m:
                break
            v, tau, beta = householder(w[row:, col])
            if tau != 0.0:
                blk = w[row:, col:]
                blk -= tau * np.outer(v, v @ blk)
                if return_uv:
                    uu = u[:, row:]
                    uu -= tau * np.outer(uu @ v, v)
            w[row, col] = beta
            w[row + 1:, col] = 0.0
        # LQ sweep on the tile row + trailing update from the right.
        c1 = c0 + tile
        for j in range(bw):
            row, col = r0 + j, c1 + j
            if col >= n:
                break
            v, tau, beta = householder(w[row, col:])
            if tau != 0.0:
                blk = w[row:, col:]
                blk -= tau * np.outer(blk @ v, v)
                if return_uv:
                    vb = vv[:, col:]
                    vb -= tau * np.outer(vb @ v, v)
            w[row, col] = beta
            w[row, col + 1:] = 0.0
    band = np.triu(np.tril(w[:n, :n], tile), 0)
    if return_uv:
        return band, u, vv, w
    return band


# ---------------------------------------------------------------------------
# Stage 2: band -> bidiagonal by Householder bulge chasing
# ---------------------------------------------------------------------------

def chase_task(bm: np.ndarray, p: int, c: int, tile: int) -> None:
    """One bulge-chasing step on the dense matrix ``bm`` (in place).

    Right reflector: annihilate row p beyond column c (columns c..c+L-1, the
    band edge plus the fill), applied to rows p..c+L-1.
    Left reflector: annihilate column c below the diagonal (rows c+1..c+L-1),
    applied to columns c..c+L+tile-1.  L = min(tile, n - c).
    """
    n = bm.shape[0]
    L = min(tile, n - c)
    r_end = min(c + L, n)
    v, tau, beta = householder(bm[p, c:c + L])
    if tau != 0.0:
        blk = bm[p:r_end, c:c + L]
        blk -= tau * np.outer(blk @ v, v)
    bm[p, c] = beta
    bm[p, c + 1:c + L] = 0.0
    c_end = min(c + L + tile, n)
    v, tau, beta = householder(bm[c:c + L, c])
    if tau != 0.0:
        blk = bm[c:c + L, c:c_end]
        blk -= tau * np.outer(v, v @ blk)
    bm[c, c] = beta
    bm[c + 1:c + L, c] = 0.0


def sweep_tasks(s: int, n: int, tile: int):
    """The (p, c) pairs of sweep s, in order: p_0 = s, c_0 = s + 1, then p <- c, c <- c + tile."""
    p, c = s, s + 1
    out = []
    while c < n:
        out.append((p, c))
        p, c = c, c + tile
    return out


def bulge_chase(band: np.ndarray, tile: int, return_matrix: bool = False):
    """Reduce an upper band matrix (bandwidth ``tile``) to upper bidiagonal form.

    Sweep s = 0..n-2 makes row s bidiagonal and chases the bulge it creates off
    the bottom of the matrix; sweeps run strictly one after another.
    Returns (d, e) with d = diag, e = superdiagonal.
    """
    bm = np.array(band, dtype=np.float64, copy=True)
    n = bm.shape[0]
    for s in range(n - 1):
        for p, c in sweep_tasks(s, n, tile):
            chase_task(bm, p, c, tile)
    d = np.diag(bm).copy()
    e = np.diag(bm, 1).copy()
    if return_matrix:
        return d, e, bm
    return d, e


# ---------------------------------------------------------------------------
# Stage 3 and diagnostics
# ---------------------------------------------------------------------------

def bidiag_matrix(d, e) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    n = d.size
    b = np.diag(d)
    if n > 1:
        b[np.arange(n - 1), np.arange(1, n)] = e
    return b


def bidiag_values(d, e, threads: int = 0) -> np.ndarray:
    """Singular values of the upper bidiagonal (d, e), descending (Jacobi on the dense matrix)."""
    return svd_values(bidiag_matrix(d, e), threads=threads)


def golub_kahan(a) -> tuple[np.ndarray, np.ndarray]:
    """One-stage Householder bidiagonalisation (diagnostic only): returns (d, e)."""
    w = np.array(a, dtype=np.float64, copy=True)
    if w.shape[0] < w.shape[1]:
        w = w.T.copy()
    m, n = w.shape
    for j in range(n):
        v, tau, beta = householder(w[j:, j])
        if tau != 0.0:
            blk = w[j:, j:]
            blk -= tau * np.outer(v, v @ blk)
        w[j, j] = beta
        w[j + 1:, j] = 0.0
        if j + 1 < n:
            v, tau, beta = householder(w[j, j + 1:])
            if tau != 0.0:
                blk = w[j:, j + 1:]
                blk -= tau * np.outer(blk @ v, v)
            w[j, j + 1] = beta
            w[j, j + 2:] = 0.0
    return np.diag(w[:n, :n]).copy(), np.diag(w[:n, :n], 1).copy()


def time_sweeps(a, sweeps: int, threads: int = 0) -> tuple[float, int]:
    """Wall time of the first ``sweeps`` Jacobi sweeps on ``a`` (bounded oracle timing sample).

    Returns (seconds, sweeps actually run).  Used only to time the oracle on a
    bounded sample; the values it would return are not used."""
    import time
    a64 = np.asfortranarray(np.asarray(a).astype(np.float64))
    m, n = a64.shape
    out = np.zeros(min(m, n), dtype=np.float64)
    done = ctypes.c_int(0)
    off = ctypes.c_double(0.0)
    t0 = time.perf_counter()
    _load().oracle_svd_values(a64.ctypes.data, m, n, max(1, m), out.ctypes.data, sweeps, threads,
                              ctypes.byref(done), ctypes.byref(off))
    return time.perf_counter() - t0, done.value
