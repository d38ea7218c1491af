"""Pins for the stage-level oracle functions (band reduction, bulge chase,
bidiagonal singular values) against mathematics and LAPACK, not against themselves."""
import numpy as np
import pytest
import scipy.linalg.lapack as lapack

import oracle
import workloads

U = 2.0 ** -53


def _band_mask(n, tile):
    i, j = np.indices((n, n))
    return (j >= i) & (j - i <= tile)


@pytest.mark.parametrize("m,n,tile", [(64, 64, 8), (96, 70, 16), (100, 100, 32), (77, 77, 32), (33, 33, 64)])
def test_band_reduce_structure_and_orthogonality(m, n, tile):
    a = workloads.gaussian(m, n, cfg_id=80, dtype="float64")
    band, u, v, w = oracle.band_reduce(a, tile, return_uv=True)
    # exact zeros outside the band
    assert np.all(band[~_band_mask(n, tile)] == 0.0)
    # U^T A V = [B; 0] with U, V orthogonal (independent of how the reflectors were applied)
    assert np.max(np.abs(u.T @ u - np.eye(m))) <= 20 * m * U
    assert np.max(np.abs(v.T @ v - np.eye(n))) <= 20 * n * U
    full = np.zeros((m, n))
    full[:n, :n] = band
    assert np.max(np.abs(u.T @ a @ v - full)) <= 20 * m * U * np.linalg.norm(a, 2)
    # first R entry is +-|A[:,0]|, and the Frobenius norm is preserved
    assert abs(abs(band[0, 0]) - np.linalg.norm(a[:, 0])) <= 4 * m * U * np.linalg.norm(a[:, 0])
    assert abs(np.linalg.norm(band) - np.linalg.norm(a)) <= 10 * m * U * np.linalg.norm(a)


def test_band_reduce_r_factors_match_lapack_qr():
    # The first QR sweep is a Householder QR of the first tile column: its R must equal
    # LAPACK's R of that panel up to row signs.
    a = workloads.gaussian(90, 90, cfg_id=81, dtype="float64")
    tile = 16
    band = oracle.band_reduce(a, tile)
    r = np.linalg.qr(a[:, :tile], mode="r")
    assert np.allclose(np.abs(band[:tile, :tile]), np.abs(np.triu(r)), rtol=0, atol=1e-13 * np.linalg.norm(a))


@pytest.mark.parametrize("tile", [4, 16, 32])
def test_band_preserves_singular_values(tile):
    a = workloads.cfg0_matrix()[:128, :128]
    s = oracle.svd_values(a)
    band = oracle.band_reduce(a, tile)
    assert np.max(np.abs(oracle.svd_values(band) - s)) <= 1e-13 * s[0]


@pytest.mark.parametrize("n,tile", [(50, 4), (64, 16), (97, 16), (130, 32), (40, 64)])
def test_bulge_chase_structure_and_values(n, tile):
    a = workloads.gaussian(n, n, cfg_id=82, dtype="float64")
    band = oracle.band_reduce(a, tile)
    d, e, bm = oracle.bulge_chase(band, tile, return_matrix=True)
    i, j = np.indices((n, n))
    off = (j != i) & (j != i + 1)
    assert np.max(np.abs(bm[off])) == 0.0
    s = oracle.svd_values(band)
    sb = oracle.bidiag_values(d, e)
    assert np.max(np.abs(sb - s)) <= 1e-13 * s[0]
    # column 0 is never touched by a right reflector and holds a single entry: |d0| is exact.
    assert abs(d[0]) == abs(band[0, 0])
    # Frobenius norm preserved
    assert abs(np.sqrt(np.sum(d * d) + np.sum(e * e)) - np.linalg.norm(band)) <= 10 * n * U * np.linalg.norm(band)


@pytest.mark.parametrize("n,tile", [(60, 8), (128, 32)])
def test_bulge_chase_matches_golub_kahan_up_to_signs(n, tile):
    # V e1 = e1 for every transform of both stages, so by the uniqueness of the Golub-Kahan
    # bidiagonal for a given first column of V, |d| and |e| equal those of the one-stage
    # Householder bidiagonalisation (diagnostic bound: rounding amplified by the Lanczos chain).
    a = workloads.gaussian(n, n, cfg_id=83, dtype="float64")
    band = oracle.band_reduce(a, tile)
    d, e = oracle.bulge_chase(band, tile)
    dg, eg = oracle.golub_kahan(a)
    scale = np.linalg.norm(a, 2)
    assert np.max(np.abs(np.abs(d) - np.abs(dg))) <= 1e-9 * scale
    assert np.max(np.abs(np.abs(e) - np.abs(eg))) <= 1e-9 * scale


def test_golub_kahan_values():
    a = workloads.gaussian(70, 50, cfg_id=84, dtype="float64")
    d, e = oracle.golub_kahan(a)
    s = np.linalg.svd(a, compute_uv=False)
    assert np.max(np.abs(oracle.bidiag_values(d, e) - s)) <= 1e-13 * s[0]


def _tgk_values(d, e):
    """Singular values via LAPACK dstebz (bisection) on the Golub-Kahan tridiagonal."""
    n = d.size
    off = np.zeros(2 * n - 1)
    off[0::2] = d
    off[1::2] = e
    m, w, _, _, info = lapack.dstebz(np.zeros(2 * n), off, 2, 0.0, 0.0, n + 1, 2 * n, 0.0, b"E")
    assert info == 0 and m == n
    return np.sort(np.abs(w[:n]))[::-1]


def test_bidiag_values_against_dstebz_and_special_cases():
    rng = np.random.default_rng(7)
    for n in (1, 2, 5, 40, 200):
        d = rng.standard_normal(n)
        e = rng.standard_normal(max(n - 1, 0))
        s = oracle.bidiag_values(d, e)
        assert np.max(np.abs(s - _tgk_values(d, e))) <= 4 * n * U * s[0] * 4
    d = rng.standard_normal(30)
    assert np.array_equal(oracle.bidiag_values(d, np.zeros(29)), np.sort(np.abs(d))[::-1])
    assert np.array_equal(oracle.bidiag_values(np.ones(10), np.zeros(9)), np.ones(10))


def test_band_reduce_ragged_and_wide():
    a = workloads.gaussian(45, 70, cfg_id=85, dtype="float64")
    s = oracle.svd_values(a)
    band = oracle.band_reduce(a, 16)
    assert band.shape == (45, 45)
    assert np.max(np.abs(oracle.svd_values(band) - s)) <= 1e-13 * s[0]
