"""Pins for the CPU oracle: every check compares it with something other than itself
(closed forms, invariants, exact special cases, LAPACK routines, brute force)."""
import math

import numpy as np
import pytest
import scipy.linalg.lapack as lapack

import oracle
import workloads

U = 2.0 ** -53


# ----------------------------- P1: known spectra -----------------------------

@pytest.mark.parametrize("n", [8, 33, 128, 256])
def test_known_spectrum(n):
    s = workloads.geometric_spectrum(n, 1e-3)
    a = workloads.known_spectrum(n, n, s, cfg_id=90, dtype="float64")
    sig = oracle.svd_values(a)
    assert np.max(np.abs(sig - s)) <= 10 * n * U * s[0]


def test_cfg0_matrix_matches_its_spectrum():
    sig = oracle.svd_values(workloads.cfg0_matrix())
    s = workloads.cfg0_spectrum()
    assert np.max(np.abs(sig - s)) <= 10 * 256 * U


@pytest.mark.parametrize("m,n", [(40, 25), (25, 40)])
def test_known_spectrum_rectangular(m, n):
    k = min(m, n)
    s = np.linspace(3.0, 0.5, k)
    a = workloads.known_spectrum(m, n, s, cfg_id=91, dtype="float64")
    assert np.max(np.abs(oracle.svd_values(a) - s)) <= 10 * max(m, n) * U * 3.0


# ----------------------------- P2: invariants --------------------------------

def test_frobenius_identity():
    a = workloads.gaussian(120, 90, cfg_id=92, dtype="float64")
    sig = oracle.svd_values(a)
    lhs = math.fsum(float(x) * float(x) for x in sig)
    rhs = math.fsum(float(x) * float(x) for x in a.ravel())
    assert abs(lhs - rhs) <= 10 * 120 * U * rhs


@pytest.mark.parametrize("k", [-40, -3, 5, 60])
def test_power_of_two_scaling_is_bitwise(k):
    a = workloads.gaussian(50, 50, cfg_id=93, dtype="float64")
    s1 = oracle.svd_values(a)
    s2 = oracle.svd_values(np.ldexp(a, k))
    assert np.array_equal(np.ldexp(s1, k), s2)


def test_transpose_and_permutation_invariance():
    a = workloads.gaussian(70, 60, cfg_id=94, dtype="float64")
    s = oracle.svd_values(a)
    rng = np.random.default_rng(0)
    b = a[rng.permutation(70)][:, rng.permutation(60)]
    tol = 10 * 70 * U * s[0]
    assert np.max(np.abs(oracle.svd_values(a.T) - s)) <= tol
    assert np.max(np.abs(oracle.svd_values(b) - s)) <= tol


def test_bitwise_independent_of_thread_count():
    a = workloads.gaussian(130, 101, cfg_id=95, dtype="float64")
    ref = oracle.svd_values(a, threads=1)
    for t in (2, 3, 8):
        assert np.array_equal(oracle.svd_values(a, threads=t), ref)


# ----------------------------- P3: closed forms / brute force -----------------

def test_two_by_two_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b, c, d = rng.standard_normal(4) * 10.0 ** rng.uniform(-3, 3)
        p = math.hypot(a + d, c - b)
        q = math.hypot(a - d, b + c)
        want = np.array([(p + q) / 2, abs(p - q) / 2])
        got = oracle.svd_values(np.array([[a, b], [c, d]]))
        assert np.max(np.abs(got - want)) <= 4 * U * want[0] * 4


def test_three_by_three_symmetric_functions():
    rng = np.random.default_rng(2)
    for _ in range(100):
        a = rng.standard_normal((3, 3))
        s = oracle.svd_values(a)
        # e1 = sum sigma^2 = |A|_F^2; e2 = sum_{i<j} sigma_i^2 sigma_j^2 = sum of squared 2x2 minors
        # (Cauchy-Binet); e3 = sigma1 sigma2 sigma3 = |det A| (cofactor expansion written out).
        e1 = float(np.sum(a * a))
        minors = 0.0
        for r in [(0, 1), (0, 2), (1, 2)]:
            for c in [(0, 1), (0, 2), (1, 2)]:
                m = a[r[0], c[0]] * a[r[1], c[1]] - a[r[0], c[1]] * a[r[1], c[0]]
                minors += m * m
        det = (a[0, 0] * (a[1, 1] * a[2, 2] - a[1, 2] * a[2, 1])
               - a[0, 1] * (a[1, 0] * a[2, 2] - a[1, 2] * a[2, 0])
               + a[0, 2] * (a[1, 0] * a[2, 1] - a[1, 1] * a[2, 0]))
        s2 = s * s
        assert abs(s2.sum() - e1) <= 1e-13 * e1
        assert abs(s2[0] * s2[1] + s2[0] * s2[2] + s2[1] * s2[2] - minors) <= 1e-12 * e1 * e1
        assert abs(s.prod() - abs(det)) <= 1e-12 * s[0] ** 3


def test_diagonal_and_permutation_exact():
    rng = np.random.default_rng(3)
    d = rng.standard_normal(40) * 10.0 ** rng.uniform(-5, 5, 40)
    want = np.sort(np.abs(d))[::-1]
    assert np.array_equal(oracle.svd_values(np.diag(d)), want)
    p = np.diag(d)[rng.permutation(40)][:, rng.permutation(40)]
    assert np.array_equal(oracle.svd_values(p), want)


def test_rank_one_and_orthogonal():
    rng = np.random.default_rng(4)
    u = rng.standard_normal(60)
    v = rng.standard_normal(45)
    s = oracle.svd_values(np.outer(u, v))
    s1 = np.linalg.norm(u) * np.linalg.norm(v)
    assert abs(s[0] - s1) <= 10 * 60 * U * s1
    assert np.all(s[1:] <= 10 * 60 * U * s1)
    q = workloads.haar_orthogonal(50, rng)
    assert np.max(np.abs(oracle.svd_values(q) - 1.0)) <= 10 * 50 * U


def test_zero_and_empty():
    assert np.array_equal(oracle.svd_values(np.zeros((5, 3))), np.zeros(3))
    assert oracle.svd_values(np.zeros((0, 4))).size == 0
    with pytest.raises(oracle.OracleError):
        oracle.svd_values(np.array([[1.0, np.nan], [0.0, 1.0]]))


@pytest.mark.parametrize("m,n", [(100, 100), (150, 80)])
def test_lapack_cross_checks(m, n):
    a = workloads.gaussian(m, n, cfg_id=96, dtype="float64")
    s = oracle.svd_values(a)
    ref_sdd = np.linalg.svd(a, compute_uv=False)
    sva, _, _, work, _, info = lapack.dgejsv(a, jobu=3, jobv=3)
    assert info == 0
    ref_jsv = np.sort(sva * work[0] / work[1])[::-1]
    tol = 10 * max(m, n) * U * s[0]
    assert np.max(np.abs(s - ref_sdd)) <= tol
    assert np.max(np.abs(s - ref_jsv)) <= tol


def test_float32_input_is_promoted_exactly():
    a64 = workloads.gaussian(40, 40, cfg_id=97, dtype="float32")
    a32 = workloads.as_dtype(a64, "float32")
    assert np.array_equal(oracle.svd_values(a32), oracle.svd_values(a32.astype(np.float64)))


# ----------------------------- reflector convention --------------------------

def test_householder_matches_dlarfg():
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 30):
        for zero_alpha in (False, True):
            x = rng.standard_normal(n)
            if zero_alpha:
                x[0] = 0.0
            v, tau, beta = oracle.householder(x)
            alpha_l, xl, tau_l = lapack.dlarfg(n, x[0], x[1:].copy() if n > 1 else np.zeros(1))
            assert abs(beta - alpha_l) <= 4 * U * abs(alpha_l)
            assert abs(tau - tau_l) <= 8 * U
            if n > 1:
                assert np.allclose(v[1:], xl[: n - 1], rtol=1e-14, atol=0)
            h = np.eye(n) - tau * np.outer(v, v)
            assert np.allclose(h @ x, np.r_[beta, np.zeros(n - 1)], atol=1e-14 * np.linalg.norm(x))
            assert np.allclose(h @ h.T, np.eye(n), atol=1e-15 * 8)
