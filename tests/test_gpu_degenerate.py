"""GPU parity on structurally degenerate inputs, and the contract for non-finite input.

Degenerate structures reach the paths where a reflector is the identity (a zero
tail: tau = 0 in the panels and in the chase), where singular values coincide
(bisection on clustered values) or vanish, and the multi-chunk TSQR tree of tall
and wide shapes; each is checked against the oracle on the same matrix, plus the
values the mathematics fixes (identity: all ones; one nonzero entry: that
entry's magnitude and zeros).  Non-finite input has no singular values: every
entry point writes NaN (the header states this for each of them).
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import U32, U64, banner, gate, sigma_errors, to_dev, torch_cuda, valid_config

pytestmark = pytest.mark.gpu


def _svdv():
    import paper_2608_21227_amd as svdv
    return svdv


def _rng(seed):
    return np.random.default_rng(20260 + seed)


def _matrix(case: str) -> np.ndarray:
    """float64 matrices of each degenerate structure (seeded)."""
    if case == "rank_deficient":  # rank 75 of 300: 225 zero singular values in exact arithmetic
        r = _rng(1)
        return r.standard_normal((300, 75)) @ r.standard_normal((75, 300))
    if case == "identity":  # every value 1: one cluster of 257
        return np.eye(257)
    if case == "zero_blocks":  # zero columns and rows inside: identity reflectors on the way
        a = _rng(2).standard_normal((300, 300))
        a[:, 120:140] = 0.0
        a[50:60, :] = 0.0
        return a
    if case == "bidiagonal":  # already reduced: every reflector of stage 1 has a zero tail
        r = _rng(3)
        return np.diag(r.standard_normal(280)) + np.diag(r.standard_normal(279), 1)
    if case == "single_entry":
        a = np.zeros((200, 200))
        a[37, 121] = -3.5
        return a
    if case == "graded":  # rows scaled over 2^0 .. 2^-63
        a = _rng(4).standard_normal((256, 256))
        return a * np.ldexp(1.0, -(np.arange(256) // 4))[:, None]
    if case == "clustered":  # known spectrum with three tight clusters
        s = np.concatenate([np.full(90, 1.0), np.full(90, 0.5) + 1e-9 * np.arange(90), np.full(60, 1e-3)])
        return workloads.known_spectrum(240, 240, s, cfg_id=90, dtype="float64")
    if case == "tall_multichunk":  # panels taller than one chunk: a TSQR tree
        return _rng(5).standard_normal((2300, 40))
    if case == "wide_multichunk":  # the transpose path, then a TSQR tree
        return _rng(6).standard_normal((40, 2300))
    raise ValueError(case)


CASES = ["rank_deficient", "identity", "zero_blocks", "bidiagonal", "single_entry", "graded", "clustered",
         "tall_multichunk", "wide_multichunk"]


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("case", CASES)
def test_degenerate_structures_match_oracle(dtype, case):
    torch = torch_cuda()
    svdv = _svdv()
    a = workloads.as_dtype(_matrix(case), dtype)
    ref = oracle.svd_values(a.astype(np.float64))
    m, n = a.shape
    configs = [None]
    cfg32 = valid_config(svdv, m, n, dtype, 32)
    if cfg32 is not None:
        configs.append(cfg32)
    for cfg in configs:
        banner(f"degenerate {case} {dtype} {m}x{n} cfg={'default' if cfg is None else cfg}")
        s = svdv.svd_values(to_dev(a, torch, fortran=True), config=cfg).cpu().numpy().astype(np.float64)
        assert s.shape == ref.shape
        assert np.all(np.isfinite(s)) and np.all(s >= 0) and np.all(np.diff(s) <= 0)
        nw, _ = sigma_errors(s, ref)
        if dtype == "float64":
            assert nw <= 1e-12, f"{case}: normwise {nw:.3e}"
        else:
            assert nw <= 1e-5, f"{case}: normwise {nw:.3e}"
        u = U64 if dtype == "float64" else U32
        if case == "identity":
            assert np.max(np.abs(s - 1.0)) <= 64 * u
        if case == "single_entry":
            assert abs(s[0] - 3.5) <= 8 * u * 3.5
            assert np.max(s[1:]) <= 1e-9 * 3.5
        if case == "rank_deficient":
            assert np.max(s[75:]) <= (1e-12 if dtype == "float64" else 1e-5) * s[0]


# ----------------------------------------------------------------------------- non-finite input
@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("where,value", [((5, 0), np.nan), ((199, 199), np.nan), ((0, 3), np.inf),
                                         ((120, 7), -np.inf)])
def test_nonfinite_input_gives_nan(dtype, where, value):
    torch = torch_cuda()
    svdv = _svdv()
    a = workloads.as_dtype(_rng(7).standard_normal((200, 200)), dtype)
    a[where] = value
    banner(f"non-finite {dtype} at {where} = {value}")
    s = svdv.svd_values(to_dev(a, torch, fortran=True)).cpu().numpy()
    assert s.shape == (200,) and np.all(np.isnan(s))
    # the transpose path (m < n) and the band of stage 1
    w = np.ascontiguousarray(a[:150, :]).copy()
    w[min(where[0], 149), where[1]] = value
    s = svdv.svd_values(to_dev(w, torch, fortran=True)).cpu().numpy()
    assert s.shape == (150,) and np.all(np.isnan(s))
    band = svdv.stage_band(to_dev(a, torch, fortran=True)).cpu().numpy()
    assert np.all(np.isnan(band))
    # afterwards a finite matrix is unaffected (nothing of the mark is left behind)
    a[where] = 1.0
    s = svdv.svd_values(to_dev(a, torch, fortran=True)).cpu().numpy()
    gate(dtype, s, oracle.svd_values(a.astype(np.float64)))


def test_nonfinite_input_noalloc_and_batched():
    torch = torch_cuda()
    svdv = _svdv()
    mats = [workloads.as_dtype(_rng(8 + i).standard_normal((n, n)), "float32") for i, n in enumerate((90, 130, 60))]
    bad = mats[1].copy()
    bad[40, 41] = np.nan
    banner("non-finite noalloc float32 130")
    out = torch.empty(130, dtype=torch.float32, device="cuda")
    svdv.svd_values_noalloc(to_dev(bad, torch, fortran=True), out)
    assert np.all(np.isnan(out.cpu().numpy()))
    banner("non-finite batched float32 (middle matrix)")
    dev = [to_dev(x, torch, fortran=True) for x in (mats[0], bad, mats[2])]
    packed, offs = svdv.svd_values_batched(dev)
    packed = packed.cpu().numpy()
    assert np.all(np.isnan(packed[offs[1]:offs[1] + 130]))
    for i in (0, 2):
        got = packed[offs[i]:offs[i] + mats[i].shape[0]]
        assert np.all(np.isfinite(got))
        gate("float32", got, oracle.svd_values(mats[i].astype(np.float64)))


def test_nonfinite_stage_inputs_give_nan():
    torch = torch_cuda()
    svdv = _svdv()
    r = _rng(11)
    n, b = 150, 16
    band = r.standard_normal((n, b + 1))
    for dd in range(b + 1):
        band[n - dd:, dd] = 0.0
    band[70, 5] = np.nan
    banner("non-finite stage_bidiag n=150 b=16")
    d, e = svdv.stage_bidiag(to_dev(band, torch), b)
    assert np.all(np.isnan(d.cpu().numpy())) and np.all(np.isnan(e.cpu().numpy()))
    banner("stage_bidiag after a non-finite band: finite band again")
    band[70, 5] = 0.25
    d, e = svdv.stage_bidiag(to_dev(band, torch), b)
    assert np.all(np.isfinite(d.cpu().numpy())) and np.all(np.isfinite(e.cpu().numpy()))
    dv, ev = r.standard_normal(80), r.standard_normal(79)
    for (i, arr, val) in [(3, "d", np.nan), (78, "e", np.inf), (0, "d", -np.inf)]:
        d2, e2 = dv.copy(), ev.copy()
        (d2 if arr == "d" else e2)[i] = val
        for out_dtype in (torch.float64, torch.float32):
            banner(f"non-finite stage_values {arr}[{i}] = {val} -> {out_dtype}")
            s = svdv.stage_values(to_dev(d2, torch), to_dev(e2, torch), out_dtype=out_dtype).cpu().numpy()
            assert np.all(np.isnan(s))
    s = svdv.stage_values(to_dev(dv, torch), to_dev(ev, torch)).cpu().numpy()
    assert np.all(np.isfinite(s))


# ----------------------------------------------------------------------------- binding argument checks
def test_binding_rejects_mistyped_or_short_buffers():
    """Buffers the library would misread (wrong dtype, too short, wrong shape) raise in
    the binding before any launch."""
    torch = torch_cuda()
    svdv = _svdv()
    f32 = lambda *s: torch.zeros(*s, dtype=torch.float32, device="cuda")
    f64 = lambda *s: torch.zeros(*s, dtype=torch.float64, device="cuda")
    banner("binding argument checks (no launch)")
    with pytest.raises(ValueError, match="out holds"):
        svdv.svd_values(f32(10, 8), out=f32(7))
    with pytest.raises(TypeError, match="out must be"):
        svdv.svd_values(f32(10, 8), out=f64(8))
    with pytest.raises(TypeError, match="band must be"):
        svdv.stage_bidiag(f32(40, 17), 16)
    with pytest.raises(ValueError, match="b \\+ 1"):
        svdv.stage_bidiag(f64(40, 12), 16)
    with pytest.raises(TypeError, match="d must be"):
        svdv.stage_values(f32(10), f64(9))
    with pytest.raises(ValueError, match="e holds"):
        svdv.stage_values(f64(10), f64(5))
    with pytest.raises(TypeError, match="mats\\[1\\]"):
        svdv.svd_values_batched([f32(9, 9), f64(9, 9)])
    C = f32(30, 20).t().contiguous().t()
    with pytest.raises(ValueError, match="reflector length"):
        svdv.apply_qt(f32(20, 4).t().contiguous().t(), f32(4, 4).t().contiguous().t(), C, side=0)
    with pytest.raises(ValueError, match="column-major"):
        svdv.apply_qt(f32(30, 4), f32(4, 4).t().contiguous().t(), C, side=0)
    with pytest.raises(ValueError, match="feature columns"):
        svdv.mlp_forward(f32(svdv.MLP_NPARAM), f32(5, 4))


# ----------------------------------------------------------------------------- extreme magnitudes
@pytest.mark.parametrize("dtype,k_exact,k_sub", [("float32", 100, -132), ("float64", 1000, -1062)])
def test_extreme_magnitudes(dtype, k_exact, k_sub):
    """Staging scales the input by a power of two into [0.5, 1) before anything else
    (reading R3), so 2^k A has exactly 2^k times the values of A while 2^k A is
    exact (near the overflow threshold here), and an input in the subnormal range is
    as accurate as the same input rescaled exactly into the normal range."""
    torch = torch_cuda()
    svdv = _svdv()
    a = workloads.as_dtype(_rng(12).standard_normal((180, 150)), dtype)
    banner(f"extreme magnitudes {dtype}: 2^{k_exact}, 2^{k_sub}")
    s = svdv.svd_values(to_dev(a, torch, fortran=True)).cpu().numpy()
    big = np.ldexp(a, k_exact)
    assert np.all(np.isfinite(big)) and np.array_equal(np.ldexp(big, -k_exact), a)
    s_big = svdv.svd_values(to_dev(big, torch, fortran=True)).cpu().numpy()
    assert np.array_equal(s_big, np.ldexp(s, k_exact))
    tiny = np.ldexp(a, k_sub)  # partly subnormal: the input itself loses low bits
    assert np.min(np.abs(tiny[tiny != 0])) < np.finfo(a.dtype).tiny
    s_tiny = svdv.svd_values(to_dev(tiny, torch, fortran=True)).cpu().numpy().astype(np.float64)
    ref = np.ldexp(oracle.svd_values(np.ldexp(tiny.astype(np.float64), -k_sub)), k_sub)  # exact rescaling
    nw = np.max(np.abs(s_tiny - ref)) / ref[0]
    assert nw <= (1e-5 if dtype == "float32" else 1e-12), f"normwise {nw:.3e}"


@pytest.mark.parametrize("k", [200, 900, -600, -1000])
def test_stage_values_any_magnitude(k):
    """Stage 3 alone takes (d, e) as given: values of 2^k (d, e) are exactly 2^k times
    those of (d, e) wherever 2^k (d, e) is representable without rounding."""
    torch = torch_cuda()
    svdv = _svdv()
    r = _rng(13)
    d, e = r.standard_normal(300), r.standard_normal(299)
    banner(f"stage_values at scale 2^{k}")
    want = svdv.stage_values(to_dev(d, torch), to_dev(e, torch)).cpu().numpy()
    ds, es = np.ldexp(d, k), np.ldexp(e, k)
    assert np.array_equal(np.ldexp(ds, -k), d) and np.array_equal(np.ldexp(es, -k), e)
    got = svdv.stage_values(to_dev(ds, torch), to_dev(es, torch)).cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.array_equal(got, np.ldexp(want, k))


@pytest.mark.parametrize("k", [600, 900, -600, -900])
def test_stage_bidiag_any_magnitude(k):
    """Stage 2 alone takes the band as given: the bidiagonal of 2^k B is exactly 2^k
    times that of B (the band is scaled into range internally by a power of two)."""
    torch = torch_cuda()
    svdv = _svdv()
    r = _rng(14)
    n, b = 200, 16
    band = r.standard_normal((n, b + 1))
    for dd in range(b + 1):
        band[n - dd:, dd] = 0.0
    banner(f"stage_bidiag at scale 2^{k}")
    d0, e0 = (x.cpu().numpy() for x in svdv.stage_bidiag(to_dev(band, torch), b))
    scaled = np.ldexp(band, k)
    assert np.array_equal(np.ldexp(scaled, -k), band)
    d1, e1 = (x.cpu().numpy() for x in svdv.stage_bidiag(to_dev(scaled, torch), b))
    assert np.all(np.isfinite(d1)) and np.all(np.isfinite(e1))
    assert np.array_equal(d1, np.ldexp(d0, k)) and np.array_equal(e1, np.ldexp(e0, k))
