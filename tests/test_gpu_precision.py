"""Reduced-precision trailing updates (BF16 / FP16 MFMA operands, float32
accumulation; panel factorisation in float64 arithmetic, stage 2 and stage 3 in
float64) against float64 references.

Tolerances follow from the operand rounding: every operand of the two products
of the update is rounded to a format with unit roundoff u (BF16 2^-8, FP16
2^-11), so one update C - V T^T V^T C is perturbed by at most about
2u |V| |T| |V|^T |C| + 2u |V| |Z'| entrywise, i.e. in Frobenius norm by
4 u ||V||_F^2 ||T||_F ||C||_F.  The whole reduction applies 2 n / b updates to
a matrix of norm sigma_1; their perturbations add like a random walk, so the
singular values move by about u sqrt(2 n / b) sigma_1 (times a small constant).
That is a bound for the worst case; the measured normwise errors of whole
calls are far below it (about 0.08 u for BF16 and 0.06 u for FP16 at n = 8192,
cond 1e4), so the end-to-end gates below are one unit roundoff of the low
precision relative to sigma_1: an order of magnitude above what is measured,
and far below what a wrong update (or one in the wrong precision) would give.
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import banner, torch_cuda

pytestmark = pytest.mark.gpu

U_LOW = {2: 2.0 ** -8, 3: 2.0 ** -11}
NAMES = {2: "bf16", 3: "fp16"}


def _svdv():
    import paper_2608_21227_amd as svdv
    return svdv


@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("h,w,k,tile,threads,ib", [(100, 70, 16, 16, 1024, 1), (256, 300, 32, 32, 512, 2),
                                                   (200, 130, 64, 64, 1024, 1)])
def test_apply_qt_reduced_precision(prec, side, h, w, k, tile, threads, ib):
    torch = torch_cuda()
    svdv = _svdv()
    cfg = svdv.Config(tile=tile, threads=threads, inner_block=ib, sweep_width=1, update_precision=prec)
    assert svdv.check_config(h, w, "float32", cfg)
    rng = np.random.default_rng(h * 7 + w + k + side + 100 * prec)
    vr = h if side == 0 else w
    V = np.tril(rng.standard_normal((vr, k)), -1)
    V[np.arange(k), np.arange(k)] = 1.0
    T = np.triu(rng.standard_normal((k, k)) * 0.3)
    C = rng.standard_normal((h, w))
    V, T, C = V.astype(np.float32), T.astype(np.float32), C.astype(np.float32)
    V64, T64, C64 = V.astype(np.float64), T.astype(np.float64), C.astype(np.float64)
    Q = np.eye(vr) - V64 @ T64 @ V64.T
    want = Q.T @ C64 if side == 0 else C64 @ Q
    banner(f"apply_qt {NAMES[prec]} side={side} h={h} w={w} k={k} tile={tile}")
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x.T)).t().cuda()
    Vd, Td, Cd = dev(V), dev(T), dev(C)
    svdv.apply_qt(Vd, Td, Cd, side=side, config=cfg)
    torch.cuda.synchronize()
    got = Cd.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(got - want)
    bound = 4 * U_LOW[prec] * np.linalg.norm(V64) ** 2 * np.linalg.norm(T64) * np.linalg.norm(C64)
    assert err <= bound, f"{NAMES[prec]} update error {err:.3e} > {bound:.3e}"
    # and it really is reduced precision: clearly above float32 rounding (at the size of this product)
    assert err > 1e-6 * np.linalg.norm(want)


@pytest.mark.parametrize("prec", [2, 3])
def test_end_to_end_reduced_precision(prec):
    torch = torch_cuda()
    svdv = _svdv()
    n, b = 512, 16
    s_true = workloads.geometric_spectrum(n, 1e-4)  # cond 1e4, as the mixed-precision workload
    a = workloads.as_dtype(workloads.known_spectrum(n, n, s_true, cfg_id=3, dtype="float32"), "float32")
    ref = oracle.svd_values(a)
    cfg = svdv.Config(tile=b, threads=1024, inner_block=1, sweep_width=4, update_precision=prec)
    banner(f"end-to-end {NAMES[prec]} n={n}")
    s = svdv.svd_values(torch.from_numpy(np.ascontiguousarray(a.T)).t().cuda(), config=cfg)
    torch.cuda.synchronize()
    got = s.cpu().numpy().astype(np.float64)
    nw = np.max(np.abs(got - ref)) / ref[0]
    rel = np.max(np.abs(got - ref) / ref)
    print(f"[precision] {NAMES[prec]} n={n}: normwise {nw:.3e}, max relative {rel:.3e}", flush=True)
    assert nw <= U_LOW[prec], f"{NAMES[prec]} normwise error {nw:.3e} > {U_LOW[prec]:.3e}"
    assert np.all(np.diff(got) <= 0) and np.all(got >= 0)


# ----------------------------------------------------------------------------- mixed-precision workload
# n = 8192, A = U diag(s) V^T with s geometric from 1 to 1e-4 (cond 1e4), stored in
# float32; the stored float64 oracle values of exactly that rounded matrix
# (tests/golden/cfg3_n8192_float32.npy, written by tests/golden/make_golden.py).
# Tile 16 with the 1024-thread update: the panels run their multi-chunk tree
# (8192 rows, 2048 per chunk) and the 16-wave register strip of the update.
GOLDEN_CFG3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg3_n8192_float32.npy")


@pytest.fixture(scope="module")
def cfg3_case():
    if not os.path.exists(GOLDEN_CFG3):
        pytest.skip("cfg3 golden values not written")
    torch = torch_cuda()
    a = workloads.cfg3_matrix(8192, "float32")
    dev = torch.from_numpy(np.ascontiguousarray(a.T)).t().cuda()
    del a
    return dev, np.load(GOLDEN_CFG3)


@pytest.mark.parametrize("prec", [0, 2, 3])
def test_mixed_precision_workload_against_oracle(cfg3_case, prec):
    torch = torch_cuda()
    svdv = _svdv()
    dev, ref = cfg3_case
    cfg = svdv.Config(tile=16, threads=1024, inner_block=1, sweep_width=4, update_precision=prec)
    name = NAMES.get(prec, "fp32")
    banner(f"mixed-precision workload n=8192 cond 1e4, {name} updates")
    s = svdv.svd_values(dev, config=cfg)
    torch.cuda.synchronize()
    got = s.cpu().numpy().astype(np.float64)
    nw = float(np.max(np.abs(got - ref)) / ref[0])
    rel = float(np.max(np.abs(got - ref) / ref))
    print(f"[precision] {name} n=8192 cond 1e4: normwise {nw:.3e}, max relative {rel:.3e}", flush=True)
    assert np.all(np.isfinite(got)) and np.all(np.diff(got) <= 0)
    if prec == 0:
        from gpu_util import gate
        gate("float32", got, ref)
    else:
        assert nw <= U_LOW[prec], f"{name} normwise error {nw:.3e} > {U_LOW[prec]:.3e}"
        # the reduced precision is really in use: well above float32 rounding
        assert nw > 16 * 2.0 ** -24, f"{name} error {nw:.3e} is at float32 level"
