"""Reduced-precision trailing updates (BF16 / FP16 MFMA operands, float32
accumulation; panels, stage 2 and stage 3 unchanged) against float64 references.

Tolerances follow from the operand rounding: every operand of the two products
of the update is rounded to a format with unit roundoff u (BF16 2^-8, FP16
2^-11), so one update C - V T^T V^T C is perturbed by at most about
2u |V| |T| |V|^T |C| + 2u |V| |Z'| entrywise, i.e. in Frobenius norm by
4 u ||V||_F^2 ||T||_F ||C||_F.  The whole reduction applies 2 n / b updates to
a matrix of norm sigma_1; their perturbations add like a random walk, so the
singular values move by about u sqrt(2 n / b) sigma_1 (times a small constant,
taken as 8 below).
"""
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
    bound = 8 * U_LOW[prec] * np.sqrt(2 * n / b)
    assert nw <= bound, f"{NAMES[prec]} normwise error {nw:.3e} > {bound:.3e}"
    assert np.all(np.diff(got) <= 0) and np.all(got >= 0)
