"""Learned cost model: the GPU training kernels against the float64 reference
(oracle.mlp), and what the trained model gains over random search when the
tuner may measure only k configurations of a cell it has not seen."""
import glob
import os

import numpy as np
import pytest

from oracle import mlp as ref
from gpu_util import banner, torch_cuda

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _svdv():
    import paper_2608_21227_amd as svdv
    return svdv


def _problem(seed, n=500):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal(ref.NPARAM) * 0.2).astype(np.float32)
    X = rng.uniform(-1, 1, (n, ref.IN)).astype(np.float32)
    t = rng.standard_normal(n).astype(np.float32)
    return p, X, t


@pytest.mark.parametrize("seed,n", [(0, 1), (1, 37), (2, 500), (3, 2100)])
def test_gradient_and_forward_match_float64_reference(seed, n):
    torch = torch_cuda()
    svdv = _svdv()
    p, X, t = _problem(seed, n)
    banner(f"mlp gradient n={n}")
    pd, Xd, td = (torch.from_numpy(a).cuda() for a in (p, X, t))
    g = torch.zeros_like(pd)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    svdv.mlp_gradient(pd, Xd, td, g, loss)
    y = svdv.mlp_forward(pd, Xd)
    torch.cuda.synchronize()
    p64, X64, t64 = p.astype(np.float64), X.astype(np.float64), t.astype(np.float64)
    g_ref = ref.gradient(p64, X64, t64)
    y_ref, _ = ref.forward(p64, X64)
    g_gpu = g.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    assert rel <= 1e-4, f"gradient relative error {rel:.2e}"
    big = np.abs(g_ref) > 1e-3 * np.abs(g_ref).max()
    assert np.max(np.abs(g_gpu[big] - g_ref[big]) / np.abs(g_ref[big])) <= 1e-3
    assert np.max(np.abs(y.cpu().numpy() - y_ref)) <= 1e-5 * max(1.0, np.abs(y_ref).max())
    assert abs(float(loss.item()) - ref.loss(p64, X64, t64)) <= 1e-5 * ref.loss(p64, X64, t64)


def test_adam_matches_reference_and_training_reduces_loss():
    torch = torch_cuda()
    svdv = _svdv()
    p, X, t = _problem(7, 300)
    t = (X[:, 0] ** 2 - X[:, 1] * X[:, 2] + 0.3 * X[:, 5]).astype(np.float32)
    pd, Xd, td = (torch.from_numpy(a).cuda() for a in (p, X, t))
    g, m, v = (torch.zeros_like(pd) for _ in range(3))
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    work = svdv.mlp_work(X.shape[0], "cuda")
    # one step against the reference
    svdv.mlp_gradient(pd, Xd, td, g, loss, work)
    svdv.mlp_adam_step(pd, g, m, v, 1, 1e-3)
    torch.cuda.synchronize()
    p64 = p.astype(np.float64)
    p1, _, _ = ref.adam_step(p64, ref.gradient(p64, X.astype(np.float64), t.astype(np.float64)),
                             np.zeros_like(p64), np.zeros_like(p64), 1, 1e-3)
    assert np.max(np.abs(pd.cpu().numpy() - p1)) <= 1e-6
    l0 = ref.loss(p64, X.astype(np.float64), t.astype(np.float64))
    for k in range(2, 401):
        svdv.mlp_gradient(pd, Xd, td, g, loss, work)
        svdv.mlp_adam_step(pd, g, m, v, k, 3e-3)
    torch.cuda.synchronize()
    assert float(loss.item()) < 0.1 * l0


def test_learned_ranking_beats_random_search_on_unseen_cells():
    torch_cuda()
    from paper_2608_21227_amd import learned
    paths = sorted(glob.glob(os.path.join(ROOT, "paper_2608_21227_amd", "tuning", "tuning_*.jsonl")))
    recs = learned.load_records(paths)
    cells = sorted({(r["n"], r["dtype"]) for r in recs if r.get("status") == "ok"})
    if len(cells) < 3:
        pytest.skip("needs measurements of at least three (n, dtype) cells")
    banner(f"learned tuning over {len(cells)} cells")
    gains = []
    for held in cells:  # leave one cell out at a time
        train = [r for r in recs if (r["n"], r["dtype"]) != held]
        model = learned.CostModel().fit(train, steps=1500, seed=0)
        table = learned.cell_table(recs, *held)
        for k in (1, 5, 10):
            rm = learned.regret_topk(model, table, held[0], held[1], k)
            rr = learned.regret_random(table, k, trials=500, seed=1)
            print(f"[learned] held {held} k={k}: model regret {rm:.3f}, random regret {rr:.3f}", flush=True)
            if k == 10:
                gains.append((rr, rm))
    # over the unseen cells, the model's budget-10 search loses less than random search does
    assert np.mean([rm for _, rm in gains]) < np.mean([rr for rr, _ in gains])
