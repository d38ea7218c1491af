"""Learned tuning: a cost model that predicts a configuration's run time, so the
auto-tuner measures only its most promising candidates.

The paper's tuner picks x* = argmin_x f(K_x) over measured run times (Eq. 1),
which needs every configuration measured.  Here a small perceptron (6 -> 64 ->
64 -> 1, ReLU, float32), trained on the tuner's own measurements with the
library's GPU kernels (forward, gradient, Adam: ``mlp_*`` in the package),
predicts log run time from six features of (n, dtype, configuration).  For a
new (n, dtype) cell the valid configurations are ranked by prediction and the
best k are measured; exhaustive search stays the reference: the regret of a
budget-k search is min(measured time of the k chosen) / (exhaustive best) - 1,
and random search with the same budget is the baseline it must beat.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import Config, MLP_HIDDEN, MLP_IN, MLP_NPARAM, check_config, mlp_adam_step, mlp_forward, mlp_gradient, mlp_work
from .tuner import read_db, space


def features(n: int, dtype: str, cfg: Config) -> list[float]:
    """log2 n, dtype, log2 tile, log2 threads, log2 inner block, sweep width -- each mapped
    affinely to roughly [-1, 1] over the tuning space."""
    return [(math.log2(n) - 11.0) / 2.0,
            0.0 if dtype == "float32" else 1.0,
            math.log2(cfg.tile) - 5.0,
            (math.log2(cfg.threads) - 8.0) / 1.2,
            math.log2(cfg.inner_block) - 1.5,
            (cfg.sweep_width - 4.5) / 2.5]


def records_to_xy(records):
    """(X, log-time) of the valid measured records."""
    X, y = [], []
    for r in records:
        if r.get("status") != "ok":
            continue
        X.append(features(r["n"], r["dtype"], Config(**r["config"])))
        y.append(math.log(r["median_ms"]))
    return np.asarray(X, dtype=np.float32), np.asarray(y, dtype=np.float64)


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (float32)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((MLP_IN, MLP_HIDDEN)) * math.sqrt(2.0 / MLP_IN)
    W2 = rng.standard_normal((MLP_HIDDEN, MLP_HIDDEN)) * math.sqrt(2.0 / MLP_HIDDEN)
    w3 = rng.standard_normal(MLP_HIDDEN) * math.sqrt(1.0 / MLP_HIDDEN)
    p = np.concatenate([W1.ravel(), np.zeros(MLP_HIDDEN), W2.ravel(), np.zeros(MLP_HIDDEN), w3, [0.0]])
    assert p.size == MLP_NPARAM
    return p.astype(np.float32)


@dataclass
class CostModel:
    params: object = None  # float32 CUDA tensor
    mean: float = 0.0      # log-time standardisation of the training targets
    std: float = 1.0
    losses: list = None

    def fit(self, records, steps: int = 2000, lr: float = 3e-3, seed: int = 0, device="cuda"):
        """Full-batch Adam on the standardised log times (all arithmetic in the GPU kernels)."""
        import torch
        X, y = records_to_xy(records)
        if len(X) == 0:
            raise ValueError("no valid measurements to train on")
        self.mean, self.std = float(y.mean()), float(y.std() or 1.0)
        t = ((y - self.mean) / self.std).astype(np.float32)
        Xd = torch.from_numpy(X).to(device)
        td = torch.from_numpy(t).to(device)
        p = torch.from_numpy(init_params(seed)).to(device)
        g = torch.zeros_like(p)
        m = torch.zeros_like(p)
        v = torch.zeros_like(p)
        loss = torch.zeros(1, dtype=torch.float32, device=device)
        work = mlp_work(len(X), device)
        self.losses = []
        for k in range(1, steps + 1):
            mlp_gradient(p, Xd, td, g, loss, work)
            mlp_adam_step(p, g, m, v, k, lr)
            if k == 1 or k % 250 == 0 or k == steps:
                self.losses.append((k, float(loss.item())))
        self.params = p
        return self

    def predict(self, n: int, dtype: str, cfgs) -> np.ndarray:
        """Predicted run times (ms) of the configurations."""
        import torch
        X = torch.tensor([features(n, dtype, c) for c in cfgs], dtype=torch.float32, device=self.params.device)
        y = mlp_forward(self.params, X).cpu().numpy().astype(np.float64)
        return np.exp(y * self.std + self.mean)


def cell_table(records, n: int, dtype: str) -> dict:
    """key -> measured median ms of the valid configurations of one (n, dtype) cell."""
    from .tuner import key_of
    return {key_of(Config(**r["config"])): r["median_ms"] for r in records
            if r.get("n") == n and r.get("dtype") == dtype and r.get("status") == "ok"}


def valid_configs(n: int, dtype: str):
    return [c for c in space() if check_config(n, n, dtype, c)]


def regret_topk(model: CostModel, table: dict, n: int, dtype: str, k: int) -> float:
    """Measure (look up) the k configurations the model ranks best; regret against the exhaustive best."""
    from .tuner import key_of
    cfgs = [c for c in valid_configs(n, dtype) if key_of(c) in table]
    pred = model.predict(n, dtype, cfgs)
    order = np.argsort(pred, kind="stable")[:k]
    best_chosen = min(table[key_of(cfgs[i])] for i in order)
    return best_chosen / min(table.values()) - 1.0


def regret_random(table: dict, k: int, trials: int = 500, seed: int = 0) -> float:
    """Mean regret of measuring k configurations drawn uniformly without replacement."""
    rng = np.random.default_rng(seed)
    times = np.asarray(list(table.values()))
    best = times.min()
    out = [times[rng.choice(times.size, size=min(k, times.size), replace=False)].min() / best - 1.0
           for _ in range(trials)]
    return float(np.mean(out))


def load_records(paths):
    recs = []
    for p in paths:
        recs.extend(read_db(p))
    return recs
