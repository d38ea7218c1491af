"""Auto-tuner for the svdv configuration space (the paper's Eq. 1: x* = argmin_x f(K_x)).

The search space is tile x threads x inner_block x sweep_width.  Every
configuration is measured the way the paper's runtime observer does it: one
warm-up call excluded from the metric, then `reps` calls timed with stream
events, the median kept.  Configurations the library reports as unsupported
are recorded as invalid and skipped (they do not stop the run).  Results are
appended to a JSONL database so an interrupted run resumes where it stopped;
a torn last line is ignored.

"Median configuration": the valid configurations sorted by their median time,
the one at index floor((N-1)/2) (the lower median -- a real, re-runnable
configuration).  "Plain": the fixed a-priori default below, chosen before any
tuning.
"""
from __future__ import annotations

import itertools
import json
import os
import statistics
import time
from typing import Callable, Iterable

from . import Config, Unsupported, check_config

TILES = (16, 32, 64, 128)
THREADS = (64, 128, 256, 512, 1024)
INNER = (1, 2, 4, 8)
SWEEP = tuple(range(1, 9))
PLAIN = Config(tile=32, threads=256, inner_block=1, sweep_width=1)

_HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(_HERE, "tuned.json")


def space(tiles=TILES, threads=THREADS, inner=INNER, sweep=SWEEP) -> list[Config]:
    return [Config(t, th, ib, sw) for t, th, ib, sw in itertools.product(tiles, threads, inner, sweep)]


def key_of(cfg: Config) -> str:
    return f"{cfg.tile}/{cfg.threads}/{cfg.inner_block}/{cfg.sweep_width}/{cfg.update_precision}"


# --------------------------------------------------------------------------- database

def read_db(path: str) -> list[dict]:
    """Records of a JSONL database; a torn (unparsable) line is dropped."""
    out = []
    if not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            try:
                out.append(json.loads(line))
            except json.JSONDecodeError:
                continue
    return out


def append_db(path: str, rec: dict) -> None:
    """Append one record; a torn last line (an interrupted write, no newline) is
    closed first so the new record starts a line of its own."""
    torn = False
    if os.path.exists(path) and os.path.getsize(path) > 0:
        with open(path, "rb") as f:
            f.seek(-1, os.SEEK_END)
            torn = f.read(1) != b"\n"
    with open(path, "a") as f:
        f.write(("\n" if torn else "") + json.dumps(rec) + "\n")
        f.flush()
        os.fsync(f.fileno())


# --------------------------------------------------------------------------- measurement

def robust_median(times: list[float]) -> float:
    return float(statistics.median(times))


def measure_fn(a, cfg: Config, reps: int, warmup: int = 1) -> list[float]:
    """Per-call milliseconds of svd_values on the device-resident matrix `a` (torch tensor)."""
    import torch
    from . import svd_values
    for _ in range(warmup):
        svd_values(a, config=cfg)
    st = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    evs[0].record(st)
    for i in range(reps):
        svd_values(a, config=cfg)
        evs[i + 1].record(st)
    torch.cuda.synchronize()
    return [evs[i].elapsed_time(evs[i + 1]) for i in range(reps)]


def tune(n: int, dtype: str, configs: Iterable[Config], db_path: str,
         measure: Callable[[Config], list[float]], is_valid: Callable[[Config], bool] | None = None,
         max_retries: int = 2, progress: Callable[[str], None] | None = None) -> list[dict]:
    """Measure every configuration not yet in the database (resume), skipping invalid ones.

    A measurement with a non-positive time or a spread (max/min) above 3x is
    repeated up to `max_retries` times (timing safeguard); the last one is kept
    and flagged."""
    done = {r["key"] for r in read_db(db_path) if r.get("n") == n and r.get("dtype") == dtype}
    is_valid = is_valid or (lambda c: check_config(n, n, dtype, c))
    for cfg in configs:
        k = key_of(cfg)
        if k in done:
            continue
        rec = {"n": n, "dtype": dtype, "key": k, "config": cfg.as_dict(), "ts": time.time()}
        if not is_valid(cfg):
            rec.update(status="invalid")
        else:
            try:
                times, flagged = None, False
                for attempt in range(max_retries + 1):
                    times = measure(cfg)
                    bad = min(times) <= 0 or (max(times) / min(times) > 3.0)
                    if not bad:
                        break
                    flagged = True
                rec.update(status="ok", times_ms=times, median_ms=robust_median(times), remeasured=flagged)
            except Unsupported as e:
                rec.update(status="invalid", detail=str(e))
        append_db(db_path, rec)
        done.add(k)
        if progress:
            progress(f"{k} {rec['status']} {rec.get('median_ms', '')}")
    return [r for r in read_db(db_path) if r.get("n") == n and r.get("dtype") == dtype]


def summarize(records: list[dict]) -> dict:
    """argmin (Eq. 1), lower-median configuration and counts over the valid records."""
    ok = sorted((r for r in records if r.get("status") == "ok"), key=lambda r: r["median_ms"])
    if not ok:
        return {"valid": 0, "invalid": sum(1 for r in records if r.get("status") == "invalid")}
    med = ok[(len(ok) - 1) // 2]
    return {
        "valid": len(ok),
        "invalid": sum(1 for r in records if r.get("status") == "invalid"),
        "best": ok[0]["config"], "best_ms": ok[0]["median_ms"],
        "median": med["config"], "median_ms": med["median_ms"],
        "worst_ms": ok[-1]["median_ms"],
        "ratio_median_over_best": med["median_ms"] / ok[0]["median_ms"],
    }


# --------------------------------------------------------------------------- tuned table

def load_table(path: str = TABLE_PATH) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_table(table: dict, path: str = TABLE_PATH) -> None:
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def _entry(table: dict, n: int, dtype: str):
    return table.get(f"{n}_{dtype}")


def lookup(table: dict, n: int, dtype: str) -> Config | None:
    e = _entry(table, n, dtype)
    return Config(**e["best"]) if e else None


def lookup_median(table: dict, n: int, dtype: str) -> Config | None:
    e = _entry(table, n, dtype)
    return Config(**e["median"]) if e else None


# --------------------------------------------------------------------------- command line

def main(argv=None) -> None:
    """python -m paper_2608_21227_amd.tuner --n 4096 --dtype float32 [--reps 5] [--db PATH] [--limit K]

    Measures the whole space at one (n, dtype) cell on the current GPU (resuming
    from the database), prints the summary and records best and median in the
    tuned table."""
    import argparse
    import sys
    import numpy as np
    import torch
    from . import default_config
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--dtype", default="float32", choices=["float32", "float64"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--db", default=None)
    ap.add_argument("--table", default=TABLE_PATH)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--time-budget", type=float, default=0.0, help="stop measuring after this many seconds")
    ap.add_argument("--slow-ms", type=float, default=500.0)
    ap.add_argument("--tiles", default=None, help="comma-separated tile sizes to search (default: all)")
    args = ap.parse_args(argv)
    n, dtype = args.n, args.dtype
    db = args.db or os.path.join(_HERE, "tuning", f"tuning_{n}_{dtype}.jsonl")
    os.makedirs(os.path.dirname(db) or ".", exist_ok=True)
    rng = np.random.default_rng(np.random.SeedSequence(260821227, spawn_key=(1, n, 0 if dtype == "float32" else 1)))
    a_np = rng.standard_normal((n, n)).astype(dtype)
    a = torch.from_numpy(np.ascontiguousarray(a_np.T)).t().cuda()
    t0 = time.time()
    tiles = tuple(int(x) for x in args.tiles.split(",")) if args.tiles else TILES
    cfgs = space(tiles=tiles)
    order = np.random.default_rng(args.seed).permutation(len(cfgs))  # interleave so a partial run is a fair sample
    cfgs = [cfgs[i] for i in order]

    def measure(cfg):
        if args.time_budget and time.time() - t0 > args.time_budget:
            raise TimeoutError
        # configurations slower than `slow_ms` per call get one timed call after the
        # warm-up (their rank is not in doubt and they would dominate the run time)
        first = measure_fn(a, cfg, 1, warmup=1)
        if first[0] > args.slow_ms:
            return first
        return measure_fn(a, cfg, args.reps, warmup=0)

    try:
        recs = tune(n, dtype, cfgs, db, measure, progress=lambda m: print("[tune]", m, flush=True))
    except TimeoutError:
        print("[tune] time budget reached; partial database kept", flush=True)
        recs = [r for r in read_db(db) if r.get("n") == n and r.get("dtype") == dtype]
    summ = summarize(recs)
    summ["plain_ms"] = next((r["median_ms"] for r in recs if r.get("key") == key_of(PLAIN) and r.get("status") == "ok"), None)
    summ["default"] = default_config(n, n, dtype).as_dict()
    print(json.dumps(summ), flush=True)
    if summ.get("valid"):
        table = load_table(args.table)
        table[f"{n}_{dtype}"] = {k: summ[k] for k in ("best", "best_ms", "median", "median_ms", "valid", "invalid",
                                                      "ratio_median_over_best", "plain_ms")}
        if tiles != TILES:
            table[f"{n}_{dtype}"]["tiles"] = list(tiles)
        save_table(table, args.table)


if __name__ == "__main__":
    main()
