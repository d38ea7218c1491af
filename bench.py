"""Headline benchmark: singular values of a dense n=4096 float32 matrix (i.i.d. N(0,1)) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 4096] [--dtype float32] [--no-cpu]

A step is one call of the whole hot path (input staging, stage 1 band
reduction, band packing, stage 2 bulge chase, stage 3 bisection) on the same
device-resident input.  The metric is GFLOP/s on the nominal 4n^3/3 basis for
the tuned configuration; the median and plain (untuned default)
configurations of the auto-tuner's space are timed the same way beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_2608_21227_amd as svdv  # noqa: E402
import workloads  # noqa: E402
from paper_2608_21227_amd import tuner  # noqa: E402

PEAKS = {"hbm_GBs": 8000.0, "fp32_TF": 157.3, "fp64_TF": 78.6, "fp64_vec_TF": 78.6}


def chase_flops(n: int, b: int) -> float:
    """Algorithmic flops of one bulge-chase launch: per task 4 flops per element of the right
    (rows p+1..c+L-1 x L) and left (L x columns c+1..c+L+b-1) reflector applications."""
    total = 0.0
    for s in range(n - 1):
        p, c = s, s + 1
        while c < n:
            L = min(b, n - c)
            rend = min(c + L, n)
            cend = min(c + L + b, n)
            total += 4.0 * (rend - p - 1) * L + 4.0 * L * (cend - c - 1)
            p, c = c, c + b
    return total


def time_config(a, cfg, steps: int, warmup: int, torch):
    for _ in range(warmup):
        svdv.svd_values(a, config=cfg)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        s = svdv.svd_values(a, config=cfg)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall, s


def stage_breakdown(a, cfg, reps: int, torch):
    """Median per-stage times and per-kernel-class statistics of `reps` timed calls."""
    acc, kacc = {}, {"update": [], "panel": []}
    svdv.set_timing(True)
    for _ in range(reps):
        svdv.svd_values(a, config=cfg)
        for k, v in svdv.last_timing().items():
            acc.setdefault(k, []).append(v)
    # kernel-class statistics in separate calls (their per-launch events lengthen stage 1)
    svdv.set_timing(True, kernels=True)
    for _ in range(reps):
        svdv.svd_values(a, config=cfg)
        for kind in kacc:
            kacc[kind].append(svdv.last_kernel_stats(kind))
    svdv.set_timing(False)
    torch.cuda.synchronize()
    kstats = {}
    for kind, lst in kacc.items():
        med = sorted(lst, key=lambda r: r["ms"])[len(lst) // 2]
        kstats[kind] = med
    return {k: float(np.median(v)) for k, v in acc.items()}, kstats


def counters_for(kind: str, cfg, field: str):
    """A figure from the committed rocprofv3 counter summaries (profiles/traffic.json),
    if they were taken for this kernel class and configuration with the current
    kernel source: HBM bytes per launch, or the MFMA busy fraction."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    e = rec.get(kind)
    if not e or e.get("config") != cfg.as_dict():
        return None
    src = os.path.join(ROOT, "paper_2608_21227_amd", "csrc", e["source"])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != e.get("source_sha256"):
            return None  # the kernel changed since the counters were taken
    return e.get(field)


def traffic_for(kind: str, cfg):
    """HBM bytes per launch from the committed counters (see counters_for)."""
    return counters_for(kind, cfg, "bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(a_np: np.ndarray, n: int, dtype: str):
    """The float64 Jacobi oracle on this host's cores, on a bounded sample of the headline
    workload: one sweep of the same matrix, scaled by the number of sweeps the oracle takes
    to converge on it (recorded beside the stored oracle values when they were computed)."""
    import oracle
    info_path = os.path.join(ROOT, "tests", "golden", f"cfg1_n{n}_{dtype}.json")
    if os.path.exists(info_path):
        with open(info_path) as f:
            sweeps_total, src = int(json.load(f)["sweeps"]), "recorded when the stored oracle values were computed"
    else:
        sweeps_total, src = 18, "assumed (no record for this matrix)"
    threads = os.cpu_count() or 1
    secs, done = oracle.time_sweeps(a_np, 1, threads=threads)
    est = secs * sweeps_total
    gflops = (4.0 / 3.0) * n ** 3 / est / 1e9
    return {"value": round(gflops, 4), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"1 of the {sweeps_total} Jacobi sweeps the oracle needs on this n={n} {dtype} matrix "
                      f"(sweep count {src}): {secs:.1f} s, float64, OpenMP on {threads} threads of "
                      f"{_cpu_model()}; whole-run estimate {est:.0f} s"}


def cpu_lapack(a_np: np.ndarray, n: int, dtype: str, reps: int = 2):
    """Context beside the oracle: LAPACK's divide-and-conquer driver (numpy.linalg.svd
    without vectors: sgesdd for float32, dgesdd for float64) on this host's cores, on the
    same matrix, median of `reps` calls (several seconds each at n = 4096), on the same
    4n^3/3 basis.  A comparator only."""
    import threadpoolctl
    info = threadpoolctl.threadpool_info()
    blas = next((i for i in info if i.get("user_api") == "blas"), {})
    a = np.asfortranarray(a_np)
    np.linalg.svd(a[:256, :256], compute_uv=False)  # starts the thread pool
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        np.linalg.svd(a, compute_uv=False)
        ts.append(time.perf_counter() - t0)
    secs = float(np.median(ts))
    return {"value": round((4.0 / 3.0) * n ** 3 / secs / 1e9, 3), "unit": "GFLOP/s",
            "cores": int(blas.get("num_threads") or 0), "kind": "lapack",
            "sample": f"numpy.linalg.svd(compute_uv=False) ({'s' if dtype == 'float32' else 'd'}gesdd, "
                      f"{blas.get('internal_api', '?')} {blas.get('version', '?')}) on the same n={n} {dtype} matrix, "
                      f"median of {reps}: {secs:.2f} s on {_cpu_model()}"}


def batched_report(torch, count: int = 512, reps: int = 5):
    """512 square matrices, sizes uniform in [32, 512], known log-uniform spectra, float32:
    one batched call per repetition (the matrices grouped by their tuned configuration, each
    group one graph replay); throughput on the 4n^3/3 basis summed over the batch, and the
    per-matrix error against the stored float64 oracle values of exactly the rounded matrices."""
    mats, spectra = workloads.cfg2_batch(count, 32, 512, "float32")
    devs = [torch.from_numpy(np.ascontiguousarray(a.T)).t().cuda() for a in mats]
    packed, offs = svdv.svd_values_batched(devs)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        packed, _ = svdv.svd_values_batched(devs, out=packed)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    got = packed.cpu().numpy().astype(np.float64)
    flops = sum(4.0 / 3.0 * len(s) ** 3 for s in spectra)
    configs = {svdv.default_config(len(s), len(s), "float32") for s in spectra}  # one group per configuration
    rep = {"workload": f"{count} square float32 matrices, n uniform in [32, 512], log-uniform spectra in [1e-4, 1]",
           "ms_per_batch": round(ms, 4), "gflops": round(flops / (ms * 1e-3) / 1e9, 3),
           "configurations": [c.as_dict() for c in sorted(configs, key=lambda c: tuple(c.as_dict().values()))],
           "configuration_note": "tuned per size (nearest measured cell); a group whose tuned update workgroup has "
                                 "no register strip runs the widest one that has",
           "launch": "one hipGraph replay per configuration group, the groups concurrent on their own streams"}
    gold = os.path.join(ROOT, "tests", "golden", f"cfg2_b{count}_float32.npy")
    if os.path.exists(gold):
        ref_all = np.load(gold)
        nw, rel, pos = [], [], 0
        for s, o in zip(spectra, offs):
            k = len(s)
            ref = ref_all[pos:pos + k]
            pos += k
            d = np.abs(got[o:o + k] - ref)
            nw.append(float(d.max() / ref[0]))
            rel.append(float(np.max(d / ref)))
        rep.update(reference="float64 oracle (stored values)", max_normwise_err=max(nw),
                   median_normwise_err=float(np.median(nw)), max_relative_err=max(rel))
    return rep


def precision_report(torch, n: int = 8192):
    """n = 8192 float32 matrix with geometric spectrum (cond 1e4): trailing updates in float32,
    BF16 and FP16 MFMA (float32 accumulation), errors against the stored float64 oracle values."""
    gold = os.path.join(ROOT, "tests", "golden", f"cfg3_n{n}_float32.npy")
    if not os.path.exists(gold):
        return None
    ref = np.load(gold)
    a = torch.from_numpy(np.ascontiguousarray(workloads.cfg3_matrix(n, "float32").T)).t().cuda()
    rep = {"workload": f"{n}x{n} float32, A = U diag(s) V^T, s geometric 1 -> 1e-4", "reference": "float64 oracle"}
    for name, prec in (("fp32", 0), ("bf16", 2), ("fp16", 3)):
        cfg = svdv.Config(tile=16, threads=1024, inner_block=1, sweep_width=4, update_precision=prec)
        svdv.svd_values(a, config=cfg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = svdv.svd_values(a, config=cfg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        got = s.cpu().numpy().astype(np.float64)
        d = np.abs(got - ref)
        rep[name] = {"normwise": float(d.max() / ref[0]), "max_rel": float(np.max(d / ref)), "ms": round(dt * 1e3, 2)}
    return rep


# The paper's Table 2 (trailing-update kernel alone, tile 64, 16384 x 16384 float32):
# optimal / median milliseconds on the two AMD GPUs it measured (context, other hardware).
PAPER_TABLE2_MS = {"MI300X": (1.8, 12.0), "MI210": (5.7, 32.0)}


def paper_protocol_report(torch, n: int = 16384, tile: int = 64, reps: int = 5):
    """The paper's own protocol, for context: the trailing-update kernel alone (svdv_apply_qt,
    Algorithm 2's operation: C <- (I - V T V^T)^T C with `tile` reflectors) on an n x n float32
    N(0,1) matrix, over the kernel-parameter space at fixed tile (threads x inner_block); one
    warm-up and `reps` event-timed launches per configuration, median kept; optimal and median
    configuration times and their ratio, beside the paper's Table 2."""
    g = torch.Generator(device="cuda").manual_seed(260821227)
    C = torch.randn(n, n, device="cuda", dtype=torch.float32, generator=g).t()  # column-major view
    # reflector entries of size 1/sqrt(n) (as a Householder vector's are): the ~70
    # launches of the sweep, all on the same C, keep its values finite
    V = torch.randn(tile, n, device="cuda", dtype=torch.float32, generator=g).t() / np.sqrt(n)
    V = torch.tril(V, -1) + torch.eye(n, tile, device="cuda", dtype=torch.float32)
    V = V.t().contiguous().t()  # unit lower trapezoidal, column-major
    Tm = (torch.triu(torch.randn(tile, tile, device="cuda", dtype=torch.float32, generator=g)) * 0.01).t().contiguous().t()
    st = torch.cuda.current_stream()
    times = {}
    for threads in (64, 128, 256, 512, 1024):
        for ib in (1, 2, 4, 8):
            cfg = svdv.Config(tile=tile, threads=threads, inner_block=ib, sweep_width=1)
            try:
                svdv.apply_qt(V, Tm, C, side=0, config=cfg)
            except svdv.Unsupported:
                continue  # configuration outside the kernel's register/LDS limits
            ts = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                svdv.apply_qt(V, Tm, C, side=0, config=cfg)
                e1.record(st)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            times[(threads, ib)] = float(np.median(ts))
    if not times:
        return None
    order = sorted(times, key=lambda kk: times[kk])
    best, med = order[0], order[(len(order) - 1) // 2]
    flops = 4.0 * n * n * tile
    return {"workload": f"trailing-update kernel alone, {n}x{n} float32 N(0,1), tile {tile}, one launch",
            "configs_valid": len(times), "optimal_ms": round(times[best], 4), "median_ms": round(times[med], 4),
            "median_over_optimal": round(times[med] / times[best], 3),
            "optimal_config": {"threads": best[0], "inner_block": best[1]},
            "median_config": {"threads": med[0], "inner_block": med[1]},
            "optimal_tflops": round(flops / (times[best] * 1e-3) / 1e12, 3),
            "paper_table2_ms_context": {k: {"optimal": v[0], "median": v[1]} for k, v in PAPER_TABLE2_MS.items()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--dtype", default="float32", choices=["float32", "float64"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-tuned", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and reduced-precision reports")
    ap.add_argument("--paper-protocol", action="store_true",
                    help="run only the trailing-update kernel sweep at 16384^2, tile 64, and print its report")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU: --gpus must be 1 (the split over several GPUs is a design, not implemented)"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.paper_protocol:
        print("[bench] paper protocol (update kernel alone, 16384^2, tile 64)", file=sys.stderr, flush=True)
        print(json.dumps({"paper_protocol": paper_protocol_report(torch)}))
        return
    n, dtype = args.n, args.dtype
    print(f"[bench] generating n={n} {dtype} input", file=sys.stderr, flush=True)
    a_np = workloads.cfg1_matrix(n, dtype)
    a = torch.from_numpy(np.ascontiguousarray(a_np.T)).t().cuda()  # column-major on device
    nominal = (4.0 / 3.0) * n ** 3

    table = tuner.load_table()
    tuned = tuner.lookup(table, n, dtype) or svdv.default_config(n, n, dtype)
    plain = tuner.PLAIN
    median = tuner.lookup_median(table, n, dtype)
    res = {}
    order = [("tuned", tuned)] + ([] if args.only_tuned else [("plain", plain)] + ([("median", median)] if median else []))
    for name, cfg in order:
        print(f"[bench] timing {name} {cfg}", file=sys.stderr, flush=True)
        ms, wall, s = time_config(a, cfg, args.steps, args.warmup, torch)
        res[name] = {"config": cfg.as_dict(), "ms": ms, "gflops": nominal / (ms * 1e-3) / 1e9, "wall_s": wall}
        if name == "tuned":
            s_tuned = s.cpu().numpy().astype(np.float64)
    print("[bench] stage breakdown", file=sys.stderr, flush=True)
    stages, kstats = stage_breakdown(a, tuned, 3, torch)

    # parity spot check against the stored oracle values (full size)
    gold = os.path.join(ROOT, "tests", "golden", f"cfg1_n{n}_{dtype}.npy")
    parity = None
    if os.path.exists(gold):
        ref = np.load(gold)
        diff = np.abs(s_tuned - ref)
        parity = {"normwise": float(diff.max() / ref[0]), "max_rel": float(np.max(diff / ref))}
        # the parity gate of the tests: float64 normwise <= 1e-12; float32 normwise <= 1e-5
        # and per-value relative <= 1e-5 * cond (cond of the oracle's values)
        if dtype == "float64":
            parity["gate"] = "normwise <= 1e-12"
            parity["pass"] = parity["normwise"] <= 1e-12
        else:
            cond = float(ref[0] / ref[-1])
            parity["gate"] = f"normwise <= 1e-5 and max_rel <= 1e-5 * cond ({cond:.4g})"
            parity["pass"] = parity["normwise"] <= 1e-5 and parity["max_rel"] <= 1e-5 * cond

    # roofline of each hot kernel class, measured live (events on the library's stream)
    b = tuned.tile
    es = 4 if dtype == "float32" else 8
    ridge = (PEAKS["fp32_TF"] if dtype == "float32" else PEAKS["fp64_TF"]) * 1e12 / (PEAKS["hbm_GBs"] * 1e9)
    kinds = {}
    t_chase = stages.get("chase_kernel", stages.get("chase", float("nan"))) * 1e-3
    fl = chase_flops(n, b)
    kinds["chase"] = {"kernel": "k_chase_* (stage 2 bulge chase, float64; one launch per call)", "launches": 1,
                      "ms": t_chase * 1e3, "bound": "alu", "achieved": fl / t_chase / 1e12,
                      "peak": PEAKS["fp64_vec_TF"], "unit": "TFLOP/s", "flops_per_launch": fl}
    for kind, name in (("update", "k_larfb_* (stage 1 trailing update, Algorithm 2's operation)"),
                       ("panel", "k_chunk_qr (stage 1 panel QR/LQ)")):
        ks = kstats[kind]
        t = ks["ms"] * 1e-3
        if not ks["launches"] or t <= 0:
            continue
        inten = ks["flops"] / ks["bytes"]
        if kind == "update" and inten >= ridge:
            ach, peak, unit, bound = ks["flops"] / t / 1e12, (PEAKS["fp32_TF"] if dtype == "float32" else PEAKS["fp64_TF"]), "TFLOP/s", "mfma"
        else:
            ach, peak, unit, bound = ks["bytes"] / t / 1e9, PEAKS["hbm_GBs"], "GB/s", "hbm"
        kinds[kind] = {"kernel": name, "launches": ks["launches"], "ms": ks["ms"], "bound": bound, "achieved": ach,
                       "peak": peak, "unit": unit, "avg_launch_us": 1e3 * ks["ms"] / ks["launches"],
                       "alg_flops": ks["flops"], "alg_bytes": ks["bytes"]}
    dom = max(kinds, key=lambda k: kinds[k]["ms"])
    rooflines = {}
    for k, v in kinds.items():
        rooflines[k] = {"bound": v["bound"], "achieved": round(v["achieved"], 6), "peak": v["peak"], "unit": v["unit"],
                        "frac": round(v["achieved"] / v["peak"], 6), "ms_per_step": round(v["ms"], 4),
                        "launches_per_step": v["launches"], "kernel": v["kernel"]}
    roofline = dict(rooflines[dom])
    roofline["traffic"] = traffic_for(dom, tuned)
    # HBM bytes per launch from the committed counters (when taken for this kernel
    # source and configuration) over the launch time measured here
    for k, v in kinds.items():
        tb = traffic_for(k, tuned)
        if tb:
            rooflines[k]["hbm_GBs_from_counters"] = round(tb / (v["ms"] * 1e-3 / v["launches"]) / 1e9, 3)
            if k == dom:
                roofline["hbm_GBs_from_counters"] = rooflines[k]["hbm_GBs_from_counters"]
        busy = counters_for(k, tuned, "mfma_busy")
        if busy is not None:
            rooflines[k]["mfma_busy_from_counters"] = busy
    t_stage1 = stages.get("stage1", float("nan")) * 1e-3
    s1_flops = 8.0 / 3.0 * n ** 3

    tuned_ms = res["tuned"]["ms"]
    out = {
        "metric": "SVD-values GFLOP/s (4n³/3 basis) tuned vs median config, n=4096 FP32, 1 MI355X",
        "value": round(res["tuned"]["gflops"], 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tuned_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == "float32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"dense {n}x{n} {dtype} i.i.d. N(0,1) singular values (two-stage: band, bulge chase, bisection)",
                   "n": n, "tuned": res["tuned"]["config"]},
        "median_gflops": round(res["median"]["gflops"], 3) if "median" in res else None,
        "plain_gflops": round(res["plain"]["gflops"], 3) if "plain" in res else None,
        "tuned_over_median": round(res["median"]["ms"] / tuned_ms, 3) if "median" in res else None,
        "tuned_over_plain": round(res["plain"]["ms"] / tuned_ms, 3) if "plain" in res else None,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "stage1_roofline_frac": round(max(s1_flops / (PEAKS["fp32_TF" if dtype == "float32" else "fp64_TF"] * 1e12),
                                          4 * (4 if dtype == "float32" else 8) * n ** 3 / (3 * b) / (PEAKS["hbm_GBs"] * 1e9))
                                      / t_stage1, 5),
        "roofline": roofline,
        "rooflines": rooflines,
        "parity_vs_oracle": parity,
    }
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a_np, n, dtype)
        print("[bench] cpu context (LAPACK gesdd)", file=sys.stderr, flush=True)
        out["cpu_lapack"] = cpu_lapack(a_np, n, dtype)
    if not args.no_extras:
        print("[bench] batched workload", file=sys.stderr, flush=True)
        out["batched"] = batched_report(torch)
        print("[bench] reduced-precision updates", file=sys.stderr, flush=True)
        out["precision"] = precision_report(torch)
        print("[bench] paper protocol (update kernel alone, 16384^2, tile 64)", file=sys.stderr, flush=True)
        out["paper_protocol"] = paper_protocol_report(torch)
    print(json.dumps(out))
    if parity is not None and not parity["pass"]:
        print(f"[bench] parity gate failed: {parity}", file=sys.stderr, flush=True)
        sys.exit(3)


if __name__ == "__main__":
    main()
