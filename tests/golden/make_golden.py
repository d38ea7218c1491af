"""Writes the stored oracle singular values used by the full-size GPU parity tests.

Calls only the CPU oracle (``oracle.svd_values``) on the seeded workloads of
``workloads``; nothing here touches the GPU path.  Output: one ``.npy`` file of
float64 singular values (descending) per (workload, n, dtype).

    python tests/golden/make_golden.py [--sizes 1024 2048 4096] [--threads 8]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def path_for(name: str) -> str:
    return os.path.join(HERE, name + ".npy")


def write_info(name: str, info: dict, secs: float, threads: int) -> None:
    """Sidecar record of the oracle run that wrote `name` (Jacobi sweeps to convergence,
    wall time and threads of this machine), read by the bench's CPU baseline."""
    import json
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump({"sweeps": int(info["sweeps"]), "seconds": round(secs, 2), "threads": int(threads or os.cpu_count()),
                   "offmax": float(info["offmax"])}, f)
        f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="*", default=[1024, 2048, 4096])
    ap.add_argument("--dtypes", nargs="*", default=["float32", "float64"])
    ap.add_argument("--cfg3", action="store_true", help="also the n=8192 cond-1e4 matrix (slow)")
    ap.add_argument("--cfg2", action="store_true",
                    help="also the batch of 512 float32 matrices (n uniform in [32, 512]): one packed array of "
                         "every matrix's values in batch order")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--info", nargs="*", default=[],
                    help="re-run the oracle on these stored workloads (e.g. cfg1_n4096_float32) only to record their "
                         "sweep counts; the stored values are left as they are")
    args = ap.parse_args()
    jobs = [(f"cfg1_n{n}_{dt}", lambda n=n, dt=dt: workloads.cfg1_matrix(n, dt))
            for n in args.sizes for dt in args.dtypes]
    if args.cfg3:
        jobs.append(("cfg3_n8192_float32", lambda: workloads.cfg3_matrix(8192, "float32")))
    for name in args.info:
        _, nn, dt = name.split("_")
        a = workloads.cfg1_matrix(int(nn[1:]), dt)
        t = time.time()
        info = {}
        s = oracle.svd_values(a, threads=args.threads, info=info)
        ok = np.array_equal(s, np.load(path_for(name)))
        write_info(name, info, time.time() - t, args.threads)
        print(f"{name}: sweeps={info['sweeps']} in {time.time() - t:.1f}s, same values as stored: {ok}", flush=True)
    if args.cfg2:
        out = path_for("cfg2_b512_float32")
        if os.path.exists(out):
            print("exists", out, flush=True)
        else:
            t = time.time()
            mats, _ = workloads.cfg2_batch(512, 32, 512, "float32")
            vals = [oracle.svd_values(a, threads=args.threads) for a in mats]
            np.save(out, np.concatenate(vals))
            print(f"cfg2_b512_float32: {time.time() - t:.1f}s, {sum(len(v) for v in vals)} values", flush=True)
    for name, make in jobs:
        out = path_for(name)
        if os.path.exists(out):
            print("exists", out, flush=True)
            continue
        a = make()
        t = time.time()
        info = {}
        s = oracle.svd_values(a, threads=args.threads, info=info)
        np.save(out, s)
        write_info(name, info, time.time() - t, args.threads)
        print(f"{name}: {time.time() - t:.1f}s sweeps={info['sweeps']}", flush=True)


if __name__ == "__main__":
    main()
