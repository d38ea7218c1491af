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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="*", default=[1024, 2048, 4096])
    ap.add_argument("--dtypes", nargs="*", default=["float32", "float64"])
    ap.add_argument("--cfg3", action="store_true", help="also the n=8192 cond-1e4 matrix (slow)")
    ap.add_argument("--cfg2", action="store_true",
                    help="also the batch of 512 float32 matrices (n uniform in [32, 512]): one packed array of "
                         "every matrix's values in batch order")
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    jobs = [(f"cfg1_n{n}_{dt}", lambda n=n, dt=dt: workloads.cfg1_matrix(n, dt))
            for n in args.sizes for dt in args.dtypes]
    if args.cfg3:
        jobs.append(("cfg3_n8192_float32", lambda: workloads.cfg3_matrix(8192, "float32")))
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
        print(f"{name}: {time.time() - t:.1f}s sweeps={info['sweeps']}", flush=True)


if __name__ == "__main__":
    main()
