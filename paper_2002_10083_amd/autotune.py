"""Run the tuner on the benchmark workload and record the result:
python -m paper_2002_10083_amd.autotune [--n N]"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--key", default="iterate")
    args = ap.parse_args()
    import torch
    from mclgen import config1_graph
    from paper_2002_10083_amd import mcl, tuning
    W = config1_graph(n=args.n, n_clusters=max(1, args.n // 20))
    A = mcl.DeviceCSC.from_host(W)
    mcl.normalize_(A)

    def run(policy, scale):
        G, _, st = mcl.iterate(A, bin_policy=policy, est_scale=scale)
        del G
        return st

    t = time.time()
    policy, scale, rep = tuning.tune(run)
    rep["tune_s"] = round(time.time() - t, 1)
    rep["gpu"] = torch.cuda.get_device_name(0)
    tuning.save_policy(args.key, policy, scale, rep)
    print("tuned", hex(policy), scale, rep, flush=True)


if __name__ == "__main__":
    main()
