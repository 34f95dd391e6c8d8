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
    ap.add_argument("--copy-to", default=None, help="also write the table to this file")
    args = ap.parse_args()
    import torch
    from mclgen import config1_graph
    from paper_2002_10083_amd import mcl, tuning
    W = config1_graph(n=args.n, n_clusters=max(1, args.n // 20))
    A = mcl.DeviceCSC.from_host(W)
    mcl.normalize_(A)

    def run(policy, scale, keys):
        G, _, st = mcl.iterate(A, bin_policy=policy, est_scale=scale, cohen_keys=keys)
        del G
        return st

    t = time.time()
    policy, scale, keys, rep = tuning.tune(run)
    rep["tune_s"] = round(time.time() - t, 1)
    rep["gpu"] = torch.cuda.get_device_name(0)
    tuning.save_policy(args.key, policy, scale, keys, rep)
    if args.copy_to:
        tuning.save_policy(args.key, policy, scale, keys, rep, path=args.copy_to)
    print("tuned", hex(policy), scale, keys, rep, flush=True)


if __name__ == "__main__":
    main()
