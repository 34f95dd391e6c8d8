"""Run the tuner on a benchmark workload and record the result:
python -m paper_2002_10083_amd.autotune [--n N] [--workload iterate|batched --key KEY]"""
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
    ap.add_argument("--persist-only", action="store_true",
                    help="keep the stored launch shapes of --key and only decide whether bins 0-6 "
                         "accumulate in one persistent launch")
    ap.add_argument("--scale-only", default=None,
                    help="keep the stored launch shapes and key count of --key and choose the estimate "
                         "scale (table sizing margin) from this comma-separated list")
    ap.add_argument("--workload", default="iterate", choices=["iterate", "batched"],
                    help="iterate: one fused iteration of the 1M-vertex graph; batched: the first three "
                         "iterations of the 20,000-component graph, all components per call")
    args = ap.parse_args()
    import torch
    from mclgen import config1_graph, config3_graph
    from paper_2002_10083_amd import mcl, tuning
    if args.workload == "batched":
        W = config3_graph()
        comp = torch.from_numpy(W.comp_ptr).cuda()
    else:
        W = config1_graph(n=args.n, n_clusters=max(1, args.n // 20))
        comp = None
    A = mcl.DeviceCSC.from_host(W)
    mcl.normalize_(A)

    def run(policy, scale, keys):
        if comp is None:
            G, _, st = mcl.iterate(A, bin_policy=policy, est_scale=scale, cohen_keys=keys)
            del G
            return st
        # three iterations, per-bin times and columns summed
        X, tot = A, None
        active = torch.ones(comp.numel() - 1, dtype=torch.uint8, device="cuda")
        for it in range(3):
            X, _, st = mcl.iterate(X, bin_policy=policy, est_scale=scale, cohen_keys=keys, comp_ptr=comp,
                                   active=active, iteration=it)
            if tot is None:
                tot = st
            else:
                for k in ("bin_ms", "bin_cols"):
                    tot[k] = [a + b for a, b in zip(tot[k], st[k])]
                tot["n_overflow"] += st["n_overflow"]
        return tot

    t = time.time()
    if args.scale_only:
        import json
        policy, scale, keys = tuning.load_policy(args.key)
        with open(tuning.TUNED) as f:
            rep = json.load(f).get(args.key, {})
        for k in ("bin_policy", "est_scale", "cohen_keys"):
            rep.pop(k, None)
        times = {}
        for sc in [float(x) for x in args.scale_only.split(",")]:
            best = None
            for _ in range(2):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st = run(policy, sc, keys)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t1) * 1e3
                best = dt if best is None else min(best, dt)
            times[sc] = round(best, 3)
            print("scale %.2f: %.1f ms (overflow %d)" % (sc, best, st["n_overflow"]), flush=True)
        scale = min(times, key=lambda k: times[k])
        rep["scale_ms"] = {str(k): v for k, v in times.items()}
        tuning.save_policy(args.key, policy, scale, keys, rep)
        if args.copy_to:
            tuning.save_policy(args.key, policy, scale, keys, rep, path=args.copy_to)
        print("tuned", hex(policy), scale, keys, times, flush=True)
        return
    if args.persist_only:
        policy, scale, keys = tuning.load_policy(args.key)
        with open(tuning.TUNED) as f:
            import json
            rep = json.load(f).get(args.key, {})
        rep.pop("bin_policy", None)
        rep.pop("est_scale", None)
        rep.pop("cohen_keys", None)
        policy, rep["persist"] = tuning.decide_persist(run, policy, scale, keys)
        tuning.save_policy(args.key, policy, scale, keys, rep)
        if args.copy_to:
            tuning.save_policy(args.key, policy, scale, keys, rep, path=args.copy_to)
        print("tuned", hex(policy), scale, keys, rep["persist"], flush=True)
        return
    if args.workload == "batched":
        # three iterations per trial: one measurement each, only the launch
        # shapes that were within 30 % of the best on the 1M-vertex graph,
        # and that graph's Cohen key count and margin
        _, sc0, k0 = tuning.load_policy("iterate")
        policy, scale, keys, rep = tuning.tune(run, reps=1, candidates=tuning.candidates_from("iterate"),
                                               scales=(sc0,), keys=(k0,))
    else:
        policy, scale, keys, rep = tuning.tune(run)
    policy, rep["persist"] = tuning.decide_persist(run, policy, scale, keys)
    rep["tune_s"] = round(time.time() - t, 1)
    rep["gpu"] = torch.cuda.get_device_name(0)
    tuning.save_policy(args.key, policy, scale, keys, rep)
    if args.copy_to:
        tuning.save_policy(args.key, policy, scale, keys, rep, path=args.copy_to)
    print("tuned", hex(policy), scale, keys, rep, flush=True)


if __name__ == "__main__":
    main()
