"""Train the warm-start network on the generated instances of the
learned-start study.

    python -m paper_2402_08134_amd.train_warmstart --out weights/warmstart.bin

Instances (workloads.warm_instance): ids 0..1799 are the training pool --
stochastic block model graphs (even ids) and Gaussian-kernel similarities
(odd ids), n uniform in [4096, 32768], k in {16, 32, 64}; ids 1800..1999 are
held out and never touched here.  For each training instance, in id order
until --count instances or the --budget seconds of data preparation are used
up: a plain FP32 run from the random start until the stall rule stops it
(at most 1000 iterations), the LAI basis (l = k + 16, q = 2), the entry
features and the aligned targets; --entries entries of each instance are
drawn at random into the training pool.  The network is shared by all
columns, all k and both kinds of input, and is trained with Adam on shuffled
batches of the pool.  Everything runs on the GPU through the library except
data generation and the target alignment (an assignment problem on the
host).  Writes the network (library file format) and a JSON record of the
run beside it (--out + ".json").
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--count", type=int, default=1800, help="training instances (ids 0..count-1)")
    ap.add_argument("--budget", type=float, default=600.0, help="seconds of data preparation at most")
    ap.add_argument("--entries", type=int, default=65536, help="entries drawn from each instance")
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    sys.path.insert(0, ROOT)
    import torch
    import paper_2402_08134_amd as P
    from paper_2402_08134_amd import warmstart as WSP
    import workloads

    def log(msg):
        print(msg, flush=True)

    rng = np.random.default_rng(args.seed)
    t0 = time.time()
    Fs, Ts, used = [], [], []
    for i in list(workloads.WARM_TRAIN_IDS)[:args.count]:
        if time.time() - t0 > args.budget:
            break
        spec = workloads.warm_instance(i)
        n, k = spec["n"], spec["k"]
        X = workloads.warm_instance_data(spec)
        if spec["kind"] == "sbm":
            Xd = (torch.from_numpy(X.indptr.astype(np.int32)).cuda(), torch.from_numpy(X.indices.astype(np.int32)).cuda(),
                  torch.from_numpy(X.data).cuda(), n)
        else:
            Xd = X
        F, T, iters = WSP.instance_data(Xd, k, k + 16, 2, seed=1, max_iters=1000)
        m = min(args.entries, n * k)
        idx = np.sort(rng.choice(n * k, size=m, replace=False))
        Fs.append(F[torch.from_numpy(idx).cuda()].contiguous())
        Ts.append(torch.from_numpy(T[idx]).cuda())
        used.append({"id": i, "kind": spec["kind"], "n": n, "k": k, "plain_iterations": int(iters)})
        del F, X, Xd
        log(f"instance {i}: {spec['kind']} n={n} k={k} plain iterations {iters}  [{time.time() - t0:.0f}s]")
    Fp = torch.cat(Fs)
    Tp = torch.cat(Ts)
    del Fs, Ts
    t1 = time.time()
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, args.seed + 7)
    losses = WSP.train_pooled(net, Fp, Tp, args.epochs, args.lr, args.batch, seed=args.seed, log=log,
                              lr_final=args.lr_final)
    log(f"trained on {Fp.shape[0]} entries of {len(used)} instances in {time.time() - t1:.0f}s")
    WSP.save(net, args.out)
    meta = {"instances": len(used), "ids": [u["id"] for u in used], "entries_per_instance": args.entries,
            "pool_entries": int(Fp.shape[0]), "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "lr_final": args.lr_final,
            "seed": args.seed, "losses": losses, "prep_seconds": round(t1 - t0, 1),
            "train_seconds": round(time.time() - t1, 1), "per_instance": used}
    with open(args.out + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(json.dumps({k: v for k, v in meta.items() if k not in ("ids", "per_instance")}))


if __name__ == "__main__":
    main()
