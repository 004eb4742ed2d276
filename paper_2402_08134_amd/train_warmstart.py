"""Train the warm-start network on synthetic dense similarity instances.

    python -m paper_2402_08134_amd.train_warmstart --out weights.npz

Instances: Gaussian-kernel matrices of equal-weight Gaussian mixtures (k
components in R^{2k}, the construction of the dense benchmarks), n drawn
uniformly from [n_min, n_max], k from --ks.  For each: a plain FP32 run from
the random start until the stall rule stops it, the LAI basis (l = k + 16,
q = 2), the entry features and the aligned targets.  The network is shared by
all columns and all k, and is trained with Adam on shuffled batches of
entries pooled from every instance; the last instances are held out and
evaluated: iterations to r* = r_conv + 1e-3 from the random start and from
the learned start.  Everything runs on the GPU except data generation and
the target alignment.
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
    ap.add_argument("--instances", type=int, default=24)
    ap.add_argument("--held-out", type=int, default=3)
    ap.add_argument("--n-min", type=int, default=3000)
    ap.add_argument("--n-max", type=int, default=8192)
    ap.add_argument("--ks", default="16,32,64")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
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
    ks = [int(v) for v in args.ks.split(",")]
    t0 = time.time()
    train, held = [], []
    for i in range(args.instances):
        n = int(rng.integers(args.n_min, args.n_max + 1))
        k = int(ks[rng.integers(len(ks))])
        X, _ = workloads.gaussian_kernel(n, 2 * k, k, seed=1000 + i, dtype=np.float32)
        Xd = torch.from_numpy(X).cuda()
        if i >= args.instances - args.held_out:
            held.append((Xd, k))
            log(f"instance {i}: n={n} k={k} held out  [{time.time() - t0:.0f}s]")
            continue
        F, T, iters = WSP.instance_data(Xd, k, k + 16, 2, seed=1)
        train.append((F, T))
        del Xd
        log(f"instance {i}: n={n} k={k} plain iterations {iters}  [{time.time() - t0:.0f}s]")
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, args.seed + 7)
    losses = WSP.train(net, train, args.epochs, args.lr, args.batch, seed=args.seed, log=log)
    log(f"trained in {time.time() - t0:.0f}s")
    evals = []
    for Xd, k in held:
        o = P.symnmf_default_options(stop_mode=P.STOP_STALL, check_every=4)
        ref = P.symnmf_create(Xd, k, 0.0, 0, 5, o)
        P.symnmf_iterate(ref, 4000)
        r_star = P.symnmf_residual(ref, P.RESID_EXACT)[0] + 1e-3

        def iters_from(netw):
            o = P.symnmf_default_options(stop_mode=P.STOP_TARGET, target=r_star, check_every=1)
            c = P.symnmf_create(Xd, k, 0.0, 0, 5, o)
            if netw is not None:
                P.symnmf_lai(c, k + 16, 2)
                P.symnmf_warmstart(c, netw)
                P.symnmf_refine(c, P.STOP_TARGET, r_star)
            return P.symnmf_iterate(c, 4000)

        ev = {"n": int(Xd.shape[0]), "k": k, "random": iters_from(None), "learned": iters_from(net)}
        evals.append(ev)
        log(f"held out n={ev['n']} k={k}: iterations to r*: random {ev['random']}, learned {ev['learned']}")
    meta = {"instances": args.instances, "held_out": args.held_out, "n_range": [args.n_min, args.n_max],
            "ks": ks, "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "seed": args.seed,
            "losses": losses, "held_out_eval": evals}
    WSP.save(net, args.out, meta)
    log(json.dumps(meta))


if __name__ == "__main__":
    main()
