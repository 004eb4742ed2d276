"""Benchmark: SymNMF time-to-residual on one MI355X.

Workload: dense similarity, n = 16384, k = 32, FP32 -- the Gaussian-kernel
matrix of a 32-component Gaussian mixture in R^64 (zero diagonal), the
synthetic stand-in for the paper's dense Web-of-Science similarity matrix.

One step = one whole solve from the data resident in HBM: create (scalars
pass, random init), then regularised HALS iterations until the normalised
residual reaches r* = r_conv + 1e-3, where r_conv is the residual at which the
plain random-init method stops under the paper's rule (no drop > 1e-4 for four
iterations).  `value` is seconds per solve with the learned start (LAI basis
l = k + 16, q = 2, the trained network of paper_2402_08134_amd/weights, the
least-squares scale fit, then iterations on X); the plain random-start solve,
the LAI method (Algorithm LAI-SymNMF followed by refinement on X) and the
learned start followed by LAI iterations are reported beside it.

Also reported: the live roofline of the dominant kernel (the X H product,
timed with HIP events on the solve stream inside the timed solves), the
per-phase device time, and the FP64 CPU oracle timed on a bounded sample on
the host cores.  `--pmc-probe` runs the short fixed workload the rocprofv3
counter passes are taken on.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--dim", type=int, default=64)
    ap.add_argument("--comps", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run the short counter-collection workload and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.pmc_probe:
        pmc_probe(args)
        return

    import numpy as np
    import torch
    import paper_2402_08134_amd as P
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    P.lib()
    n, k = args.n, args.k
    l, q = k + 16, 2
    t0 = time.time()
    Xh, _ = workloads.gaussian_kernel(n, args.dim, args.comps, seed=0, dtype=np.float32)
    log(f"[bench] generated X n={n} in {time.time() - t0:.1f}s")
    X = torch.from_numpy(Xh).cuda()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    # Reference convergence level (untimed): plain random init, paper's rule.
    o = P.symnmf_default_options(stop_mode=P.STOP_STALL, check_every=8)
    ctx = P.symnmf_create(X, k, 0.0, 0, 1, o)
    iters_conv = P.symnmf_iterate(ctx, 2000)
    r_conv = P.symnmf_residual(ctx, P.RESID_EXACT)[0]
    r_star = r_conv + 1e-3
    del ctx
    log(f"[bench] plain converged: {iters_conv} iterations, residual {r_conv:.6f}; r* = {r_star:.6f}")

    def solve_plain(seed):
        o = P.symnmf_default_options(stop_mode=P.STOP_TARGET, target=r_star, check_every=4, timing=1)
        c = P.symnmf_create(X, k, 0.0, 0, seed, o)
        it = P.symnmf_iterate(c, 4000)
        return c, it

    def solve_learned(seed, lai_first):
        # learned start: LAI basis, network, scale fit; then (optionally LAI
        # iterations until their own residual stalls, then) refinement on X
        o = P.symnmf_default_options(stop_mode=P.STOP_STALL if lai_first else P.STOP_TARGET,
                                     target=r_star, check_every=4, timing=1)
        c = P.symnmf_create(X, k, 0.0, 0, seed, o)
        P.symnmf_lai(c, l, q)
        beta = P.symnmf_warmstart(c, net)
        it = P.symnmf_iterate(c, 2000) if lai_first else 0
        P.symnmf_refine(c, P.STOP_TARGET, r_star)
        it2 = P.symnmf_iterate(c, 4000)
        return c, it + it2, it2, beta

    def solve_lai(seed):
        # LAI phase until its own residual stalls, then refinement on X.
        o = P.symnmf_default_options(stop_mode=P.STOP_STALL, check_every=8, timing=1)
        c = P.symnmf_create(X, k, 0.0, 0, seed, o)
        P.symnmf_lai(c, l, q)
        it = P.symnmf_iterate(c, 2000)
        P.symnmf_refine(c, P.STOP_TARGET, r_star)
        it2 = P.symnmf_iterate(c, 4000)
        return c, it + it2, it2

    from paper_2402_08134_amd import warmstart as WSP
    net = WSP.load(os.path.join(WSP.WEIGHTS_DIR, "warmstart_gk.npz"))

    for w in range(args.warmup):
        solve_plain(100 + w)
        solve_lai(100 + w)
        solve_learned(100 + w, False)
        solve_learned(100 + w, True)
    torch.cuda.synchronize()

    # timed: plain
    seeds = [1 + s for s in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_iters = []
    ctxs = []
    for sd in seeds:
        c, it = solve_plain(sd)
        plain_iters.append(it)
        ctxs.append(c)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / args.steps
    plain_res = [P.symnmf_residual(c, P.RESID_EXACT)[0] for c in ctxs]
    plain_phases = phase_totals(P, ctxs)
    del ctxs

    # timed: LAI + refinement
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lai_iters, lai_refine, ctxs = [], [], []
    for sd in seeds:
        c, it, it2 = solve_lai(sd)
        lai_iters.append(it)
        lai_refine.append(it2)
        ctxs.append(c)
    torch.cuda.synchronize()
    t_lai = (time.perf_counter() - t0) / args.steps
    lai_res = [P.symnmf_residual(c, P.RESID_EXACT)[0] for c in ctxs]
    lai_phases = phase_totals(P, ctxs)
    del ctxs
    learned = {}
    for lai_first in (False, True):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, its2, betas, ctxs = [], [], [], []
        for sd in seeds:
            c, it, it2, beta = solve_learned(sd, lai_first)
            its.append(it)
            its2.append(it2)
            betas.append(beta)
            ctxs.append(c)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        res = [P.symnmf_residual(c, P.RESID_EXACT)[0] for c in ctxs]
        ph = phase_totals(P, ctxs)
        del ctxs
        name = "learned_then_lai" if lai_first else "learned"
        learned[name] = {"s_per_solve": t, "iterations": its, "iterations_on_X": its2, "beta": betas,
                         "final_residual": res, "speedup_vs_plain": None,
                         "phases_ms_per_solve": {kk: v[0] / args.steps for kk, v in ph.items()}}
        log(f"[bench] {name} {t * 1e3:.2f} ms/solve iters {its} (on X {its2}) res {res}")
    log(f"[bench] plain {t_plain * 1e3:.2f} ms/solve iters {plain_iters} res {plain_res}")
    log(f"[bench] lai   {t_lai * 1e3:.2f} ms/solve iters {lai_iters} (refine {lai_refine}) res {lai_res}")

    # Live roofline of the dominant kernel, the X H product of each
    # half-iteration (one GEMM launch): its device time comes from the HIP
    # events the library records around that launch on the solve stream
    # during the timed plain solves above.
    ms, calls = plain_phases["product"]
    t_prod = ms / 1e3 / calls
    alg_bytes = float(n) * n * 4 + 2.0 * n * k * 4
    achieved = alg_bytes / t_prod / 1e9
    log(f"[bench] X*H product {t_prod * 1e6:.1f} us over {calls} launches -> {achieved:.0f} GB/s algorithmic")
    traffic = stored_traffic(n, k)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(Xh, k, int(np.median(plain_iters)))

    for v in learned.values():
        v["speedup_vs_plain"] = t_plain / v["s_per_solve"]
    t_learned = learned["learned"]["s_per_solve"]
    out = {
        "metric": "SymNMF time-to-residual (s) and X*H GB/s or MFMA %, learned-init vs plain",
        "value": t_learned,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_learned * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"dense Gaussian-kernel similarity n={n} k={k} FP32 "
                               f"(32-component GMM in R^64), HALS to r*=r_conv+1e-3; value: learned start "
                               f"(LAI basis l={l}, q={q}, network, scale fit) then iterations on X",
                   "n": n, "k": k, "r_conv": r_conv, "r_star": r_star,
                   "plain": {"s_per_solve": t_plain, "iterations": plain_iters, "final_residual": plain_res},
                   "learned_vs_plain": t_plain / t_learned,
                   **learned,
                   "plain_iterations": plain_iters,
                   "lai": {"l": l, "q": q, "s_per_solve": t_lai, "iterations": lai_iters,
                           "refine_iterations": lai_refine, "speedup_vs_plain": t_plain / t_lai}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_gemm_mfma<float,2,4,true> (X H, one launch per half-iteration)",
                     "us_per_launch": t_prod * 1e6, "launches": calls,
                     "algorithmic_bytes_per_launch": alg_bytes},
        "phases_ms_per_solve": {"plain": {kk: v[0] / args.steps for kk, v in plain_phases.items()},
                                "lai": {kk: v[0] / args.steps for kk, v in lai_phases.items()}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def phase_totals(P, ctxs):
    """Summed (ms, launches) per phase over the contexts of a timed loop."""
    names = {P.PHASE_PRODUCT: "product", P.PHASE_UPDATE: "update", P.PHASE_SAMPLE: "sample", P.PHASE_LAI: "lai"}
    tot = {v: [0.0, 0] for v in names.values()}
    for c in ctxs:
        st = P.symnmf_get_stats(c)
        for ph, name in names.items():
            tot[name][0] += st.phase_ms[ph]
            tot[name][1] += st.phase_calls[ph]
    return tot


def stored_traffic(n, k):
    """HBM bytes per launch of the product kernel from the committed
    rocprofv3 counter summary, or None when that summary is missing, was
    taken at another size, or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_gemm_mfma_f32_gk16384_k32_pmc.txt")
    src = os.path.join(ROOT, "paper_2402_08134_amd", "csrc", "k_dense.hip")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            key, _, val = line.partition(":")
            kv[key.strip()] = val.strip()
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("k_dense.hip sha256") != digest or kv.get("n") != str(n) or kv.get("k") != str(k):
        return None
    try:
        return float(kv["hbm bytes per launch (scaled)"])
    except (KeyError, ValueError):
        return None


def pmc_probe(args):
    """Short fixed workload for the rocprofv3 counter passes: a 1 GiB device
    copy (the calibration kernel of known traffic), then ten plain
    iterations at the bench size."""
    import numpy as np
    import torch
    import paper_2402_08134_amd as P
    import workloads
    Xh, _ = workloads.gaussian_kernel(args.n, args.dim, args.comps, seed=0, dtype=np.float32)
    X = torch.from_numpy(Xh).cuda()
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("[pmc-probe] copies done (3 x 1 GiB read + 1 GiB write)")
    c = P.symnmf_create(X, args.k, 0.0, 0, 1)
    P.symnmf_iterate(c, 10)
    torch.cuda.synchronize()
    log("[pmc-probe] 10 plain iterations done")


def cpu_baseline(Xh, k, iters_gpu):
    """The FP64 oracle (as it stands) on the host: two plain HALS iterations
    on the same matrix, scaled to the iterations the GPU needed."""
    import numpy as np
    from oracle import symnmf as O
    t0 = time.perf_counter()
    sc = O.data_scalars(Xh)
    t_sc = time.perf_counter() - t0
    H0 = O.initial_factor(Xh.shape[0], k, sc["zeta"], 1)
    it = 2
    t0 = time.perf_counter()
    O.plain_symnmf(Xh, k, sc["maxval"], H0, it)
    t_it = (time.perf_counter() - t0) / it
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return {"value": t_sc + t_it * iters_gpu, "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": f"{it} plain HALS iterations + scalars pass on the same X, "
                      f"scaled to {iters_gpu} iterations ({t_it:.2f} s/iteration)"}


if __name__ == "__main__":
    main()
