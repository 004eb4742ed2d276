"""Benchmark: SymNMF time-to-residual on one MI355X.

Workload: dense similarity, n = 16384, k = 32, FP32 -- the Gaussian-kernel
matrix of a 32-component Gaussian mixture in R^64 (zero diagonal), the
synthetic stand-in for the paper's dense Web-of-Science similarity matrix.

One step = one whole solve from the data resident in HBM: create (scalars
pass, random init), then regularised HALS iterations until the normalised
residual reaches r* = r_conv + 1e-3, where r_conv is the residual at which the
plain random-init method stops under the paper's rule (no drop > 1e-4 for four
iterations).  The HALS methods timed: plain (random start, iterations on X),
lai (Algorithm LAI-SymNMF from the random start until its own residual
stalls, then refinement on X until the residual on X is r*), learned (the learned start -- LAI basis
l = k + 16, q = 2, the trained network of paper_2402_08134_amd/weights and
the least-squares scale fit -- then iterations on X) and learned_lai (the
learned start, LAI iterations as in lai, then refinement on X); also
learned_lai_ada, the same with the basis of Algorithm Ada-RRF (q chosen on
the fly, tolerance 1e-3, at most 10 rounds) instead of q = 2.  The PGNCG
rows (Section 2.1.3) follow the paper's protocol instead -- iterate until the
stall rule stops them, and report time and residual: pgncg (random start, on
X), lai_pgncg (Algorithm LAI-PGNCG-SymNMF) and lai_pgncg_ir (then refinement
on X).  `value` is seconds per solve of learned_lai; every method's time,
iteration counts, final residuals and speed-up over plain are in
`config.methods`.

The timed solves replay their iterations from HIP graphs and record no
events.  A second pass runs each method once more with HIP events around
every phase's launches (eager launches): it gives the per-phase device time
and the live roofline of the dominant kernel (the X H product).  Also
reported: the FP64 CPU oracle timed on a bounded sample on the host cores.
`--pmc-probe` runs the short fixed workload the rocprofv3 counter passes are
taken on (with `--workload sparse`: the CSR product's).

The default run also measures the other workloads and puts their records
under config.workloads (each with its own roofline; --only-headline skips
them): sparse (SBM graph n = 2^20, k = 64: plain CSR HALS, BF16 gathers,
leverage-score sampling, SpMM roofline), precision (n = 65536, k = 64 in FP32
and BF16, product rates against HBM and the matrix-core peaks, the FP64
oracle's check of both) and warmstart (the learned start against the random
start on the 200 held-out generated instances).  Each can also be run alone
with --workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0


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
    ap.add_argument("--only-headline", action="store_true",
                    help="default workload only, without the sparse, precision and learned-start workloads")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run the short counter-collection workload and exit")
    ap.add_argument("--workload", choices=["dense", "sparse", "precision", "warmstart"], default="dense",
                    help="dense: the Gaussian-kernel similarity (default, the headline line); "
                         "sparse: the normalised SBM graph, plain CSR HALS vs leverage-score sampling; "
                         "precision: n = 65536, k = 64 dense similarity in FP32 and BF16; "
                         "warmstart: learned start vs random start on the held-out generated instances")
    ap.add_argument("--warm-count", type=int, default=200, help="held-out instances evaluated")
    ap.add_argument("--warm-first", type=int, default=0, help="index of the first held-out instance")
    ap.add_argument("--warm-weights", default=None, help="network file (default: the committed one)")
    ap.add_argument("--warm-out", default=None, help="also write the per-instance records to this JSON file")
    ap.add_argument("--precision-n", type=int, default=65536)
    ap.add_argument("--precision-oracle-iters", type=int, default=2,
                    help="iterations of the precision workload's oracle check (the converged run: 80)")
    ap.add_argument("--sparse-n", type=int, default=1 << 20)
    ap.add_argument("--sparse-k", type=int, default=64)
    ap.add_argument("--sparse-s", type=int, default=8192)
    ap.add_argument("--sparse-iters", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.pmc_probe:
        if args.workload == "sparse":
            pmc_probe_sparse(args)
        else:
            pmc_probe(args)
        return
    if args.workload == "sparse":
        print(json.dumps(bench_sparse(args)), flush=True)
        return
    if args.workload == "precision":
        print(json.dumps(bench_precision(args)), flush=True)
        return
    if args.workload == "warmstart":
        print(json.dumps(bench_warmstart(args)), flush=True)
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
    torch.cuda.synchronize()

    # Reference convergence level (untimed): plain random init, paper's rule.
    o = P.symnmf_default_options(stop_mode=P.STOP_STALL, check_every=8)
    ctx = P.symnmf_create(X, k, 0.0, 0, 1, o)
    iters_conv = P.symnmf_iterate(ctx, 2000)
    r_conv = P.symnmf_residual(ctx, P.RESID_EXACT)[0]
    r_star = r_conv + 1e-3
    del ctx
    log(f"[bench] plain converged: {iters_conv} iterations, residual {r_conv:.6f}; r* = {r_star:.6f}")

    from paper_2402_08134_amd import warmstart as WSP
    net = WSP.load(os.path.join(WSP.WEIGHTS_DIR, "warmstart.bin"))

    def solve(method, seed, timing):
        """One solve to r* (PGNCG methods: to the stall rule); returns
        (context, iterations, iterations on X)."""
        if "pgncg" in method:
            o = P.symnmf_default_options(rule=P.RULE_PGNCG, stop_mode=P.STOP_STALL, check_every=8, timing=timing)
            c = P.symnmf_create(X, k, 0.0, 0, seed, o)
            if method == "pgncg":
                it = P.symnmf_iterate(c, 4000)
                return c, it, it
            P.symnmf_lai(c, l, q)
            it = P.symnmf_iterate(c, 2000)
            if method == "lai_pgncg":
                return c, it, 0
            P.symnmf_refine(c, P.STOP_STALL)
            it2 = P.symnmf_iterate(c, 4000)
            return c, it + it2, it2
        lai_stage = method in ("lai", "learned_lai", "learned_lai_ada")
        # LAI stage until its own residual stalls (stopping it at r* instead
        # leaves the residual on X far above r*: measured slower); then
        # iterations on X until the residual on X is r*
        o = P.symnmf_default_options(stop_mode=P.STOP_STALL if lai_stage else P.STOP_TARGET,
                                     target=r_star, check_every=8 if lai_stage else 4, timing=timing)
        c = P.symnmf_create(X, k, 0.0, 0, seed, o)
        if method == "plain":
            it = P.symnmf_iterate(c, 4000)
            return c, it, it
        if method.endswith("_ada"):
            P.symnmf_lai_adaptive(c, l, 10, 1e-3)
        else:
            P.symnmf_lai(c, l, q)
        if method.startswith("learned"):
            P.symnmf_warmstart(c, net, want_beta=False)
        it = P.symnmf_iterate(c, 2000) if lai_stage else 0
        P.symnmf_refine(c, P.STOP_TARGET, r_star)
        it2 = P.symnmf_iterate(c, 4000)
        return c, it + it2, it2

    methods = ["plain", "lai", "learned", "learned_lai", "learned_lai_ada", "pgncg", "lai_pgncg", "lai_pgncg_ir"]
    # Warm-up: as many contexts alive at once as the timed loop keeps, so the
    # library's device-block cache holds their buffers (a service solving
    # repeatedly runs from that cache; device allocation is not solve time).
    for w in range(args.warmup):
        for m in methods:
            live = [solve(m, 100 + w * args.steps + s, 0)[0] for s in range(args.steps)]
            torch.cuda.synchronize()
            del live
    torch.cuda.synchronize()

    # Timed: whole solves, graphs on, no per-launch events.
    seeds = [1 + s for s in range(args.steps)]
    res = {}
    for m in methods:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, its_x, ctxs = [], [], []
        for sd in seeds:
            c, it, itx = solve(m, sd, 0)
            its.append(it)
            its_x.append(itx)
            ctxs.append(c)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        finals = [P.symnmf_residual(c, P.RESID_EXACT) for c in ctxs]
        final = [float(v[0]) for v in finals]
        beta = [P.symnmf_get_stats(c).warm_beta for c in ctxs]
        del ctxs
        res[m] = {"s_per_solve": t, "iterations": its, "iterations_on_X": its_x, "final_residual": final,
                  "final_residual_HHt": [float(v[1]) for v in finals],
                  "stop": "stall rule" if "pgncg" in m else "r*"}
        if m.startswith("learned"):
            res[m]["warm_beta"] = beta
        log(f"[bench] {m:12s} {t * 1e3:8.2f} ms/solve  iterations {its} (on X {its_x})  final residual "
            f"{['%.6f' % v for v in final]}")
    t_plain = res["plain"]["s_per_solve"]
    for m in methods:
        res[m]["speedup_vs_plain"] = t_plain / res[m]["s_per_solve"]

    # Phase pass: the same solves once more with HIP events around every
    # phase's launches (eager launches); the product kernel's average launch
    # time gives the live roofline of the dominant kernel.
    phases = {}
    for m in methods:
        c, _, _ = solve(m, seeds[0], 1)
        phases[m] = phase_totals(P, [c])
        del c
    ms, calls = phases["plain"]["product"]
    t_prod = ms / 1e3 / calls
    alg_bytes = float(n) * n * 4 + 2.0 * n * k * 4
    achieved = alg_bytes / t_prod / 1e9
    log(f"[bench] X*H product {t_prod * 1e6:.1f} us over {calls} launches -> {achieved:.0f} GB/s algorithmic")
    traffic = stored_traffic("k_gemm_cols_f32_gk16384_k32_pmc.txt", "k_dense.hip", n, k)

    # The dominant kernel of the timed learned_lai solve by device time is
    # the LAI update (two launches per LAI iteration): timed alone on a
    # context in LAI mode after the learned start (HIP events around every
    # update launch).  Algorithmic bytes per launch: U (its n x l FP32 copy),
    # the source factor and the old factor read, the new factor written
    # (n x k FP32 each): n (4 l + 12 k).
    o = P.symnmf_default_options(timing=1)
    c = P.symnmf_create(X, k, 0.0, 0, seeds[0], o)
    P.symnmf_lai(c, l, q)
    P.symnmf_warmstart(c, net, want_beta=False)
    P.symnmf_iterate(c, 40)
    ph = phase_totals(P, [c])
    del c
    t_upd = ph["update"][0] / 1e3 / ph["update"][1]
    t_red = ph["reduce"][0] / 1e3 / ph["reduce"][1]
    alg_upd = float(n) * (4.0 * l + 12.0 * k)
    ach_upd = alg_upd / t_upd / 1e9
    log(f"[bench] LAI update {t_upd * 1e6:.1f} us over {ph['update'][1]} launches -> {ach_upd:.0f} GB/s "
        f"algorithmic; partial-sum reduction {t_red * 1e6:.1f} us")
    traffic_upd = stored_traffic("k_update_lai_gk16384_k32_l48_pmc.txt", "k_update.hip", n, k)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] oracle: one learned_lai solve on the host ...")
        cpu = cpu_baseline(Xh, k, l, q, net_params_host(P, net), r_star)
        log(f"[bench] oracle learned_lai solve {cpu['value']:.1f} s ({cpu['sample']})")

    t_val = res["learned_lai"]["s_per_solve"]
    out = {
        "metric": "SymNMF time-to-residual (s) and X*H GB/s or MFMA %, learned-init vs plain",
        "value": t_val,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_val * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"dense Gaussian-kernel similarity n={n} k={k} FP32 (32-component GMM in R^64), "
                               f"HALS to r* = r_conv + 1e-3; value: learned start (LAI basis l={l}, q={q}, "
                               f"trained network, scale fit), LAI iterations, refinement on X",
                   "n": n, "k": k, "l": l, "q": q, "r_conv": r_conv, "r_star": r_star,
                   "learned_vs_plain": t_plain / t_val,
                   "methods": res,
                   # the X H product (the plain method's dominant kernel)
                   "roofline_xh": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                                   "kernel": "k_gemm_cols<2, 2, true> (X H read along rows of X)",
                                   "us_per_launch": t_prod * 1e6, "launches": calls,
                                   "algorithmic_bytes_per_launch": alg_bytes,
                                   "mfma_tflops": 2.0 * n * n * k / t_prod / 1e12,
                                   "mfma_frac": 2.0 * n * n * k / t_prod / 1e12 / FP32_MFMA_PEAK_TFLOPS}},
        "roofline": {"bound": "hbm", "achieved": ach_upd, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach_upd / HBM_PEAK_GBS, "traffic": traffic_upd,
                     "kernel": "k_update<32, 48, float, float, float, 2, 8> (fused LAI update: U M + alpha F, "
                               "HALS sweep, new factor, block partials of F^T F and U^T F; two launches per LAI "
                               "iteration, the largest device-time share of the learned_lai solve)",
                     "us_per_launch": t_upd * 1e6, "launches": ph["update"][1],
                     "algorithmic_bytes_per_launch": alg_upd,
                     "reduction_us_per_launch": t_red * 1e6},
        "phases_ms_per_solve": {m: {kk: v[0] for kk, v in ph.items()} for m, ph in phases.items()},
        "cpu_baseline": cpu,
    }
    if not args.only_headline:
        # the other workloads, each with its own roofline: the sparse graph,
        # the precision sweep and the learned-start study
        del X, Xh, net
        torch.cuda.empty_cache()
        P.symnmf_trim_cache()
        others = {}
        for name, fn in (("sparse", bench_sparse), ("precision", bench_precision), ("warmstart", bench_warmstart)):
            t0 = time.time()
            r = fn(args) if name != "warmstart" else fn(args, log_each=False)
            r = {kk: v for kk, v in r.items() if kk not in ("n_gpus", "scaling", "vs_baseline", "data", "steps",
                                                          "warmup")}
            r["bench_seconds"] = round(time.time() - t0, 1)
            others[name] = r
            log(f"[bench] workload {name} done in {r['bench_seconds']} s")
            torch.cuda.empty_cache()
            P.symnmf_trim_cache()
        out["config"]["workloads"] = others
    print(json.dumps(out), flush=True)


def nnz_gb_bf16(nnz, k):
    """Bytes of BF16 factor rows gathered by one CSR product."""
    return nnz * k * 2.0


def bench_sparse(args):
    """Sparse graph workload: X = D^-1/2 A D^-1/2 of a stochastic block model
    (64 equal blocks, average degree 32, p_in / p_out = 20) in CSR int32 /
    FP32, k = 64 -- the synthetic stand-in for the paper's normalised
    citation graph.  Its community structure is weak (three quarters of the
    edges cross blocks), so a rank-64 fit leaves most of ||X|| unexplained
    and the plain method stalls within a few iterations near residual 1: a
    time-to-residual figure says little here.  Reported instead: seconds per
    iteration and the residual after a fixed number of iterations for plain
    HALS with the CSR product, for the same with BF16 gathers of the factor
    rows (the precision option of the CSR product) and for leverage-score
    sampled HALS (s rows, tau = 1/s), the per-phase device time, and the live
    roofline of the SpMM.  `value` is seconds per LvS iteration."""
    import numpy as np
    import torch
    import paper_2402_08134_amd as P
    import workloads
    n, k, s_rows = args.sparse_n, args.sparse_k, args.sparse_s
    iters = args.sparse_iters
    t0 = time.time()
    Xs, _ = workloads.sbm(n, 64, 32.0, 20.0, seed=0)
    log(f"[bench] generated SBM n={n} nnz={Xs.nnz} in {time.time() - t0:.1f}s")
    Xd = (torch.from_numpy(Xs.indptr.astype(np.int32)).cuda(), torch.from_numpy(Xs.indices.astype(np.int32)).cuda(),
          torch.from_numpy(Xs.data.astype(np.float32)).cuda(), n)
    torch.cuda.synchronize()

    def run(method, seed, timing, count):
        o = P.symnmf_default_options(timing=timing, resid_every=iters)
        if method == "plain_bf16":
            o.compute_dtype = P.BF16
        c = P.symnmf_create(Xd, k, 0.0, s_rows if method == "lvs" else 0, seed, o)
        P.symnmf_iterate(c, count)
        return c

    methods = ["plain", "plain_bf16", "lvs"]
    for m in methods:
        run(m, 100, 0, 2)
    torch.cuda.synchronize()
    res = {}
    for m in methods:
        c = run(m, 1, 0, 1)          # create and one iteration outside the timed region
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.symnmf_iterate(c, iters)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / iters
        r = P.symnmf_residual(c, P.RESID_EXACT)
        st = P.symnmf_get_stats(c)
        res[m] = {"s_per_iteration": t, "iterations": iters + 1, "residual": r[0], "residual_HHt": r[1]}
        if m == "lvs":
            res[m].update({"s": s_rows, "deterministic_rows": int(st.s_D), "sampled_rows": int(st.sample_rows),
                           "theta_over_k": st.theta_over_k})
        del c
        log(f"[bench] {m:10s} {t * 1e3:8.3f} ms/iteration  residual after {iters + 1} iterations {r[0]:.6f}")
    rb, rf = res["plain_bf16"]["residual"], res["plain"]["residual"]
    res["plain_bf16"]["residual_rel_diff_vs_fp32"] = abs(rb - rf) / rf
    phases = {}
    for m in methods:
        c = run(m, 1, 1, iters)
        phases[m] = {kk: v[0] / iters for kk, v in phase_totals(P, [c]).items()}
        if m == "plain":
            ph = phase_totals(P, [c])
            ms, calls = ph["product"]
        if m == "plain_bf16":
            msb, callsb = phase_totals(P, [c])["product"]
        del c
    t_bf = msb / 1e3 / callsb
    res["plain_bf16"]["spmm_us_per_launch"] = t_bf * 1e6
    log(f"[bench] SpMM with BF16 gathers {t_bf * 1e6:.1f} us per launch "
        f"({nnz_gb_bf16(Xs.nnz, k) / t_bf / 1e9:.0f} GB/s of BF16 row gathers); residual after {iters + 1} "
        f"iterations differs from FP32 by {res['plain_bf16']['residual_rel_diff_vs_fp32']:.1e} (relative)")
    t_prod = ms / 1e3 / calls
    nnz = Xs.nnz
    alg_bytes = nnz * 8.0 + 4.0 * (n + 1) + 2.0 * n * k * 4
    achieved = alg_bytes / t_prod / 1e9
    gather = nnz * k * 4.0
    log(f"[bench] SpMM {t_prod * 1e6:.1f} us over {calls} launches -> {achieved:.0f} GB/s algorithmic, "
        f"{gather / t_prod / 1e9:.0f} GB/s of row gathers")
    t_val = res["lvs"]["s_per_iteration"]
    out = {
        "metric": "SymNMF time-to-residual (s) and X*H GB/s or MFMA %, learned-init vs plain",
        "value": t_val, "unit": "s", "n_gpus": 1, "steps": iters, "warmup": 1,
        "ms_per_step": t_val * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sparse SBM graph n={n} nnz={nnz} k={k} CSR int32/FP32 (64 blocks, average "
                               f"degree 32, p_in/p_out = 20); value: seconds per leverage-score sampled HALS "
                               f"iteration, s={s_rows}, tau=1/s",
                   "n": n, "nnz": int(nnz), "k": k, "lvs_vs_plain_per_iteration":
                       res["plain"]["s_per_iteration"] / t_val, "methods": res},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": stored_traffic("k_csr_spmm_vec_sbm2p20_k64_pmc.txt", "k_sparse.hip", n, k),
                     "kernel": "k_csr_spmm_vec<float, float, float, 16, 4> (X H, one launch per half-iteration)",
                     "us_per_launch": t_prod * 1e6, "launches": calls, "algorithmic_bytes_per_launch": alg_bytes,
                     "row_gather_bytes_per_launch": gather,
                     # the gather-bound ceiling: the nnz 256-byte factor rows at the HBM peak
                     "row_gather_gbs": gather / t_prod / 1e9,
                     "row_gather_frac": gather / t_prod / 1e9 / HBM_PEAK_GBS},
        "phases_ms_per_iteration": phases,
        "cpu_baseline": None,
    }
    return out


WARM_WEIGHTS = "warmstart.bin"


def warm_solve(P, X, k, r_star, method, nets, seed=1):
    """One solve of a learned-start study instance to r* = r_conv + 1e-3,
    create included.  plain: random start, iterations on X.  lai: random
    start, LAI iterations (l = k + 16, q = 2) until their own residual
    stalls, then refinement on X until r*.  learned / untrained: the start
    from the trained / untrained network on the LAI basis, then iterations on
    X; learned_lai / untrained_lai: that start, then LAI iterations and
    refinement as in lai.  Returns (context, iterations, iterations on X)."""
    l, q = k + 16, 2
    lai_stage = method.endswith("lai")
    o = P.symnmf_default_options(stop_mode=P.STOP_STALL if lai_stage else P.STOP_TARGET,
                                 target=r_star, check_every=8 if lai_stage else 4)
    c = P.symnmf_create(X, k, 0.0, 0, seed, o)
    if method == "plain":
        it = P.symnmf_iterate(c, 3000)
        return c, it, it
    P.symnmf_lai(c, l, q)
    if method.startswith("learned"):
        P.symnmf_warmstart(c, nets["learned"], want_beta=False)
    elif method.startswith("untrained"):
        P.symnmf_warmstart(c, nets["untrained"], want_beta=False)
    it = P.symnmf_iterate(c, 2000) if lai_stage else 0
    P.symnmf_refine(c, P.STOP_TARGET, r_star)
    it2 = P.symnmf_iterate(c, 3000)
    return c, it + it2, it2


def bench_warmstart(args, log_each=True):
    """The learned start on the held-out instances of the learned-start study
    (workloads.warm_instance, ids 1800..1999: SBM graphs and Gaussian-kernel
    similarities, n in [4096, 32768], k in {16, 32, 64}).  Per instance: the
    plain method from the random start until the stall rule gives r_conv;
    then each method is timed once to r* = r_conv + 1e-3 (wall clock around
    the whole solve, create included, device synchronised on both sides).
    Reports the per-instance time ratios of learned vs plain (the network's
    start, then the same iterations on X), learned_lai vs lai (so that the
    LAI's own gain is not credited to the network), learned_lai vs plain,
    and the untrained network's starts as the ablation; medians, fractions
    of wins and histograms of the iteration counts."""
    import numpy as np
    import torch
    import paper_2402_08134_amd as P
    from paper_2402_08134_amd import warmstart as WSP
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    P.lib()
    wpath = args.warm_weights or os.path.join(WSP.WEIGHTS_DIR, WARM_WEIGHTS)
    nets = {"learned": WSP.load(wpath), "untrained": P.symnmf_mlp_create(P.MLP_HIDDEN, 7)}
    methods = ["plain", "lai", "learned", "learned_lai", "untrained", "untrained_lai"]
    ids = list(workloads.WARM_HELD_OUT_IDS)[args.warm_first:args.warm_first + args.warm_count]

    def device_X(spec):
        X = workloads.warm_instance_data(spec)
        if spec["kind"] == "sbm":
            return (torch.from_numpy(X.indptr.astype(np.int32)).cuda(),
                    torch.from_numpy(X.indices.astype(np.int32)).cuda(), torch.from_numpy(X.data).cuda(), spec["n"])
        return X

    # warm-up on a small instance: library load, kernels, graph instantiation
    wspec = dict(workloads.warm_instance(ids[0]), n=4096)
    for kind in ("sbm", "gmm"):
        Xw = device_X(dict(wspec, kind=kind))
        for m in methods:
            c, _, _ = warm_solve(P, Xw, wspec["k"], 2.0, m, nets)
            del c
        del Xw
    torch.cuda.synchronize()

    recs = []
    t_all = time.time()
    for i in ids:
        spec = workloads.warm_instance(i)
        n, k = spec["n"], spec["k"]
        X = device_X(spec)
        torch.cuda.synchronize()
        o = P.symnmf_default_options(stop_mode=P.STOP_STALL, check_every=8)
        ref = P.symnmf_create(X, k, 0.0, 0, 1, o)
        it_conv = P.symnmf_iterate(ref, 3000)
        r_conv = P.symnmf_residual(ref, P.RESID_EXACT)[0]
        del ref
        r_star = r_conv + 1e-3
        rec = {"id": i, "kind": spec["kind"], "n": n, "k": k, "r_conv": r_conv, "plain_conv_iterations": it_conv}
        for m in methods:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c, it, itx = warm_solve(P, X, k, r_star, m, nets)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            r = P.symnmf_residual(c, P.RESID_EXACT)[0]
            del c
            rec[m] = {"s": t, "iterations": it, "iterations_on_X": itx, "residual": r, "reached": bool(r <= r_star)}
        recs.append(rec)
        del X
        if log_each:
            log(f"[warm] {i} {spec['kind']} n={n} k={k} r*={r_star:.5f}: " +
                " ".join(f"{m} {rec[m]['s'] * 1e3:.1f}ms/{rec[m]['iterations']}" for m in methods) +
                f"  [{time.time() - t_all:.0f}s]")

    def pair(a, b, sel=None):
        rs = [r for r in recs if sel is None or sel(r)]
        if not rs:
            return None
        ratio = np.array([r[a]["s"] / r[b]["s"] if r[a]["reached"] else np.inf for r in rs])
        iratio = np.array([r[a]["iterations"] / max(r[b]["iterations"], 1) for r in rs])
        return {"instances": len(rs), "median_time_ratio": float(np.median(ratio)),
                "geomean_time_ratio": float(np.exp(np.mean(np.log(ratio)))) if np.all(np.isfinite(ratio)) else None,
                "fraction_faster": float(np.mean(ratio < 1.0)),
                "median_iteration_ratio": float(np.median(iratio)),
                "not_reached": int(sum(1 for r in rs if not r[a]["reached"]))}

    kinds = {"all": None, "sbm": lambda r: r["kind"] == "sbm", "gmm": lambda r: r["kind"] == "gmm"}
    for kk in (16, 32, 64):
        kinds[f"k{kk}"] = (lambda kk_: (lambda r: r["k"] == kk_))(kk)
    pairs = {"learned_vs_plain": ("learned", "plain"), "learned_lai_vs_lai": ("learned_lai", "lai"),
             "learned_lai_vs_plain": ("learned_lai", "plain"), "lai_vs_plain": ("lai", "plain"),
             "untrained_vs_plain": ("untrained", "plain"), "untrained_lai_vs_lai": ("untrained_lai", "lai")}
    summary = {name: {g: pair(a, b, sel) for g, sel in kinds.items()} for name, (a, b) in pairs.items()}
    edges = [0, 5, 10, 20, 40, 80, 160, 320, 640, 1280, 100000]
    hist = {m: np.histogram([r[m]["iterations"] for r in recs], bins=edges)[0].tolist() for m in methods}
    if args.warm_out:
        with open(args.warm_out, "w") as f:
            json.dump(recs, f)
    med = summary["learned_vs_plain"]["all"]["median_time_ratio"]
    return {
        "metric": "learned-start vs random-start time to r* = r_conv + 1e-3 (median per-instance time ratio, "
                  "learned / plain)",
        "value": med,
        "unit": "ratio",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(recs)} held-out generated instances (ids {ids[0]}..{ids[-1]}; SBM graphs and "
                               f"Gaussian-kernel similarities, n in [4096, 32768], k in {{16, 32, 64}}), "
                               f"HALS, l = k + 16, q = 2",
                   "weights": os.path.basename(wpath), "pairs": summary,
                   "iteration_histogram": {"bin_edges": edges, **hist},
                   "median_s": {m: float(np.median([r[m]["s"] for r in recs])) for m in methods},
                   "eval_seconds": round(time.time() - t_all, 1)},
    }


def bench_precision(args):
    """Precision sweep at n = 65536, k = 64 (64-component mixture in R^128):
    the products X H and X Omega in FP32 and in BF16 (X converted once, FP32
    accumulation on MFMA), everything else in FP32 / FP64.  Time to
    r* = r_conv + 1e-3 (r_conv: where plain FP32 stops under the stall rule)
    for plain, LAI (l = k + 16, q = 2) and the learned start, in both
    precisions; the live roofline of the BF16 X H product.  The oracle leg
    runs two FP64 iterations on the host on the same X bits and start, and
    the GPU's relative residual error after those two iterations is reported
    for both precisions.  `value` is the fastest BF16 method's time."""
    import numpy as np
    import torch
    import paper_2402_08134_amd as P
    from paper_2402_08134_amd import warmstart as WSP
    import workloads
    n, k = args.precision_n, 64
    l, q = k + 16, 2
    t0 = time.time()
    X = workloads.gpu_gaussian_kernel(n, 128, 64, seed=0)
    log(f"[bench] generated X n={n} on the GPU in {time.time() - t0:.1f}s")
    net = WSP.load(os.path.join(WSP.WEIGHTS_DIR, "warmstart.bin"))
    o = P.symnmf_default_options(stop_mode=P.STOP_STALL, check_every=8)
    ref = P.symnmf_create(X, k, 0.0, 0, 1, o)
    iters_conv = P.symnmf_iterate(ref, 2000)
    r_conv = P.symnmf_residual(ref, P.RESID_EXACT)[0]
    r_star = r_conv + 1e-3
    del ref
    log(f"[bench] plain FP32 converged: {iters_conv} iterations, residual {r_conv:.6f}; r* = {r_star:.6f}")

    def solve(method, prec, seed, timing):
        lai_stage = method != "plain"
        o = P.symnmf_default_options(stop_mode=P.STOP_STALL if lai_stage else P.STOP_TARGET, target=r_star,
                                     check_every=8 if lai_stage else 4, timing=timing)
        if prec == "bf16":
            o.compute_dtype = P.BF16
        c = P.symnmf_create(X, k, 0.0, 0, seed, o)
        if method == "plain":
            it = P.symnmf_iterate(c, 600)
            return c, it, it
        P.symnmf_lai(c, l, q)
        if method == "learned_lai":
            P.symnmf_warmstart(c, net, want_beta=False)
        it = P.symnmf_iterate(c, 2000)
        P.symnmf_refine(c, P.STOP_TARGET, r_star)
        it2 = P.symnmf_iterate(c, 600)
        return c, it + it2, it2

    res = {}
    for prec in ("f32", "bf16"):
        for m in ("plain", "lai", "learned_lai"):
            solve(m, prec, 100, 0)          # warm-up (graphs, caches)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c, it, itx = solve(m, prec, 1, 0)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            r = P.symnmf_residual(c, P.RESID_EXACT)[0]
            del c
            res[f"{m}_{prec}"] = {"s_per_solve": t, "iterations": it, "iterations_on_X": itx, "final_residual": r,
                                  "reached_r_star": bool(r <= r_star + 1e-12)}
            log(f"[bench] {m:12s} {prec:5s} {t * 1e3:9.2f} ms/solve  iterations {it} (on X {itx})  residual {r:.6f}")
    # live roofline of the BF16 product (dominant kernel of the BF16 solves),
    # and the FP32 products' rate against the FP32 matrix-core peak (X H at
    # k = 64 is bound by the matrix cores in FP32: 2 n^2 k flop on 4 n^2
    # bytes)
    products = {}
    for prec in ("bf16", "f32"):
        c, it, _ = solve("plain", prec, 1, 1)
        ph = phase_totals(P, [c])
        r = P.symnmf_residual(c, P.RESID_EXACT)[0]
        del c
        ms_, calls_ = ph["product"]
        t_ = ms_ / 1e3 / calls_
        xb = 2 if prec == "bf16" else 4
        alg_ = float(n) * n * xb + 2.0 * n * k * 4
        products[prec] = {"us_per_launch": t_ * 1e6, "launches": calls_, "algorithmic_bytes_per_launch": alg_,
                          "hbm_gbs": alg_ / t_ / 1e9, "hbm_frac": alg_ / t_ / 1e9 / HBM_PEAK_GBS,
                          "tflops": 2.0 * n * n * k / t_ / 1e12,
                          "mfma_frac": 2.0 * n * n * k / t_ / 1e12 /
                                       (BF16_MFMA_PEAK_TFLOPS if prec == "bf16" else FP32_MFMA_PEAK_TFLOPS),
                          "plain_iterations": it, "plain_final_residual": r}
        log(f"[bench] {prec:5s} X*H {t_ * 1e6:8.1f} us over {calls_} launches -> {alg_ / t_ / 1e9:.0f} GB/s "
            f"algorithmic, {2.0 * n * n * k / t_ / 1e12:.1f} TFLOP/s")
    res["products"] = products
    t_prod = products["bf16"]["us_per_launch"] / 1e6
    calls = products["bf16"]["launches"]
    alg_bytes = products["bf16"]["algorithmic_bytes_per_launch"]
    achieved = alg_bytes / t_prod / 1e9
    best = min((v["s_per_solve"], kk) for kk, v in res.items()
               if kk.endswith("bf16") and kk != "products" and v["reached_r_star"])
    cpu = None if args.no_cpu_baseline else precision_oracle_leg(X, k, res, args.precision_oracle_iters)
    out = {
        "metric": "SymNMF time-to-residual (s) and X*H GB/s or MFMA %, learned-init vs plain",
        "value": best[0], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": best[0] * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"dense Gaussian-kernel similarity n={n} k={k} (64-component GMM in R^128), "
                               f"products in BF16 with FP32 accumulation vs FP32; value: {best[1]}",
                   "n": n, "k": k, "l": l, "q": q, "r_conv_fp32": r_conv, "r_star": r_star, "methods": res},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_gemm_cols_bf16<NT, VEC> (X H in BF16, one launch per half-iteration)",
                     "us_per_launch": t_prod * 1e6, "launches": calls, "algorithmic_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
    }
    del X
    return out


def precision_oracle_leg(X, k, res, iters=2):
    """The FP64 oracle on the host: `iters` plain HALS iterations (2 by
    default; --precision-oracle-iters for a run as long as the converged
    GPU run) on the same X bits and start as the GPU's FP32 and BF16 runs of
    as many iterations; timed (the baseline) and compared (relative residual
    error of each precision)."""
    import numpy as np
    import torch
    import paper_2402_08134_amd as P
    from oracle import symnmf as O
    n = X.shape[0]
    Xh = X.cpu().numpy()
    out = {}
    for prec in ("f32", "bf16"):
        o = P.symnmf_default_options()
        if prec == "bf16":
            o.compute_dtype = P.BF16
        c = P.symnmf_create(X, k, 0.0, 0, 1, o)
        P.symnmf_iterate(c, iters)
        out[prec] = P.symnmf_residual(c, P.RESID_EXACT)[0]
        del c
    log(f"[bench] oracle: scalars + {iters} FP64 iterations on the host ...")
    t0 = time.perf_counter()
    sc = O.data_scalars(Xh)
    H0 = O.initial_factor(n, k, sc["zeta"], 1).astype(np.float32).astype(np.float64)
    done = [0]

    def progress(r):
        done[0] += 1
        if iters > 2:
            log(f"[bench] oracle iteration {done[0]}/{iters}: residual {r:.6f} [{time.perf_counter() - t0:.0f}s]")
        return False

    Wo, Ho, hist = O.plain_symnmf(Xh, k, sc["maxval"], H0, iters, stop=progress)
    t = time.perf_counter() - t0
    ro = O.residual_direct(Xh, Wo, Ho) / np.sqrt(sc["normsq"])
    errs = {p: abs(v - ro) / ro for p, v in out.items()}
    log(f"[bench] oracle residual after {iters} iterations {ro:.6f}; GPU relative error FP32 {errs['f32']:.2e} "
        f"BF16 {errs['bf16']:.2e}; oracle time {t:.1f}s")
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return {"value": t, "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": f"scalars pass + {iters} plain FP64 HALS iterations at full size on the same X bits and start",
            "iterations": iters, "residual_oracle": ro,
            "residual_gpu": out, "gpu_relative_error": errs}


def phase_totals(P, ctxs):
    """Summed (ms, launches) per phase over the contexts of a timed loop."""
    names = {P.PHASE_PRODUCT: "product", P.PHASE_UPDATE: "update", P.PHASE_SAMPLE: "sample", P.PHASE_LAI: "lai",
             P.PHASE_WARM: "warm", P.PHASE_REDUCE: "reduce"}
    tot = {v: [0.0, 0] for v in names.values()}
    for c in ctxs:
        st = P.symnmf_get_stats(c)
        for ph, name in names.items():
            tot[name][0] += st.phase_ms[ph]
            tot[name][1] += st.phase_calls[ph]
    return tot


def stored_traffic(summary, source, n, k):
    """HBM bytes per launch of a kernel from a committed rocprofv3 counter
    summary (profiles/<summary>), or None when that summary is missing, was
    taken at another size, or the kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    src = os.path.join(ROOT, "paper_2402_08134_amd", "csrc", source)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            key, _, val = line.partition(":")
            kv[key.strip()] = val.strip()
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get(f"{source} sha256") != digest or kv.get("n") != str(n) or kv.get("k") != str(k):
        return None
    try:
        return float(kv["hbm bytes per launch (scaled)"])
    except (KeyError, ValueError):
        return None


def pmc_probe(args):
    """Short fixed workload for the rocprofv3 counter passes: a 1 GiB device
    copy (the calibration kernel of known traffic), then ten plain
    iterations at the bench size, then the learned start and ten LAI
    iterations."""
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
    from paper_2402_08134_amd import warmstart as WSP
    net = WSP.load(os.path.join(WSP.WEIGHTS_DIR, WARM_WEIGHTS))
    c = P.symnmf_create(X, args.k, 0.0, 0, 1)
    P.symnmf_lai(c, args.k + 16, 2)
    P.symnmf_warmstart(c, net, want_beta=False)
    P.symnmf_iterate(c, 10)
    torch.cuda.synchronize()
    log("[pmc-probe] learned start and 10 LAI iterations done")


def pmc_probe_sparse(args):
    """Counter-collection workload for the CSR product: the SBM of the sparse
    bench, three 1 GiB device copies (the calibration kernel of known
    traffic), then three plain HALS iterations with the FP32 product and three
    with BF16 gathers of the factor rows."""
    import numpy as np
    import torch
    import paper_2402_08134_amd as P
    import workloads
    n, k = args.sparse_n, args.sparse_k
    Xs, _ = workloads.sbm(n, 64, 32.0, 20.0, seed=0)
    Xd = (torch.from_numpy(Xs.indptr.astype(np.int32)).cuda(), torch.from_numpy(Xs.indices.astype(np.int32)).cuda(),
          torch.from_numpy(Xs.data.astype(np.float32)).cuda(), n)
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("[pmc-probe] copies done (3 x 1 GiB read + 1 GiB write)")
    for bf in (False, True):
        o = P.symnmf_default_options(resid_every=100)
        if bf:
            o.compute_dtype = P.BF16
        c = P.symnmf_create(Xd, k, 0.0, 0, 1, o)
        P.symnmf_iterate(c, 3)
        torch.cuda.synchronize()
        log(f"[pmc-probe] 3 plain iterations done ({'BF16' if bf else 'FP32'} gathers)")
        del c


def cpu_baseline(Xh, k, l, q, net_params, r_star, seed=1):
    """The FP64 oracle (as it stands) on the host cores, timed on the method
    `value` times, learned_lai, on the same X: scalars pass, Algorithms RRF +
    Apx-EVD (Householder QR, eigh) from the same sketch bits, the learned
    start (features, the same network parameters, scale fit), LAI iterations
    until the stall rule, then iterations on X until r*."""
    import numpy as np
    from oracle import symnmf as O
    from oracle import warmstart as WS
    n = Xh.shape[0]
    t0 = time.perf_counter()
    sc = O.data_scalars(Xh)
    X64 = np.asarray(Xh, dtype=np.float64)
    U, lam = O.apx_evd(lambda M: X64 @ M, O.sketch_omega(n, l, seed), q)
    H0 = WS.warm_start(net_params, U, lam, sc["rowsum"], k, lambda B: X64 @ B)
    if H0 is None:
        H0 = O.initial_factor(n, k, sc["zeta"], seed)
    W, H, h1 = O.lai_symnmf(U, lam, k, sc["maxval"], H0, 2000, stop=O.StallRule(1e-4, 4))
    W, H, h2 = O.anls(lambda B: X64 @ B, sc["normsq"], H, sc["maxval"], 4000, W0=W, target=r_star)
    t = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    return {"value": t, "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": f"one whole learned_lai solve on the same X (n={n}, k={k}, l={l}, q={q}): "
                      f"{len(h1)} LAI iterations + {len(h2)} on X, final residual {h2[-1]:.6f}"}


def net_params_host(P, net):
    """The network's parameters as the oracle's list of (W, b) layers."""
    import numpy as np
    import torch
    from oracle import warmstart as WS
    p = torch.empty(P.symnmf_mlp_num_params(net), dtype=torch.float32, device="cuda")
    P.symnmf_mlp_get_params(net, p)
    v = p.cpu().double().numpy()
    out, o = [], 0
    sizes = WS.layer_sizes()
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append((v[o:o + a * b].reshape(a, b), v[o + a * b:o + a * b + b]))
        o += a * b + b
    return out


if __name__ == "__main__":
    main()
