"""GPU parity of the CSR path and of leverage-score sampling (Algorithm
LvS-SymNMF with hybrid sampling) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import symnmf as O
import workloads

from gpu_common import P, torch, require_gpu, dev, host, rel, factor, round_to, csr_dev, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _sbm(n=6000, blocks=12, deg=24.0, seed=0):
    X, lab = workloads.sbm(n, blocks, deg, 20.0, seed=seed)
    return X


def _X64(X):
    return sp.csr_matrix((X.data.astype(np.float64), X.indices, X.indptr), shape=X.shape)


@pytest.mark.parametrize("c", [1, 10, 16, 33, 64, 80])
def test_spmm_parity(c):
    X = _sbm(5003, 7, 20.0, seed=c)
    ctx = P.symnmf_create(csr_dev(X), min(c, 64), 0.0, 0, 0)
    B = workloads.random_factor(X.shape[0], c, seed=c)
    Bd = dev(B, torch.float32)
    Yd = torch.empty_like(Bd)
    P.symnmf_apply_x(ctx, Bd, Yd)
    ref = _X64(X) @ round_to(B, torch.float32)
    assert rel(host(Yd), ref) <= 1e-6


def test_csr_plain_parity_and_exact_residual():
    X = _sbm()
    n, k = X.shape[0], 12
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, 0, 3)
    iters = 25
    P.symnmf_iterate(ctx, iters)
    X64 = _X64(X)
    sc = O.data_scalars(X64)
    H0 = round_to(O.initial_factor(n, k, sc["zeta"], 3), torch.float32)
    Wo, Ho, hist = O.plain_symnmf(X64, k, sc["maxval"], H0, iters)
    hg = np.array(P.symnmf_history(ctx))
    log(f"csr plain: history max rel {np.max(np.abs(hg - hist) / hist):.2e}")
    assert np.max(np.abs(hg - hist) / hist) <= 1e-4
    r = P.symnmf_residual(ctx, P.RESID_EXACT)
    ro = O.residual_direct(X64, Wo, Ho) / np.sqrt(sc["normsq"])
    assert abs(r[0] - ro) / ro <= 1e-4


@pytest.mark.parametrize("k", [16, 32, 33, 64])
def test_leverage_parity(k):
    # k = 16, 32, 64: rows read as float4 pieces and transposed across the
    # lanes; k = 33 (padded to 64): rows staged in LDS
    X = _sbm()
    n = X.shape[0]
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, 100, 0)
    H = workloads.random_factor(n, k, seed=5) ** 2
    P.symnmf_set_factor(ctx, P.H, dev(H))
    lev = torch.empty(n, dtype=torch.float64, device="cuda")
    P.symnmf_leverage(ctx, P.H, lev)
    lo = O.leverage_scores(round_to(H, torch.float32))
    lg = host(lev)
    assert rel(lg, lo) <= 1e-10
    assert abs(lg.sum() - k) <= 1e-9 * k


@pytest.mark.parametrize("n,k,s", [(20000, 16, 3000), (40003, 64, 4000)])
def test_lvs_bitwise_reproducible(n, k, s):
    # the sampled slab's entries land in their segments by atomics and are
    # then put in column order: two runs give the same bits (k = 64 and
    # n >= 32768: the blocked sampled update)
    X = _sbm(n, 16, 24.0, seed=9)
    out = []
    for _ in range(2):
        ctx = P.symnmf_create(csr_dev(X), k, 0.0, s, 5)
        P.symnmf_iterate(ctx, 3)
        out.append((factor(ctx, P.H), factor(ctx, P.W)))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("tau", [-1.0, 0.3e-3, 0.0])
def test_sampler_bitwise(tau):
    n, k, s = 20000, 16, 2000
    X = _sbm(n, 10, 8.0, seed=2)
    o = P.symnmf_default_options(tau=tau)
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, s, 77, o)
    lev = workloads.skewed_scores(n, k, seed=3, heavy=40)
    cap = n
    rows = torch.empty(cap, dtype=torch.int32, device="cuda")
    w = torch.empty(cap, dtype=torch.float64, device="cuda")
    for h in (0, 1, 5):
        cnt = P.symnmf_sample(ctx, dev(lev), h, rows, w)
        tau_eff = 1.0 / s if tau < 0 else tau
        ro, wo, info = O.hybrid_sample(lev, k, s, tau_eff, 77, h)
        rg = rows[:cnt].cpu().numpy()
        wg = w[:cnt].cpu().numpy()
        log(f"sampler tau={tau} h={h}: rows {cnt} (det {info['s_D']})")
        assert cnt == ro.shape[0]
        assert np.array_equal(rg, ro)
        assert np.array_equal(wg, wo)
        st = P.symnmf_get_stats(ctx)
        assert st.s_D == info["s_D"]


def test_lvs_half_step_identical_inputs():
    X = _sbm(8000, 16, 30.0, seed=4)
    n, k, s = X.shape[0], 16, 800
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, s, 9)
    alpha = P.symnmf_get_stats(ctx).alpha
    H = workloads.random_factor(n, k, seed=6, scale=0.2)
    W = workloads.random_factor(n, k, seed=7, scale=0.2)
    P.symnmf_set_factor(ctx, P.H, dev(H))
    P.symnmf_set_factor(ctx, P.W, dev(W))
    H32, W32 = round_to(H, torch.float32), round_to(W, torch.float32)
    P.symnmf_half_step(ctx, 0, 4)
    Wo, info = O.lvs_half_step(_X64(X), H32, W32, alpha, s, 1.0 / s, 9, 4)
    log(f"lvs half step: rows {len(info['rows'])} det {info['s_D']}")
    assert rel(factor(ctx, P.W), Wo) <= 1e-5


def test_lvs_run_parity():
    X = _sbm(8000, 16, 30.0, seed=5)
    n, k, s = X.shape[0], 16, 1000
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, s, 21)
    iters = 8
    P.symnmf_iterate(ctx, iters)
    X64 = _X64(X)
    sc = O.data_scalars(X64)
    H0 = round_to(O.initial_factor(n, k, sc["zeta"], 21), torch.float32)
    Wo, Ho, hist = O.lvs_symnmf(X64, k, sc["maxval"], H0, iters, s, 1.0 / s, 21)
    hg = np.array(P.symnmf_history(ctx))
    log(f"lvs run: gpu {hg[-1]:.6f} oracle {hist[-1]:.6f}")
    assert np.max(np.abs(hg - hist) / hist) <= 1e-4
    r = P.symnmf_residual(ctx, P.RESID_EXACT)
    ro = O.residual_direct(X64, Wo, Ho) / np.sqrt(sc["normsq"])
    assert abs(r[0] - ro) / ro <= 1e-4


def test_lvs_tau_zero_matches_plain():
    X = _sbm(3000, 6, 20.0, seed=6)
    k = 8
    o = P.symnmf_default_options(tau=0.0)
    a = P.symnmf_create(csr_dev(X), k, 0.0, 50, 2, o)
    b = P.symnmf_create(csr_dev(X), k, 0.0, 0, 2)
    P.symnmf_iterate(a, 5)
    P.symnmf_iterate(b, 5)
    assert rel(factor(a, P.H), factor(b, P.H)) <= 1e-5


@pytest.mark.parametrize("case", [(66_001, 64, 0, np.float32), (66_001, 64, 6000, np.float32),
                                  (66_001, 64, 500, np.float32),
                                  (66_001, 52, 0, np.float32), (66_001, 60, 5000, np.float32),
                                  (40_003, 50, 0, np.float32),
                                  (65_600, 10, 0, np.float32), (65_600, 40, 3000, np.float32),
                                  (65_551, 33, 0, np.float64), (65_551, 64, 4000, np.float64),
                                  (40_003, 32, 0, np.float32), (40_003, 20, 3000, np.float32)])
def test_long_factor_half_step(case):
    # long factors: every one of the update's blocks walks several row chunks
    # (grid stride), and n is ragged against the chunk; every padded width:
    # at 64 with FP32 factors the blocked sweep (k = 64, and k = 52, 60 with
    # padding columns), k = 50 (not a multiple of 4) the 8-lanes-per-row
    # kernel, as at width 32 and for FP64.  Sampled: about 3 entries per row
    # at s = 6000 (most rows' later entries beyond the chunk's held ones) and
    # 0.25 at s = 500 (nearly all of them held)
    n, k, s, vt = case
    log(f"long factor half step n={n} k={k} s={s} {np.dtype(vt).name}")
    X = _sbm(n, 32, 16.0, seed=n + k)
    X = sp.csr_matrix((X.data.astype(vt), X.indices, X.indptr), shape=X.shape)
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, s, 3)
    alpha = P.symnmf_get_stats(ctx).alpha
    H = workloads.random_factor(n, k, seed=8, scale=0.2)
    W = workloads.random_factor(n, k, seed=9, scale=0.2)
    td = torch.float64 if vt == np.float64 else torch.float32
    P.symnmf_set_factor(ctx, P.H, dev(H))
    P.symnmf_set_factor(ctx, P.W, dev(W))
    Hr, Wr = round_to(H, td), round_to(W, td)
    P.symnmf_half_step(ctx, 0, 2)
    X64 = _X64(X)
    if s:
        Wo, _ = O.lvs_half_step(X64, Hr, Wr, alpha, s, 1.0 / s, 3, 2)
    else:
        Wo = O.hals_gy(Hr.T @ Hr + alpha * np.eye(k), X64 @ Hr + alpha * Hr, Wr)
    e = rel(factor(ctx, P.W), Wo)
    log(f"   W rel {e:.2e}")
    assert e <= (1e-12 if vt == np.float64 else 1e-5)


def test_lvs_hub_rows_half_step():
    # two hub rows adjacent to a third of the graph: with a large sample their
    # slab segments hold hundreds of entries (the segment order's one-lane
    # sort past 64 entries, the chunk's held extras summed over hundreds of
    # rows, and the per-block fallback past the chunk's held rows)
    n, k, s = 40003, 64, 12000
    X = _sbm(n, 16, 24.0, seed=21).tolil()
    rng = np.random.default_rng(5)
    for hub in (7, 20011):
        nb = rng.choice(n, n // 3, replace=False)
        nb = nb[nb != hub]
        X[hub, nb] = 0.5
        X[nb, hub] = 0.5
    X = sp.csr_matrix(X, dtype=np.float32)
    X.sort_indices()
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, s, 3)
    alpha = P.symnmf_get_stats(ctx).alpha
    H = workloads.random_factor(n, k, seed=8, scale=0.2)
    W = workloads.random_factor(n, k, seed=9, scale=0.2)
    P.symnmf_set_factor(ctx, P.H, dev(H))
    P.symnmf_set_factor(ctx, P.W, dev(W))
    Hr, Wr = round_to(H, torch.float32), round_to(W, torch.float32)
    P.symnmf_half_step(ctx, 0, 2)
    Wg = factor(ctx, P.W)
    Wo, _ = O.lvs_half_step(_X64(X), Hr, Wr, alpha, s, 1.0 / s, 3, 2)
    e = rel(Wg, Wo)
    log(f"lvs hub rows n={n} k={k} s={s}: W rel {e:.2e}")
    assert e <= 1e-5
    P.symnmf_set_factor(ctx, P.W, dev(W))
    P.symnmf_half_step(ctx, 0, 2)
    assert np.array_equal(factor(ctx, P.W), Wg)   # the same bits again


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_long_factor_plain_run(compute):
    # k = 64 on a long factor (n >= 32768): the HALS sweep runs blocked (16
    # columns at a time, the other columns' terms on the FP64 matrix cores)
    # in whole iterations.  The residual history comes from the trace
    # identity with the update's dot product; with BF16 gathers every
    # product reads the row copy the update writes.
    X = _sbm(66001, 32, 16.0, seed=5)
    n, k, iters = X.shape[0], 64, 3
    log(f"long factor plain run n={n} k={k} {compute}")
    o = _bf16_opts() if compute == "bf16" else P.symnmf_default_options()
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, 0, 3, o)
    P.symnmf_iterate(ctx, iters)
    X64 = _X64(X)
    sc = O.data_scalars(X64)
    H0 = round_to(O.initial_factor(n, k, sc["zeta"], 3), torch.float32)
    Wo, Ho, hist = O.plain_symnmf(X64, k, sc["maxval"], H0, iters)
    hg = np.array(P.symnmf_history(ctx))
    tol = 1e-4 if compute == "f32" else 1e-3
    eh = np.max(np.abs(hg - hist) / hist)
    r = P.symnmf_residual(ctx, P.RESID_EXACT)[0]
    ro = O.residual_trace(sc["normsq"], Wo, Ho, X64 @ Wo) / np.sqrt(sc["normsq"])
    log(f"   history max rel {eh:.2e}; exact residual gpu {r:.8f} oracle {ro:.8f}")
    assert eh <= tol
    assert abs(r - ro) / ro <= tol
    if compute == "f32":
        e = rel(factor(ctx, P.H), Ho)
        log(f"   H rel {e:.2e}")
        assert e <= 1e-4


def _bf16_opts(**kw):
    o = P.symnmf_default_options(**kw)
    o.compute_dtype = P.BF16
    return o


@pytest.mark.parametrize("n,k", [(6007, 16), (6007, 33), (6007, 64), (66001, 64)])
def test_bf16_gather_half_steps(n, k):
    # the product gathers a BF16 copy of the source rows (FP32 values, FP64
    # sums); both half-steps, so the copy written by the update is used too
    # (at n = 66001, k = 64 by the blocked sweep)
    X = _sbm(n, 12 if n < 10000 else 32, 24.0 if n < 10000 else 16.0, seed=k)
    n = X.shape[0]
    log(f"bf16 gathers n={n} k={k}")
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, 0, 4, _bf16_opts())
    alpha = P.symnmf_get_stats(ctx).alpha
    H = round_to(workloads.random_factor(n, k, seed=10, scale=0.2), torch.float32)
    W = round_to(workloads.random_factor(n, k, seed=11, scale=0.2), torch.float32)
    P.symnmf_set_factor(ctx, P.H, dev(H))
    P.symnmf_set_factor(ctx, P.W, dev(W))
    X64 = _X64(X)
    P.symnmf_half_step(ctx, 0, 0)
    Wo = O.hals_gy(H.T @ H + alpha * np.eye(k), X64 @ round_to(H, torch.bfloat16) + alpha * H, W)
    e = rel(factor(ctx, P.W), Wo)
    log(f"   W rel {e:.2e}")
    assert e <= 1e-5
    P.symnmf_half_step(ctx, 1, 1)
    Wr = round_to(Wo, torch.float32)
    Ho = O.hals_gy(Wr.T @ Wr + alpha * np.eye(k), X64 @ round_to(Wr, torch.bfloat16) + alpha * Wr, H)
    e = rel(factor(ctx, P.H), Ho)
    log(f"   H rel {e:.2e}")
    assert e <= 1e-4


def test_bf16_gather_run_residual_and_graphs():
    # against the FP64 oracle on FP32 data: the relative residual within 1e-3;
    # graph replay bit-identical to eager launches
    X = _sbm(5000, 10, 20.0, seed=12)
    n, k, iters = X.shape[0], 20, 12
    out = []
    for graphs in (0, 1):
        ctx = P.symnmf_create(csr_dev(X), k, 0.0, 0, 8, _bf16_opts(graphs=graphs))
        P.symnmf_iterate(ctx, iters)
        out.append((factor(ctx, P.H), P.symnmf_residual(ctx, P.RESID_EXACT)[0],
                    P.symnmf_get_stats(ctx).graph_launches))
    assert out[0][2] == 0 and out[1][2] > 0
    assert np.array_equal(out[0][0], out[1][0])
    X64 = _X64(X)
    sc = O.data_scalars(X64)
    H0 = round_to(O.initial_factor(n, k, sc["zeta"], 8), torch.float32)
    Wo, Ho, hist = O.plain_symnmf(X64, k, sc["maxval"], H0, iters)
    ro = O.residual_direct(X64, Wo, Ho) / np.sqrt(sc["normsq"])
    log(f"bf16 gathers: residual gpu {out[0][1]:.6f} oracle {ro:.6f}")
    assert abs(out[0][1] - ro) / ro <= 1e-3


def test_bf16_gather_unsupported():
    X = _sbm(2000, 4, 20.0, seed=1)
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_create(csr_dev(X), 4, 0.0, 0, 0, _bf16_opts(rule=P.RULE_PGNCG))
    assert e.value.code == P.E_UNSUPPORTED
    X64 = _X64(X)
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_create(csr_dev(X64), 4, 0.0, 0, 0, _bf16_opts())
    assert e.value.code == P.E_UNSUPPORTED
    o = P.symnmf_default_options()
    o.compute_dtype = P.F64
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_create(csr_dev(X), 4, 0.0, 0, 0, o)
    assert e.value.code == P.E_UNSUPPORTED
