"""GPU parity of the dense path (products, HALS, residuals, plain iteration)
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import symnmf as O
import workloads

from gpu_common import P, torch, require_gpu, dev, host, rel, factor, round_to, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _ctx(X, k, dtype, seed=0, compute=None, **opt):
    o = P.symnmf_default_options(**opt)
    if compute is not None:
        o.compute_dtype = compute
    return P.symnmf_create(dev(X, dtype), k, 0.0, 0, seed, o)


@pytest.mark.parametrize("case", [
    ("f64", 1000, 10), ("f64", 333, 7), ("f32", 1000, 32), ("f32", 769, 48), ("f32", 257, 80), ("bf16", 900, 64),
    ("bf16", 515, 20)])
def test_product_parity(case):
    kind, n, c = case
    log(f"product {case}")
    X, _ = workloads.gaussian_kernel(n, 16, 6, seed=n, dtype=np.float64)
    B = workloads.random_factor(n, c, seed=c)
    if kind == "f64":
        ctx = _ctx(X, min(c, 64), torch.float64)
        Bd = dev(B)
        Yd = torch.empty_like(Bd)
        P.symnmf_apply_x(ctx, Bd, Yd)
        assert rel(host(Yd), X @ B) <= 1e-13
    elif kind == "f32":
        ctx = _ctx(X, min(c, 64), torch.float32)
        Bd = dev(B, torch.float32)
        Yd = torch.empty_like(Bd)
        P.symnmf_apply_x(ctx, Bd, Yd)
        X32, B32 = round_to(X, torch.float32), round_to(B, torch.float32)
        assert rel(host(Yd), X32 @ B32) <= 2e-6
    else:
        ctx = _ctx(X, min(c, 64), torch.float32, compute=P.BF16)
        Bd = dev(B, torch.float32)
        Yd = torch.empty_like(Bd)
        P.symnmf_apply_x(ctx, Bd, Yd)
        Xb = round_to(round_to(X, torch.float32), torch.bfloat16)
        Bb = round_to(B, torch.bfloat16)
        # same rounded operands, FP32 accumulation vs FP64
        assert rel(host(Yd), Xb @ Bb) <= 2e-6
        # and the precision error against the FP32 data stays at BF16 level
        assert rel(host(Yd), X @ B) <= 1e-2


def test_scalars_and_initial_factor():
    X, _ = workloads.planted(1000, 10, noise=0.01, seed=0)
    ctx = _ctx(X, 10, torch.float64, seed=0)
    st = P.symnmf_get_stats(ctx)
    sc = O.data_scalars(X)
    assert st.normsq == pytest.approx(sc["normsq"], rel=1e-13)
    assert st.zeta == pytest.approx(sc["zeta"], rel=1e-13)
    assert st.maxval == sc["maxval"] and st.alpha == sc["maxval"]
    H0 = O.initial_factor(1000, 10, sc["zeta"], seed=0)
    assert rel(factor(ctx, P.H), H0) <= 1e-14
    assert rel(factor(ctx, P.W), H0) <= 1e-14


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_hals_half_step_identical_inputs(dtype):
    n, k = 1111, 13
    X, _ = workloads.gaussian_kernel(n, 8, 5, seed=3, dtype=np.float64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ctx = _ctx(X, k, tdt)
    alpha = float(X.max())
    H = workloads.random_factor(n, k, seed=1, scale=0.3)
    W = workloads.random_factor(n, k, seed=2, scale=0.3)
    P.symnmf_set_factor(ctx, P.H, dev(H))
    P.symnmf_set_factor(ctx, P.W, dev(W))
    if dtype == "f32":
        X, H, W = round_to(X, tdt), round_to(H, tdt), round_to(W, tdt)
    P.symnmf_half_step(ctx, 0)
    Wo = O.hals_symmetric(O.apply_x(X, H), H, W, alpha)
    tol = 1e-12 if dtype == "f64" else 2e-6
    assert rel(factor(ctx, P.W), Wo) <= tol
    assert (factor(ctx, P.W) == 0).any()          # projection exercised
    P.symnmf_half_step(ctx, 1)
    Ho = O.hals_symmetric(O.apply_x(X, Wo), Wo, H, alpha)
    assert rel(factor(ctx, P.H), Ho) <= (1e-12 if dtype == "f64" else 5e-6)


def test_planted_fp64_100_iterations():
    # Planted, FP64, n = 1000, k = 10, alpha = max(X), 100 iterations, seed 0.
    X, _ = workloads.planted(1000, 10, noise=0.01, seed=0)
    ctx = _ctx(X, 10, torch.float64, seed=0)
    assert P.symnmf_iterate(ctx, 100) == 100
    sc = O.data_scalars(X)
    H0 = O.initial_factor(1000, 10, sc["zeta"], seed=0)
    Wo, Ho, hist = O.plain_symnmf(X, 10, sc["maxval"], H0, 100)
    Wg, Hg = factor(ctx, P.W), factor(ctx, P.H)
    log(f"planted: factor rel W {rel(Wg, Wo):.2e} H {rel(Hg, Ho):.2e}")
    assert rel(Wg, Wo) <= 1e-8 and rel(Hg, Ho) <= 1e-8
    hg = np.array(P.symnmf_history(ctx))
    assert hg.shape == hist.shape
    assert np.max(np.abs(hg - hist) / hist) <= 1e-9
    r = P.symnmf_residual(ctx, P.RESID_EXACT)
    ro = O.residual_direct(X, Wo, Ho) / np.linalg.norm(X)
    ro2 = O.residual_direct(X, Ho, Ho) / np.linalg.norm(X)
    assert abs(r[0] - ro) / ro <= 1e-10 and abs(r[1] - ro2) / ro2 <= 1e-9
    rf = P.symnmf_residual(ctx, P.RESID_FAST)
    assert abs(rf[0] - ro) / ro <= 1e-8


def _compute(name):
    return {"f32": None, "bf16": P.BF16}[name]


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_gaussian_kernel_plain_parity(compute):
    # Dense similarity (Gaussian kernel of a mixture), ragged n, FP32 / BF16.
    n, k = 2300, 32
    X, _ = workloads.gaussian_kernel(n, 64, 32, seed=1, dtype=np.float32)
    ctx = _ctx(X, k, torch.float32, seed=5, compute=_compute(compute))
    iters = 30
    P.symnmf_iterate(ctx, iters)
    sc = O.data_scalars(X)
    H0 = round_to(O.initial_factor(n, k, sc["zeta"], seed=5), torch.float32)
    Wo, Ho, hist = O.plain_symnmf(X, k, sc["maxval"], H0, iters)
    ro = O.residual_direct(X, Wo, Ho) / np.sqrt(sc["normsq"])
    r = P.symnmf_residual(ctx, P.RESID_EXACT)
    log(f"gk {compute}: residual gpu {r[0]:.8f} oracle {ro:.8f}")
    tol = 1e-3 if compute == "bf16" else 1e-4
    assert abs(r[0] - ro) / ro <= tol
    hg = np.array(P.symnmf_history(ctx))
    assert np.max(np.abs(hg - hist) / hist) <= 10 * tol


def test_stop_rules():
    X, _ = workloads.planted(600, 6, noise=0.02, seed=4)
    o = P.symnmf_default_options(stop_mode=P.STOP_STALL, check_every=3)
    ctx = P.symnmf_create(dev(X), 6, 0.0, 0, 1, o)
    done = P.symnmf_iterate(ctx, 500)
    hist = np.array(P.symnmf_history(ctx))
    assert len(hist) == done < 500
    # the oracle's stall rule stops at the same iteration on the same history
    rule = O.StallRule(1e-4, 4)
    stops = [rule(r) for r in hist]
    assert stops[-1] and not any(stops[:-1])
    assert P.symnmf_iterate(ctx, 10) == 0          # stays stopped
    r = P.symnmf_residual(ctx, P.RESID_FAST)       # residual still computed after a stop
    assert abs(r[0] - hist[-1]) <= 1e-9
    target = float(hist[20])
    o = P.symnmf_default_options(stop_mode=P.STOP_TARGET, target=target, check_every=5)
    ctx = P.symnmf_create(dev(X), 6, 0.0, 0, 1, o)
    done = P.symnmf_iterate(ctx, 500)
    h2 = np.array(P.symnmf_history(ctx))
    assert done <= 21 and len(h2) == done
    assert h2[-1] <= target and np.all(h2[:-1] > target)
    # stall-or-target: the target when it comes first, else the stall rule
    o = P.symnmf_default_options(stop_mode=P.STOP_STALL_OR_TARGET, target=target, check_every=5)
    ctx = P.symnmf_create(dev(X), 6, 0.0, 0, 1, o)
    assert P.symnmf_iterate(ctx, 500) == done
    o = P.symnmf_default_options(stop_mode=P.STOP_STALL_OR_TARGET, target=0.0, check_every=3)
    ctx = P.symnmf_create(dev(X), 6, 0.0, 0, 1, o)
    assert P.symnmf_iterate(ctx, 500) == len(hist)


def test_determinism_and_edge_sizes():
    X, _ = workloads.gaussian_kernel(300, 8, 4, seed=9, dtype=np.float32)
    outs = []
    for _ in range(2):
        ctx = _ctx(X, 5, torch.float32, seed=3)
        P.symnmf_iterate(ctx, 7)
        outs.append((factor(ctx, P.W), factor(ctx, P.H), P.symnmf_history(ctx)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]
    # k = 1, and n = k (one tile, ragged everywhere)
    for n, k in ((50, 1), (17, 17), (130, 64)):
        Xs, _ = workloads.planted(n, k, noise=0.01, seed=n)
        ctx = _ctx(Xs, k, torch.float64, seed=2)
        P.symnmf_iterate(ctx, 3)
        sc = O.data_scalars(Xs)
        H0 = O.initial_factor(n, k, sc["zeta"], 2)
        Wo, Ho, _ = O.plain_symnmf(Xs, k, sc["maxval"], H0, 3)
        assert rel(factor(ctx, P.H), Ho) <= 1e-11


def test_invalid_arguments():
    X, _ = workloads.planted(100, 4, noise=0.01, seed=1)
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_create(dev(X), 0, 0.0, 0, 0)
    assert e.value.code == P.E_INVALID
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_create(dev(X), 65, 0.0, 0, 0)
    assert e.value.code == P.E_INVALID
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_create(dev(X), 4, 0.0, 10, 0)          # sampling needs CSR
    assert e.value.code == P.E_UNSUPPORTED
    Xn = X.copy()
    Xn[3, 5] = np.nan
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_create(dev(Xn), 4, 0.0, 0, 0)
    assert e.value.code == P.E_INVALID
    ctx = P.symnmf_create(dev(X), 4, 0.0, 0, 0)
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_residual(ctx, P.RESID_LAI)
    assert e.value.code == P.E_STATE
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_lai(ctx, 2, 1)                          # l < k
    assert e.value.code == P.E_INVALID


@pytest.mark.parametrize("case", ["dense_f32", "dense_f64", "lai", "csr", "bpp", "stall"])
def test_graph_replay_matches_eager(case):
    """Iterations replayed from HIP graphs equal directly launched ones, bit
    for bit, over several replays with other work and synchronisation in
    between, and with iteration counts that are not multiples of a block."""
    import scipy.sparse  # noqa: F401
    if case == "csr":
        Xs, _ = workloads.sbm(3000, 6, 20.0, 20.0, seed=3)
        make = lambda o: P.symnmf_create(  # noqa: E731
            (dev(Xs.indptr.astype(np.int32)), dev(Xs.indices.astype(np.int32)), dev(Xs.data), 3000), 8, 0.0, 0, 2, o)
    else:
        X, _ = workloads.gaussian_kernel(1300, 16, 8, seed=4, dtype=np.float64)
        dt = torch.float64 if case == "dense_f64" else torch.float32
        make = lambda o: P.symnmf_create(dev(X, dt), 12, 0.0, 0, 2, o)  # noqa: E731
    kw = {}
    if case == "bpp":
        kw["rule"] = P.RULE_BPP
    if case == "stall":
        kw.update(stop_mode=P.STOP_STALL, check_every=4, stop_tol=1e-6)
    a = make(P.symnmf_default_options(graphs=1, **kw))
    b = make(P.symnmf_default_options(graphs=0, **kw))
    if case == "lai":
        P.symnmf_lai(a, 24, 1)
        P.symnmf_lai(b, 24, 1)
    done_a = done_b = 0
    for chunk in (3, 8, 13, 8, 5, 16):
        done_a += P.symnmf_iterate(a, chunk)
        done_b += P.symnmf_iterate(b, chunk)
        ra = P.symnmf_residual(a, P.RESID_FAST)
        rb = P.symnmf_residual(b, P.RESID_FAST)
        assert ra == rb
        assert np.array_equal(factor(a, P.H), factor(b, P.H))
        assert np.array_equal(factor(a, P.W), factor(b, P.W))
    assert done_a == done_b
    assert P.symnmf_history(a) == P.symnmf_history(b)
    assert P.symnmf_get_stats(a).graph_launches > 0 and P.symnmf_get_stats(b).graph_launches == 0
    if case == "lai":
        # and after switching to X
        P.symnmf_refine(a)
        P.symnmf_refine(b)
        P.symnmf_iterate(a, 11)
        P.symnmf_iterate(b, 11)
        assert np.array_equal(factor(a, P.H), factor(b, P.H))


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_precision_k64_parity(compute):
    # The precision sweep's shape at a size the oracle finishes quickly:
    # 64-component mixture in R^128, k = 64, FP32 X, products in FP32 or BF16.
    n, k, iters = 6000, 64, 10
    X, _ = workloads.gaussian_kernel(n, 128, 64, seed=2, dtype=np.float32)
    ctx = _ctx(X, k, torch.float32, seed=3, compute=_compute(compute))
    P.symnmf_iterate(ctx, iters)
    sc = O.data_scalars(X)
    H0 = round_to(O.initial_factor(n, k, sc["zeta"], seed=3), torch.float32)
    Wo, Ho, hist = O.plain_symnmf(X, k, sc["maxval"], H0, iters)
    ro = O.residual_direct(X, Wo, Ho) / np.sqrt(sc["normsq"])
    r = P.symnmf_residual(ctx, P.RESID_EXACT)[0]
    log(f"precision k=64 {compute}: residual gpu {r:.8f} oracle {ro:.8f} rel {abs(r - ro) / ro:.2e}")
    assert abs(r - ro) / ro <= (1e-3 if compute == "bf16" else 1e-4)
