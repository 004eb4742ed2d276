"""GPU parity of the LAI path (Algorithms RRF, Apx-EVD, LAI-SymNMF) against
the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import symnmf as O
import workloads

from gpu_common import P, torch, require_gpu, dev, host, rel, factor, round_to, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("dtype,compute", [("f64", None), ("f32", None), ("f32", "bf16")])
def test_lai_parity(dtype, compute):
    n, k, l, q, seed = 1500, 16, 32, 2, 11
    X, _ = workloads.gaussian_kernel(n, 32, 16, seed=7, dtype=np.float64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    o = P.symnmf_default_options()
    if compute == "bf16":
        o.compute_dtype = P.BF16
    ctx = P.symnmf_create(dev(X, tdt), k, 0.0, 0, seed, o)
    P.symnmf_lai(ctx, l, q)
    U = torch.empty((n, l), dtype=torch.float64, device="cuda")
    lam = torch.empty(l, dtype=torch.float64, device="cuda")
    P.symnmf_get_lai(ctx, U, lam)
    Ug, lg = host(U), host(lam)
    Xo = round_to(X, tdt)
    if compute == "bf16":
        Xo = round_to(Xo, torch.bfloat16)
    Om = O.sketch_omega(n, l, seed)
    Uo, lo = O.apx_evd(lambda M: O.apply_x(Xo, M), Om, q)
    assert np.abs(Ug.T @ Ug - np.eye(l)).max() <= 1e-12
    assert np.all(np.diff(lg) <= 0)
    tol = {"f64": 1e-10, "f32": 2e-4, "bf16": 2e-2}[compute or dtype]
    log(f"lai {dtype}/{compute}: lam rel {rel(lg, lo):.2e}")
    assert rel(lg, lo) <= tol
    XLg = (Ug * lg) @ Ug.T
    XLo = (Uo * lo) @ Uo.T
    assert rel(XLg, XLo) <= 10 * tol
    # LAI iterations: residual against U Lambda U^T, same start
    iters = 20
    P.symnmf_iterate(ctx, iters)
    sc = O.data_scalars(Xo)
    H0 = round_to(O.initial_factor(n, k, sc["zeta"], seed), tdt)
    Wo, Ho, hist = O.lai_symnmf(Uo, lo, k, sc["maxval"], H0, iters)
    hg = np.array(P.symnmf_history(ctx))
    rtol = {"f64": 1e-8, "f32": 1e-4, "bf16": 1e-3}[compute or dtype]
    log(f"lai {dtype}/{compute}: history max rel {np.max(np.abs(hg - hist) / hist):.2e}")
    assert np.max(np.abs(hg - hist) / hist) <= rtol
    r = P.symnmf_residual(ctx, P.RESID_LAI)
    assert abs(r[0] - hist[-1]) / hist[-1] <= rtol
    # residual against the full X (the quantity the paper reports)
    re = P.symnmf_residual(ctx, P.RESID_EXACT)
    ro = O.residual_direct(Xo, Wo, Ho) / np.linalg.norm(Xo)
    assert abs(re[0] - ro) / ro <= rtol


@pytest.mark.parametrize("case", [(1500, 32, 48, "f32"), (1500, 64, 80, "f32"), (1333, 30, 46, "f64"),
                                  (1333, 64, 96, "f64"), (1100, 40, 56, "f32")])
def test_lai_wide_parity(case):
    # wider factors and bases: padded widths 32 and 64 take the update layout
    # with 8 lanes per row and 64-row chunks (n ragged against the chunk);
    # k = 64 with l = 96 in FP64 (staging too large for LDS) and width 48
    # keep 16 lanes per row
    n, k, l, dtype = case
    log(f"lai wide n={n} k={k} l={l} {dtype}")
    q, seed, iters = 1, 3, 10
    X, _ = workloads.gaussian_kernel(n, 2 * k, k, seed=k + l, dtype=np.float64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ctx = P.symnmf_create(dev(X, tdt), k, 0.0, 0, seed)
    P.symnmf_lai(ctx, l, q)
    P.symnmf_iterate(ctx, iters)
    Xo = round_to(X, tdt)
    Uo, lo = O.apx_evd(lambda M: O.apply_x(Xo, M), O.sketch_omega(n, l, seed), q)
    sc = O.data_scalars(Xo)
    H0 = round_to(O.initial_factor(n, k, sc["zeta"], seed), tdt)
    Wo, Ho, hist = O.lai_symnmf(Uo, lo, k, sc["maxval"], H0, iters)
    hg = np.array(P.symnmf_history(ctx))
    rtol = 1e-8 if dtype == "f64" else 1e-4
    log(f"   history max rel {np.max(np.abs(hg - hist) / hist):.2e}, H rel {rel(factor(ctx, P.H), Ho):.2e}")
    assert np.max(np.abs(hg - hist) / hist) <= rtol
    assert rel(factor(ctx, P.H), Ho) <= (1e-6 if dtype == "f64" else 1e-2)


def test_lai_exact_low_rank_input():
    # X of rank r <= l: the LAI reproduces X, so the LAI residual against
    # U Lambda U^T equals the residual against X.
    n, k, l = 700, 6, 12
    _, H0 = workloads.planted(n, 8, noise=0.0, seed=3)
    X = H0 @ H0.T
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, 4)
    P.symnmf_lai(ctx, l, 1)
    U = torch.empty((n, l), dtype=torch.float64, device="cuda")
    lam = torch.empty(l, dtype=torch.float64, device="cuda")
    P.symnmf_get_lai(ctx, U, lam)
    Ug, lg = host(U), host(lam)
    assert rel((Ug * lg) @ Ug.T, X) <= 1e-11
    P.symnmf_iterate(ctx, 5)
    a = P.symnmf_residual(ctx, P.RESID_LAI)
    b = P.symnmf_residual(ctx, P.RESID_EXACT)
    assert abs(a[0] - b[0]) <= 1e-9


def test_lai_rejects_bad_rank():
    X, _ = workloads.planted(200, 4, noise=0.01, seed=1)
    ctx = P.symnmf_create(dev(X), 4, 0.0, 0, 0)
    for l in (3, 97, 201):
        with pytest.raises(P.SymNMFError):
            P.symnmf_lai(ctx, l, 1)


def test_lai_then_refinement_parity():
    # LAI-HALS followed by iterative refinement on the full X.
    n, k, l, q, seed = 1200, 12, 28, 2, 5
    X, _ = workloads.gaussian_kernel(n, 16, 12, seed=8, dtype=np.float64)
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, seed)
    P.symnmf_lai(ctx, l, q)
    P.symnmf_iterate(ctx, 12)
    P.symnmf_refine(ctx, P.STOP_NONE, 0.0)
    assert P.symnmf_get_stats(ctx).mode == P.MODE_PLAIN
    P.symnmf_iterate(ctx, 6)
    sc = O.data_scalars(X)
    H0 = O.initial_factor(n, k, sc["zeta"], seed)
    Uo, lo = O.apx_evd(lambda M: X @ M, O.sketch_omega(n, l, seed), q)
    W1, H1, h1 = O.lai_symnmf(Uo, lo, k, sc["maxval"], H0, 12)
    W2, H2, h2 = O.anls(lambda B: X @ B, sc["normsq"], H1, sc["maxval"], 6, W0=W1)
    hg = np.array(P.symnmf_history(ctx))
    assert len(hg) == 18
    assert np.max(np.abs(hg[12:] - h2) / h2) <= 1e-8
    assert rel(factor(ctx, P.H), H2) <= 1e-7
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_refine(ctx, P.STOP_NONE, 0.0)      # no longer in LAI mode
    assert e.value.code == P.E_STATE


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ada_rrf_parity(dtype):
    # Algorithm Ada-RRF: the same number of rounds as the oracle (its residual
    # drops are 2.5e-2 then 6.2e-4 against the 1e-3 tolerance, far from a tie),
    # the same last QB residual, and the same Apx-EVD of the resulting basis.
    n, k, l, seed = 1500, 16, 32, 11
    X, _ = workloads.gaussian_kernel(n, 32, 16, seed=7, dtype=np.float64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Xo = round_to(X, tdt)
    ctx = P.symnmf_create(dev(X, tdt), k, 0.0, 0, seed)
    rounds, r = P.symnmf_lai_adaptive(ctx, l, 10, 1e-3)
    nx = float(np.sum(Xo * Xo))
    Qo, rounds_o, res = O.ada_rrf(lambda M: O.apply_x(Xo, M), nx, O.sketch_omega(n, l, seed), 10, 1e-3)
    log(f"ada-rrf {dtype}: rounds gpu {rounds} oracle {rounds_o}; residual gpu {r:.8f} oracle {res[-1]:.8f}")
    assert rounds == rounds_o == 2
    assert abs(r - res[-1]) / res[-1] <= (1e-10 if dtype == "f64" else 1e-5)
    Uo, lo = O.apx_evd(lambda M: O.apply_x(Xo, M), None, 0, Q=Qo)
    lam = torch.empty(l, dtype=torch.float64, device="cuda")
    P.symnmf_get_lai(ctx, None, lam)
    assert rel(host(lam), lo) <= (1e-10 if dtype == "f64" else 2e-4)
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_lai_adaptive(ctx, l, 0, 1e-3)
    assert e.value.code == P.E_INVALID


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_lai_on_csr_parity(dtype):
    """Algorithms RRF, Apx-EVD and LAI-SymNMF on a sparse graph (the
    algorithms need only products with X, which run through the CSR kernel),
    then the learned start's features and refinement on the CSR X."""
    from oracle import warmstart as WS
    from gpu_common import csr_dev
    import scipy.sparse as sp
    n, k, l, q, seed, iters = 3001, 8, 24, 2, 6, 8
    Xs, _ = workloads.sbm(n, 8, 24.0, 20.0, seed=4)
    if dtype == "f64":
        Xs = sp.csr_matrix((Xs.data.astype(np.float64), Xs.indices, Xs.indptr), shape=Xs.shape)
    X64 = sp.csr_matrix((Xs.data.astype(np.float64), Xs.indices, Xs.indptr), shape=Xs.shape)
    ctx = P.symnmf_create(csr_dev(Xs), k, 0.0, 0, seed)
    P.symnmf_lai(ctx, l, q)
    U = torch.empty((n, l), dtype=torch.float64, device="cuda")
    lam = torch.empty(l, dtype=torch.float64, device="cuda")
    P.symnmf_get_lai(ctx, U, lam)
    Ug, lg = host(U), host(lam)
    Uo, lo = O.apx_evd(lambda M: X64 @ M, O.sketch_omega(n, l, seed), q)
    tol = 1e-10 if dtype == "f64" else 1e-4
    S = np.arange(0, n, 37)
    e_l, e_x = rel(lg, lo), rel((Ug[S] * lg) @ Ug.T, (Uo[S] * lo) @ Uo.T)
    log(f"csr lai {dtype}: lambda rel {e_l:.2e}, sampled U Lambda U^T rows rel {e_x:.2e}")
    assert np.abs(Ug.T @ Ug - np.eye(l)).max() <= 1e-12
    assert e_l <= tol and e_x <= 10 * tol
    sc = O.data_scalars(X64)
    F = torch.empty((n * k, P.MLP_FEATURES), dtype=torch.float32, device="cuda")
    P.symnmf_warm_features(ctx, F)
    Fo = WS.features(Ug, lg, sc["rowsum"], k)
    assert max(rel(host(F)[:, c], Fo[:, c]) for c in range(P.MLP_FEATURES)) <= 1e-5
    H0 = factor(ctx, P.H)
    P.symnmf_iterate(ctx, iters)
    Wo, Ho, hist = O.lai_symnmf(Ug, lg, k, sc["maxval"], H0, iters)
    hg = np.array(P.symnmf_history(ctx))
    rtol = 1e-8 if dtype == "f64" else 1e-4
    log(f"csr lai {dtype}: {iters} LAI iterations, history max rel {np.max(np.abs(hg - hist) / hist):.2e}")
    assert np.max(np.abs(hg - hist) / hist) <= rtol
    P.symnmf_refine(ctx, P.STOP_NONE, 0.0)
    P.symnmf_iterate(ctx, 3)
    W2, H2, h2 = O.anls(lambda B: X64 @ B, sc["normsq"], Ho, sc["maxval"], 3, W0=Wo)
    hg = np.array(P.symnmf_history(ctx))
    assert np.max(np.abs(hg[iters:] - h2) / h2) <= rtol
