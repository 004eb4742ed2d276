"""GPU parity of the BPP update rule (exact per-row NLS by block principal
pivoting) against the FP64 oracle's exact NLS (brute-force enumeration for
k <= 10, Lawson-Hanson above), through the C ABI: single half-steps from
identical inputs in the plain, LAI and LvS modes, KKT conditions of the GPU
result itself, and whole runs."""
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


def _bpp_opts(**kw):
    return P.symnmf_default_options(rule=P.RULE_BPP, **kw)


def _kkt(x, G, Y):
    """Largest violations of the NLS optimality conditions of every row:
    x >= 0, g = G x - y >= 0, x * g = 0 (scaled by the data)."""
    g = x @ G - Y
    ys = np.linalg.norm(Y)
    return {"neg_x": float(max(0.0, -x.min())), "neg_g": float(max(0.0, -g.min()) / ys),
            "compl": float(np.abs(x * g).max() / (ys * ys / np.linalg.norm(G)))}


@pytest.mark.parametrize("case", [("f64", 1111, 8), ("f64", 1111, 13), ("f32", 1500, 32), ("f64", 320, 64)])
def test_bpp_half_step_identical_inputs(case):
    kind, n, k = case
    log(f"bpp half step {case}")
    # clustered X and a factor whose columns each straddle two clusters: the
    # exact solution needs both active and bound variables
    X, H0 = workloads.planted(n, k, noise=0.01, seed=3)
    tdt = torch.float64 if kind == "f64" else torch.float32
    ctx = P.symnmf_create(dev(X, tdt), k, 0.0, 0, 0, _bpp_opts())
    alpha = float(round_to(X, tdt).max())
    H = H0 + np.roll(H0, 1, axis=1)
    W = workloads.random_factor(n, k, seed=2, scale=0.3)
    W[W < 0.1] = 0.0                      # a start support that is not the answer
    P.symnmf_set_factor(ctx, P.H, dev(H))
    P.symnmf_set_factor(ctx, P.W, dev(W))
    if kind == "f32":
        X, H = round_to(X, tdt), round_to(H, tdt)
    P.symnmf_half_step(ctx, 0)
    G = H.T @ H + alpha * np.eye(k)
    Y = O.apply_x(X, H) + alpha * H
    Wo = O.nls_gy(G, Y)
    Wg = factor(ctx, P.W)
    err = rel(Wg, Wo)
    kkt = _kkt(Wg, G, Y)
    log(f"bpp {case}: rel {err:.2e} zeros {np.mean(Wo == 0):.2f} kkt {kkt}")
    assert 0.05 < np.mean(Wo == 0) < 0.95          # both sets non-trivial
    tol = 1e-11 if kind == "f64" else 2e-5
    assert err <= tol
    assert np.array_equal(Wg == 0, Wo == 0) or kind == "f32"
    if kind == "f64":
        assert kkt["neg_x"] == 0.0 and kkt["neg_g"] <= 1e-12 and kkt["compl"] <= 1e-12
    assert P.symnmf_get_stats(ctx).flags & P.FLAG_BPP_CAP == 0


def test_bpp_planted_fp64_run():
    n, k, iters = 1000, 12, 15
    X, _ = workloads.planted(n, k, noise=0.01, seed=2)
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, 4, _bpp_opts())
    P.symnmf_iterate(ctx, iters)
    sc = O.data_scalars(X)
    H0 = O.initial_factor(n, k, sc["zeta"], 4)
    Wo, Ho, hist = O.plain_symnmf(X, k, sc["maxval"], H0, iters, rule="nls")
    hg = np.array(P.symnmf_history(ctx))
    log(f"bpp planted: W {rel(factor(ctx, P.W), Wo):.2e} H {rel(factor(ctx, P.H), Ho):.2e} "
        f"r {hg[-1]:.6f} / {hist[-1]:.6f}")
    assert rel(factor(ctx, P.W), Wo) <= 1e-9 and rel(factor(ctx, P.H), Ho) <= 1e-9
    assert np.max(np.abs(hg - hist) / hist) <= 1e-10


def test_bpp_gaussian_kernel_f32_run():
    n, k, iters = 2300, 32, 6
    X, _ = workloads.gaussian_kernel(n, 64, 32, seed=1, dtype=np.float32)
    ctx = P.symnmf_create(dev(X, torch.float32), k, 0.0, 0, 5, _bpp_opts())
    P.symnmf_iterate(ctx, iters)
    sc = O.data_scalars(X)
    H0 = round_to(O.initial_factor(n, k, sc["zeta"], 5), torch.float32)
    Wo, Ho, hist = O.plain_symnmf(X, k, sc["maxval"], H0, iters, rule="nls")
    r = P.symnmf_residual(ctx, P.RESID_EXACT)[0]
    ro = O.residual_direct(X, Wo, Ho) / np.sqrt(sc["normsq"])
    log(f"bpp gk f32: residual gpu {r:.8f} oracle {ro:.8f}")
    assert abs(r - ro) / ro <= 1e-4
    hg = np.array(P.symnmf_history(ctx))
    assert np.max(np.abs(hg - hist) / hist) <= 1e-4


def test_bpp_lai_fp64_run():
    n, k, l, q, iters, seed = 1200, 10, 26, 2, 8, 3
    X, _ = workloads.gaussian_kernel(n, 16, 10, seed=8, dtype=np.float64)
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, seed, _bpp_opts())
    P.symnmf_lai(ctx, l, q)
    P.symnmf_iterate(ctx, iters)
    Uo, lo = O.apx_evd(lambda M: O.apply_x(X, M), O.sketch_omega(n, l, seed), q)
    sc = O.data_scalars(X)
    H0 = O.initial_factor(n, k, sc["zeta"], seed)
    Wo, Ho, hist = O.lai_symnmf(Uo, lo, k, sc["maxval"], H0, iters, rule="nls")
    hg = np.array(P.symnmf_history(ctx))
    log(f"bpp lai: H {rel(factor(ctx, P.H), Ho):.2e} hist {np.max(np.abs(hg - hist) / hist):.2e}")
    assert rel(factor(ctx, P.H), Ho) <= 1e-7
    assert np.max(np.abs(hg - hist) / hist) <= 1e-9


def test_bpp_lvs_half_step_identical_inputs():
    X, _ = workloads.sbm(8000, 16, 30.0, 20.0, seed=4)
    n, k, s = X.shape[0], 16, 800
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, s, 9, _bpp_opts())
    alpha = P.symnmf_get_stats(ctx).alpha
    H = workloads.random_factor(n, k, seed=6, scale=0.2)
    W = workloads.random_factor(n, k, seed=7, scale=0.2)
    P.symnmf_set_factor(ctx, P.H, dev(H))
    P.symnmf_set_factor(ctx, P.W, dev(W))
    H32, W32 = round_to(H, torch.float32), round_to(W, torch.float32)
    P.symnmf_half_step(ctx, 0, 4)
    X64 = sp.csr_matrix((X.data.astype(np.float64), X.indices, X.indptr), shape=X.shape)
    Wo, info = O.lvs_half_step(X64, H32, W32, alpha, s, 1.0 / s, 9, 4, rule="nls")
    err = rel(factor(ctx, P.W), Wo)
    log(f"bpp lvs half step: rows {len(info['rows'])} rel {err:.2e}")
    assert err <= 1e-5


def test_bpp_rows_with_zero_target_are_zero():
    # Rows of X and H zeroed together give a zero right-hand side; their exact
    # NLS solution is the zero row, whatever the start support.
    n, k = 200, 6
    X, _ = workloads.planted(n, k, noise=0.0, seed=1)
    alpha = float(X.max())
    H = workloads.random_factor(n, k, seed=3, scale=0.5)
    H[::3] = 0.0
    X[::3, :] = 0.0
    X[:, ::3] = 0.0
    ctx = P.symnmf_create(dev(X), k, alpha, 0, 0, _bpp_opts())
    P.symnmf_set_factor(ctx, P.H, dev(H))
    P.symnmf_set_factor(ctx, P.W, dev(workloads.random_factor(n, k, seed=4, scale=0.5)))
    P.symnmf_half_step(ctx, 0)
    Wo = O.nls_gy(H.T @ H + alpha * np.eye(k), O.apply_x(X, H) + alpha * H)
    Wg = factor(ctx, P.W)
    assert np.all(Wg[::3] == 0.0) and np.all(Wo[::3] == 0.0)
    assert rel(Wg, Wo) <= 1e-12
