"""GPU parity of PGNCG and LAI-PGNCG (Section 2.1.3; Algorithm
LAI-PGNCG-SymNMF) against the FP64 oracle, through the C ABI: dense FP64 and
FP32 X, CSR X, every padded rank width, one and many CG steps, the LAI
operator, graph replay, the stop rule and argument errors."""
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


def _opts(cg_iters=5, **kw):
    return P.symnmf_default_options(rule=P.RULE_PGNCG, cg_iters=cg_iters, **kw)


def _h0(X, n, k, seed, dtype):
    sc = O.data_scalars(X)
    return round_to(O.initial_factor(n, k, sc["zeta"], seed=seed), dtype)


def _hist(ctx):
    return np.array(P.symnmf_history(ctx))


def test_dense_fp64_parity():
    # ragged n (15 chunks of 64 rows + 40), k = 10 (padded to 16)
    n, k, iters = 1000, 10, 15
    X, _ = workloads.gaussian_kernel(n, 20, 10, seed=7, dtype=np.float64)
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, 3, _opts())
    P.symnmf_iterate(ctx, iters)
    Ho, ho = O.plain_pgncg(X, _h0(X, n, k, 3, torch.float64), iters, 5)
    hg, Hg = _hist(ctx), factor(ctx, P.H)
    log(f"fp64: history rel {rel(hg, ho):.2e}, H rel {rel(Hg, Ho):.2e}, last {hg[-1]:.6f}")
    assert len(hg) == iters
    assert rel(hg, ho) <= 1e-10
    assert rel(Hg, Ho) <= 1e-8
    assert np.array_equal(factor(ctx, P.W), Hg)  # W is kept equal to H


@pytest.mark.parametrize("case", [(2300, 32, 5), (1100, 48, 1), (1100, 48, 12), (777, 64, 5), (70, 1, 3)])
def test_dense_fp32_parity(case):
    n, k, cg = case
    log(f"fp32 case n={n} k={k} cg_iters={cg}")
    iters = 12
    X, _ = workloads.gaussian_kernel(n, max(2 * k, 4), max(k, 2), seed=n + k, dtype=np.float32)
    X = np.asarray(X, dtype=np.float32)
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, 5, _opts(cg))
    P.symnmf_iterate(ctx, iters)
    X64 = X.astype(np.float64)
    Ho, ho = O.plain_pgncg(X64, _h0(X64, n, k, 5, torch.float32), iters, cg)
    hg = _hist(ctx)
    r = P.symnmf_residual(ctx, P.RESID_EXACT)[1]
    ro = O.residual_direct(X64, Ho, Ho) / np.linalg.norm(X64)
    log(f"   residual gpu {r:.8f} oracle {ro:.8f}; history rel {rel(hg, ho):.2e}; H rel {rel(factor(ctx, P.H), Ho):.2e}")
    assert abs(r - ro) / ro <= 1e-4
    assert np.max(np.abs(hg - ho) / ho) <= 1e-3


def test_csr_parity():
    X, _ = workloads.sbm(3000, 8, 24.0, 20.0, seed=11)
    n, k, iters = X.shape[0], 16, 10
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, 0, 2, _opts())
    P.symnmf_iterate(ctx, iters)
    X64 = sp.csr_matrix((X.data.astype(np.float64), X.indices, X.indptr), shape=X.shape)
    Ho, ho = O.plain_pgncg(X64, _h0(X64, n, k, 2, torch.float32), iters, 5)
    hg = _hist(ctx)
    log(f"csr: history rel {rel(hg, ho):.2e}, H rel {rel(factor(ctx, P.H), Ho):.2e}")
    assert np.max(np.abs(hg - ho) / ho) <= 1e-3
    assert rel(factor(ctx, P.H), Ho) <= 1e-3


def test_lai_pgncg_parity_and_refinement():
    n, k, l, q, iters = 1500, 16, 32, 2, 10
    X, _ = workloads.gaussian_kernel(n, 32, 16, seed=4, dtype=np.float64)
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, 6, _opts())
    P.symnmf_lai(ctx, l, q)
    P.symnmf_iterate(ctx, iters)
    U, lam = O.apx_evd(lambda M: O.apply_x(X, M), O.sketch_omega(n, l, 6), q)
    Ho, ho = O.lai_pgncg(U, lam, _h0(X, n, k, 6, torch.float64), iters, 5)
    hg, Hg = _hist(ctx), factor(ctx, P.H)
    log(f"lai: history rel {rel(hg, ho):.2e}, H rel {rel(Hg, Ho):.2e}")
    assert rel(hg, ho) <= 1e-8 and rel(Hg, Ho) <= 1e-6
    # refinement continues on X from the LAI factor (Section 3.3)
    P.symnmf_refine(ctx)
    P.symnmf_iterate(ctx, 5)
    Hr, hr = O.plain_pgncg(X, Ho, 5, 5)
    log(f"refined: H rel {rel(factor(ctx, P.H), Hr):.2e}")
    assert rel(_hist(ctx)[iters:], hr) <= 1e-8 and rel(factor(ctx, P.H), Hr) <= 1e-6


@pytest.mark.parametrize("lai", [False, True])
def test_graph_replay_matches_eager(lai):
    n, k = 1300, 24
    X, _ = workloads.gaussian_kernel(n, 48, 24, seed=8, dtype=np.float32)
    out = []
    for graphs in (0, 1):
        ctx = P.symnmf_create(dev(X, torch.float32), k, 0.0, 0, 1, _opts(4, graphs=graphs))
        if lai:
            P.symnmf_lai(ctx, k + 16, 1)
        P.symnmf_iterate(ctx, 20)
        st = P.symnmf_get_stats(ctx)
        out.append((factor(ctx, P.H), _hist(ctx), st.graph_launches))
    assert out[0][2] == 0 and out[1][2] > 0
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_stop_rule():
    n, k = 1200, 12
    X, _ = workloads.gaussian_kernel(n, 24, 12, seed=9, dtype=np.float32)
    ctx = P.symnmf_create(dev(X, torch.float32), k, 0.0, 0, 4,
                          _opts(3, stop_mode=P.STOP_STALL, stop_tol=1e-3, check_every=2))
    done = P.symnmf_iterate(ctx, 500)
    hg = _hist(ctx)
    assert 0 < done < 500 and len(hg) == done
    # the stall rule holds exactly at the stop and at no earlier iteration
    rule = O.StallRule(tol=1e-3, patience=4)
    fired = [rule(r) for r in hg]
    assert fired[-1] and not any(fired[:-1])
    # stopped: later calls do nothing
    H1 = factor(ctx, P.H)
    assert P.symnmf_iterate(ctx, 5) == 0 and np.array_equal(factor(ctx, P.H), H1)


def test_invalid_arguments():
    X, _ = workloads.planted(200, 4, noise=0.01, seed=0)
    for cg in (0, 65):
        with pytest.raises(P.SymNMFError) as e:
            P.symnmf_create(dev(X), 4, 0.0, 0, 0, _opts(cg))
        assert e.value.code == P.E_INVALID
    ctx = P.symnmf_create(dev(X), 4, 0.0, 0, 0, _opts())
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_half_step(ctx, 0)
    assert e.value.code == P.E_UNSUPPORTED
    Xs, _ = workloads.sbm(2000, 4, 20.0, 20.0, seed=1)
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_create(csr_dev(Xs), 4, 0.0, 64, 0, _opts())
    assert e.value.code == P.E_UNSUPPORTED
