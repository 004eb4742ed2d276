"""Parity at the benchmark sizes, in the launch configurations bench.py
times: the dense similarity n = 16384, k = 32 (FP32; plain iterations, and
the LAI basis l = 48, q = 2 with the learned start and LAI iterations), a
LAI run past n = 32768 (the update's U prefetch), the precision sweep
n = 65536, k = 64 (FP32 and BF16 products, both half-steps, the LAI path at
l = 80) and the sparse graph n = 2^20,
k = 64.  The FP64 oracle computes sampled output rows one by one (a row of
X H, a row of the HALS update given the exact Gram) or, at n = 16384, whole
plain iterations; at n = 2^20 a property that holds at any size is checked
too (leverage scores sum to k)."""
import os

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


def _rows(n, count, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=count, replace=False))


@pytest.fixture(scope="module")
def dense16k():
    X, _ = workloads.gaussian_kernel(16384, 64, 32, seed=0, dtype=np.float32)
    return X


def test_dense_16384_product_and_half_step(dense16k):
    X = dense16k
    n, k = X.shape[0], 32
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, 1)
    alpha = P.symnmf_get_stats(ctx).alpha
    H = factor(ctx, P.H)
    W0 = factor(ctx, P.W)
    S = _rows(n, 128, 1)
    XS = X[S].astype(np.float64)
    # the product in the benchmark's configuration (k_gemm_cols, 8 row splits)
    Y = torch.empty((n, k), dtype=torch.float32, device="cuda")
    P.symnmf_apply_x(ctx, dev(H, torch.float32), Y)
    Yo = XS @ H
    e = rel(host(Y)[S], Yo)
    log(f"n=16384 X H sampled rows: rel {e:.2e}")
    assert e <= 2e-6
    # one W half-step: sampled rows of the HALS sweep with the exact Gram
    P.symnmf_half_step(ctx, 0, 0)
    G = H.T @ H + alpha * np.eye(k)
    Wo = O.hals_gy(G, Yo + alpha * H[S], W0[S])
    e = rel(factor(ctx, P.W)[S], Wo)
    log(f"n=16384 W half-step sampled rows: rel {e:.2e}")
    assert e <= 1e-5


def test_dense_16384_three_iterations(dense16k):
    X = dense16k
    n, k, iters = X.shape[0], 32, 3
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, 5)
    P.symnmf_iterate(ctx, iters)
    sc = O.data_scalars(X)
    H0 = round_to(O.initial_factor(n, k, sc["zeta"], seed=5), torch.float32)
    Wo, Ho, hist = O.plain_symnmf(X, k, sc["maxval"], H0, iters)
    hg = np.array(P.symnmf_history(ctx))
    log(f"n=16384 three iterations: history gpu {hg} oracle {hist}")
    assert np.max(np.abs(hg - hist) / hist) <= 1e-4
    assert rel(factor(ctx, P.H), Ho) <= 1e-4


def test_dense_16384_lai_learned_start_and_iterations(dense16k):
    """The benchmark's value path at its size: RRF + Apx-EVD (l = 48, q = 2;
    the sketch is bit-identical on both sides) against the oracle's
    Householder / eigh version; then, from the device's basis, the learned
    start's features, network and scale fit, and LAI iterations."""
    from oracle import warmstart as WS
    from paper_2402_08134_amd import warmstart as WSP
    X = dense16k
    n, k, l, q, seed = X.shape[0], 32, 48, 2, 1
    X64 = X.astype(np.float64)
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, seed)
    P.symnmf_lai(ctx, l, q)
    U = torch.empty((n, l), dtype=torch.float64, device="cuda")
    lam = torch.empty(l, dtype=torch.float64, device="cuda")
    P.symnmf_get_lai(ctx, U, lam)
    Ug, lg = host(U), host(lam)
    Uo, lo = O.apx_evd(lambda M: X64 @ M, O.sketch_omega(n, l, seed), q)
    S = _rows(n, 96, 4)
    e_lam = rel(lg, lo)
    e_xl = rel((Ug[S] * lg) @ Ug.T, (Uo[S] * lo) @ Uo.T)
    log(f"n=16384 l=48 q=2: lambda rel {e_lam:.2e}, sampled rows of U Lambda U^T rel {e_xl:.2e}, "
        f"|U^T U - I| {np.abs(Ug.T @ Ug - np.eye(l)).max():.1e}")
    assert np.abs(Ug.T @ Ug - np.eye(l)).max() <= 1e-12
    assert e_lam <= 1e-4 and e_xl <= 1e-3
    # learned start from the device's basis
    rowsum = O.data_scalars(X64)["rowsum"]
    F = torch.empty((n * k, P.MLP_FEATURES), dtype=torch.float32, device="cuda")
    P.symnmf_warm_features(ctx, F)
    Fo = WS.features(Ug, lg, rowsum, k)
    Fg = host(F)
    e_f = max(rel(Fg[:, c], Fo[:, c]) for c in range(P.MLP_FEATURES))
    net = WSP.load(os.path.join(WSP.WEIGHTS_DIR, "warmstart.bin"))
    p = torch.empty(P.symnmf_mlp_num_params(net), dtype=torch.float32, device="cuda")
    P.symnmf_mlp_get_params(net, p)
    ps = []
    v, o_ = host(p), 0
    for a, b in zip(WS.layer_sizes()[:-1], WS.layer_sizes()[1:]):
        ps.append((v[o_:o_ + a * b].reshape(a, b), v[o_ + a * b:o_ + a * b + b]))
        o_ += a * b + b
    beta = P.symnmf_warmstart(ctx, net)
    H0g = factor(ctx, P.H)
    H0o = WS.warm_start(ps, Ug, lg, rowsum, k, lambda B: X64 @ B)
    e_h0 = rel(H0g, H0o)
    log(f"n=16384 learned start: features max rel {e_f:.2e}, beta {beta:.6f}, H0 rel {e_h0:.2e}")
    assert e_f <= 1e-5 and e_h0 <= 1e-5
    # LAI iterations from that start, against the oracle on the same basis
    iters = 5
    P.symnmf_iterate(ctx, iters)
    Wo, Ho, hist = O.lai_symnmf(Ug, lg, k, O.data_scalars(X64)["maxval"], H0g, iters)
    hg = np.array(P.symnmf_history(ctx))
    e_hist = float(np.max(np.abs(hg - hist) / hist))
    log(f"n=16384 {iters} LAI iterations: history max rel {e_hist:.2e}, H rel {rel(factor(ctx, P.H), Ho):.2e}")
    assert e_hist <= 1e-4 and rel(factor(ctx, P.H), Ho) <= 1e-4


def test_lai_iterations_past_32768_rows():
    """LAI iterations at n = 40000, k = 16 (padded width 16, 16 lanes per row,
    each block prefetching its next chunk of U), against the oracle on the
    device's basis; the basis itself is checked for orthonormality and for
    its eigenvalues against Rayleigh quotients formed on the host."""
    n, k, l, q, seed = 40000, 16, 32, 1, 2
    X = workloads.gpu_gaussian_kernel(n, 32, 16, seed=3)
    ctx = P.symnmf_create(X, k, 0.0, 0, seed)
    P.symnmf_lai(ctx, l, q)
    U = torch.empty((n, l), dtype=torch.float64, device="cuda")
    lam = torch.empty(l, dtype=torch.float64, device="cuda")
    P.symnmf_get_lai(ctx, U, lam)
    Ug, lg = host(U), host(lam)
    assert np.abs(Ug.T @ Ug - np.eye(l)).max() <= 1e-12
    # Rayleigh quotients u_j^T X u_j for the top four, X streamed in row blocks
    top = Ug[:, :4]
    XU = np.zeros_like(top)
    for r0 in range(0, n, 4096):
        XU[r0:r0 + 4096] = host(X[r0:r0 + 4096]) @ top
    rq = np.einsum("ij,ij->j", top, XU)
    log(f"n=40000: lambda[:4] {lg[:4]}, Rayleigh quotients {rq}")
    assert rel(lg[:4], rq) <= 1e-5
    H0 = factor(ctx, P.H)
    maxval = P.symnmf_get_stats(ctx).maxval
    del X
    torch.cuda.empty_cache()
    iters = 4
    P.symnmf_iterate(ctx, iters)
    Wo, Ho, hist = O.lai_symnmf(Ug, lg, k, maxval, H0, iters)
    hg = np.array(P.symnmf_history(ctx))
    e = float(np.max(np.abs(hg - hist) / hist))
    log(f"n=40000 {iters} LAI iterations: history max rel {e:.2e}, H rel {rel(factor(ctx, P.H), Ho):.2e}")
    assert e <= 1e-4 and rel(factor(ctx, P.H), Ho) <= 1e-4


def test_lai_65536_width_64():
    """The precision sweep's LAI path at its size: n = 65536, k = 64, l = 80,
    q = 2 (padded width 64: the update with the vector partial tile and U
    loaded where it is used, l / 16 = 5 tiles), against the oracle on the
    device's basis, checked as at n = 40000."""
    n, k, l, q, seed = 65536, 64, 80, 2, 1
    X = workloads.gpu_gaussian_kernel(n, 128, 64, seed=0)
    ctx = P.symnmf_create(X, k, 0.0, 0, seed)
    P.symnmf_lai(ctx, l, q)
    U = torch.empty((n, l), dtype=torch.float64, device="cuda")
    lam = torch.empty(l, dtype=torch.float64, device="cuda")
    P.symnmf_get_lai(ctx, U, lam)
    Ug, lg = host(U), host(lam)
    assert np.abs(Ug.T @ Ug - np.eye(l)).max() <= 1e-12
    top = Ug[:, :4]
    XU = np.zeros_like(top)
    for r0 in range(0, n, 4096):
        XU[r0:r0 + 4096] = host(X[r0:r0 + 4096]) @ top
    rq = np.einsum("ij,ij->j", top, XU)
    log(f"n=65536: lambda[:4] {lg[:4]}, Rayleigh quotients {rq}")
    assert rel(lg[:4], rq) <= 1e-5
    H0 = factor(ctx, P.H)
    maxval = P.symnmf_get_stats(ctx).maxval
    del X
    torch.cuda.empty_cache()
    iters = 4
    P.symnmf_iterate(ctx, iters)
    Wo, Ho, hist = O.lai_symnmf(Ug, lg, k, maxval, H0, iters)
    hg = np.array(P.symnmf_history(ctx))
    e = float(np.max(np.abs(hg - hist) / hist))
    log(f"n=65536 {iters} LAI iterations: history max rel {e:.2e}, H rel {rel(factor(ctx, P.H), Ho):.2e}")
    assert e <= 1e-4 and rel(factor(ctx, P.H), Ho) <= 1e-4


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_precision_65536_products(compute):
    n, k = 65536, 64
    X = workloads.gpu_gaussian_kernel(n, 128, 64, seed=0)
    o = P.symnmf_default_options()
    if compute == "bf16":
        o.compute_dtype = P.BF16
    ctx = P.symnmf_create(X, k, 0.0, 0, 1, o)
    H = factor(ctx, P.H)
    Y = torch.empty((n, k), dtype=torch.float32, device="cuda")
    P.symnmf_apply_x(ctx, dev(H, torch.float32), Y)
    S = _rows(n, 64, 2)
    XS = host(X[torch.from_numpy(S).cuda()])
    del ctx, X
    torch.cuda.empty_cache()
    Yg = host(Y)[S]
    if compute == "f32":
        e = rel(Yg, XS @ H)
        log(f"n=65536 FP32 X H sampled rows: rel {e:.2e}")
        assert e <= 1e-5
    else:
        e = rel(Yg, round_to(XS, torch.bfloat16) @ round_to(H, torch.bfloat16))
        e2 = rel(Yg, XS @ H)
        log(f"n=65536 BF16 X H sampled rows: rel {e:.2e} (vs FP32 data {e2:.2e})")
        assert e <= 1e-5 and e2 <= 1e-2


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_precision_65536_half_steps(compute):
    # both half-steps at the precision sweep's size, where the HALS sweep runs
    # blocked (16-column blocks, the other columns' terms on the FP64 matrix
    # cores, split-K product partials); the second product reads the
    # transposed panel the first update wrote.  Sampled rows against the
    # sweep with the exact Gram, (1) on the library's own product X F (the
    # same inputs: the sweep itself within 1e-5) and (2) on the FP64 product:
    # there the FP32 product's own error over 65536 terms (about 1e-5) comes
    # out of the sweep amplified, measured 8.5e-5 with either sweep layout
    n, k = 65536, 64
    X = workloads.gpu_gaussian_kernel(n, 128, 64, seed=0)
    o = P.symnmf_default_options()
    if compute == "bf16":
        o.compute_dtype = P.BF16
    ctx = P.symnmf_create(X, k, 0.0, 0, 1, o)
    alpha = P.symnmf_get_stats(ctx).alpha
    H = factor(ctx, P.H)
    W0 = factor(ctx, P.W)
    P.symnmf_half_step(ctx, 0, 0)
    W = factor(ctx, P.W)
    P.symnmf_half_step(ctx, 1, 1)
    H1 = factor(ctx, P.H)
    S = _rows(n, 64, 4)
    Sd = torch.from_numpy(S).cuda()
    prods = []
    for F in (H, W):
        Y = torch.empty((n, k), dtype=torch.float32, device="cuda")
        P.symnmf_apply_x(ctx, dev(F, torch.float32), Y)
        prods.append(host(Y[Sd]))
    XS = host(X[Sd])
    del ctx, X
    torch.cuda.empty_cache()
    GH, GW = H.T @ H + alpha * np.eye(k), W.T @ W + alpha * np.eye(k)
    e = rel(W[S], O.hals_gy(GH, prods[0] + alpha * H[S], W0[S]))
    e2 = rel(H1[S], O.hals_gy(GW, prods[1] + alpha * W[S], H[S]))
    q = (lambda A: round_to(A, torch.bfloat16)) if compute == "bf16" else (lambda A: A)
    f = rel(W[S], O.hals_gy(GH, q(XS) @ q(H) + alpha * H[S], W0[S]))
    f2 = rel(H1[S], O.hals_gy(GW, q(XS) @ q(W) + alpha * W[S], H[S]))
    log(f"n=65536 {compute} half-steps sampled rows: on the library's product W rel {e:.2e}, H rel {e2:.2e}; "
        f"on the FP64 product W rel {f:.2e}, H rel {f2:.2e}")
    assert e <= 1e-5 and e2 <= 1e-5
    assert f <= 2e-4 and f2 <= 2e-4


def test_sparse_2pow20_spmm_and_leverage():
    X, _ = workloads.sbm(1 << 20, 64, 32.0, 20.0, seed=0)
    n, k = X.shape[0], 64
    ctx = P.symnmf_create(csr_dev(X), k, 0.0, 0, 1)
    H = factor(ctx, P.H)
    Y = torch.empty((n, k), dtype=torch.float32, device="cuda")
    P.symnmf_apply_x(ctx, dev(H, torch.float32), Y)
    S = _rows(n, 256, 3)
    X64 = sp.csr_matrix((X.data.astype(np.float64), X.indices, X.indptr), shape=X.shape)
    e = rel(host(Y)[S], X64[S] @ H)
    log(f"n=2^20 SpMM sampled rows: rel {e:.2e}")
    assert e <= 1e-6
    lev = torch.empty(n, dtype=torch.float64, device="cuda")
    P.symnmf_leverage(ctx, P.H, lev)
    lg = host(lev)
    tot = float(lg.sum())
    log(f"n=2^20 leverage scores of H: sum {tot:.10f} (k = {k})")
    assert abs(tot - k) <= 1e-8 * k
    # sampled rows: l_i = h_i (H^T H)^-1 h_i^T with the exact FP64 Gram
    Gi = np.linalg.inv(H.T @ H)
    lo = np.einsum("ij,jk,ik->i", H[S], Gi, H[S])
    assert rel(lg[S], lo) <= 1e-9
