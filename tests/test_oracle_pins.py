"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics,
not by the oracle itself: published known answers, closed forms, invariants,
special cases that reduce to textbook routines, and brute force.

Each test names the oracle function(s) it pins and why a plausible mistake in
them (dropped term, wrong sign or index, transposed operand) would fail it.
"""
import os

import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy import stats

from oracle import philox
from oracle import symnmf as O
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# RNG: Philox-4x32-10 against the published known-answer vectors.
# --------------------------------------------------------------------------

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(np.array([v[0:4]], dtype=np.uint32), (v[4], v[5]))[0]
        assert [int(x) for x in out] == v[6:10]


def test_philox_stream_layout_and_uniform():
    # value e is word pair (e mod 2) of block e div 2; uniform = (v >> 11) 2^-53
    seed = (7 << 32) | 123
    v = philox.u64_stream(seed, 9, 5, 3)
    w = philox.philox4x32_10(np.array([[2, 0, 5, 3]], dtype=np.uint32), (123, 7))[0].astype(np.uint64)
    assert v[4] == (w[0] | (w[1] << np.uint64(32)))
    assert v[5] == (w[2] | (w[3] << np.uint64(32)))
    u = philox.uniform(seed, 200000, 0, philox.TAG_H0)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_philox_gaussian_and_draws():
    z = philox.gaussian(11, 200000, 0, philox.TAG_OMEGA)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    d = philox.draws(3, 60000, 1, philox.TAG_SAMPLE, 6)
    assert d.min() >= 0 and d.max() <= 5
    cnt = np.bincount(d, minlength=6)
    assert stats.chisquare(cnt).pvalue > 1e-3
    # the draw is floor(v * bound / 2^64): bound 2^64 returns v itself
    v = philox.u64_stream(3, 5, 1, philox.TAG_SAMPLE)
    assert [int(x) for x in philox.draws(3, 5, 1, philox.TAG_SAMPLE, 1 << 64)] == [int(x) for x in v]


def test_sketch_log_against_the_math_library():
    """The sketch's own logarithm agrees with the platform log to a few ulps
    on (0, 1] (relative where |ln x| > 1/4; near x = 1, where ln x -> 0, an
    absolute bound; the reduction's e ln 2 + ln m can cancel up to a factor 2
    for x in [1/2, sqrt(1/2)), hence 8 half-ulps), and is exact at x = 1."""
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.integers(0, 2 ** 53, 200000, dtype=np.uint64),
                        np.array([0, 1, 2 ** 52, 2 ** 53 - 1, 2 ** 53 - 2], dtype=np.uint64)])
    x = ((np.uint64(1) << np.uint64(53)) - a).astype(np.float64) * 2.0 ** -53
    L = philox.log_unit(a)
    ref = np.array([math.log(v) for v in x])
    far = np.abs(ref) > 0.25
    assert np.max(np.abs(L - ref)[far] / np.abs(ref[far])) <= 8 * 2.0 ** -53
    assert np.max(np.abs(L - ref)[~far]) <= 4 * 2.0 ** -53
    assert L[-5] == 0.0                                   # x = 1
    # ln 2^-j = -j ln 2 to the accuracy of the split constant
    for j in (1, 2, 10, 52, 53):
        v = philox.log_unit(np.array([2 ** 53 - 2 ** (53 - j)], dtype=np.uint64))[0]
        assert abs(v + j * math.log(2.0)) <= 2 * j * 2.0 ** -53


def test_sketch_cosine_identities():
    """cos(2 pi u) of the sketch: exact at quarter turns, even, the
    Pythagorean identity with the quarter-turn shift (sin), and within a
    few ulps of the platform cosine (whose own argument 2 pi u is rounded)."""
    q = np.array([0, 2 ** 51, 2 ** 52, 3 * 2 ** 51], dtype=np.uint64)
    assert list(philox.cos_turn(q)) == [1.0, 0.0, -1.0, 0.0]
    rng = np.random.default_rng(2)
    b = rng.integers(1, 2 ** 53, 200000, dtype=np.uint64)
    b = b[(b % np.uint64(2 ** 51)) != np.uint64(2 ** 50)]   # off the half-quadrant ties
    c = philox.cos_turn(b)
    assert np.array_equal(philox.cos_turn((np.uint64(1) << np.uint64(53)) - b), c)
    s = philox.cos_turn((b - np.uint64(2 ** 51)) % np.uint64(2 ** 53))   # cos(x - pi/2) = sin x
    assert np.max(np.abs(c * c + s * s - 1.0)) <= 6 * 2.0 ** -53
    u = b.astype(np.float64) * 2.0 ** -53
    assert np.max(np.abs(c - np.cos(2.0 * np.pi * u))) <= 8 * 2.0 ** -53


# --------------------------------------------------------------------------
# Scalars and initialisation.
# --------------------------------------------------------------------------

def test_data_scalars_hand_example():
    X = np.array([[0.0, 2.0, 1.0], [2.0, 0.0, 3.0], [1.0, 3.0, 0.0]])
    sc = O.data_scalars(X)
    assert sc["normsq"] == 2 * (4 + 1 + 9)
    assert sc["zeta"] == 12.0 / 9.0
    assert sc["maxval"] == 3.0
    assert np.array_equal(sc["rowsum"], [3.0, 5.0, 4.0])
    scs = O.data_scalars(sp.csr_matrix(X))
    assert scs["normsq"] == sc["normsq"] and scs["zeta"] == sc["zeta"] and scs["maxval"] == 3.0


def test_initial_factor_range_and_scale():
    zeta, k = 0.37, 8
    H = O.initial_factor(5000, k, zeta, seed=9)
    top = 2.0 * np.sqrt(zeta / k)
    assert H.min() >= 0 and H.max() < top
    assert abs(H.mean() / (top / 2) - 1.0) < 0.01


# --------------------------------------------------------------------------
# HALS.
# --------------------------------------------------------------------------

def test_hals_three_forms_agree():
    # eq. symhals_update1 (explicit R_i), eq. symhals_update2 (efficient) and
    # the Update(G, Y) form are the same sweep (Appendix A derivation).
    rng = np.random.default_rng(0)
    n, k, alpha = 50, 4, 0.7
    A = rng.uniform(size=(n, n))
    X = A + A.T
    W = rng.uniform(size=(n, k))
    H = rng.uniform(size=(n, k))
    w1 = O.hals_explicit(X, W, H, alpha)
    w2 = O.hals_symmetric(X @ H, H, W, alpha)
    w3 = O.hals_gy(H.T @ H + alpha * np.eye(k), X @ H + alpha * H, W)
    assert np.allclose(w1, w2, rtol=1e-13, atol=1e-13)
    assert np.allclose(w2, w3, rtol=1e-13, atol=1e-13)


def test_hals_rank_one_closed_form():
    # k = 1: the sweep is the nonnegative rank-one regularised solve
    # w = [(X h + alpha h) / (h^T h + alpha)]_+ , independent of the old w.
    rng = np.random.default_rng(1)
    n, alpha = 40, 2.5
    A = rng.standard_normal((n, n))
    X = A + A.T
    h = rng.uniform(size=(n, 1))
    w = O.hals_symmetric(X @ h, h, rng.uniform(size=(n, 1)), alpha)
    expect = np.maximum((X @ h[:, 0] + alpha * h[:, 0]) / (h[:, 0] @ h[:, 0] + alpha), 0)
    assert np.allclose(w[:, 0], expect, rtol=1e-14, atol=1e-14)
    assert (expect == 0).any()   # the projection is exercised


def test_hals_columns_are_exact_coordinate_minimisers():
    # After its update, column i satisfies the KKT conditions of
    # min_{w_i >= 0} of the regularised objective with the other columns
    # fixed; check the last column (untouched afterwards) under several
    # column orders.
    rng = np.random.default_rng(2)
    n, k, alpha = 60, 5, 1.3
    A = rng.standard_normal((n, n))
    X = A + A.T
    H = rng.uniform(size=(n, k))
    W0 = rng.uniform(size=(n, k))
    for perm in [np.arange(k), np.roll(np.arange(k), 2), np.arange(k)[::-1]]:
        Hp, Wp = H[:, perm], W0[:, perm]
        G = Hp.T @ Hp + alpha * np.eye(k)
        Y = X @ Hp + alpha * Hp
        Wn = O.hals_symmetric(X @ Hp, Hp, Wp, alpha)
        g = Wn @ G[:, -1] - Y[:, -1]          # gradient / 2 w.r.t. the last column
        w = Wn[:, -1]
        scale = np.abs(Y[:, -1]).max()
        assert w.min() >= 0
        assert np.all(g[w > 0] == pytest.approx(0.0, abs=1e-12 * scale))
        assert np.all(g[w == 0] >= -1e-12 * scale)


def test_hals_planted_fixed_point():
    # X = H0 H0^T, W = H = H0: Y = H0 (G0 + alpha I), G = G0 + alpha I, so the
    # sweep and the exact NLS both return H0.
    X, H0 = workloads.planted(200, 5, noise=0.0, seed=3)
    alpha = X.max()
    G = H0.T @ H0 + alpha * np.eye(5)
    Y = X @ H0 + alpha * H0
    assert np.allclose(O.hals_symmetric(X @ H0, H0, H0, alpha), H0, rtol=1e-13, atol=1e-13)
    assert np.allclose(O.nls_gy(G, Y), H0, rtol=1e-12, atol=1e-12)
    assert np.allclose(O.nls_gy(G, Y, method="lh"), H0, rtol=1e-10, atol=1e-10)


# --------------------------------------------------------------------------
# Exact NLS (the result BPP computes).
# --------------------------------------------------------------------------

def _random_gy(n, k, seed, alpha=0.5):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((3 * k, k))
    G = A.T @ A + alpha * np.eye(k)
    Y = rng.standard_normal((n, k)) * 2.0
    return G, Y


def test_nls_brute_force_equals_lawson_hanson():
    for k in (1, 3, 6, 8):
        G, Y = _random_gy(200, k, seed=k)
        xb = O.nls_gy(G, Y, method="brute")
        xl = O.nls_gy(G, Y, method="lh")
        assert np.allclose(xb, xl, rtol=1e-9, atol=1e-10)


def test_nls_kkt():
    for k, method in ((8, "brute"), (24, "lh")):
        G, Y = _random_gy(300, k, seed=100 + k)
        X = O.nls_gy(G, Y, method=method)
        g = X @ G - Y
        ny = np.abs(Y).max()
        assert X.min() >= 0
        assert g.min() >= -1e-9 * ny
        assert np.abs(X * g).max() <= 1e-9 * ny * ny
        assert ((X > 0) & (X < 1e9)).any() and (X == 0).any()


# --------------------------------------------------------------------------
# Residual identity and ANLS behaviour.
# --------------------------------------------------------------------------

def test_residual_trace_identity():
    rng = np.random.default_rng(4)
    n, k = 120, 6
    A = rng.uniform(size=(n, n))
    X = A + A.T
    W = rng.uniform(size=(n, k))
    H = rng.uniform(size=(n, k))
    d = O.residual_direct(X, W, H)
    assert d == pytest.approx(np.linalg.norm(X - W @ H.T), rel=1e-13)
    t = O.residual_trace(float(np.sum(X * X)), W, H, X @ W)
    assert t == pytest.approx(d, rel=1e-10)
    Xs = sp.csr_matrix(np.where(X > 1.2, X, 0.0))
    assert O.residual_direct(Xs, W, H) == pytest.approx(np.linalg.norm(Xs.toarray() - W @ H.T), rel=1e-13)


def _surrogate(X, W, H, alpha):
    return np.linalg.norm(X - W @ H.T) ** 2 + alpha * np.linalg.norm(W - H) ** 2


@pytest.mark.parametrize("rule", ["hals", "nls"])
def test_anls_monotone(rule):
    # Each half-step is an exact (NLS) or coordinate-exact (HALS) block
    # minimisation of the surrogate, so it cannot increase it.
    X, _ = workloads.planted(150, 4, noise=0.05, seed=5)
    alpha = X.max()
    H0 = O.initial_factor(150, 4, X.mean(), seed=1)
    W, H = H0.copy(), H0.copy()
    f = _surrogate(X, W, H, alpha)
    I = np.eye(4)
    for _ in range(15):
        if rule == "hals":
            W = O.hals_symmetric(X @ H, H, W, alpha)
        else:
            W = O.nls_gy(H.T @ H + alpha * I, X @ H + alpha * H)
        f1 = _surrogate(X, W, H, alpha)
        assert f1 <= f * (1 + 1e-12)
        if rule == "hals":
            H = O.hals_symmetric(X @ W, W, H, alpha)
        else:
            H = O.nls_gy(W.T @ W + alpha * I, X @ W + alpha * W)
        f = _surrogate(X, W, H, alpha)
        assert f <= f1 * (1 + 1e-12)


def test_planted_convergence_noiseless():
    # Noiseless planted X = H0 H0^T: the method reaches a near-zero residual.
    X, H0 = workloads.planted(300, 5, noise=0.0, seed=6)
    alpha = X.max()
    Hi = O.initial_factor(300, 5, X.mean(), seed=2)
    W, H, hist = O.plain_symnmf(X, 5, alpha, Hi, 8000, rule="hals", target=1e-6)
    assert hist[-1] <= 1e-6
    assert O.residual_direct(X, W, H) / np.linalg.norm(X) <= 1.1e-6


def test_planted_noisy_reaches_noise_floor():
    X, H0 = workloads.planted(300, 5, noise=0.01, seed=7)
    floor = np.linalg.norm(X - H0 @ H0.T) / np.linalg.norm(X)
    Hi = O.initial_factor(300, 5, X.mean(), seed=3)
    W, H, hist = O.plain_symnmf(X, 5, X.max(), Hi, 400, rule="hals")
    assert hist[-1] <= floor + 1e-3


def test_stall_rule():
    s = O.StallRule(1e-4, 4)
    seq = [1.0, 0.5, 0.49995, 0.4999, 0.49985, 0.4998]
    out = [s(r) for r in seq]
    assert out == [False, False, False, False, False, True]
    s = O.StallRule(1e-4, 4)
    assert not any(s(r) for r in [1.0, 0.99995, 0.9999, 0.5, 0.49995])


def test_projected_gradient_zero_at_stationary_point():
    X, H0 = workloads.planted(100, 4, noise=0.0, seed=8)
    alpha = X.max()
    pg = O.projected_gradient_norm(X @ H0, X @ H0, H0, H0, alpha)
    assert pg <= 1e-9 * np.linalg.norm(X @ H0)
    H1 = H0 * 1.1
    assert O.projected_gradient_norm(X @ H1, X @ H1, H1, H1, alpha) > 1e-3


# --------------------------------------------------------------------------
# Randomized range finder / Apx-EVD / LAI.
# --------------------------------------------------------------------------

def test_rrf_exact_low_rank_reconstructs():
    rng = np.random.default_rng(10)
    n, r, l = 300, 6, 10
    B = rng.standard_normal((n, r))
    X = B @ np.diag([9, 7, 5, -3, 2, 1.5]) @ B.T / n
    Om = O.sketch_omega(n, l, seed=4)
    U, lam = O.apx_evd(lambda M: X @ M, Om, q=1)
    assert np.allclose(U.T @ U, np.eye(l), atol=1e-12)
    assert np.linalg.norm(U @ np.diag(lam) @ U.T - X) <= 1e-12 * np.linalg.norm(X)
    # eigenvalues: the nonzero ones equal those of eigh(X), sorted descending
    ev = np.linalg.eigh(X)[0]
    ev = ev[np.argsort(-ev)]
    nz = np.concatenate([ev[:5], ev[-1:]])          # five positive, one negative
    assert np.allclose(np.sort(lam[np.abs(lam) > 1e-9])[::-1], np.sort(nz)[::-1], rtol=1e-10)
    # eigenvectors of the two largest eigenvalues match eigh(X)'s up to the sign rule
    evals, evecs = np.linalg.eigh(X)
    for j, idx in enumerate(np.argsort(-evals)[:2]):
        v = evecs[:, idx]
        v = v * np.sign(v[np.argmax(np.abs(v))])
        assert np.allclose(U[:, j], v, atol=1e-10)


def test_qb_residual_identity_and_bounds():
    # ||QB - X||^2 = ||X||^2 - ||B||^2 for orthonormal Q (Appendix Ada-RRF),
    # and the Apx-EVD error is at most twice the QB error (Section 3.3).
    rng = np.random.default_rng(11)
    n, l = 250, 12
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = 0.8 ** np.arange(n)
    X = (V * d) @ V.T
    Q = O.rrf(lambda M: X @ M, O.sketch_omega(n, l, 5), q=1)
    Bm = Q.T @ X
    qb = np.linalg.norm(Q @ Bm - X)
    assert qb ** 2 == pytest.approx(np.linalg.norm(X) ** 2 - np.linalg.norm(Bm) ** 2, rel=1e-8)
    U, lam = O.apx_evd(lambda M: X @ M, O.sketch_omega(n, l, 5), q=1)
    evd = np.linalg.norm(U @ np.diag(lam) @ U.T - X)
    assert evd <= 2 * qb * (1 + 1e-12)
    # the best rank-l error is a lower bound
    assert qb >= np.sqrt(np.sum(d[l:] ** 2)) * (1 - 1e-12)


def test_ada_rrf_checks_and_special_cases():
    # Algorithm Ada-RRF: every reported check equals the QB residual formed
    # directly; an infinite tolerance stops at the second check; a tolerance
    # of -infinity runs q_max rounds and then spans the RRF basis with
    # q = q_max; an exact rank-r input (r <= l) is captured at once.
    rng = np.random.default_rng(12)
    n, l = 300, 14
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    d = 0.9 ** np.arange(n)
    X = (V * d) @ V.T
    nx = float(np.sum(X * X))
    Om = O.sketch_omega(n, l, 6)
    # residual checks against the direct formation ||Q Q^T X - X|| / ||X||
    Q0 = O._qr_positive(X @ Om)
    Q, rounds, res = O.ada_rrf(lambda M: X @ M, nx, Om, q_max=1, tol=-np.inf)
    assert rounds == 1 and len(res) == 1
    assert res[0] == pytest.approx(np.linalg.norm(Q0 @ (Q0.T @ X) - X) / np.sqrt(nx), rel=1e-9)
    # the first check is compared with +infinity, so even an infinite
    # tolerance stops only at the second check
    Q, rounds, res = O.ada_rrf(lambda M: X @ M, nx, Om, q_max=5, tol=np.inf)
    assert rounds == 1 and len(res) == 2
    Q, rounds, res = O.ada_rrf(lambda M: X @ M, nx, Om, q_max=3, tol=-np.inf)
    Qr = O.rrf(lambda M: X @ M, Om, 3)
    assert rounds == 3 and len(res) == 3
    assert np.linalg.norm(Q @ Q.T - Qr @ Qr.T) <= 1e-9
    # the residual of the best rank-l approximation bounds every check
    assert min(res) >= np.sqrt(np.sum(d[l:] ** 2) / nx) * (1 - 1e-12)
    # exact low rank: the first check is ~0, the second stops the loop
    r = 9
    Z = rng.random((n, r))
    Xl = Z @ Z.T
    nl = float(np.sum(Xl * Xl))
    Q, rounds, res = O.ada_rrf(lambda M: Xl @ M, nl, Om, q_max=6, tol=1e-3)
    assert rounds == 1 and len(res) == 2 and res[0] <= 1e-6
    assert np.linalg.norm(Q @ (Q.T @ Xl) - Xl) <= 1e-10 * np.linalg.norm(Xl)


def test_lai_equals_plain_when_input_is_low_rank():
    # X of exact rank <= l: U Lambda U^T = X, so LAI-SymNMF reproduces the
    # plain iteration.
    n, k, l = 200, 4, 8
    _, H0 = workloads.planted(n, k, noise=0.0, seed=12)
    X = H0 @ H0.T
    U, lam = O.apx_evd(lambda M: X @ M, O.sketch_omega(n, l, 6), q=1)
    Hi = O.initial_factor(n, k, X.mean(), 4)
    alpha = X.max()
    W1, H1, h1 = O.plain_symnmf(X, k, alpha, Hi, 20)
    W2, H2, h2 = O.lai_symnmf(U, lam, k, alpha, Hi, 20)
    assert np.allclose(H1, H2, rtol=1e-8, atol=1e-10)
    assert np.allclose(h1, h2, rtol=1e-7, atol=1e-9)


# --------------------------------------------------------------------------
# Leverage scores and hybrid sampling.
# --------------------------------------------------------------------------

def test_leverage_invariants():
    rng = np.random.default_rng(13)
    n, k = 400, 7
    A = rng.uniform(size=(n, k))
    lev = O.leverage_scores(A)
    assert lev.min() >= 0 and lev.max() <= 1 + 1e-12
    assert lev.sum() == pytest.approx(k, rel=1e-12)
    # thin-SVD basis gives the same scores; so does any invertible mixing
    Usvd = np.linalg.svd(A, full_matrices=False)[0]
    assert np.allclose(lev, np.sum(Usvd ** 2, axis=1), rtol=1e-10, atol=1e-14)
    M = rng.standard_normal((k, k)) + 3 * np.eye(k)
    assert np.allclose(lev, O.leverage_scores(A @ M), rtol=1e-9, atol=1e-14)
    E = np.zeros((n, k))
    E[:k] = np.eye(k)
    assert np.allclose(O.leverage_scores(E), np.r_[np.ones(k), np.zeros(n - k)], atol=1e-14)


def test_hybrid_sample_structure():
    n, k, s = 3000, 8, 400
    lev = workloads.skewed_scores(n, k, seed=14)
    tau = 1.0 / s
    rows, w, info = O.hybrid_sample(lev, k, s, tau, seed=5, half_iter=3)
    det = lev / k >= tau
    assert info["s_D"] == det.sum() and info["s_D"] > 0
    assert np.all(np.diff(rows) > 0)
    assert set(np.nonzero(det)[0]) <= set(rows)
    assert np.all(w[np.isin(rows, np.nonzero(det)[0])] == 1.0)
    assert info["counts"].sum() == s - info["s_D"]
    assert info["counts"][det].sum() == 0
    # tau = 0: every row is deterministic, S = I
    rows0, w0, info0 = O.hybrid_sample(lev, k, s, 0.0, seed=5, half_iter=3)
    assert np.array_equal(rows0, np.arange(n)) and np.all(w0 == 1.0) and info0["s_R"] == 0


def test_hybrid_sample_distribution_chi2():
    # Draw frequencies follow p~_i = w_i / W_R over the random rows.
    n, k, s = 50, 3, 20000
    lev = workloads.skewed_scores(n, k, seed=15, heavy=2)
    tau = 0.2
    rows, w, info = O.hybrid_sample(lev, k, s, tau, seed=8, half_iter=0)
    det = lev / k >= tau
    wq = np.floor(lev * 2.0 ** 40) * (~det)
    p = wq / wq.sum()
    cnt = info["counts"][~det]
    res = stats.chisquare(cnt, p[~det] * cnt.sum())
    assert res.pvalue > 1e-3


@pytest.mark.slow
def test_hybrid_sample_unbiased_gram():
    # E[H^T S^T S H] = H^T H over the random part (Section 5.2 uses
    # E||S H||^2 = ||H||^2 to justify the same alpha).
    rng = np.random.default_rng(16)
    n, k, s = 300, 3, 60
    H = rng.uniform(size=(n, k)) ** 3
    lev = O.leverage_scores(H)
    G = H.T @ H
    acc = np.zeros((k, k))
    acc2 = np.zeros((k, k))
    T = 3000
    for seed in range(T):
        rows, w, _ = O.hybrid_sample(lev, k, s, 1.0 / s, seed, 0)
        Gs = H[rows].T @ (w[:, None] * H[rows])
        acc += Gs
        acc2 += Gs * Gs
    mean = acc / T
    sd = np.sqrt(np.maximum(acc2 / T - mean ** 2, 0) / T)
    assert np.all(np.abs(mean - G) <= 5 * sd + 1e-12)


def test_lvs_with_tau_zero_is_plain():
    # tau = 0 keeps every row with weight 1: LvS-SymNMF reduces to the plain
    # regularised HALS iteration.
    X, _ = workloads.planted(120, 4, noise=0.02, seed=17)
    Xs = sp.csr_matrix(X)
    alpha = X.max()
    Hi = O.initial_factor(120, 4, X.mean(), 5)
    W1, H1, h1 = O.plain_symnmf(X, 4, alpha, Hi, 5)
    W2, H2, h2 = O.lvs_symnmf(Xs, 4, alpha, Hi, 5, s=60, tau=0.0, seed=1)
    assert np.allclose(H1, H2, rtol=1e-12, atol=1e-13)
    assert np.allclose(h1, h2, rtol=1e-10)


def test_lvs_sampled_operands_match_an_explicit_sketch():
    # Algorithm LvS-SymNMF with the hybrid S of Section 4.2 (eq. SH), built
    # here row by row from the draw list: one row e_i^T for each deterministic
    # row (p_i = l_i / k >= tau) and one row e_r^T / sqrt(s_R p_r) for every
    # random draw r (eq. lev_score_S, p_r = l_r / (k - theta)).  The sampled
    # NLS operands are G = H^T S^T S H + alpha I and Y = X S^T S H + alpha H,
    # and the new factor is the HALS sweep on them.  tau = 1/s gives both
    # kinds of rows and weights far from 1.
    rng = np.random.default_rng(21)
    n, k, s = 90, 4, 30
    H = rng.uniform(0.1, 1.0, size=(n, k)) ** 2
    H[[3, 17, 50, 71]] *= 9.0
    B = rng.uniform(size=(n, n))
    X = B + B.T
    W = rng.uniform(size=(n, k))
    alpha, tau = 0.7, 1.0 / s
    new, info = O.lvs_half_step(X, H, W, alpha, s, tau, seed=9, half_iter=5)
    # leverage scores from the SVD (eq. lev_score_def), not from a QR
    Uh = np.linalg.svd(H, full_matrices=False)[0]
    lev = np.sum(Uh * Uh, axis=1)
    assert np.allclose(info["lev"], lev, rtol=1e-12, atol=1e-15)
    lev = info["lev"]                 # the exact bits the draws were made from
    det = lev / k >= tau
    s_D = int(det.sum())
    assert 0 < s_D < s
    theta = float(lev[det].sum())
    s_R = s - s_D
    # draw j: r = floor(v_j W_R / 2^64) on the integer weights w_i =
    # floor(l_i 2^40) of the random rows; the row is the first whose running
    # sum of w exceeds r (linear scan)
    w = [0 if det[i] else int(np.floor(lev[i] * 2.0 ** 40)) for i in range(n)]
    W_R = sum(w)
    v = philox.u64_stream(9, s_R, 5, philox.TAG_SAMPLE)
    drawn = []
    for x in v:
        r = (int(x) * W_R) >> 64
        acc = 0
        for i in range(n):
            acc += w[i]
            if acc > r:
                drawn.append(i)
                break
    assert len(drawn) == s_R
    S = np.zeros((s_D + s_R, n))
    for j, i in enumerate(np.nonzero(det)[0]):
        S[j, i] = 1.0
    for j, i in enumerate(drawn):
        S[s_D + j, i] = 1.0 / np.sqrt(s_R * lev[i] / (k - theta))
    SH = S @ H
    G = SH.T @ SH + alpha * np.eye(k)
    Y = X @ (S.T @ SH) + alpha * H
    assert np.abs(np.diag(S.T @ S) - 1.0).max() > 0.5       # weights really differ from 1
    assert np.linalg.norm(info["G"] - G) <= 1e-8 * np.linalg.norm(G)
    assert np.linalg.norm(info["Y"] - Y) <= 1e-8 * np.linalg.norm(Y)
    assert np.allclose(new, O.hals_gy(G, Y, W), rtol=1e-8, atol=1e-10)


def test_sampled_nls_error_shrinks_with_samples():
    # Theorem 1 flavour: the leverage-sampled NLS solution approaches the
    # exact one as s grows (median over trials).
    rng = np.random.default_rng(18)
    m, k, alpha = 2000, 4, 1e-3
    A = rng.uniform(size=(m, k)) ** 2
    b = A @ rng.uniform(size=(k, 3)) + 0.1 * rng.standard_normal((m, 3))
    G = A.T @ A + alpha * np.eye(k)
    xstar = O.nls_gy(G, (A.T @ b).T + 0.0)
    lev = O.leverage_scores(A)
    errs = []
    for s in (40, 400, 4000):
        e = []
        for t in range(30):
            rows, w, _ = O.hybrid_sample(lev, k, s, 1.0 / s, 100 + t, 0)
            Gs = A[rows].T @ (w[:, None] * A[rows]) + alpha * np.eye(k)
            Ys = (A[rows].T @ (w[:, None] * b[rows])).T
            e.append(np.linalg.norm(O.nls_gy(Gs, Ys) - xstar) / np.linalg.norm(xstar))
        errs.append(np.median(e))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05


# --------------------------------------------------------------------------
# PGNCG (Section 2.1.3; Algorithm LAI-PGNCG-SymNMF).
# --------------------------------------------------------------------------

def _vec(A):
    return A.reshape(-1, order="F")


def _explicit_jacobian(H):
    """J = -(H kron I_n) - K (H kron I_n) with K the perfect shuffle
    (K vec(A) = vec(A^T) for n x n A), as written in Section 2.1.3."""
    n, k = H.shape
    HI = np.kron(H, np.eye(n))
    K = np.zeros((n * n, n * n))
    for i in range(n):
        for j in range(n):
            K[j + n * i, i + n * j] = 1.0
    return -HI - K @ HI


def _sym(n, seed):
    A = np.random.default_rng(seed).random((n, n))
    return A + A.T


def test_pgncg_operators_match_kronecker_jacobian_and_calculus():
    # gn_normal_apply and gn_gradient against (a) the paper's Kronecker form of
    # J and (b) central differences of r(H) = vec(X - H H^T), which are exact
    # for a quadratic.  A dropped term (P^T H), a transposed Gram or a wrong
    # sign in either fails.
    n, k = 5, 3
    rng = np.random.default_rng(0)
    X = _sym(n, 1)
    H = rng.random((n, k))
    P = rng.standard_normal((n, k))
    J = _explicit_jacobian(H)
    h = 1e-3
    Jfd = np.empty_like(J)
    for c in range(n * k):
        E = np.zeros(n * k)
        E[c] = h
        Ep = E.reshape((n, k), order="F")
        Jfd[:, c] = (_vec(X - (H + Ep) @ (H + Ep).T) - _vec(X - (H - Ep) @ (H - Ep).T)) / (2 * h)
    assert np.allclose(J, Jfd, rtol=0, atol=1e-10)
    r = _vec(X - H @ H.T)
    assert np.allclose(_vec(O.gn_normal_apply(H, P)), J.T @ (J @ _vec(P)), rtol=1e-12, atol=1e-12)
    assert np.allclose(_vec(O.gn_gradient(X @ H, H)), J.T @ r, rtol=1e-12, atol=1e-12)


def test_pgncg_direction_is_the_gauss_newton_step():
    # With enough CG steps the direction is the minimum-norm least-squares
    # solution of J z = r, i.e. the Gauss-Newton step -z of min ||J p + r||.
    n, k = 6, 2
    rng = np.random.default_rng(2)
    X = _sym(n, 3)
    H = rng.random((n, k)) + 0.2
    J = _explicit_jacobian(H)
    z = np.linalg.lstsq(J, _vec(X - H @ H.T), rcond=None)[0]
    Z = O.gn_direction(X @ H, H, 60)
    assert np.linalg.norm(_vec(Z) - z) <= 1e-8 * np.linalg.norm(z)
    # one CG step is the steepest-descent step with the exact line search
    g = O.gn_gradient(X @ H, H)
    a = np.sum(g * g) / np.sum(g * O.gn_normal_apply(H, g))
    assert np.allclose(O.gn_direction(X @ H, H, 1), a * g, rtol=1e-13, atol=0)


def test_pgncg_zero_residual_converges_quadratically():
    # X = H* H*^T with H* > 0: Gauss-Newton on a zero-residual problem
    # converges quadratically from a nearby positive start, the projection
    # inactive (the residual roughly squares each iteration).
    n, k = 30, 3
    rng = np.random.default_rng(4)
    Hs = 0.5 + rng.random((n, k))
    X = Hs @ Hs.T
    H0 = Hs * (1.0 + 0.05 * rng.standard_normal((n, k)))
    H, hist = O.plain_pgncg(X, H0, 3, 10)
    rfin = O.residual_direct(X, H, H) / np.linalg.norm(X)
    assert hist[0] > 1e-2 and hist[1] < 1e-3 and hist[2] < 1e-6 and rfin < 1e-10
    # the logged entry t is the residual of the factor iteration t starts from
    assert hist[0] == pytest.approx(O.residual_direct(X, H0, H0) / np.linalg.norm(X), rel=1e-10)


def test_lai_pgncg_with_a_full_basis_is_plain_pgncg():
    # U Lambda U^T = X exactly when U holds all n eigenvectors
    n, k = 40, 3
    X, _ = workloads.gaussian_kernel(n, 6, 3, seed=5, dtype=np.float64)
    lam, U = np.linalg.eigh(X)
    H0 = O.initial_factor(n, k, O.data_scalars(X)["zeta"], seed=6)
    Hp, hp = O.plain_pgncg(X, H0, 6, 4)
    Hl, hl = O.lai_pgncg(U, lam, H0, 6, 4)
    assert np.allclose(Hl, Hp, rtol=1e-9, atol=1e-12) and np.allclose(hl, hp, rtol=1e-9)
    assert hp[-1] < hp[0]
