"""Pins of the warm-start oracle (oracle/warmstart.py) against facts that do
not restate its code: central finite differences for every gradient, Adam's
closed-form behaviour under a constant gradient and its scale invariance,
softplus limits, brute-force minimisation for the scale fit, brute-force
enumeration of permutations for the column matching, and the algebraic
properties of features, anchors and targets."""
import numpy as np
import pytest

from oracle import philox
from oracle import warmstart as WS


def _random_params(sizes, rng, scale=0.7):
    return [(rng.standard_normal((a, b)) * scale, rng.standard_normal(b) * 0.3)
            for a, b in zip(sizes[:-1], sizes[1:])]


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    sizes = [4, 6, 5, 6, 3]
    params = _random_params(sizes, rng)
    X = rng.standard_normal((5, 4))
    T = np.abs(rng.standard_normal((5, 3)))
    _, grads = WS.loss_and_grads(params, X, T)
    h = 1e-6
    for L, (W, b) in enumerate(params):
        for which, P in ((0, W), (1, b)):
            fd = np.zeros_like(P)
            for idx in np.ndindex(P.shape):
                orig = P[idx]
                P[idx] = orig + h
                lp = WS.loss_only(params, X, T)
                P[idx] = orig - h
                lm = WS.loss_only(params, X, T)
                P[idx] = orig
                fd[idx] = (lp - lm) / (2 * h)
            g = grads[L][which]
            assert np.linalg.norm(g - fd) <= 1e-7 * max(np.linalg.norm(fd), 1e-12) + 1e-10, (L, which)


def test_gradient_of_input_layer_sees_relu_mask():
    # a unit that is off for every row gets exactly zero gradient
    rng = np.random.default_rng(1)
    sizes = [3, 4, 4, 4, 2]
    params = _random_params(sizes, rng)
    W, b = params[0]
    b = b.copy()
    b[2] = -1e3
    params[0] = (W, b)
    X = rng.standard_normal((6, 3))
    _, grads = WS.loss_and_grads(params, X, np.ones((6, 2)))
    assert np.all(grads[0][0][:, 2] == 0.0) and grads[0][1][2] == 0.0


def test_softplus_limits_and_derivative():
    assert WS.softplus(0.0) == pytest.approx(np.log(2.0), rel=1e-15)
    assert WS.softplus(50.0) == pytest.approx(50.0, rel=1e-15)
    assert WS.softplus(-50.0) == pytest.approx(np.exp(-50.0), rel=1e-12)
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (WS.softplus(z + h) - WS.softplus(z - h)) / (2 * h)
    assert np.max(np.abs(fd - WS.sigmoid(z))) <= 1e-9


def test_adam_constant_gradient_moves_by_lr_per_step():
    # with a constant gradient the bias-corrected moments equal g and g^2,
    # so every step moves each parameter by lr * g / (|g| + eps)
    rng = np.random.default_rng(2)
    params = [(rng.standard_normal((3, 2)), rng.standard_normal(2))]
    g = [(rng.standard_normal((3, 2)), rng.standard_normal(2))]
    opt = WS.Adam(params, lr=0.01)
    p = params
    for _ in range(7):
        p = opt.step(p, g)
    for (W0, b0), (W1, b1), (gW, gb) in zip(params, p, g):
        assert np.allclose(W1, W0 - 7 * 0.01 * gW / (np.abs(gW) + 1e-8), rtol=0, atol=1e-13)
        assert np.allclose(b1, b0 - 7 * 0.01 * gb / (np.abs(gb) + 1e-8), rtol=0, atol=1e-13)


def test_adam_is_invariant_to_gradient_scale():
    rng = np.random.default_rng(3)
    params = [(rng.standard_normal((4, 3)), rng.standard_normal(3))]
    seq = [[(rng.standard_normal((4, 3)), rng.standard_normal(3))] for _ in range(5)]
    a = WS.Adam(params, lr=0.003, eps=0.0)
    b = WS.Adam(params, lr=0.003, eps=0.0)
    pa, pb = params, params
    for g in seq:
        pa = a.step(pa, g)
        pb = b.step(pb, [(1000.0 * gW, 1000.0 * gb) for gW, gb in g])
    assert np.allclose(pa[0][0], pb[0][0], rtol=0, atol=1e-12)
    assert np.allclose(pa[0][1], pb[0][1], rtol=0, atol=1e-12)


def test_init_params_follow_the_philox_stream():
    sizes = WS.layer_sizes()
    assert sizes == [6, 64, 64, 64, 1]
    params = WS.init_params(sizes, seed=11)
    for L, (W, b) in enumerate(params):
        a = np.sqrt(6.0 / sizes[L])
        assert W.shape == (sizes[L], sizes[L + 1]) and np.all(b == 0.0)
        assert np.abs(W).max() <= a
        u = philox.uniform(11, W.size, L, WS.TAG_MLP)
        assert np.array_equal(W.ravel(), (2.0 * u - 1.0) * a)
        # uniform on [-a, a]: variance a^2 / 3 (checked where the sample is large)
        if W.size >= 1000:
            assert abs(W.var() / (a * a / 3.0) - 1.0) < 0.1


def test_scale_fit_is_the_least_squares_multiple():
    rng = np.random.default_rng(4)
    n, k = 60, 4
    Ht = np.abs(rng.standard_normal((n, k)))
    M = np.abs(rng.standard_normal((n, n)))
    X = M + M.T
    beta = WS.scale_fit(X @ Ht, Ht)
    S = Ht @ Ht.T
    # golden-section search of ||X - c S||^2 over c, with no use of the formula
    lo, hi = 0.0, 10.0 * np.abs(X).max() / max(S.max(), 1e-300)
    f = lambda c: np.sum((X - c * S) ** 2)
    gr = (np.sqrt(5) - 1) / 2
    for _ in range(200):
        c1, c2 = hi - gr * (hi - lo), lo + gr * (hi - lo)
        if f(c1) < f(c2):
            hi = c2
        else:
            lo = c1
    # (a comparison search resolves the minimiser to about sqrt(eps) relative)
    assert beta * beta == pytest.approx(0.5 * (lo + hi), rel=1e-6)
    # an exact multiple is recovered
    assert WS.scale_fit((2.5 * S) @ Ht, Ht) ** 2 == pytest.approx(2.5, rel=1e-13)
    assert WS.scale_fit(-S @ Ht, Ht) is None


@pytest.mark.parametrize("k", [3, 5, 6])
def test_column_matching_equals_brute_force(k):
    rng = np.random.default_rng(k)
    A = np.abs(rng.standard_normal((40, k)))
    H = np.abs(rng.standard_normal((40, k)))
    assert np.array_equal(WS.match_columns(A, H), WS.match_columns_brute(A, H))
    # a permuted, lightly perturbed copy is matched back to its source columns
    p = rng.permutation(k)
    Hp = A[:, p] * (1.0 + 0.01 * rng.random((40, k)))
    perm = WS.match_columns(A, Hp)
    assert np.array_equal(p[perm], np.arange(k))


def test_features_anchors_and_targets():
    rng = np.random.default_rng(5)
    n, l, k = 50, 8, 3
    U, _ = np.linalg.qr(rng.standard_normal((n, l)))
    lam = np.array([4.0, 2.0, 1.0, 0.5, 0.1, 0.0, -0.1, -0.2])
    d = np.full(n, 3.0)
    F = WS.features(U, lam, d, k).reshape(n, k, 6)
    a = F[:, :, 0]
    # each column of a is sqrt(n) times a unit vector, signed to its larger part
    assert np.allclose((a ** 2).sum(axis=0), n)
    assert np.all(np.linalg.norm(np.maximum(a, 0), axis=0) >= np.linalg.norm(np.maximum(-a, 0), axis=0))
    assert np.allclose(np.abs(a), np.sqrt(n) * np.abs(U[:, :k]))
    assert np.allclose(F[:, 0, 1] ** 2, (a ** 2).sum(axis=1))           # row norm
    assert np.allclose(F[:, :, 2], a.max(axis=1, keepdims=True))        # row max
    assert np.all(F[:, :, 3] <= 0) and np.all(F[:, :, 3].max(axis=1) == 0)
    assert np.allclose(F[0, :, 4], [1.0, 0.5, 0.25])
    assert np.all(F[:, :, 5] == 0.0)                                    # constant degree -> log 1
    d2 = d.copy()
    d2[0] = 0.0                                                          # isolated vertex: clamped log
    assert WS.features(U, lam, d2, k)[0, 5] == pytest.approx(np.log(1e-6))
    u = np.array([1.0, 1.0, -3.0, 0.0])
    A = WS.anchors(u[:, None], 1)
    assert np.allclose(A[:, 0], [0, 0, 1, 0])               # the larger (negative) part
    A = WS.anchors(U, k)
    assert np.all(A >= 0) and np.allclose(np.linalg.norm(A, axis=0), 1.0)
    # the anchors are the normalised positive parts of the signed features
    assert np.allclose(A, np.maximum(a, 0) / np.linalg.norm(np.maximum(a, 0), axis=0))
    H = np.abs(rng.standard_normal((n, k)))
    T = WS.targets(H, U, k)
    assert np.linalg.norm(T) == pytest.approx(np.sqrt(n * k), rel=1e-13)
    # the targets do not depend on the column order of H*
    assert np.allclose(WS.targets(H[:, [2, 0, 1]], U, k), T, rtol=0, atol=1e-14)


def test_warm_start_recovers_an_exact_multiple():
    # if X is exactly c Ht Ht^T for the network's own output, the start is
    # sqrt(c) Ht whatever the network
    rng = np.random.default_rng(6)
    n, l, k = 40, 7, 3
    U, _ = np.linalg.qr(rng.standard_normal((n, l)))
    lam = np.linspace(3.0, 0.5, l)
    d = rng.random(n) + 0.5
    params = WS.init_params(WS.layer_sizes(), 3)
    Ht = WS.predict(params, WS.features(U, lam, d, k)).reshape(n, k)
    X = 2.25 * Ht @ Ht.T
    H0 = WS.warm_start(params, U, lam, d, k, lambda B: X @ B)
    assert np.allclose(H0, 1.5 * Ht, rtol=1e-12, atol=0)
