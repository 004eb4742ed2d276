"""GPU parity of the learned warm start against the FP64 oracle
(oracle/warmstart.py), through the C ABI: initialisation, forward pass,
gradients, Adam steps, entry features, the scaled start, the fallback, and a
test that a network trained on the GPU shortens the way to the target
residual compared with the random start."""
import os

import numpy as np
import pytest

from oracle import symnmf as O
from oracle import warmstart as WS
import workloads

from gpu_common import P, torch, require_gpu, dev, host, rel, factor, round_to, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def _unflat(v, sizes=None):
    sizes = sizes or WS.layer_sizes()
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = v[o:o + a * b].reshape(a, b)
        o += a * b
        out.append((W, v[o:o + b]))
        o += b
    return out


def _params(net):
    p = torch.empty(P.symnmf_mlp_num_params(net), dtype=torch.float32, device="cuda")
    P.symnmf_mlp_get_params(net, p)
    return host(p)


def _random_features(rows, seed):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((rows, 6))
    F[:, 4] = rng.random(rows)
    return round_to(F, torch.float32)


def _trained_like(seed):
    """Parameters with some dead units and non-trivial biases (FP32 values)."""
    rng = np.random.default_rng(seed)
    ps = WS.init_params(WS.layer_sizes(), seed)
    ps = [(W, rng.standard_normal(W.shape[1]) * 0.3) for W, _ in ps]
    return _unflat(round_to(_flat(ps), torch.float32))


def test_mlp_init_matches_oracle():
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 17)
    assert P.symnmf_mlp_num_params(net) == 8833
    ref = round_to(_flat(WS.init_params(WS.layer_sizes(), 17)), torch.float32)
    assert np.array_equal(_params(net), ref)


def test_mlp_save_and_load(tmp_path):
    """A saved network loads back with the same parameters and outputs; files
    that are not the library's format are refused."""
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 3)
    P.symnmf_mlp_set_params(net, dev(_flat(_trained_like(8)), torch.float32))
    path = str(tmp_path / "net.bin")
    P.symnmf_mlp_save(net, path)
    assert os.path.getsize(path) == 24 + 4 * 8833
    back = P.symnmf_mlp_load(path)
    assert np.array_equal(_params(back), _params(net))
    F = dev(_random_features(999, 5), torch.float32)
    Y1 = torch.empty(999, dtype=torch.float32, device="cuda")
    Y2 = torch.empty_like(Y1)
    P.symnmf_mlp_forward(net, F, Y1)
    P.symnmf_mlp_forward(back, F, Y2)
    assert torch.equal(Y1, Y2)
    raw = open(path, "rb").read()
    for bad in (raw[:-4], raw + b"\0", b"XYMNMLP1" + raw[8:]):
        p2 = str(tmp_path / "bad.bin")
        open(p2, "wb").write(bad)
        with pytest.raises(P.SymNMFError) as e:
            P.symnmf_mlp_load(p2)
        assert e.value.code == P.E_INVALID
    with pytest.raises(P.SymNMFError):
        P.symnmf_mlp_load(str(tmp_path / "missing.bin"))


@pytest.mark.parametrize("rows", [1, 257, 5000])
def test_mlp_forward_parity(rows):
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 3)
    ps = _trained_like(4)
    P.symnmf_mlp_set_params(net, dev(_flat(ps), torch.float32))
    F = _random_features(rows, rows)
    Y = torch.empty(rows, dtype=torch.float32, device="cuda")
    P.symnmf_mlp_forward(net, dev(F, torch.float32), Y)
    yo = WS.predict(ps, F).ravel()
    assert rel(host(Y), yo) <= 1e-5


def test_mlp_gradient_parity():
    rows = 3001                    # several blocks, entry ranges with a ragged tail
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 5)
    ps = _trained_like(6)
    P.symnmf_mlp_set_params(net, dev(_flat(ps), torch.float32))
    F = _random_features(rows, 7)
    T = round_to(np.abs(np.random.default_rng(8).standard_normal(rows)), torch.float32)
    g = torch.empty(P.symnmf_mlp_num_params(net), dtype=torch.float32, device="cuda")
    loss = P.symnmf_mlp_gradient(net, dev(F, torch.float32), dev(T, torch.float32), g)
    lo, go = WS.loss_and_grads(ps, F, T[:, None])
    assert loss == pytest.approx(lo, rel=1e-6)
    gg = _unflat(host(g))
    for L, ((gW, gb), (oW, ob)) in enumerate(zip(gg, go)):
        log(f"grad layer {L}: W {rel(gW, oW):.2e} b {rel(gb, ob):.2e}")
        assert rel(gW, oW) <= 1e-4 and rel(gb, ob) <= 1e-4


def test_mlp_adam_steps_parity():
    rows = 2048
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 9)
    p0 = _unflat(round_to(_flat(WS.init_params(WS.layer_sizes(), 9)), torch.float32))
    F = _random_features(rows, 10)
    T = round_to(np.abs(np.random.default_rng(11).standard_normal(rows)), torch.float32)
    Fd, Td = dev(F, torch.float32), dev(T, torch.float32)
    opt = WS.Adam(p0, lr=1e-3)
    po = p0
    for _ in range(5):
        P.symnmf_mlp_train_step(net, Fd, Td, 1e-3)
        _, go = WS.loss_and_grads(po, F, T[:, None])
        po = opt.step(po, go)
    pg = _params(net)
    moved = _flat(po) - _flat(p0)
    err = np.linalg.norm(pg - _flat(po)) / np.linalg.norm(moved)
    log(f"adam: deviation / displacement {err:.2e}")
    assert err <= 1e-3


def _lai_instance(n, k, l, q, seed, dtype=torch.float32):
    X, _ = workloads.gaussian_kernel(n, 2 * k, k, seed=seed, dtype=np.float64)
    X = round_to(X, dtype)
    ctx = P.symnmf_create(dev(X, dtype), k, 0.0, 0, seed)
    P.symnmf_lai(ctx, l, q)
    Uo, lo = O.apx_evd(lambda M: O.apply_x(X, M), O.sketch_omega(n, l, seed), q)
    return X, ctx, Uo, lo


def test_warm_features_parity():
    n, k, l, q = 1500, 16, 32, 2
    X, ctx, Uo, lo = _lai_instance(n, k, l, q, 3, torch.float64)
    F = torch.empty((n * k, 6), dtype=torch.float32, device="cuda")
    P.symnmf_warm_features(ctx, F)
    Fo = WS.features(Uo, lo, O.data_scalars(X)["rowsum"], k)
    Fg = host(F)
    for c in range(6):
        log(f"feature {c}: rel {rel(Fg[:, c], Fo[:, c]):.2e}")
        assert rel(Fg[:, c], Fo[:, c]) <= 1e-5


def test_warmstart_parity_and_scale():
    n, k, l, q = 1500, 16, 32, 2
    X, ctx, Uo, lo = _lai_instance(n, k, l, q, 4, torch.float64)
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 21)
    ps = _unflat(_params(net))
    beta = P.symnmf_warmstart(ctx, net)
    Ho = WS.warm_start(ps, Uo, lo, O.data_scalars(X)["rowsum"], k, lambda B: O.apply_x(X, B))
    Ht = WS.predict(ps, WS.features(Uo, lo, O.data_scalars(X)["rowsum"], k)).reshape(n, k)
    assert beta == pytest.approx(WS.scale_fit(O.apply_x(X, Ht), Ht), rel=1e-5)
    assert rel(factor(ctx, P.H), Ho) <= 1e-5 and rel(factor(ctx, P.W), Ho) <= 1e-5
    # the iterations continue from it (LAI mode, then the full X)
    P.symnmf_iterate(ctx, 3)
    P.symnmf_refine(ctx)
    P.symnmf_iterate(ctx, 3)
    assert np.isfinite(P.symnmf_residual(ctx, P.RESID_EXACT)[0])


def test_warmstart_keeps_random_start_when_the_fit_fails():
    # a network whose output underflows to zero: ||Ht^T Ht|| = 0, no scale
    # exists, and the random start is kept
    n, k, l = 600, 6, 16
    X, _ = workloads.gaussian_kernel(n, 8, 6, seed=2, dtype=np.float64)
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, 2)
    H0 = factor(ctx, P.H)
    P.symnmf_lai(ctx, l, 1)
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 1)
    v = np.zeros(P.symnmf_mlp_num_params(net))
    v[-1] = -200.0                                  # b4: softplus(-200) = 0 in FP32
    P.symnmf_mlp_set_params(net, dev(v, torch.float32))
    assert P.symnmf_warmstart(ctx, net) == 0.0
    assert np.array_equal(factor(ctx, P.H), H0) and np.array_equal(factor(ctx, P.W), H0)


def test_warmstart_requires_lai():
    X, _ = workloads.planted(200, 4, noise=0.01, seed=0)
    ctx = P.symnmf_create(dev(X), 4, 0.0, 0, 0)
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 1)
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_warmstart(ctx, net)
    assert e.value.code == P.E_STATE
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_mlp_create(32, 1)
    assert e.value.code == P.E_INVALID


def test_trained_network_shortens_the_solve():
    """Train on six instances on the GPU, then compare iterations to
    r* = r_conv + 1e-3 on two held-out instances: random start, the untrained
    network's start and the trained network's start."""
    from paper_2402_08134_amd import warmstart as WSP
    k, l, q = 16, 32, 2
    data = []
    for i in range(6):
        n = 1600 + 150 * i
        X, _ = workloads.gaussian_kernel(n, 2 * k, k, seed=200 + i, dtype=np.float32)
        F, T, it = WSP.instance_data(dev(X), k, l, q, seed=1)
        data.append((F, T))
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 7)
    untrained = P.symnmf_mlp_create(P.MLP_HIDDEN, 7)
    losses = WSP.train(net, data, epochs=10, lr=1e-3, batch=4096, seed=0)
    log(f"training losses {['%.4f' % v for v in losses]}")
    assert losses[-1] < losses[0]
    gains = []
    for j in range(2):
        n = 1900 + 300 * j
        X, _ = workloads.gaussian_kernel(n, 2 * k, k, seed=300 + j, dtype=np.float32)
        Xd = dev(X)
        o = P.symnmf_default_options(stop_mode=P.STOP_STALL, check_every=4)
        ref = P.symnmf_create(Xd, k, 0.0, 0, 5, o)
        P.symnmf_iterate(ref, 2000)
        r_star = P.symnmf_residual(ref, P.RESID_EXACT)[0] + 1e-3

        def iters_from(netw):
            o = P.symnmf_default_options(stop_mode=P.STOP_TARGET, target=r_star, check_every=1)
            c = P.symnmf_create(Xd, k, 0.0, 0, 5, o)
            if netw is not None:
                P.symnmf_lai(c, l, q)
                assert P.symnmf_warmstart(c, netw) > 0
                P.symnmf_refine(c, P.STOP_TARGET, r_star)
            return P.symnmf_iterate(c, 4000)

        it_r, it_u, it_t = iters_from(None), iters_from(untrained), iters_from(net)
        log(f"held-out n={n}: iterations to r*: random {it_r}, untrained net {it_u}, trained net {it_t}")
        gains.append((it_r, it_u, it_t))
    assert all(t < r for r, u, t in gains)
    assert sum(t for _, _, t in gains) < sum(u for _, u, _ in gains)
