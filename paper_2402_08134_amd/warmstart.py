"""Training and use of the learned warm start, over the C ABI.

The network, its features, its gradients and its Adam steps run in the
library (symnmf_mlp_*, symnmf_warm_features, symnmf_warmstart).  This module
only prepares training data on the host -- the converged factor of a plain
run, its columns matched to the spectral anchors (an assignment problem) and
rescaled -- shuffles it, and loops over batches.  PyTorch holds device
memory.

Targets of one instance: with c_j = U[:, j] (the LAI basis), the anchor of
column j is the part (positive or negative) of c_j with the larger norm,
normalised; the columns of the converged H* are permuted to maximise the
total cosine with the anchors, then H* is divided by ||H*||_F / sqrt(n k).
Entry (i, j) of the result is the target of feature row (i, j).
"""
import os

import numpy as np
from scipy.optimize import linear_sum_assignment

import paper_2402_08134_amd as P


def spectral_anchors(U, k):
    U = np.asarray(U, dtype=np.float64)[:, :k]
    pos = np.maximum(U, 0.0)
    neg = np.maximum(-U, 0.0)
    take_pos = np.linalg.norm(pos, axis=0) >= np.linalg.norm(neg, axis=0)
    A = np.where(take_pos[None, :], pos, neg)
    nrm = np.linalg.norm(A, axis=0)
    nrm[nrm == 0] = 1.0
    return A / nrm


def align_targets(H, U, k):
    """n x k targets (float32) of a converged factor H (host arrays)."""
    H = np.asarray(H, dtype=np.float64)
    n = H.shape[0]
    A = spectral_anchors(U, k)
    hn = np.linalg.norm(H, axis=0)
    hn[hn == 0] = 1.0
    cos = (A.T @ H) / hn[None, :]
    rows, cols = linear_sum_assignment(-cos)
    perm = np.empty(k, dtype=np.int64)
    perm[rows] = cols
    scale = np.linalg.norm(H) / np.sqrt(n * k)
    return (H[:, perm] / scale).astype(np.float32)


def instance_data(X, k, l, q, seed, max_iters=2000):
    """Features (device, (n k) x 6) and targets (host, n k) of one symmetric
    X (a dense device tensor, or a (row_ptr, col_idx, values, n) tuple of
    device tensors for CSR): plain run from the random start until the stall
    rule stops it, then the LAI basis of the same X."""
    import torch
    dense = not isinstance(X, tuple)
    n = X.shape[0] if dense else int(X[3])
    device = X.device if dense else X[0].device
    o = P.symnmf_default_options(stop_mode=P.STOP_STALL, check_every=8)
    ctx = P.symnmf_create(X, k, 0.0, 0, seed, o)
    iters = P.symnmf_iterate(ctx, max_iters)
    dt = torch.float64 if ctx.fdtype == P.F64 else torch.float32
    Hd = torch.empty((n, k), dtype=dt, device=device)
    P.symnmf_get_factor(ctx, P.H, Hd)
    P.symnmf_lai(ctx, l, q)
    U = torch.empty((n, l), dtype=torch.float64, device=device)
    P.symnmf_get_lai(ctx, U, None)
    F = torch.empty((n * k, P.MLP_FEATURES), dtype=torch.float32, device=device)
    P.symnmf_warm_features(ctx, F)
    torch.cuda.synchronize()
    T = align_targets(Hd.cpu().numpy(), U.cpu().numpy(), k).reshape(-1)
    return F, T, iters


def train(net, data, epochs, lr, batch, seed=0, log=None):
    """Adam over shuffled batches of entries pooled from every instance.
    data: list of (F device tensor, T host array).  Returns the mean loss of
    each epoch."""
    import torch
    dev = data[0][0].device
    Fh = np.concatenate([F.cpu().numpy() for F, _ in data])
    Th = np.concatenate([T for _, T in data]).astype(np.float32)
    rng = np.random.default_rng(seed)
    losses = []
    for ep in range(epochs):
        perm = rng.permutation(Fh.shape[0])
        Fd = torch.from_numpy(np.ascontiguousarray(Fh[perm])).to(dev)
        Td = torch.from_numpy(np.ascontiguousarray(Th[perm])).to(dev)
        tot, cnt = 0.0, 0
        for s in range(0, Fh.shape[0] - batch + 1, batch):
            loss = P.symnmf_mlp_train_step(net, Fd[s:s + batch], Td[s:s + batch], lr)
            tot += loss
            cnt += 1
        losses.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.5f}")
    return losses


def train_pooled(net, F, T, epochs, lr, batch, seed=0, log=None, lr_final=None):
    """Adam over shuffled batches of a pooled entry set (F: device (m, 6)
    FP32, T: device (m,) FP32); the step size goes geometrically from lr in
    the first epoch to lr_final (default lr) in the last.  Returns the mean
    loss of each epoch."""
    import torch
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    m = F.shape[0]
    losses = []
    lr_final = lr if lr_final is None else lr_final
    for ep in range(epochs):
        step = lr * (lr_final / lr) ** (ep / max(epochs - 1, 1))
        perm = torch.randperm(m, generator=g).to(F.device)
        Fs = F.index_select(0, perm).contiguous()
        Ts = T.index_select(0, perm).contiguous()
        tot, cnt = 0.0, 0
        for s in range(0, m - batch + 1, batch):
            tot += P.symnmf_mlp_train_step(net, Fs[s:s + batch], Ts[s:s + batch], step)
            cnt += 1
        losses.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.5f}")
        del Fs, Ts
    return losses


def save(net, path):
    """The network's parameters in the library's file format."""
    P.symnmf_mlp_save(net, path)


def load(path, stream=None):
    """A network from a file written by save (symnmf_mlp_load), or from the
    older .npz files (parameters array and hidden width)."""
    if not path.endswith(".npz"):
        return P.symnmf_mlp_load(path, stream)
    import torch
    z = np.load(path, allow_pickle=False)
    if int(z["hidden"]) != P.MLP_HIDDEN:
        raise ValueError(f"{path}: hidden width {int(z['hidden'])} is not supported")
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 0, stream)
    p = torch.from_numpy(z["params"].astype(np.float32)).cuda()
    P.symnmf_mlp_set_params(net, p)
    torch.cuda.synchronize()
    return net


WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
