"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds inputs (data matrices, starting factors, test
vectors).  It holds none of the factorisation's arithmetic and is shared by
the tests, the oracle checks and the benchmark.

Stand-ins (the paper's datasets are not available):
* dense similarity (the Web of Science hypergraph adjacency of Section 5.1 is
  a dense symmetric nonnegative similarity matrix): a Gaussian-kernel matrix
  of points drawn from a Gaussian mixture, zero diagonal;
* sparse graph (the normalised, zero-diagonal citation graph of Section 5.2):
  a stochastic block model, symmetrically normalised D^-1/2 A D^-1/2;
* planted: X = H0 H0^T + small symmetric noise with a block-dominant H0.
"""
import numpy as np
import scipy.sparse as sp


def planted(n=1000, k=10, noise=0.01, seed=0, block=None):
    """X = H0 H0^T + E.  H0[i, c] ~ U[0, 1] when c is row i's block
    (block = n // k rows each), else U[0, 0.1]; E = noise * |N(0, 1)| drawn for
    i <= j and mirrored.  FP64.  Returns (X, H0)."""
    rng = np.random.default_rng(seed)
    block = block or max(n // k, 1)
    H0 = rng.uniform(0.0, 0.1, size=(n, k))
    owner = np.minimum(np.arange(n) // block, k - 1)
    H0[np.arange(n), owner] = rng.uniform(0.0, 1.0, size=n)
    X = H0 @ H0.T
    if noise > 0:
        E = noise * np.abs(rng.standard_normal((n, n)))
        E = np.triu(E)
        E = E + np.triu(E, 1).T
        X = X + E
    X = 0.5 * (X + X.T)
    return X, H0


def gmm_points(n, dim, comps, seed):
    """Points of an equal-weight Gaussian mixture: means ~ N(0, 4 I), unit
    covariance."""
    rng = np.random.default_rng(seed)
    means = 2.0 * rng.standard_normal((comps, dim))
    lab = rng.integers(0, comps, size=n)
    P = means[lab] + rng.standard_normal((n, dim))
    return P, lab


def gaussian_kernel(n=16384, dim=64, comps=32, seed=0, dtype=np.float32, median_pairs=1 << 22):
    """X_ij = exp(-||x_i - x_j||^2 / median^2), zero diagonal, bitwise symmetric.

    median = lower median of the pairwise distances over i < j (exact up to
    n = 16384, else over `median_pairs` random pairs)."""
    P, lab = gmm_points(n, dim, comps, seed)
    sq = np.sum(P * P, axis=1)
    rng = np.random.default_rng(seed + 1)
    if n <= 16384:
        iu = np.triu_indices(n, 1) if n <= 4096 else None
        if iu is not None:
            D2 = np.maximum(sq[:, None] + sq[None, :] - 2.0 * (P @ P.T), 0.0)
            d2 = D2[iu]
        else:
            parts = []
            for r0 in range(0, n, 2048):
                blk = np.maximum(sq[r0:r0 + 2048, None] + sq[None, :] - 2.0 * (P[r0:r0 + 2048] @ P.T), 0.0)
                for r in range(blk.shape[0]):
                    i = r0 + r
                    parts.append(blk[r, i + 1:])
            d2 = np.concatenate(parts)
    else:
        i = rng.integers(0, n, size=median_pairs)
        j = rng.integers(0, n, size=median_pairs)
        keep = i != j
        i, j = i[keep], j[keep]
        d2 = np.maximum(np.sum((P[i] - P[j]) ** 2, axis=1), 0.0)
    m = (d2.shape[0] - 1) // 2
    med2 = float(np.partition(d2, m)[m])
    del d2
    X = np.empty((n, n), dtype=dtype)
    for r0 in range(0, n, 2048):
        blk = np.maximum(sq[r0:r0 + 2048, None] + sq[None, :] - 2.0 * (P[r0:r0 + 2048] @ P.T), 0.0)
        X[r0:r0 + 2048] = np.exp(-blk / med2).astype(dtype)
    # mirror the upper triangle so X is bitwise symmetric, then zero the diagonal
    for r0 in range(0, n, 2048):
        r1 = min(r0 + 2048, n)
        for c0 in range(0, r0, 2048):
            X[r0:r1, c0:c0 + 2048] = X[c0:c0 + 2048, r0:r1].T
        blk = X[r0:r1, r0:r1]
        low = np.tril_indices(r1 - r0, -1)
        blk[low] = blk.T[low]
    np.fill_diagonal(X, 0)
    return X, lab


def gpu_gaussian_kernel(n, dim, comps, seed, median_on_gpu=False):
    """The Gaussian-kernel similarity of gaussian_kernel (same points, same
    sampled-pairs median for n > 16384), formed on the GPU in FP64 blocks
    and stored as FP32 (a torch tensor on the GPU), bitwise symmetric, zero
    diagonal.  For sizes whose host copy would be too large.  With
    median_on_gpu the squared distances of the sampled pairs are formed and
    ranked on the GPU (same pairs and definition; the rounding of the
    distances may differ in the last bits)."""
    import torch
    Pp, _ = gmm_points(n, dim, comps, seed)
    rng = np.random.default_rng(seed + 1)
    i = rng.integers(0, n, size=1 << 22)
    j = rng.integers(0, n, size=1 << 22)
    keep = i != j
    if median_on_gpu:
        Pg = torch.from_numpy(Pp).cuda()
        ii = torch.from_numpy(i[keep]).cuda()
        jj = torch.from_numpy(j[keep]).cuda()
        d2g = torch.zeros(ii.shape[0], dtype=torch.float64, device="cuda")
        for c0 in range(0, dim, 16):
            d2g += ((Pg[ii, c0:c0 + 16] - Pg[jj, c0:c0 + 16]) ** 2).sum(1)
        d2g.clamp_min_(0.0)
        m = (d2g.shape[0] - 1) // 2
        med2 = float(torch.kthvalue(d2g, m + 1).values)
        del Pg, ii, jj, d2g
    else:
        d2 = np.maximum(np.sum((Pp[i[keep]] - Pp[j[keep]]) ** 2, axis=1), 0.0)
        m = (d2.shape[0] - 1) // 2
        med2 = float(np.partition(d2, m)[m])
    Pd = torch.from_numpy(Pp).cuda()
    sq = (Pd * Pd).sum(1)
    X = torch.empty((n, n), dtype=torch.float32, device="cuda")
    B = 8192
    for i0 in range(0, n, B):
        i1 = min(i0 + B, n)
        for j0 in range(i0, n, B):
            j1 = min(j0 + B, n)
            blk = sq[i0:i1, None] + sq[None, j0:j1] - 2.0 * (Pd[i0:i1] @ Pd[j0:j1].T)
            blk = torch.exp(-blk.clamp_min(0.0) / med2).float()
            if j0 == i0:
                up = torch.triu(blk)
                blk = up + torch.triu(blk, 1).T
            X[i0:i1, j0:j1] = blk
            if j0 != i0:
                X[j0:j1, i0:i1] = blk.T
    X.fill_diagonal_(0.0)
    torch.cuda.synchronize()
    return X


def sbm(n=1 << 20, blocks=64, avg_degree=32.0, ratio=20.0, seed=0):
    """Stochastic block model, equal contiguous blocks, simple undirected graph
    without self loops, X = D^-1/2 A D^-1/2 as CSR (int32 indices, FP32
    values, sorted columns).  p_in = ratio * p_out with the expected degree
    b p_in + (n - b) p_out = avg_degree (b = n / blocks).  Isolated vertices
    keep an empty row.  Edges are drawn as random pairs per block pair with
    Binomial counts and de-duplicated."""
    rng = np.random.default_rng(seed)
    b = n // blocks
    p_out = avg_degree / (ratio * (b - 1) + (n - b))
    p_in = ratio * p_out
    src, dst = [], []
    # within-block edges
    m_in = rng.binomial(b * (b - 1) // 2, min(p_in, 1.0), size=blocks)
    for B in range(blocks):
        u = rng.integers(0, b, size=m_in[B]) + B * b
        v = rng.integers(0, b, size=m_in[B]) + B * b
        src.append(u)
        dst.append(v)
    # cross-block edges: pairs (u, v) with different blocks
    cross_pairs = (n * n - blocks * b * b) // 2
    m_out = rng.binomial(cross_pairs, min(p_out, 1.0))
    u = rng.integers(0, n, size=int(m_out * 1.02) + 16)
    v = rng.integers(0, n, size=u.shape[0])
    keep = (u // b) != (v // b)
    src.append(u[keep][:m_out])
    dst.append(v[keep][:m_out])
    u = np.concatenate(src).astype(np.int64)
    v = np.concatenate(dst).astype(np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a, c = np.minimum(u, v), np.maximum(u, v)
    key = np.unique(a * n + c)
    a, c = key // n, key % n
    rows = np.concatenate([a, c])
    cols = np.concatenate([c, a])
    A = sp.csr_matrix((np.ones(rows.shape[0], dtype=np.float64), (rows, cols)), shape=(n, n))
    A.sum_duplicates()
    A.sort_indices()
    deg = np.asarray(A.sum(axis=1)).ravel()
    dinv = np.zeros(n)
    nz = deg > 0
    dinv[nz] = 1.0 / np.sqrt(deg[nz])
    Dm = sp.diags(dinv)
    X = (Dm @ A @ Dm).tocsr()
    X.sort_indices()
    X = sp.csr_matrix((X.data.astype(np.float32), X.indices.astype(np.int32), X.indptr.astype(np.int32)),
                      shape=(n, n))
    labels = np.arange(n) // b
    return X, labels


# Instances of the learned-start study: 2000 generated problems, ids 0..1799
# for training and 1800..1999 held out.  Instance i: a stochastic block model
# graph when i is even, a Gaussian-kernel similarity when i is odd;
# n uniform in [4096, 32768], k uniform in {16, 32, 64}.  SBM: k equal
# blocks, average degree 32, p_in / p_out = 20, X = D^-1/2 A D^-1/2.
# Gaussian kernel: k equal-weight components in R^(2k), FP32, median over
# 2^22 sampled pairs.
WARM_TRAIN_IDS = range(0, 1800)
WARM_HELD_OUT_IDS = range(1800, 2000)


def warm_instance(i):
    """Kind, n, k and data seed of instance i of the learned-start study."""
    rng = np.random.default_rng([20240208, int(i)])
    n = 4096 + int(rng.integers(0, 28673))
    k = (16, 32, 64)[int(rng.integers(0, 3))]
    return {"id": int(i), "kind": "sbm" if i % 2 == 0 else "gmm", "n": n, "k": k, "seed": 100000 + int(i)}


def warm_instance_data(spec):
    """The matrix of an instance: a scipy CSR (SBM) or a GPU tensor (Gaussian
    kernel, formed on the GPU)."""
    if spec["kind"] == "sbm":
        X, _ = sbm(spec["n"], spec["k"], 32.0, 20.0, seed=spec["seed"])
        return X
    return gpu_gaussian_kernel(spec["n"], 2 * spec["k"], spec["k"], spec["seed"], median_on_gpu=True)


def random_factor(n, k, seed, scale=1.0, zero_cols=()):
    """A nonnegative n x k matrix with U[0, scale) entries (optionally with
    some all-zero columns)."""
    rng = np.random.default_rng(seed)
    H = rng.uniform(0.0, scale, size=(n, k))
    for c in zero_cols:
        H[:, c] = 0.0
    return H


def skewed_scores(n, k, seed, heavy=8):
    """A positive length-n vector summing to k with a few large entries: the
    shape of leverage scores of a matrix with a handful of dominant rows.
    Used only as a sampler input."""
    rng = np.random.default_rng(seed)
    v = rng.pareto(1.5, size=n) + 0.05
    big = rng.choice(n, size=min(heavy, n), replace=False)
    v[big] *= n / (10.0 * heavy)
    v = v / v.sum() * k
    return np.minimum(v, 1.0)
