"""FP64 oracle of the learned warm start (test infrastructure only).

The paper starts every run from a random H (Section 5, experimental setup)
and names SVD-based starts only as an alternative.  This project adds a
learned start built on the LAI basis of Section 3: a small MLP maps features
of each entry of H, taken from the spectral embedding of its row and column
(plus the row's log degree), to a nonnegative initial value; the result is
scaled to fit X, and the ordinary iterations continue from it.
Nothing here is in the paper; the definitions below are this project's, and
the HIP library implements the same definitions independently.

Definitions
-----------
entries    the network runs once per entry (i, j) of H, j < k, with weights
           shared by all columns (the LAI basis and the columns of a
           converged H are both arbitrary in order and rotation from one
           instance to the next, so only a column-shared map transfers).
features   with c_j = sqrt(n) U[:, j] (U the n x l LAI basis, eigenvalues
           descending), s_j = +1 when ||max(c_j, 0)|| >= ||max(-c_j, 0)||
           else -1, a_ij = s_j c_ij, r_i = ||(c_i0, ..., c_i,k-1)||,
           m_i = max_{j<k} a_ij and d the row sums of X:
           f_ij = [a_ij, r_i, m_i, a_ij - m_i, lam_j / lam_0,
                   log(max(d_i / mean(d), 1e-6))]          (6 values)
           stored row-major over (i, j).
network    sizes [6, 64, 64, 64, 1]: h_1..h_3 = relu(h_{L-1} W_L + b_L),
           z = h_3 W_4 + b_4, output y = softplus(z) = log(1 + e^z).
           W_L is (in x out) row-major, b_L has `out` entries.
init       W_L = (2u - 1) sqrt(6 / in) with u the Philox uniforms of stream
           (seed, sub = L - 1, tag MLP), row-major order; b_L = 0.
loss       L = 1 / (2N) sum ||y - t||^2 over the N entries of a batch.
Adam       Kingma and Ba: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
           p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
start      Ht[i, j] = y_ij; H0 = W0 = beta Ht with
           beta^2 = tr(Ht^T X Ht) / ||Ht^T Ht||_F^2 (the least-squares
           multiple c of Ht Ht^T closest to X).
anchors    max(s_j c_j, 0) normalised, j < k (an NNDSVD-style nonnegative
           anchor, Boutsidis and Gallopoulos).
targets    a converged H* of the plain method, columns matched to the anchors
           by maximum total cosine (assignment problem), then divided by
           ||H*||_F / sqrt(n k); entry (i, j) of the result is the target of
           feature row f_ij.
"""
import itertools

import numpy as np
from scipy.optimize import linear_sum_assignment

from . import philox

TAG_MLP = 6
D_IN = 6
HIDDEN = 64
DEPTH = 3


def features(U, lam, rowsum, k):
    """(n k) x 6 feature rows, one per entry of H (definition above)."""
    U = np.asarray(U, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    n = U.shape[0]
    c = np.sqrt(n) * U[:, :k]
    s = np.array([1.0 if np.linalg.norm(np.maximum(c[:, j], 0.0)) >= np.linalg.norm(np.maximum(-c[:, j], 0.0))
                  else -1.0 for j in range(k)])
    a = c * s
    r = np.sqrt(np.sum(c * c, axis=1))
    m = a.max(axis=1)
    d = np.asarray(rowsum, dtype=np.float64)
    logd = np.log(np.maximum(d / d.mean(), 1e-6))
    F = np.empty((n, k, 6))
    F[:, :, 0] = a
    F[:, :, 1] = r[:, None]
    F[:, :, 2] = m[:, None]
    F[:, :, 3] = a - m[:, None]
    F[:, :, 4] = (lam[:k] / lam[0])[None, :]
    F[:, :, 5] = logd[:, None]
    return F.reshape(n * k, 6)


def anchors(U, k):
    """n x k nonnegative unit-norm anchors from the first k columns of U: the
    part (positive or negative) of larger norm."""
    U = np.asarray(U, dtype=np.float64)
    A = np.empty((U.shape[0], k))
    for j in range(k):
        p = np.maximum(U[:, j], 0.0)
        m = np.maximum(-U[:, j], 0.0)
        a = p if np.linalg.norm(p) >= np.linalg.norm(m) else m
        nrm = np.linalg.norm(a)
        A[:, j] = a / nrm if nrm > 0 else 0.0
    return A


def match_columns(A, H):
    """Permutation perm (column perm[j] of H goes to position j) maximising
    sum_j cos(A[:, j], H[:, perm[j]]), by the assignment problem."""
    C = _cosines(A, H)
    rows, cols = linear_sum_assignment(-C)
    perm = np.empty(A.shape[1], dtype=np.int64)
    perm[rows] = cols
    return perm


def match_columns_brute(A, H):
    """The same maximiser by enumerating every permutation (tiny k only)."""
    C = _cosines(A, H)
    k = C.shape[0]
    best, arg = -np.inf, None
    for p in itertools.permutations(range(k)):
        s = sum(C[j, p[j]] for j in range(k))
        if s > best:
            best, arg = s, p
    return np.array(arg, dtype=np.int64)


def _cosines(A, H):
    na = np.linalg.norm(A, axis=0)
    nh = np.linalg.norm(H, axis=0)
    na[na == 0] = 1.0
    nh[nh == 0] = 1.0
    return (A.T @ H) / np.outer(na, nh)


def targets(Hstar, U, k):
    """Training targets of one instance (definition above)."""
    H = np.asarray(Hstar, dtype=np.float64)
    n = H.shape[0]
    perm = match_columns(anchors(U, k), H)
    return H[:, perm] / (np.linalg.norm(H) / np.sqrt(n * k))


def scale_fit(XHt, Ht):
    """beta with beta^2 = tr(Ht^T X Ht) / ||Ht^T Ht||_F^2, given XHt = X Ht;
    None when that ratio is not positive."""
    Ht = np.asarray(Ht, dtype=np.float64)
    num = float(np.sum(Ht * XHt))
    G = Ht.T @ Ht
    den = float(np.sum(G * G))
    if not (num > 0.0 and den > 0.0):
        return None
    return np.sqrt(num / den)


# ----------------------------------------------------------------------------
# The network
# ----------------------------------------------------------------------------

def layer_sizes(d_in=D_IN, hidden=HIDDEN, out=1):
    return [d_in] + [hidden] * DEPTH + [out]


def init_params(sizes, seed):
    """List of (W, b) per layer (definition above)."""
    params = []
    for L in range(len(sizes) - 1):
        fan_in, fan_out = sizes[L], sizes[L + 1]
        u = philox.uniform(seed, fan_in * fan_out, L, TAG_MLP).reshape(fan_in, fan_out)
        params.append(((2.0 * u - 1.0) * np.sqrt(6.0 / fan_in), np.zeros(fan_out)))
    return params


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(params, X):
    """Returns (activations h_0 = X, h_1, ..., h_D; pre-activation z; y)."""
    h = [np.asarray(X, dtype=np.float64)]
    for W, b in params[:-1]:
        h.append(np.maximum(h[-1] @ W + b, 0.0))
    W, b = params[-1]
    z = h[-1] @ W + b
    return h, z, softplus(z)


def loss_and_grads(params, X, T):
    """Loss of the batch and its gradient for every (W, b), by backprop."""
    h, z, y = forward(params, X)
    N = X.shape[0]
    diff = y - np.asarray(T, dtype=np.float64)
    loss = 0.5 * float(np.sum(diff * diff)) / N
    dz = diff * sigmoid(z) / N
    grads = [None] * len(params)
    for L in range(len(params) - 1, -1, -1):
        W, _ = params[L]
        grads[L] = (h[L].T @ dz, dz.sum(axis=0))
        if L > 0:
            dz = (dz @ W.T) * (h[L] > 0.0)
    return loss, grads


def loss_only(params, X, T):
    _, _, y = forward(params, X)
    diff = y - np.asarray(T, dtype=np.float64)
    return 0.5 * float(np.sum(diff * diff)) / X.shape[0]


class Adam:
    """Adam state for a parameter list (definition above)."""

    def __init__(self, params, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for L, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for i, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[L][i] + (1.0 - self.b1) * g
                v = self.b2 * self.v[L][i] + (1.0 - self.b2) * g * g
                self.m[L] = (m, self.m[L][1]) if i == 0 else (self.m[L][0], m)
                self.v[L] = (v, self.v[L][1]) if i == 0 else (self.v[L][0], v)
                new.append(p - self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append((new[0], new[1]))
        return out


def predict(params, F):
    """Network output for the feature rows F (one value per row)."""
    return forward(params, F)[2]


def warm_start(params, U, lam, rowsum, k, X_apply):
    """H0 of the learned start: the network on every entry, then the scale
    fit against X (X_apply(B) = X B).  None when the fit is not positive."""
    n = U.shape[0]
    Ht = predict(params, features(U, lam, rowsum, k)).reshape(n, k)
    beta = scale_fit(X_apply(Ht), Ht)
    return None if beta is None else beta * Ht
