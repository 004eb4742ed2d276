"""FP64 oracle for randomized SymNMF (test infrastructure only).

Notation follows the paper: X is the symmetric m x m data matrix (here n x n),
k the rank, alpha the symmetric regulariser of the surrogate objective
(Section 2.1.1, eq. surrogate_symnmf_obj), W and H the two n x k factors.
The paper writes the product with the data as Y = H^T X (k x m); this oracle
keeps the transposed, row-major form Y = X H (n x k), which is the same data.

Every function cites the passage it follows.  Where the paper is silent the
reading used is stated in the docstring (the list of readings is kept with the
design notes of the project).
"""
import itertools

import numpy as np
import scipy.sparse as sp
from scipy.optimize import nnls

from . import philox

# ----------------------------------------------------------------------------
# Products with the data matrix.  X may be a dense ndarray (FP64 or FP32; FP32
# is upcast block by block, never in full) or a scipy CSR matrix.
# ----------------------------------------------------------------------------

_ROW_BLOCK = 4096


def apply_x(X, B):
    """Return X @ B in FP64 (X dense or CSR, B n x c)."""
    B = np.asarray(B, dtype=np.float64)
    if sp.issparse(X):
        return np.asarray(X @ B, dtype=np.float64)
    if X.dtype == np.float64:
        return X @ B
    out = np.empty((X.shape[0], B.shape[1]), dtype=np.float64)
    for r0 in range(0, X.shape[0], _ROW_BLOCK):
        out[r0:r0 + _ROW_BLOCK] = X[r0:r0 + _ROW_BLOCK].astype(np.float64) @ B
    return out


def data_scalars(X):
    """One-time scalars of X used by the method.

    ||X||_F^2 (= tr(X^T X), computed once, Appendix "Fast residual evaluation"),
    the mean zeta of all n^2 entries and max(X) (Section 5: the random
    initialisation scales by zeta; alpha = max(X)), and the row sums.
    """
    if sp.issparse(X):
        v = X.data.astype(np.float64)
        n = X.shape[0]
        rowsum = np.asarray(X.astype(np.float64).sum(axis=1)).ravel()
        mx = v.max() if v.size else 0.0
        if X.nnz < n * n:
            mx = max(mx, 0.0)   # implicit zeros take part in max and mean
        return dict(normsq=float(v @ v), zeta=float(v.sum()) / (n * n), maxval=float(mx), rowsum=rowsum)
    n = X.shape[0]
    normsq = 0.0
    total = 0.0
    mx = -np.inf
    rowsum = np.empty(n)
    for r0 in range(0, n, _ROW_BLOCK):
        blk = X[r0:r0 + _ROW_BLOCK].astype(np.float64)
        normsq += float(np.sum(blk * blk))
        rs = blk.sum(axis=1)
        rowsum[r0:r0 + _ROW_BLOCK] = rs
        total += float(rs.sum())
        mx = max(mx, float(blk.max()))
    return dict(normsq=normsq, zeta=total / (n * n), maxval=mx, rowsum=rowsum)


# ----------------------------------------------------------------------------
# Initialisation (Section 5, experimental setup): entries uniform on [0, 1),
# scaled by 2*sqrt(zeta/k), zeta the average of all entries of X.
# Reading: the starting W of the HALS sweeps equals H.
# ----------------------------------------------------------------------------

def initial_factor(n, k, zeta, seed):
    u = philox.uniform(seed, n * k, 0, philox.TAG_H0).reshape(n, k)
    return u * (2.0 * np.sqrt(zeta / k))


# ----------------------------------------------------------------------------
# Update rules.
# ----------------------------------------------------------------------------

def hals_symmetric(XH, H, W, alpha):
    """One sweep of the efficient regularised SymHALS rule for W given H
    (Section 2.1.2, eq. symhals_update2), columns i = 1..k in order, each
    column using the already-updated earlier columns of W:

        w_i <- [ ((X - W H^T + alpha I) h_i + ||h_i||^2 w_i) / (||h_i||^2 + alpha) ]_+

    with (X - W H^T + alpha I) h_i = (XH)_i - W (H^T h_i) + alpha h_i.
    The rule for H given W is the same call with the roles swapped.
    """
    W = np.array(W, dtype=np.float64, copy=True)
    H = np.asarray(H, dtype=np.float64)
    HtH = H.T @ H
    for i in range(H.shape[1]):
        hh = HtH[i, i]
        num = XH[:, i] - W @ HtH[:, i] + alpha * H[:, i] + hh * W[:, i]
        W[:, i] = np.maximum(num / (hh + alpha), 0.0)
    return W


def hals_explicit(X, W, H, alpha):
    """The same sweep written with the explicit residual R_i = X - sum_{j != i}
    w_j h_j^T (Section 2.1.2, eq. symhals_update1; derivation in Appendix A).
    Only for tiny n (forms n x n matrices)."""
    W = np.array(W, dtype=np.float64, copy=True)
    H = np.asarray(H, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    n, k = H.shape
    for i in range(k):
        R = X.copy()
        for j in range(k):
            if j != i:
                R -= np.outer(W[:, j], H[:, j])
        hi = H[:, i]
        W[:, i] = np.maximum((R + alpha * np.eye(n)) @ hi / (hi @ hi + alpha), 0.0)
    return W


def hals_gy(G, Y, W):
    """HALS as an Update(G, Y) rule (Appendix "Update() function"):
    w_i <- [ w_i + (Y_i - (W G)_i) / G_ii ]_+ for i = 1..k in order, with the
    regularised pair G = H^T H + alpha I, Y = X H + alpha H (or their sampled
    counterparts in Algorithm LvS-SymNMF)."""
    W = np.array(W, dtype=np.float64, copy=True)
    for i in range(G.shape[0]):
        W[:, i] = np.maximum(W[:, i] + (Y[:, i] - W @ G[:, i]) / G[i, i], 0.0)
    return W


def nls_gy(G, Y, method="auto"):
    """Exact nonnegative least squares for every row (Appendix "Update()":
    ANLS solves min_{x >= 0} x^T G x - 2 x^T y per row).  With alpha > 0 the
    matrix G is positive definite and the minimiser is unique.

    k <= 10: brute force over all 2^k supports F; the minimiser is the
    candidate with smallest objective among the solutions of G_FF x_F = y_F
    that are nonnegative.  Larger k: scipy's Lawson-Hanson NNLS on the
    Cholesky-transformed system ||L^T x - L^{-1} y||, G = L L^T.
    method: "auto" (as above), "brute" or "lh" to force one of the two.
    (This defines the result that block principal pivoting must reach.)
    """
    G = np.asarray(G, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    n, k = Y.shape
    if method == "brute" or (method == "auto" and k <= 10):
        best = np.zeros((n, k))
        best_obj = np.zeros(n)       # F = {} gives x = 0 with objective 0
        for r in range(1, k + 1):
            for F in itertools.combinations(range(k), r):
                F = list(F)
                xF = np.linalg.solve(G[np.ix_(F, F)], Y[:, F].T).T
                ok = np.all(xF >= 0.0, axis=1)
                x = np.zeros((n, k))
                x[:, F] = xF
                obj = np.einsum('ij,jk,ik->i', x, G, x) - 2.0 * np.einsum('ij,ij->i', x, Y)
                better = ok & (obj < best_obj)
                best[better] = x[better]
                best_obj[better] = obj[better]
        return best
    L = np.linalg.cholesky(G)
    A = L.T
    out = np.empty((n, k))
    for j in range(n):
        b = np.linalg.solve(L, Y[j])
        out[j], _ = nnls(A, b, maxiter=50 * k)
    return out


# ----------------------------------------------------------------------------
# Residuals (Appendix "Stopping criteria").
# ----------------------------------------------------------------------------

def residual_direct(X, W, H):
    """||X - W H^T||_F by forming the difference block by block."""
    W = np.asarray(W, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    if sp.issparse(X):
        Xd = X.toarray().astype(np.float64)
        return float(np.linalg.norm(Xd - W @ H.T))
    s = 0.0
    for r0 in range(0, X.shape[0], _ROW_BLOCK):
        d = X[r0:r0 + _ROW_BLOCK].astype(np.float64) - W[r0:r0 + _ROW_BLOCK] @ H.T
        s += float(np.sum(d * d))
    return float(np.sqrt(s))


def residual_trace(normsq, W, H, XW):
    """||X - W H^T||_F by the trace identity (Appendix "Fast residual
    evaluation"): tr(X^T X) + tr(H W^T W H^T) - 2 tr(W^T X H), reusing the
    latest product XW (tr(W^T X H) = tr(H^T X W) for symmetric X)."""
    W = np.asarray(W, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    r2 = normsq + float(np.sum((W.T @ W) * (H.T @ H))) - 2.0 * float(np.sum(H * XW))
    return float(np.sqrt(max(r2, 0.0)))


def projected_gradient_norm(XH, XW, W, H, alpha):
    """Projected gradient norm (Appendix "Projected gradients") for the
    regularised surrogate.  Reading: the gradients include the alpha terms,
    grad_W = 2(W H^T H - X H + alpha (W - H)) and symmetrically for H; an entry
    counts when it is negative or its variable is positive."""
    gW = 2.0 * (W @ (H.T @ H) - XH + alpha * (W - H))
    gH = 2.0 * (H @ (W.T @ W) - XW + alpha * (H - W))
    pW = np.where((gW < 0) | (W > 0), gW, 0.0)
    pH = np.where((gH < 0) | (H > 0), gH, 0.0)
    return float(np.sqrt(np.sum(pW * pW) + np.sum(pH * pH)))


class StallRule:
    """Stop once the normalised residual has failed to drop by more than
    `tol` for `patience` consecutive iterations (Section 5.1 setup: 1e-4,
    four iterations).  Reading: the drop is the absolute difference of
    consecutive normalised residuals."""

    def __init__(self, tol=1e-4, patience=4):
        self.tol, self.patience, self.prev, self.count = tol, patience, None, 0

    def __call__(self, r):
        if self.prev is not None:
            self.count = self.count + 1 if (self.prev - r) <= self.tol else 0
        self.prev = r
        return self.count >= self.patience


# ----------------------------------------------------------------------------
# Alternating updates (Section 2.1.1 eq. ANLS4symNMF; order W then H as in
# Algorithms LAI-SymNMF and LvS-SymNMF).
# ----------------------------------------------------------------------------

def anls(X_apply, normsq, H0, alpha, iters, rule="hals", W0=None, stop=None, target=None):
    """Alternating updates of W from H, then H from W.

    X_apply(B) returns the data product X @ B (or the LAI product).
    One iteration = W-update then H-update; after it the normalised residual
    (trace identity against the matrix X_apply represents) is recorded.
    rule: "hals" (eq. symhals_update2, one sweep) or "nls" (exact NLS, the
    result block principal pivoting computes).
    Returns W, H and the residual history.
    """
    H = np.array(H0, dtype=np.float64, copy=True)
    W = H.copy() if W0 is None else np.array(W0, dtype=np.float64, copy=True)
    k = H.shape[1]
    I = np.eye(k)
    hist = []
    nx = np.sqrt(normsq)
    for _ in range(iters):
        XH = X_apply(H)
        if rule == "hals":
            W = hals_symmetric(XH, H, W, alpha)
        else:
            W = nls_gy(H.T @ H + alpha * I, XH + alpha * H)
        XW = X_apply(W)
        if rule == "hals":
            H = hals_symmetric(XW, W, H, alpha)
        else:
            H = nls_gy(W.T @ W + alpha * I, XW + alpha * W)
        r = residual_trace(normsq, W, H, XW) / nx
        hist.append(r)
        if target is not None and r <= target:
            break
        if stop is not None and stop(r):
            break
    return W, H, np.array(hist)


def plain_symnmf(X, k, alpha, H0, iters, rule="hals", stop=None, target=None):
    """Deterministic regularised SymNMF on the full X."""
    sc = data_scalars(X)
    return anls(lambda B: apply_x(X, B), sc["normsq"], H0, alpha, iters, rule, stop=stop, target=target)


# ----------------------------------------------------------------------------
# Randomized range finder and approximate EVD (Section 2.2.1, Algorithms RRF
# and Apx-EVD).
# ----------------------------------------------------------------------------

def sketch_omega(n, l, seed):
    """The Gaussian test matrix Omega (n x l), row-major value e = i*l + j."""
    return philox.gaussian(seed, n * l, 0, philox.TAG_OMEGA).reshape(n, l)


def _qr_positive(Y):
    """Thin Householder QR with the sign of each column chosen so that
    diag(R) > 0 (reading: the paper does not fix the sign convention)."""
    Q, R = np.linalg.qr(Y)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def rrf(X_apply, Omega, q):
    """Orthonormal basis of the range of (X X^T)^q X Omega.

    Reading: the basis is re-orthonormalised after every application of X
    (2q+1 applications), as the adaptive variant of the appendix does; in
    exact arithmetic this equals the single QR of Algorithm RRF because the
    positive-diagonal Q factor of X^(2q+1) Omega is unique."""
    Q = _qr_positive(X_apply(Omega))
    for _ in range(2 * q):
        Q = _qr_positive(X_apply(Q))
    return Q


def ada_rrf(X_apply, normsq, Omega, q_max, tol=1e-3):
    """Algorithm Ada-RRF (appendix "Adaptive Randomized Range Finder") for a
    symmetric X.  Q = qr(X Omega); then, while at most q_max rounds:
    B^T = X^T Q (= X Q), the normalised QB residual
    sqrt((||X||^2 - ||B||_F^2) / ||X||^2) (the trace identity of that
    appendix), Q = qr(B^T); stop when the residual fell by less than `tol`
    since the previous check (reading: absolute decrease, first check compared
    with +infinity); otherwise Y = X Q and Q = qr(Y).
    Returns (Q, number of completed rounds, residuals of the checks)."""
    Q = _qr_positive(X_apply(Omega))
    prev = np.inf
    res = []
    rounds = 0
    for _ in range(q_max):
        B = X_apply(Q)
        r = np.sqrt(max(normsq - float(np.sum(B * B)), 0.0) / normsq)
        res.append(r)
        Q = _qr_positive(B)
        if prev - r < tol:
            break
        prev = r
        Q = _qr_positive(X_apply(Q))
        rounds += 1
    return Q, rounds, res


def apx_evd(X_apply, Omega, q, Q=None):
    """Algorithm Apx-EVD: Q = RRF, T = Q^T X Q (one more product with X),
    T = Q_T Lambda Q_T^T, U = Q Q_T.  A basis Q computed elsewhere (Ada-RRF)
    may be passed instead of running RRF with q.

    Readings: eigenvalues sorted descending and negative ones kept (the PSD
    projection is commented out in the source); each column of U is signed so
    that its entry of largest magnitude is positive (first such row on ties).
    """
    if Q is None:
        Q = rrf(X_apply, Omega, q)
    T = Q.T @ X_apply(Q)
    T = 0.5 * (T + T.T)
    lam, V = np.linalg.eigh(T)
    order = np.argsort(-lam, kind="stable")
    lam, V = lam[order], V[:, order]
    U = Q @ V
    idx = np.argmax(np.abs(U), axis=0)
    sgn = np.sign(U[idx, np.arange(U.shape[1])])
    sgn[sgn == 0] = 1.0
    return U * sgn, lam


def lai_symnmf(U, lam, k, alpha, H0, iters, rule="hals", stop=None, target=None):
    """Algorithm LAI-SymNMF: the alternating updates on X_L = U Lambda U^T,
    whose products are U (Lambda (U^T B)) (Y_H = (H^T V) U^T + alpha H^T with
    V = U Lambda, transposed).  Residuals are against X_L, whose squared
    Frobenius norm is ||Lambda||^2 because U has orthonormal columns
    (Appendix "Residual computation for LAI-NMF")."""
    U = np.asarray(U, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    normsq = float(lam @ lam)
    return anls(lambda B: U @ (lam[:, None] * (U.T @ B)), normsq, H0, alpha, iters, rule,
                stop=stop, target=target)


# ----------------------------------------------------------------------------
# Projected Gauss-Newton with conjugate gradients on the SymNMF objective
# min_{H >= 0} ||X - H H^T||_F (Section 2.1.3, eq. symnmf_obj; Algorithm
# LAI-PGNCG-SymNMF in the appendix on LAI-SymNMF).
# ----------------------------------------------------------------------------

def gn_gradient(XH, H):
    """g = J^T r with r = vec(X - H H^T): g = -2 (X H - H (H^T H))
    (Section 2.1.3; XH is the data product of H)."""
    return -2.0 * (XH - H @ (H.T @ H))


def gn_normal_apply(H, P):
    """J^T J vec(P) for the Jacobian J = -(H kron I) - P_mm (H kron I) of
    r(H) = vec(X - H H^T): 2 (P H^T H + H P^T H) (Section 2.1.3; the
    CG product of Algorithm LAI-PGNCG-SymNMF)."""
    return 2.0 * (P @ (H.T @ H) + H @ (P.T @ H))


def gn_direction(XH, H, cg_iters):
    """Z ~ (J^T J)^+ g by at most cg_iters conjugate-gradient steps from Z = 0
    on the normal equations J^T J z = J^T r (Section 2.1.3).  The new factor
    is max(H - Z, 0).

    Readings (the printed pseudo-code updates neither the direction nor uses
    a separate step name): standard CG, the step length a = e / <P, J^T J P>
    with e = ||R||_F^2, then R <- R - a J^T J P, Z <- Z + a P and the
    direction P <- R + (e_new / e) P.  CG stops early (its last Z kept) when
    <P, J^T J P> is not positive: J^T J is singular along directions H S with
    S skew-symmetric, and R = 0 at a stationary point."""
    R = gn_gradient(XH, H)
    P = R.copy()
    Z = np.zeros_like(H)
    e = float(np.sum(R * R))
    for _ in range(cg_iters):
        Y = gn_normal_apply(H, P)
        pap = float(np.sum(P * Y))
        if not pap > 0.0:
            break
        a = e / pap
        Z = Z + a * P
        R = R - a * Y
        e_new = float(np.sum(R * R))
        P = R + (e_new / e) * P
        e = e_new
    return Z


def pgncg(X_apply, normsq, H0, iters, cg_iters, stop=None, target=None):
    """PGNCG-SymNMF: H <- max(H - Z, 0) with Z from gn_direction, one data
    product X H per iteration.  X_apply(B) is X @ B, or the LAI product
    U (Lambda (U^T B)) for Algorithm LAI-PGNCG-SymNMF.

    Reading (the paper gives no logging rule for this method): entry t of the
    history is the normalised residual ||X - H_t H_t^T||_F / ||X||_F of the
    factor iteration t starts from, by the trace identity with the product
    that iteration computes anyway (Appendix "Fast residual evaluation");
    the stop rule sees it before the step, so a stop keeps H_t.
    Returns H and the history."""
    H = np.array(H0, dtype=np.float64, copy=True)
    nx = np.sqrt(normsq)
    hist = []
    for _ in range(iters):
        XH = X_apply(H)
        r = residual_trace(normsq, H, H, XH) / nx
        hist.append(r)
        if target is not None and r <= target:
            break
        if stop is not None and stop(r):
            break
        H = np.maximum(H - gn_direction(XH, H, cg_iters), 0.0)
    return H, np.array(hist)


def plain_pgncg(X, H0, iters, cg_iters, stop=None, target=None):
    """PGNCG-SymNMF on the full X."""
    sc = data_scalars(X)
    return pgncg(lambda B: apply_x(X, B), sc["normsq"], H0, iters, cg_iters, stop=stop, target=target)


def lai_pgncg(U, lam, H0, iters, cg_iters, stop=None, target=None):
    """Algorithm LAI-PGNCG-SymNMF: X H replaced by U (Lambda (U^T H)), the
    residual taken against U Lambda U^T (squared norm ||Lambda||^2)."""
    U = np.asarray(U, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    return pgncg(lambda B: U @ (lam[:, None] * (U.T @ B)), float(lam @ lam), H0, iters, cg_iters,
                 stop=stop, target=target)


# ----------------------------------------------------------------------------
# Leverage scores and hybrid sampling (Section 2.2.2 eq. lev_score_def and
# lev_score_S; Section 4.2 hybrid sampling, eq. SH).
# ----------------------------------------------------------------------------

LEV_QUANT_BITS = 40


def leverage_scores(A):
    """l_i(A) = ||Q_A[i, :]||^2 for an orthonormal basis Q_A of range(A)
    (eq. lev_score_def); Q_A from Householder QR."""
    Q, _ = np.linalg.qr(np.asarray(A, dtype=np.float64))
    return np.sum(Q * Q, axis=1)


def hybrid_sample(lev, k, s, tau, seed, half_iter):
    """Hybrid leverage-score sampling matrix S (Section 4.2, eq. SH).

    Rows with p_i = l_i / k >= tau are kept deterministically (weight 1).  The
    remaining rows are drawn s_R = s - s_D times with replacement with
    probability proportional to l_i (p~_i = l_i / (k - theta)); a row drawn c
    times gets weight c / (s_R p~_i) on its row of S^T S (eq. lev_score_S:
    each draw contributes 1/(s_R p~_i)).

    Readings (the paper does not fix the discretisation): p~_i is realised
    exactly with integer weights w_i = floor(l_i * 2^40) and W_R = sum w_i, so
    p~_i = w_i / W_R; draw j takes r = floor(v_j W_R / 2^64) from Philox value
    v_j of stream (seed, half_iter, SAMPLE) and selects the smallest i whose
    inclusive prefix sum of w exceeds r.  The weight is computed as
    (c * W_R) / (s_R * w_i) in FP64 with that operation order.

    Returns (rows ascending int64, weights float64, info dict).
    """
    lev = np.asarray(lev, dtype=np.float64)
    n = lev.shape[0]
    p = lev / k
    det = p >= tau
    s_D = int(det.sum())
    theta = float(lev[det].sum())
    s_R = max(int(s) - s_D, 0)
    w = np.where(det, 0.0, np.floor(lev * float(2 ** LEV_QUANT_BITS))).astype(np.uint64)
    W_R = int(sum(int(x) for x in w)) if n < 4096 else int(w.sum(dtype=np.uint64))
    counts = np.zeros(n, dtype=np.int64)
    if s_R > 0 and W_R > 0:
        r = philox.draws(seed, s_R, half_iter, philox.TAG_SAMPLE, W_R)
        prefix = np.cumsum(w, dtype=np.uint64)
        idx = np.searchsorted(prefix, r.astype(np.uint64), side="right")
        counts = np.bincount(idx, minlength=n).astype(np.int64)
    rows = np.nonzero(det | (counts > 0))[0]
    weights = np.empty(rows.shape[0], dtype=np.float64)
    for j, i in enumerate(rows):
        if det[i]:
            weights[j] = 1.0
        else:
            weights[j] = (float(counts[i]) * float(W_R)) / (float(s_R) * float(w[i]))
    info = dict(s_D=s_D, theta=theta, s_R=s_R, W_R=W_R, counts=counts)
    return rows, weights, info


def lvs_half_step(X, src, dst, alpha, s, tau, seed, half_iter, rule="hals"):
    """One half-iteration of Algorithm LvS-SymNMF: new `dst` from `src`.

    Leverage scores of src, hybrid S, then Update(G, Y) with the sampled
    G = src^T S^T S src + alpha I and Y = X S^T S src + alpha src (the sampling
    acts on the rows of src only; the alpha block is kept exactly,
    Section 4.1)."""
    src = np.asarray(src, dtype=np.float64)
    k = src.shape[1]
    lev = leverage_scores(src)
    rows, wts, info = hybrid_sample(lev, k, s, tau, seed, half_iter)
    Hs = src[rows]
    WHs = wts[:, None] * Hs
    G = Hs.T @ WHs + alpha * np.eye(k)
    if sp.issparse(X):
        Xc = X.tocsc()[:, rows]
        Y = np.asarray(Xc @ WHs) + alpha * src
    else:
        Y = np.asarray(X[:, rows], dtype=np.float64) @ WHs + alpha * src
    if rule == "hals":
        new = hals_gy(G, Y, dst)
    else:
        new = nls_gy(G, Y)
    info["lev"] = lev
    info["rows"] = rows
    info["weights"] = wts
    info["G"] = G
    info["Y"] = Y
    return new, info


def lvs_symnmf(X, k, alpha, H0, iters, s, tau, seed, rule="hals", t0=0):
    """Algorithm LvS-SymNMF for `iters` iterations.  Half-iteration index
    h = 2 t + side (side 0 updates W from H, side 1 updates H from W) selects
    the Philox sub-stream of the draws.  Residuals are exact (full product)."""
    sc = data_scalars(X)
    nx = np.sqrt(sc["normsq"])
    H = np.array(H0, dtype=np.float64, copy=True)
    W = H.copy()
    hist = []
    for t in range(t0, t0 + iters):
        W, _ = lvs_half_step(X, H, W, alpha, s, tau, seed, 2 * t, rule)
        H, _ = lvs_half_step(X, W, H, alpha, s, tau, seed, 2 * t + 1, rule)
        hist.append(residual_trace(sc["normsq"], W, H, apply_x(X, W)) / nx)
    return W, H, np.array(hist)
