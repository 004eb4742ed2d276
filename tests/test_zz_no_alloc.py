"""The learned start without device allocation (symnmf_warmstart_noalloc):
its temporaries live in the library's static per-GPU scratch array.  Checked
through the C ABI against symnmf_warmstart on identically prepared contexts,
on two calls in a row (the second with a smaller input, so stale contents of
the larger first call would show), in FP32 and FP64, and the size limit."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads

from gpu_common import P, torch, require_gpu, dev, factor, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _prepared(X, k, l, q, seed):
    ctx = P.symnmf_create(dev(X), k, 0.0, 0, seed)
    P.symnmf_lai(ctx, l, q)
    return ctx


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_noalloc_warmstart_matches_the_allocating_call(dtype):
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 11)
    for n, k, l in ((2400, 32, 48), (900, 8, 24)):   # second call smaller
        X, _ = workloads.gaussian_kernel(n, 2 * k, k, seed=n + k, dtype=dtype)
        log(f"warmstart_noalloc n={n} k={k} l={l} dtype={np.dtype(dtype).name}")
        a = _prepared(X, k, l, 2, 3)
        b = _prepared(X, k, l, 2, 3)
        beta_a = P.symnmf_warmstart(a, net)
        beta_b = P.symnmf_warmstart_noalloc(b, net)
        assert beta_a > 0 and beta_b == beta_a
        for which in (P.W, P.H):
            assert np.array_equal(factor(a, which), factor(b, which))
        # the solve continues identically from both starts
        P.symnmf_iterate(a, 3)
        P.symnmf_iterate(b, 3)
        assert P.symnmf_history(a) == P.symnmf_history(b)


def test_noalloc_warmstart_rejects_sizes_beyond_the_scratch():
    n, k = 40000, 64                                   # n k FP32 needs 80 MB > 64 MiB
    A = sp.diags(np.ones(n - 1), 1, format="csr", dtype=np.float32)
    A = (A + A.T).tocsr()
    A.sort_indices()
    X = (dev(A.indptr.astype(np.int32)), dev(A.indices.astype(np.int32)), dev(A.data), n)
    ctx = P.symnmf_create(X, k, 0.0, 0, 1)
    net = P.symnmf_mlp_create(P.MLP_HIDDEN, 1)
    with pytest.raises(P.SymNMFError) as e:
        P.symnmf_warmstart_noalloc(ctx, net)
    assert e.value.code == P.E_INVALID and "scratch" in str(e.value)
