"""Bit-identical random streams on both sides (the shared generator
contract): the Gaussian sketch Omega of Algorithm RRF and the random initial
factor of the experimental setup, 2^20 values each, device against the
oracle's own implementation of the same published definitions (Philox-4x32-10
and Box-Muller with the library's own logarithm and cosine)."""
import hashlib

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import philox
from oracle import symnmf as O

from gpu_common import P, torch, require_gpu, dev, host, factor, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _path_graph(n, dtype=np.float64):
    """CSR of a path graph with unit weights: every sum over it is exact, so
    the mean of X (and with it the scale of the random start) is the same
    number on both sides whatever the summation order."""
    A = sp.diags(np.ones(n - 1), 1, format="csr", dtype=dtype)
    A = (A + A.T).tocsr()
    A.sort_indices()
    return A, (dev(A.indptr.astype(np.int32)), dev(A.indices.astype(np.int32)), dev(A.data), n)


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()[:16]


@pytest.mark.parametrize("n,l,seed", [(16384, 64, 1), (16384, 64, (1 << 40) + 3), (1000, 48, 7)])
def test_sketch_bitwise(n, l, seed):
    _, X = _path_graph(n)
    ctx = P.symnmf_create(X, 4, 0.0, 0, seed)
    Om = torch.empty((n, l), dtype=torch.float64, device="cuda")
    P.symnmf_get_sketch(ctx, l, Om)
    g = host(Om)
    o = O.sketch_omega(n, l, seed)
    log(f"sketch n={n} l={l} seed={seed}: device {_digest(g)} oracle {_digest(o)}")
    assert _digest(g) == _digest(o)
    assert np.array_equal(g.view(np.uint64), o.view(np.uint64))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_initial_factor_bitwise(dtype):
    n, k, seed = 16384, 64, 9
    A, X = _path_graph(n, dtype)
    ctx = P.symnmf_create(X, k, 0.0, 0, seed)
    zeta = O.data_scalars(A.astype(np.float64))["zeta"]
    ho = O.initial_factor(n, k, zeta, seed)
    if dtype == np.float32:
        ho = ho.astype(np.float32).astype(np.float64)
    hg = factor(ctx, P.H)
    log(f"initial factor {np.dtype(dtype).name} n={n} k={k}: device {_digest(hg)} oracle {_digest(ho)}")
    assert np.array_equal(hg, ho) and np.array_equal(factor(ctx, P.W), ho)
    # the uniform stream itself: u = H0 / scale is exact in FP64
    if dtype == np.float64:
        u = philox.uniform(seed, n * k, 0, philox.TAG_H0).reshape(n, k)
        assert np.array_equal(hg, u * (2.0 * np.sqrt(zeta / k)))
