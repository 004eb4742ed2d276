"""Host-side part of the learned warm start against the oracle (no GPU).

The training targets are built on the host by the package (column matching
by the assignment problem, then the RMS rescale); the oracle defines the same
targets independently.  The inputs make a slip visible: the columns of H are
a known permutation of noisy anchors with very different norms, so a
transposed cosine matrix, a permutation applied the wrong way round or a
per-column instead of a global rescale all change the result."""
import numpy as np
import pytest

from oracle import warmstart as OW
from paper_2402_08134_amd import warmstart as WS


def _instance(n, l, k, seed):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((n, l)))[0]
    A = OW.anchors(U, k)
    perm = rng.permutation(k)
    scales = rng.uniform(0.2, 5.0, size=k)
    H = np.empty((n, k))
    for j in range(k):
        H[:, perm[j]] = scales[j] * (A[:, j] + 0.02 * rng.uniform(size=n))
    return H, U, perm


@pytest.mark.parametrize("n,l,k,seed", [(60, 8, 3, 0), (200, 21, 5, 1), (500, 32, 16, 2), (1000, 80, 64, 3)])
def test_align_targets_equals_oracle_targets(n, l, k, seed):
    H, U, perm = _instance(n, l, k, seed)
    got = WS.align_targets(H, U, k)
    want = OW.targets(H, U, k)
    assert got.dtype == np.float32 and got.shape == (n, k)
    assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want))
    # the planted matching is recovered: column perm[j] of H lands on anchor j
    for j in range(k):
        assert np.allclose(got[:, j], H[:, perm[j]] / (np.linalg.norm(H) / np.sqrt(n * k)), rtol=1e-6)


def test_align_targets_matching_is_the_brute_force_optimum():
    # k = 5: every permutation enumerated (the assignment problem's optimum)
    rng = np.random.default_rng(7)
    n, l, k = 120, 9, 5
    U = np.linalg.qr(rng.standard_normal((n, l)))[0]
    H = rng.uniform(size=(n, k)) ** 3
    got = WS.align_targets(H, U, k)
    perm = OW.match_columns_brute(OW.anchors(U, k), H)
    want = H[:, perm] / (np.linalg.norm(H) / np.sqrt(n * k))
    assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want))


def test_spectral_anchors_equal_oracle_anchors():
    rng = np.random.default_rng(8)
    U = np.linalg.qr(rng.standard_normal((300, 24)))[0]
    U[:, 3] = 0.0                     # a zero column stays zero
    got = WS.spectral_anchors(U, 16)
    want = OW.anchors(U, 16)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-15)
