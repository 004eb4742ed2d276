"""Shared helpers of the GPU parity tests (inputs -> device, comparisons)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2402_08134_amd as P  # noqa: E402


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()  # raises if the library is missing: no fallback


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().to(torch.float64).numpy()


def csr_dev(X):
    """scipy CSR -> (row_ptr, col_idx, values, n) GPU tensors."""
    return (dev(X.indptr.astype(np.int32)), dev(X.indices.astype(np.int32)), dev(X.data), X.shape[0])


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def factor(ctx, which):
    dt = torch.float64 if ctx.fdtype == P.F64 else torch.float32
    out = torch.empty((ctx.n, ctx.k), dtype=dt, device="cuda")
    P.symnmf_get_factor(ctx, which, out)
    return host(out)


def round_to(a, dtype):
    """Values of `a` as stored in `dtype` (FP64 result)."""
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(torch.float64).numpy()


def log(msg):
    print(msg, flush=True)
