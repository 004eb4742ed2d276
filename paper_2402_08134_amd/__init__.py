"""Python binding of libsymnmf (randomized symmetric NMF on MI355X / gfx950).

Argument marshalling only: every function forwards to the C entry point of the
same name in ``libsymnmf.so`` (declared in ``include/symnmf.h``).  PyTorch
tensors are used for device memory and the stream; no torch operation takes
part in a solve.  There is no fallback: if the library is not built or no GPU
is present, the calls raise.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsymnmf.so")

OK, E_INVALID, E_UNSUPPORTED, E_NOMEM, E_DEVICE, E_NUMERIC, E_STATE = range(7)
DENSE, CSR = 0, 1
F64, F32, BF16 = 0, 1, 2
RULE_HALS, RULE_BPP, RULE_PGNCG = 0, 1, 2
STOP_NONE, STOP_STALL, STOP_TARGET, STOP_STALL_OR_TARGET = 0, 1, 2, 3
RESID_FAST, RESID_EXACT, RESID_LAI = 0, 1, 2
W, H = 0, 1
MODE_PLAIN, MODE_LAI, MODE_LVS = 0, 1, 2
PHASE_PRODUCT, PHASE_UPDATE, PHASE_SAMPLE, PHASE_LAI, PHASE_WARM, PHASE_REDUCE = 0, 1, 2, 3, 4, 5
NUM_PHASES = 6
MLP_FEATURES, MLP_HIDDEN = 6, 64
FLAG_LEV_SHIFT, FLAG_CHOLQR_SHIFT, FLAG_BPP_CAP = 1, 2, 4


class SymNMFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"symnmf error {code}: {msg}")
        self.code = code


class Matrix(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("nnz", ctypes.c_int64), ("values", ctypes.c_void_p),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("rule", ctypes.c_int32), ("compute_dtype", ctypes.c_int32),
                ("stop_mode", ctypes.c_int32), ("stop_tol", ctypes.c_double), ("stop_patience", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("target", ctypes.c_double), ("tau", ctypes.c_double),
                ("resid_every", ctypes.c_int32), ("max_history", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("graphs", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class Stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("mode", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("stopped", ctypes.c_int32), ("k", ctypes.c_int32), ("l", ctypes.c_int32), ("n", ctypes.c_int64),
                ("alpha", ctypes.c_double), ("zeta", ctypes.c_double), ("normsq", ctypes.c_double),
                ("maxval", ctypes.c_double), ("last_residual", ctypes.c_double), ("s_D", ctypes.c_int64),
                ("sample_rows", ctypes.c_int64), ("theta_over_k", ctypes.c_double), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 7), ("warm_beta", ctypes.c_double), ("phase_ms", ctypes.c_double * NUM_PHASES),
                ("phase_calls", ctypes.c_int64 * NUM_PHASES), ("graph_launches", ctypes.c_int64)]


_VP = ctypes.c_void_p
_SIGS = {
    "symnmf_default_options": (ctypes.c_int, [ctypes.POINTER(Options)]),
    "symnmf_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.POINTER(Matrix), ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(Options), _VP]),
    "symnmf_lai": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "symnmf_refine": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_double]),
    "symnmf_lai_adaptive": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "symnmf_iterate": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "symnmf_residual": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "symnmf_set_factor": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, ctypes.c_int32]),
    "symnmf_get_factor": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, ctypes.c_int32]),
    "symnmf_get_lai": (ctypes.c_int, [_VP, _VP, _VP]),
    "symnmf_apply_x": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP]),
    "symnmf_get_sketch": (ctypes.c_int, [_VP, ctypes.c_int32, _VP]),
    "symnmf_half_step": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "symnmf_leverage": (ctypes.c_int, [_VP, ctypes.c_int32, _VP]),
    "symnmf_sample": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, _VP, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64)]),
    "symnmf_history": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32)]),
    "symnmf_get_stats": (ctypes.c_int, [_VP, ctypes.POINTER(Stats)]),
    "symnmf_last_error": (ctypes.c_char_p, [_VP]),
    "symnmf_destroy": (None, [_VP]),
    "symnmf_trim_cache": (ctypes.c_int, []),
    "symnmf_mlp_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int32, ctypes.c_uint64, _VP]),
    "symnmf_mlp_num_params": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    "symnmf_mlp_set_params": (ctypes.c_int, [_VP, _VP]),
    "symnmf_mlp_get_params": (ctypes.c_int, [_VP, _VP]),
    "symnmf_mlp_forward": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, _VP]),
    "symnmf_mlp_gradient": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, _VP, ctypes.POINTER(ctypes.c_double)]),
    "symnmf_mlp_train_step": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_double)]),
    "symnmf_mlp_save": (ctypes.c_int, [_VP, ctypes.c_char_p]),
    "symnmf_mlp_load": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_char_p, _VP]),
    "symnmf_mlp_last_error": (ctypes.c_char_p, [_VP]),
    "symnmf_mlp_destroy": (None, [_VP]),
    "symnmf_warm_features": (ctypes.c_int, [_VP, _VP]),
    "symnmf_warmstart": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(ctypes.c_double)]),
    "symnmf_warmstart_noalloc": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def lib():
    """Load libsymnmf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2402_08134_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != OK:
        msg = lib().symnmf_last_error(ctx)
        raise SymNMFError(rc, msg.decode() if msg else "")


def _dtype_code(t):
    import torch
    return {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[t.dtype]


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def symnmf_default_options(**overrides):
    o = Options()
    _check(lib().symnmf_default_options(ctypes.byref(o)))
    for key, v in overrides.items():
        setattr(o, key, v)
    return o


class Context:
    """A symnmf_ctx* plus references to the borrowed device arrays of X."""

    def __init__(self, handle, keep, k, n, fdtype):
        self.handle = handle
        self._keep = keep
        self.k, self.n, self.fdtype = k, n, fdtype

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.symnmf_destroy(h)


def symnmf_create(X, k, alpha=0.0, s=0, seed=0, options=None, stream=None):
    """X: a dense symmetric torch tensor on the GPU (n x n), or a tuple
    (row_ptr int32, col_idx int32, values, n) of GPU tensors for CSR."""
    import torch
    m = Matrix()
    if isinstance(X, tuple):
        rp, ci, val, n = X
        m.kind, m.dtype, m.n, m.ld, m.nnz = CSR, _dtype_code(val), n, n, ci.numel()
        m.values, m.row_ptr, m.col_idx = val.data_ptr(), rp.data_ptr(), ci.data_ptr()
        keep = (rp, ci, val)
        n = int(n)
        dt = m.dtype
    else:
        assert X.dim() == 2 and X.shape[0] == X.shape[1] and X.stride(1) == 1
        n = X.shape[0]
        m.kind, m.dtype, m.n, m.ld, m.nnz = DENSE, _dtype_code(X), n, X.stride(0), 0
        m.values = X.data_ptr()
        keep = (X,)
        dt = m.dtype
    opt = options if options is not None else symnmf_default_options()
    cd = opt.compute_dtype if opt.compute_dtype >= 0 else dt
    fdtype = F64 if cd == F64 else F32
    h = ctypes.c_void_p()
    rc = lib().symnmf_create(ctypes.byref(h), ctypes.byref(m), int(k), float(alpha), int(s), int(seed),
                             ctypes.byref(opt), _stream_ptr(stream))
    _check(rc, None)
    return Context(h, keep + (opt,), int(k), n, fdtype)


def symnmf_lai(ctx, l, q):
    _check(lib().symnmf_lai(ctx.handle, int(l), int(q)), ctx.handle)


def symnmf_lai_adaptive(ctx, l, q_max=10, tol=1e-3):
    """Returns (completed rounds, last QB residual)."""
    rounds = ctypes.c_int32()
    res = ctypes.c_double()
    _check(lib().symnmf_lai_adaptive(ctx.handle, int(l), int(q_max), float(tol), ctypes.byref(rounds),
                                     ctypes.byref(res)), ctx.handle)
    return rounds.value, res.value


def symnmf_refine(ctx, stop_mode=STOP_NONE, target=0.0):
    _check(lib().symnmf_refine(ctx.handle, int(stop_mode), float(target)), ctx.handle)


def symnmf_iterate(ctx, iters):
    done = ctypes.c_int32()
    _check(lib().symnmf_iterate(ctx.handle, int(iters), ctypes.byref(done)), ctx.handle)
    return done.value


def symnmf_residual(ctx, mode=RESID_FAST):
    out = (ctypes.c_double * 2)()
    _check(lib().symnmf_residual(ctx.handle, int(mode), out), ctx.handle)
    return out[0], out[1]


def symnmf_set_factor(ctx, which, src):
    assert src.is_contiguous() and src.shape == (ctx.n, ctx.k)
    _check(lib().symnmf_set_factor(ctx.handle, int(which), src.data_ptr(), _dtype_code(src)), ctx.handle)


def symnmf_get_factor(ctx, which, dst):
    assert dst.is_contiguous() and dst.shape == (ctx.n, ctx.k)
    _check(lib().symnmf_get_factor(ctx.handle, int(which), dst.data_ptr(), _dtype_code(dst)), ctx.handle)


def symnmf_get_lai(ctx, U=None, lam=None):
    _check(lib().symnmf_get_lai(ctx.handle, U.data_ptr() if U is not None else None,
                                lam.data_ptr() if lam is not None else None), ctx.handle)


def symnmf_apply_x(ctx, B, Y):
    assert B.is_contiguous() and Y.is_contiguous() and B.shape == Y.shape and B.shape[0] == ctx.n
    _check(lib().symnmf_apply_x(ctx.handle, B.data_ptr(), int(B.shape[1]), Y.data_ptr()), ctx.handle)


def symnmf_get_sketch(ctx, l, Omega):
    import torch
    assert Omega.is_contiguous() and Omega.dtype == torch.float64 and Omega.numel() == ctx.n * l
    _check(lib().symnmf_get_sketch(ctx.handle, int(l), Omega.data_ptr()), ctx.handle)


def symnmf_half_step(ctx, side, half_iter=0):
    _check(lib().symnmf_half_step(ctx.handle, int(side), int(half_iter)), ctx.handle)


def symnmf_leverage(ctx, which, lev):
    assert lev.is_contiguous() and lev.numel() == ctx.n
    _check(lib().symnmf_leverage(ctx.handle, int(which), lev.data_ptr()), ctx.handle)


def symnmf_sample(ctx, lev, half_iter, rows, weights):
    cnt = ctypes.c_int64()
    _check(lib().symnmf_sample(ctx.handle, lev.data_ptr(), int(half_iter), rows.data_ptr(), weights.data_ptr(),
                               int(rows.numel()), ctypes.byref(cnt)), ctx.handle)
    return cnt.value


def symnmf_history(ctx, cap=4096):
    buf = (ctypes.c_double * cap)()
    cnt = ctypes.c_int32()
    _check(lib().symnmf_history(ctx.handle, buf, int(cap), ctypes.byref(cnt)), ctx.handle)
    return [buf[i] for i in range(cnt.value)]


def symnmf_get_stats(ctx):
    st = Stats()
    st.struct_size = ctypes.sizeof(Stats)
    _check(lib().symnmf_get_stats(ctx.handle, ctypes.byref(st)), ctx.handle)
    return st


def symnmf_trim_cache():
    _check(lib().symnmf_trim_cache())


def symnmf_destroy(ctx):
    h, ctx.handle = ctx.handle, None
    if h:
        lib().symnmf_destroy(h)


# ---- learned warm start -------------------------------------------------------

class Mlp:
    """A symnmf_mlp* (the warm-start network)."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.symnmf_mlp_destroy(h)


def _mcheck(rc, net):
    if rc != OK:
        msg = lib().symnmf_mlp_last_error(net.handle if net is not None else None)
        raise SymNMFError(rc, msg.decode() if msg else "")


def symnmf_mlp_create(hidden=MLP_HIDDEN, seed=0, stream=None):
    h = ctypes.c_void_p()
    _mcheck(lib().symnmf_mlp_create(ctypes.byref(h), int(hidden), int(seed), _stream_ptr(stream)), None)
    return Mlp(h)


def symnmf_mlp_save(net, path):
    _mcheck(lib().symnmf_mlp_save(net.handle, os.fsencode(path)), net)


def symnmf_mlp_load(path, stream=None):
    h = ctypes.c_void_p()
    _mcheck(lib().symnmf_mlp_load(ctypes.byref(h), os.fsencode(path), _stream_ptr(stream)), None)
    return Mlp(h)


def symnmf_mlp_num_params(net):
    c = ctypes.c_int64()
    _mcheck(lib().symnmf_mlp_num_params(net.handle, ctypes.byref(c)), net)
    return c.value


def symnmf_mlp_set_params(net, params):
    assert params.is_contiguous() and params.numel() == symnmf_mlp_num_params(net)
    _mcheck(lib().symnmf_mlp_set_params(net.handle, params.data_ptr()), net)


def symnmf_mlp_get_params(net, out):
    assert out.is_contiguous() and out.numel() == symnmf_mlp_num_params(net)
    _mcheck(lib().symnmf_mlp_get_params(net.handle, out.data_ptr()), net)


def symnmf_mlp_forward(net, F, Y):
    assert F.is_contiguous() and Y.is_contiguous() and F.shape[0] == Y.numel() and F.shape[1] == MLP_FEATURES
    _mcheck(lib().symnmf_mlp_forward(net.handle, F.data_ptr(), int(F.shape[0]), Y.data_ptr()), net)


def symnmf_mlp_gradient(net, F, T, grad):
    assert F.is_contiguous() and T.is_contiguous() and grad.is_contiguous()
    loss = ctypes.c_double()
    _mcheck(lib().symnmf_mlp_gradient(net.handle, F.data_ptr(), T.data_ptr(), int(F.shape[0]), grad.data_ptr(),
                                      ctypes.byref(loss)), net)
    return loss.value


def symnmf_mlp_train_step(net, F, T, lr, want_loss=True):
    assert F.is_contiguous() and T.is_contiguous() and F.shape[0] == T.numel()
    loss = ctypes.c_double()
    _mcheck(lib().symnmf_mlp_train_step(net.handle, F.data_ptr(), T.data_ptr(), int(F.shape[0]), float(lr),
                                        ctypes.byref(loss) if want_loss else None), net)
    return loss.value if want_loss else None


def symnmf_mlp_destroy(net):
    h, net.handle = net.handle, None
    if h:
        lib().symnmf_mlp_destroy(h)


def symnmf_warm_features(ctx, F):
    assert F.is_contiguous() and F.numel() == ctx.n * ctx.k * MLP_FEATURES
    _check(lib().symnmf_warm_features(ctx.handle, F.data_ptr()), ctx.handle)


def symnmf_warmstart(ctx, net, want_beta=True):
    """Returns beta (synchronises), or None with want_beta=False (stream-ordered;
    the value is then in symnmf_get_stats(ctx).warm_beta)."""
    beta = ctypes.c_double()
    _check(lib().symnmf_warmstart(ctx.handle, net.handle, ctypes.byref(beta) if want_beta else None), ctx.handle)
    return beta.value if want_beta else None


def symnmf_warmstart_noalloc(ctx, net, want_beta=True):
    """symnmf_warmstart with its temporaries in the library's static device
    scratch (no device allocation); same return value."""
    beta = ctypes.c_double()
    _check(lib().symnmf_warmstart_noalloc(ctx.handle, net.handle, ctypes.byref(beta) if want_beta else None),
           ctx.handle)
    return beta.value if want_beta else None
