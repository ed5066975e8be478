"""ctypes binding of ``liblrsdp.so`` (the C ABI declared in include/lrsdp.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Device buffers are torch tensors on the context's device; their
pointers are handed to the library, which never allocates on the solve path.
The binding raises ``LrsdpUnavailable`` when the built library is missing; it
has no fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblrsdp.so")

OK, NOT_CONVERGED = 0, 1
EINVAL, ENOMEM, EHIP, ENUMERIC, EUNSUPPORTED = -1, -2, -3, -4, -5
F64, F32, F32_BF16IN = 0, 1, 2
MAXCUT, COMPLETION, GENERAL = 1, 2, 3
C_AUTO, C_SPARSE, C_DENSE = 0, 1, 2
ORDER_INPUT, ORDER_DEGREE = 0, 1


class LrsdpUnavailable(ImportError):
    pass


class LrsdpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lrsdp error {code}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [
        ("prec", C.c_int), ("rank", C.c_int), ("ld", C.c_int), ("lbfgs_mem", C.c_int),
        ("tol", C.c_double), ("max_outer", C.c_int), ("max_inner", C.c_int),
        ("max_iter_total", C.c_int64), ("time_limit_s", C.c_double),
        ("sigma0", C.c_double), ("sigma_factor", C.c_double), ("sigma_max_ratio", C.c_double),
        ("feas_decrease", C.c_double), ("eta0", C.c_double), ("eta_factor", C.c_double),
        ("eta_min", C.c_double), ("check_every", C.c_int), ("refresh_every", C.c_int),
        ("profile", C.c_int), ("verbose", C.c_int), ("phase2", C.c_int), ("switch_err1", C.c_double),
        ("admm_check", C.c_int), ("max_admm", C.c_int), ("precond", C.c_int),
        ("rank_max", C.c_int), ("rank_trigger", C.c_int), ("rank_scale", C.c_double), ("rank_seed", C.c_int64),
        ("reopt", C.c_int), ("reopt_factor", C.c_double), ("max_reopt", C.c_int), ("cert_iters", C.c_int),
    ]


class Result(C.Structure):
    _fields_ = [
        ("obj", C.c_double), ("dual", C.c_double), ("err1", C.c_double), ("err1_inf", C.c_double),
        ("err3", C.c_double), ("sigma", C.c_double), ("seconds", C.c_double),
        ("outer", C.c_int64), ("inner", C.c_int64), ("status", C.c_int),
        ("spmm_launches", C.c_int), ("spmm_ms", C.c_double), ("spmm_bytes", C.c_double),
        ("admm_iters", C.c_int64), ("admm_fallbacks", C.c_int64), ("rank_final", C.c_int64),
        ("reopt_rounds", C.c_int64), ("err2", C.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ProblemInfo(C.Structure):
    _fields_ = [
        ("kind", C.c_int), ("n", C.c_int64), ("m", C.c_int64), ("nnz", C.c_int64),
        ("n1", C.c_int64), ("n2", C.c_int64), ("weights", C.c_int), ("max_row_nnz", C.c_int64),
        ("c_l1", C.c_double), ("b_l1", C.c_double), ("b_inf", C.c_double), ("c_dense", C.c_int),
        ("node_order", C.c_int),
    ]


class Cert(C.Structure):
    _fields_ = [
        ("lambda_min", C.c_double), ("resid", C.c_double), ("lambda_lb", C.c_double),
        ("dual_bound", C.c_double), ("err2", C.c_double), ("by", C.c_double),
        ("iters", C.c_int64), ("status", C.c_int), ("block", C.c_int), ("lambda_max", C.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Proof(C.Structure):
    _fields_ = [
        ("shift", C.c_double), ("lambda_lb", C.c_double), ("margin", C.c_double), ("dual_bound", C.c_double),
        ("by", C.c_double), ("pivot", C.c_int64), ("status", C.c_int), ("reserved", C.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


PROOF_MAX_N = 8192

_P = C.c_void_p
_I64 = C.c_int64
_SIGS = {
    "lrsdp_last_error": (C.c_char_p, []),
    "lrsdp_version": (C.c_char_p, []),
    "lrsdp_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "lrsdp_ctx_destroy": (None, [_P]),
    "lrsdp_problem_maxcut": (C.c_int, [_I64, _I64, _P, _P, _P, C.POINTER(_P)]),
    "lrsdp_problem_maxcut_ex": (C.c_int, [_I64, _I64, _P, _P, _P, C.c_int, C.POINTER(_P)]),
    "lrsdp_problem_completion": (C.c_int, [_I64, _I64, _I64, _P, _P, _P, C.POINTER(_P)]),
    "lrsdp_problem_general": (C.c_int, [_I64, _I64, _P, _P, _P, _I64, _I64, _P, _P, _P, _P, _P, C.POINTER(_P)]),
    "lrsdp_problem_general_ex": (C.c_int, [_I64, _I64, _P, _P, _P, _I64, _I64, _P, _P, _P, _P, _P, C.c_int,
                                           C.POINTER(_P)]),
    "lrsdp_problem_block_ranks": (C.c_int, [_P, _P]),
    "lrsdp_problem_general_blocks": (C.c_int, [_I64, _P, _I64, _P, _P, _P, _P, _I64, _I64, _P, _P, _P, _P, _P, _P,
                                               C.POINTER(_P)]),
    "lrsdp_problem_destroy": (None, [_P]),
    "lrsdp_problem_get_info": (C.c_int, [_P, C.POINTER(ProblemInfo)]),
    "lrsdp_problem_device_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "lrsdp_problem_upload": (C.c_int, [_P, _P, _P, C.c_size_t]),
    "lrsdp_options_default": (None, [C.POINTER(Options)]),
    "lrsdp_workspace_bytes": (C.c_int, [_P, C.POINTER(Options), C.POINTER(C.c_size_t)]),
    "lrsdp_solve": (C.c_int, [_P, _P, C.POINTER(Options), _P, C.c_size_t, _P, _P, C.POINTER(Result)]),
    "lrsdp_k_spmm": (C.c_int, [_P, _P, C.c_int, _P, _I64, _P, _P]),
    "lrsdp_k_constraint": (C.c_int, [_P, _P, C.c_int, _P, _P, _I64, _P]),
    "lrsdp_k_ls_coeffs": (C.c_int, [_P, _P, C.c_int, _P, _P, _I64, _P, C.c_double, _P, _P, _P, _P]),
    "lrsdp_k_cubic": (C.c_int, [_P, _P, _P]),
    "lrsdp_k_alm": (C.c_int, [_P, _P, C.c_int, _P, _I64, _P, C.c_double, _P, _P]),
    "lrsdp_k_alm_noalloc": (C.c_int, [_P, _P, C.c_int, _P, _I64, _P, C.c_double, _P]),
    "lrsdp_k_alm_noalloc_max_bytes": (C.c_size_t, []),
    "lrsdp_k_lbfgs_dir": (C.c_int, [_P, C.c_int, _I64, _I64, _P, _P, _P, C.c_int, _P]),
    "lrsdp_k_admm": (C.c_int, [_P, _P, C.c_int, _P, _P, _I64, _P, C.c_double, C.c_int, C.c_double, C.c_int, _P,
                                C.c_size_t]),
    "lrsdp_admm_workspace_bytes": (C.c_int, [_P, C.c_int, _I64, C.POINTER(C.c_size_t)]),
    "lrsdp_mlp_param_count": (C.c_int, []),
    "lrsdp_ws_features": (C.c_int, [_P, _P, _P, _P]),
    "lrsdp_mlp_forward": (C.c_int, [_P, _P, C.c_int, _P, _I64, _P]),
    "lrsdp_mlp_grad": (C.c_int, [_P, _P, C.c_int, _P, _P, _I64, _P, _P, _P]),
    "lrsdp_mlp_adam": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, C.c_float]),
    "lrsdp_mlp_train": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _I64, C.c_int, C.c_int, C.c_float, _P, _P]),
    "lrsdp_mlp_train_work_floats": (C.c_int, []),
    "lrsdp_warmstart": (C.c_int, [_P, _P, _P, C.c_int, C.c_double, C.c_double, _P, _P, C.POINTER(C.c_double)]),
    "lrsdp_ws_targets": (C.c_int, [_P, _P, _P, _P, C.c_double, _P]),
    "lrsdp_certify_workspace_bytes": (C.c_int, [_P, C.c_int, C.POINTER(C.c_size_t)]),
    "lrsdp_certify": (C.c_int, [_P, _P, _P, C.c_int, C.c_double, C.c_uint64, _P, C.c_size_t, C.POINTER(Cert)]),
    "lrsdp_certify_dense": (C.c_int, [_P, _P, C.c_double, C.POINTER(Proof)]),
}

_lib = None


def load():
    """Load the built library (raises LrsdpUnavailable if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LrsdpUnavailable(
            f"{LIB_PATH} not found: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


def _check(rc):
    if rc < 0:
        raise LrsdpError(rc, load().lrsdp_last_error().decode())
    return rc


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def default_options(**kw) -> Options:
    o = Options()
    load().lrsdp_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def padded_ld(rank: int, prec: int) -> int:
    """Smallest row stride >= rank whose row bytes are a multiple of 16 (the
    float32 stride for LRSDP_F32_BF16IN)."""
    per = 2 if prec == F64 else 4
    return ((rank + per - 1) // per) * per


def elem_dtype(prec: int):
    import torch
    return torch.float64 if prec == F64 else torch.float32


class Context:
    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load()
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = C.c_void_p()
        _check(lib.lrsdp_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().lrsdp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """Host-built problem; ``upload`` places it in a torch-owned device buffer."""

    def __init__(self, handle, nblocks=1):
        self.handle = handle
        self.dev = None
        self.nblocks = nblocks   # blocks of a general problem (lrsdp_problem_block_ranks reads one rank each)

    @classmethod
    def maxcut(cls, n, u, v, w=None, node_order=None):
        """node_order: None or ORDER_INPUT (lrsdp_problem_maxcut), ORDER_DEGREE
        (lrsdp_problem_maxcut_ex)."""
        lib = load()
        ua, up = _host(u, np.int32)
        va, vp = _host(v, np.int32)
        if w is not None:
            wa, wp = _host(w, np.float64)
        else:
            wp = None
        h = C.c_void_p()
        if node_order is None:
            _check(lib.lrsdp_problem_maxcut(int(n), len(ua), up, vp, wp, C.byref(h)))
        else:
            _check(lib.lrsdp_problem_maxcut_ex(int(n), len(ua), up, vp, wp, int(node_order), C.byref(h)))
        return cls(h)

    @classmethod
    def completion(cls, n1, n2, i, j, Mij):
        lib = load()
        ia, ip = _host(i, np.int32)
        ja, jp = _host(j, np.int32)
        ma, mp = _host(Mij, np.float64)
        h = C.c_void_p()
        _check(lib.lrsdp_problem_completion(int(n1), int(n2), len(ia), ip, jp, mp, C.byref(h)))
        return cls(h)

    @classmethod
    def general(cls, n, c_row, c_col, c_val, m, a_con, a_row, a_col, a_val, b, c_storage=None):
        """min <C, X> s.t. <A_k, X> = b_k: C and the A_k as triplets, each
        off-diagonal entry given once (it stands for both (r, c) and (c, r)).
        c_storage: None (automatic), C_SPARSE or C_DENSE."""
        lib = load()
        cr, crp = _host(c_row, np.int32)
        cc, ccp = _host(c_col, np.int32)
        cv, cvp = _host(c_val, np.float64)
        ak, akp = _host(a_con, np.int32)
        ar, arp = _host(a_row, np.int32)
        ac, acp = _host(a_col, np.int32)
        av, avp = _host(a_val, np.float64)
        bb, bp = _host(b, np.float64)
        if not (len(cr) == len(cc) == len(cv)) or not (len(ak) == len(ar) == len(ac) == len(av)) or len(bb) != m:
            raise ValueError("triplet arrays of different lengths, or len(b) != m")
        h = C.c_void_p()
        _check(lib.lrsdp_problem_general_ex(int(n), len(cr), crp, ccp, cvp, int(m), len(ak), akp, arp, acp, avp, bp,
                                            C_AUTO if c_storage is None else int(c_storage), C.byref(h)))
        return cls(h)

    @classmethod
    def general_blocks(cls, block_n, c_blk, c_row, c_col, c_val, m, a_con, a_blk, a_row, a_col, a_val, b,
                       block_rank=None):
        """Several PSD blocks laid out one after another in one factor; triplets
        carry a block id and block-local indices."""
        lib = load()
        bn, bnp = _host(block_n, np.int64)
        arrs = [_host(x, t) for x, t in ((c_blk, np.int32), (c_row, np.int32), (c_col, np.int32), (c_val, np.float64),
                                         (a_con, np.int32), (a_blk, np.int32), (a_row, np.int32), (a_col, np.int32),
                                         (a_val, np.float64), (b, np.float64))]
        (cb, cbp), (cr, crp), (cc, ccp), (cv, cvp), (ak, akp), (ab, abp), (ar, arp), (ac, acp), (av, avp), (bb, bp) = arrs
        if not (len(cb) == len(cr) == len(cc) == len(cv)) or not (len(ak) == len(ab) == len(ar) == len(ac) == len(av)) \
                or len(bb) != m:
            raise ValueError("triplet arrays of different lengths, or len(b) != m")
        h = C.c_void_p()
        _check(lib.lrsdp_problem_general_blocks(len(bn), bnp, len(cb), cbp, crp, ccp, cvp, int(m), len(ak), akp, abp,
                                                arp, acp, avp, bp, C.byref(h)))
        prob = cls(h, nblocks=len(bn))
        if block_rank is not None:
            prob.set_block_ranks(block_rank)
        return prob

    def set_block_ranks(self, block_rank):
        """lrsdp_problem_block_ranks: the rank of each block's factor (before upload)."""
        ra, rp = _host(block_rank, np.int32)
        if len(ra) != self.nblocks:
            raise ValueError(f"{len(ra)} block ranks for {self.nblocks} blocks")
        _check(load().lrsdp_problem_block_ranks(self.handle, rp))
        return self

    @property
    def info(self) -> ProblemInfo:
        inf = ProblemInfo()
        _check(load().lrsdp_problem_get_info(self.handle, C.byref(inf)))
        return inf

    def device_bytes(self) -> int:
        b = C.c_size_t()
        _check(load().lrsdp_problem_device_bytes(self.handle, C.byref(b)))
        return b.value

    def upload(self, ctx: Context):
        import torch
        nbytes = self.device_bytes()
        self.dev = torch.empty(nbytes, dtype=torch.uint8, device=ctx.torch_device)
        _check(load().lrsdp_problem_upload(ctx.handle, self.handle, _ptr(self.dev), nbytes))
        return self

    def close(self):
        if getattr(self, "handle", None):
            load().lrsdp_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(prob: Problem, opts: Options) -> int:
    b = C.c_size_t()
    _check(load().lrsdp_workspace_bytes(prob.handle, C.byref(opts), C.byref(b)))
    return b.value


def solve(ctx: Context, prob: Problem, R, y, opts: Options, workspace=None):
    """Run the solve in place on device tensors R (n x ld) and y (m, float64).

    Returns (status, Result).  ``workspace`` may be a preallocated uint8 device
    tensor of at least ``workspace_bytes`` bytes.
    """
    import torch
    need = workspace_bytes(prob, opts)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=ctx.torch_device)
    res = Result()
    rc = _check(load().lrsdp_solve(ctx.handle, prob.handle, C.byref(opts), _ptr(workspace),
                                   workspace.numel(), _ptr(R), _ptr(y), C.byref(res)))
    return rc, res


# ---- kernel entry points --------------------------------------------------------
def k_spmm(ctx, prob, prec, V, ytil, Y):
    _check(load().lrsdp_k_spmm(ctx.handle, prob.handle, prec, _ptr(V), V.shape[1], _ptr(ytil), _ptr(Y)))


def k_constraint(ctx, prob, prec, U, V, out):
    _check(load().lrsdp_k_constraint(ctx.handle, prob.handle, prec, _ptr(U), _ptr(V), U.shape[1], _ptr(out)))


def k_ls_coeffs(ctx, prob, prec, R, D, y, sigma, work, out, q1=None, q2=None):
    _check(load().lrsdp_k_ls_coeffs(ctx.handle, prob.handle, prec, _ptr(R), _ptr(D), R.shape[1], _ptr(y),
                                    float(sigma), _ptr(work), _ptr(out), _ptr(q1), _ptr(q2)))


def k_cubic(ctx, a, tau):
    _check(load().lrsdp_k_cubic(ctx.handle, _ptr(a), _ptr(tau)))


def k_alm(ctx, prob, prec, R, y, sigma, work, out):
    _check(load().lrsdp_k_alm(ctx.handle, prob.handle, prec, _ptr(R), R.shape[1], _ptr(y), float(sigma),
                              _ptr(work), _ptr(out)))


def k_alm_noalloc(ctx, prob, prec, R, y, sigma, out):
    """lrsdp_k_alm without a caller work buffer (the library's static array)."""
    _check(load().lrsdp_k_alm_noalloc(ctx.handle, prob.handle, prec, _ptr(R), R.shape[1], _ptr(y), float(sigma),
                                      _ptr(out)))


def k_alm_noalloc_max_bytes() -> int:
    return load().lrsdp_k_alm_noalloc_max_bytes()


def k_lbfgs_dir(ctx, prec, G, S, Y, D):
    k = len(S)
    sp = (C.c_void_p * max(k, 1))(*[t.data_ptr() for t in S])
    yp = (C.c_void_p * max(k, 1))(*[t.data_ptr() for t in Y])
    _check(load().lrsdp_k_lbfgs_dir(ctx.handle, prec, G.shape[0], G.shape[1], _ptr(G),
                                    C.cast(sp, C.c_void_p), C.cast(yp, C.c_void_p), k, _ptr(D)))


# ---- learned warm start ----------------------------------------------------------
def mlp_param_count() -> int:
    return load().lrsdp_mlp_param_count()


def ws_features(ctx, prob, feat, stats):
    _check(load().lrsdp_ws_features(ctx.handle, prob.handle, _ptr(feat), _ptr(stats)))


PARAM_F32, PARAM_BF16 = 0, 1


def _param_dtype(params):
    import torch
    if params.dtype == torch.float32:
        return PARAM_F32
    if params.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        return PARAM_BF16
    raise TypeError(f"MLP parameters must be float32 or bfloat16, not {params.dtype}")


def mlp_forward(ctx, params, feat, out):
    _check(load().lrsdp_mlp_forward(ctx.handle, _ptr(params), _param_dtype(params), _ptr(feat), feat.shape[0],
                                    _ptr(out)))


def mlp_grad(ctx, params, feat, target, grad, loss, work):
    _check(load().lrsdp_mlp_grad(ctx.handle, _ptr(params), _param_dtype(params), _ptr(feat), _ptr(target),
                                 feat.shape[0], _ptr(grad), _ptr(loss) if loss is not None else None, _ptr(work)))


def mlp_adam(ctx, params, m, v, grad, step, lr):
    _check(load().lrsdp_mlp_adam(ctx.handle, _ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(step), float(lr)))


def mlp_train_work_floats() -> int:
    return load().lrsdp_mlp_train_work_floats()


def mlp_train(ctx, master, params_bf16, m, v, feat, target, first_step, steps, lr, work, loss_hist=None):
    _check(load().lrsdp_mlp_train(ctx.handle, _ptr(master), _ptr(params_bf16), _ptr(m), _ptr(v), _ptr(feat),
                                  _ptr(target), feat.shape[0], int(first_step), int(steps), float(lr), _ptr(work),
                                  _ptr(loss_hist) if loss_hist is not None else None))


def warmstart(ctx, prob, params, work, y0, log_ratio_range=(-10.0, 10.0)):
    """Fill y0 (device float64) and return the predicted sigma0."""
    s = C.c_double()
    lo, hi = log_ratio_range
    _check(load().lrsdp_warmstart(ctx.handle, prob.handle, _ptr(params), _param_dtype(params), float(lo), float(hi),
                                  _ptr(work), _ptr(y0), C.byref(s)))
    return s.value


def ws_targets(ctx, prob, stats, y, sigma_final, target):
    _check(load().lrsdp_ws_targets(ctx.handle, prob.handle, _ptr(stats), _ptr(y), float(sigma_final),
                                   _ptr(target)))


def admm_workspace_bytes(prob, prec, ld):
    b = C.c_size_t()
    _check(load().lrsdp_admm_workspace_bytes(prob.handle, prec, ld, C.byref(b)))
    return b.value


def k_admm(ctx, prob, prec, U, V, y, sigma, iters, cg_tol=1e-12, cg_max=1000, work=None):
    """Splitting iterations in place (completion, general: CG half-steps; `work` is
    allocated here when None)."""
    import torch
    nb = admm_workspace_bytes(prob, prec, U.shape[1])
    if work is None and nb:
        work = torch.empty(nb, dtype=torch.uint8, device=U.device)
    wb = 0 if work is None else work.numel() * work.element_size()
    _check(load().lrsdp_k_admm(ctx.handle, prob.handle, prec, _ptr(U), _ptr(V), U.shape[1], _ptr(y),
                               float(sigma), int(iters), float(cg_tol), int(cg_max), _ptr(work), wb))


def certify_workspace_bytes(prob, max_iter):
    b = C.c_size_t()
    _check(load().lrsdp_certify_workspace_bytes(prob.handle, max_iter, C.byref(b)))
    return b.value


def certify(ctx, prob, y, max_iter=300, tol=1e-6, seed=15049, work=None):
    """Smallest eigenvalue of C - A*(y) (y: device float64) and the dual bound it
    gives; returns a Cert.  `work` is a device uint8 tensor (allocated here if None)."""
    import torch
    if work is None:
        work = torch.empty(certify_workspace_bytes(prob, max_iter), dtype=torch.uint8, device=ctx.torch_device)
    out = Cert()
    _check(load().lrsdp_certify(ctx.handle, prob.handle, _ptr(y), max_iter, tol, seed, _ptr(work),
                                work.numel() * work.element_size(), C.byref(out)))
    return out


def certify_dense(prob, y, shift):
    """lrsdp_certify_dense: proof that lambda_min(C - A*(y)) >= shift - margin
    (host Cholesky of C - A*(y) - shift I; y: host float64, m entries); returns a
    Proof (status 0: proven, 1: the factorisation failed at `pivot`)."""
    ya, yp = _host(y, np.float64)
    if len(ya) != prob.info.m:
        raise ValueError(f"y has {len(ya)} entries, the problem {prob.info.m}")
    out = Proof()
    _check(load().lrsdp_certify_dense(prob.handle, yp, float(shift), C.byref(out)))
    return out
