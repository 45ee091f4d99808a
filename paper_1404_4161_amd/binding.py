"""Thin ctypes binding of libchfsi.so (include/chfsi.h).

Argument marshalling only: every step runs in the library's HIP kernels.
Matrices are torch complex128 tensors on the GPU in COLUMN-MAJOR layout
(stride(0) == 1); ``colmajor(t)`` makes such a copy.  Workspaces are
allocated with torch when not given.  The functions carry the C names.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import (POINTER, Structure, c_char, c_double, c_float, c_int, c_longlong,
                    c_size_t, c_ulonglong, c_void_p)

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchfsi.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "chfsi.h")

CHFSI_OK, CHFSI_INVALID_ARG, CHFSI_NOT_HPD, CHFSI_NO_CONVERGENCE = 0, 1, 2, 3
CHFSI_NONFINITE, CHFSI_DEVICE_ERROR, CHFSI_ALLOC_ERROR = 4, 5, 6
CHFSI_LOG_FIELDS = 24
CHFSI_MLP_FEATURES = 8
CHFSI_MLP_PARAMS = 4818


class ChfsiOpts(Structure):
    _fields_ = [("tol", c_double), ("deg0", c_int), ("deg_max", c_int), ("max_iter", c_int),
                ("lanczos_steps", c_int), ("alpha_rule", c_int), ("degree_mode", c_int),
                ("reuse_b_factor", c_int), ("precision", c_int), ("seed", c_ulonglong),
                ("degree_jitter", c_double), ("first_rule", c_int), ("log_capacity", c_int),
                ("log", POINTER(c_double)), ("mlp", POINTER(c_float)),
                ("seq_rates", POINTER(c_double)), ("rr_refine", c_int)]


class ChfsiInfo(Structure):
    _fields_ = [("iters", c_int), ("converged", c_int), ("filter_launches", c_int),
                ("cholqr_shifted", c_int), ("b_factor_reused", c_int),
                ("filter_iters_fp32", c_int),
                ("matvecs", c_longlong),
                ("filter_matvecs", c_longlong), ("filter_flops", c_double),
                ("filter_seconds", c_double), ("total_seconds", c_double),
                ("max_resid", c_double), ("beta", c_double), ("norm_h", c_double),
                ("step_seconds", c_double * 8), ("filter_flops_fp32", c_double),
                ("filter_seconds_fp32", c_double), ("log_records", c_int),
                ("learned_cols", c_int), ("fallback_cols", c_int), ("learned_raised", c_int),
                ("filter_steps_bf16", c_int), ("filter_flops_bf16", c_double),
                ("rr_refined", c_int), ("rr_dense", c_int),
                ("filter_steps_fp16", c_int), ("filter_flops_fp16", c_double),
                ("filter_flops_fp64_mfma", c_double)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "step_seconds"}
        d["step_seconds"] = list(self.step_seconds)
        return d


_SIGS = {
    "chfsi_default_opts": (c_int, [POINTER(ChfsiOpts)]),
    "chfsi_workspace_bytes": (c_size_t, [c_int, c_int, c_int, c_int, POINTER(ChfsiOpts)]),
    "chfsi_solve": (c_int, [c_int, c_int, c_int, c_void_p, c_int, c_void_p, c_int, c_double,
                            c_void_p, c_int, POINTER(c_double), POINTER(c_double), c_void_p, c_int,
                            c_void_p, c_size_t, POINTER(ChfsiOpts), c_void_p, POINTER(ChfsiInfo)]),
    "chfsi_status_string": (ctypes.c_char_p, [c_int]),
    "chfsi_batch_workspace_bytes": (c_size_t, [c_int, POINTER(ChfsiOpts)]),
    "chfsi_solve_batch": (c_int, [c_int, POINTER(c_int), POINTER(c_int), POINTER(c_int),
                                  POINTER(c_void_p), POINTER(c_int), POINTER(c_void_p),
                                  POINTER(c_int), c_double, POINTER(c_void_p), POINTER(c_int),
                                  POINTER(POINTER(c_double)), POINTER(POINTER(c_double)),
                                  POINTER(c_void_p), POINTER(c_int), POINTER(c_void_p),
                                  POINTER(c_size_t), c_void_p, c_size_t, POINTER(ChfsiOpts), c_int,
                                  c_void_p, POINTER(ChfsiInfo), POINTER(c_int)]),
    "chfsi_step_workspace_bytes": (c_size_t, [c_int, c_int]),
    "chfsi_filter": (c_int, [c_int, c_int, c_void_p, c_int, c_void_p, c_int, POINTER(c_int),
                             c_double, c_double, c_double, c_void_p, c_size_t, c_void_p,
                             POINTER(c_double), POINTER(c_int)]),
    "chfsi_defect_workspace_bytes": (c_size_t, [c_int, c_int]),
    "chfsi_filter_defect": (c_int, [c_int, c_int, c_void_p, c_int, c_void_p, c_int, c_void_p,
                                    c_int, POINTER(c_double), POINTER(c_int), c_double, c_double,
                                    c_double, c_void_p, c_int, c_void_p, c_size_t, c_void_p,
                                    POINTER(c_double)]),
    "chfsi_defect_split_workspace_bytes": (c_size_t, [c_int, c_int]),
    "chfsi_filter_defect_split": (c_int, [c_int, c_int, c_void_p, c_int, c_void_p, c_int,
                                          c_void_p, c_int, POINTER(c_double), POINTER(c_int),
                                          c_double, c_double, c_double, c_int, c_void_p, c_int,
                                          c_void_p, c_size_t, c_void_p, POINTER(c_double),
                                          POINTER(c_double)]),
    "chfsi_filter_defect_fp16": (c_int, [c_int, c_int, c_void_p, c_int, c_void_p, c_int,
                                         c_void_p, c_int, POINTER(c_double), POINTER(c_int),
                                         c_double, c_double, c_double, c_int, c_void_p, c_int,
                                         c_void_p, c_size_t, c_void_p, POINTER(c_double),
                                         POINTER(c_double)]),
    "chfsi_eigh_workspace_bytes": (c_size_t, [c_int]),
    "chfsi_eigh_projected": (c_int, [c_int, c_void_p, c_int, c_void_p, c_int, POINTER(c_double),
                                     c_int, c_void_p, c_size_t, c_void_p, POINTER(c_int)]),
    "chfsi_orthonormalize": (c_int, [c_int, c_int, c_void_p, c_int, c_int, c_void_p, c_int,
                                     c_void_p, c_size_t, c_void_p, POINTER(c_int)]),
    "chfsi_rayleigh_ritz": (c_int, [c_int, c_int, c_void_p, c_int, c_void_p, c_int, c_void_p,
                                    c_int, POINTER(c_double), POINTER(c_double), c_void_p,
                                    c_size_t, c_void_p]),
    "chfsi_lanczos_bounds": (c_int, [c_int, c_void_p, c_int, c_int, c_ulonglong, c_void_p,
                                     c_size_t, c_void_p, POINTER(c_double), POINTER(c_double),
                                     POINTER(c_double)]),
    "chfsi_filter_noalloc_need_bytes": (c_size_t, [c_int, c_int]),
    "chfsi_filter_noalloc": (c_int, [c_int, c_int, c_void_p, c_int, c_void_p, c_int,
                                     POINTER(c_int), c_double, c_double, c_double, c_void_p,
                                     POINTER(c_double), POINTER(c_int)]),
    "chfsi_reduce_workspace_bytes": (c_size_t, [c_int]),
    "chfsi_reduce_standard": (c_int, [c_int, c_void_p, c_int, c_void_p, c_int, c_void_p, c_int,
                                      c_void_p, c_int, c_void_p, c_size_t, c_void_p]),
    "chfsi_split_schedule": (c_int, [c_int, c_int, POINTER(c_double), POINTER(c_double),
                                     POINTER(c_int), c_double, c_double, c_double, c_double,
                                     c_int, POINTER(ctypes.c_byte)]),
    "chfsi_degrees": (c_int, [c_int, POINTER(c_double), POINTER(c_double), c_int, c_double,
                              c_double, c_double, c_int, POINTER(c_int)]),
    "chfsi_degree_features": (c_int, [c_double, c_double, c_double, c_double, c_double, c_double,
                                      c_double, c_double, c_int, POINTER(c_double)]),
    "chfsi_degrees_learned": (c_int, [c_int, POINTER(c_double), POINTER(c_double), c_int, c_double,
                                      c_double, c_double, c_double, c_double, c_int, c_int,
                                      POINTER(c_float), c_void_p, c_size_t, c_void_p,
                                      POINTER(c_int), POINTER(c_float), POINTER(c_int)]),
    "chfsi_degrees_sequence": (c_int, [c_int, POINTER(c_double), POINTER(c_double),
                                       POINTER(c_double), c_int, c_double, c_double, c_double,
                                       c_int, POINTER(c_int), POINTER(c_int)]),
    "chfsi_mlp_workspace_bytes": (c_size_t, [c_int]),
    "chfsi_mlp_forward": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "chfsi_mlp_gradient": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_size_t, c_void_p]),
    "chfsi_mlp_adam": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_int, c_void_p]),
    "chfsi_mlp_train": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_int, c_float, c_void_p,
                                c_size_t, c_void_p, POINTER(c_float)]),
    "chfsi_autotune_workspace_bytes": (c_size_t, [c_int, c_int]),
    "chfsi_autotune_filter": (c_int, [c_int, POINTER(c_int), POINTER(c_int), c_void_p, c_size_t,
                                      c_void_p, POINTER(c_int), POINTER(c_double)]),
    "chfsi_autotune_set": (c_int, [c_int, c_int, c_int]),
    "chfsi_autotune_reset": (c_int, []),
    "chfsi_zgemm": (c_int, [c_char, c_char, c_int, c_int, c_int, POINTER(c_double), c_void_p,
                            c_int, c_void_p, c_int, POINTER(c_double), c_void_p, c_int, c_void_p,
                            c_size_t, c_void_p]),
}

_lib = None


class ChfsiError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: status {status} ({chfsi_status_string(status)})")
        self.status = status


def lib():
    """Load libchfsi.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1404_4161_amd.build`")
        # torch first: its HIP runtime (libamdhip64, soname libamdhip64.so.7)
        # is then the one libchfsi.so binds to.  Loaded the other way round,
        # the process would hold two HIP runtimes and only one of them can
        # open the GPU.
        _torch()
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def header_functions():
    """Names of the functions include/chfsi.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chfsi_[a-z_0-9]+)\s*\(", text)))


# ---------------------------------------------------------------------------
# torch helpers

def _torch():
    import torch
    return torch


def colmajor(t):
    """Column-major copy (stride(0) == 1) of a 2-D tensor."""
    return t.transpose(0, 1).contiguous().transpose(0, 1)


def _ld(t):
    if t.dim() == 2 and t.numel() == 0:
        return max(t.shape[0], 1)
    if t.dim() != 2 or (t.stride(0) != 1 and t.shape[0] > 1):
        raise ValueError("expected a column-major 2-D tensor (stride(0) == 1)")
    return max(t.stride(1), t.shape[0], 1)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream, device):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _work(nbytes, device, work=None):
    torch = _torch()
    if work is not None:
        if work.numel() * work.element_size() < nbytes:
            raise ValueError("workspace too small")
        return work
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _check(status, where):
    if status != CHFSI_OK:
        raise ChfsiError(status, where)


# ---------------------------------------------------------------------------
# C ABI wrappers (same names)

def chfsi_default_opts():
    o = ChfsiOpts()
    _check(lib().chfsi_default_opts(ctypes.byref(o)), "chfsi_default_opts")
    return o


def chfsi_status_string(status):
    return lib().chfsi_status_string(int(status)).decode()


def chfsi_workspace_bytes(n, nev, nex, generalized, opts=None):
    return int(lib().chfsi_workspace_bytes(n, nev, nex, int(bool(generalized)),
                                           ctypes.byref(opts) if opts is not None else None))


def chfsi_solve(A, B, nev, nex, tol, X0=None, opts=None, X=None, work=None, stream=None,
                raise_on_error=True, Lambda0=None, log=None, mlp=None, seq_rates=None):
    """Solve A x = lambda B x (B None: standard).  Lambda0: the Ritz values
    that go with X0 (optional).  log: float64 numpy array (cap, 24) that
    receives convergence records (opts.log / log_capacity); mlp: float32
    numpy blob of the degree network (opts.mlp); seq_rates: float64 numpy
    array of k per-vector speeds, in/out (opts.seq_rates).  Returns (status,
    Lambda[k] numpy, X (n x k column-major tensor), info dict)."""
    torch = _torch()
    n = A.shape[0]
    k = nev + nex
    dev = A.device
    if X is None:
        X = colmajor(torch.empty((n, k), dtype=torch.complex128, device=dev))
    o = ChfsiOpts.from_buffer_copy(opts if opts is not None else chfsi_default_opts())
    if log is not None:
        if log.dtype != np.float64 or not log.flags.c_contiguous or log.ndim != 2 \
                or log.shape[1] != CHFSI_LOG_FIELDS:
            raise ValueError("log must be a C-contiguous float64 array (cap, 24)")
        o.log = log.ctypes.data_as(POINTER(c_double))
        o.log_capacity = log.shape[0]
    if mlp is not None:
        if mlp.dtype != np.float32 or not mlp.flags.c_contiguous or mlp.size != CHFSI_MLP_PARAMS:
            raise ValueError("mlp must be a contiguous float32 blob of CHFSI_MLP_PARAMS entries")
        o.mlp = mlp.ctypes.data_as(POINTER(c_float))
    if seq_rates is not None:
        if seq_rates.dtype != np.float64 or not seq_rates.flags.c_contiguous \
                or seq_rates.size != k:
            raise ValueError("seq_rates must be a contiguous float64 array of k entries")
        o.seq_rates = seq_rates.ctypes.data_as(POINTER(c_double))
    wb = chfsi_workspace_bytes(n, nev, nex, B is not None, o)
    w = _work(wb, dev, work)
    lam = (c_double * k)()
    lam0 = None if Lambda0 is None else (c_double * k)(*[float(v) for v in Lambda0])
    info = ChfsiInfo()
    st = lib().chfsi_solve(n, nev, nex, _ptr(A), _ld(A), _ptr(B), _ld(B) if B is not None else 0,
                           float(tol), _ptr(X0), _ld(X0) if X0 is not None else 0, lam0, lam,
                           _ptr(X),
                           _ld(X), _ptr(w), wb, ctypes.byref(o), _stream(stream, dev),
                           ctypes.byref(info))
    if raise_on_error and st not in (CHFSI_OK, CHFSI_NO_CONVERGENCE):
        raise ChfsiError(st, "chfsi_solve")
    return st, np.array(lam[:]), X, info.as_dict()


def chfsi_step_workspace_bytes(n, k):
    return int(lib().chfsi_step_workspace_bytes(n, k))


def chfsi_filter(H, Y, degrees, c, e, gamma, work=None, stream=None):
    """Alg. 2 in place on Y; returns (flops, launches)."""
    n, k = Y.shape
    deg = (c_int * k)(*[int(x) for x in degrees])
    wb = chfsi_step_workspace_bytes(n, k)
    w = _work(wb, Y.device, work)
    fl = c_double(0.0)
    ln = c_int(0)
    _check(lib().chfsi_filter(n, k, _ptr(H), _ld(H), _ptr(Y), _ld(Y), deg, c, e, gamma, _ptr(w),
                              wb, _stream(stream, Y.device), ctypes.byref(fl), ctypes.byref(ln)),
           "chfsi_filter")
    return fl.value, ln.value


def chfsi_filter_noalloc_need_bytes(n, k):
    return int(lib().chfsi_filter_noalloc_need_bytes(n, k))


def chfsi_filter_noalloc(H, Y, degrees, c, e, gamma, stream=None):
    """chfsi_filter without a workspace (the library's static device
    scratch); in place on Y; returns (flops, launches)."""
    n, k = Y.shape
    deg = (c_int * k)(*[int(x) for x in degrees])
    fl = c_double(0.0)
    ln = c_int(0)
    _check(lib().chfsi_filter_noalloc(n, k, _ptr(H), _ld(H), _ptr(Y), _ld(Y), deg, c, e, gamma,
                                      _stream(stream, Y.device), ctypes.byref(fl),
                                      ctypes.byref(ln)),
           "chfsi_filter_noalloc")
    return fl.value, ln.value


def chfsi_filter_defect(H, Q, Z, mu, degrees, c, e, gamma, Y=None, work=None, stream=None):
    """Mixed-precision Alg. 2 on Ritz vectors Q (Z = H Q, Ritz values mu);
    returns (Y, executed FP32 flops)."""
    torch = _torch()
    n, k = Q.shape
    if Y is None:
        Y = colmajor(torch.empty((n, k), dtype=torch.complex128, device=Q.device))
    m = (c_double * k)(*[float(x) for x in mu])
    deg = (c_int * k)(*[int(x) for x in degrees])
    wb = int(lib().chfsi_defect_workspace_bytes(n, k))
    w = _work(wb, Q.device, work)
    fl = c_double(0.0)
    _check(lib().chfsi_filter_defect(n, k, _ptr(H), _ld(H), _ptr(Q), _ld(Q), _ptr(Z), _ld(Z), m,
                                     deg, c, e, gamma, _ptr(Y), _ld(Y), _ptr(w), wb,
                                     _stream(stream, Q.device), ctypes.byref(fl)),
           "chfsi_filter_defect")
    return Y, fl.value


def chfsi_filter_defect_split(H, Q, Z, mu, degrees, c, e, gamma, bf16_steps, Y=None, work=None,
                              stream=None, fp16=False):
    """chfsi_filter_defect with its first bf16_steps steps in BF16-split
    form (FP16-split with fp16=True: chfsi_filter_defect_fp16); returns (Y,
    split-step flops, FP32-step flops)."""
    torch = _torch()
    n, k = Q.shape
    if Y is None:
        Y = colmajor(torch.empty((n, k), dtype=torch.complex128, device=Q.device))
    m = (c_double * k)(*[float(x) for x in mu])
    deg = (c_int * k)(*[int(x) for x in degrees])
    wb = int(lib().chfsi_defect_split_workspace_bytes(n, k))
    w = _work(wb, Q.device, work)
    f16, f32 = c_double(0.0), c_double(0.0)
    name = "chfsi_filter_defect_fp16" if fp16 else "chfsi_filter_defect_split"
    _check(getattr(lib(), name)(n, k, _ptr(H), _ld(H), _ptr(Q), _ld(Q), _ptr(Z), _ld(Z), m, deg,
                                c, e, gamma, int(bf16_steps), _ptr(Y), _ld(Y), _ptr(w), wb,
                                _stream(stream, Q.device), ctypes.byref(f16),
                                ctypes.byref(f32)),
           name)
    return Y, f16.value, f32.value


def chfsi_eigh_projected(G, mode=1, W=None, work=None, stream=None):
    """Eigenpairs of the k x k Hermitian device matrix G (Rayleigh-Ritz's
    projected problem): mode 0 zheevd, 1 refinement with zheevd fallback,
    2 refinement only.  Returns (mu ascending numpy, W column-major tensor,
    refined flag)."""
    torch = _torch()
    k = G.shape[0]
    if W is None:
        W = colmajor(torch.empty((k, k), dtype=torch.complex128, device=G.device))
    mu = (c_double * k)()
    wb = int(lib().chfsi_eigh_workspace_bytes(k))
    w = _work(wb, G.device, work)
    ref = c_int(0)
    _check(lib().chfsi_eigh_projected(k, _ptr(G), _ld(G), _ptr(W), _ld(W), mu, int(mode), _ptr(w),
                                      wb, _stream(stream, G.device), ctypes.byref(ref)),
           "chfsi_eigh_projected")
    return np.array(mu[:]), W, ref.value


def chfsi_orthonormalize(Y, QL=None, work=None, stream=None):
    n, k = Y.shape
    nl = 0 if QL is None else QL.shape[1]
    wb = chfsi_step_workspace_bytes(n, max(k, nl))
    w = _work(wb, Y.device, work)
    sh = c_int(0)
    _check(lib().chfsi_orthonormalize(n, k, _ptr(Y), _ld(Y), nl, _ptr(QL),
                                      _ld(QL) if QL is not None else n, _ptr(w), wb,
                                      _stream(stream, Y.device), ctypes.byref(sh)),
           "chfsi_orthonormalize")
    return sh.value


def chfsi_rayleigh_ritz(H, Q, Z, work=None, stream=None):
    n, k = Q.shape
    mu = (c_double * k)()
    res = (c_double * k)()
    wb = chfsi_step_workspace_bytes(n, k)
    w = _work(wb, Q.device, work)
    _check(lib().chfsi_rayleigh_ritz(n, k, _ptr(H), _ld(H), _ptr(Q), _ld(Q), _ptr(Z), _ld(Z), mu,
                                     res, _ptr(w), wb, _stream(stream, Q.device)),
           "chfsi_rayleigh_ritz")
    return np.array(mu[:]), np.array(res[:])


def chfsi_lanczos_bounds(H, steps=20, seed=0, work=None, stream=None):
    n = H.shape[0]
    wb = chfsi_step_workspace_bytes(n, 1)
    w = _work(wb, H.device, work)
    up, lo, hi = c_double(), c_double(), c_double()
    _check(lib().chfsi_lanczos_bounds(n, _ptr(H), _ld(H), steps, seed, _ptr(w), wb,
                                      _stream(stream, H.device), ctypes.byref(up),
                                      ctypes.byref(lo), ctypes.byref(hi)),
           "chfsi_lanczos_bounds")
    return up.value, lo.value, hi.value


def chfsi_reduce_workspace_bytes(n):
    return int(lib().chfsi_reduce_workspace_bytes(n))


def chfsi_reduce_standard(A, B, H=None, L=None, work=None, stream=None):
    torch = _torch()
    n = A.shape[0]
    if H is None:
        H = colmajor(torch.empty((n, n), dtype=torch.complex128, device=A.device))
    if L is None:
        L = colmajor(torch.empty((n, n), dtype=torch.complex128, device=A.device))
    wb = chfsi_reduce_workspace_bytes(n)
    w = _work(wb, A.device, work)
    _check(lib().chfsi_reduce_standard(n, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(H), _ld(H),
                                       _ptr(L), _ld(L), _ptr(w), wb, _stream(stream, A.device)),
           "chfsi_reduce_standard")
    return H, L


def chfsi_degrees(mu, res, n_wanted, alpha, beta, tol_abs, deg_max=40):
    k = len(mu)
    m = (c_double * k)(*[float(x) for x in mu])
    r = (c_double * k)(*[float(x) for x in res])
    d = (c_int * k)()
    _check(lib().chfsi_degrees(k, m, r, int(n_wanted), float(alpha), float(beta), float(tol_abs),
                               int(deg_max), d), "chfsi_degrees")
    return np.array(d[:], dtype=np.int64)


def chfsi_split_schedule(mu, res, deg, n_wanted, c, e, tol, norm_h, form):
    """Per-step split forms of an FP32 defect filter (host only): array of
    max(deg) entries, 0 = FP32 step, form (1 BF16, 2 FP16) = split step."""
    k = len(deg)
    m = (c_double * k)(*[float(x) for x in mu])
    r = (c_double * k)(*[float(x) for x in res])
    d = (c_int * k)(*[int(x) for x in deg])
    out = (ctypes.c_byte * max(max(int(x) for x in deg), 1))()
    _check(lib().chfsi_split_schedule(int(n_wanted), k, m, r, d, float(c), float(e), float(tol),
                                      float(norm_h), int(form), out), "chfsi_split_schedule")
    return np.array(out[:], dtype=np.int64)


def chfsi_zgemm(opa, opb, alpha, A, B, beta, C, work=None, stream=None):
    M, N = C.shape
    K = A.shape[1] if opa in "Nn" else A.shape[0]
    al = (c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (c_double * 2)(complex(beta).real, complex(beta).imag)
    wb = 16 * max(M * N * 64, 1)
    w = _work(wb, C.device, work)
    _check(lib().chfsi_zgemm(opa.encode(), opb.encode(), M, N, K, al, _ptr(A), _ld(A), _ptr(B),
                             _ld(B), be, _ptr(C), _ld(C), _ptr(w), wb, _stream(stream, C.device)),
           "chfsi_zgemm")
    return C


def chfsi_degree_features(mu, res, gap, alpha, beta, gamma, norm_h, tol_abs, loop):
    """The 8 network inputs of one vector, or None when |t| <= 1."""
    f = (c_double * CHFSI_MLP_FEATURES)()
    st = lib().chfsi_degree_features(float(mu), float(res), float(gap), float(alpha), float(beta),
                                     float(gamma), float(norm_h), float(tol_abs), int(loop), f)
    return None if st != CHFSI_OK else np.array(f[:])


def _f32_blob(params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != CHFSI_MLP_PARAMS:
        raise ValueError("parameter blob must hold CHFSI_MLP_PARAMS floats")
    return p


def chfsi_degrees_learned(mu, res, n_wanted, alpha, beta, gamma, norm_h, tol_abs, loop, params,
                          deg_max=40, device="cuda", work=None, stream=None):
    """Learned degrees; returns (deg, pred, src) numpy arrays."""
    k = len(mu)
    p = _f32_blob(params)
    m = (c_double * k)(*[float(x) for x in mu])
    r = (c_double * k)(*[float(x) for x in res])
    d = (c_int * k)()
    pr = (c_float * k)()
    sr = (c_int * k)()
    wb = int(lib().chfsi_mlp_workspace_bytes(k))
    torch = _torch()
    dev = torch.device(device)
    w = _work(wb, dev, work)
    _check(lib().chfsi_degrees_learned(k, m, r, int(n_wanted), float(alpha), float(beta),
                                       float(gamma), float(norm_h), float(tol_abs), int(loop),
                                       int(deg_max), p.ctypes.data_as(POINTER(c_float)), _ptr(w),
                                       wb, _stream(stream, dev), d, pr, sr),
           "chfsi_degrees_learned")
    return (np.array(d[:], dtype=np.int64), np.array(pr[:], dtype=np.float32),
            np.array(sr[:], dtype=np.int64))


def _f32_dev(t, shape):
    torch = _torch()
    if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected a contiguous float32 tensor of shape {shape}")
    return t


def chfsi_mlp_forward(X, params, stream=None):
    """y = net(X) for X (n, 8) float32 on the GPU; returns y (n,)."""
    torch = _torch()
    n = X.shape[0]
    _f32_dev(X, (n, CHFSI_MLP_FEATURES))
    _f32_dev(params, (CHFSI_MLP_PARAMS,))
    y = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(lib().chfsi_mlp_forward(n, _ptr(X), _ptr(params), _ptr(y), _stream(stream, X.device)),
           "chfsi_mlp_forward")
    return y


def chfsi_mlp_gradient(X, T, params, work=None, stream=None):
    """Gradient of the mean squared error; returns (grad tensor, sum of
    squared errors)."""
    torch = _torch()
    n = X.shape[0]
    _f32_dev(X, (n, CHFSI_MLP_FEATURES))
    _f32_dev(T, (n,))
    _f32_dev(params, (CHFSI_MLP_PARAMS,))
    g = torch.empty(CHFSI_MLP_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    wb = int(lib().chfsi_mlp_workspace_bytes(n))
    w = _work(wb, X.device, work)
    _check(lib().chfsi_mlp_gradient(n, _ptr(X), _ptr(T), _ptr(params), _ptr(g), _ptr(loss),
                                    _ptr(w), wb, _stream(stream, X.device)),
           "chfsi_mlp_gradient")
    return g, float(loss.item())


def chfsi_mlp_adam(params, grad, m, v, lr, t, stream=None):
    """One Adam step in place on params (and the moments m, v)."""
    for x in (params, grad, m, v):
        _f32_dev(x, (CHFSI_MLP_PARAMS,))
    _check(lib().chfsi_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), float(lr), int(t),
                                _stream(stream, params.device)), "chfsi_mlp_adam")


def chfsi_mlp_train(X, T, params, steps, lr, work=None, stream=None):
    """`steps` full-batch Adam steps in place on params; returns the mean
    squared error before each step (numpy)."""
    n = X.shape[0]
    _f32_dev(X, (n, CHFSI_MLP_FEATURES))
    _f32_dev(T, (n,))
    _f32_dev(params, (CHFSI_MLP_PARAMS,))
    losses = (c_float * max(int(steps), 1))()
    wb = int(lib().chfsi_mlp_workspace_bytes(n))
    w = _work(wb, X.device, work)
    _check(lib().chfsi_mlp_train(n, _ptr(X), _ptr(T), _ptr(params), int(steps), float(lr), _ptr(w),
                                 wb, _stream(stream, X.device), losses), "chfsi_mlp_train")
    return np.array(losses[:int(steps)], dtype=np.float64)


def chfsi_batch_workspace_bytes(count, opts=None):
    return int(lib().chfsi_batch_workspace_bytes(int(count), ctypes.byref(opts)
                                                 if opts is not None else None))


def chfsi_solve_batch(As, Bs, nevs, nexs, tol, X0s=None, opts=None, Lambda0s=None, Xs=None,
                      works=None, stream=None, graph=False, raise_on_error=True, serial=False,
                      own_defect=False):
    """Solve len(As) independent problems in lockstep (grouped filter
    launches).  Bs / X0s / Lambda0s: lists (entries may be None) or None.
    Returns (status, [Lambda numpy], [X tensors], [info dicts], [statuses])."""
    torch = _torch()
    count = len(As)
    dev = As[0].device
    o = opts if opts is not None else chfsi_default_opts()
    ns = [a.shape[0] for a in As]
    ks = [nevs[q] + nexs[q] for q in range(count)]
    if Xs is None:
        Xs = [colmajor(torch.empty((ns[q], ks[q]), dtype=torch.complex128, device=dev))
              for q in range(count)]
    wbs = [chfsi_workspace_bytes(ns[q], nevs[q], nexs[q], Bs is not None and Bs[q] is not None, o)
           for q in range(count)]
    if works is None:
        works = [_work(wbs[q], dev) for q in range(count)]
    bw = chfsi_batch_workspace_bytes(count, o)
    bwork = _work(bw, dev)
    I = c_int * count
    P = c_void_p * count
    lam = [(c_double * ks[q])() for q in range(count)]
    lam_ptrs = (POINTER(c_double) * count)(*[ctypes.cast(x, POINTER(c_double)) for x in lam])
    lam0 = None
    keep = []
    if Lambda0s is not None:
        arrs = []
        for q in range(count):
            if Lambda0s[q] is None:
                arrs.append(None)
            else:
                a = (c_double * ks[q])(*[float(v) for v in Lambda0s[q]])
                keep.append(a)
                arrs.append(ctypes.cast(a, POINTER(c_double)))
        lam0 = (POINTER(c_double) * count)(*arrs)
    b_ptrs = b_lds = None
    if Bs is not None:
        b_ptrs = P(*[None if b is None else b.data_ptr() for b in Bs])
        b_lds = I(*[0 if b is None else _ld(b) for b in Bs])
    x0_ptrs = x0_lds = None
    if X0s is not None:
        x0_ptrs = P(*[None if x is None else x.data_ptr() for x in X0s])
        x0_lds = I(*[0 if x is None else _ld(x) for x in X0s])
    infos = (ChfsiInfo * count)()
    sts = I()
    st = lib().chfsi_solve_batch(
        count, I(*ns), I(*[int(v) for v in nevs]), I(*[int(v) for v in nexs]),
        P(*[a.data_ptr() for a in As]), I(*[_ld(a) for a in As]), b_ptrs, b_lds, float(tol),
        x0_ptrs, x0_lds, lam0, lam_ptrs, P(*[x.data_ptr() for x in Xs]), I(*[_ld(x) for x in Xs]),
        P(*[w.data_ptr() for w in works]), (c_size_t * count)(*wbs), _ptr(bwork), bw,
        ctypes.byref(o), (1 if graph else 0) | (2 if serial else 0) | (4 if own_defect else 0), _stream(stream, dev), infos,
        sts)
    if raise_on_error and st not in (CHFSI_OK, CHFSI_NO_CONVERGENCE):
        raise ChfsiError(st, "chfsi_solve_batch")
    return (st, [np.array(l[:]) for l in lam], Xs, [i.as_dict() for i in infos],
            [int(v) for v in sts])


# filter-step variants (CHFSI_FILTER_VARIANTS): 0 / 1 64 x 64 tiles, 4M
# split, K 8 / 16 deep; 2 128 x 128 tiles; 3 / 4 as 0 / 1 with the 3M split;
# 5 / 6 operands loaded straight into LDS, 3M / 4M
FILTER_VARIANTS = 7
DEFAULT_FILTER_VARIANT = 5   # taken where no shape was measured


def chfsi_autotune_filter(ns, Ns, device="cuda", stream=None):
    """Time the filter-step variants on each (n, N) launch shape and record
    the fastest; returns (variants, tflops (count x FILTER_VARIANTS,
    complex-equivalent)) numpy arrays."""
    torch = _torch()
    count = len(ns)
    dev = torch.device(device)
    wb = int(lib().chfsi_autotune_workspace_bytes(max(ns), max(Ns)))
    w = _work(wb, dev)
    v = (c_int * count)()
    tf = (c_double * (FILTER_VARIANTS * count))()
    _check(lib().chfsi_autotune_filter(count, (c_int * count)(*ns), (c_int * count)(*Ns), _ptr(w),
                                       wb, _stream(stream, dev), v, tf), "chfsi_autotune_filter")
    return np.array(v[:]), np.array(tf[:]).reshape(count, FILTER_VARIANTS)


def chfsi_autotune_set(n, N, variant):
    _check(lib().chfsi_autotune_set(int(n), int(N), int(variant)), "chfsi_autotune_set")


def chfsi_autotune_reset():
    _check(lib().chfsi_autotune_reset(), "chfsi_autotune_reset")


def chfsi_degrees_sequence(mu, res, speed, n_wanted, alpha, beta, tol_abs, deg_max=40):
    """Sequence-calibrated degrees (host); returns (deg, src) numpy arrays."""
    k = len(mu)
    m = (c_double * k)(*[float(x) for x in mu])
    r = (c_double * k)(*[float(x) for x in res])
    sp = None if speed is None else (c_double * k)(*[float(x) for x in speed])
    d = (c_int * k)()
    sr = (c_int * k)()
    _check(lib().chfsi_degrees_sequence(k, m, r, sp, int(n_wanted), float(alpha), float(beta),
                                        float(tol_abs), int(deg_max), d, sr),
           "chfsi_degrees_sequence")
    return np.array(d[:], dtype=np.int64), np.array(sr[:], dtype=np.int64)
