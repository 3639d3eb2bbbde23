"""Python binding of the C ABI in ``include/dl.h`` (argument marshalling only).

Every function here passes device pointers of torch tensors and the current
HIP stream to the library ``libdl_mi355.so``; all arithmetic runs in the HIP
kernels.  If the library has not been built the first call raises: there is
no other implementation to fall back to.

Layouts (row-major): D ``[n][p]`` float32, Y ``[m][p]`` float32,
X_idx ``[m][s]`` int32 (-1 = unused slot), X_val ``[m][s]`` float32.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdl_mi355.so")

DL_OK, DL_EINVAL, DL_EWORKSPACE, DL_EHIP, DL_ENUMERIC, DL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PREC_FP32, PREC_BF16 = 0, 1
RULE_AKSVD, RULE_SGK, RULE_NSGK = 0, 1, 2


class DLError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int), ("n", ctypes.c_int), ("m", ctypes.c_int), ("s", ctypes.c_int),
        ("group_size", ctypes.c_int), ("precision", ctypes.c_int), ("rule", ctypes.c_int),
        ("pivot_fp64_threshold", ctypes.c_float), ("tol_corr", ctypes.c_float),
        ("tol_pivot", ctypes.c_float), ("omp_lanes_per_signal", ctypes.c_int),
        ("omp_atoms_per_lane", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("fp64_pivot_recomputes", ctypes.c_longlong), ("early_stops", ctypes.c_longlong),
        ("unused_atoms", ctypes.c_longlong), ("zero_updates", ctypes.c_longlong),
        ("nonfinite", ctypes.c_longlong), ("fallbacks", ctypes.c_longlong),
    ]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class _Problem(ctypes.Structure):
    _fields_ = [("prm", _Params), ("Y", ctypes.c_void_p), ("D", ctypes.c_void_p),
                ("X_idx", ctypes.c_void_p), ("X_val", ctypes.c_void_p),
                ("rmse", ctypes.c_void_p)]


_lib = None
_vp = ctypes.c_void_p
_PP = ctypes.POINTER(_Params)
_PB = ctypes.POINTER(_Problem)

# name -> (restype, argtypes); the same list is checked against the header by the tests
SIGNATURES = {
    "dl_abi_version": (ctypes.c_int, []),
    "dl_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "dl_params_default": (ctypes.c_int, [_PP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "dl_workspace_size": (ctypes.c_size_t, [_PP]),
    "dl_workspace_init": (ctypes.c_int, [_PP, _vp, ctypes.c_size_t, _vp]),
    "dl_gram": (ctypes.c_int, [_PP, _vp, _vp, _vp]),
    "dl_corr": (ctypes.c_int, [_PP, _vp, _vp, _vp, _vp]),
    "dl_products": (ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "dl_omp": (ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "dl_csr": (ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "dl_jau_update": (ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "dl_jau_update_nsgk": (ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                          ctypes.c_size_t, _vp]),
    "dl_rmse": (ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "dl_iterate": (ctypes.c_int, [_PP, _vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp,
                                  ctypes.c_size_t, _vp]),
    "dl_rmse_noalloc": (ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _vp, _vp]),
    "dl_read_stats": (ctypes.c_int, [_PP, _vp, ctypes.c_size_t, ctypes.POINTER(Stats), _vp]),
    "dl_iterate_record": (ctypes.c_int, [_PP, _vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp,
                                         ctypes.c_size_t, _vp]),
    "dl_proposal_workspace_size": (ctypes.c_size_t, [_PP]),
    "dl_code_proposed": (ctypes.c_int, [_PP, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                        _vp, ctypes.c_size_t, _vp]),
    "dl_iterate_proposed": (ctypes.c_int, [_PP, _vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp,
                                           _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp]),
    "dl_mlp_param_count": (ctypes.c_size_t, [ctypes.c_void_p]),
    "dl_mlp_workspace_size": (ctypes.c_size_t, [ctypes.c_void_p]),
    "dl_mlp_init": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "dl_mlp_train_step": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp, ctypes.c_int, ctypes.c_int,
                                         _vp, ctypes.c_int, _vp, ctypes.c_int, _vp]),
    "dl_mlp_read": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp, _vp,
                                   ctypes.POINTER(ctypes.c_double), _vp]),
    "dl_mlp_forward": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp, ctypes.c_int, _vp, _vp]),
    "dl_topk": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]),
    "dl_batch_workspace_size": (ctypes.c_size_t, [_PB, ctypes.c_int]),
    "dl_iterate_batched": (ctypes.c_int, [_PB, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t,
                                          _vp]),
    "dl_autotune": (ctypes.c_int, [_PB, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t, _vp]),
    "dl_profile_enable": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "dl_profile_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]),
}

# kernel ids of dl_profile_read (enum dl_kernel)
KERNELS = ["gram", "corr", "omp", "csr_count", "csr_scan", "csr_scatter", "upd_pass1",
           "upd_reduce", "upd_pass2", "upd_eupdate", "rmse", "misc", "mlp", "propose"]


def lib():
    """Load ``libdl_mi355.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1509_05054_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    try:
        return lib().dl_status_string(int(status)).decode()
    except Exception:  # library missing: still report the number
        return f"status {status}"


def _check(status: int, what: str):
    if status != DL_OK:
        raise DLError(status, what)


@dataclass
class Params:
    p: int
    n: int
    m: int
    s: int
    group_size: int | None = None
    precision: int = PREC_FP32
    rule: int = RULE_AKSVD
    pivot_fp64_threshold: float = 1e-6
    tol_corr: float = 1e-5
    tol_pivot: float = 1e-10
    omp_lanes_per_signal: int = 0
    omp_atoms_per_lane: int = 0

    def c(self) -> _Params:
        return _Params(self.p, self.n, self.m, self.s,
                       self.n if self.group_size is None else self.group_size,
                       self.precision, self.rule, self.pivot_fp64_threshold, self.tol_corr,
                       self.tol_pivot, self.omp_lanes_per_signal, self.omp_atoms_per_lane)

    def ref(self):
        self._c = self.c()  # keep alive for the call
        return ctypes.byref(self._c)


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def workspace_size(prm: Params) -> int:
    n = lib().dl_workspace_size(prm.ref())
    if n == 0:
        raise DLError(DL_EINVAL, "dl_workspace_size")
    return int(n)


def workspace(prm: Params, device="cuda") -> torch.Tensor:
    """Allocate (torch caching allocator) and initialise a workspace for ``prm``."""
    ws = torch.empty(workspace_size(prm), dtype=torch.uint8, device=device)
    _check(lib().dl_workspace_init(prm.ref(), _ptr(ws), ws.numel(), _stream()), "dl_workspace_init")
    return ws


def gram(prm: Params, D, G, stream=None):
    _check(lib().dl_gram(prm.ref(), _ptr(D), _ptr(G), _stream(stream)), "dl_gram")


def corr(prm: Params, D, Y, A0, stream=None):
    _check(lib().dl_corr(prm.ref(), _ptr(D), _ptr(Y), _ptr(A0), _stream(stream)), "dl_corr")


def products(prm: Params, D, Y, G, A0, ws, stream=None):
    _check(lib().dl_products(prm.ref(), _ptr(D), _ptr(Y), _ptr(G), _ptr(A0), _ptr(ws), ws.numel(),
                             _stream(stream)), "dl_products")


def omp(prm: Params, D, Y, X_idx, X_val, ws, stream=None):
    _check(lib().dl_omp(prm.ref(), _ptr(D), _ptr(Y), _ptr(X_idx), _ptr(X_val), _ptr(ws),
                        ws.numel(), _stream(stream)), "dl_omp")


def csr(prm: Params, X_idx, row_ptr, users, ws, stream=None):
    _check(lib().dl_csr(prm.ref(), _ptr(X_idx), _ptr(row_ptr), _ptr(users), _ptr(ws),
                        ws.numel(), _stream(stream)), "dl_csr")


def jau_update(prm: Params, Y, D, X_idx, X_val, ws, stream=None):
    _check(lib().dl_jau_update(prm.ref(), _ptr(Y), _ptr(D), _ptr(X_idx), _ptr(X_val), _ptr(ws),
                               ws.numel(), _stream(stream)), "dl_jau_update")


def jau_update_nsgk(prm: Params, Y, D, X_idx, X_val, Xprev_idx, Xprev_val, ws, stream=None):
    """NSGK atom update of D (eq. 7) from this coding X and the previous one."""
    _check(lib().dl_jau_update_nsgk(prm.ref(), _ptr(Y), _ptr(D), _ptr(X_idx), _ptr(X_val),
                                    _ptr(Xprev_idx), _ptr(Xprev_val), _ptr(ws), ws.numel(),
                                    _stream(stream)), "dl_jau_update_nsgk")


def rmse(prm: Params, Y, D, X_idx, X_val, out, ws, stream=None):
    _check(lib().dl_rmse(prm.ref(), _ptr(Y), _ptr(D), _ptr(X_idx), _ptr(X_val), _ptr(out),
                         _ptr(ws), ws.numel(), _stream(stream)), "dl_rmse")


def rmse_noalloc(prm: Params, Y, D, X_idx, X_val, out, stream=None):
    """dl_rmse with the library's static scratch (no workspace, no allocation)."""
    _check(lib().dl_rmse_noalloc(prm.ref(), _ptr(Y), _ptr(D), _ptr(X_idx), _ptr(X_val),
                                 _ptr(out), _stream(stream)), "dl_rmse_noalloc")


def iterate(prm: Params, Y, D, iters, X_idx, X_val, rmse_out, ws, stream=None):
    _check(lib().dl_iterate(prm.ref(), _ptr(Y), _ptr(D), int(iters), _ptr(X_idx), _ptr(X_val),
                            _ptr(rmse_out), _ptr(ws), ws.numel(), _stream(stream)), "dl_iterate")


class _MlpParams(ctypes.Structure):
    _fields_ = [("in_dim", ctypes.c_int), ("hidden", ctypes.c_int), ("out_dim", ctypes.c_int),
                ("batch", ctypes.c_int), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("pos_weight", ctypes.c_float)]


@dataclass
class MlpParams:
    in_dim: int
    hidden: int
    out_dim: int
    batch: int = 4096
    lr: float = 3e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    pos_weight: float = 1.0

    def ref(self):
        self._c = _MlpParams(self.in_dim, self.hidden, self.out_dim, self.batch, self.lr,
                             self.beta1, self.beta2, self.eps, self.pos_weight)
        return ctypes.cast(ctypes.pointer(self._c), ctypes.c_void_p)


def mlp_param_count(q: MlpParams) -> int:
    n = lib().dl_mlp_param_count(q.ref())
    if n == 0:
        raise DLError(DL_EINVAL, "dl_mlp_param_count")
    return int(n)


def mlp_workspace(q: MlpParams, params, device="cuda") -> torch.Tensor:
    """Allocate the network workspace and load the packed FP32 parameters."""
    size = lib().dl_mlp_workspace_size(q.ref())
    if size == 0:
        raise DLError(DL_EINVAL, "dl_mlp_workspace_size")
    ws = torch.empty(int(size), dtype=torch.uint8, device=device)
    _check(lib().dl_mlp_init(q.ref(), _ptr(params), _ptr(ws), ws.numel(), _stream()), "dl_mlp_init")
    return ws


def mlp_train_step(q: MlpParams, ws, Y, hist, pairs, step, stream=None):
    m, p = Y.shape
    s = hist.shape[1]
    _check(lib().dl_mlp_train_step(q.ref(), _ptr(ws), ws.numel(), _ptr(Y), m, p, _ptr(hist), s,
                                   _ptr(pairs), int(step), _stream(stream)), "dl_mlp_train_step")


def mlp_read(q: MlpParams, ws, params=None, grads=None, want_loss=False, stream=None):
    loss = ctypes.c_double(0.0)
    _check(lib().dl_mlp_read(q.ref(), _ptr(ws), ws.numel(), _ptr(params), _ptr(grads),
                             ctypes.byref(loss) if want_loss else None, _stream(stream)),
           "dl_mlp_read")
    return loss.value if want_loss else None


def mlp_forward(q: MlpParams, ws, X, logits, stream=None):
    _check(lib().dl_mlp_forward(q.ref(), _ptr(ws), ws.numel(), _ptr(X), X.shape[0], _ptr(logits),
                                _stream(stream)), "dl_mlp_forward")


def topk(logits, k, out, stream=None):
    rows, cols = logits.shape
    _check(lib().dl_topk(rows, cols, int(k), _ptr(logits), _ptr(out), _stream(stream)), "dl_topk")


def profile_enable(on: bool, max_launches: int = 1 << 16):
    """Per-kernel HIP-event timing inside the library (measurement only)."""
    _check(lib().dl_profile_enable(int(bool(on)), int(max_launches)), "dl_profile_enable")


def profile_read() -> dict:
    """{kernel: (total_ms, launches)} since the last read; waits for the events."""
    k = len(KERNELS)
    ms = (ctypes.c_double * k)()
    cnt = (ctypes.c_longlong * k)()
    _check(lib().dl_profile_read(ms, cnt, k), "dl_profile_read")
    return {KERNELS[i]: (float(ms[i]), int(cnt[i])) for i in range(k)}


def iterate_record(prm: Params, Y, D, iters, X_idx, X_val, rmse_out, hist, rref, ws, stream=None):
    _check(lib().dl_iterate_record(prm.ref(), _ptr(Y), _ptr(D), int(iters), _ptr(X_idx),
                                   _ptr(X_val), _ptr(rmse_out), _ptr(hist), _ptr(rref), _ptr(ws),
                                   ws.numel(), _stream(stream)), "dl_iterate_record")


class _Proposal(ctypes.Structure):
    _fields_ = [("cand", ctypes.c_void_p), ("k", ctypes.c_int), ("margin", ctypes.c_float),
                ("audit_every", ctypes.c_int)]


def proposal_workspace(prm: Params, device="cuda") -> torch.Tensor:
    n = lib().dl_proposal_workspace_size(prm.ref())
    if n == 0:
        raise DLError(DL_EINVAL, "dl_proposal_workspace_size")
    return torch.empty(int(n), dtype=torch.uint8, device=device)


def code_proposed(prm: Params, cand, margin, D, Y, rref, X_idx, X_val, ws, pws, stream=None):
    pr = _Proposal(ctypes.c_void_p(cand.data_ptr()), cand.shape[1], float(margin), 0)
    _check(lib().dl_code_proposed(prm.ref(), ctypes.cast(ctypes.pointer(pr), ctypes.c_void_p),
                                  _ptr(D), _ptr(Y), _ptr(rref), _ptr(X_idx), _ptr(X_val), _ptr(ws),
                                  ws.numel(), _ptr(pws), pws.numel(), _stream(stream)),
           "dl_code_proposed")


def iterate_proposed(prm: Params, cand, margin, audit_every, Y, D, iters, rref, X_idx, X_val,
                     rmse_out, ws, pws, stream=None):
    pr = _Proposal(ctypes.c_void_p(cand.data_ptr()), cand.shape[1], float(margin), int(audit_every))
    _check(lib().dl_iterate_proposed(prm.ref(), ctypes.cast(ctypes.pointer(pr), ctypes.c_void_p),
                                     _ptr(Y), _ptr(D), int(iters), _ptr(rref), _ptr(X_idx),
                                     _ptr(X_val), _ptr(rmse_out), _ptr(ws), ws.numel(), _ptr(pws),
                                     pws.numel(), _stream(stream)), "dl_iterate_proposed")


def read_stats(prm: Params, ws, stream=None, allow_nonfinite=False) -> dict:
    st = Stats()
    rc = lib().dl_read_stats(prm.ref(), _ptr(ws), ws.numel(), ctypes.byref(st), _stream(stream))
    if rc == DL_ENUMERIC and allow_nonfinite:
        return st.as_dict()
    _check(rc, "dl_read_stats")
    return st.as_dict()


# ---------------------------------------------------------------- batched problems
@dataclass
class Problem:
    """One problem of a batched call: parameters and its device tensors
    (Y [m][p], D [n][p] in/out, X_idx/X_val [m][s] out, rmse [iters] float64 out)."""
    prm: Params
    Y: torch.Tensor
    D: torch.Tensor
    X_idx: torch.Tensor
    X_val: torch.Tensor
    rmse: torch.Tensor | None = None


def _problem_array(problems):
    arr = (_Problem * len(problems))()
    for k, pb in enumerate(problems):
        arr[k].prm = pb.prm.c()
        arr[k].Y = _ptr(pb.Y).value if pb.Y is not None else None
        arr[k].D = _ptr(pb.D).value if pb.D is not None else None
        arr[k].X_idx = _ptr(pb.X_idx).value if pb.X_idx is not None else None
        arr[k].X_val = _ptr(pb.X_val).value if pb.X_val is not None else None
        arr[k].rmse = _ptr(pb.rmse).value if pb.rmse is not None else None
    return arr


def batch_workspace(problems, device="cuda") -> torch.Tensor:
    n = lib().dl_batch_workspace_size(_problem_array(problems), len(problems))
    if n == 0:
        raise DLError(DL_EINVAL, "dl_batch_workspace_size")
    return torch.empty(int(n), dtype=torch.uint8, device=device)


def iterate_batched(problems, iters, ws, stream=None):
    arr = _problem_array(problems)
    _check(lib().dl_iterate_batched(arr, len(problems), int(iters), _ptr(ws), ws.numel(),
                                    _stream(stream)), "dl_iterate_batched")


def autotune(problems, ws, reps=3, stream=None):
    """Time the OMP launch shapes and store the fastest in the ``prm``
    (``omp_lanes_per_signal``, ``omp_atoms_per_lane``) of every problem that
    shares the persistent launches; returns every problem's shape ((0, 0):
    the default, kept by the problems that run alone)."""
    arr = _problem_array(problems)
    _check(lib().dl_autotune(arr, len(problems), int(reps), _ptr(ws), ws.numel(),
                             _stream(stream)), "dl_autotune")
    out = []
    for k, pb in enumerate(problems):
        pb.prm.omp_lanes_per_signal = int(arr[k].prm.omp_lanes_per_signal)
        pb.prm.omp_atoms_per_lane = int(arr[k].prm.omp_atoms_per_lane)
        out.append((pb.prm.omp_lanes_per_signal, pb.prm.omp_atoms_per_lane))
    return out
