"""Thin ctypes binding of librcscm (include/rcscm.h).

Argument marshalling only: every step of the estimation runs in the HIP
kernels of librcscm.so.  torch provides device memory and the stream.
Importing this module does not need a GPU; creating a Context does.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librcscm.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "rcscm.h")

OK, EINVAL, ESHAPE, ENOTNULL, ENOTPSD, ENONFINITE, EDEVICE, ENOMEM, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7, -8
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "ENOTNULL", -4: "ENOTPSD",
                -5: "ENONFINITE", -6: "EDEVICE", -7: "ENOMEM", -8: "ESTATE"}
RULES = {"naive": 0, "accel": 1, "first": 2}
SCHEDULES = {"auto": 0, "stream": 1, "resident": 2}
LAMSUMS = {"f64": 0, "kahan32": 1}
FLAG_GRAPH = 1
FLAG_CHECKPOINT = 2
FLAG_RUN_ONLY = 4
FLAG_NAIVE_RECOMPUTE = 8


class RcscmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("rh0", ctypes.c_float), ("ru0", ctypes.c_float), ("lam0", ctypes.c_float),
                ("rule", ctypes.c_int), ("schedule", ctypes.c_int), ("lamsum", ctypes.c_int),
                ("block", ctypes.c_int), ("chunk", ctypes.c_int), ("flags", ctypes.c_uint)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "rcscm_default_params": (None, [ctypes.POINTER(Params)]),
    "rcscm_version": (_I, []),
    "rcscm_create": (_I, [ctypes.POINTER(_P), _I, _I, _I, ctypes.POINTER(Params), _P]),
    "rcscm_create_batch": (_I, [ctypes.POINTER(_P), _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                                ctypes.POINTER(Params), _P]),
    "rcscm_init": (_I, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "rcscm_iterate": (_I, [_P, _I]),
    "rcscm_extract": (_I, [_P, _P, _P, _P, _P]),
    "rcscm_set_state": (_I, [_P, _P, _P, _P]),
    "rcscm_get_state": (_I, [_P, _P, _P, _P]),
    "rcscm_sync": (_I, [_P]),
    "rcscm_objective": (_I, [_P, ctypes.POINTER(ctypes.c_double)]),
    "rcscm_backward": (_I, [_P, _P, _P, _P, _P, _P]),
    "rcscm_destroy": (None, [_P]),
    "rcscm_last_error": (ctypes.c_char_p, [_P]),
    "rcscm_workspace_bytes": (ctypes.c_size_t, [_I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                                                ctypes.POINTER(Params)]),
    "rcscm_get_schedule": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "rcscm_backproject": (_I, [_P, _P, _P, ctypes.POINTER(_I), _P, _P, _P, _P, _P]),
    "rcscm_run": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _I, _P, _P, _P, _P]),
    "rcscm_set_run_classes": (_I, [_P, _I, ctypes.POINTER(_I)]),
    "rcscm_get_run_classes": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "rcscm_run_noalloc": (_I, [_I, _I, _I, ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P, _P,
                               _P, _I, _P, _P, _P, _P, _I]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Loads librcscm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1908_01964_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions declared in include/rcscm.h."""
    with open(HEADER_PATH) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rcscm_[a-z_]+)\s*\(", text)))


def default_params() -> Params:
    p = Params()
    lib().rcscm_default_params(ctypes.byref(p))
    return p


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("arrays passed to librcscm must be device tensors")
    if not t.is_contiguous():
        raise ValueError("arrays passed to librcscm must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check(status: int, handle=None):
    if status != OK:
        msg = lib().rcscm_last_error(handle).decode()
        raise RcscmError(status, msg)


def workspace_bytes(I: int, Js: Sequence[int], Ms: Sequence[int], **kw) -> int:
    U = len(Js)
    p = _params(**kw)
    Ja = (ctypes.c_int * U)(*Js)
    Ma = (ctypes.c_int * U)(*Ms)
    return int(lib().rcscm_workspace_bytes(U, I, Ja, Ma, ctypes.byref(p)))


def _params(alpha=1.1, beta=1e-16, rh0=1.0, ru0=1.0, lam0=1.0, rule="accel", schedule="auto",
            lamsum="f64", block=0, chunk=0, graph=False, checkpoint=False,
            run_only=False, naive_recompute=False) -> Params:
    p = default_params()
    p.alpha, p.beta = float(alpha), float(beta)
    p.rh0, p.ru0, p.lam0 = float(rh0), float(ru0), float(lam0)
    p.rule = RULES[rule] if isinstance(rule, str) else int(rule)
    p.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    p.lamsum = LAMSUMS[lamsum] if isinstance(lamsum, str) else int(lamsum)
    p.block, p.chunk = int(block), int(chunk)
    p.flags = ((FLAG_GRAPH if graph else 0) | (FLAG_CHECKPOINT if checkpoint else 0)
               | (FLAG_RUN_ONLY if run_only else 0)
               | (FLAG_NAIVE_RECOMPUTE if naive_recompute else 0))
    return p


class Context:
    """One estimation problem (a single utterance, or a ragged batch of U utterances).

    Arrays use the batch layout of include/rcscm.h: per-utterance arrays
    concatenated in utterance order (for U = 1 the natural [I, J, M] shapes).
    """

    def __init__(self, I: int, Js: Sequence[int], Ms: Sequence[int], device=None, stream=None,
                 run_classes=None, **params):
        self.I, self.Js, self.Ms = int(I), [int(j) for j in Js], [int(m) for m in Ms]
        self.U = len(self.Js)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        self.params = _params(**params)
        self.nbins = sum(self.I * j for j in self.Js)
        self.nrows = self.U * self.I
        # element counts of x, a (and b) and Rp in the batch layout, checked at every call
        self._nx = sum(self.I * j * m for j, m in zip(self.Js, self.Ms))
        self._na = sum(self.I * m for m in self.Ms)
        self._nr = sum(self.I * m * m for m in self.Ms)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            if self.U == 1:
                st = lib().rcscm_create(ctypes.byref(h), self.I, self.Js[0], self.Ms[0],
                                        ctypes.byref(self.params),
                                        ctypes.c_void_p(self.stream.cuda_stream))
            else:
                Ja = (ctypes.c_int * self.U)(*self.Js)
                Ma = (ctypes.c_int * self.U)(*self.Ms)
                st = lib().rcscm_create_batch(ctypes.byref(h), self.U, self.I, Ja, Ma,
                                              ctypes.byref(self.params),
                                              ctypes.c_void_p(self.stream.cuda_stream))
        _check(st, None)
        self._h = h
        self._keep = []  # tensors the library borrows (x for the naive rule)
        if run_classes:
            self.set_run_classes(run_classes)

    @classmethod
    def single(cls, I: int, J: int, M: int, **kw) -> "Context":
        return cls(I, [J], [M], **kw)

    # -- lifecycle ---------------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().rcscm_destroy(self._h)
            self._h = None
        self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- calls -------------------------------------------------------------------------------
    def init(self, x: torch.Tensor, a: torch.Tensor, Rp: torch.Tensor, b: torch.Tensor,
             rh0: Optional[torch.Tensor] = None, ru0: Optional[torch.Tensor] = None,
             lam0: Optional[torch.Tensor] = None):
        self._check_sizes(x, a, Rp, b, rh0, ru0, lam0)
        _check(lib().rcscm_init(self._h, _ptr(x), _ptr(a), _ptr(Rp), _ptr(b), _ptr(rh0), _ptr(ru0),
                                _ptr(lam0)), self._h)
        self._keep = [x]
        return self

    def iterate(self, K: int):
        _check(lib().rcscm_iterate(self._h, int(K)), self._h)
        return self

    def extract(self, s_hat: bool = True, out=None):
        """Returns dict(rh, ru, lam[, s_hat]) as new device tensors (batch layout)."""
        dev = self.device
        if out is None:
            out = dict(rh=torch.empty(self.nbins, dtype=torch.float32, device=dev),
                       ru=torch.empty(self.nbins, dtype=torch.float32, device=dev),
                       lam=torch.empty(self.nrows, dtype=torch.float32, device=dev))
            if s_hat:
                out["s_hat"] = torch.empty(self.nbins, dtype=torch.complex64, device=dev)
        _check(lib().rcscm_extract(self._h, _ptr(out.get("rh")), _ptr(out.get("ru")),
                                   _ptr(out.get("lam")), _ptr(out.get("s_hat"))), self._h)
        return out

    def run(self, x, a, Rp, b, K: int, rh0=None, ru0=None, lam0=None, out=None, s_hat=True):
        """init + iterate(K) + extract in one call (a single fused launch where possible)."""
        self._check_sizes(x, a, Rp, b, rh0, ru0, lam0)
        dev = self.device
        if out is None:
            out = dict(rh=torch.empty(self.nbins, dtype=torch.float32, device=dev),
                       ru=torch.empty(self.nbins, dtype=torch.float32, device=dev),
                       lam=torch.empty(self.nrows, dtype=torch.float32, device=dev))
            if s_hat:
                out["s_hat"] = torch.empty(self.nbins, dtype=torch.complex64, device=dev)
        _check(lib().rcscm_run(self._h, _ptr(x), _ptr(a), _ptr(Rp), _ptr(b), _ptr(rh0), _ptr(ru0),
                               _ptr(lam0), int(K), _ptr(out.get("rh")), _ptr(out.get("ru")),
                               _ptr(out.get("lam")), _ptr(out.get("s_hat"))), self._h)
        self._keep = [x]
        return out

    def set_state(self, rh: torch.Tensor, ru: torch.Tensor, lam: torch.Tensor):
        for t, n in ((rh, self.nbins), (ru, self.nbins), (lam, self.nrows)):
            if t.dtype != torch.float32 or t.numel() != n:
                raise ValueError("state arrays must be float32 with the batch sizes")
        _check(lib().rcscm_set_state(self._h, _ptr(rh), _ptr(ru), _ptr(lam)), self._h)
        return self

    def get_state(self, out=None):
        """Copies the current state into dict(rh, ru, lam) device tensors (batch layout)."""
        dev = self.device
        if out is None:
            out = dict(rh=torch.empty(self.nbins, dtype=torch.float32, device=dev),
                       ru=torch.empty(self.nbins, dtype=torch.float32, device=dev),
                       lam=torch.empty(self.nrows, dtype=torch.float32, device=dev))
        for k, n in (("rh", self.nbins), ("ru", self.nbins), ("lam", self.nrows)):
            if out[k].dtype != torch.float32 or out[k].numel() != n:
                raise ValueError("state arrays must be float32 with the batch sizes")
        _check(lib().rcscm_get_state(self._h, _ptr(out["rh"]), _ptr(out["ru"]), _ptr(out["lam"])),
               self._h)
        return out

    def sync(self):
        _check(lib().rcscm_sync(self._h), self._h)
        return self

    def status(self) -> int:
        return int(lib().rcscm_sync(self._h))

    def objective(self) -> float:
        v = ctypes.c_double()
        _check(lib().rcscm_objective(self._h, ctypes.byref(v)), self._h)
        return float(v.value)

    def backward(self, x: torch.Tensor, grad_s_hat: torch.Tensor, want_x=True, want_rh0=True,
                 want_lam0=True):
        dev = self.device
        gx = torch.empty_like(x) if want_x else None
        grh = torch.empty(self.nbins, dtype=torch.float32, device=dev) if want_rh0 else None
        glam = torch.empty(self.nrows, dtype=torch.float32, device=dev) if want_lam0 else None
        _check(lib().rcscm_backward(self._h, _ptr(x), _ptr(grad_s_hat), _ptr(gx), _ptr(grh),
                                    _ptr(glam)), self._h)
        return gx, grh, glam

    def backward_into(self, x: torch.Tensor, grad_s_hat: torch.Tensor, grad_x=None, grad_rh0=None,
                      grad_lam0=None):
        """rcscm_backward into caller-allocated outputs (any of them may be None)."""
        _check(lib().rcscm_backward(self._h, _ptr(x), _ptr(grad_s_hat), _ptr(grad_x),
                                    _ptr(grad_rh0), _ptr(grad_lam0)), self._h)
        return grad_x, grad_rh0, grad_lam0

    def backproject(self, x: torch.Tensor, W: torch.Tensor, target, want_ru0=True,
                    want_lam0=True):
        """a, R', b (and r^u_0, lambda_0) from demixing matrices W (eq. (11), eqs. (22)-(23))."""
        dev = self.device
        na = sum(self.I * m for m in self.Ms)
        nr = sum(self.I * m * m for m in self.Ms)
        if W.dtype != torch.complex128 or W.numel() != nr:
            raise ValueError(f"W must be complex128 with {nr} elements")
        tg = [int(target)] * self.U if isinstance(target, int) else [int(t) for t in target]
        a = torch.empty(na, dtype=torch.complex128, device=dev)
        b = torch.empty(na, dtype=torch.complex128, device=dev)
        Rp = torch.empty(nr, dtype=torch.complex128, device=dev)
        ru0 = torch.empty(self.nbins, dtype=torch.float32, device=dev) if want_ru0 else None
        lam0 = torch.empty(self.nrows, dtype=torch.float32, device=dev) if want_lam0 else None
        T = (ctypes.c_int * self.U)(*tg)
        _check(lib().rcscm_backproject(self._h, _ptr(x), _ptr(W), T, _ptr(a), _ptr(Rp), _ptr(b),
                                       _ptr(ru0), _ptr(lam0)), self._h)
        return a, Rp, b, ru0, lam0

    def set_run_classes(self, table):
        """Workgroup classes of run()'s fused launch: entries (M, j_max, nt, bpl); [] = built-in."""
        flat = [int(v) for e in table for v in e]
        arr = (ctypes.c_int * max(1, len(flat)))(*flat)
        _check(lib().rcscm_set_run_classes(self._h, len(table), arr), self._h)
        return self

    def run_classes(self):
        """The classes run() launches: list of dict(M, nt, bpl, rows, J)."""
        n = ctypes.c_int()
        _check(lib().rcscm_get_run_classes(self._h, 0, None, ctypes.byref(n)), self._h)
        cap = max(1, n.value)
        arr = (ctypes.c_int * (5 * cap))()
        _check(lib().rcscm_get_run_classes(self._h, cap, arr, ctypes.byref(n)), self._h)
        return [dict(M=arr[5 * k], nt=arr[5 * k + 1], bpl=arr[5 * k + 2], rows=arr[5 * k + 3],
                     J=arr[5 * k + 4]) for k in range(n.value)]

    def schedule(self):
        s, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().rcscm_get_schedule(self._h, ctypes.byref(s), ctypes.byref(b),
                                        ctypes.byref(c)), self._h)
        names = {v: k for k, v in SCHEDULES.items()}
        return dict(schedule=names[s.value], block=b.value, chunk=c.value)

    # -- helpers -----------------------------------------------------------------------------
    def _check_sizes(self, x, a, Rp, b, rh0, ru0, lam0):
        nx, na, nr = self._nx, self._na, self._nr
        for t, n, dt, name in ((x, nx, torch.complex64, "x"), (a, na, torch.complex128, "a"),
                               (Rp, nr, torch.complex128, "Rp"), (b, na, torch.complex128, "b")):
            if t.dtype != dt or t.numel() != n:
                raise ValueError(f"{name} must be {dt} with {n} elements (got {t.dtype}, "
                                 f"{t.numel()})")
        for t, n, name in ((rh0, self.nbins, "rh0"), (ru0, self.nbins, "ru0"),
                           (lam0, self.nrows, "lam0")):
            if t is not None and (t.dtype != torch.float32 or t.numel() != n):
                raise ValueError(f"{name} must be float32 with {n} elements")


def run_noalloc(I: int, J: int, M: int, x, a, Rp, b, K: int, out: dict, rh0=None, ru0=None,
                lam0=None, stream=None, check=True, **params):
    """rcscm_run_noalloc: one utterance, no context, no device allocation by the library.

    out holds caller-allocated device tensors rh, ru (float32 [I*J]), lam (float32 [I]) and
    s_hat (complex64 [I*J]); any may be missing.  check=False only enqueues (capturable)."""
    p = _params(**params)
    st = torch.cuda.current_stream() if stream is None else stream
    _check(lib().rcscm_run_noalloc(int(I), int(J), int(M), ctypes.byref(p),
                                   ctypes.c_void_p(st.cuda_stream), _ptr(x), _ptr(a), _ptr(Rp),
                                   _ptr(b), _ptr(rh0), _ptr(ru0), _ptr(lam0), int(K),
                                   _ptr(out.get("rh")), _ptr(out.get("ru")), _ptr(out.get("lam")),
                                   _ptr(out.get("s_hat")), 1 if check else 0), None)
    return out


def to_device(problem_or_list, device="cuda"):
    """Packs one synthetic Problem (or a list of them) into device tensors in batch layout."""
    probs = problem_or_list if isinstance(problem_or_list, (list, tuple)) else [problem_or_list]

    def cat(arrs, dtype):
        return torch.cat([torch.from_numpy(v).reshape(-1) for v in arrs]).to(dtype).to(device)
    x = cat([p.x for p in probs], torch.complex64)
    a = cat([p.a for p in probs], torch.complex128)
    Rp = cat([p.Rp for p in probs], torch.complex128)
    b = cat([p.b for p in probs], torch.complex128)
    return x, a, Rp, b
