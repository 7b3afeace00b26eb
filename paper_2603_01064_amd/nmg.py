"""Thin Python binding of the C ABI in ``include/nmg.h`` (argument marshalling only).

Every computation runs in the HIP library ``_lib/libnmg.so``; this module only
checks tensor dtypes/devices/shapes and passes raw device pointers and the
current HIP stream.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libnmg.so")

NMG_OK = 0
NMG_NOT_CONVERGED = 1
NMG_DIVERGED = 2
NMG_ERR_NONFINITE = -5
PRECISION = {"fp64": 0, "fp32": 1, "mixed": 2}
MASK = {"band": 0, "ramp": 1, "cycle": 2}  # "cycle": the combined loss eq. loss_1
MAX_LAYERS = 7


class NMGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nmg status {code}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int), ("s", ctypes.c_double), ("trunc", ctypes.c_double),
        ("levels", ctypes.c_int), ("max_batch", ctypes.c_int), ("n_layers", ctypes.c_int),
        ("channels", ctypes.c_int * (MAX_LAYERS + 1)), ("ksize", ctypes.c_int), ("n_weight_sets", ctypes.c_int),
        ("operator_form", ctypes.c_int), ("smoother_arch", ctypes.c_int), ("fno_width", ctypes.c_int),
        ("fno_layers", ctypes.c_int), ("fno_modes", ctypes.c_int), ("fno_ksize", ctypes.c_int),
    ]


class RequestResult(ctypes.Structure):
    """``nmg_request_result``: one finished serving request."""
    _fields_ = [("id", ctypes.c_longlong), ("status", ctypes.c_int), ("cycles", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class SolveStats(ctypes.Structure):
    """``nmg_solve_stats``: the outcome of one right-hand side of a solve."""
    _fields_ = [("cycles", ctypes.c_int), ("status", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("done_ms", ctypes.c_double)]


class _CycleOpts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("use_fprime", ctypes.c_int),
                ("precision", ctypes.c_int)]


_lib = None


def load_library():
    """Loads ``libnmg.so``; raises ``ImportError`` if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, Z, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_int
    sig = {
        "nmg_setup_hierarchy": (S, [ctypes.POINTER(_Problem), ctypes.POINTER(P)]),
        "nmg_destroy": (None, [P]),
        "nmg_last_error": (ctypes.c_char_p, []),
        "nmg_load_smoother_weights": (S, [P, I, I, P, Z]),
        "nmg_get_smoother_weights": (S, [P, I, I, P, Z]),
        "nmg_set_jacobi_smoother": (S, [P, I, D]),
        "nmg_prepare": (S, [P, I, P, P]),
        "nmg_apply_operator": (S, [P, I, I, P, P, P, I, P]),
        "nmg_apply_smoother": (S, [P, I, I, P, P, P, P, I, P]),
        "nmg_apply_fprime": (S, [P, I, I, P, P, I, P]),
        "nmg_vcycle": (S, [P, I, P, P, P, P, ctypes.POINTER(_CycleOpts), P]),
        "nmg_solve": (S, [P, I, P, P, P, P, D, I, ctypes.POINTER(_CycleOpts), P, P, P]),
        "nmg_loss_grad": (S, [P, I, I, P, P, I, I, I, I, P, P]),
        "nmg_loss_forward": (S, [P, I, I, P, P, I, I, I, P, P]),
        "nmg_rollout": (S, [P, I, P, P, P, P, P, ctypes.POINTER(_CycleOpts), P]),
        "nmg_get_gradient": (S, [P, I, I, P, Z]),
        "nmg_adam_step": (S, [P, I, D, D, D, D, P]),
        "nmg_train_step": (S, [P, I, I, P, P, I, I, I, D, P, P]),
        "nmg_level_size": (I, [P, I]),
        "nmg_alpha_floor": (S, [P, ctypes.POINTER(ctypes.c_double)]),
        "nmg_profile_enable": (S, [P, I]),
        "nmg_set_graphs": (S, [P, I]),
        "nmg_profile_levels": (S, [P, I]),
        "nmg_profile_sample": (S, [P, I]),
        "nmg_profile_rhs": (S, [P, P]),
        "nmg_serve_submit": (S, [P, ctypes.c_longlong, D, I, P, P]),
        "nmg_serve_step": (S, [P, D, I, ctypes.POINTER(_CycleOpts), P, ctypes.POINTER(ctypes.c_int), P]),
        "nmg_serve_pending": (S, [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "nmg_serve_reset": (S, [P]),
        "nmg_request_bytes": (S, [P, I, ctypes.POINTER(ctypes.c_size_t)]),
        "nmg_pool_create": (S, [ctypes.c_size_t, ctypes.POINTER(P)]),
        "nmg_pool_destroy": (None, [P]),
        "nmg_pool_add": (S, [P, P, ctypes.POINTER(ctypes.c_int)]),
        "nmg_pool_submit": (S, [P, I, ctypes.c_longlong, D, I, P, P]),
        "nmg_pool_step": (S, [P, D, I, ctypes.POINTER(_CycleOpts), P, P, I, ctypes.POINTER(ctypes.c_int)]),
        "nmg_pool_pending": (S, [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_size_t)]),
        "nmg_profile_query": (S, [P, I, I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
        "nmg_debug_transfer_map": (S, [P, I, I, P, P]),
        "nmg_debug_factor": (S, [P, I, I, P, P]),
        "nmg_debug_option": (S, [P, I, I]),
        "nmg_apply_fprime_noalloc": (S, [P, I, I, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code: int) -> int:
    if code < 0:
        msg = _lib.nmg_last_error()
        raise NMGError(code, msg.decode() if msg else "")
    return code


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _require(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


@dataclass
class Problem:
    """Mirror of ``nmg_problem``."""
    n: int
    s: float
    levels: int
    dim: int = 2
    trunc: float = 4.0
    max_batch: int = 1
    channels: Sequence[int] = (1, 32, 32, 1)
    ksize: int = 3
    n_weight_sets: int = 1
    operator: str = "normal"   # "normal": alpha I + K^T K; "kernel": alpha I + K; "aniso": alpha D + K (1D)
    fno: Optional[Tuple[int, int, int, int]] = None   # (width C, Fourier layers, modes k, ksize): FNO smoother

    def to_c(self) -> _Problem:
        p = _Problem()
        p.dim, p.n, p.s, p.trunc = self.dim, self.n, self.s, self.trunc
        p.levels, p.max_batch = self.levels, self.max_batch
        p.n_layers = len(self.channels) - 1
        for i, c in enumerate(self.channels):
            p.channels[i] = int(c)
        p.ksize, p.n_weight_sets = self.ksize, self.n_weight_sets
        forms = {"normal": 0, "kernel": 1, "aniso": 2}
        if self.operator not in forms:
            raise ValueError(f"operator must be one of {sorted(forms)}, not {self.operator!r}")
        p.operator_form = forms[self.operator]
        if self.fno is not None:
            p.smoother_arch = 1
            p.fno_width, p.fno_layers, p.fno_modes, p.fno_ksize = (int(v) for v in self.fno)
        return p

    def weight_count(self) -> int:
        if self.fno is not None:
            C, nl, k, ks = self.fno
            rm = 2 * C * C * k * k if self.dim == 2 else C * C * k
            return 2 * C + nl * (2 * rm + C * C * ks ** self.dim + C) + C + 1
        kk = self.ksize ** self.dim
        return sum(a * b * kk for a, b in zip(self.channels[:-1], self.channels[1:]))


@dataclass
class Handle:
    """An ``nmg_handle`` plus the problem it was built for."""
    problem: Problem
    ptr: ctypes.c_void_p = field(default_factory=ctypes.c_void_p)
    _serve_refs: dict = field(default_factory=dict)
    _next_id: int = 0

    # -- lifetime --------------------------------------------------------
    def close(self):
        if self.ptr:
            _lib.nmg_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- geometry --------------------------------------------------------
    def level_size(self, level: int) -> int:
        return int(_lib.nmg_level_size(self.ptr, level))

    def request_bytes(self, precision: str = "mixed") -> int:
        """Device bytes one request slot occupies in a solve of ``precision``."""
        out = ctypes.c_size_t(0)
        _check(_lib.nmg_request_bytes(self.ptr, PRECISION[precision], ctypes.byref(out)))
        return int(out.value)

    def alpha_floor(self) -> float:
        """Alphas at or below this value leave the operator indefinite and are rejected."""
        out = ctypes.c_double()
        _check(_lib.nmg_alpha_floor(self.ptr, ctypes.byref(out)))
        return float(out.value)

    def level_shape(self, level: int, batch: int):
        n = self.level_size(level)
        return (batch, n) if self.problem.dim == 1 else (batch, n, n)

    # -- smoothers -------------------------------------------------------
    def load_smoother_weights(self, level: int, weight_set: int, layers) -> None:
        flat = np.concatenate([np.asarray(w, dtype=np.float32).reshape(-1) for w in layers])
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        _check(_lib.nmg_load_smoother_weights(self.ptr, level, weight_set,
                                              flat.ctypes.data_as(ctypes.c_void_p), flat.size))

    def get_smoother_weights(self, level: int, weight_set: int = 0) -> np.ndarray:
        out = np.empty(self.problem.weight_count(), dtype=np.float32)
        _check(_lib.nmg_get_smoother_weights(self.ptr, level, weight_set, out.ctypes.data_as(ctypes.c_void_p),
                                             out.size))
        return out

    def set_jacobi_smoother(self, level: int, omega: float) -> None:
        _check(_lib.nmg_set_jacobi_smoother(self.ptr, level, float(omega)))

    # -- operators and cycle -----------------------------------------------
    def prepare(self, alpha) -> None:
        import torch
        _require(alpha, torch.float64, name="alpha")
        _check(_lib.nmg_prepare(self.ptr, alpha.numel(), _ptr(alpha), _stream()))

    def apply_operator(self, level: int, x, alpha, precision: str = "fp64"):
        import torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        B = alpha.numel()
        _require(x, dt, self.level_shape(level, B), "x")
        _require(alpha, torch.float64, (B,), "alpha")
        y = torch.empty_like(x)
        _check(_lib.nmg_apply_operator(self.ptr, level, B, _ptr(alpha), _ptr(x), _ptr(y), PRECISION[precision],
                                       _stream()))
        return y

    def apply_smoother(self, level: int, b, alpha=None, weight_set=None, precision: str = "fp64"):
        """``h = ||b|| N_l(b/||b||)`` (or weighted Jacobi) on level ``level``."""
        import torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        B = b.shape[0]
        _require(b, dt, self.level_shape(level, B), "b")
        ws = ctypes.c_void_p()
        if weight_set is not None:
            _require(weight_set, torch.int32, (B,), "weight_set")
            ws = _ptr(weight_set)
        ap = ctypes.c_void_p()
        if alpha is not None:
            _require(alpha, torch.float64, (B,), "alpha")
            ap = _ptr(alpha)
        out = torch.empty_like(b)
        _check(_lib.nmg_apply_smoother(self.ptr, level, B, ap, ws, _ptr(b), _ptr(out), PRECISION[precision],
                                       _stream()))
        return out

    def apply_fprime(self, level: int, h, precision: str = "fp64"):
        """``F'_l(h)`` on level ``level``."""
        import torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        B = h.shape[0]
        _require(h, dt, self.level_shape(level, B), "h")
        out = torch.empty_like(h)
        _check(_lib.nmg_apply_fprime(self.ptr, level, B, _ptr(h), _ptr(out), PRECISION[precision], _stream()))
        return out

    def apply_fprime_noalloc(self, level: int, h, out):
        """``nmg_apply_fprime_noalloc``: the BF16 ``F'_l(h)`` into the caller's
        ``out`` with the library's fixed device scratch (no allocation)."""
        import torch
        B = h.shape[0]
        _require(h, torch.float32, self.level_shape(level, B), "h")
        _require(out, torch.float32, self.level_shape(level, B), "out")
        _check(_lib.nmg_apply_fprime_noalloc(self.ptr, level, B, _ptr(h), _ptr(out), _stream()))
        return out

    def vcycle(self, y, x, alpha, weight_set=None, nu1: int = 1, nu2: int = 1, use_fprime: bool = False,
               precision: str = "fp64"):
        """In-place ``x <- MG(x, y)``; call ``prepare(alpha)`` first."""
        import torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        B = alpha.numel()
        shape = self.level_shape(0, B)
        _require(y, dt, shape, "y")
        _require(x, dt, shape, "x")
        _require(alpha, torch.float64, (B,), "alpha")
        ws = ctypes.c_void_p()
        if weight_set is not None:
            _require(weight_set, torch.int32, (B,), "weight_set")
            ws = _ptr(weight_set)
        o = _CycleOpts(nu1, nu2, 1 if use_fprime else 0, PRECISION[precision])
        _check(_lib.nmg_vcycle(self.ptr, B, _ptr(alpha), ws, _ptr(y), _ptr(x), ctypes.byref(o), _stream()))
        return x

    def solve(self, b, alpha, weight_set=None, rtol: float = 1e-6, max_cycles: int = 100, nu1: int = 1,
              nu2: int = 1, use_fprime: bool = False, precision: str = "mixed", x=None, history: bool = False,
              done_ms=None):
        """Returns ``(x, cycles, history_or_None, status)``; ``done_ms`` (a float64
        NumPy array of length B) receives per right-hand-side convergence times
        (-1 where a right-hand side did not converge).  The per right-hand-side
        outcome (cycles, status, final relative residual, time) of the last solve
        is kept in ``self.last_stats`` as a dict of NumPy arrays."""
        import torch
        B = alpha.numel()
        shape = self.level_shape(0, B)
        _require(b, torch.float64, shape, "b")
        _require(alpha, torch.float64, (B,), "alpha")
        if x is None:
            x = torch.empty_like(b)
        _require(x, torch.float64, shape, "x")
        ws = ctypes.c_void_p()
        if weight_set is not None:
            _require(weight_set, torch.int32, (B,), "weight_set")
            ws = _ptr(weight_set)
        stats = (SolveStats * B)()
        hist = np.empty((B, max_cycles + 1), dtype=np.float64) if history else None
        o = _CycleOpts(nu1, nu2, 1 if use_fprime else 0, PRECISION[precision])
        st = _check(_lib.nmg_solve(self.ptr, B, _ptr(alpha), ws, _ptr(b), _ptr(x), float(rtol), int(max_cycles),
                                   ctypes.byref(o), stats,
                                   hist.ctypes.data_as(ctypes.c_void_p) if hist is not None else ctypes.c_void_p(),
                                   _stream()))
        self.last_stats = {
            "cycles": np.array([r.cycles for r in stats], dtype=np.int32),
            "status": np.array([r.status for r in stats], dtype=np.int32),
            "rel_residual": np.array([r.rel_residual for r in stats], dtype=np.float64),
            "done_ms": np.array([r.done_ms for r in stats], dtype=np.float64),
        }
        if done_ms is not None:
            done_ms[:] = np.where(self.last_stats["status"] == NMG_OK, self.last_stats["done_ms"], -1.0)
        return x, self.last_stats["cycles"].copy(), hist, st

    # -- serving (continuous batching) --------------------------------------
    def serve_submit(self, b, x, alpha: float, weight_set: int = 0, rid: int | None = None) -> int:
        """Queues one request: ``b`` (float64 [ny, n] device tensor) is solved into
        ``x`` (same shape) when the request finishes.  Both tensors are kept
        alive by the handle until then.  Returns the request id."""
        import torch
        _require(b, torch.float64, self.level_shape(0, 1)[1:], "b")
        _require(x, torch.float64, self.level_shape(0, 1)[1:], "x")
        if rid is None:
            rid = self._next_id
        self._next_id = max(self._next_id, rid) + 1
        _check(_lib.nmg_serve_submit(self.ptr, int(rid), float(alpha), int(weight_set), _ptr(b), _ptr(x)))
        self._serve_refs[int(rid)] = (b, x)
        return int(rid)

    def serve_step(self, rtol: float = 1e-6, max_cycles: int = 100, nu1: int = 1, nu2: int = 1,
                   use_fprime: bool = False, precision: str = "mixed"):
        """One engine step; returns the list of finished :class:`RequestResult`."""
        done = (RequestResult * self.problem.max_batch)()
        nd = ctypes.c_int(0)
        o = _CycleOpts(nu1, nu2, 1 if use_fprime else 0, PRECISION[precision])
        _check(_lib.nmg_serve_step(self.ptr, float(rtol), int(max_cycles), ctypes.byref(o), done, ctypes.byref(nd),
                                   _stream()))
        out = [done[i] for i in range(nd.value)]
        for r in out:
            self._serve_refs.pop(int(r.id), None)
        return out

    def serve_pending(self):
        """``(queued, active)`` request counts."""
        q, a = ctypes.c_int(0), ctypes.c_int(0)
        _check(_lib.nmg_serve_pending(self.ptr, ctypes.byref(q), ctypes.byref(a)))
        return q.value, a.value

    def serve_reset(self) -> None:
        _check(_lib.nmg_serve_reset(self.ptr))
        self._serve_refs.clear()

    # -- training ----------------------------------------------------------
    def loss_grad(self, e, alpha, weight_set: int = 0, mask: str = "ramp", use_fprime: bool = False,
                  precision: str = "fp64", zero_grad: bool = True) -> np.ndarray:
        import torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        B = alpha.numel()
        _require(e, dt, self.level_shape(0, B), "e")
        _require(alpha, torch.float64, (B,), "alpha")
        losses = np.zeros(max(1, self.problem.levels - 1), dtype=np.float64)
        _check(_lib.nmg_loss_grad(self.ptr, weight_set, B, _ptr(alpha), _ptr(e), MASK[mask], int(use_fprime),
                                  PRECISION[precision], int(zero_grad), losses.ctypes.data_as(ctypes.c_void_p),
                                  _stream()))
        return losses

    def loss_forward(self, e, alpha, weight_set: int = 0, mask: str = "ramp", use_fprime: bool = False,
                     precision: str = "fp64") -> np.ndarray:
        """The losses of :meth:`loss_grad` without the adjoint (gradients untouched)."""
        import torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        B = alpha.numel()
        _require(e, dt, self.level_shape(0, B), "e")
        _require(alpha, torch.float64, (B,), "alpha")
        losses = np.zeros(max(1, self.problem.levels - 1), dtype=np.float64)
        _check(_lib.nmg_loss_forward(self.ptr, weight_set, B, _ptr(alpha), _ptr(e), MASK[mask], int(use_fprime),
                                     PRECISION[precision], losses.ctypes.data_as(ctypes.c_void_p), _stream()))
        return losses

    def rollout(self, e, alpha, k, weight_set=None, nu1: int = 1, nu2: int = 0, use_fprime: bool = False,
                precision: str = "fp32"):
        """Algorithm 5 DataGeneration in place on ``e``: sample ``i`` goes
        through ``k[i]`` cycles ``e <- e - MG(0, A e)``; returns ``y = A e``."""
        import torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        B = alpha.numel()
        _require(e, dt, self.level_shape(0, B), "e")
        _require(alpha, torch.float64, (B,), "alpha")
        ks = np.ascontiguousarray(np.asarray(k, dtype=np.int32).reshape(-1))
        if ks.size != B:
            raise ValueError(f"k must have {B} entries")
        ws = ctypes.c_void_p()
        if weight_set is not None:
            _require(weight_set, torch.int32, (B,), "weight_set")
            ws = _ptr(weight_set)
        y = torch.empty_like(e)
        o = _CycleOpts(nu1, nu2, 1 if use_fprime else 0, PRECISION[precision])
        _check(_lib.nmg_rollout(self.ptr, B, _ptr(alpha), ws, ks.ctypes.data_as(ctypes.c_void_p), _ptr(e), _ptr(y),
                                ctypes.byref(o), _stream()))
        return y

    def get_gradient(self, level: int, weight_set: int = 0) -> np.ndarray:
        out = np.empty(self.problem.weight_count(), dtype=np.float64)
        _check(_lib.nmg_get_gradient(self.ptr, level, weight_set, out.ctypes.data_as(ctypes.c_void_p), out.size))
        return out

    def adam_step(self, weight_set: int = 0, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8) -> None:
        _check(_lib.nmg_adam_step(self.ptr, weight_set, lr, beta1, beta2, eps, _stream()))

    def train_step(self, e, alpha, weight_set: int = 0, mask: str = "ramp", use_fprime: bool = False,
                   precision: str = "mixed", lr: float = 1e-3) -> np.ndarray:
        import torch
        dt = torch.float64 if precision == "fp64" else torch.float32
        B = alpha.numel()
        _require(e, dt, self.level_shape(0, B), "e")
        _require(alpha, torch.float64, (B,), "alpha")
        losses = np.zeros(max(1, self.problem.levels - 1), dtype=np.float64)
        _check(_lib.nmg_train_step(self.ptr, weight_set, B, _ptr(alpha), _ptr(e), MASK[mask], int(use_fprime),
                                   PRECISION[precision], float(lr), losses.ctypes.data_as(ctypes.c_void_p),
                                   _stream()))
        return losses

    # -- profiling ---------------------------------------------------------
    KERNELS = {"smoother": 0, "operator": 1, "restrict": 2, "prolong": 3, "coarse": 4, "fprime": 5, "refine": 6,
               "norm": 7}

    def debug_option(self, option: int, value: int) -> None:
        """``nmg_debug_option`` (1 = NMG_DEBUG_FP32_HANDOFF, 2 = NMG_DEBUG_SEPARATE_RESTRICT)."""
        _check(_lib.nmg_debug_option(self.ptr, int(option), int(value)))

    def set_graphs(self, enable: bool) -> None:
        """Replay solve iterations as captured HIP graphs (default) or launch eagerly."""
        _check(_lib.nmg_set_graphs(self.ptr, 1 if enable else 0))

    def profile_enable(self, kinds=("smoother",)) -> None:
        """Times the given kernel families (empty: profiling off)."""
        mask = 0
        for k in kinds:
            mask |= 1 << self.KERNELS[k]
        _check(_lib.nmg_profile_enable(self.ptr, mask))

    def profile_sample(self, period: int) -> None:
        """Time only every ``period``-th solve iteration."""
        _check(_lib.nmg_profile_sample(self.ptr, int(period)))

    def profile_rhs(self) -> int:
        """Active right-hand sides summed over the timed solve iterations."""
        v = ctypes.c_longlong(0)
        _check(_lib.nmg_profile_rhs(self.ptr, ctypes.byref(v)))
        return v.value

    def profile_levels(self, levels=None) -> None:
        """Time only the given levels (None: all levels)."""
        mask = 0xFFFF if levels is None else sum(1 << int(l) for l in levels)
        _check(_lib.nmg_profile_levels(self.ptr, mask))

    def profile_query(self, kind: str, level: int = -1):
        """``(total_ms, launches)`` of one kernel family (level -1: all levels)."""
        ms = ctypes.c_double(0.0)
        cnt = ctypes.c_int(0)
        _check(_lib.nmg_profile_query(self.ptr, self.KERNELS[kind], level, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    # -- introspection -----------------------------------------------------
    def debug_transfer_map(self, level: int, kind: int):
        ncount = self.level_size(level + 1) if kind == 0 else self.level_size(level)
        per = 3 if kind == 0 else 2
        idx = np.zeros((ncount, per), dtype=np.int32)
        w = np.zeros((ncount, per), dtype=np.float32)
        _check(_lib.nmg_debug_transfer_map(self.ptr, level, kind, idx.ctypes.data_as(ctypes.c_void_p),
                                           w.ctypes.data_as(ctypes.c_void_p)))
        return idx, w

    def debug_factor(self, level: int, which: int):
        r = ctypes.c_int(0)
        _check(_lib.nmg_debug_factor(self.ptr, level, which, ctypes.c_void_p(), ctypes.byref(r)))
        n = self.level_size(level)
        out = np.zeros((n, 2 * r.value + 1), dtype=np.float64)
        _check(_lib.nmg_debug_factor(self.ptr, level, which, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(r)))
        return out, r.value


def setup_hierarchy(problem: Problem) -> Handle:
    """``nmg_setup_hierarchy``: builds the hierarchy and returns a handle."""
    load_library()
    p = problem.to_c()
    h = Handle(problem=problem)
    _check(_lib.nmg_setup_hierarchy(ctypes.byref(p), ctypes.byref(h.ptr)))
    return h


def load_smoother_weights(h: Handle, level: int, weight_set: int, layers) -> None:
    h.load_smoother_weights(level, weight_set, layers)


def vcycle(h: Handle, *args, **kw):
    return h.vcycle(*args, **kw)


def solve(h: Handle, *args, **kw):
    return h.solve(*args, **kw)


def train_step(h: Handle, *args, **kw):
    return h.train_step(*args, **kw)


class Pool:
    """``nmg_pool``: continuous batching over several handles (one per grid
    size, say) with admission by a device-memory budget.  Handles stay owned
    by the caller and must outlive the pool."""

    def __init__(self, hbm_budget_bytes: int):
        load_library()
        self.ptr = ctypes.c_void_p()
        _check(_lib.nmg_pool_create(ctypes.c_size_t(int(hbm_budget_bytes)), ctypes.byref(self.ptr)))
        self.members = []
        self._refs = {}
        self._next_id = 0

    def add(self, handle: Handle) -> int:
        m = ctypes.c_int(-1)
        _check(_lib.nmg_pool_add(self.ptr, handle.ptr, ctypes.byref(m)))
        self.members.append(handle)
        return m.value

    def submit(self, member: int, b, x, alpha: float, weight_set: int = 0, rid: int | None = None) -> int:
        """Queues a request for ``member``; ``b``/``x`` are float64 device
        tensors of that member's grid, kept alive until the request finishes.
        Synchronises the current stream first, so ``b`` is ready for the
        pool's own streams."""
        import torch
        h = self.members[member]
        _require(b, torch.float64, h.level_shape(0, 1)[1:], "b")
        _require(x, torch.float64, h.level_shape(0, 1)[1:], "x")
        if rid is None:
            rid = self._next_id
        self._next_id = max(self._next_id, rid) + 1
        torch.cuda.current_stream().synchronize()
        _check(_lib.nmg_pool_submit(self.ptr, int(member), int(rid), float(alpha), int(weight_set), _ptr(b),
                                    _ptr(x)))
        self._refs[int(rid)] = (b, x)
        return int(rid)

    def step(self, rtol: float = 1e-6, max_cycles: int = 100, nu1: int = 1, nu2: int = 1, use_fprime: bool = False,
             precision: str = "mixed"):
        """Admission plus one outer iteration of every member with work;
        returns ``[(member, RequestResult), ...]`` of finished requests."""
        q, a = self.pending()[:2]
        cap = max(1, a + q)
        done = (RequestResult * cap)()
        dm = (ctypes.c_int * cap)()
        nd = ctypes.c_int(0)
        o = _CycleOpts(nu1, nu2, 1 if use_fprime else 0, PRECISION[precision])
        _check(_lib.nmg_pool_step(self.ptr, float(rtol), int(max_cycles), ctypes.byref(o), done, dm, cap,
                                  ctypes.byref(nd)))
        out = [(int(dm[i]), done[i]) for i in range(nd.value)]
        for _, r in out:
            self._refs.pop(int(r.id), None)
        return out

    def pending(self):
        """``(queued, active, bytes_in_flight)``."""
        q, a, by = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_size_t(0)
        _check(_lib.nmg_pool_pending(self.ptr, ctypes.byref(q), ctypes.byref(a), ctypes.byref(by)))
        return q.value, a.value, by.value

    def close(self) -> None:
        if self.ptr:
            _lib.nmg_pool_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()
            self._refs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
