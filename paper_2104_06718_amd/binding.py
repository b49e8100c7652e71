"""ctypes binding of the C ABI in include/ld.h (argument marshalling only).

Every step of the bounding method runs in the HIP library; this module only
turns torch tensors into device pointers and structs.  It fails loudly when the
built library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libld_mi355x.so")

LD_OK, LD_E_ARG, LD_E_SHAPE, LD_E_NUMERIC, LD_E_NOMEM, LD_E_DEVICE, LD_E_UNSUPPORTED, LD_E_STATE = \
    0, -1, -2, -3, -4, -5, -6, -7
LD_LINEAR, LD_CONV2D = 0, 1
LD_FP32, LD_BF16, LD_FP64 = 0, 1, 2
LD_INIT_CROWN, LD_INIT_ZERO, LD_INIT_GIVEN, LD_INIT_WK = 0, 1, 2, 3
LD_ENGINE_AUTO, LD_ENGINE_RESIDENT, LD_ENGINE_LAYERWISE = 0, 1, 2
TAU_DEFAULT = 2.0 ** -20

_PREC = {"fp32": LD_FP32, "bf16": LD_BF16, "fp64": LD_FP64, LD_FP32: LD_FP32, LD_BF16: LD_BF16, LD_FP64: LD_FP64}
_INIT = {"crown": LD_INIT_CROWN, "zero": LD_INIT_ZERO, "given": LD_INIT_GIVEN, "wk": LD_INIT_WK}
_ENGINE = {"auto": LD_ENGINE_AUTO, "resident": LD_ENGINE_RESIDENT, "layerwise": LD_ENGINE_LAYERWISE}

EXPORTED = ["ld_create_net", "ld_destroy_net", "ld_net_layer_width", "ld_net_num_layers",
            "ld_set_validation", "ld_state_create", "ld_state_destroy", "ld_state_set_rho",
            "ld_state_get_rho", "ld_state_get_rho_f64", "ld_state_get_step", "ld_state_reset",
            "ld_state_set_tracking", "ld_state_get_best", "ld_init_duals", "ld_dual_eval", "ld_dual_eval_noalloc", "ld_dual_eval_f64", "ld_rounding_margin",
            "ld_step", "ld_autotune", "ld_tuned_config", "ld_tuned_engine", "ld_tile_candidates",
            "ld_set_tuned_config", "ld_profile_iteration",
            "ld_intermediate_bounds", "ld_fsb_branch", "ld_bab", "ld_branch_children", "ld_sigmoid_hull", "ld_sigmoid_inner_min", "ld_prox_step", "ld_prox_get_step", "ld_prox_profile_iteration", "ld_final_bound", "ld_last_error"]


class LDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"LD error {code}: {msg}")
        self.code = code


class ld_layer(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("in_c", ctypes.c_int), ("in_h", ctypes.c_int), ("in_w", ctypes.c_int),
                ("out_c", ctypes.c_int), ("out_h", ctypes.c_int), ("out_w", ctypes.c_int), ("kh", ctypes.c_int),
                ("kw", ctypes.c_int), ("stride", ctypes.c_int), ("pad", ctypes.c_int),
                ("W", ctypes.c_void_p), ("b", ctypes.c_void_p)]


class ld_batch(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int), ("l0", ctypes.c_void_p), ("u0", ctypes.c_void_p),
                ("l", ctypes.POINTER(ctypes.c_void_p)), ("u", ctypes.POINTER(ctypes.c_void_p)),
                ("c", ctypes.c_void_p)]


class ld_opts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("total_iters", ctypes.c_int), ("lr0", ctypes.c_float),
                ("lr_end", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("precision", ctypes.c_int), ("init", ctypes.c_int),
                ("tie_tau", ctypes.c_float), ("engine", ctypes.c_int)]


_lib = None


class ld_prox_opts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("total_iters", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("eta0", ctypes.c_float), ("eta_end", ctypes.c_float), ("mu", ctypes.c_float),
                ("precision", ctypes.c_int), ("init", ctypes.c_int), ("tie_tau", ctypes.c_float)]


class ld_bab_opts(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int), ("root_iters", ctypes.c_int), ("iters", ctypes.c_int),
                ("root_lr0", ctypes.c_float), ("root_lr_end", ctypes.c_float), ("lr0", ctypes.c_float),
                ("lr_end", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("threshold", ctypes.c_float), ("gap", ctypes.c_float), ("max_rounds", ctypes.c_int),
                ("max_subproblems", ctypes.c_int), ("precision", ctypes.c_int), ("tie_tau", ctypes.c_float)]


class ld_bab_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("lower", ctypes.c_double), ("incumbent", ctypes.c_double),
                ("rounds", ctypes.c_int), ("leaves", ctypes.c_int), ("bounded", ctypes.c_longlong),
                ("max_open", ctypes.c_longlong)]


BAB_STATUS = {0: "verified", 1: "falsified", 2: "solved", 3: "limit"}


class ld_tile(ctypes.Structure):
    _fields_ = [("tn", ctypes.c_int), ("mwaves", ctypes.c_int), ("kwaves", ctypes.c_int), ("splits", ctypes.c_int),
                ("form", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def load_library(path: Optional[str] = None):
    """Load the built shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: build the HIP library first "
                          f"(python -m paper_2104_06718_amd.build or __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    V, I, P = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER
    lib.ld_last_error.restype = ctypes.c_char_p
    lib.ld_create_net.argtypes = [P(ld_layer), I, P(V)]
    lib.ld_destroy_net.argtypes = [V]
    lib.ld_destroy_net.restype = None
    lib.ld_net_layer_width.argtypes = [V, I, P(I)]
    lib.ld_net_num_layers.argtypes = [V, P(I)]
    lib.ld_set_validation.argtypes = [I]
    lib.ld_set_validation.restype = None
    lib.ld_state_create.argtypes = [V, I, P(V)]
    lib.ld_state_destroy.argtypes = [V]
    lib.ld_state_destroy.restype = None
    lib.ld_state_set_rho.argtypes = [V, P(V), V]
    lib.ld_state_get_rho.argtypes = [V, P(V), V]
    lib.ld_state_get_rho_f64.argtypes = [V, P(V), V]
    lib.ld_state_get_step.argtypes = [V, V, P(I)]
    lib.ld_state_reset.argtypes = [V, V]
    lib.ld_state_set_tracking.argtypes = [V, I, V]
    lib.ld_state_get_best.argtypes = [V, V, V, V]
    lib.ld_profile_iteration.argtypes = [V, P(ld_batch), V, P(ld_opts), I, P(ctypes.c_double), P(I), I, P(I), V]
    lib.ld_init_duals.argtypes = [V, P(ld_batch), I, I, P(V), V]
    lib.ld_dual_eval.argtypes = [V, P(ld_batch), P(V), V, P(V), I, ctypes.c_float, V]
    lib.ld_dual_eval_f64.argtypes = [V, P(ld_batch), P(V), V, P(V), ctypes.c_float, V]
    lib.ld_dual_eval_noalloc.argtypes = [V, P(ld_batch), P(V), V, P(V), I, ctypes.c_float, V]
    lib.ld_rounding_margin.argtypes = [V, P(ld_batch), P(V), V, V]
    lib.ld_step.argtypes = [V, P(ld_batch), V, P(ld_opts), V]
    lib.ld_autotune.argtypes = [V, P(ld_batch), P(ld_opts), V]
    lib.ld_tuned_config.argtypes = [V, I, I, I, I, P(ld_tile), P(ctypes.c_double)]
    lib.ld_tuned_engine.argtypes = [V, I, I, P(I), P(I), P(ctypes.c_double), P(ctypes.c_double)]
    lib.ld_tile_candidates.argtypes = [V, I, I, I, P(ld_tile), I, P(I)]
    lib.ld_set_tuned_config.argtypes = [V, I, I, I, I, P(ld_tile)]
    lib.ld_final_bound.argtypes = [V, P(ld_batch), V, V, V, V, V, ctypes.c_float, V]
    lib.ld_intermediate_bounds.argtypes = [V, P(ld_batch), P(ld_opts), I, V, V, V]
    lib.ld_fsb_branch.argtypes = [V, P(ld_batch), V, V, V, V, V]
    lib.ld_bab.argtypes = [V, P(ld_batch), P(ld_bab_opts), P(ld_bab_result), P(ctypes.c_float), V]
    lib.ld_sigmoid_hull.argtypes = [ctypes.c_longlong, V, V, V, V, V]
    lib.ld_sigmoid_inner_min.argtypes = [ctypes.c_longlong, V, V, V, V, V, V, V, V, V, V]
    lib.ld_branch_children.argtypes = [V, P(ld_batch), V, V, P(V), V, V, P(V), P(V), V, P(V), V]
    lib.ld_prox_step.argtypes = [V, P(ld_batch), V, P(ld_prox_opts), V]
    lib.ld_prox_get_step.argtypes = [V, P(I)]
    lib.ld_prox_profile_iteration.argtypes = [V, P(ld_batch), V, P(ld_prox_opts), I, P(ctypes.c_double), P(I), I,
                                              P(I), V]
    for name in EXPORTED:
        getattr(lib, name)
    if path is None:
        _lib = lib
    return lib


def _check(rc: int):
    if rc != LD_OK:
        raise LDError(rc, load_library().ld_last_error().decode())


def _ptrs(tensors: Sequence[Optional[torch.Tensor]]):
    arr = (ctypes.c_void_p * max(len(tensors), 1))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


class Net:
    """A ReLU network (list of layer dicts/specs), copied to the device by ld_create_net.

    Each layer: kind ('linear' | 'conv'), W, b (host float32 arrays),
    in_shape (C,H,W), out_shape (C,H,W), stride, pad.
    """

    def __init__(self, layers):
        import numpy as np
        self.lib = load_library()
        arr = (ld_layer * len(layers))()
        self._keep = []
        self.widths = []
        for i, L in enumerate(layers):
            get = (lambda k: L[k]) if isinstance(L, dict) else (lambda k: getattr(L, k))
            W = np.ascontiguousarray(np.asarray(get("W"), dtype=np.float32))
            b = np.ascontiguousarray(np.asarray(get("b"), dtype=np.float32))
            self._keep += [W, b]
            ins, outs = tuple(get("in_shape")), tuple(get("out_shape"))
            kind = get("kind")
            a = arr[i]
            a.kind = LD_LINEAR if kind == "linear" else LD_CONV2D
            a.in_c, a.in_h, a.in_w = ins
            a.out_c, a.out_h, a.out_w = outs
            if kind == "linear":
                a.kh = a.kw = a.stride = 1
                a.pad = 0
            else:
                a.kh, a.kw = W.shape[2], W.shape[3]
                a.stride, a.pad = int(get("stride")), int(get("pad"))
            a.W = W.ctypes.data
            a.b = b.ctypes.data
        h = ctypes.c_void_p()
        _check(self.lib.ld_create_net(arr, len(layers), ctypes.byref(h)))
        self.handle = h
        self.n = len(layers)
        w = ctypes.c_int()
        self.widths = []
        for k in range(self.n + 1):
            _check(self.lib.ld_net_layer_width(h, k, ctypes.byref(w)))
            self.widths.append(w.value)
        self._keep = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.ld_destroy_net(h)
            self.handle = None


class Batch:
    """Device arrays of B subdomains (float32 CUDA tensors; see ld_batch in include/ld.h)."""

    def __init__(self, l0, u0, l, u, c):
        self.l0 = _dev_f32(l0, "l0")
        self.u0 = _dev_f32(u0, "u0")
        self.l = [_dev_f32(t, "l[k]") for t in l]
        self.u = [_dev_f32(t, "u[k]") for t in u]
        self.c = _dev_f32(c, "c")
        self.B = int(l0.shape[0])
        self._la = _ptrs(self.l)
        self._ua = _ptrs(self.u)
        self.struct = ld_batch(self.B, self.l0.data_ptr(), self.u0.data_ptr(),
                               ctypes.cast(self._la, ctypes.POINTER(ctypes.c_void_p)),
                               ctypes.cast(self._ua, ctypes.POINTER(ctypes.c_void_p)), self.c.data_ptr())

    @staticmethod
    def from_instance(inst, device="cuda"):
        t = lambda a: torch.from_numpy(a).to(device)  # noqa: E731
        return Batch(t(inst.l0), t(inst.u0), [t(a) for a in inst.l], [t(a) for a in inst.u], t(inst.c))


class State:
    """Ascent state (rho, Adam moments, step counter) of B subdomains."""

    def __init__(self, net: Net, B: int):
        self.lib = net.lib
        self.net = net
        self.B = B
        h = ctypes.c_void_p()
        _check(self.lib.ld_state_create(net.handle, B, ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.ld_state_destroy(h)
            self.handle = None

    def set_rho(self, rho: List[torch.Tensor], stream=None):
        _check(self.lib.ld_state_set_rho(self.handle, _ptrs([_dev_f32(r, "rho") for r in rho]), _stream(stream)))

    def get_rho(self, stream=None) -> List[torch.Tensor]:
        out = [torch.empty((self.B, w), device="cuda", dtype=torch.float32) for w in self.net.widths[1:-1]]
        _check(self.lib.ld_state_get_rho(self.handle, _ptrs(out), _stream(stream)))
        return out

    def get_rho64(self, stream=None) -> List[torch.Tensor]:
        """The duals in FP64 (the FP64 engine's own, or the FP32 duals widened)."""
        out = [torch.empty((self.B, w), device="cuda", dtype=torch.float64) for w in self.net.widths[1:-1]]
        _check(self.lib.ld_state_get_rho_f64(self.handle, _ptrs(out), _stream(stream)))
        return out

    def reset(self, stream=None):
        _check(self.lib.ld_state_reset(self.handle, _stream(stream)))

    def set_tracking(self, on: bool = True, stream=None):
        """Keep the ascent's best dual value from now on (ld_state_set_tracking)."""
        _check(self.lib.ld_state_set_tracking(self.handle, int(bool(on)), _stream(stream)))

    def best(self, stream=None):
        """(best_q float64 [B], best_t int32 [B]) of the tracked steps (ld_state_get_best)."""
        q = torch.empty(self.B, device="cuda", dtype=torch.float64)
        t = torch.empty(self.B, device="cuda", dtype=torch.int32)
        _check(self.lib.ld_state_get_best(self.handle, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                          _stream(stream)))
        return q, t

    def step_count(self, stream=None) -> int:
        t = ctypes.c_int()
        _check(self.lib.ld_state_get_step(self.handle, _stream(stream), ctypes.byref(t)))
        return t.value

    def prox_step_count(self) -> int:
        t = ctypes.c_int()
        _check(self.lib.ld_prox_get_step(self.handle, ctypes.byref(t)))
        return t.value


def set_validation(on: bool):
    load_library().ld_set_validation(1 if on else 0)


def init_duals(net: Net, batch: Batch, init="crown", precision="fp32", stream=None) -> List[torch.Tensor]:
    out = [torch.empty((batch.B, w), device="cuda", dtype=torch.float32) for w in net.widths[1:-1]]
    _check(net.lib.ld_init_duals(net.handle, ctypes.byref(batch.struct), _INIT[init], _PREC[precision],
                                 _ptrs(out), _stream(stream)))
    return out


def dual_eval(net: Net, batch: Batch, rho: List[torch.Tensor], supergrad=True, precision="fp32",
              tau: float = TAU_DEFAULT, stream=None):
    """q(rho) [B] (float64) and, if requested, the supergradient per hidden layer."""
    q = torch.empty(batch.B, device="cuda", dtype=torch.float64)
    rho = [_dev_f32(r, "rho") for r in rho]
    s = None
    sp = None
    if supergrad:
        s = [torch.empty_like(r) for r in rho]
        sp = _ptrs(s)
    _check(net.lib.ld_dual_eval(net.handle, ctypes.byref(batch.struct), _ptrs(rho), ctypes.c_void_p(q.data_ptr()),
                                sp, _PREC[precision], ctypes.c_float(tau), _stream(stream)))
    return q, s


def dual_eval_noalloc(net: Net, batch: Batch, rho: List[torch.Tensor], q: torch.Tensor,
                      supergrad: Optional[List[torch.Tensor]] = None, precision="fp32", tau: float = TAU_DEFAULT,
                      stream=None):
    """ld_dual_eval_noalloc into caller-given outputs: q (float64 [B]) and, if given,
    supergrad (float32 [B, n_k] per hidden layer).  The library allocates nothing."""
    rho = [_dev_f32(r, "rho") for r in rho]
    sp = _ptrs([_dev_f32(t, "supergrad") for t in supergrad]) if supergrad is not None else None
    _check(net.lib.ld_dual_eval_noalloc(net.handle, ctypes.byref(batch.struct), _ptrs(rho),
                                        ctypes.c_void_p(q.data_ptr()), sp, _PREC[precision], ctypes.c_float(tau),
                                        _stream(stream)))


def dual_eval_f64(net: Net, batch: Batch, rho: List[torch.Tensor], supergrad=True, tau: float = TAU_DEFAULT,
                  stream=None):
    """q(rho) [B] and, if requested, the supergradient, both in FP64, at FP64 duals."""
    q = torch.empty(batch.B, device="cuda", dtype=torch.float64)
    for r in rho:
        if not (r.is_cuda and r.dtype == torch.float64 and r.is_contiguous()):
            raise ValueError("rho must be contiguous float64 CUDA tensors")
    s = sp = None
    if supergrad:
        s = [torch.empty_like(r) for r in rho]
        sp = _ptrs(s)
    _check(net.lib.ld_dual_eval_f64(net.handle, ctypes.byref(batch.struct), _ptrs(list(rho)),
                                    ctypes.c_void_p(q.data_ptr()), sp, ctypes.c_float(tau), _stream(stream)))
    return q, s


def rounding_margin(net: Net, batch: Batch, rho: List[torch.Tensor], stream=None) -> torch.Tensor:
    """Per-subdomain bound (float64 [B]) on how far the FP32-operand dual value at
    rho can exceed the exact q(rho) (ld_rounding_margin)."""
    m = torch.empty(batch.B, device="cuda", dtype=torch.float64)
    rho = [_dev_f32(r, "rho") for r in rho]
    _check(net.lib.ld_rounding_margin(net.handle, ctypes.byref(batch.struct), _ptrs(rho),
                                      ctypes.c_void_p(m.data_ptr()), _stream(stream)))
    return m


def step(net: Net, batch: Batch, state: State, iters: int, total_iters: Optional[int] = None, lr0=1e-2,
         lr_end=1e-4, beta1=0.9, beta2=0.999, eps=1e-8, precision="fp32", init="crown",
         tau: float = TAU_DEFAULT, engine="auto", stream=None):
    o = _opts(iters, total_iters, lr0, lr_end, beta1, beta2, eps, precision, init, tau, engine)
    _check(net.lib.ld_step(net.handle, ctypes.byref(batch.struct), state.handle, ctypes.byref(o), _stream(stream)))


def sigmoid_hull(l: torch.Tensor, u: torch.Tensor, stream=None):
    """Tangent points (t_up, t_lo) of the sigmoid's hull on [l, u] (ld_sigmoid_hull)."""
    l, u = _dev_f32(l, "l"), _dev_f32(u, "u")
    if l.shape != u.shape:
        raise ValueError("l and u differ in shape")
    tu, tl = torch.empty_like(l), torch.empty_like(l)
    _check(load_library().ld_sigmoid_hull(l.numel(), l.data_ptr(), u.data_ptr(), tu.data_ptr(), tl.data_ptr(),
                                          _stream(stream)))
    return tu, tl


def sigmoid_inner_min(rho, g, l, u, t_up, t_lo, stream=None):
    """(xB*, x*, value) of the sigmoid P_k inner minimisation (ld_sigmoid_inner_min)."""
    a = [_dev_f32(t, name) for t, name in ((rho, "rho"), (g, "g"), (l, "l"), (u, "u"), (t_up, "t_up"),
                                           (t_lo, "t_lo"))]
    if any(t.shape != a[0].shape for t in a):
        raise ValueError("operands differ in shape")
    xb, x = torch.empty_like(a[0]), torch.empty_like(a[0])
    val = torch.empty(a[0].shape, device="cuda", dtype=torch.float64)
    _check(load_library().ld_sigmoid_inner_min(a[0].numel(), *[t.data_ptr() for t in a], xb.data_ptr(), x.data_ptr(),
                                               val.data_ptr(), _stream(stream)))
    return xb, x, val


def fsb_branch(net: Net, batch: Batch, candidates=False, stream=None):
    """FSB's split per subdomain (ld_fsb_branch): (layer [B] int32, index [B] int32,
    value [B] float64) and, if asked, the prefilter's candidates [B, n-1, 2]."""
    B = batch.B
    layer = torch.empty(B, device="cuda", dtype=torch.int32)
    index = torch.empty(B, device="cuda", dtype=torch.int32)
    value = torch.empty(B, device="cuda", dtype=torch.float64)
    cand = torch.empty((B, len(net.widths) - 2, 2), device="cuda", dtype=torch.int32) if candidates else None
    _check(net.lib.ld_fsb_branch(net.handle, ctypes.byref(batch.struct), ctypes.c_void_p(layer.data_ptr()),
                                 ctypes.c_void_p(index.data_ptr()), ctypes.c_void_p(value.data_ptr()),
                                 ctypes.c_void_p(cand.data_ptr()) if cand is not None else None, _stream(stream)))
    return (layer, index, value, cand) if candidates else (layer, index, value)


def bab(net: Net, root: Batch, threshold=0.0, gap=0.0, batch=64, root_iters=100, iters=50, root_lr0=1e-2,
        root_lr_end=1e-4, lr0=1e-3, lr_end=1e-4, beta1=0.9, beta2=0.999, eps=1e-8, max_rounds=1000,
        max_subproblems=1 << 16, precision="fp32", tau: float = TAU_DEFAULT, stream=None):
    """Branch and bound on one property (ld_bab): root is a Batch of one subdomain.
    Returns a dict with status ('verified', 'falsified', 'solved', 'limit'), lower,
    incumbent, rounds, leaves, bounded, max_open and x_best (the incumbent's input,
    a float32 CPU tensor, or None)."""
    o = ld_bab_opts(int(batch), int(root_iters), int(iters), root_lr0, root_lr_end, lr0, lr_end, beta1, beta2, eps,
                    float(threshold), float(gap), int(max_rounds), int(max_subproblems), _PREC[precision], tau)
    r = ld_bab_result()
    x = (ctypes.c_float * net.widths[0])(*([float("nan")] * net.widths[0]))
    _check(net.lib.ld_bab(net.handle, ctypes.byref(root.struct), ctypes.byref(o), ctypes.byref(r), x,
                          _stream(stream)))
    xb = torch.tensor(list(x), dtype=torch.float32)
    return dict(status=BAB_STATUS[r.status], lower=r.lower, incumbent=r.incumbent, rounds=r.rounds, leaves=r.leaves,
                bounded=r.bounded, max_open=r.max_open, x_best=None if bool(torch.isnan(xb).all()) else xb)


def branch_children(net: Net, batch: Batch, layer: torch.Tensor, index: torch.Tensor, rho=None, stream=None):
    """The 2B children of the splits (ld_branch_children): a Batch and, if the
    parents' duals are given, the children's warm-start duals."""
    B = batch.B
    w = net.widths
    l0 = torch.empty((2 * B, w[0]), device="cuda", dtype=torch.float32)
    u0 = torch.empty_like(l0)
    lo = [torch.empty((2 * B, x), device="cuda", dtype=torch.float32) for x in w[1:-1]]
    hi = [torch.empty_like(x) for x in lo]
    c = torch.empty((2 * B, w[-1]), device="cuda", dtype=torch.float32)
    layer = layer.to(device="cuda", dtype=torch.int32).contiguous()
    index = index.to(device="cuda", dtype=torch.int32).contiguous()
    rp = ro = None
    rho_out = None
    if rho is not None:
        rho = [_dev_f32(r, "rho") for r in rho]
        rho_out = [torch.empty((2 * B, r.shape[1]), device="cuda", dtype=torch.float32) for r in rho]
        rp, ro = _ptrs(rho), _ptrs(rho_out)
    _check(net.lib.ld_branch_children(net.handle, ctypes.byref(batch.struct), ctypes.c_void_p(layer.data_ptr()),
                                      ctypes.c_void_p(index.data_ptr()), rp, ctypes.c_void_p(l0.data_ptr()),
                                      ctypes.c_void_p(u0.data_ptr()), _ptrs(lo), _ptrs(hi),
                                      ctypes.c_void_p(c.data_ptr()), ro, _stream(stream)))
    kids = Batch(l0, u0, lo, hi, c)
    return (kids, rho_out) if rho is not None else kids


def intermediate_bounds(sub: Net, batch: Batch, iters: int, total_iters: Optional[int] = None, lr0=1e-2,
                        lr_end=1e-4, beta1=0.9, beta2=0.999, eps=1e-8, precision="fp32", init="crown",
                        tau: float = TAU_DEFAULT, engine="auto", max_problems=0, stream=None):
    """LD bounds (lo, hi), each [B, n_j] float32, on the pre-activations of the last
    layer of `sub` (the network of the first j layers) for every subdomain of
    `batch` (ld_intermediate_bounds; batch.c is not read)."""
    nj = sub.widths[-1]
    lo = torch.empty((batch.B, nj), device="cuda", dtype=torch.float32)
    hi = torch.empty_like(lo)
    o = _opts(iters, total_iters, lr0, lr_end, beta1, beta2, eps, precision, init, tau, engine)
    _check(sub.lib.ld_intermediate_bounds(sub.handle, ctypes.byref(batch.struct), ctypes.byref(o), int(max_problems),
                                          ctypes.c_void_p(lo.data_ptr()), ctypes.c_void_p(hi.data_ptr()),
                                          _stream(stream)))
    return lo, hi


def prox_step(net: Net, batch: Batch, state: State, iters: int, total_iters: Optional[int] = None,
              inner_iters=2, eta0=10.0, eta_end=500.0, mu=0.3, precision="fp32", init="crown",
              tau: float = TAU_DEFAULT, stream=None):
    """`iters` outer iterations of the proximal solver (ld_prox_step)."""
    o = ld_prox_opts(iters, iters if total_iters is None else total_iters, inner_iters, eta0, eta_end, mu,
                     _PREC[precision], _INIT[init], tau)
    _check(net.lib.ld_prox_step(net.handle, ctypes.byref(batch.struct), state.handle, ctypes.byref(o),
                                _stream(stream)))


def prox_profile_iteration(net: Net, batch: Batch, state: State, reps=20, total_iters=100, inner_iters=2,
                           eta0=10.0, eta_end=500.0, mu=0.3, precision="fp32", tau: float = TAU_DEFAULT,
                           stream=None):
    """[(slot, average us per launch)] of one proximal outer iteration (ld_prox_profile_iteration)."""
    o = ld_prox_opts(1, total_iters, inner_iters, eta0, eta_end, mu, _PREC[precision], _INIT["crown"], tau)
    avg = (ctypes.c_double * 64)()
    kinds = (ctypes.c_int * 64)()
    ns = ctypes.c_int()
    _check(net.lib.ld_prox_profile_iteration(net.handle, ctypes.byref(batch.struct), state.handle, ctypes.byref(o),
                                             reps, avg, kinds, 64, ctypes.byref(ns), _stream(stream)))
    return [(kinds[i], avg[i]) for i in range(ns.value)]


def autotune(net: Net, batch: Batch, total_iters=500, lr0=1e-2, lr_end=1e-4, beta1=0.9, beta2=0.999, eps=1e-8,
             precision="fp32", tau: float = TAU_DEFAULT, stream=None):
    """Run the autotuner for (batch.B, precision); returns tuning_info()."""
    o = _opts(1, total_iters, lr0, lr_end, beta1, beta2, eps, precision, "crown", tau)
    _check(net.lib.ld_autotune(net.handle, ctypes.byref(batch.struct), ctypes.byref(o), _stream(stream)))
    return tuning_info(net, batch.B, precision)


def tuning_info(net: Net, B: int, precision="fp32"):
    """Tuned engine and per-contraction configuration for (B, precision), or None."""
    eng, conc, ul, ur = ctypes.c_int(), ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    rc = net.lib.ld_tuned_engine(net.handle, int(B), _PREC[precision], ctypes.byref(eng), ctypes.byref(conc),
                                 ctypes.byref(ul), ctypes.byref(ur))
    if rc == LD_E_STATE:
        return None
    _check(rc)
    names = {v: k for k, v in _ENGINE.items()}
    out = dict(engine=names[eng.value], concurrent_phases=bool(conc.value), us_per_iter_layerwise=ul.value,
               us_per_iter_resident=ur.value, layers=[])
    t, us = ld_tile(), ctypes.c_double()
    for k in range(1, len(net.widths) - 1):
        for d, dname in ((1, "transposed"), (0, "forward")):
            _check(net.lib.ld_tuned_config(net.handle, int(B), _PREC[precision], k, d, ctypes.byref(t),
                                           ctypes.byref(us)))
            out["layers"].append(dict(layer=k, dir=dname, us=us.value, **t.as_dict()))
    return out


def tile_candidates(net: Net, B: int, k: int, direction: str):
    """Candidate launch configurations (dicts with tn, mwaves, kwaves, splits,
    form) of a contraction (direction 'forward' or 'transposed' of hidden layer k)."""
    d = 1 if direction == "transposed" else 0
    cnt = ctypes.c_int()
    _check(net.lib.ld_tile_candidates(net.handle, int(B), int(k), d, None, 0, ctypes.byref(cnt)))
    n = cnt.value
    arr = (ld_tile * max(n, 1))()
    _check(net.lib.ld_tile_candidates(net.handle, int(B), int(k), d, arr, n, ctypes.byref(cnt)))
    return [arr[i].as_dict() for i in range(n)]


def set_tuned_config(net: Net, B: int, precision: str, k: int, direction: str, tile: dict):
    """Pin one contraction's configuration (a dict from tile_candidates)."""
    d = 1 if direction == "transposed" else 0
    t = ld_tile(**{f: int(tile[f]) for f, _ in ld_tile._fields_})
    _check(net.lib.ld_set_tuned_config(net.handle, int(B), _PREC[precision], int(k), d, ctypes.byref(t)))


def _opts(iters, total_iters, lr0, lr_end, beta1, beta2, eps, precision, init, tau, engine="auto"):
    return ld_opts(int(iters), int(total_iters if total_iters is not None else iters), lr0, lr_end, beta1, beta2,
                   eps, _PREC[precision], _INIT[init], tau, _ENGINE[engine])


def profile_iteration(net: Net, batch: Batch, state: State, reps=10, total_iters=500, lr0=1e-2, lr_end=1e-4,
                      beta1=0.9, beta2=0.999, eps=1e-8, precision="fp32", init="crown", tau: float = TAU_DEFAULT,
                      stream=None):
    """Average duration (us) of every kernel launch of one ascent iteration, with its kind."""
    o = _opts(reps, total_iters, lr0, lr_end, beta1, beta2, eps, precision, init, tau)
    avg = (ctypes.c_double * 64)()
    kinds = (ctypes.c_int * 64)()
    ns = ctypes.c_int()
    _check(net.lib.ld_profile_iteration(net.handle, ctypes.byref(batch.struct), state.handle, ctypes.byref(o),
                                        int(reps), avg, kinds, 64, ctypes.byref(ns), _stream(stream)))
    return [(kinds[i], avg[i]) for i in range(ns.value)]


def final_bound(net: Net, batch: Batch, state: State, tau: float = TAU_DEFAULT, stream=None):
    B = batch.B
    d = dict(bound=torch.empty(B, device="cuda", dtype=torch.float64),
             q_final=torch.empty(B, device="cuda", dtype=torch.float64),
             primal=torch.empty(B, device="cuda", dtype=torch.float64),
             feasible=torch.empty(B, device="cuda", dtype=torch.int32))
    _check(net.lib.ld_final_bound(net.handle, ctypes.byref(batch.struct), state.handle,
                                  *(ctypes.c_void_p(d[k].data_ptr()) for k in ("bound", "q_final", "primal",
                                                                               "feasible")),
                                  ctypes.c_float(tau), _stream(stream)))
    return d


class LDDual(torch.autograd.Function):
    """q(rho) as a differentiable function of the duals (Section 5.1, eq:nonprox_problem).

    ``LDDual.apply(net, batch, precision, tau, *rho) -> q`` ([B], float64).  The
    dual is concave and piecewise linear; its supergradient at rho is
    s_k = xB*_k - (W_k x*_{k-1} + b_k) (Algorithm 1), which backward returns,
    scaled by the incoming gradient of each subdomain's q.  Forward keeps only
    the duals: backward recomputes every layer's inner minimisers and forward
    products in one more library call instead of storing them, so the memory
    held between forward and backward is the size of rho itself.  Where several
    minimisers exist (a kink) the returned element is the one the tie rule
    selects, a valid supergradient.
    """

    @staticmethod
    def forward(ctx, net: Net, batch: Batch, precision: str, tau: float, *rho):
        q, _ = dual_eval(net, batch, list(rho), supergrad=False, precision=precision, tau=tau)
        ctx.net, ctx.batch, ctx.precision, ctx.tau = net, batch, precision, tau
        ctx.save_for_backward(*rho)
        return q

    @staticmethod
    def backward(ctx, grad_q):
        rho = ctx.saved_tensors
        _, s = dual_eval(ctx.net, ctx.batch, list(rho), supergrad=True, precision=ctx.precision, tau=ctx.tau)
        w = grad_q.to(torch.float64).unsqueeze(1)
        grads = [(w * sk.to(torch.float64)).to(r.dtype) for sk, r in zip(s, rho)]
        return (None, None, None, None, *grads)


def ld_dual(net: Net, batch: Batch, rho: Sequence[torch.Tensor], precision="fp32",
            tau: float = TAU_DEFAULT) -> torch.Tensor:
    """Differentiable q(rho): ``ld_dual(net, batch, rho).sum().backward()`` fills
    every rho_k.grad with the supergradient s_k."""
    return LDDual.apply(net, batch, precision, tau, *rho)
