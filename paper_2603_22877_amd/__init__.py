"""MI355X-native FourierSMT hot path: Python binding of ``libfsmt.so``.

Every function here marshals arguments for one C-ABI call of the same name (see
``include/fsmt.h``); all arithmetic runs in the HIP kernels. PyTorch provides device
memory and streams only. Tensors are float32 on the handle's device, shaped [R][n]
(any strides, e.g. a transposed [n][R] buffer viewed as [R][n]).
"""
from __future__ import annotations

import ctypes as ct
from typing import Optional

import numpy as np

from . import _abi
from ._abi import (FSMT_ACCUMULATE, FSMT_HOST_ONLY, FSMT_MSG_AUTO, FSMT_MSG_LDS, FSMT_PROJ_BOX,  # noqa: F401
                   FSMT_PROJ_UNIT, FsmtError)

__all__ = ["XBDD", "xbdd_compile", "xbdd_free", "xbdd_info", "xbdd_export_diagram", "cop_forward",
           "cop_backward", "pgd_step", "round_and_check", "erwa_update", "fsmt_solve_batched", "fsmt_solve_batched_noalloc", "fsmt_solve_status", "FsmtError",
           "FSMT_ACCUMULATE", "FSMT_HOST_ONLY", "view", "lib"]


def lib():
    return _abi.load()


_PROBLEM_FIELDS = (("atom_ptr", np.int64), ("atom_var", np.int32), ("atom_coef", np.float64),
                   ("atom_rhs", np.float64), ("atom_op", np.int8), ("con_kind", np.int32),
                   ("con_ptr", np.int64), ("con_lit", np.int32), ("con_param", np.int32),
                   ("expr_ptr", np.int64), ("expr_ops", np.int32), ("real_lo", np.float64),
                   ("real_hi", np.float64))


class XBDD:
    """Owner of a compiled handle (``xbdd_compile`` result); freed by :meth:`free`."""

    def __init__(self, ptr: int, problem):
        self.ptr = ptr
        self.n_bool = int(problem.n_bool)
        self.n_real = int(problem.n_real)
        self.n_cons = int(problem.con_kind.shape[0])
        self.n_atoms = int(problem.atom_rhs.shape[0])

    @property
    def handle(self):
        if not self.ptr:
            raise ValueError("handle already freed")
        return ct.c_void_p(self.ptr)

    def free(self) -> None:
        if self.ptr:
            lib().xbdd_free(ct.c_void_p(self.ptr))
            self.ptr = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def xbdd_compile(problem, device: Optional[int] = None, max_nodes: int = 0,
                 projection: int = 0, messages: int = 0) -> XBDD:
    """Compile a problem (object with the ``workloads.format.Problem`` arrays).

    ``device``: HIP device index, None for the current one, or FSMT_HOST_ONLY.
    ``projection``: FSMT_PROJ_UNIT (box + unit atoms, default) or FSMT_PROJ_BOX.
    ``messages``: FSMT_MSG_AUTO (closed forms for recognized families, registers when the
    other diagrams are small; default), FSMT_MSG_LDS or FSMT_MSG_GENERIC (no closed forms).
    """
    keep = {}
    s = _abi.Problem()
    s.n_bool, s.n_real = int(problem.n_bool), int(problem.n_real)
    s.n_atoms, s.n_cons = int(problem.atom_rhs.shape[0]), int(problem.con_kind.shape[0])
    for name, dt in _PROBLEM_FIELDS:
        arr = np.ascontiguousarray(getattr(problem, name), dtype=dt)
        if arr.size == 0:
            arr = np.zeros(1, dt)
        keep[name] = arr
        setattr(s, name, arr.ctypes.data)
    o = _abi.CompileOpts()
    o.device = -1 if device is None else int(device)
    o.max_nodes = int(max_nodes)
    o.projection = int(projection)
    o.messages = int(messages)
    out = ct.c_void_p()
    _abi.check(lib().xbdd_compile(ct.byref(s), ct.byref(o), ct.byref(out)))
    return XBDD(out.value, problem)


def xbdd_free(h: XBDD) -> None:
    h.free()


def xbdd_info(h: XBDD) -> dict:
    st = _abi.Stats()
    _abi.check(lib().xbdd_info(h.handle, ct.byref(st)))
    return {k: getattr(st, k) for k, _ in st._fields_}


def xbdd_export_diagram(h: XBDD, c: int, max_nodes: int = 4096, max_slots: int = 4096) -> dict:
    nn, ns, nb, root = ct.c_int32(), ct.c_int32(), ct.c_int32(), ct.c_int32()
    nodes = np.zeros(3 * max_nodes, np.int32)
    sup = np.zeros(max_slots, np.int32)
    _abi.check(lib().xbdd_export_diagram(h.handle, int(c), max_nodes, max_slots, ct.byref(nn),
                                         ct.byref(ns), ct.byref(nb), ct.byref(root),
                                         nodes.ctypes.data, sup.ctypes.data))
    return dict(n_nodes=nn.value, n_slots=ns.value, n_bslots=nb.value, root=root.value,
                nodes=nodes[:3 * nn.value].reshape(-1, 3).copy(), support=sup[:ns.value].copy())


# ---------------------------------------------------------------------- tensors -> views
def view(t, rows: Optional[int] = None) -> _abi.View:
    """fsmt_view of a float32 tensor: 2-D [R][n]; a 1-D tensor [n] becomes a broadcast row."""
    import torch
    if t is None:
        return _abi.View()
    if t.dtype != torch.float32:
        raise TypeError("float32 tensor expected")
    v = _abi.View()
    v.data = t.data_ptr() if t.numel() > 0 else None
    if t.dim() == 1:
        v.rows, v.cols = 1, t.shape[0]
        v.stride_r, v.stride_v = 0, t.stride(0)
    elif t.dim() == 2:
        v.rows, v.cols = t.shape
        v.stride_r, v.stride_v = t.stride()
    else:
        raise ValueError("1-D or 2-D tensor expected")
    return v


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def cop_forward(h: XBDD, a, b, kappa: float, w, obj, unsat=None, flags: int = 0, stream=None):
    _abi.check(lib().cop_forward(h.handle, view(a), view(b), float(kappa), view(w), _ptr(obj),
                                 view(unsat), int(flags), _stream(stream)))


def cop_backward(h: XBDD, a, b, kappa: float, w, obj, grad_a, grad_b, flags: int = 0, stream=None):
    _abi.check(lib().cop_backward(h.handle, view(a), view(b), float(kappa), view(w), _ptr(obj),
                                  view(grad_a), view(grad_b), int(flags), _stream(stream)))


def pgd_step(h: XBDD, a, b, grad_a, grad_b, eta_a: float, eta_b: float, gmap_sq=None,
             flags: int = 0, stream=None):
    _abi.check(lib().pgd_step(h.handle, view(a), view(b), view(grad_a), view(grad_b),
                              float(eta_a), float(eta_b), _ptr(gmap_sq), int(flags),
                              _stream(stream)))


def round_and_check(h: XBDD, a, b, x, sat_bits, n_unsat, verdict, stream=None):
    _abi.check(lib().round_and_check(h.handle, view(a), view(b), _ptr(x), _ptr(sat_bits),
                                     _ptr(n_unsat), _ptr(verdict), _stream(stream)))


def erwa_update(h: XBDD, R: int, sat_bits, w, hist, level: int, rho: float = 0.5,
                gamma: float = 2.0, tau: int = 1, normalize: bool = True, stream=None):
    _abi.check(lib().erwa_update(h.handle, int(R), _ptr(sat_bits), _ptr(w), _ptr(hist), int(level),
                                 float(rho), float(gamma), int(tau), int(bool(normalize)),
                                 _stream(stream)))


def fsmt_solve_batched(handles, opts: _abi.SolveOpts, states, stream=None):
    n = len(handles)
    harr = (ct.c_void_p * n)(*[h.ptr for h in handles])
    sarr = (_abi.SolveState * n)(*states)
    _abi.check(lib().fsmt_solve_batched(ct.cast(harr, ct.c_void_p), n, ct.byref(opts),
                                        ct.cast(sarr, ct.c_void_p), _stream(stream)))


def fsmt_solve_batched_noalloc(handles, opts: _abi.SolveOpts, states, stream=None):
    """The allocation-free solver call (persistent schedule, library-owned device scratch)."""
    n = len(handles)
    harr = (ct.c_void_p * n)(*[h.ptr for h in handles])
    sarr = (_abi.SolveState * n)(*states)
    _abi.check(lib().fsmt_solve_batched_noalloc(ct.cast(harr, ct.c_void_p), n, ct.byref(opts),
                                                ct.cast(sarr, ct.c_void_p), _stream(stream)))


def fsmt_solve_status(states, stream=None):
    """Synchronize the stream and raise FsmtError(FSMT_EABORTED) if a solver call gave up."""
    n = len(states)
    sarr = (_abi.SolveState * n)(*states)
    _abi.check(lib().fsmt_solve_status(ct.cast(sarr, ct.c_void_p), n, _stream(stream)))
