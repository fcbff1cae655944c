"""Batched evaluation of many instances of one formulation (binding only).

The instances (ExaModel objects whose pattern trees are identical, sizes may
differ) are evaluated together: one evaluation launch over the tiles of every
instance and selected callback, one launch of every instance's reductions,
replayed from a HIP graph; see exa_batch_* in include/exa.h.  Inputs and
outputs are the concatenations of the per-instance arrays (``offsets()``).
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np
import torch

from ._lib import EV_BATCH, LIB, UNITS, UNSTAGED, BatchIO, BatchOptions, check
from .model import ExaModel, _stream

_F64 = torch.float64
# io field -> (length kind, callback whose output it is, or None for inputs)
_OUTS = {"f": ("B", "obj"), "g": ("x", "grad"), "c": ("y", "cons"), "jac": ("jac", "jac"),
         "hess": ("hess", "hess"), "jv": ("y", "jprod"), "jtw": ("x", "jtprod"), "hv": ("x", "hprod"),
         "lag": ("x", "lag"), "theta_bar": ("theta", "adjoint")}
_INS = {"x": "x", "y": "y", "v": "x", "w": "y", "wx": "x"}


class ExaBatch:
    def __init__(self, models: Sequence[ExaModel], *, autotune: bool = True, block: int = 256,
                 epl: int = 4, fuse: bool = True, units: str = "jac_hess", use_graph: bool = True,
                 xcd_aware: bool = True):
        self.models = list(models)  # the models must outlive the batch
        arr = (C.c_void_p * len(self.models))(*[m.handle.value for m in self.models])
        opt = BatchOptions(1 if autotune else 0, block, epl, 1 if fuse else 0, UNITS[units],
                           1 if use_graph else 0, 1 if xcd_aware else 0, 0)
        h = C.c_void_p()
        check(LIB.exa_batch_create(arr, len(self.models), C.byref(opt), C.byref(h)))
        self._h = h
        B = len(self.models)
        self.B = B
        off = np.zeros(5 * (B + 1), dtype=np.int64)
        check(LIB.exa_batch_offsets(h, off.ctypes.data_as(C.POINTER(C.c_int64))))
        self._off = off.reshape(B + 1, 5)

    # -- layout --------------------------------------------------------------
    def offsets(self) -> np.ndarray:
        """(B + 1, 5) starts of each instance in x (nvar), y (ncon), jac
        (nnzj), hess (nnzh) and theta (ntheta) arrays; row B holds totals."""
        return self._off

    def total(self, what: str) -> int:
        if what == "B":
            return self.B
        return int(self._off[-1, {"x": 0, "y": 1, "jac": 2, "hess": 3, "theta": 4}[what]])

    def slice(self, what: str, i: int) -> slice:
        k = {"x": 0, "y": 1, "jac": 2, "hess": 3, "theta": 4}[what]
        return slice(int(self._off[i, k]), int(self._off[i + 1, k]))

    def concat(self, arrays, device="cuda:0"):
        return torch.as_tensor(np.concatenate([np.asarray(a, dtype=np.float64) for a in arrays]),
                               device=device)

    concat_x = concat
    concat_y = concat

    def empty(self, what: str, device="cuda:0"):
        return torch.empty(self.total(what), dtype=_F64, device=device)

    # -- parameters ----------------------------------------------------------
    def set_theta(self, theta):
        """Replace the batch's parameters (device [sum ntheta])."""
        t = self._p(theta, self.total("theta"), "theta")
        check(LIB.exa_batch_set_theta(self._h, t, _stream(theta.get_device())))

    # -- evaluation ----------------------------------------------------------
    @staticmethod
    def _p(t, n, name):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != _F64 \
                or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be a contiguous float64 device tensor with {n} entries")
        return C.c_void_p(t.data_ptr())

    def _io(self, x, y, obj_weight, v, w, wx, outs):
        io = BatchIO()
        io.x = self._p(x, self.total("x"), "x")
        io.y = self._p(y, self.total("y"), "y")
        io.obj_weight = float(obj_weight)
        io.v = self._p(v, self.total("x"), "v")
        io.w = self._p(w, self.total("y"), "w")
        io.wx = self._p(wx, self.total("x"), "wx")
        mask = 0
        for name, (kind, cb) in _OUTS.items():
            t = outs.get(name)
            if t is not None:
                setattr(io, name, self._p(t, self.total(kind), name))
                mask |= EV_BATCH[cb]
        if mask == 0:
            raise ValueError("no output given: nothing to evaluate")
        return io, mask

    def evaluate(self, x, y=None, obj_weight=1.0, v=None, w=None, wx=None, **outs):
        """Every callback whose output is given, for every instance, in one
        call (outputs: f, g, c, jac, hess, jv, jtw, hv, lag, theta_bar)."""
        unknown = set(outs) - set(_OUTS)
        if unknown:
            raise TypeError(f"unknown outputs {sorted(unknown)}")
        io, mask = self._io(x, y, obj_weight, v, w, wx, outs)
        check(LIB.exa_batch_eval(self._h, mask, C.byref(io), _stream(x.get_device())))
        return outs

    def bind(self, x, y=None, obj_weight=1.0, v=None, w=None, wx=None, **outs):
        """A zero-argument callable evaluating the given outputs at fixed
        tensors (the ctypes record is built once)."""
        io, mask = self._io(x, y, obj_weight, v, w, wx, outs)
        keep = (x, y, v, w, wx, outs)
        fn, h, dev = LIB.exa_batch_eval, self._h, x.get_device()

        def call():
            check(fn(h, mask, C.byref(io), _stream(dev)))
        call._keep = keep
        return call

    def eval(self, x, y, obj_weight, jac=None, hess=None):
        """Jacobian and/or Hessian values of every instance."""
        self.evaluate(x, y, obj_weight, jac=jac, hess=hess)

    # -- schedule and measurement ---------------------------------------------
    @staticmethod
    def mask(callbacks) -> int:
        m = 0
        for c in callbacks:
            m |= EV_BATCH[c]
        return m

    def schedule(self, callbacks=("jac", "hess")) -> dict:
        out = np.zeros(6, dtype=np.int64)
        check(LIB.exa_batch_schedule(self._h, self.mask(callbacks), out.ctypes.data_as(C.POINTER(C.c_int64))))
        d = dict(zip(["block", "points_per_lane", "fused", "units", "tiles", "tuned_ns"], out.tolist()))
        d["unstaged"] = int(bool(d["units"] & UNSTAGED))
        d["units"] = {v: k for k, v in UNITS.items()}[d["units"] & ~UNSTAGED]
        return d

    def set_schedule(self, callbacks, block: int, points_per_lane: int, fused: bool = True,
                     units: str = "jac_hess", unstaged: bool = False):
        u = UNITS[units] | (UNSTAGED if unstaged else 0)
        check(LIB.exa_batch_set_schedule(self._h, self.mask(callbacks), block, points_per_lane,
                                         1 if fused else 0, u))

    def kernel_bytes(self, callbacks=("jac", "hess")) -> dict:
        out = np.zeros(4, dtype=np.int64)
        check(LIB.exa_batch_bytes(self._h, self.mask(callbacks), out.ctypes.data_as(C.POINTER(C.c_int64))))
        return dict(zip(["eval_read", "eval_write", "reduce_read", "reduce_write"], out.tolist()))

    def timing(self, enable: bool = True):
        check(LIB.exa_batch_timing(self._h, 1 if enable else 0))

    def timing_read(self) -> dict:
        out = np.zeros(4, dtype=np.float64)
        check(LIB.exa_batch_timing_read(self._h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return dict(calls=int(out[0]), eval_us=float(out[1]), reduce_calls=int(out[2]), reduce_us=float(out[3]))

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            check(LIB.exa_batch_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
