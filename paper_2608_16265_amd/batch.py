"""Batched evaluation of many instances of one formulation (binding only).

The instances (ExaModel objects whose pattern trees are identical, sizes may
differ) are evaluated by one persistent kernel launch replayed from a HIP
graph; see exa_batch_* in include/exa.h.  Inputs and outputs are the
concatenations of the per-instance arrays.
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np
import torch

from ._lib import LIB, BatchOptions, CB_HESS, CB_JAC, check
from .model import ExaModel, _stream


class ExaBatch:
    def __init__(self, models: Sequence[ExaModel], *, autotune: bool = True, block: int = 256,
                 epl: int = 4, grid: int = 0, use_graph: bool = True, fuse: bool = True,
                 xcd_aware: bool = True, separate: bool = False):
        self.models = list(models)  # the models must outlive the batch
        arr = (C.c_void_p * len(self.models))(*[m.handle.value for m in self.models])
        opt = BatchOptions(1 if autotune else 0, block, epl, grid, 1 if use_graph else 0,
                           1 if fuse else 0, 1 if xcd_aware else 0, 1 if separate else 0)
        h = C.c_void_p()
        check(LIB.exa_batch_create(arr, len(self.models), C.byref(opt), C.byref(h)))
        self._h = h
        B = len(self.models)
        off = np.zeros(4 * (B + 1), dtype=np.int64)
        check(LIB.exa_batch_offsets(h, off.ctypes.data_as(C.POINTER(C.c_int64))))
        self._off = off.reshape(B + 1, 4)

    def offsets(self) -> np.ndarray:
        """(B + 1, 4) starts of each instance in x, y, jac and hess arrays."""
        return self._off

    def total(self, what: str) -> int:
        return int(self._off[-1, {"x": 0, "y": 1, "jac": 2, "hess": 3}[what]])

    def concat_x(self, xs):
        return torch.as_tensor(np.concatenate([np.asarray(x, dtype=np.float64) for x in xs]),
                               device="cuda:0")

    def concat_y(self, ys):
        return torch.as_tensor(np.concatenate([np.asarray(y, dtype=np.float64) for y in ys]),
                               device="cuda:0")

    @staticmethod
    def _p(t, n, name):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 \
                or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be a contiguous float64 device tensor with {n} entries")
        return C.c_void_p(t.data_ptr())

    def eval(self, x, y, obj_weight, jac=None, hess=None):
        mask = (CB_JAC if jac is not None else 0) | (CB_HESS if hess is not None else 0)
        px = self._p(x, self.total("x"), "x")
        py = self._p(y, self.total("y"), "y") if hess is not None else None
        check(LIB.exa_batch_eval(self._h, mask, px, py, float(obj_weight),
                                 self._p(jac, self.total("jac"), "jac"),
                                 self._p(hess, self.total("hess"), "hess"), _stream(x.get_device())))

    def kernel_bytes(self, jac: bool = True, hess: bool = True):
        mask = (CB_JAC if jac else 0) | (CB_HESS if hess else 0)
        rd, wr = C.c_int64(), C.c_int64()
        check(LIB.exa_batch_bytes(self._h, mask, C.byref(rd), C.byref(wr)))
        return rd.value, wr.value

    def schedule(self) -> dict:
        out = np.zeros(6, dtype=np.int64)
        check(LIB.exa_batch_schedule(self._h, out.ctypes.data_as(C.POINTER(C.c_int64))))
        return dict(zip(["block", "points_per_lane", "grid", "tiles", "tuned_ns", "combined"],
                        out.tolist()))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            check(LIB.exa_batch_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
