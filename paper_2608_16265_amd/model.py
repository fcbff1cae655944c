"""Python binding of the evaluator: argument marshalling only.

Every callback runs in the HIP kernels of libexa.so; this module converts a
model description (exa_modeling.Model) into the C descriptors, checks tensor
arguments and forwards device pointers and the current torch stream.
"""
from __future__ import annotations

import ctypes as C
from typing import List

import numpy as np
import torch

from . import _lib
from ._lib import LIB, PatternDesc, Options, check


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class _Descriptors:
    """C pattern descriptors plus the numpy arrays that keep them alive."""

    def __init__(self, model):
        self.keep: List = []
        pats = model.patterns
        self.arr = (PatternDesc * max(1, len(pats)))()
        for i, p in enumerate(pats):
            nodes = p.nodes()
            icn = list(p.data.icols)
            fcn = list(p.data.fcols)
            op = np.array([_lib.OPCODE[n.op] for n in nodes], dtype=np.int32)
            a = np.empty(len(nodes), dtype=np.int32)
            b = np.empty(len(nodes), dtype=np.int32)
            off = np.zeros(len(nodes), dtype=np.int64)
            val = np.zeros(len(nodes), dtype=np.float64)
            for j, n in enumerate(nodes):
                a[j], b[j] = n.a, n.b
                if n.op == "const":
                    val[j] = n.value
                elif n.op == "data":
                    a[j] = fcn.index(n.col)
                elif n.op in ("var", "param"):
                    a[j] = -1 if n.col is None else icn.index(n.col)
                    off[j] = n.off
            icols = [np.ascontiguousarray(p.data.icols[c], dtype=np.int32) for c in icn]
            fcols = [np.ascontiguousarray(p.data.fcols[c], dtype=np.float64) for c in fcn]
            ic_ptrs = (C.POINTER(C.c_int32) * max(1, len(icols)))(*[_ptr(c, C.c_int32) for c in icols])
            fc_ptrs = (C.POINTER(C.c_double) * max(1, len(fcols)))(*[_ptr(c, C.c_double) for c in fcols])
            d = self.arr[i]
            d.kind = _lib.KIND[p.kind]
            d.nnodes = len(nodes)
            d.op, d.a, d.b = _ptr(op, C.c_int32), _ptr(a, C.c_int32), _ptr(b, C.c_int32)
            d.off, d.val = _ptr(off, C.c_int64), _ptr(val, C.c_double)
            d.ndata = p.ndata
            d.n_icols, d.n_fcols = len(icols), len(fcols)
            d.icols, d.fcols = ic_ptrs, fc_ptrs
            d.target = p.target
            d.row_icol = icn.index(p.row_col) if p.kind == "aug" else -1
            d.row_off = p.row_off
            keep = [op, a, b, off, val, icols, fcols, ic_ptrs, fc_ptrs]
            if p.kind == "con":
                lc = np.ascontiguousarray(p.lcon, dtype=np.float64)
                uc = np.ascontiguousarray(p.ucon, dtype=np.float64)
                d.lcon, d.ucon = _ptr(lc, C.c_double), _ptr(uc, C.c_double)
                keep += [lc, uc]
            self.keep.append(keep)
        self.n = len(pats)


# torch's query of the raw current-stream handle costs ~0.06 us, against
# ~2.7 us for building a torch.cuda.Stream object; the public call remains as
# the fallback for torch builds without it.
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream(dev=None):
    """Handle of torch's current HIP stream on device index `dev` (the current
    device when None), the stream every callback is enqueued on."""
    if dev is None:
        dev = torch.cuda.current_device()
    if _raw_stream is not None:
        return C.c_void_p(_raw_stream(dev))
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


_F64 = torch.float64


class ExaModel:
    """A compiled model on the current HIP device (Sec. 3.2 ExaModel)."""

    def __init__(self, model, *, host_only: bool = False, block: int = 256, epl: int = 4,
                 autotune: bool = False, fuse: bool = False, eval_per_mode: bool = False,
                 cache_dir: str = None, max_device_bytes: int = 0):
        self.description = model
        desc = _Descriptors(model)
        xl = np.ascontiguousarray(model.xl, dtype=np.float64)
        xu = np.ascontiguousarray(model.xu, dtype=np.float64)
        th = np.ascontiguousarray(model.theta, dtype=np.float64)
        opt = Options(1 if host_only else 0, block, epl, 1 if autotune else 0, 1 if fuse else 0,
                      1 if eval_per_mode else 0)
        opt.cache_dir = cache_dir.encode() if cache_dir else None
        opt.max_device_bytes = int(max_device_bytes)
        h = C.c_void_p()
        check(LIB.exa_create(desc.arr, desc.n, model.nvar, _ptr(xl, C.c_double), _ptr(xu, C.c_double),
                             model.ntheta, _ptr(th, C.c_double) if th.size else None,
                             C.byref(opt), C.byref(h)))
        self._h = h
        self.host_only = host_only
        n, m, nj, nh = (C.c_int64() for _ in range(4))
        check(LIB.exa_dims(h, C.byref(n), C.byref(m), C.byref(nj), C.byref(nh)))
        self.nvar, self.ncon, self.nnzj, self.nnzh = n.value, m.value, nj.value, nh.value
        self.ntheta = model.ntheta

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            check(LIB.exa_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- meta ---------------------------------------------------------------
    def bounds(self):
        xl, xu = np.empty(self.nvar), np.empty(self.nvar)
        gl, gu = np.empty(self.ncon), np.empty(self.ncon)
        check(LIB.exa_bounds(self._h, _ptr(xl, C.c_double), _ptr(xu, C.c_double),
                             _ptr(gl, C.c_double), _ptr(gu, C.c_double)))
        return xl, xu, gl, gu

    def jac_structure(self):
        r = np.empty(self.nnzj, dtype=np.int32)
        c = np.empty(self.nnzj, dtype=np.int32)
        check(LIB.exa_jac_structure(self._h, _ptr(r, C.c_int32), _ptr(c, C.c_int32)))
        return r, c

    def hess_structure(self):
        r = np.empty(self.nnzh, dtype=np.int32)
        c = np.empty(self.nnzh, dtype=np.int32)
        check(LIB.exa_hess_structure(self._h, _ptr(r, C.c_int32), _ptr(c, C.c_int32)))
        return r, c

    def generated_source(self) -> str:
        n = C.c_int64()
        check(LIB.exa_generated_source(self._h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value + 1)
        check(LIB.exa_generated_source(self._h, buf, n.value + 1, C.byref(n)))
        return buf.value.decode()

    def compile_check(self):
        """Compile the generated kernels for gfx950 (no GPU needed)."""
        check(LIB.exa_compile_check(self._h))

    def pattern_info(self, p: int) -> dict:
        out = np.zeros(8, dtype=np.int64)
        check(LIB.exa_pattern_info(self._h, p, _ptr(out, C.c_int64)))
        keys = ["kind", "ndata", "o1step", "o2step", "pstep", "o0", "o1", "o2"]
        return dict(zip(keys, out.tolist()))

    def kernel_bytes(self, callback: str):
        """(read, write) algorithmic bytes of one launch of a callback's
        evaluation kernel under its current schedule."""
        rd, wr = C.c_int64(), C.c_int64()
        check(LIB.exa_kernel_bytes(self._h, _lib.CALLBACKS.index(callback), C.byref(rd), C.byref(wr)))
        return rd.value, wr.value

    def schedule(self, callback: str) -> dict:
        out = np.zeros(4, dtype=np.int64)
        check(LIB.exa_schedule(self._h, _lib.CALLBACKS.index(callback), _ptr(out, C.c_int64)))
        return dict(block=int(out[0]), points_per_lane=int(out[1]), fused=int(out[2]) & 1,
                    unstaged=(int(out[2]) >> 1) & 1, tiles=int(out[3]))

    def device_bytes(self) -> int:
        out = C.c_int64()
        check(LIB.exa_device_bytes(self._h, C.byref(out)))
        return out.value

    def build_info(self) -> dict:
        out = np.zeros(6, dtype=np.float64)
        check(LIB.exa_build_info(self._h, out.ctypes.data_as(C.POINTER(C.c_double))))
        origin = {-1: "host_only", 0: "compiled", 1: "cache", 2: "shared"}[int(out[3])]
        return dict(host_ms=float(out[0]), codegen_ms=float(out[1]), compile_ms=float(out[2]), origin=origin,
                    device_bytes=int(out[4]), cache=bool(out[5]))

    def counters(self):
        out = np.zeros(9, dtype=np.int64)
        check(LIB.exa_counters(self._h, _ptr(out, C.c_int64)))
        return dict(zip(["obj", "grad", "cons", "jac", "hess", "jprod", "jtprod", "hprod", "adjoint"],
                        out.tolist()))

    # -- tensor plumbing ------------------------------------------------------
    @staticmethod
    def _dev(t, n, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype is not _F64 or t.numel() != n or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor with {n} entries")
        return C.c_void_p(t.data_ptr())

    def _out(self, out, n, ref, name):
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=ref.device)
        self._dev(out, n, name)
        return out

    # -- callbacks (Sec. 2.1.3) ---------------------------------------------
    def obj(self, x, out=None):
        """Device scalar tensor holding f(x)."""
        px = self._dev(x, self.nvar, "x")
        out = self._out(out, 1, x, "out")
        check(LIB.exa_obj(self._h, px, C.c_void_p(out.data_ptr()), _stream(x.get_device())))
        return out

    def obj_host(self, x) -> float:
        """f(x) as a Python float (the call waits for the stream)."""
        px = self._dev(x, self.nvar, "x")
        f = C.c_double()
        check(LIB.exa_obj_host(self._h, px, C.byref(f), _stream(x.get_device())))
        return f.value

    def grad(self, x, out=None):
        px = self._dev(x, self.nvar, "x")
        out = self._out(out, self.nvar, x, "out")
        check(LIB.exa_grad(self._h, px, C.c_void_p(out.data_ptr()), _stream(x.get_device())))
        return out

    def cons(self, x, out=None):
        px = self._dev(x, self.nvar, "x")
        out = self._out(out, self.ncon, x, "out")
        check(LIB.exa_cons(self._h, px, C.c_void_p(out.data_ptr()), _stream(x.get_device())))
        return out

    def jac_coord(self, x, out=None):
        px = self._dev(x, self.nvar, "x")
        out = self._out(out, self.nnzj, x, "out")
        check(LIB.exa_jac_coord(self._h, px, C.c_void_p(out.data_ptr()), _stream(x.get_device())))
        return out

    def hess_coord(self, x, y, obj_weight=1.0, out=None):
        px = self._dev(x, self.nvar, "x")
        py = self._dev(y, self.ncon, "y")
        out = self._out(out, self.nnzh, x, "out")
        check(LIB.exa_hess_coord(self._h, px, py, float(obj_weight), C.c_void_p(out.data_ptr()),
                                 _stream(x.get_device())))
        return out

    def jac_hess_coord(self, x, y, obj_weight=1.0, jac=None, hess=None):
        """Jacobian and Hessian values from one launch (bit-identical to the
        separate callbacks)."""
        px = self._dev(x, self.nvar, "x")
        py = self._dev(y, self.ncon, "y")
        jac = self._out(jac, self.nnzj, x, "jac")
        hess = self._out(hess, self.nnzh, x, "hess")
        check(LIB.exa_jac_hess_coord(self._h, px, py, float(obj_weight), C.c_void_p(jac.data_ptr()),
                                     C.c_void_p(hess.data_ptr()), _stream(x.get_device())))
        return jac, hess

    def jprod(self, x, v, out=None):
        px, pv = self._dev(x, self.nvar, "x"), self._dev(v, self.nvar, "v")
        out = self._out(out, self.ncon, x, "out")
        check(LIB.exa_jprod(self._h, px, pv, C.c_void_p(out.data_ptr()), _stream(x.get_device())))
        return out

    def jtprod(self, x, w, out=None):
        px, pw = self._dev(x, self.nvar, "x"), self._dev(w, self.ncon, "w")
        out = self._out(out, self.nvar, x, "out")
        check(LIB.exa_jtprod(self._h, px, pw, C.c_void_p(out.data_ptr()), _stream(x.get_device())))
        return out

    def hprod(self, x, y, obj_weight, v, out=None):
        px, py = self._dev(x, self.nvar, "x"), self._dev(y, self.ncon, "y")
        pv = self._dev(v, self.nvar, "v")
        out = self._out(out, self.nvar, x, "out")
        check(LIB.exa_hprod(self._h, px, py, float(obj_weight), pv, C.c_void_p(out.data_ptr()),
                            _stream(x.get_device())))
        return out

    def lag_grad(self, x, y, obj_weight=1.0, out=None):
        """sigma grad f(x) + J(x)^T y (exa_lag_grad)."""
        px, py = self._dev(x, self.nvar, "x"), self._dev(y, self.ncon, "y")
        out = self._out(out, self.nvar, x, "out")
        check(LIB.exa_lag_grad(self._h, px, py, float(obj_weight), C.c_void_p(out.data_ptr()),
                               _stream(x.get_device())))
        return out

    _CSC = {"jac": 0, "hess": 1}

    def csc_structure(self, which: str):
        """(colptr [nvar+1], rowval) of the compressed sparse columns of the
        Jacobian ("jac") or of the Hessian's lower triangle ("hess")."""
        k = self._CSC[which]
        nnz = C.c_int64()
        check(LIB.exa_csc_dims(self._h, k, C.byref(nnz)))
        colptr = np.empty(self.nvar + 1, dtype=np.int32)
        rowval = np.empty(nnz.value, dtype=np.int32)
        check(LIB.exa_csc_structure(self._h, k, _ptr(colptr, C.c_int32), _ptr(rowval, C.c_int32)))
        return colptr, rowval

    def csc_values(self, which: str, coo, out=None):
        """Compressed-column values from COO values (exa_csc_values)."""
        k = self._CSC[which]
        nnz = C.c_int64()
        check(LIB.exa_csc_dims(self._h, k, C.byref(nnz)))
        pc = self._dev(coo, self.nnzj if k == 0 else self.nnzh, "coo")
        out = self._out(out, nnz.value, coo, "out")
        check(LIB.exa_csc_values(self._h, k, pc, C.c_void_p(out.data_ptr()), _stream(coo.get_device())))
        return out

    def adjoint_theta(self, x, y, obj_weight, w, out=None):
        px, py = self._dev(x, self.nvar, "x"), self._dev(y, self.ncon, "y")
        pw = self._dev(w, self.nvar, "w")
        out = self._out(out, self.ntheta, x, "out")
        check(LIB.exa_adjoint_theta(self._h, px, py, float(obj_weight), pw,
                                    C.c_void_p(out.data_ptr()), _stream(x.get_device())))
        return out

    # -- several callbacks at one point (exa_eval) -----------------------------
    _EV_OUT = (("obj", "f", "f"), ("grad", "g", "n"), ("cons", "c", "m"), ("jac", "jac", "nnzj"),
               ("hess", "hess", "nnzh"), ("jprod", "jv", "m"), ("jtprod", "jtw", "n"),
               ("hprod", "hv", "n"))

    def _eval_args(self, x, y, obj_weight, v, w, outs):
        sizes = {"f": 1, "n": self.nvar, "m": self.ncon, "nnzj": self.nnzj, "nnzh": self.nnzh}
        a = _lib.EvalArgs()
        keep = [x]
        a.x = self._dev(x, self.nvar, "x")
        for cb, field, size in self._EV_OUT:
            t = outs.get(field)
            if t is None:
                continue
            a.mask |= _lib.EV[cb]
            setattr(a, field, self._dev(t, sizes[size], field))
            keep.append(t)
        if a.mask == 0:
            raise ValueError("give at least one output tensor (f, g, c, jac, hess, jv, jtw, hv)")
        for name, t, n, bits in (("y", y, self.ncon, ("hess", "hprod")), ("v", v, self.nvar, ("jprod", "hprod")),
                                 ("w", w, self.ncon, ("jtprod",))):
            if any(a.mask & _lib.EV[b] for b in bits):
                if t is None:
                    raise ValueError(f"{name} is needed by the selected callbacks")
                setattr(a, name, self._dev(t, n, name))
                keep.append(t)
        a.obj_weight = float(obj_weight)
        return a, keep

    def evaluate(self, x, y=None, obj_weight=1.0, v=None, w=None, *, f=None, g=None, c=None, jac=None,
                 hess=None, jv=None, jtw=None, hv=None):
        """Every callback whose output tensor is given, at one point, through
        exa_eval: one evaluation launch plus at most one reduction launch (one
        more for segments over 1,024 entries), each output bit-identical to
        its own callback's.  Outputs: f (obj), g
        (grad), c (cons), jac, hess, jv (jprod), jtw (jtprod), hv (hprod)."""
        a, _ = self._eval_args(x, y, obj_weight, v, w, dict(f=f, g=g, c=c, jac=jac, hess=hess, jv=jv, jtw=jtw,
                                                             hv=hv))
        check(LIB.exa_eval(self._h, C.byref(a), _stream(x.get_device())))

    def bind(self, x, y=None, obj_weight=1.0, v=None, w=None, *, f=None, g=None, c=None, jac=None, hess=None,
             jv=None, jtw=None, hv=None):
        """A reusable exa_eval call over fixed tensors: the arguments are
        checked once, and each call of the result evaluates the selected
        callbacks on the tensors' current contents (the caller updates them in
        place).  The bound tensors are kept alive by the returned object."""
        a, keep = self._eval_args(x, y, obj_weight, v, w, dict(f=f, g=g, c=c, jac=jac, hess=hess, jv=jv,
                                                                jtw=jtw, hv=hv))
        return BoundEval(self, a, keep, x.get_device())

    def eval_schedule(self, callbacks) -> dict:
        """Schedule exa_eval uses for a set of callback names (after its first
        call with that set)."""
        out = np.zeros(4, dtype=np.int64)
        check(LIB.exa_eval_schedule(self._h, self._eval_mask(callbacks), _ptr(out, C.c_int64)))
        return dict(block=int(out[0]), points_per_lane=int(out[1]), fused=int(out[2]) & 1,
                    one_pass=(int(out[2]) >> 1) & 1, jac_hess=(int(out[2]) >> 2) & 1,
                    unstaged=(int(out[2]) >> 4) & 1, tiles=int(out[3]))

    UNITS = {"per_callback": 0, "jac_hess": 1, "one_pass": 2}

    def set_eval_schedule(self, callbacks, block: int, points_per_lane: int, fused: bool = False,
                          units="per_callback", unstaged: bool = False):
        """Fix exa_eval's schedule for a set of callback names (no tuning):
        units is "per_callback" (Jacobian and Hessian tiles apart),
        "jac_hess" (Jacobian + Hessian units) or "one_pass"; unstaged stores
        each lane's Jacobian and Hessian values itself."""
        u = self.UNITS[units] if isinstance(units, str) else int(units)
        u |= _lib.UNSTAGED if unstaged else 0
        check(LIB.exa_eval_set_schedule(self._h, self._eval_mask(callbacks), int(block), int(points_per_lane),
                                        1 if fused else 0, u))

    @staticmethod
    def _eval_mask(callbacks) -> int:
        mask = 0
        for cb in callbacks:
            mask |= _lib.EV[cb]
        return mask

    def eval_bytes(self, callbacks) -> dict:
        """Algorithmic bytes of exa_eval's two launches for a set of callback
        names: {eval_read, eval_write, reduce_read, reduce_write}."""
        out = np.zeros(4, dtype=np.int64)
        check(LIB.exa_eval_bytes(self._h, self._eval_mask(callbacks), _ptr(out, C.c_int64)))
        return dict(zip(("eval_read", "eval_write", "reduce_read", "reduce_write"), out.tolist()))

    def eval_timing(self, enable: bool = True):
        """Turn on (or off) HIP-event timing of exa_eval's launches."""
        check(LIB.exa_eval_timing(self._h, 1 if enable else 0))

    def eval_timing_read(self) -> dict:
        """Average launch durations (us) of the exa_eval calls recorded since
        timing was turned on or last read."""
        out = np.zeros(4, dtype=np.float64)
        check(LIB.exa_eval_timing_read(self._h, _ptr(out, C.c_double)))
        return dict(calls=int(out[0]), eval_us=float(out[1]), reduce_calls=int(out[2]), reduce_us=float(out[3]))

    def set_theta(self, theta):
        pt = self._dev(theta, self.ntheta, "theta")
        check(LIB.exa_set_theta(self._h, pt, _stream(theta.get_device())))


class BoundEval:
    """exa_eval with its arguments fixed (see ExaModel.bind)."""

    def __init__(self, model, args, keep, device):
        self._model = model  # the model outlives the call
        self._args = args
        self._keep = keep
        self._ref = C.byref(args)
        self._dev = device

    @property
    def obj_weight(self) -> float:
        return self._args.obj_weight

    @obj_weight.setter
    def obj_weight(self, value: float):
        self._args.obj_weight = float(value)

    def __call__(self):
        check(LIB.exa_eval(self._model._h, self._ref, _stream(self._dev)))
