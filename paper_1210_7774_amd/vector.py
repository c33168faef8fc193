"""The bridge: a numpy-like front end that records array operations as vector
bytecode for the engine in libmgx.so (include/ve.h) and hands a batch over
when data is needed (the paper's "Bridge" section: instructions are collected
until the program reads an array).

Argument marshalling only: every element operation runs in the engine's
generated HIP kernels; torch provides device memory and the stream.

    import paper_1210_7774_amd.vector as vx
    eng = vx.Engine()
    full = eng.asarray(torch_tensor)            # caller-owned memory, no copy
    center, up = full[1:-1, 1:-1], full[:-2, 1:-1]
    work = eng.empty(center.shape)
    work[...] = center
    work += 0.2 * (up + center)
    center[...] = work
    eng.flush()                                  # or read: work.torch()

Temporaries record a free when Python drops them, which lets the engine
skip storing values nothing reads again.
"""
from __future__ import annotations

import ctypes
import math
import weakref

import numpy as np

from . import _abi

_DT = {"float64": _abi.VE_F64, "float32": _abi.VE_F32}
_ITEM = {_abi.VE_F64: 8, _abi.VE_F32: 4}


def _torch():
    import torch
    return torch


class VEError(RuntimeError):
    pass


class Engine:
    """One vector engine on the current device and stream."""

    def __init__(self, stream=None, batch_limit: int = 4096):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("the vector engine needs a ROCm GPU; there is no CPU path")
        self._L = _abi.lib()
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        h = ctypes.c_void_p(0)
        self._check(self._L.ve_create(ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)), "ve_create", None)
        self._h = h
        self._pending = []
        self._limit = batch_limit
        self._keep = []        # tensors bound as array-bases (kept alive)
        self._self = weakref.ref(self)

    # ---- plumbing
    def _check(self, rc, where, h="self"):
        if rc != _abi.VE_OK:
            msg = ""
            if h is not None and getattr(self, "_h", None):
                msg = self._L.ve_last_error(self._h).decode()
            raise VEError("%s failed (%d): %s" % (where, rc, msg))

    def _new_base(self, dtype: int, nelem: int, ptr=None) -> "_Base":
        bid = ctypes.c_int(0)
        self._check(self._L.ve_base_new(self._h, dtype, int(nelem), ctypes.c_void_p(ptr) if ptr else None,
                                        ctypes.byref(bid)), "ve_base_new")
        return _Base(self, bid.value, dtype, nelem)

    def record(self, op, out, ins=()):
        """Append one instruction (op name, out view, inputs) to the batch."""
        self._pending.append((op, out, tuple(ins)))
        if len(self._pending) >= self._limit:
            self.flush()

    def flush(self):
        """Execute the recorded batch (stream-ordered)."""
        if not self._pending or not self._h:
            return
        batch, self._pending = self._pending, []
        arr = _abi.ve_batch(batch)
        self._check(self._L.ve_execute(self._h, arr, len(batch)), "ve_execute")

    def execute(self, instrs):
        """Run raw (op, out, ins) instructions after the pending batch."""
        self.flush()
        arr = _abi.ve_batch(list(instrs))
        self._check(self._L.ve_execute(self._h, arr, len(instrs)), "ve_execute")

    def base_ptr(self, bid: int) -> int:
        p = ctypes.c_void_p(0)
        self._check(self._L.ve_base_ptr(self._h, bid, ctypes.byref(p)), "ve_base_ptr")
        return p.value or 0

    def register(self, expr: str, nin: int) -> int:
        """A user-defined element-wise operation; returns its opcode."""
        op = ctypes.c_int(0)
        self._check(self._L.ve_register(self._h, expr.encode(), nin, ctypes.byref(op)), "ve_register")
        return op.value

    def stats(self) -> dict:
        s = _abi.VeStats()
        self._check(self._L.ve_stats_get(self._h, ctypes.byref(s)), "ve_stats_get")
        return {k: getattr(s, k) for k, _ in s._fields_}

    def profile(self, on: bool):
        self.flush()
        self._check(self._L.ve_profile(self._h, int(bool(on))), "ve_profile")

    def profile_read(self):
        self.flush()
        buf = (_abi.VeKernelTiming * 256)()
        n = ctypes.c_int(0)
        self._check(self._L.ve_profile_read(self._h, buf, 256, ctypes.byref(n)), "ve_profile_read")
        return [(buf[i].name.decode(), buf[i].launches, buf[i].avg_ms, buf[i].bytes_per_launch)
                for i in range(min(n.value, 256))]

    def close(self):
        if getattr(self, "_h", None):
            try:
                self.flush()
            finally:
                self._L.ve_destroy(self._h)
                self._h = None
                self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- array constructors
    def asarray(self, t) -> "Array":
        """Wrap a float64 / float32 CUDA tensor (its storage becomes a
        caller-owned array-base; no copy)."""
        torch = _torch()
        if not t.is_cuda or t.dtype not in (torch.float64, torch.float32):
            raise TypeError("a float64 or float32 CUDA tensor is required")
        dt = _abi.VE_F64 if t.dtype == torch.float64 else _abi.VE_F32
        st = t.untyped_storage()
        nelem = st.nbytes() // _ITEM[dt]
        b = self._new_base(dt, nelem, st.data_ptr())
        self._keep.append(st)
        return Array(b, t.storage_offset(), tuple(t.shape), tuple(t.stride()))

    def empty(self, shape, dtype="float64") -> "Array":
        shape = (shape,) if isinstance(shape, int) else tuple(shape)
        b = self._new_base(_DT[dtype], math.prod(shape))
        return Array(b, 0, shape, _contig(shape))

    def full(self, shape, value, dtype="float64") -> "Array":
        a = self.empty(shape, dtype)
        a[...] = float(value)
        return a

    def zeros(self, shape, dtype="float64") -> "Array":
        return self.full(shape, 0.0, dtype)


def _contig(shape):
    st, s = [], 1
    for n in reversed(shape):
        st.append(s)
        s *= n
    return tuple(reversed(st))


class _Base:
    """An array-base; records a free when Python drops it."""

    def __init__(self, eng: Engine, bid: int, dtype: int, nelem: int):
        self.eng_ref = weakref.ref(eng)
        self.id = bid
        self.dtype = dtype
        self.nelem = nelem

    def __del__(self):
        eng = self.eng_ref()
        if eng is not None and getattr(eng, "_h", None):
            # appended without the flush check: a free may be recorded while
            # a batch is being handed over, and must follow it
            eng._pending.append(("free", (self.id, 0, (1,), (1,)), ()))


def _bshape(a, b):
    """numpy broadcasting of two shapes."""
    n = max(len(a), len(b))
    a = (1,) * (n - len(a)) + tuple(a)
    b = (1,) * (n - len(b)) + tuple(b)
    out = []
    for x, y in zip(a, b):
        if x != y and x != 1 and y != 1:
            raise ValueError("shapes %s and %s do not broadcast" % (a, b))
        out.append(max(x, y))
    return tuple(out)


class Array:
    """A view of an array-base (numpy semantics for indexing and arithmetic;
    element operations are recorded, not run)."""

    __array_priority__ = 1000

    def __init__(self, base: _Base, offset: int, shape, strides):
        self._base = base
        self.offset = offset
        self.shape = tuple(shape)
        self.strides = tuple(strides)

    # ---- properties
    @property
    def eng(self) -> Engine:
        e = self._base.eng_ref()
        if e is None:
            raise VEError("the engine of this array is gone")
        return e

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def size(self):
        return math.prod(self.shape)

    @property
    def dtype(self):
        return "float64" if self._base.dtype == _abi.VE_F64 else "float32"

    def view_tuple(self):
        if not self.shape:
            return (self._base.id, self.offset, (1,), (1,))
        return (self._base.id, self.offset, self.shape, self.strides)

    # ---- indexing
    def __getitem__(self, key) -> "Array":
        if not isinstance(key, tuple):
            key = (key,)
        if len(key) == len(self.shape) and all(type(k) is slice for k in key):
            # the common case: one slice per axis
            off, shape, strides = self.offset, [], []
            for k, n, s in zip(key, self.shape, self.strides):
                start, stop, step = k.indices(n)
                m = len(range(start, stop, step))
                if m > 0:
                    off += start * s
                shape.append(m)
                strides.append(step * s)
            return Array(self._base, off, shape, strides)
        if any(k is Ellipsis for k in key):
            i = [k is Ellipsis for k in key].index(True)
            fill = self.ndim - (len(key) - 1)
            key = key[:i] + (slice(None),) * fill + key[i + 1:]
        key = key + (slice(None),) * (self.ndim - len(key))
        if len(key) > self.ndim:
            raise IndexError("too many indices")
        off, shape, strides = self.offset, [], []
        for k, n, s in zip(key, self.shape, self.strides):
            if isinstance(k, (int, np.integer)):
                k = int(k)
                if k < 0:
                    k += n
                if not 0 <= k < n:
                    raise IndexError("index out of range")
                off += k * s
            elif isinstance(k, slice):
                start, stop, step = k.indices(n)
                m = len(range(start, stop, step))
                off += start * s if m > 0 else 0
                shape.append(m)
                strides.append(step * s)
            else:
                raise TypeError("basic indexing only (ints, slices, ...)")
        return Array(self._base, off, shape, strides)

    def __setitem__(self, key, value):
        dst = self[key]
        dst._assign(value)

    def _assign(self, value):
        if isinstance(value, Array):
            value = value._broadcast_to(self.shape)
            self.eng.record("copy", self.view_tuple(), (value.view_tuple(),))
        else:
            self.eng.record("copy", self.view_tuple(), (float(value),))

    def _broadcast_to(self, shape) -> "Array":
        if self.shape == tuple(shape):
            return self
        shape = tuple(shape)
        if _bshape(self.shape, shape) != shape:
            raise ValueError("cannot broadcast %s to %s" % (self.shape, shape))
        pad = len(shape) - self.ndim
        strides = [0] * pad + [0 if n == 1 and m != 1 else s for n, m, s in
                               zip(self.shape, shape[pad:], self.strides)]
        return Array(self._base, self.offset, shape, strides)

    # ---- element-wise operations
    def _binary(self, op, other, reverse=False, out=None) -> "Array":
        eng = self.eng
        if isinstance(other, Array):
            shape = self.shape if self.shape == other.shape else _bshape(self.shape, other.shape)
            a, b = self._broadcast_to(shape), other._broadcast_to(shape)
            if a.dtype != b.dtype:
                a, b = _promote(a), _promote(b)
            ins = [a.view_tuple(), b.view_tuple()]
            dt = a.dtype
        else:
            shape = self.shape
            ins = [self.view_tuple(), float(other)]
            dt = self.dtype
        if reverse:
            ins = ins[::-1]
        if out is None:
            out = eng.empty(shape, dt)
        eng.record(op, out.view_tuple(), ins)
        return out

    def _unary(self, op) -> "Array":
        out = self.eng.empty(self.shape, self.dtype)
        self.eng.record(op, out.view_tuple(), (self.view_tuple(),))
        return out

    def __add__(self, o): return self._binary("add", o)
    def __radd__(self, o): return self._binary("add", o, reverse=True)
    def __sub__(self, o): return self._binary("subtract", o)
    def __rsub__(self, o): return self._binary("subtract", o, reverse=True)
    def __mul__(self, o): return self._binary("multiply", o)
    def __rmul__(self, o): return self._binary("multiply", o, reverse=True)
    def __truediv__(self, o): return self._binary("divide", o)
    def __rtruediv__(self, o): return self._binary("divide", o, reverse=True)
    def __pow__(self, o): return self._binary("power", o)
    def __rpow__(self, o): return self._binary("power", o, reverse=True)
    def __gt__(self, o): return self._binary("greater", o)
    def __ge__(self, o): return self._binary("greater_equal", o)
    def __lt__(self, o): return self._binary("less", o)
    def __le__(self, o): return self._binary("less_equal", o)
    def __neg__(self): return self._unary("negative")
    def __abs__(self): return self._unary("absolute")

    def _inplace(self, op, o):
        self._binary(op, o._broadcast_to(self.shape) if isinstance(o, Array) else o, out=self)
        return self

    def __iadd__(self, o): return self._inplace("add", o)
    def __isub__(self, o): return self._inplace("subtract", o)
    def __imul__(self, o): return self._inplace("multiply", o)
    def __itruediv__(self, o): return self._inplace("divide", o)

    def copy(self) -> "Array":
        out = self.eng.empty(self.shape, self.dtype)
        out._assign(self)
        return out

    def sum(self) -> "Array":
        out = self.eng.empty((1,), self.dtype)
        self.eng.record("add_reduce", out.view_tuple(), (self.view_tuple(),))
        return out

    def max(self) -> "Array":
        out = self.eng.empty((1,), self.dtype)
        self.eng.record("maximum_reduce", out.view_tuple(), (self.view_tuple(),))
        return out

    # ---- reading
    def torch(self):
        """A new torch tensor with this view's values (flushes the batch and
        copies through the engine; stream-ordered)."""
        torch = _torch()
        eng = self.eng
        t = torch.empty(self.shape, dtype=torch.float64 if self.dtype == "float64" else torch.float32,
                        device="cuda")
        if self.size:
            dst = eng.asarray(t)
            dst._assign(self)
            eng.flush()
        return t

    def numpy(self) -> np.ndarray:
        return self.torch().cpu().numpy()

    def __float__(self):
        if self.size != 1:
            raise TypeError("only one-element arrays convert to float")
        return float(self.numpy().reshape(-1)[0])


def _promote(a: Array) -> Array:
    if a.dtype == "float64":
        return a
    out = a.eng.empty(a.shape, "float64")
    out._assign(a)
    return out


def _ufunc(op):
    def f(x):
        return x._unary(op)
    f.__name__ = op
    return f


sqrt, exp, log, sin, cos, tanh = (_ufunc(n) for n in ("sqrt", "exp", "log", "sin", "cos", "tanh"))


def maximum(a: Array, b) -> Array:
    return a._binary("maximum", b)


def minimum(a: Array, b) -> Array:
    return a._binary("minimum", b)


def where(c: Array, a: Array, b: Array) -> Array:
    shape = _bshape(_bshape(c.shape, a.shape), b.shape)
    out = c.eng.empty(shape, a.dtype)
    c.eng.record("where", out.view_tuple(), (c._broadcast_to(shape).view_tuple(), a._broadcast_to(shape).view_tuple(),
                                             b._broadcast_to(shape).view_tuple()))
    return out
