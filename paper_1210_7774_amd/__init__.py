"""MI355X-native geometric multigrid for Poisson / diffusion problems.

Thin Python binding of libmgx.so (include/mg.h): torch tensors supply device
memory and the stream; every level operation runs in the library's HIP
kernels.  There is no CPU path -- constructing a solver without the built
library, or on a machine without a GPU, raises.

    s = Solver(n=4095, dim=2)                     # Poisson, V(2,2) RB-GS, FP64
    u = torch.zeros(n, n, dtype=torch.float64, device="cuda")
    status, stats = s.solve(u, f, rtol=1e-10)
"""
from __future__ import annotations

import ctypes

from . import _abi
from ._abi import MGError

__all__ = ["Solver", "BatchSolver", "MGError", "Stats", "NWEIGHTS", "jacobi5"]

NWEIGHTS = _abi.NWEIGHTS

Stats = _abi.Stats

_SMOOTHERS = {"rbgs": _abi.MG_SM_RBGS, "jacobi": _abi.MG_SM_JACOBI, "learned": _abi.MG_SM_LEARNED}
_PRECISIONS = {"f64": _abi.MG_P_F64, "f32": _abi.MG_P_F32_IR, "bf16": _abi.MG_P_F32_BF16_IR}
_CYCLES = {"V": _abi.MG_CYCLE_V, "W": _abi.MG_CYCLE_W, "F": _abi.MG_CYCLE_F}


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_f64(t, shape, name):
    torch = _torch()
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("%s must be a float64 CUDA tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


def make_options(nu1=2, nu2=2, smoother="rbgs", precision="f64", ncoarse=0, max_cycles=100, use_graph=False,
                 omega=0.0, stream=None, learned=None, cycle="V", fmg=False, zero_start=False) -> _abi.Options:
    o = _abi.Options()
    _abi.lib().mg_options_default(ctypes.byref(o))
    o.nu1, o.nu2 = nu1, nu2
    o.smoother = _SMOOTHERS[smoother]
    o.precision = _PRECISIONS[precision]
    o.ncoarse = ncoarse
    o.max_cycles = max_cycles
    o.inner_cycles = 1
    o.use_graph = int(bool(use_graph))
    o.omega = omega
    o.learned = ctypes.c_void_p(learned.data_ptr()) if learned is not None else None
    o.stream = _stream_handle(stream)
    o.cycle = _CYCLES[cycle]
    o.fmg = int(bool(fmg))
    o.zero_start = int(bool(zero_start))
    return o


def make_grid(n, dim, pitch=None) -> _abi.Grid:
    g = _abi.Grid()
    g.dim = dim
    for ax in range(3):
        g.n[ax] = n if ax < dim else 1
        g.pitch[ax] = 0
    if pitch is not None:
        for ax, p in enumerate(pitch):
            g.pitch[ax] = p
    return g


class Solver:
    """One system on one GPU: -div(a grad u) = f (a None: Poisson) on n^dim
    interior nodes, homogeneous Dirichlet boundary.

    u and f are float64 CUDA tensors of shape (n,)*dim (contiguous, x the
    last index); a is a float64 CUDA tensor of shape (n+2, n+2) (dim 2).
    smoother="learned" takes `learned`, the network's FP32 weights (a CUDA
    tensor of NWEIGHTS numbers, read at setup), with precision "f32"/"bf16".
    cycle is "V", "W" or "F"; fmg=True starts solve() with one
    full-multigrid pass (precision "f64"); zero_start=True makes solve()
    start from u = 0 without reading the u passed in."""

    def __init__(self, n: int, dim: int = 2, a=None, nu1=2, nu2=2, smoother="rbgs", precision="f64",
                 ncoarse=0, max_cycles=100, use_graph=False, omega=0.0, stream=None, learned=None, cycle="V",
                 fmg=False, zero_start=False):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a ROCm GPU; there is no CPU path")
        L = _abi.lib()
        self.n, self.dim = n, dim
        self.shape = (n,) * dim
        self._a = a
        self._tune_tag = "%s|%s|nu%d,%d" % (precision, smoother, nu1, nu2)
        if cycle not in _CYCLES:
            raise ValueError("cycle must be one of %s" % sorted(_CYCLES))
        if a is not None:
            _check_f64(a, (n + 2,) * dim, "a")
        self.grid = make_grid(n, dim)
        self.op = _abi.Operator(_abi.MG_OP_DIFFUSION if a is not None else _abi.MG_OP_POISSON,
                                ctypes.c_void_p(a.data_ptr()) if a is not None else None)
        if learned is not None:
            if learned.dtype != torch.float32 or not learned.is_cuda or learned.numel() != _abi.NWEIGHTS:
                raise TypeError("learned must be a float32 CUDA tensor of %d weights" % _abi.NWEIGHTS)
            learned = learned.contiguous()
        self._learned = learned
        self.opts = make_options(nu1, nu2, smoother, precision, ncoarse, max_cycles, use_graph, omega, stream,
                                 learned, cycle, fmg, zero_start)
        nbytes = ctypes.c_size_t(0)
        rc = L.mg_workspace_size(ctypes.byref(self.grid), ctypes.byref(self.op), ctypes.byref(self.opts),
                                 ctypes.byref(nbytes))
        if rc != _abi.MG_OK:
            raise MGError(rc, "mg_workspace_size")
        self.workspace = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device="cuda")
        self.handle = ctypes.c_void_p(0)
        rc = L.mg_setup(ctypes.byref(self.grid), ctypes.byref(self.op), ctypes.byref(self.opts),
                        _ptr(self.workspace), nbytes.value, ctypes.byref(self.handle))
        if rc != _abi.MG_OK:
            raise MGError(rc, "mg_setup", L.mg_last_error(None).decode())

    def _err(self, rc, where):
        detail = _abi.lib().mg_last_error(self.handle).decode() if self.handle else ""
        return MGError(rc, where, detail)

    def solve(self, u, f, rtol=1e-10, raise_on_error=True):
        """Solve in place on u (initial guess on entry).  Returns (status, Stats)."""
        _check_f64(u, self.shape, "u")
        _check_f64(f, self.shape, "f")
        st = _abi.Stats()
        rc = _abi.lib().mg_solve(self.handle, _ptr(u), _ptr(f), float(rtol), ctypes.byref(st))
        if rc < 0 and raise_on_error:
            raise self._err(rc, "mg_solve")
        return rc, st

    def vcycle(self, u, f):
        _check_f64(u, self.shape, "u")
        _check_f64(f, self.shape, "f")
        rc = _abi.lib().mg_vcycle(self.handle, _ptr(u), _ptr(f))
        if rc != _abi.MG_OK:
            raise self._err(rc, "mg_vcycle")

    def residual_norm(self, u, f) -> float:
        _check_f64(u, self.shape, "u")
        _check_f64(f, self.shape, "f")
        out = ctypes.c_double(0.0)
        rc = _abi.lib().mg_residual_norm(self.handle, _ptr(u), _ptr(f), ctypes.byref(out))
        if rc != _abi.MG_OK:
            raise self._err(rc, "mg_residual_norm")
        return out.value

    def scaled_residual(self, u, f, s=None):
        """s = D^-1 (f - A u) in FP64 (2D); returns s."""
        _check_f64(u, self.shape, "u")
        _check_f64(f, self.shape, "f")
        if s is None:
            s = _torch().empty_like(u)
        _check_f64(s, self.shape, "s")
        rc = _abi.lib().mg_scaled_residual(self.handle, _ptr(u), _ptr(f), _ptr(s))
        if rc != _abi.MG_OK:
            raise self._err(rc, "mg_scaled_residual")
        return s

    def residual(self, u, f, r):
        rc = _abi.lib().mg_residual(self.handle, _ptr(u), _ptr(f), _ptr(r))
        if rc != _abi.MG_OK:
            raise self._err(rc, "mg_residual")

    def smooth_restrict(self, u, f, u_out, fc):
        rc = _abi.lib().mg_smooth_restrict(self.handle, _ptr(u), _ptr(f), _ptr(u_out), _ptr(fc))
        if rc != _abi.MG_OK:
            raise self._err(rc, "mg_smooth_restrict")

    def correct_smooth(self, u, uc, f, u_out):
        rc = _abi.lib().mg_correct_smooth(self.handle, _ptr(u), _ptr(uc), _ptr(f), _ptr(u_out))
        if rc != _abi.MG_OK:
            raise self._err(rc, "mg_correct_smooth")

    def autotune(self, u, f, reps=10, cache=None):
        """Time the fused 2D level kernels' launch shapes on (u, f) and keep
        the fastest; u is smoothed in place.  Returns {n: (block height,
        tiled)}, which tune_set() accepts.  cache: a JSON file path; a stored
        entry for this device, precision, operator and size is applied
        without timing, a miss is tuned and stored."""
        _check_f64(u, self.shape, "u")
        _check_f64(f, self.shape, "f")
        op = ("diffusion" if self._a is not None else "poisson") + "%dd" % len(self.shape)
        return _autotune(self, [u], [f], reps, cache, [self.shape[0]], op)

    def tune_get(self):
        return _tune_get(self)

    def tune_set(self, choices):
        _tune_set(self, choices)

    def profile(self, on: bool, finest_only: bool = False):
        """Per-kernel HIP-event timing on (all launches, or only the finest
        level's) or off."""
        rc = _abi.lib().mg_profile(self.handle, (2 if finest_only else 1) if on else 0)
        if rc != _abi.MG_OK:
            raise self._err(rc, "mg_profile")

    def kernel_timings(self):
        """Per kernel class: dict name -> (launches, avg_ms, bytes_per_launch)."""
        return _read_timings(self)

    def close(self):
        if self.handle:
            _abi.lib().mg_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _read_timings(obj):
    buf = (_abi.KernelTiming * 256)()
    cnt = ctypes.c_int(0)
    rc = _abi.lib().mg_profile_read(obj.handle, buf, 256, ctypes.byref(cnt))
    if rc != _abi.MG_OK:
        raise MGError(rc, "mg_profile_read")
    out = {}
    for i in range(cnt.value):
        k = buf[i]
        out[k.name.decode()] = (k.launches, k.avg_ms, k.bytes_per_launch)
    return out


def jacobi5(inp, iters=4, out=None, work=None, stream=None):
    """The paper's fixed-iteration Jacobi benchmark: `iters` iterations of
    0.2 * (centre + up + down + left + right) on the interior of the 2D
    float64 CUDA tensor `inp` (its outer ring is a fixed boundary).  Returns
    out (allocated if None); `inp` is unchanged.  work: scratch of the same
    shape for iters > 4 (allocated if None)."""
    torch = _torch()
    if inp.dim() != 2:
        raise ValueError("a 2D tensor is required")
    _check_f64(inp, inp.shape, "inp")
    if not inp.is_contiguous():
        raise ValueError("inp must be contiguous")
    if out is None:
        out = torch.empty_like(inp)
    _check_f64(out, inp.shape, "out")
    if iters > 4 and work is None:
        work = torch.empty_like(inp)
    if work is not None:
        _check_f64(work, inp.shape, "work")
    rows, cols = inp.shape
    rc = _abi.lib().mg_jacobi5(_ptr(inp), _ptr(out), _ptr(work), int(rows), int(cols), int(iters),
                               _stream_handle(stream))
    if rc != _abi.MG_OK:
        raise MGError(rc, "mg_jacobi5", _abi.lib().mg_last_error(None).decode())
    return out


def _autotune(obj, us, fs, reps, cache, sizes, operator):
    if cache:
        from . import tunecache
        torch = _torch()
        key = tunecache.key(torch.cuda.get_device_name(), obj._tune_tag, operator, sizes)
        hit = tunecache.load(cache, key)
        if hit is not None:
            try:
                _tune_set(obj, hit)
                return _tune_get(obj)
            except MGError:
                pass  # an entry this handle cannot apply is a miss: tune again and rewrite it
        choice = _autotune(obj, us, fs, reps, None, sizes, operator)
        tunecache.store(cache, key, choice)
        return choice
    k = len(us)
    up = (ctypes.c_void_p * k)(*[u.data_ptr() for u in us])
    fp = (ctypes.c_void_p * k)(*[f.data_ptr() for f in fs])
    rc = _abi.lib().mg_autotune(obj.handle, up, fp, int(reps))
    if rc != _abi.MG_OK:
        raise MGError(rc, "mg_autotune", _abi.lib().mg_last_error(obj.handle).decode())
    return _tune_get(obj)


def _tune_get(obj):
    L = _abi.lib()
    cnt = ctypes.c_int(0)
    rc = L.mg_tune_get(obj.handle, None, None, None, 0, ctypes.byref(cnt))
    if rc != _abi.MG_OK:
        raise MGError(rc, "mg_tune_get")
    m = cnt.value
    n, hb, tl = (ctypes.c_int * max(m, 1))(), (ctypes.c_int * max(m, 1))(), (ctypes.c_int * max(m, 1))()
    rc = L.mg_tune_get(obj.handle, n, hb, tl, m, ctypes.byref(cnt))
    if rc != _abi.MG_OK:
        raise MGError(rc, "mg_tune_get")
    return {int(n[i]): (int(hb[i]), bool(tl[i])) for i in range(m)}


def _tune_set(obj, choices):
    for n, (hb, tiled) in dict(choices).items():
        rc = _abi.lib().mg_tune_set(obj.handle, int(n), int(hb), 1 if tiled else 0)
        if rc != _abi.MG_OK:
            raise MGError(rc, "mg_tune_set")


class BatchSolver:
    """Many independent 2D systems of uneven sizes solved together: equal-size
    levels share one launch per phase, converged systems drop out."""

    def __init__(self, ns, coefs=None, nu1=2, nu2=2, precision="f32", max_cycles=100, use_graph=False,
                 stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("BatchSolver needs a ROCm GPU; there is no CPU path")
        L = _abi.lib()
        self.ns = [int(n) for n in ns]
        k = len(self.ns)
        self._tune_tag = "%s|rbgs|nu%d,%d" % (precision, nu1, nu2)
        self.grids = (_abi.Grid * k)()
        self.ops = (_abi.Operator * k)()
        self._coefs = coefs
        for s, n in enumerate(self.ns):
            self.grids[s] = make_grid(n, 2)
            if coefs is not None:
                _check_f64(coefs[s], (n + 2, n + 2), "a[%d]" % s)
                self.ops[s] = _abi.Operator(_abi.MG_OP_DIFFUSION, ctypes.c_void_p(coefs[s].data_ptr()))
            else:
                self.ops[s] = _abi.Operator(_abi.MG_OP_POISSON, None)
        self.opts = make_options(nu1, nu2, "rbgs", precision, 0, max_cycles, use_graph, 0.0, stream)
        nbytes = ctypes.c_size_t(0)
        rc = L.mg_workspace_size_batch(k, self.grids, self.ops, ctypes.byref(self.opts), ctypes.byref(nbytes))
        if rc != _abi.MG_OK:
            raise MGError(rc, "mg_workspace_size_batch")
        self.workspace = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device="cuda")
        self.handle = ctypes.c_void_p(0)
        rc = L.mg_setup_batch(k, self.grids, self.ops, ctypes.byref(self.opts), _ptr(self.workspace), nbytes.value,
                              ctypes.byref(self.handle))
        if rc != _abi.MG_OK:
            raise MGError(rc, "mg_setup_batch", L.mg_last_error(None).decode())

    def solve(self, us, fs, rtol=1e-10, raise_on_error=True):
        k = len(self.ns)
        up = (ctypes.c_void_p * k)(*[u.data_ptr() for u in us])
        fp = (ctypes.c_void_p * k)(*[f.data_ptr() for f in fs])
        st = (_abi.Stats * k)()
        rc = _abi.lib().mg_solve_batch(self.handle, up, fp, float(rtol), st)
        if rc < 0 and raise_on_error:
            detail = _abi.lib().mg_last_error(self.handle).decode()
            raise MGError(rc, "mg_solve_batch", detail)
        return rc, list(st)

    def autotune(self, us, fs, reps=10, cache=None):
        """As Solver.autotune, over all systems at once (shared launches)."""
        for s, n in enumerate(self.ns):
            _check_f64(us[s], (n, n), "u[%d]" % s)
            _check_f64(fs[s], (n, n), "f[%d]" % s)
        op = ("diffusion" if self._coefs is not None else "poisson") + "2d-batch"
        return _autotune(self, us, fs, reps, cache, self.ns, op)

    def tune_get(self):
        return _tune_get(self)

    def tune_set(self, choices):
        _tune_set(self, choices)

    def profile(self, on: bool, finest_only: bool = False):
        rc = _abi.lib().mg_profile(self.handle, (2 if finest_only else 1) if on else 0)
        if rc != _abi.MG_OK:
            raise MGError(rc, "mg_profile")

    def kernel_timings(self):
        return _read_timings(self)

    def close(self):
        if self.handle:
            _abi.lib().mg_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
