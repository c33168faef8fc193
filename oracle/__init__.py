"""The oracle: a plain, slow CPU multigrid that the HIP path is checked against.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the product
library: the level operations live in ``mg_oracle.c`` / ``mg_core.inc`` (plain
C, IEEE FP64 with an FP32 build of the same source, ``-ffp-contract=off``), the
learned-smoother reference lives in ``learned.py`` (numpy FP64), the paper's
fixed-iteration Jacobi benchmark in ``jacobi5.py`` (numpy FP64 array views).

Arrays are numpy, interior-only, x fastest: shape ``(n,)``, ``(n, n)`` or
``(n, n, n)`` indexed ``[k][j][i]``.  A nodal coefficient covers the ``(n+2)^d``
nodes including the boundary.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "mg_oracle.c"), os.path.join(_HERE, "mg_core.inc")]

RBGS, JACOBI, LEX = 0, 1, 2
F64, F32, BF16 = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, no contraction of a*b+c)."""
    newest = max(os.path.getmtime(s) for s in _SRC)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC[0], "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Opts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("smoother", ctypes.c_int),
                ("ncoarse", ctypes.c_int), ("bf16", ctypes.c_int), ("omega", ctypes.c_double)]


@dataclass
class Opts:
    nu1: int = 2
    nu2: int = 2
    smoother: int = RBGS
    ncoarse: int = 3
    omega: float | None = None   # None: 2d/(2d+1), the smoothing-optimal Jacobi weight
    bf16: bool = False

    def c(self, d: int) -> _Opts:
        om = self.omega if self.omega is not None else 2.0 * d / (2.0 * d + 1.0)
        return _Opts(self.nu1, self.nu2, self.smoother, self.ncoarse, int(self.bf16), om)


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        for sfx, P, R in (("f64", _D, ctypes.c_double), ("f32", _F, ctypes.c_float)):
            g = lambda nm: getattr(_lib, "%s_%s" % (nm, sfx))  # noqa: E731
            g("orc_apply").argtypes = [ctypes.c_int, ctypes.c_int, R, P, P, P]
            g("orc_residual").argtypes = [ctypes.c_int, ctypes.c_int, R, P, P, P, P]
            g("orc_sweep").argtypes = [ctypes.c_int, ctypes.c_int, R, P, P, P, ctypes.c_int, R, ctypes.c_int]
            g("orc_restrict").argtypes = [ctypes.c_int, ctypes.c_int, P, P]
            g("orc_prolong_add").argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int]
            g("orc_coarsen_coef").argtypes = [ctypes.c_int, ctypes.c_int, P, P]
            g("orc_dot").argtypes = [ctypes.c_long, P, P]
            g("orc_dot").restype = R
            g("orc_assemble").argtypes = [ctypes.c_int, ctypes.c_int, R, P, _D]
            g("orc_vcycle").argtypes = [ctypes.c_int, ctypes.c_int, R, P, P, P, ctypes.POINTER(_Opts)]
            g("orc_cycle").argtypes = [ctypes.c_int, ctypes.c_int, R, P, P, P, ctypes.POINTER(_Opts), ctypes.c_int]
            g("orc_fmg").argtypes = [ctypes.c_int, ctypes.c_int, R, P, P, P, ctypes.POINTER(_Opts), ctypes.c_int,
                                     ctypes.c_int]
        _lib.orc_lu_solve.argtypes = [ctypes.c_int, _D, _D, _D]
        _lib.orc_lu_solve.restype = ctypes.c_int
        _lib.orc_bf16_round.argtypes = [ctypes.c_float]
        _lib.orc_bf16_round.restype = ctypes.c_float
        _lib.orc_solve.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, ctypes.POINTER(_Opts),
                                   ctypes.c_double, ctypes.c_int, _D, ctypes.POINTER(ctypes.c_int)]
        _lib.orc_solve.restype = ctypes.c_int
        _lib.orc_solve_cycles.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, ctypes.POINTER(_Opts), ctypes.c_int,
                                          ctypes.c_int, ctypes.c_double, ctypes.c_int, _D,
                                          ctypes.POINTER(ctypes.c_int)]
        _lib.orc_solve_cycles.restype = ctypes.c_int
        _lib.orc_solve_ir.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, ctypes.POINTER(_Opts),
                                      ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, _D,
                                      ctypes.POINTER(ctypes.c_int)]
        _lib.orc_solve_ir.restype = ctypes.c_int
        _lib.orc_solve_ir_cycles.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, ctypes.POINTER(_Opts),
                                             ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                             _D, ctypes.POINTER(ctypes.c_int)]
        _lib.orc_solve_ir_cycles.restype = ctypes.c_int
    return _lib


def _dt(x):
    return np.float32 if x.dtype == np.float32 else np.float64


def _p(x, dt):
    if x is None:
        return None
    assert x.dtype == dt and x.flags.c_contiguous, (x.dtype, dt)
    return x.ctypes.data_as(_F if dt == np.float32 else _D)


def _sfx(dt):
    return "f32" if dt == np.float32 else "f64"


def _dn(u):
    return u.ndim, u.shape[0]


def h_of(n: int) -> float:
    return 1.0 / (n + 1)


def apply(u, a=None, h=None):
    """A u (A includes the 1/h^2)."""
    d, n = _dn(u)
    dt = _dt(u)
    out = np.empty_like(u)
    getattr(lib(), "orc_apply_" + _sfx(dt))(d, n, h_of(n) if h is None else h, _p(a, dt), _p(u, dt), _p(out, dt))
    return out


def residual(u, f, a=None, h=None):
    d, n = _dn(u)
    dt = _dt(u)
    r = np.empty_like(u)
    getattr(lib(), "orc_residual_" + _sfx(dt))(d, n, h_of(n) if h is None else h, _p(a, dt), _p(u, dt),
                                              _p(f, dt), _p(r, dt))
    return r


def sweep(u, f, a=None, kind=RBGS, omega=None, bf16=False, h=None, nsweeps=1):
    """In-place smoothing sweep(s) on u; returns u."""
    d, n = _dn(u)
    dt = _dt(u)
    om = omega if omega is not None else 2.0 * d / (2.0 * d + 1.0)
    fn = getattr(lib(), "orc_sweep_" + _sfx(dt))
    for _ in range(nsweeps):
        fn(d, n, h_of(n) if h is None else h, _p(a, dt), _p(u, dt), _p(f, dt), kind, om, int(bf16))
    return u


def restrict(r):
    d, n = _dn(r)
    dt = _dt(r)
    nc = (n - 1) // 2
    rc = np.empty((nc,) * d, dtype=dt)
    getattr(lib(), "orc_restrict_" + _sfx(dt))(d, n, _p(r, dt), _p(rc, dt))
    return rc


def prolong_add(ec, u, bf16=False):
    """u += P ec (in place); returns u."""
    d, nc = _dn(ec)
    dt = _dt(u)
    assert u.shape[0] == 2 * nc + 1
    getattr(lib(), "orc_prolong_add_" + _sfx(dt))(d, nc, _p(ec, dt), _p(u, dt), int(bf16))
    return u


def coarsen_coef(a, d):
    n = a.shape[0] - 2
    nc = (n - 1) // 2
    dt = _dt(a)
    ac = np.empty((nc + 2,) * d, dtype=dt)
    getattr(lib(), "orc_coarsen_coef_" + _sfx(dt))(d, n, _p(a, dt), _p(ac, dt))
    return ac


def assemble(d, n, a=None, h=None, dtype=np.float64):
    m = n ** d
    M = np.empty((m, m), dtype=np.float64)
    getattr(lib(), "orc_assemble_" + _sfx(dtype))(d, n, h_of(n) if h is None else h, _p(a, dtype),
                                                 M.ctypes.data_as(_D))
    return M


def lu_solve(M, b):
    M = np.ascontiguousarray(M, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty_like(b)
    rc = lib().orc_lu_solve(M.shape[0], M.ctypes.data_as(_D), b.ctypes.data_as(_D), x.ctypes.data_as(_D))
    if rc != 0:
        raise np.linalg.LinAlgError("singular")
    return x


def vcycle(u, f, a=None, opts: Opts | None = None, h=None):
    """One V-cycle in place on u (FP64 or float by the dtype of u)."""
    d, n = _dn(u)
    dt = _dt(u)
    o = (opts or Opts()).c(d)
    getattr(lib(), "orc_vcycle_" + _sfx(dt))(d, n, h_of(n) if h is None else h, _p(a, dt), _p(u, dt),
                                            _p(f, dt), ctypes.byref(o))
    return u


CYCLES = {"V": 0, "W": 1, "F": 2}


def cycle(u, f, a=None, opts: Opts | None = None, h=None, kind="V"):
    """One V-, W- or F-cycle in place on u (FP64 or float by the dtype of u)."""
    d, n = _dn(u)
    dt = _dt(u)
    o = (opts or Opts()).c(d)
    getattr(lib(), "orc_cycle_" + _sfx(dt))(d, n, h_of(n) if h is None else h, _p(a, dt), _p(u, dt), _p(f, dt),
                                           ctypes.byref(o), CYCLES[kind])
    return u


def fmg(f, a=None, opts: Opts | None = None, h=None, kind="V", ncyc=1):
    """Full multigrid from scratch: returns u (FP64 or float by the dtype of f)."""
    d, n = _dn(f)
    dt = _dt(f)
    u = np.zeros_like(f)
    o = (opts or Opts()).c(d)
    getattr(lib(), "orc_fmg_" + _sfx(dt))(d, n, h_of(n) if h is None else h, _p(a, dt), _p(u, dt), _p(f, dt),
                                         ctypes.byref(o), CYCLES[kind], ncyc)
    return u


def bf16_round(x):
    x = np.asarray(x, dtype=np.float32)
    return np.vectorize(lambda v: lib().orc_bf16_round(float(v)), otypes=[np.float32])(x)


@dataclass
class SolveResult:
    u: np.ndarray
    status: int
    cycles: int
    hist: np.ndarray

    @property
    def rho_avg(self) -> float:
        k = self.cycles
        return float((self.hist[k] / self.hist[0]) ** (1.0 / k)) if k > 0 else 0.0


def solve(f, a=None, opts: Opts | None = None, tol=1e-10, maxc=100, u0=None, kind="V", fmg=False):
    """Cycles (V, W or F) from u0 (default 0) until rel. residual <= tol
    (FP64); fmg: the first step is a full-multigrid pass from scratch."""
    d, n = _dn(f)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    hist = np.zeros(maxc + 1)
    cyc = ctypes.c_int(0)
    o = (opts or Opts()).c(d)
    rc = lib().orc_solve_cycles(d, n, _p(a, np.float64), _p(u, np.float64), _p(f, np.float64), ctypes.byref(o),
                                CYCLES[kind], int(bool(fmg)), tol, maxc, hist.ctypes.data_as(_D), ctypes.byref(cyc))
    return SolveResult(u, rc, cyc.value, hist[: cyc.value + 1].copy())


def solve_ir(f, a=None, opts: Opts | None = None, prec=F32, inner=1, tol=1e-10, maxc=100, u0=None, kind="V"):
    """Iterative refinement with an FP64 outer loop and inner cycles (V, W or
    F) in prec."""
    d, n = _dn(f)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64, copy=True)
    hist = np.zeros(maxc + 1)
    cyc = ctypes.c_int(0)
    o = (opts or Opts()).c(d)
    rc = lib().orc_solve_ir_cycles(d, n, _p(a, np.float64), _p(u, np.float64), _p(f, np.float64), ctypes.byref(o),
                                   prec, inner, CYCLES[kind], tol, maxc, hist.ctypes.data_as(_D), ctypes.byref(cyc))
    return SolveResult(u, rc, cyc.value, hist[: cyc.value + 1].copy())
