"""ctypes declarations of the C-ABI in include/mg.h (argument marshalling only).

Loading fails loudly when libmgx.so has not been built: there is no CPU
fallback for any entry point.
"""
from __future__ import annotations

import ctypes
import functools
import struct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# MGX_LIBRARY may point at another build of the same library (tuning runs)
LIB_PATH = os.environ.get("MGX_LIBRARY") or os.path.join(HERE, "libmgx.so")

MG_OK = 0
MG_NOT_CONVERGED = 1
MG_FELL_BACK = 2
MG_ERR_ARG = -1
MG_ERR_UNSUPPORTED = -2
MG_ERR_HIP = -3
MG_ERR_NONFINITE = -4
MG_ERR_DIVERGED = -5
MG_ERR_WORKSPACE = -6

MG_OP_POISSON = 0
MG_OP_DIFFUSION = 1
MG_SM_RBGS = 0
MG_SM_JACOBI = 1
MG_SM_LEARNED = 2
MG_P_F64 = 0
MG_P_F32_IR = 1
MG_P_F32_BF16_IR = 2
MG_CYCLE_V = 0
MG_CYCLE_W = 1
MG_CYCLE_F = 2
MG_MAX_CYCLES = 200
MG_MONITOR_CONTINUE = 0
MG_MONITOR_FALLBACK = 1
MG_MONITOR_DIVERGED = 2

# every function declared in include/mg.h
EXPORTS = ("mg_options_default", "mg_workspace_size", "mg_setup", "mg_vcycle", "mg_residual_norm", "mg_solve",
           "mg_smooth_restrict", "mg_correct_smooth", "mg_residual", "mg_destroy", "mg_status_str",
           "mg_last_error", "mg_workspace_size_batch", "mg_setup_batch", "mg_solve_batch", "mg_profile",
           "mg_profile_read", "mg_learned_scratch_bytes", "mg_learned_loss_grad", "mg_learned_apply",
           "mg_learned_train", "mg_learned_crop", "mg_scaled_residual", "mg_autotune", "mg_tune_get",
           "mg_tune_set", "mg_jacobi5", "mg_jacobi5_static", "mg_learned_step", "mg_monitor")
NWEIGHTS = 4896


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("pitch", ctypes.c_longlong * 3)]


class Operator(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("a", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("smoother", ctypes.c_int),
                ("precision", ctypes.c_int), ("ncoarse", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("inner_cycles", ctypes.c_int), ("use_graph", ctypes.c_int), ("omega", ctypes.c_double),
                ("learned", ctypes.c_void_p), ("stream", ctypes.c_void_p), ("cycle", ctypes.c_int),
                ("fmg", ctypes.c_int),
                ("zero_start", ctypes.c_int)]


class KernelTiming(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double),
                ("avg_ms", ctypes.c_double), ("bytes_per_launch", ctypes.c_double)]


class TrainOptions(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("patch", ctypes.c_int), ("border", ctypes.c_int),
                ("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


class TrainStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("loss_first_epoch", ctypes.c_double), ("loss_last_epoch", ctypes.c_double),
                ("ms", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("rel_res", ctypes.c_double), ("rho_avg", ctypes.c_double),
                ("rho_asym", ctypes.c_double), ("fell_back", ctypes.c_int),
                ("hist", ctypes.c_double * (MG_MAX_CYCLES + 1))]

    def history(self):
        return [self.hist[i] for i in range(self.cycles + 1)]


# ---- the vector-bytecode engine (include/ve.h)
VE_EXPORTS = ("ve_create", "ve_destroy", "ve_base_new", "ve_base_ptr", "ve_execute", "ve_plan", "ve_kernel_source",
              "ve_register", "ve_stats_get", "ve_profile", "ve_profile_read", "ve_last_error")
VE_OK, VE_ERR_ARG, VE_ERR_UNSUPPORTED, VE_ERR_HIP, VE_ERR_COMPILE = 0, -1, -2, -3, -4
VE_MAX_NDIM, VE_MAX_IN = 4, 3
VE_F64, VE_F32 = 0, 1
VE_OPCODES = {"sync": 1, "discard": 2, "free": 3, "copy": 10, "negative": 11, "absolute": 12, "sqrt": 13, "exp": 14,
              "log": 15, "sin": 16, "cos": 17, "tanh": 18, "add": 30, "subtract": 31, "multiply": 32, "divide": 33,
              "maximum": 34, "minimum": 35, "power": 36, "greater": 37, "greater_equal": 38, "less": 39,
              "less_equal": 40, "equal": 41, "not_equal": 42, "where": 50, "add_reduce": 60, "maximum_reduce": 61}
VE_USER = 100


class VeView(ctypes.Structure):
    _fields_ = [("base", ctypes.c_int), ("ndim", ctypes.c_int), ("offset", ctypes.c_longlong),
                ("shape", ctypes.c_longlong * VE_MAX_NDIM), ("stride", ctypes.c_longlong * VE_MAX_NDIM)]


class VeInstr(ctypes.Structure):
    _fields_ = [("opcode", ctypes.c_int), ("out", VeView), ("in_", VeView * VE_MAX_IN),
                ("cst", ctypes.c_double * VE_MAX_IN)]


class VeStats(ctypes.Structure):
    _fields_ = [("instructions", ctypes.c_longlong), ("kernels", ctypes.c_longlong), ("compiled", ctypes.c_longlong),
                ("cache_hits", ctypes.c_longlong), ("stores_elided", ctypes.c_longlong),
                ("staged", ctypes.c_longlong), ("compile_ms", ctypes.c_double)]


class VeKernelTiming(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double),
                ("avg_ms", ctypes.c_double), ("bytes_per_launch", ctypes.c_double)]


_VIEW = struct.Struct("=iiq4q4q")           # VeView: 80 bytes
_NOVIEW = _VIEW.pack(-1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0)
_Z4 = (0, 0, 0, 0)


def _view_bytes(v):
    try:
        return _view_bytes_cached(v)
    except TypeError:          # unhashable (lists): pack without the cache
        return _view_bytes_cached.__wrapped__(v)


@functools.lru_cache(maxsize=8192)
def _view_bytes_cached(v):
    base, off, shape, strides = v
    n = len(shape)
    sh = tuple(shape) + _Z4[n:]
    st = tuple(strides) + _Z4[n:]
    return _VIEW.pack(base, n, off, sh[0], sh[1], sh[2], sh[3], st[0], st[1], st[2], st[3])


_HEAD = struct.Struct("=i4x")


def _instr_bytes_uncached(op, out, ins):
    code = VE_OPCODES[op] if isinstance(op, str) else int(op)
    cst = [0.0, 0.0, 0.0]
    views = []
    for k in range(VE_MAX_IN):
        v = ins[k] if k < len(ins) else None
        if isinstance(v, tuple):
            views.append(_view_bytes(v))
        else:
            views.append(_NOVIEW)
            if v is not None:
                cst[k] = float(v)
    return _HEAD.pack(code) + _view_bytes(out) + b"".join(views) + struct.pack("=3d", *cst)


# a program that loops records the same instructions again and again
_instr_bytes_cached = functools.lru_cache(maxsize=16384)(_instr_bytes_uncached)


def _instr_bytes(op, out, ins):
    try:
        return _instr_bytes_cached(op, out, ins)
    except TypeError:          # unhashable (lists): pack without the cache
        return _instr_bytes_uncached(op, out, ins)


def ve_batch(instrs):
    """A VeInstr array from (op, out, ins) tuples: op a name or an opcode,
    views (base, offset, shape, strides), inputs views or float constants
    (packed field by field in the C layout: opcode, padding, out, in[3],
    cst[3])."""
    parts = [_instr_bytes(op, out, ins) for op, out, ins in instrs]
    n = max(len(instrs), 1)
    arr = (VeInstr * n)()
    if parts:
        ctypes.memmove(arr, b"".join(parts), ctypes.sizeof(VeInstr) * len(parts))
    return arr


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmgx.so is not built (run `python -m paper_1210_7774_amd.build`); "
                           "there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    H = ctypes.c_void_p
    st = ctypes.c_int
    L.mg_options_default.argtypes = [P(Options)]
    L.mg_options_default.restype = None
    L.mg_workspace_size.argtypes = [P(Grid), P(Operator), P(Options), P(ctypes.c_size_t)]
    L.mg_setup.argtypes = [P(Grid), P(Operator), P(Options), ctypes.c_void_p, ctypes.c_size_t, P(H)]
    L.mg_vcycle.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p]
    L.mg_residual_norm.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p, P(ctypes.c_double)]
    L.mg_solve.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, P(Stats)]
    L.mg_smooth_restrict.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.mg_correct_smooth.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.mg_residual.argtypes = [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.mg_destroy.argtypes = [H]
    L.mg_status_str.argtypes = [st]
    L.mg_status_str.restype = ctypes.c_char_p
    L.mg_last_error.argtypes = [H]
    L.mg_last_error.restype = ctypes.c_char_p
    L.mg_workspace_size_batch.argtypes = [ctypes.c_int, P(Grid), P(Operator), P(Options), P(ctypes.c_size_t)]
    L.mg_setup_batch.argtypes = [ctypes.c_int, P(Grid), P(Operator), P(Options), ctypes.c_void_p, ctypes.c_size_t,
                                 P(H)]
    L.mg_solve_batch.argtypes = [H, P(ctypes.c_void_p), P(ctypes.c_void_p), ctypes.c_double, P(Stats)]
    V = ctypes.c_void_p
    L.mg_learned_scratch_bytes.argtypes = [ctypes.c_int, ctypes.c_int]
    L.mg_learned_scratch_bytes.restype = ctypes.c_size_t
    L.mg_learned_loss_grad.argtypes = [V, V, V, ctypes.c_int, ctypes.c_int, ctypes.c_int, V, P(ctypes.c_double), V, V,
                                       ctypes.c_size_t, V]
    L.mg_learned_apply.argtypes = [V, ctypes.c_int, ctypes.c_int, ctypes.c_int, V, V, V, ctypes.c_size_t, V]
    L.mg_learned_train.argtypes = [V, V, V, ctypes.c_int, V, P(TrainOptions), V, P(ctypes.c_double), P(TrainStats), V,
                                   ctypes.c_size_t, V]
    L.mg_learned_crop.argtypes = [V, V, V, V, ctypes.c_int, V, V, ctypes.c_int, ctypes.c_int, V, V, V, V]
    L.mg_scaled_residual.argtypes = [H, V, V, V]
    L.mg_autotune.argtypes = [H, P(ctypes.c_void_p), P(ctypes.c_void_p), ctypes.c_int]
    L.mg_tune_get.argtypes = [H, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int), ctypes.c_int, P(ctypes.c_int)]
    L.mg_tune_set.argtypes = [H, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.mg_jacobi5.argtypes = [V, V, V, ctypes.c_int, ctypes.c_int, ctypes.c_int, V]
    L.mg_jacobi5_static.argtypes = [V, V, ctypes.c_int, ctypes.c_int, ctypes.c_int, V]
    L.mg_learned_step.argtypes = [V, V, V, V, ctypes.c_int, ctypes.c_int, V, V, ctypes.c_size_t, V]
    L.mg_monitor.argtypes = [P(ctypes.c_double), ctypes.c_int, ctypes.c_int, ctypes.c_double]
    L.mg_monitor.restype = ctypes.c_int
    L.mg_profile.argtypes = [H, ctypes.c_int]
    L.mg_profile_read.argtypes = [H, P(KernelTiming), ctypes.c_int, P(ctypes.c_int)]
    E = ctypes.c_void_p
    L.ve_create.argtypes = [V, P(E)]
    L.ve_destroy.argtypes = [E]
    L.ve_base_new.argtypes = [E, ctypes.c_int, ctypes.c_longlong, V, P(ctypes.c_int)]
    L.ve_base_ptr.argtypes = [E, ctypes.c_int, P(V)]
    L.ve_execute.argtypes = [E, P(VeInstr), ctypes.c_int]
    L.ve_plan.argtypes = [P(VeInstr), ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int)]
    L.ve_kernel_source.argtypes = [P(VeInstr), ctypes.c_int, P(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                   ctypes.c_char_p, ctypes.c_size_t, P(ctypes.c_size_t)]
    L.ve_register.argtypes = [E, ctypes.c_char_p, ctypes.c_int, P(ctypes.c_int)]
    L.ve_stats_get.argtypes = [E, P(VeStats)]
    L.ve_profile.argtypes = [E, ctypes.c_int]
    L.ve_profile_read.argtypes = [E, P(VeKernelTiming), ctypes.c_int, P(ctypes.c_int)]
    L.ve_last_error.argtypes = [E]
    L.ve_last_error.restype = ctypes.c_char_p
    for nm in VE_EXPORTS[:-1]:
        getattr(L, nm).restype = st
    for nm in ("mg_workspace_size", "mg_setup", "mg_vcycle", "mg_residual_norm", "mg_solve", "mg_smooth_restrict",
               "mg_correct_smooth", "mg_residual", "mg_destroy", "mg_workspace_size_batch", "mg_setup_batch",
               "mg_solve_batch", "mg_profile", "mg_profile_read", "mg_learned_loss_grad", "mg_learned_apply",
               "mg_learned_train", "mg_learned_crop", "mg_scaled_residual", "mg_autotune", "mg_tune_get",
               "mg_tune_set", "mg_jacobi5", "mg_jacobi5_static", "mg_learned_step"):
        getattr(L, nm).restype = st
    _lib = L
    return L


def status_str(s: int) -> str:
    return lib().mg_status_str(s).decode()


class MGError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = "%s: %s (%d)" % (where, status_str(status), status)
        if detail:
            msg += ": " + detail
        super().__init__(msg)
