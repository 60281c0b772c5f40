"""Python binding of the MI355X ECMG_jcg library (include/ecmg.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libecmg.so.  Importing this module fails loudly if the library has not been
built (``python -m paper_1506_02983_amd.build`` or ``__graft_entry__.build()``);
there is no CPU fallback.

Fields are given as numpy functions ``fn(x, y, z, face)`` evaluated with
broadcasting (see ``workloads``), as constants, or as torch functions evaluated
on the device (``device_fields=True``), which samples every field with torch on
the GPU through the library's device-callback interface.
"""
from __future__ import annotations

import atexit
import ctypes
import dataclasses
import os
import sys
import weakref
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libecmg.so")

OK, EINVAL, ENOMEM, ENOTCONV, EBREAKDOWN, EDEVICE, ESTATE, ECALLBACK, ENOENT = 0, -1, -2, -3, -4, -5, -6, -7, -8
DIRICHLET, ROBIN = 0, 1
FP64, MIXED = 0, 1
SERENDIPITY20, LAGRANGE27 = 0, 1
JCG, CG = 0, 1                      # iteration on the JCG levels: ECMG_jcg / ECMG_cg
VEC_U, VEC_W, VEC_UTILDE, VEC_F, VEC_DINV, VEC_NONE = 0, 1, 2, 3, 4, -1
# ecmg_level_info.path: the kernels a level ran on
PATH_DENSE, PATH_PERSISTENT, PATH_TILED, PATH_TILED_UNFOLDED, PATH_COLUMN, PATH_GATHER, PATH_MIXED, PATH_QUEUE = range(8)
K_PASSA, K_PASSB, K_INIT, K_EXPF, K_EXPT, K_PASSA32, K_PASSB32, K_PERSIST, K_MIXSTART, K_MIXUPDATE = range(10)

_STATUS = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", ENOTCONV: "ENOTCONV", EBREAKDOWN: "EBREAKDOWN",
           EDEVICE: "EDEVICE", ESTATE: "ESTATE", ECALLBACK: "ECALLBACK", ENOENT: "ENOENT"}

HOST_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
DEVICE_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_void_p)


class Field(ctypes.Structure):
    _fields_ = [("value", ctypes.c_double), ("host", HOST_FN), ("device", DEVICE_FN), ("user", ctypes.c_void_p)]


class ProblemC(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3), ("n0", ctypes.c_int32 * 3),
                ("levels", ctypes.c_int32), ("face_type", ctypes.c_int32 * 6),
                ("beta", Field), ("f", Field), ("g_D", Field), ("alpha", Field), ("g_R", Field)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("interp", ctypes.c_int32),
                ("keep_w", ctypes.c_int32), ("inner_tol", ctypes.c_double), ("dsolve_tol", ctypes.c_double),
                ("chunk", ctypes.c_int32), ("timing", ctypes.c_int32), ("hip_stream", ctypes.c_void_p),
                ("persistent_nodes", ctypes.c_int64), ("dsolve_dense_max", ctypes.c_int64),
                ("autotune", ctypes.c_int32), ("tune_cache", ctypes.c_char_p), ("method", ctypes.c_int32),
                ("speculate", ctypes.c_int32), ("fold_blocks", ctypes.c_int32), ("true_residual", ctypes.c_int32),
                ("batch_graph", ctypes.c_int32), ("columns", ctypes.c_int32), ("gather_nodes", ctypes.c_int64),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_user", ctypes.c_void_p)]


class TuneResult(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("path", ctypes.c_int32), ("kz", ctypes.c_int32), ("seg", ctypes.c_int32),
                ("nwg", ctypes.c_int32), ("candidates", ctypes.c_int32), ("us_default", ctypes.c_double),
                ("us_best", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["path"] = {1: "persistent", 3: "gather"}.get(self.path, "tiled")
        return d


class LevelInfo(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("outer_steps", ctypes.c_int32), ("status", ctypes.c_int32),
                ("path", ctypes.c_int32), ("rre", ctypes.c_double), ("nf", ctypes.c_double),
                ("ms", ctypes.c_double), ("rre_true", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# Every symbol include/ecmg.h declares (checked by the CPU test suite).
EXPORTS = ["ecmg_default_options", "ecmg_create", "ecmg_setup", "ecmg_solve", "ecmg_solve_extrapolated",
           "ecmg_solve_fixed",
           "ecmg_extrapolate", "ecmg_prolongate", "ecmg_jcg", "ecmg_apply", "ecmg_get", "ecmg_set",
           "ecmg_device_view", "ecmg_norms", "ecmg_level_dims", "ecmg_plan_bytes", "ecmg_kernel_times",
           "ecmg_reset_kernel_times", "ecmg_last_error", "ecmg_destroy", "ecmg_solve_batch",
           "ecmg_extrapolate_batch", "ecmg_server_create", "ecmg_server_submit", "ecmg_server_step",
           "ecmg_server_poll", "ecmg_server_stats", "ecmg_server_completed", "ecmg_server_times", "ecmg_server_reset_stats",
           "ecmg_server_destroy",
           "ecmg_autotune", "ecmg_tune_lookup", "ecmg_set_timing", "ecmg_cascadic_schedule",
           "ecmg_solve_levels", "ecmg_tolerance_schedule", "ecmg_autotune_batch", "ecmg_norms_noalloc"]

_lib = None

# Contexts and servers still open at interpreter exit are closed by an exit
# handler registered after torch's (so it runs first, while the HIP runtime and
# torch's allocator are still up); __del__ makes no library call once the
# interpreter is finalizing.
_live = weakref.WeakSet()
_finalizing = sys.is_finalizing       # kept: module globals may be gone when __del__ runs at exit


def _close_live():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:  # noqa: BLE001
            pass


def load_library(path: str = LIB_PATH):
    """Load libecmg.so; raises ImportError if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libecmg.so not built at %s: run __graft_entry__.build()" % path)
    # torch bundles its own HIP runtime.  Load it first so that libecmg.so binds
    # to the same runtime (its libamdhip64.so.7 dependency is then already
    # resolved): one process, one HIP runtime, shared device memory and streams.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    atexit.register(_close_live)        # after torch's own exit handlers, so it runs before them
    L = ctypes.CDLL(path)
    P, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.ecmg_default_options.argtypes = [ctypes.POINTER(Options)]
    L.ecmg_default_options.restype = None
    L.ecmg_create.argtypes = [ctypes.POINTER(Options), ctypes.POINTER(P)]
    L.ecmg_setup.argtypes = [P, ctypes.POINTER(ProblemC)]
    L.ecmg_solve.argtypes = [P, dbl, P]
    L.ecmg_solve_extrapolated.argtypes = [P, dbl, P]
    L.ecmg_solve_fixed.argtypes = [P, P, P]
    L.ecmg_extrapolate.argtypes = [P, i32, P]
    L.ecmg_prolongate.argtypes = [P, i32]
    L.ecmg_jcg.argtypes = [P, i32, dbl, i32, P]
    L.ecmg_apply.argtypes = [P, i32, P, P]
    L.ecmg_get.argtypes = [P, i32, i32, P]
    L.ecmg_set.argtypes = [P, i32, i32, P]
    L.ecmg_device_view.argtypes = [P, i32, i32, ctypes.POINTER(P), P, P]
    L.ecmg_norms.argtypes = [P, i32, i32, i32, P, i32, P]
    L.ecmg_norms_noalloc.argtypes = [P, i32, i32, i32, P]
    L.ecmg_level_dims.argtypes = [P, i32, P]
    L.ecmg_plan_bytes.argtypes = [ctypes.POINTER(ProblemC), i32, ctypes.POINTER(ctypes.c_size_t)]
    L.ecmg_kernel_times.argtypes = [P, i32, i32, P]
    L.ecmg_reset_kernel_times.argtypes = [P]
    L.ecmg_set_timing.argtypes = [P, i32]
    L.ecmg_cascadic_schedule.argtypes = [i32, i32, dbl, P]
    L.ecmg_solve_levels.argtypes = [P, P, P]
    L.ecmg_autotune_batch.argtypes = [P, i32, dbl, ctypes.c_char_p, P]
    L.ecmg_tolerance_schedule.argtypes = [i32, dbl, dbl, P]
    L.ecmg_last_error.argtypes = [P]
    L.ecmg_last_error.restype = ctypes.c_char_p
    L.ecmg_destroy.argtypes = [P]
    L.ecmg_destroy.restype = None
    L.ecmg_solve_batch.argtypes = [P, i32, dbl, P]
    L.ecmg_extrapolate_batch.argtypes = [P, i32]
    L.ecmg_server_create.argtypes = [ctypes.POINTER(Options), ctypes.c_size_t, ctypes.POINTER(P)]
    L.ecmg_server_submit.argtypes = [P, ctypes.POINTER(ProblemC), dbl, P, ctypes.POINTER(ctypes.c_uint64)]
    L.ecmg_server_step.argtypes = [P, ctypes.POINTER(i32)]
    L.ecmg_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(i32), P]
    L.ecmg_server_stats.argtypes = [P, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                    ctypes.POINTER(ctypes.c_int64)]
    L.ecmg_server_completed.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), i32, ctypes.POINTER(i32)]
    L.ecmg_server_times.argtypes = [P, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.ecmg_server_reset_stats.argtypes = [P]
    L.ecmg_server_destroy.argtypes = [P]
    L.ecmg_server_destroy.restype = None
    L.ecmg_autotune.argtypes = [P, i32, ctypes.c_char_p, P]
    L.ecmg_tune_lookup.argtypes = [ctypes.c_char_p, i32, i32, i32, i32, P]
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def tune_lookup(path: str, n, precision: int = FP64) -> Optional[dict]:
    """The choice a tuning cache holds for a JCG level of n = (nx, ny, nz)
    elements (host only; None if there is none)."""
    L = load_library()
    r = TuneResult()
    rc = L.ecmg_tune_lookup(path.encode(), int(precision), int(n[0]), int(n[1]), int(n[2]), ctypes.byref(r))
    if rc == ENOENT:
        return None
    if rc != OK:
        raise EcmgError(rc, (L.ecmg_last_error(None) or b"").decode())
    return r.as_dict()


def cascadic_schedule(levels: int, m_L: int, beta: float) -> List[int]:
    """Per-level iteration counts of the original ECMG (Algorithm 3, eq. ee)
    for Solver.solve_fixed: 0 on the two DSOLVE grids, ceil(m_L beta^(L-j)) on
    fine grid j (host only)."""
    L = load_library()
    out = (ctypes.c_int32 * int(levels))()
    rc = L.ecmg_cascadic_schedule(int(levels), int(m_L), float(beta), out)
    if rc != OK:
        raise EcmgError(rc, (L.ecmg_last_error(None) or b"").decode())
    return list(out)


def tolerance_schedule(levels: int, eps_finest: float, ratio: float) -> List[float]:
    """Per-level relative tolerances for Solver.solve_levels: 0 on the two
    DSOLVE grids, min(1, eps_finest * ratio^(levels-1-l)) on level l (host only)."""
    L = load_library()
    out = (ctypes.c_double * int(levels))()
    rc = L.ecmg_tolerance_schedule(int(levels), float(eps_finest), float(ratio), out)
    if rc != OK:
        raise EcmgError(rc, (L.ecmg_last_error(None) or b"").decode())
    return list(out)


class EcmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_STATUS.get(code, "?"), code, msg))
        self.code = code


# ---------------------------------------------------------------------------
# fields
# ---------------------------------------------------------------------------

def _host_callback(fn):
    """Wrap a numpy field fn(x, y, z, face) as a tensor-product host callback."""
    def cb(face, nx, ny, nz, px, py, pz, pout, user):
        try:
            x = np.ctypeslib.as_array(ctypes.cast(px, ctypes.POINTER(ctypes.c_double)), shape=(nx,))
            y = np.ctypeslib.as_array(ctypes.cast(py, ctypes.POINTER(ctypes.c_double)), shape=(ny,))
            z = np.ctypeslib.as_array(ctypes.cast(pz, ctypes.POINTER(ctypes.c_double)), shape=(nz,))
            out = np.ctypeslib.as_array(ctypes.cast(pout, ctypes.POINTER(ctypes.c_double)), shape=(nz, ny, nx))
            v = fn(x[None, None, :], y[None, :, None], z[:, None, None], int(face))
            out[...] = np.broadcast_to(v, (nz, ny, nx))
            return 0
        except Exception:                      # noqa: BLE001 - reported as ECMG_ECALLBACK
            import traceback
            traceback.print_exc()
            return 1
    return HOST_FN(cb)


class _DevArray:
    def __init__(self, ptr, shape):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": "<f8", "data": (int(ptr), False),
                                         "version": 3, "strides": None}


def _device_callback(fn):
    """Wrap a field fn(x, y, z, face) written with array methods torch supports
    as a device callback evaluated by torch on the GPU."""
    import torch

    def cb(face, nx, ny, nz, px, py, pz, pout, stream, user):
        try:
            torch.cuda.init()
            dev = torch.device("cuda", torch.cuda.current_device())
            with torch.cuda.stream(torch.cuda.ExternalStream(int(stream), device=dev)):
                x = torch.as_tensor(_DevArray(px, (nx,)), device="cuda")
                y = torch.as_tensor(_DevArray(py, (ny,)), device="cuda")
                z = torch.as_tensor(_DevArray(pz, (nz,)), device="cuda")
                out = torch.as_tensor(_DevArray(pout, (nz, ny, nx)), device="cuda")
                v = fn(x[None, None, :], y[None, :, None], z[:, None, None], int(face))
                out.copy_(torch.as_tensor(v, dtype=torch.float64, device="cuda").expand(nz, ny, nx))
            return 0
        except Exception:                      # noqa: BLE001
            import traceback
            traceback.print_exc()
            return 1
    return DEVICE_FN(cb)


def _field(fn, device: bool, keep: list) -> Field:
    f = Field()
    c = getattr(fn, "constant", None)
    if c is not None or isinstance(fn, (int, float)):
        f.value = float(c if c is not None else fn)
        return f
    if device:
        cb = _device_callback(fn)
        f.device = cb
    else:
        cb = _host_callback(fn)
        f.host = cb
    keep.append(cb)
    return f


def problem_struct(problem, device_fields: bool = False):
    """ctypes ecmg_problem for a workloads.Problem; returns (struct, keepalive)."""
    keep: list = []
    p = ProblemC()
    for d in range(3):
        p.lo[d] = float(problem.lo[d])
        p.hi[d] = float(problem.hi[d])
        p.n0[d] = int(problem.n0[d])
    p.levels = int(problem.levels)
    for f in range(6):
        p.face_type[f] = int(problem.face_type[f])
    p.beta = _field(problem.beta, device_fields, keep)
    p.f = _field(problem.f, device_fields, keep)
    p.g_D = _field(problem.gD, device_fields, keep)
    p.alpha = _field(problem.alpha, device_fields, keep)
    p.g_R = _field(problem.gR, device_fields, keep)
    return p, keep


# ---------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------

def _torch_allocator_hooks():
    """(alloc, free) callbacks that take the library's device memory from
    PyTorch's caching allocator, on the library's stream."""
    import torch

    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                      torch.cuda.ExternalStream(int(stream or 0)))
        except Exception:                      # noqa: BLE001 - reported as ECMG_ENOMEM
            return None

    def free(ptr, stream, user):
        torch.cuda.caching_allocator_delete(int(ptr))

    return ALLOC_FN(alloc), FREE_FN(free)


class Solver:
    """One ECMG_jcg (or, with method=CG, ECMG_cg) context: one problem
    hierarchy resident on the device."""

    def __init__(self, precision: int = FP64, interp: int = SERENDIPITY20, keep_w: bool = True,
                 max_iter: int = 20000, dsolve_tol: float = 1e-14, inner_tol: float = 1e-4,
                 chunk: int = 0, timing: bool = False, stream=None, persistent_nodes: int = -1,
                 dsolve_dense_max: Optional[int] = None, autotune: int = 0, tune_cache: Optional[str] = None,
                 method: int = JCG, speculate: bool = True, fold_blocks: int = -1, true_residual: bool = False,
                 batch_graph: bool = True, columns: bool = True, gather_nodes: int = -1,
                 torch_allocator: bool = False):
        self.L = load_library()
        o = Options()
        self.L.ecmg_default_options(ctypes.byref(o))
        o.precision, o.interp, o.keep_w, o.max_iter = precision, interp, int(keep_w), max_iter
        o.dsolve_tol, o.inner_tol, o.chunk, o.timing = dsolve_tol, inner_tol, chunk, int(timing)
        o.hip_stream = stream
        o.persistent_nodes = persistent_nodes
        if dsolve_dense_max is not None:
            o.dsolve_dense_max = dsolve_dense_max
        o.autotune = int(autotune)
        o.tune_cache = tune_cache.encode() if tune_cache else None
        o.method = int(method)
        o.speculate = int(speculate)
        o.fold_blocks = int(fold_blocks)
        o.true_residual = int(true_residual)
        o.batch_graph = int(batch_graph)
        o.columns = int(columns)
        o.gather_nodes = int(gather_nodes)
        self._hooks = None
        if torch_allocator:
            self._hooks = _torch_allocator_hooks()
            o.alloc, o.free = self._hooks
        self.opt = o
        h = ctypes.c_void_p()
        self._check(self.L.ecmg_create(ctypes.byref(o), ctypes.byref(h)), None)
        self.h = h
        self.levels = 0
        self._keep = None
        _live.add(self)

    def _check(self, rc, h="self"):
        if rc != OK:
            msg = self.L.ecmg_last_error(self.h if h == "self" else None)
            raise EcmgError(rc, (msg or b"").decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.L.ecmg_destroy(self.h)
            self.h = None

    def __del__(self):
        if _finalizing is None or _finalizing():
            return
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- calls --------------------------------------------------------------
    def setup(self, problem, device_fields: bool = False):
        p, keep = problem_struct(problem, device_fields)
        self._keep = (p, keep)
        self._check(self.L.ecmg_setup(self.h, ctypes.byref(p)))
        self.levels = int(problem.levels)
        return self

    def _infos(self):
        return (LevelInfo * self.levels)()

    def autotune(self, iters: int = 8, cache: Optional[str] = None) -> List[dict]:
        """Time the candidate JCG configurations of every JCG level (after setup),
        keep the fastest for later solves, merge them into the JSON cache.
        iters <= 0 times each level over its iteration count in the last solve."""
        out = (TuneResult * max(self.levels - 2, 1))()
        self._check(self.L.ecmg_autotune(self.h, int(iters), cache.encode() if cache else None, out))
        return [r.as_dict() for r in out[:max(self.levels - 2, 0)]]

    def solve(self, rel_tol: float, allow_fail: bool = False, extrapolate: bool = False) -> List[dict]:
        """ecmg_solve; extrapolate=True: ecmg_solve_extrapolated (EXP_true on
        the finest level enqueued behind the cascade, one wait)."""
        info = self._infos()
        fn = self.L.ecmg_solve_extrapolated if extrapolate else self.L.ecmg_solve
        rc = fn(self.h, float(rel_tol), info)
        if not allow_fail:
            self._check(rc)
        return [i.as_dict() for i in info]

    def solve_levels(self, rel_tol: Sequence[float], allow_fail: bool = False) -> List[dict]:
        """ecmg_solve with one relative tolerance per level (entries 0, 1 ignored)."""
        info = self._infos()
        arr = (ctypes.c_double * self.levels)(*[float(v) for v in rel_tol])
        rc = self.L.ecmg_solve_levels(self.h, arr, info)
        if not allow_fail:
            self._check(rc)
        return [i.as_dict() for i in info]

    def solve_fixed(self, iters: Sequence[int]) -> List[dict]:
        info = self._infos()
        arr = (ctypes.c_int32 * self.levels)(*[int(v) for v in iters])
        self._check(self.L.ecmg_solve_fixed(self.h, arr, info))
        return [i.as_dict() for i in info]

    def dims(self, level: int) -> tuple:
        n = (ctypes.c_int64 * 3)()
        self._check(self.L.ecmg_level_dims(self.h, int(level), n))
        return tuple(int(v) for v in n)

    def nodes(self, level: int) -> int:
        n = self.dims(level)
        return (n[0] + 1) * (n[1] + 1) * (n[2] + 1)

    def extrapolate(self, level: int = -1, out: bool = True) -> Optional[np.ndarray]:
        if level < 0:
            level = self.levels - 1
        buf = np.empty(self.nodes(level)) if out else None
        self._check(self.L.ecmg_extrapolate(self.h, int(level), None if buf is None else buf.ctypes.data))
        return buf

    def prolongate(self, level: int):
        self._check(self.L.ecmg_prolongate(self.h, int(level)))

    def jcg(self, level: int, rel_tol: float, fixed_iters: int = -1, allow_fail: bool = False) -> dict:
        info = LevelInfo()
        rc = self.L.ecmg_jcg(self.h, int(level), float(rel_tol), int(fixed_iters), ctypes.byref(info))
        if not allow_fail:
            self._check(rc)
        d = info.as_dict()
        d["rc"] = rc
        return d

    def apply(self, level: int, v: np.ndarray) -> np.ndarray:
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert v.size == self.nodes(level)
        out = np.empty_like(v)
        self._check(self.L.ecmg_apply(self.h, int(level), v.ctypes.data, out.ctypes.data))
        return out

    def get(self, level: int, which: int = VEC_U) -> np.ndarray:
        if level < 0:
            level = self.levels - 1
        out = np.empty(self.nodes(level))
        self._check(self.L.ecmg_get(self.h, int(level), int(which), out.ctypes.data))
        return out

    def set(self, level: int, which: int, v: np.ndarray):
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert v.size == self.nodes(level)
        self._check(self.L.ecmg_set(self.h, int(level), int(which), v.ctypes.data))

    def device_view(self, level: int, which: int = VEC_U):
        """(device pointer, (nx+1, ny+1, nz+1), row pitch in elements)."""
        ptr = ctypes.c_void_p()
        dims = (ctypes.c_int64 * 3)()
        pitch = ctypes.c_int64()
        self._check(self.L.ecmg_device_view(self.h, int(level), int(which), ctypes.byref(ptr), dims,
                                            ctypes.byref(pitch)))
        return int(ptr.value), tuple(int(v) for v in dims), int(pitch.value)

    def norms(self, level: int, which: int, minus_which: int = VEC_NONE, minus=None):
        """(max, RMS) of vec[which] - vec[minus_which] - minus; ``minus`` is a
        numpy array or a contiguous float64 torch tensor on the device."""
        out = (ctypes.c_double * 2)()
        on_dev, ptr = 0, None
        if minus is not None and type(minus).__module__.startswith("torch"):
            import torch
            assert minus.is_cuda and minus.dtype == torch.float64 and minus.is_contiguous()
            assert minus.numel() == self.nodes(level if level >= 0 else self.levels - 1)
            torch.cuda.current_stream().synchronize()   # the library works on its own stream
            on_dev, ptr = 1, minus.data_ptr()
        elif minus is not None:
            m = np.ascontiguousarray(minus, dtype=np.float64)
            ptr = m.ctypes.data
        self._check(self.L.ecmg_norms(self.h, int(level), int(which), int(minus_which), ptr, on_dev, out))
        return float(out[0]), float(out[1])

    def norms_noalloc(self, level: int, which: int, minus_which: int = VEC_NONE):
        """ecmg_norms_noalloc: (max, RMS) of vec[which] - vec[minus_which] with
        the reduction's scratch in the library's static device array."""
        out = (ctypes.c_double * 2)()
        self._check(self.L.ecmg_norms_noalloc(self.h, int(level), int(which), int(minus_which), out))
        return float(out[0]), float(out[1])

    def kernel_times(self, level: int, kind: int) -> tuple:
        out = (ctypes.c_double * 2)()
        self._check(self.L.ecmg_kernel_times(self.h, int(level), int(kind), out))
        return float(out[0]), int(out[1])

    def reset_kernel_times(self):
        self._check(self.L.ecmg_reset_kernel_times(self.h))

    def set_timing(self, classes) -> None:
        """Time these kernel classes from now on (an iterable of class numbers,
        or -1 for all, 0 for none)."""
        mask = classes if isinstance(classes, int) else sum(1 << int(k) for k in classes)
        self._check(self.L.ecmg_set_timing(self.h, int(mask)))


def solve_batch(solvers: Sequence["Solver"], rel_tol: float, allow_fail: bool = False) -> List[List[dict]]:
    """ecmg_solve_batch over set-up solvers; returns each box's level infos."""
    L = load_library()
    n = len(solvers)
    handles = (ctypes.c_void_p * n)(*[s.h for s in solvers])
    total = sum(s.levels for s in solvers)
    info = (LevelInfo * total)()
    rc = L.ecmg_solve_batch(handles, n, float(rel_tol), info)
    if rc != OK and not allow_fail:
        msg = L.ecmg_last_error(solvers[0].h)
        raise EcmgError(rc, (msg or b"").decode())
    out, k = [], 0
    for s in solvers:
        out.append([info[k + l].as_dict() for l in range(s.levels)])
        k += s.levels
    return out


def autotune_batch(solvers: Sequence["Solver"], rel_tol: float, cache: Optional[str] = None) -> dict:
    """ecmg_autotune_batch: time the batched solve of these solvers under the
    candidate nodes-per-workgroup and segment settings, keep the fastest on all
    of them (and in the JSON cache)."""
    L = load_library()
    n = len(solvers)
    handles = (ctypes.c_void_p * n)(*[s.h for s in solvers])
    r = TuneResult()
    rc = L.ecmg_autotune_batch(handles, n, float(rel_tol), cache.encode() if cache else None, ctypes.byref(r))
    if rc != OK:
        msg = L.ecmg_last_error(solvers[0].h)
        raise EcmgError(rc, (msg or b"").decode())
    d = r.as_dict()
    d["path"] = "batch"
    d["nodes_per_workgroup"] = d.pop("nwg")
    return d


def extrapolate_batch(solvers: Sequence["Solver"]) -> None:
    """ecmg_extrapolate_batch: EXP_true on the finest level of every solver."""
    L = load_library()
    n = len(solvers)
    handles = (ctypes.c_void_p * n)(*[s.h for s in solvers])
    rc = L.ecmg_extrapolate_batch(handles, n)
    if rc != OK:
        msg = L.ecmg_last_error(solvers[0].h)
        raise EcmgError(rc, (msg or b"").decode())


class Server:
    """ecmg_server: continuous batching of independent requests (FP64).

    submit() queues a problem (its field structures are kept alive here until
    the request is released; the server's set-up thread calls them); step()
    takes in the requests set up since the last step, advances every active
    request by one level and finishes completed ones; result() returns U~ on
    the finest grid."""

    def __init__(self, hbm_budget_bytes: int, device_fields: bool = True, **opts):
        self.L = load_library()
        o = Options()
        self.L.ecmg_default_options(ctypes.byref(o))
        for k, v in opts.items():
            setattr(o, k, v.encode() if isinstance(v, str) else v)
        self.h = ctypes.c_void_p()
        rc = self.L.ecmg_server_create(ctypes.byref(o), int(hbm_budget_bytes), ctypes.byref(self.h))
        if rc != OK:
            raise EcmgError(rc, (self.L.ecmg_last_error(None) or b"").decode())
        self.device_fields = device_fields
        self._req = {}
        _live.add(self)

    def _check(self, rc):
        if rc != OK:
            raise EcmgError(rc, (self.L.ecmg_last_error(None) or b"").decode())

    def submit(self, problem, rel_tol: float, want_result: bool = True) -> int:
        p, keep = problem_struct(problem, self.device_fields)
        n = [int(v) << (problem.levels - 1) for v in problem.n0]
        out = np.empty((n[2] + 1, n[1] + 1, n[0] + 1)) if want_result else None
        t = ctypes.c_uint64()
        self._check(self.L.ecmg_server_submit(self.h, ctypes.byref(p), float(rel_tol),
                                              out.ctypes.data if out is not None else None, ctypes.byref(t)))
        self._req[t.value] = (p, keep, out, problem.levels)
        return t.value

    def step(self) -> int:
        d = ctypes.c_int32()
        self._check(self.L.ecmg_server_step(self.h, ctypes.byref(d)))
        return d.value

    def poll(self, ticket: int):
        """(state, infos): state 0 queued, 1 running, 2 done, < 0 error."""
        st = ctypes.c_int32()
        levels = self._req[ticket][3]
        info = (LevelInfo * levels)()
        self._check(self.L.ecmg_server_poll(self.h, ticket, ctypes.byref(st), info))
        return st.value, ([i.as_dict() for i in info] if st.value == 2 else None)

    def result(self, ticket: int):
        return self._req[ticket][2]

    def release(self, ticket: int):
        """Drop the kept problem structures and result of a finished request
        (the set-up thread calls the field callbacks until it is set up, and
        U~ is written to the result buffer when it is done)."""
        if ticket in self._req:
            st, _ = self.poll(ticket)
            if st in (0, 1):
                raise EcmgError(ESTATE, "request %d is still %s" % (ticket, "queued" if st == 0 else "running"))
        self._req.pop(ticket, None)

    def stats(self) -> dict:
        p50, p99, sps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        done = ctypes.c_int64()
        self._check(self.L.ecmg_server_stats(self.h, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(sps),
                                             ctypes.byref(done)))
        st, tk, fi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self.L.ecmg_server_times(self.h, ctypes.byref(st), ctypes.byref(tk), ctypes.byref(fi)))
        return {"p50_ms": p50.value, "p99_ms": p99.value, "solves_per_s": sps.value, "done": done.value,
                "host_ms": {"setup": st.value, "steps": tk.value, "finish": fi.value}}

    def completed(self) -> list:
        """Tickets of the requests finished (done or failed) since the last call."""
        out = []
        buf = (ctypes.c_uint64 * 256)()
        n = ctypes.c_int32()
        while True:
            self._check(self.L.ecmg_server_completed(self.h, buf, 256, ctypes.byref(n)))
            out.extend(buf[:n.value])
            if n.value < 256:
                return out

    def reset_stats(self):
        self._check(self.L.ecmg_server_reset_stats(self.h))

    def close(self):
        if self.h:
            self.L.ecmg_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        if _finalizing is None or _finalizing():
            return
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def plan_bytes(problem, precision: int = FP64) -> int:
    L = load_library()
    p, keep = problem_struct(problem)
    out = ctypes.c_size_t()
    rc = L.ecmg_plan_bytes(ctypes.byref(p), int(precision), ctypes.byref(out))
    if rc != OK:
        raise EcmgError(rc, (L.ecmg_last_error(None) or b"").decode())
    return int(out.value)


def last_error() -> str:
    return (load_library().ecmg_last_error(None) or b"").decode()
