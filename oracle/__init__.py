"""CPU FP64 oracle for the ECMG_jcg cascade (arXiv 1506.02983).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library (which must not fall
back to it).  The arithmetic lives in ``ecmg_oracle.c`` (plain C, FP64); this
module marshals arguments and runs Algorithm 4 step by step:

  O1 grid          level l has n0*2^l elements per axis (Section 4.1, Algorithm 4)
  O2 coefficients  beta at element centroids, alpha at Robin face-element centroids
  O3 matrix        Q1 element matrices by Gauss quadrature, assembled CSR (Section 2)
  O4 load          2x2x2 Gauss per element, 2x2 per Robin face element (Section 2)
  O5 system        Dirichlet lifting b = F - A_FD g_D; the ||f_h|| of the stopping
                   test is the norm of (b on free nodes, g_D on Dirichlet nodes),
                   i.e. of the right-hand side with Dirichlet identity rows
  O6 DSOLVE        banded Cholesky on the two coarsest grids
  O7 JCG           PCG with M = diag(A_FF) while ||r||_2 > eps ||f_h||_2; ECMG_cg
                   (Section 4.1) the same recurrence with M = I
  O7b schedule     eq. ee: the fixed per-grid CG counts of Algorithm 3
  O8 EXP_finite    eqs. jiedian, zhongdian, inter (Section 4.3)
  O9 cascade       Algorithm 4
  O10 EXP_true     eqs. t1 and chenlin (Sections 4.2.1, 4.3)
  O11 norms        max norm and the discrete L2 norm of the tables, the root mean
                   square over all nodes (Section 5)
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

from workloads import DIRICHLET, ROBIN, Problem, tensor_eval

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ecmg_oracle.c")
_SO = os.path.join(_HERE, "libecmg_oracle.so")
_GAUSS = 1.0 / math.sqrt(3.0)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("face_type", ctypes.c_int32 * 6)]


class _CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        G = ctypes.POINTER(_Grid)
        C = ctypes.POINTER(_CSR)
        i64, dbl = ctypes.c_int64, ctypes.c_double
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_dirichlet_mask.argtypes = [G, P]
        L.orc_element_stiffness.argtypes = [dbl, dbl, dbl, P]
        L.orc_face_mass.argtypes = [dbl, dbl, P]
        L.orc_csr_nnz.argtypes = [G]
        L.orc_csr_nnz.restype = i64
        L.orc_assemble.argtypes = [G, P, P, P, P, P]
        L.orc_load.argtypes = [G, P, P, P]
        L.orc_spmv.argtypes = [C, P, P, P]
        L.orc_diagonal.argtypes = [C, P]
        L.orc_lift.argtypes = [C, P, P, P, P]
        L.orc_lift.restype = dbl
        L.orc_rhs_norm.argtypes = [i64, P, P, P]
        L.orc_rhs_norm.restype = dbl
        L.orc_jcg.argtypes = [C, P, P, P, P, dbl, i64, i64, dbl, P, P, P, P]
        L.orc_dsolve.argtypes = [G, C, P, P, P]
        L.orc_serendipity_weight.argtypes = [ctypes.c_int] * 3 + [dbl] * 3
        L.orc_serendipity_weight.restype = dbl
        L.orc_exp_finite_node.argtypes = [i64, i64, i64, P, P, i64, i64, i64]
        L.orc_exp_finite_node.restype = dbl
        L.orc_exp_finite_node_lagrange27.argtypes = [i64, i64, i64, P, P, i64, i64, i64]
        L.orc_exp_finite_node_lagrange27.restype = dbl
        L.orc_exp_finite.argtypes = [G, P, P, P, ctypes.c_int]
        L.orc_exp_finite_points.argtypes = [i64, i64, i64, P, P, P, i64, P, ctypes.c_int]
        L.orc_exp_true_node.argtypes = [i64, i64, i64, P, P, i64, i64, i64]
        L.orc_exp_true_node.restype = dbl
        L.orc_exp_true.argtypes = [G, P, P, P]
        L.orc_exp_true_points.argtypes = [i64, i64, i64, P, P, P, i64, P]
        L.orc_apply_rows.argtypes = [G, P, P, P, P, i64, P]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops (timing of the baseline)."""
    lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------------------
# O1/O2: grid and point sets
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Grid:
    n: tuple            # elements per axis
    lo: tuple
    hi: tuple
    face_type: tuple

    @property
    def h(self):
        return tuple((self.hi[d] - self.lo[d]) / self.n[d] for d in range(3))

    @property
    def nodes(self):
        return tuple(n + 1 for n in self.n)

    @property
    def num_nodes(self):
        return (self.n[0] + 1) * (self.n[1] + 1) * (self.n[2] + 1)

    def c(self) -> _Grid:
        g = _Grid()
        g.nx, g.ny, g.nz = self.n
        g.hx, g.hy, g.hz = self.h
        for f in range(6):
            g.face_type[f] = int(self.face_type[f])
        return g

    # coordinates along axis d
    def node_coords(self, d):
        return self.lo[d] + np.arange(self.n[d] + 1) * self.h[d]

    def centroid_coords(self, d):
        return self.lo[d] + (np.arange(self.n[d]) + 0.5) * self.h[d]

    def gauss_coords(self, d):
        """Two Gauss points per element, element e's at its origin + (1 -/+ 1/sqrt3) h/2."""
        h = self.h[d]
        e0 = self.lo[d] + np.arange(self.n[d]) * h
        out = np.empty(2 * self.n[d])
        out[0::2] = e0 + (1.0 - _GAUSS) * h / 2.0
        out[1::2] = e0 + (1.0 + _GAUSS) * h / 2.0
        return out

    def face_plane(self, f):
        d = f // 2
        return np.array([self.lo[d] if f % 2 == 0 else self.hi[d]])


def grid_of(problem: Problem, level: int) -> Grid:
    return Grid(problem.n_at(level), tuple(map(float, problem.lo)), tuple(map(float, problem.hi)),
                tuple(problem.face_type))


def _face_eval(fn, grid: Grid, f: int, kind: str) -> np.ndarray:
    """Evaluate a field on face f's face elements: 'centroid' or 'gauss' points,
    returned as a flat array with the face's first in-plane axis fastest."""
    ax = f // 2
    sets = []
    for d in range(3):
        if d == ax:
            sets.append(grid.face_plane(f))
        elif kind == "centroid":
            sets.append(grid.centroid_coords(d))
        else:
            sets.append(grid.gauss_coords(d))
    return tensor_eval(fn, sets[0], sets[1], sets[2], face=f).ravel()


# ---------------------------------------------------------------------------
# O3-O5: discretisation of one level
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Level:
    grid: Grid
    beta: np.ndarray
    alpha: List[Optional[np.ndarray]]
    dmask: np.ndarray
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    D: np.ndarray
    F: np.ndarray
    gD: np.ndarray      # g_D on Dirichlet nodes, 0 elsewhere
    b: np.ndarray
    nb: float           # ||b||_2 over free nodes
    nf: float = 0.0     # ||f_h||_2 of the stopping test (b and g_D rows)

    def csr(self) -> _CSR:
        c = _CSR()
        c.n = self.grid.num_nodes
        c.nnz = self.col.size
        c.rowptr, c.col, c.val = _ptr(self.rowptr), _ptr(self.col), _ptr(self.val)
        return c

    def dense(self) -> np.ndarray:
        n = self.grid.num_nodes
        A = np.zeros((n, n))
        for r in range(n):
            s, e = self.rowptr[r], self.rowptr[r + 1]
            A[r, self.col[s:e]] = self.val[s:e]
        return A


def coefficients(problem: Problem, grid: Grid):
    """O2: beta per element (centroid), alpha per Robin face element (centroid)."""
    beta = tensor_eval(problem.beta, grid.centroid_coords(0), grid.centroid_coords(1),
                       grid.centroid_coords(2)).ravel()
    alpha = [None] * 6
    for f in range(6):
        if grid.face_type[f] == ROBIN:
            alpha[f] = np.ascontiguousarray(_face_eval(problem.alpha, grid, f, "centroid"))
    return beta, alpha


def dirichlet_mask(grid: Grid) -> np.ndarray:
    m = np.zeros(grid.num_nodes, dtype=np.uint8)
    lib().orc_dirichlet_mask(ctypes.byref(grid.c()), _ptr(m))
    return m


def assemble(grid: Grid, beta: np.ndarray, alpha) -> tuple:
    L = lib()
    g = grid.c()
    nnz = int(L.orc_csr_nnz(ctypes.byref(g)))
    rowptr = np.zeros(grid.num_nodes + 1, dtype=np.int64)
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz)
    ap = (ctypes.c_void_p * 6)(*[_ptr(a) for a in alpha])
    L.orc_assemble(ctypes.byref(g), _ptr(beta), ap, _ptr(rowptr), _ptr(col), _ptr(val))
    assert rowptr[-1] == nnz
    return rowptr, col, val


def load_vector(problem: Problem, grid: Grid) -> np.ndarray:
    """O4: F by 2x2x2 Gauss on f and 2x2 Gauss on g_R over Robin faces."""
    fg = tensor_eval(problem.f, grid.gauss_coords(0), grid.gauss_coords(1), grid.gauss_coords(2)).ravel()
    gR = [None] * 6
    for f in range(6):
        if grid.face_type[f] == ROBIN:
            gR[f] = np.ascontiguousarray(_face_eval(problem.gR, grid, f, "gauss"))
    F = np.zeros(grid.num_nodes)
    gp = (ctypes.c_void_p * 6)(*[_ptr(a) for a in gR])
    lib().orc_load(ctypes.byref(grid.c()), _ptr(fg), gp, _ptr(F))
    return F


def discretize(problem: Problem, level: int) -> Level:
    grid = grid_of(problem, level)
    beta, alpha = coefficients(problem, grid)
    dmask = dirichlet_mask(grid)
    rowptr, col, val = assemble(grid, beta, alpha)
    F = load_vector(problem, grid)
    gD = tensor_eval(problem.gD, grid.node_coords(0), grid.node_coords(1), grid.node_coords(2)).ravel()
    gD = np.where(dmask == 1, gD, 0.0)
    lv = Level(grid, beta, alpha, dmask, rowptr, col, val, np.zeros(grid.num_nodes), F, gD,
               np.zeros(grid.num_nodes), 0.0)
    c = lv.csr()
    lib().orc_diagonal(ctypes.byref(c), _ptr(lv.D))
    lv.nb = float(lib().orc_lift(ctypes.byref(c), _ptr(dmask), _ptr(F), _ptr(gD), _ptr(lv.b)))
    lv.nf = float(lib().orc_rhs_norm(grid.num_nodes, _ptr(dmask), _ptr(lv.b), _ptr(gD)))
    return lv


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------

def spmv(lv: Level, v: np.ndarray) -> np.ndarray:
    """(A v) on free rows, 0 on Dirichlet rows (all columns used)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    y = np.zeros_like(v)
    lib().orc_spmv(ctypes.byref(lv.csr()), _ptr(lv.dmask), _ptr(v), _ptr(y))
    return y


def dsolve(lv: Level) -> np.ndarray:
    x = lv.gD.copy()
    st = lib().orc_dsolve(ctypes.byref(lv.grid.c()), ctypes.byref(lv.csr()), _ptr(lv.dmask), _ptr(lv.F), _ptr(x))
    if st != 0:
        raise RuntimeError("oracle DSOLVE failed (%d)" % st)
    return x


@dataclasses.dataclass
class JCGResult:
    x: np.ndarray
    iters: int
    rre: float
    rre_true: float
    status: int
    hist: np.ndarray


JCG_METHOD = 0      # Section 4.1: CG preconditioned with M = diag(A) (ECMG_jcg)
CG_METHOD = 1       # Section 4.1: ECMG_cg, the same CG with M = I


def jcg(lv: Level, x0: np.ndarray, eps: float, max_iter: int = 20000, fixed_iters: int = -1,
        method: int = JCG_METHOD) -> JCGResult:
    """Preconditioned CG of Algorithm 4 (M = diag(A)); with ``method=CG_METHOD``
    plain CG, i.e. the same recurrence with M = I on the free nodes."""
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()
    D = lv.D if method == JCG_METHOD else np.ones_like(lv.D)
    it = ctypes.c_int64(0)
    rre = ctypes.c_double(0.0)
    rrt = ctypes.c_double(0.0)
    hist = np.zeros(max(max_iter, fixed_iters) + 2)
    st = lib().orc_jcg(ctypes.byref(lv.csr()), _ptr(lv.dmask), _ptr(D), _ptr(lv.F), _ptr(x),
                       float(eps), int(max_iter), int(fixed_iters), float(lv.nf),
                       ctypes.byref(it), ctypes.byref(rre), ctypes.byref(rrt), _ptr(hist))
    return JCGResult(x, int(it.value), float(rre.value), float(rrt.value), int(st), hist[: it.value + 1])


def cascadic_schedule(levels: int, m_L: int, beta: float) -> List[int]:
    """Eq. ee (Algorithm 3): with L = levels - 2 fine grids, grid j = 1..L
    (hierarchy level j + 1) runs m_j = ceil(m_L * beta^(L - j)) CG steps; the
    two DSOLVE grids run none.  The power is taken as repeated products."""
    if levels < 3 or m_L < 1 or not (beta >= 1.0) or not math.isfinite(beta):
        raise ValueError("need levels >= 3, m_L >= 1, beta >= 1")
    L = levels - 2
    out = [0, 0]
    for j in range(1, L + 1):
        m = float(m_L)
        for _ in range(L - j):
            m *= beta
        out.append(int(math.ceil(m)))
    return out


def tolerance_schedule(levels: int, eps_finest: float, ratio: float) -> List[float]:
    """Per-level relative tolerances: eps_finest on the finest grid, each coarser
    JCG grid ``ratio`` times looser (capped at 1), 0 on the DSOLVE grids.  The
    paper fixes no schedule (Section 5 only says fine grids need a stricter
    tolerance); this geometric one is the library's."""
    if levels < 3 or not (eps_finest > 0.0) or not (ratio >= 1.0):
        raise ValueError("need levels >= 3, eps_finest > 0, ratio >= 1")
    out = [0.0, 0.0]
    for l in range(2, levels):
        e = float(eps_finest)
        for _ in range(l, levels - 1):
            e *= ratio
        out.append(min(e, 1.0))
    return out


SERENDIPITY20 = 0   # Section 4.3: 20 extrapolated nodes + serendipity (eq. inter)
LAGRANGE27 = 1      # the Remark after eq. inter: 27 nodes + tri-quadratic Lagrange


def exp_finite(grid: Grid, U1: np.ndarray, U0: np.ndarray, variant: int = SERENDIPITY20) -> np.ndarray:
    """W on every node of level ``grid`` from U1 = u_{l-1}, U0 = u_{l-2}
    (g_D is not imposed here)."""
    W = np.zeros(grid.num_nodes)
    lib().orc_exp_finite(ctypes.byref(grid.c()), _ptr(np.ascontiguousarray(U1)),
                         _ptr(np.ascontiguousarray(U0)), _ptr(W), int(variant))
    return W


def exp_finite_points(n: Sequence[int], U1, U0, pts, variant: int = SERENDIPITY20) -> np.ndarray:
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.zeros(pts.size)
    lib().orc_exp_finite_points(int(n[0]), int(n[1]), int(n[2]), _ptr(np.ascontiguousarray(U1)),
                                _ptr(np.ascontiguousarray(U0)), _ptr(pts), pts.size, _ptr(out), int(variant))
    return out


def exp_true(grid: Grid, U1: np.ndarray, U0: np.ndarray) -> np.ndarray:
    """Fourth-order extrapolation on level ``grid`` from U1 = u_l and U0 = u_{l-1}."""
    Ut = np.zeros(grid.num_nodes)
    lib().orc_exp_true(ctypes.byref(grid.c()), _ptr(np.ascontiguousarray(U1)),
                       _ptr(np.ascontiguousarray(U0)), _ptr(Ut))
    return Ut


def exp_true_points(n: Sequence[int], U1, U0, pts) -> np.ndarray:
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.zeros(pts.size)
    lib().orc_exp_true_points(int(n[0]), int(n[1]), int(n[2]), _ptr(np.ascontiguousarray(U1)),
                              _ptr(np.ascontiguousarray(U0)), _ptr(pts), pts.size, _ptr(out))
    return out


def apply_rows(grid: Grid, beta, alpha, v, pts) -> np.ndarray:
    """(A v)_r at rows ``pts`` without assembling (0 on Dirichlet rows)."""
    pts = np.ascontiguousarray(pts, dtype=np.int64)
    out = np.zeros(pts.size)
    ap = (ctypes.c_void_p * 6)(*[_ptr(a) for a in alpha])
    lib().orc_apply_rows(ctypes.byref(grid.c()), _ptr(beta), ap, _ptr(np.ascontiguousarray(v)),
                         _ptr(pts), pts.size, _ptr(out))
    return out


def element_stiffness(h) -> np.ndarray:
    K = np.zeros(64)
    lib().orc_element_stiffness(float(h[0]), float(h[1]), float(h[2]), _ptr(K))
    return K.reshape(8, 8)


def face_mass(hp, hq) -> np.ndarray:
    M = np.zeros(16)
    lib().orc_face_mass(float(hp), float(hq), _ptr(M))
    return M.reshape(4, 4)


def serendipity_weight(node_abc, xi, eta, zeta) -> float:
    a, b, c = node_abc
    return float(lib().orc_serendipity_weight(int(a), int(b), int(c), float(xi), float(eta), float(zeta)))


# ---------------------------------------------------------------------------
# O11: norms of the tables (Section 5)
# ---------------------------------------------------------------------------

def norms(v: np.ndarray, grid: Grid) -> tuple:
    """(max norm, discrete L2 norm) over all nodes; the L2 norm of the tables is
    the root mean square (sum v^2 / N)^(1/2) (Section 5, Tables of Problem 1)."""
    return float(np.max(np.abs(v))), float(math.sqrt(float(np.dot(v, v)) / v.size))


def exact_nodes(problem: Problem, grid: Grid) -> np.ndarray:
    return tensor_eval(problem.u, grid.node_coords(0), grid.node_coords(1), grid.node_coords(2)).ravel()


# ---------------------------------------------------------------------------
# O9: the cascade (Algorithm 4)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class LevelResult:
    level: int
    n: tuple
    iters: int = 0
    rre: float = 0.0
    rre_true: float = 0.0
    u: Optional[np.ndarray] = None
    W: Optional[np.ndarray] = None
    Ut: Optional[np.ndarray] = None
    err: Dict[str, float] = dataclasses.field(default_factory=dict)


def cascade(problem: Problem, eps: Optional[float] = None, fixed_iters: Optional[Sequence[int]] = None,
            max_iter: int = 20000, keep_vectors: bool = True, errors: bool = True,
            levels: Optional[Sequence[Level]] = None, variant: int = SERENDIPITY20,
            method: int = JCG_METHOD) -> List[LevelResult]:
    """Algorithm 4: DSOLVE on levels 0 and 1, then for each finer level
    W = EXP_finite(u_{l-1}, u_{l-2}), JCG from W while ||A u - f|| > eps ||f||,
    and U~ = EXP_true(u_l, u_{l-1}).  ``fixed_iters[l]`` (l >= 2) replaces the
    stopping test with an exact iteration count.  ``method=CG_METHOD`` is
    ECMG_cg (Section 4.1); with ``fixed_iters=cascadic_schedule(...)`` it is the
    original ECMG of Algorithm 3.  ``eps`` may be a sequence, one relative
    tolerance per level (the per-level schedule Section 5 motivates)."""
    eps = problem.eps if eps is None else eps
    eps_at = (lambda l: float(eps[l])) if isinstance(eps, (list, tuple, np.ndarray)) else (lambda l: float(eps))
    Lt = problem.levels
    out: List[LevelResult] = []
    us: List[np.ndarray] = []
    for l in range(Lt):
        lv = levels[l] if levels is not None else discretize(problem, l)
        res = LevelResult(l, lv.grid.n)
        if l < 2:
            u = dsolve(lv)
        else:
            W = exp_finite(lv.grid, us[l - 1], us[l - 2], variant)
            x0 = np.where(lv.dmask == 1, lv.gD, W)      # JCG starts from W with g_D imposed
            fi = -1 if fixed_iters is None else int(fixed_iters[l])
            jr = jcg(lv, x0, eps_at(l), max_iter=max_iter, fixed_iters=fi, method=method)
            if jr.status == -4:
                raise RuntimeError("oracle JCG breakdown on level %d" % l)
            u = jr.x
            res.iters, res.rre, res.rre_true = jr.iters, jr.rre, jr.rre_true
            res.W = W
        us.append(u)
        if l >= 1:
            res.Ut = exp_true(lv.grid, u, us[l - 1])
        res.u = u
        if errors:
            ue = exact_nodes(problem, lv.grid)
            res.err["U_max"], res.err["U_l2"] = norms(u - ue, lv.grid)
            if res.Ut is not None:
                res.err["Ut_max"], res.err["Ut_l2"] = norms(res.Ut - ue, lv.grid)
            if res.W is not None:
                res.err["WU_max"], res.err["WU_l2"] = norms(res.W - u, lv.grid)
                res.err["r_h"] = res.err["WU_l2"] / res.err["U_l2"] if res.err["U_l2"] > 0 else float("nan")
        out.append(res)
        if not keep_vectors and l >= 2:
            out[l - 2].u = out[l - 2].W = out[l - 2].Ut = None
    return out
