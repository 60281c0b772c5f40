"""Seeded synthetic inputs: manufactured boundary value problems of the form
-div(beta grad u) = f on a box, u = g_D on Dirichlet faces and
alpha u + beta du/dn = g_R on Robin faces (Section 1, eq. bvp).

This module holds only problem definitions (closed-form fields, box, grid
hierarchy, face types, tolerance) and the seeded generators for the batched and
serving mixes.  It holds none of the solver's arithmetic and is the only code
shared by the CPU oracle and the GPU library's tests and benchmark.

Every field is a function ``fn(x, y, z, face)`` evaluated with broadcasting on
numpy arrays or, unchanged, on torch tensors (any device); ``face`` is -1 for volume points and 0..5 (x-lo, x-hi, y-lo,
y-hi, z-lo, z-hi) when all points lie on that face, which Robin data needs for
the outward normal.  ``tensor_eval`` turns such a function into the
tensor-product sampling convention of the C interfaces: ``out[k, j, i] =
fn(x[i], y[j], z[k])``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

DIRICHLET = 0
ROBIN = 1  # Neumann is Robin with alpha == 0 (Section 1)

FACE_NAMES = ("x-lo", "x-hi", "y-lo", "y-hi", "z-lo", "z-hi")
# outward unit normal of each face: (axis, sign)
FACE_NORMAL = ((0, -1.0), (0, 1.0), (1, -1.0), (1, 1.0), (2, -1.0), (2, 1.0))

Field = Callable[[np.ndarray, np.ndarray, np.ndarray, int], np.ndarray]


def _xp(*arrays):
    """The array module of the inputs: numpy, or torch for torch tensors (fields
    are then evaluated on whatever device the tensors live on)."""
    for a in arrays:
        if type(a).__module__.startswith("torch"):
            import torch
            return torch
    return np


def _const(c: float) -> Field:
    def fn(x, y, z, face=-1):
        return 0.0 * x + 0.0 * y + 0.0 * z + float(c)
    fn.constant = float(c)  # type: ignore[attr-defined]
    return fn


@dataclasses.dataclass
class Problem:
    """A manufactured problem on a box with a uniform grid hierarchy.

    Level l has n0[d] * 2**l elements on axis d; ``levels`` counts every grid,
    including the two coarsest ones that are solved directly (Algorithm 4).
    """
    name: str
    lo: Sequence[float]
    hi: Sequence[float]
    n0: Sequence[int]
    levels: int
    face_type: Sequence[int]
    beta: Field
    f: Field
    u: Field                       # exact solution (also used as g_D)
    grad_u: Callable               # returns (ux, uy, uz)
    alpha: Field = dataclasses.field(default_factory=lambda: _const(0.0))
    eps: float = 1e-8
    grad_beta: Optional[Callable] = None

    # ---- boundary data derived from u -------------------------------------
    def gD(self, x, y, z, face=-1):
        return self.u(x, y, z, face)

    def gR(self, x, y, z, face):
        """alpha u + beta (grad u . n) on Robin face ``face`` (outward normal)."""
        axis, sign = FACE_NORMAL[face]
        g = self.grad_u(x, y, z)[axis]
        return self.alpha(x, y, z, face) * self.u(x, y, z, face) + self.beta(x, y, z, face) * sign * g

    def n_at(self, level: int):
        return tuple(int(n) * (1 << level) for n in self.n0)

    def nodes_at(self, level: int) -> int:
        nx, ny, nz = self.n_at(level)
        return (nx + 1) * (ny + 1) * (nz + 1)

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def tensor_eval(fn: Field, x, y, z, face: int = -1) -> np.ndarray:
    """Evaluate ``fn`` on the tensor product x (fastest) by y by z (slowest)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    out = fn(x[None, None, :], y[None, :, None], z[:, None, None], face)
    out = np.broadcast_to(out, (z.size, y.size, x.size))
    return np.ascontiguousarray(out, dtype=np.float64)


# ---------------------------------------------------------------------------
# The paper's three test problems (Section 5)
# ---------------------------------------------------------------------------

def paper_problem1(levels: int = 3, eps: float = 1e-9) -> Problem:
    """Problem 1: -Laplace u = (3/4) pi^2 u on the unit cube,
    u = sin(pi x/2) sin(pi y/2) sin(pi z/2); u = 0 on x=0, y=0, z=0 and zero
    normal derivative on x=1, y=1, z=1; coarsest grid 8^3 (Section 5, eq. prob1)."""
    h = 0.5 * math.pi

    def u(x, y, z, face=-1):
        xp = _xp(x, y, z)
        return xp.sin(h * x) * xp.sin(h * y) * xp.sin(h * z)

    def grad_u(x, y, z):
        xp = _xp(x, y, z)
        sx, sy, sz = xp.sin(h * x), xp.sin(h * y), xp.sin(h * z)
        cx, cy, cz = xp.cos(h * x), xp.cos(h * y), xp.cos(h * z)
        return (h * cx * sy * sz, h * sx * cy * sz, h * sx * sy * cz)

    def f(x, y, z, face=-1):
        return 0.75 * math.pi ** 2 * u(x, y, z)

    return Problem("paper-problem-1", (0, 0, 0), (1, 1, 1), (8, 8, 8), levels,
                   (DIRICHLET, ROBIN, DIRICHLET, ROBIN, DIRICHLET, ROBIN),
                   beta=_const(1.0), f=f, u=u, grad_u=grad_u, alpha=_const(0.0), eps=eps)


def paper_problem2(levels: int = 3, eps: float = 1e-12) -> Problem:
    """Problem 2: u = exp(z) sin(3 pi x/2) sin(pi y/2) on the unit cube, Dirichlet
    on x=0, y=0, z=0, z=1 and zero normal derivative on x=1, y=1; coarsest grid
    10 x 4 x 5 (Section 5, eq. prob2)."""
    a, b = 1.5 * math.pi, 0.5 * math.pi

    def u(x, y, z, face=-1):
        xp = _xp(x, y, z)
        return xp.exp(z) * xp.sin(a * x) * xp.sin(b * y)

    def grad_u(x, y, z):
        xp = _xp(x, y, z)
        e = xp.exp(z)
        return (e * a * xp.cos(a * x) * xp.sin(b * y), e * b * xp.sin(a * x) * xp.cos(b * y),
                e * xp.sin(a * x) * xp.sin(b * y))

    def f(x, y, z, face=-1):
        return (2.5 * math.pi ** 2 - 1.0) * u(x, y, z)

    return Problem("paper-problem-2", (0, 0, 0), (1, 1, 1), (10, 4, 5), levels,
                   (DIRICHLET, ROBIN, DIRICHLET, ROBIN, DIRICHLET, DIRICHLET),
                   beta=_const(1.0), f=f, u=u, grad_u=grad_u, alpha=_const(0.0), eps=eps)


def paper_problem3(levels: int = 3, eps: float = 1e-11) -> Problem:
    """Problem 3: singular u = xyz / (x^2+y^2+z^2)^(3/4), Dirichlet on every face,
    coarsest grid 8^3 (Section 5, eq. prob3)."""

    def r2(x, y, z):
        return x * x + y * y + z * z

    def u(x, y, z, face=-1):
        xp = _xp(x, y, z)
        s = r2(x, y, z)
        ss = xp.where(s > 0, s, 1.0)
        return xp.where(s > 0, x * y * z / ss ** 0.75, 0.0)

    def grad_u(x, y, z):
        xp = _xp(x, y, z)
        s = r2(x, y, z)
        ss = xp.where(s > 0, s, 1.0)
        p = ss ** -0.75
        q = -1.5 * x * y * z * ss ** -1.75
        return (xp.where(s > 0, y * z * p + q * x, 0.0), xp.where(s > 0, x * z * p + q * y, 0.0),
                xp.where(s > 0, x * y * p + q * z, 0.0))

    def f(x, y, z, face=-1):
        xp = _xp(x, y, z)
        s = r2(x, y, z)
        ss = xp.where(s > 0, s, 1.0)
        return xp.where(s > 0, 33.0 * x * y * z / (4.0 * ss ** 1.75), 0.0)

    return Problem("paper-problem-3", (0, 0, 0), (1, 1, 1), (8, 8, 8), levels,
                   (DIRICHLET,) * 6, beta=_const(1.0), f=f, u=u, grad_u=grad_u, eps=eps)


# ---------------------------------------------------------------------------
# The benchmark workloads (variable beta, Robin faces, non-cubic boxes)
# ---------------------------------------------------------------------------

def smooth_dirichlet_cube(levels: int = 4, eps: float = 1e-10) -> Problem:
    """beta = 1, u = exp(x+y+z), Dirichlet on all faces, coarsest 4^3 elements;
    4 levels end at 32^3 elements (35,937 nodes)."""

    def u(x, y, z, face=-1):
        xp = _xp(x, y, z)
        return xp.exp(x + y + z)

    def grad_u(x, y, z):
        xp = _xp(x, y, z)
        e = xp.exp(x + y + z)
        return (e, e, e)

    def f(x, y, z, face=-1):
        xp = _xp(x, y, z)
        return -3.0 * xp.exp(x + y + z)

    return Problem("smooth-dirichlet-cube-4^3", (0, 0, 0), (1, 1, 1), (4, 4, 4), levels,
                   (DIRICHLET,) * 6, beta=_const(1.0), f=f, u=u, grad_u=grad_u, eps=eps)


def variable_beta_robin_cube(levels: int = 7, eps: float = 1e-8) -> Problem:
    """beta = 1 + 0.5 S with S = sin(pi x) sin(pi y) sin(pi z), u = S + xyz on the
    unit cube; Dirichlet on x=0 and x=1, Robin (alpha = 1) on the y and z faces;
    coarsest 8^3 elements, 7 levels end at 512^3 elements (513^3 nodes)."""
    pi = math.pi

    def S(x, y, z):
        xp = _xp(x, y, z)
        return xp.sin(pi * x) * xp.sin(pi * y) * xp.sin(pi * z)

    def gradS(x, y, z):
        xp = _xp(x, y, z)
        sx, sy, sz = xp.sin(pi * x), xp.sin(pi * y), xp.sin(pi * z)
        cx, cy, cz = xp.cos(pi * x), xp.cos(pi * y), xp.cos(pi * z)
        return (pi * cx * sy * sz, pi * sx * cy * sz, pi * sx * sy * cz)

    def beta(x, y, z, face=-1):
        return 1.0 + 0.5 * S(x, y, z)

    def u(x, y, z, face=-1):
        return S(x, y, z) + x * y * z

    def grad_u(x, y, z):
        gx, gy, gz = gradS(x, y, z)
        return (gx + y * z, gy + x * z, gz + x * y)

    def f(x, y, z, face=-1):
        s = S(x, y, z)
        gx, gy, gz = gradS(x, y, z)
        ux, uy, uz = gx + y * z, gy + x * z, gz + x * y
        # -div(beta grad u) = -beta Lap u - grad beta . grad u, Lap u = -3 pi^2 S
        return 3.0 * pi * pi * s * (1.0 + 0.5 * s) - 0.5 * (gx * ux + gy * uy + gz * uz)

    return Problem("variable-beta-robin-cube-8^3", (0, 0, 0), (1, 1, 1), (8, 8, 8), levels,
                   (DIRICHLET, DIRICHLET, ROBIN, ROBIN, ROBIN, ROBIN),
                   beta=beta, f=f, u=u, grad_u=grad_u, alpha=_const(1.0), eps=eps)


def high_contrast_singular_box(levels: int = 6, eps: float = 1e-8) -> Problem:
    """Box [0,2]x[0,1]x[0,1], coarsest 16x8x8 elements (6 levels end at
    512x256x256); beta = exp(4 sin(2 pi x) cos(2 pi y)) in [e^-4, e^4];
    u = (x^2+y^2+z^2)^(1/3), singular at the corner node (Dirichlet everywhere)."""
    tp = 2.0 * math.pi

    def beta(x, y, z, face=-1):
        xp = _xp(x, y, z)
        return xp.exp(4.0 * xp.sin(tp * x) * xp.cos(tp * y)) + 0.0 * z

    def grad_beta(x, y, z):
        xp = _xp(x, y, z)
        b = beta(x, y, z)
        return (4.0 * tp * b * xp.cos(tp * x) * xp.cos(tp * y),
                -4.0 * tp * b * xp.sin(tp * x) * xp.sin(tp * y), 0.0 * b)

    def u(x, y, z, face=-1):
        return (x * x + y * y + z * z) ** (1.0 / 3.0)

    def grad_u(x, y, z):
        xp = _xp(x, y, z)
        s = x * x + y * y + z * z
        c = xp.where(s > 0, (2.0 / 3.0) / xp.where(s > 0, s, 1.0) ** (2.0 / 3.0), 0.0)
        return (c * x, c * y, c * z)

    def f(x, y, z, face=-1):
        xp = _xp(x, y, z)
        s = x * x + y * y + z * z
        ss = xp.where(s > 0, s, 1.0)
        m = xp.where(s > 0, ss ** (-2.0 / 3.0), 0.0)  # r^(-4/3)
        bx, by, bz = grad_beta(x, y, z)
        return -(10.0 / 9.0) * beta(x, y, z) * m - (2.0 / 3.0) * m * (x * bx + y * by + z * bz)

    return Problem("high-contrast-singular-box-16x8x8", (0, 0, 0), (2, 1, 1), (16, 8, 8), levels,
                   (DIRICHLET,) * 6, beta=beta, f=f, u=u, grad_u=grad_u, eps=eps,
                   grad_beta=grad_beta)


# ---------------------------------------------------------------------------
# Seeded mixes: many uneven boxes, and a request stream
# ---------------------------------------------------------------------------

def batched_box(side, n_fine, phi, a, eps: float = 1e-8) -> Problem:
    """One box of the batched mix: [0,side]^3 (per axis), Dirichlet everywhere,
    beta = 1 + 0.5 sin(2 pi (x+phi1)) sin(2 pi (y+phi2)), u = exp(a.x); three
    levels whose finest grid has ``n_fine`` elements per axis."""
    tp = 2.0 * math.pi
    p1, p2 = float(phi[0]), float(phi[1])
    a = tuple(float(v) for v in a)
    a2 = a[0] ** 2 + a[1] ** 2 + a[2] ** 2

    def beta(x, y, z, face=-1):
        xp = _xp(x, y, z)
        return 1.0 + 0.5 * xp.sin(tp * (x + p1)) * xp.sin(tp * (y + p2)) + 0.0 * z

    def u(x, y, z, face=-1):
        xp = _xp(x, y, z)
        return xp.exp(a[0] * x + a[1] * y + a[2] * z)

    def grad_u(x, y, z):
        e = u(x, y, z)
        return (a[0] * e, a[1] * e, a[2] * e)

    def f(x, y, z, face=-1):
        xp = _xp(x, y, z)
        e = u(x, y, z)
        bx = 0.5 * tp * xp.cos(tp * (x + p1)) * xp.sin(tp * (y + p2))
        by = 0.5 * tp * xp.sin(tp * (x + p1)) * xp.cos(tp * (y + p2))
        return -e * (beta(x, y, z) * a2 + a[0] * bx + a[1] * by)

    n0 = tuple(int(n) // 4 for n in n_fine)
    return Problem("batched-box", (0, 0, 0), tuple(float(s) for s in side), n0, 3,
                   (DIRICHLET,) * 6, beta=beta, f=f, u=u, grad_u=grad_u, eps=eps)


def batched_mix(n_boxes: int = 512, seed: int = 0, eps: float = 1e-8) -> List[Problem]:
    """512 independent three-level solves with uneven shapes: box sides U(0.5, 2)
    per axis, finest elements per axis drawn from {16, 24, 32, 48, 64}."""
    rng = np.random.default_rng(seed)
    choices = np.array([16, 24, 32, 48, 64])
    out = []
    for _ in range(n_boxes):
        side = rng.uniform(0.5, 2.0, size=3)
        n_fine = rng.choice(choices, size=3)
        phi = rng.uniform(0.0, 1.0, size=2)
        a = rng.uniform(-1.0, 1.0, size=3)
        out.append(batched_box(side, n_fine, phi, a, eps))
    return out


def serving_request(n_fine: int, phi, k, faces, eps: float = 1e-8) -> Problem:
    """One request of the serving mix: unit cube, coarsest 8^3, finest
    ``n_fine``^3; beta = 1.25 + 0.75 sin 2pi(x+phi1) sin 2pi(y+phi2) sin 2pi(z+phi3)
    in [0.5, 2]; u = sin(k.x); each face Dirichlet or Robin with alpha = 1."""
    tp = 2.0 * math.pi
    p = [float(v) for v in phi]
    k = [float(v) for v in k]

    def sb(x, y, z):
        xp = _xp(x, y, z)
        return (xp.sin(tp * (x + p[0])), xp.sin(tp * (y + p[1])), xp.sin(tp * (z + p[2])),
                xp.cos(tp * (x + p[0])), xp.cos(tp * (y + p[1])), xp.cos(tp * (z + p[2])))

    def beta(x, y, z, face=-1):
        s1, s2, s3, _, _, _ = sb(x, y, z)
        return 1.25 + 0.75 * s1 * s2 * s3

    def grad_beta(x, y, z):
        s1, s2, s3, c1, c2, c3 = sb(x, y, z)
        return (0.75 * tp * c1 * s2 * s3, 0.75 * tp * s1 * c2 * s3, 0.75 * tp * s1 * s2 * c3)

    def u(x, y, z, face=-1):
        xp = _xp(x, y, z)
        return xp.sin(k[0] * x + k[1] * y + k[2] * z)

    def grad_u(x, y, z):
        xp = _xp(x, y, z)
        c = xp.cos(k[0] * x + k[1] * y + k[2] * z)
        return (k[0] * c, k[1] * c, k[2] * c)

    def f(x, y, z, face=-1):
        xp = _xp(x, y, z)
        ph = k[0] * x + k[1] * y + k[2] * z
        s, c = xp.sin(ph), xp.cos(ph)
        bx, by, bz = grad_beta(x, y, z)
        kk = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
        return beta(x, y, z) * kk * s - c * (k[0] * bx + k[1] * by + k[2] * bz)

    levels = int(round(math.log2(n_fine // 8))) + 1
    return Problem("serving-request", (0, 0, 0), (1, 1, 1), (8, 8, 8), levels,
                   tuple(int(t) for t in faces), beta=beta, f=f, u=u, grad_u=grad_u,
                   alpha=_const(1.0), eps=eps, grad_beta=grad_beta)


@dataclasses.dataclass
class Request:
    arrival_s: float
    problem: Problem


def serving_stream(n_requests: int = 2100, rate_per_s: float = 50.0, seed: int = 1,
                   eps: float = 1e-8) -> List[Request]:
    """Poisson arrivals at ``rate_per_s``; finest grid per request drawn from
    {32, 64, 128, 256}^3 with weights 0.4/0.3/0.2/0.1."""
    rng = np.random.default_rng(seed)
    sizes = np.array([32, 64, 128, 256])
    w = np.array([0.4, 0.3, 0.2, 0.1])
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        n = int(rng.choice(sizes, p=w))
        phi = rng.uniform(0.0, 1.0, size=3)
        k = rng.uniform(1.0, 3.0, size=3)
        faces = rng.integers(0, 2, size=6)
        out.append(Request(t, serving_request(n, phi, k, faces, eps)))
    return out


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal vector (parity inputs for single operators)."""
    return np.random.default_rng(seed).standard_normal(n)
