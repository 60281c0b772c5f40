"""Pins the oracle's Q1 discretisation (Section 2, eqs. var and fe_equation)
against textbook facts that do not come from the oracle's own quadrature:
closed forms, energies of linear functions, consistency with -Laplace on
quadratics, exactness for trilinear solutions, and integrals of polynomials."""
import itertools
import math

import numpy as np
import pytest

import workloads
from workloads import DIRICHLET, ROBIN


def _class_coeff(h, da, db, dc):
    """Closed-form Q1 stiffness entry / beta for local nodes differing on the
    axes marked 1 (tensor product of 1-D stiffness [[1,-1],[-1,1]]/h and 1-D
    mass h[[1/3,1/6],[1/6,1/3]])."""
    hx, hy, hz = h
    K1 = lambda d, hh: (1.0 if d == 0 else -1.0) / hh
    M1 = lambda d, hh: hh * (1.0 / 3.0 if d == 0 else 1.0 / 6.0)
    return (K1(da, hx) * M1(db, hy) * M1(dc, hz) + M1(da, hx) * K1(db, hy) * M1(dc, hz) +
            M1(da, hx) * M1(db, hy) * K1(dc, hz))


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (0.25, 0.5, 0.125), (0.3, 0.07, 1.9)])
def test_element_stiffness_closed_form(orc, h):
    K = orc.element_stiffness(h)
    for a, b in itertools.product(range(8), repeat=2):
        d = [((a >> s) & 1) ^ ((b >> s) & 1) for s in range(3)]
        assert K[a, b] == pytest.approx(_class_coeff(h, *d), rel=1e-13, abs=1e-15)
    assert np.allclose(K, K.T, atol=1e-15)
    assert np.allclose(K.sum(axis=1), 0.0, atol=1e-13)
    ev = np.linalg.eigvalsh(K)
    assert abs(ev[0]) < 1e-12 and ev[1] > 1e-6      # only constants in the kernel
    # energy of a linear function u = c.x is |c|^2 |e|
    c = np.array([0.7, -1.3, 2.1])
    xs = np.array([[(a & 1) * h[0], ((a >> 1) & 1) * h[1], ((a >> 2) & 1) * h[2]] for a in range(8)])
    u = xs @ c
    assert u @ K @ u == pytest.approx(float(c @ c) * h[0] * h[1] * h[2], rel=1e-12)


def test_face_mass(orc):
    hp, hq = 0.3, 0.7
    M = orc.face_mass(hp, hq)
    assert M.sum() == pytest.approx(hp * hq, rel=1e-14)
    # int of u^2 for u = 1 + 2p - q (bilinear interpolant is exact for linear u)
    pts = [((a & 1) * hp, ((a >> 1) & 1) * hq) for a in range(4)]
    u = np.array([1 + 2 * p - q for p, q in pts])
    exact = 0.0
    # int_0^hp int_0^hq (1+2p-q)^2 dq dp, expanded by hand
    A, B = hp, hq
    exact = (A * B + 4 * A ** 3 * B / 3 + A * B ** 3 / 3 + 2 * A ** 2 * B - A * B ** 2 - A ** 2 * B ** 2)
    assert u @ M @ u == pytest.approx(exact, rel=1e-13)
    assert M[0, 0] == pytest.approx(hp * hq / 9, rel=1e-14)
    assert M[0, 1] == pytest.approx(hp * hq / 18, rel=1e-14)
    assert M[0, 3] == pytest.approx(hp * hq / 36, rel=1e-14)


def _robin_cube(n, h, beta=1.0, faces=(ROBIN,) * 6, alpha=0.0):
    p = workloads.paper_problem1(levels=1)
    return p.with_(n0=n, lo=(0, 0, 0), hi=tuple(n[d] * h[d] for d in range(3)), face_type=faces,
                   beta=workloads._const(beta), alpha=workloads._const(alpha))


def test_stencil_textbook_values(orc):
    """beta = 1, cubic h: centre 8h/3, face neighbours 0, edge neighbours -h/6,
    corners -h/12 (interior row)."""
    h = 0.25
    lv = orc.discretize(_robin_cube((4, 4, 4), (h, h, h)), 0)
    g = lv.grid
    r = 2 + 5 * (2 + 5 * 2)
    cols = lv.col[lv.rowptr[r]:lv.rowptr[r + 1]]
    vals = lv.val[lv.rowptr[r]:lv.rowptr[r + 1]]
    for c, v in zip(cols, vals):
        i, j, k = c % 5 - 2, (c // 5) % 5 - 2, c // 25 - 2
        nz = abs(i) + abs(j) + abs(k)
        want = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}[nz]
        assert v == pytest.approx(want, abs=1e-15)
    assert len(cols) == 27


@pytest.mark.parametrize("q", ["x2", "y2z", "xyz", "z2x", "xy"])
def test_stencil_consistency_on_quadratics(orc, q):
    """Interior rows of A (beta = 1) applied to nodal samples of q equal
    -Laplace q times the cell volume when q has degree <= 2 in one axis and <= 1
    in the others (the Q1 stencil is exact there)."""
    h = (0.2, 0.25, 0.125)
    lv = orc.discretize(_robin_cube((5, 4, 8), h), 0)
    g = lv.grid
    X, Y, Z = np.meshgrid(g.node_coords(0), g.node_coords(1), g.node_coords(2), indexing="ij")
    # (q, Laplace q)
    fn = {"x2": (X ** 2, 2.0 + 0 * X), "y2z": (Y ** 2 * Z, 2.0 * Z), "xyz": (X * Y * Z, 0 * X),
          "z2x": (Z ** 2 * X, 2.0 * X), "xy": (X * Y, 0 * X)}[q]
    v = fn[0].transpose(2, 1, 0).ravel()
    lap = fn[1].transpose(2, 1, 0).ravel()
    Av = np.zeros_like(v)
    for r in range(v.size):
        s, e = lv.rowptr[r], lv.rowptr[r + 1]
        Av[r] = lv.val[s:e] @ v[lv.col[s:e]]
    vol = h[0] * h[1] * h[2]
    interior = [(i + 6 * (j + 5 * k)) for i in range(1, 5) for j in range(1, 4) for k in range(1, 8)]
    assert np.allclose(Av[interior], -lap[interior] * vol, atol=1e-13)


def test_load_vector_integrals(orc):
    """F_i = int f phi_i: for f = 1 the interior entries are the cell volume, for
    linear f they are f(x_i) times the volume, and sum_i F_i = int f for any
    f that 2-point Gauss integrates exactly (degree <= 3 per axis)."""
    h = (0.2, 0.25, 0.125)
    base = _robin_cube((5, 4, 8), h, faces=(DIRICHLET,) * 6)     # no Robin load terms
    vol = h[0] * h[1] * h[2]
    for name, f, integral in (
        ("one", lambda x, y, z, face=-1: 1.0 + 0 * x * y * z, 1.0 * 1.0 * 1.0),
        ("lin", lambda x, y, z, face=-1: 1.0 + 2 * x - y + 3 * z + 0 * x * y * z, None),
        ("cubic", lambda x, y, z, face=-1: x ** 3 * y ** 2 * z + 0 * x, (1 / 4) * (1 / 3) * (1 / 2)),
    ):
        p = base.with_(f=f)
        g = orc.grid_of(p, 0)
        F = orc.load_vector(p, g)
        if integral is not None:
            assert F.sum() == pytest.approx(integral, rel=1e-13)
        X, Y, Z = np.meshgrid(g.node_coords(0), g.node_coords(1), g.node_coords(2), indexing="ij")
        fv = f(X, Y, Z).transpose(2, 1, 0).ravel()
        interior = [(i + 6 * (j + 5 * k)) for i in range(1, 5) for j in range(1, 4) for k in range(1, 8)]
        if name in ("one", "lin"):
            assert np.allclose(F[interior], fv[interior] * vol, rtol=1e-13)


def test_robin_load_integral(orc):
    """sum_i (Robin part of F_i) = int over the Robin faces of g_R."""
    base = _robin_cube((3, 4, 2), (1 / 3, 1 / 4, 1 / 2))
    p = base.with_(f=workloads._const(0.0), face_type=(DIRICHLET, ROBIN, DIRICHLET, DIRICHLET, DIRICHLET, ROBIN))
    # g_R = alpha u + beta du/dn with u = x y^2 z, alpha = 0, beta = 1
    p = p.with_(u=lambda x, y, z, face=-1: x * y * y * z, grad_u=lambda x, y, z: (y * y * z, 2 * x * y * z, x * y * y))
    g = orc.grid_of(p, 0)
    F = orc.load_vector(p, g)
    # x = 1 face: du/dx = y^2 z over [0,1]^2 -> 1/6 ; z = 1 face: du/dz = x y^2 -> 1/6
    assert F.sum() == pytest.approx(1 / 6 + 1 / 6, rel=1e-13)


@pytest.mark.parametrize("faces", [(DIRICHLET,) * 6, (DIRICHLET, ROBIN, ROBIN, DIRICHLET, ROBIN, ROBIN),
                                   (ROBIN, ROBIN, ROBIN, ROBIN, ROBIN, DIRICHLET)])
def test_trilinear_solution_reproduced(orc, faces):
    """A trilinear u lies in the Q1 space, so with constant beta (f = 0) and
    exact Robin data the discrete solution equals u at every node."""
    beta, alpha = 2.5, 1.7
    u = lambda x, y, z, face=-1: 1.0 + 0.5 * x - y + 2 * z + x * y - 0.7 * y * z + 1.3 * x * y * z
    gu = lambda x, y, z: (0.5 + y + 1.3 * y * z, -1.0 + x - 0.7 * z + 1.3 * x * z, 2.0 - 0.7 * y + 1.3 * x * y)
    p = workloads.paper_problem1(levels=2).with_(
        n0=(3, 2, 4), lo=(0.1, -0.3, 0.0), hi=(1.0, 0.5, 0.6), face_type=faces, u=u, grad_u=gu,
        beta=workloads._const(beta), alpha=workloads._const(alpha), f=workloads._const(0.0))
    for level in (0, 1):
        lv = orc.discretize(p, level)
        x = orc.dsolve(lv)
        ue = orc.exact_nodes(p, lv.grid)
        assert np.abs(x - ue).max() < 1e-12


# ---------------------------------------------------------------------------
# Variable coefficients: beta per element at its centroid, alpha per Robin
# face element at its centroid (the reading of the bilinear form of Section 2
# for coefficients that vary; every problem of Section 5 has beta = 1)
# ---------------------------------------------------------------------------

def _indicator(c, r):
    """A field that is 1 within half-widths r of the point c and 0 elsewhere."""
    def fn(x, y, z, face=-1):
        inside = (np.abs(x - c[0]) < r[0]) & (np.abs(y - c[1]) < r[1]) & (np.abs(z - c[2]) < r[2])
        return np.where(inside, 1.0, 0.0) + 0.0 * x * y * z
    return fn


def _node(n, i, j, k):
    return i + (n[0] + 1) * (j + (n[1] + 1) * k)


@pytest.mark.parametrize("e", [(0, 0, 0), (2, 3, 1), (1, 0, 1), (2, 1, 0)])
def test_beta_of_one_element_lands_on_its_nodes(orc, e):
    """A beta that is 1 around one element's centroid and 0 elsewhere gives a
    matrix that is that element's Q1 stiffness (the closed-form tensor product,
    not the oracle's quadrature) on its 8 nodes and zero everywhere else: beta is
    sampled at that centroid and multiplies that element's matrix only."""
    n, h = (3, 4, 2), (0.3, 0.25, 0.5)
    c = [(e[d] + 0.5) * h[d] for d in range(3)]
    p = _robin_cube(n, h).with_(beta=_indicator(c, [0.25 * hh for hh in h]))
    A = orc.discretize(p, 0).dense()
    want = np.zeros_like(A)
    for a, b in itertools.product(range(8), repeat=2):
        na = _node(n, e[0] + (a & 1), e[1] + ((a >> 1) & 1), e[2] + ((a >> 2) & 1))
        nb = _node(n, e[0] + (b & 1), e[1] + ((b >> 1) & 1), e[2] + ((b >> 2) & 1))
        d = [((a >> s) & 1) ^ ((b >> s) & 1) for s in range(3)]
        want[na, nb] = _class_coeff(h, *d)
    assert np.abs(A - want).max() <= 1e-14


@pytest.mark.parametrize("face, fe", [(0, (1, 0)), (1, (3, 1)), (3, (2, 1)), (4, (0, 3)), (5, (2, 2))])
def test_alpha_of_one_face_element_lands_on_its_nodes(orc, face, fe):
    """With beta = 0 and an alpha that is 1 around one Robin face element's
    centroid, the matrix is that face element's mass, alpha hp hq (1/9, 1/18,
    1/36) by the number of in-face axes on which two nodes differ, on its 4
    nodes, and zero elsewhere."""
    n, h = (3, 4, 2), (0.3, 0.25, 0.5)
    ax = face // 2
    pa, qa = [d for d in range(3) if d != ax]
    plane = 0.0 if face % 2 == 0 else n[ax] * h[ax]
    c = [0.0] * 3
    c[ax] = plane
    c[pa] = (fe[0] + 0.5) * h[pa]
    c[qa] = (fe[1] + 0.5) * h[qa]
    if fe[0] >= n[pa] or fe[1] >= n[qa]:
        pytest.skip("face element outside this face")
    r = [0.25 * hh for hh in h]
    p = _robin_cube(n, h, beta=0.0).with_(alpha=_indicator(c, r))
    A = orc.discretize(p, 0).dense()
    want = np.zeros_like(A)
    hp, hq = h[pa], h[qa]
    cls = (hp * hq / 9.0, hp * hq / 18.0, hp * hq / 36.0)
    k_face = 0 if face % 2 == 0 else n[ax]
    for a, b in itertools.product(range(4), repeat=2):
        def idx(m):
            ijk = [0, 0, 0]
            ijk[ax] = k_face
            ijk[pa] = fe[0] + (m & 1)
            ijk[qa] = fe[1] + ((m >> 1) & 1)
            return _node(n, *ijk)
        want[idx(a), idx(b)] = cls[bin(a ^ b).count("1")]
    assert np.abs(A - want).max() <= 1e-15


@pytest.mark.parametrize("mask", range(64))
def test_apply_rows_equals_assembled_rows(orc, mask):
    """The oracle's row-wise operator (used to check single rows at sizes where
    nothing is assembled) equals the assembled CSR matrix on every row, for every
    combination of Dirichlet and Robin faces, with variable beta and alpha."""
    faces = tuple(ROBIN if (mask >> f) & 1 else DIRICHLET for f in range(6))
    p = workloads.variable_beta_robin_cube(levels=1).with_(
        n0=(3, 4, 2), hi=(0.9, 1.0, 0.5), face_type=faces,
        alpha=lambda x, y, z, face=-1: 1.0 + 0.5 * x * x + 0.25 * y - 0.1 * z + 0.0 * x)
    lv = orc.discretize(p, 0)
    v = workloads.random_vector(lv.grid.num_nodes, seed=mask)
    full = orc.spmv(lv, v)
    rows = np.arange(lv.grid.num_nodes)
    got = orc.apply_rows(lv.grid, lv.beta, lv.alpha, v, rows)
    assert np.abs(got - full).max() <= 1e-14 * max(np.abs(full).max(), 1.0), mask
