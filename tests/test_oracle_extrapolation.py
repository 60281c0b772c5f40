"""Pins the oracle's EXP_finite and EXP_true (Sections 4.2-4.3) to the paper's
worked example and 1-D formulas, to polynomial reproduction, and to the
asymptotic-expansion argument the formulas are derived from (eq. asy)."""
import itertools

import numpy as np
import pytest

S20 = [(a, b, c) for c in (0, 2, 4) for b in (0, 2, 4) for a in (0, 2, 4)
       if (a == 2) + (b == 2) + (c == 2) <= 1]


def node_id(a, b, c):
    """The paper's 125-node numbering of a coarse element, x fastest."""
    return 1 + a + 5 * b + 25 * c


def test_node_numbering_matches_paper_lists():
    corners = sorted(node_id(a, b, c) for a, b, c in S20 if 2 not in (a, b, c))
    assert corners == [1, 5, 21, 25, 101, 105, 121, 125]
    assert sorted(node_id(2, b, c) for b in (0, 4) for c in (0, 4)) == [3, 23, 103, 123]
    assert sorted(node_id(a, 2, c) for a in (0, 4) for c in (0, 4)) == [11, 15, 111, 115]
    assert sorted(node_id(a, b, 2) for a in (0, 4) for b in (0, 4)) == [51, 55, 71, 75]


def test_w35_worked_example_weights(orc):
    """Section 4.3: W_35 = N(1,-1/2,-1/2) . W = 9/16 W15 - 3/16 W25 + 9/16 W55
    + 3/16 W75 - 3/16 W105 + 3/16 W115 - 1/8 W125."""
    want = {15: 9 / 16, 25: -3 / 16, 55: 9 / 16, 75: 3 / 16, 105: -3 / 16, 115: 3 / 16, 125: -1 / 8}
    assert node_id(4, 1, 1) == 35
    for m in S20:
        w = orc.serendipity_weight(m, 1.0, -0.5, -0.5)
        assert w == pytest.approx(want.get(node_id(*m), 0.0), abs=1e-15)


def test_partition_of_unity(orc):
    for a, b, c in itertools.product(range(5), repeat=3):
        s = sum(orc.serendipity_weight(m, a / 2 - 1, b / 2 - 1, c / 2 - 1) for m in S20)
        assert s == pytest.approx(1.0, abs=1e-14)


def _one_element(rng):
    """U1 on 3^3 nodes (level l-1 of one coarse element), U0 on 2^3 nodes."""
    return rng.standard_normal(27), rng.standard_normal(8)


def test_w35_worked_example_values(orc):
    rng = np.random.default_rng(3)
    U1, U0 = _one_element(rng)
    u1 = lambda a, b, c: U1[a // 2 + 3 * (b // 2) + 9 * (c // 2)]
    u0 = lambda a, b, c: U0[a // 4 + 2 * (b // 4) + 4 * (c // 4)]

    def W(a, b, c):  # eqs. jiedian and zhongdian typed from the paper
        if 2 not in (a, b, c):
            return (5 * u1(a, b, c) - u0(a, b, c)) / 4
        e = [(0, 4) if v == 2 else (v, v) for v in (a, b, c)]
        p0, p1 = (e[0][0], e[1][0], e[2][0]), (e[0][1], e[1][1], e[2][1])
        return u1(a, b, c) + (u1(*p0) - u0(*p0) + u1(*p1) - u0(*p1)) / 8

    w = {node_id(*m): W(*m) for m in S20}
    want = (9 / 16 * w[15] - 3 / 16 * w[25] + 9 / 16 * w[55] + 3 / 16 * w[75] - 3 / 16 * w[105]
            + 3 / 16 * w[115] - 1 / 8 * w[125])
    got = orc.exp_finite_points((4, 4, 4), U1, U0, [4 + 5 * (1 + 5 * 1)])[0]
    assert got == pytest.approx(want, rel=1e-14, abs=1e-14)
    for m in S20:  # the 20 nodes take the extrapolation formulas themselves
        r = m[0] + 5 * (m[1] + 5 * m[2])
        assert orc.exp_finite_points((4, 4, 4), U1, U0, [r])[0] == pytest.approx(W(*m), rel=1e-15, abs=1e-15)


def test_edge_quarter_points_reduce_to_sifen(orc):
    """On a coarse edge the interpolation reduces to the 1-D quarter-point
    formulas eqs. sifen1 and sifen2."""
    rng = np.random.default_rng(5)
    U1, U0 = _one_element(rng)
    # the edge b = c = 0 along x: U1 at a = 0, 2, 4 and U0 at a = 0, 4
    A0, Am, A1 = U1[0], U1[1], U1[2]
    B0, B1 = U0[0], U0[1]
    s1 = ((9 * A0 + 12 * Am - A1) - (3 * B0 + B1)) / 16
    s2 = ((9 * A1 + 12 * Am - A0) - (3 * B1 + B0)) / 16
    got = orc.exp_finite_points((4, 4, 4), U1, U0, [1, 3])
    assert got[0] == pytest.approx(s1, rel=1e-14, abs=1e-14)
    assert got[1] == pytest.approx(s2, rel=1e-14, abs=1e-14)


def _grid_samples(fn, n, h):
    x = np.arange(n[0] + 1) * h[0]
    y = np.arange(n[1] + 1) * h[1]
    z = np.arange(n[2] + 1) * h[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return fn(X, Y, Z).ravel()


SEREN_SPAN = [lambda x, y, z: 1 + 0 * x, lambda x, y, z: x * y * z, lambda x, y, z: x * x * y,
              lambda x, y, z: z * z * x * y, lambda x, y, z: y * y - 0.3 * x * z + x * x * z]
FULL_SPAN = SEREN_SPAN + [lambda x, y, z: x * x * y * y, lambda x, y, z: x * x * y * y * z * z]


@pytest.mark.parametrize("variant", [0, 1])
def test_polynomial_reproduction(orc, variant):
    """With U1 = U0 = q sampled (no extrapolation correction), W = q whenever q
    lies in the interpolation space: the serendipity span (variant 0) or the
    full tri-quadratic span (variant 1)."""
    nf = (8, 12, 8)
    h = (0.25, 0.1, 0.3)
    span = SEREN_SPAN if variant == 0 else FULL_SPAN
    for q in span:
        U1 = _grid_samples(q, tuple(n // 2 for n in nf), tuple(2 * v for v in h))
        U0 = _grid_samples(q, tuple(n // 4 for n in nf), tuple(4 * v for v in h))
        W = orc.exp_finite(orc.Grid(nf, (0, 0, 0), tuple(nf[d] * h[d] for d in range(3)), (0,) * 6), U1, U0, variant)
        assert np.allclose(W, _grid_samples(q, nf, h), atol=1e-12)
    if variant == 0:   # x^2 y^2 is outside the serendipity span
        q = FULL_SPAN[-2]
        U1 = _grid_samples(q, tuple(n // 2 for n in nf), tuple(2 * v for v in h))
        U0 = _grid_samples(q, tuple(n // 4 for n in nf), tuple(4 * v for v in h))
        W = orc.exp_finite(orc.Grid(nf, (0, 0, 0), tuple(nf[d] * h[d] for d in range(3)), (0,) * 6), U1, U0, 0)
        assert not np.allclose(W, _grid_samples(q, nf, h), atol=1e-8)


@pytest.mark.parametrize("variant", [0, 1])
def test_asymptotic_expansion_exactness(orc, variant):
    """eq. asy with no remainder: U^i = u + A h_i^2 (A trilinear).  EXP_finite
    then returns U^2 = u + A h_2^2 exactly where the interpolation reproduces
    u + A h_2^2 (c = 5/4 and the 1/8 of eq. zhongdian), and EXP_true returns u
    exactly (eqs. t1, chenlin)."""
    nf = (8, 8, 12)
    h2 = (0.125, 0.2, 0.1)
    u = lambda x, y, z: 1 + x * x * y - 2 * y * z * z + x * y * z
    A = lambda x, y, z: 3 - x + 2 * y * z + 0.5 * x * y * z
    H = lambda l: tuple(v * 2 ** (2 - l) for v in h2)
    U = [None] * 3
    s = [1.0, 0.25, 0.0625]          # h_i^2 / h_0^2 for the three levels
    for l in range(3):
        n = tuple(m // 2 ** (2 - l) for m in nf)
        U[l] = _grid_samples(lambda x, y, z: u(x, y, z) + A(x, y, z) * s[l], n, H(l))
    grid = orc.Grid(nf, (0, 0, 0), tuple(nf[d] * h2[d] for d in range(3)), (0,) * 6)
    W = orc.exp_finite(grid, U[1], U[0], variant)
    assert np.allclose(W, U[2], atol=1e-12)
    # EXP_true on level 2 from (U^2, U^1) and on level 1 from (U^1, U^0)
    Ut = orc.exp_true(grid, U[2], U[1])
    assert np.allclose(Ut, _grid_samples(u, nf, h2), atol=1e-12)


def test_exp_true_is_trilinear_correction(orc):
    """EXP_true = U1 + (1/3) T[U1 - U0], T = trilinear interpolation of the
    coarse-node differences (t1 at coarse nodes, chenlin at edge midpoints and
    its face/body diagonal means)."""
    rng = np.random.default_rng(11)
    nf = (6, 4, 8)
    U1 = rng.standard_normal((nf[2] + 1) * (nf[1] + 1) * (nf[0] + 1))
    U0 = rng.standard_normal((nf[2] // 2 + 1) * (nf[1] // 2 + 1) * (nf[0] // 2 + 1))
    grid = orc.Grid(nf, (0, 0, 0), (1, 1, 1), (0,) * 6)
    Ut = orc.exp_true(grid, U1, U0)
    u1 = U1.reshape(nf[2] + 1, nf[1] + 1, nf[0] + 1)
    u0 = U0.reshape(nf[2] // 2 + 1, nf[1] // 2 + 1, nf[0] // 2 + 1)
    d = u1[::2, ::2, ::2] - u0
    # trilinear prolongation of d by averaging along each axis
    T = np.zeros_like(u1)
    T[::2, ::2, ::2] = d
    T[::2, ::2, 1::2] = 0.5 * (T[::2, ::2, 0:-1:2] + T[::2, ::2, 2::2])
    T[::2, 1::2, :] = 0.5 * (T[::2, 0:-1:2, :] + T[::2, 2::2, :])
    T[1::2, :, :] = 0.5 * (T[0:-1:2, :, :] + T[2::2, :, :])
    assert np.allclose(Ut, (u1 + T / 3.0).ravel(), atol=1e-14)
