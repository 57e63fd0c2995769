"""Pins of the oracle's D, M and weighted-gap values.

Exact references are computed independently with rational arithmetic: on
axis-aligned rectangular elements the bilinear shape functions are products
of 1-D hat functions, so every mortar integral is a product of two 1-D
integrals of polynomials over intervals.
"""

from fractions import Fraction as F

import numpy as np
import pytest

import oracle
import synth


def hat(nodes, k, x_lo_hi):
    """1-D linear hat on [a, b] (nodes (a, b)); k=0 -> (b-x)/(b-a), k=1 -> (x-a)/(b-a).
    Returned as polynomial coefficients (c0, c1)."""
    a, b = nodes
    if k == 0:
        return (b / (b - a), F(-1) / (b - a))
    return (-a / (b - a), F(1) / (b - a))


def integ(p, q, lo, hi, extra=None):
    """exact integral over [lo, hi] of p(x) q(x) [extra(x)] for linear polys."""
    c = [p[0] * q[0], p[0] * q[1] + p[1] * q[0], p[1] * q[1]]
    if extra is not None:
        c = [c[0] * extra[0], c[0] * extra[1] + c[1] * extra[0], c[1] * extra[1] + c[2] * extra[0],
             c[2] * extra[1]]
    return sum(ci * (hi ** (i + 1) - lo ** (i + 1)) / (i + 1) for i, ci in enumerate(c))


# quad4 node k -> (ix, iy) corner flags, nodes CCW from (-1,-1)
CORNER = [(0, 0), (1, 0), (1, 1), (0, 1)]


def rect_pair_exact(sx, sy, mx, my, gap_line=None):
    """Exact D (4x4), M (4x4), g (4) for slave rectangle sx x sy and master
    rectangle mx x my (intervals as Fractions), standard basis.  gap_line =
    (c0, c1): master height c0 + c1 x above the flat slave."""
    lox, hix = max(sx[0], mx[0]), min(sx[1], mx[1])
    loy, hiy = max(sy[0], my[0]), min(sy[1], my[1])
    D = np.zeros((4, 4), dtype=object)
    M = np.zeros((4, 4), dtype=object)
    g = np.zeros(4, dtype=object)
    for j in range(4):
        pjx, pjy = hat(sx, CORNER[j][0], None), hat(sy, CORNER[j][1], None)
        for k in range(4):
            pkx, pky = hat(sx, CORNER[k][0], None), hat(sy, CORNER[k][1], None)
            D[j, k] = integ(pjx, pkx, lox, hix) * integ(pjy, pky, loy, hiy)
            qkx, qky = hat(mx, CORNER[k][0], None), hat(my, CORNER[k][1], None)
            M[j, k] = integ(pjx, qkx, lox, hix) * integ(pjy, qky, loy, hiy)
        if gap_line is not None:
            one = (F(1), F(0))
            g[j] = integ(pjx, one, lox, hix, extra=gap_line) * integ(pjy, one, loy, hiy)
    return D, M, g


def flat_rect(x, y, z=None):
    X = np.array([[x[0], y[0], 0], [x[1], y[0], 0], [x[1], y[1], 0], [x[0], y[1], 0]], float)
    if z is not None:
        X[:, 2] = [z(p[0]) for p in X]
    return X


def one_pair(xs, xm, prm):
    S = synth.Mesh(xs, np.array([[0, 1, 2, 3]], np.int32))
    M = synth.Mesh(xm, np.array([[0, 1, 2, 3]], np.int32))
    nv, blocks, st = oracle.eval_candidates(S, M, prm, np.array([0], np.int32), np.array([0], np.int32))
    return nv[0], blocks[0, :16].reshape(4, 4), blocks[0, 16:32].reshape(4, 4), blocks[0, 32:], st[0]


def tofloat(a):
    return np.array(a, dtype=float)


def test_identical_unit_squares_give_mass_matrix():
    xs = flat_rect((0, 1), (0, 1))
    nv, D, M, g, st = one_pair(xs, xs.copy(), oracle.params())
    assert nv == 4 and st == 0
    mass = np.array([[4, 2, 1, 2], [2, 4, 2, 1], [1, 2, 4, 2], [2, 1, 2, 4]]) / 36.0
    np.testing.assert_allclose(D, mass, atol=1e-15)
    np.testing.assert_allclose(M, mass, atol=1e-15)
    np.testing.assert_allclose(g, 0.0, atol=0)


def test_shifted_half_pair_exact():
    half = F(1, 2)
    Dx, Mx, _ = rect_pair_exact((F(0), F(1)), (F(0), F(1)), (half, half + 1), (half, half + 1))
    nv, D, M, g, st = one_pair(flat_rect((0, 1), (0, 1)), flat_rect((0.5, 1.5), (0.5, 1.5)), oracle.params())
    assert nv == 4
    np.testing.assert_allclose(D, tofloat(Dx), atol=1e-15)
    np.testing.assert_allclose(M, tofloat(Mx), atol=1e-15)
    # the hand-worked numbers (times 2304)
    np.testing.assert_allclose(D * 2304, [[4, 8, 16, 8], [8, 28, 56, 16], [16, 56, 196, 56], [8, 16, 56, 28]],
                               atol=1e-11)
    np.testing.assert_allclose(M * 2304, [[25, 5, 1, 5], [65, 25, 5, 13], [169, 65, 25, 65], [65, 13, 5, 25]],
                               atol=1e-11)
    assert abs(D.sum() - 0.25) < 1e-15


def test_tilted_master_plane_gap_exact():
    # master plane z = c0 + c1 x over a flat slave: g_j = int N_j (c0 + c1 x)
    c0, c1 = F(1, 4), F(1, 2)
    sx, sy = (F(0), F(1, 2)), (F(1, 4), F(3, 4))
    mx, my = (F(-1, 4), F(3, 4)), (F(0), F(1))
    _, _, gx = rect_pair_exact(sx, sy, mx, my, gap_line=(c0, c1))
    xs = flat_rect((0, 0.5), (0.25, 0.75))
    xm = flat_rect((-0.25, 0.75), (0.0, 1.0), z=lambda x: 0.25 + 0.5 * x)
    nv, D, M, g, st = one_pair(xs, xm, oracle.params())
    assert nv == 4 and st == 0
    np.testing.assert_allclose(g, tofloat(gx), atol=1e-15)
    assert np.all(g > 0)  # master on the +n0 side
    # flipping the master below the slave flips the sign
    xm2 = xm.copy()
    xm2[:, 2] *= -1
    _, _, _, g2, _ = one_pair(xs, xm2, oracle.params())
    np.testing.assert_allclose(g2, -g, atol=1e-15)


def test_unjittered_flat_config_exact_rational():
    ns, nm = 8, 7
    itf = synth.flat_tied(ns, nm, jitter=0.0)
    r = oracle.evaluate(itf)
    Dx = {}
    Mx = {}
    for s, m in zip(r["pair_s"], r["pair_m"]):
        si, sj = s % ns, s // ns
        mi, mj = m % nm, m // nm
        sx, sy = (F(si, ns), F(si + 1, ns)), (F(sj, ns), F(sj + 1, ns))
        mx, my = (F(mi, nm), F(mi + 1, nm)), (F(mj, nm), F(mj + 1, nm))
        D, M, _ = rect_pair_exact(sx, sy, mx, my)
        cs = itf.slave.conn[s]
        cm = itf.master.conn[m]
        for j in range(4):
            for k in range(4):
                Dx[(cs[j], cs[k])] = Dx.get((cs[j], cs[k]), 0) + D[j, k]
                Mx[(cs[j], cm[k])] = Mx.get((cs[j], cm[k]), 0) + M[j, k]
    Dc = r["D"].tocoo()
    Mc = r["M"].tocoo()
    assert set(zip(Dc.row, Dc.col)) == set(Dx)
    assert set(zip(Mc.row, Mc.col)) == set(Mx)
    for a, b, v in zip(Dc.row, Dc.col, Dc.data):
        assert abs(v - float(Dx[(a, b)])) < 1e-15
    for a, b, v in zip(Mc.row, Mc.col, Mc.data):
        assert abs(v - float(Mx[(a, b)])) < 1e-15
    np.testing.assert_array_equal(r["g"], 0.0)


@pytest.mark.parametrize("seed", [1000, 1, 2])
def test_global_invariants_jittered_flat(seed):
    itf = synth.flat_tied(8, 7, seed=seed)
    r = oracle.evaluate(itf)
    D, M, g = r["D"], r["M"], r["g"]
    # full coverage of the unit square: total D = slave area = 1
    assert abs(D.sum() - 1.0) < 1e-13
    # conservation: row sums of M equal row sums of D (partition of unity)
    np.testing.assert_allclose(np.asarray(M.sum(1)).ravel(), np.asarray(D.sum(1)).ravel(), atol=1e-15)
    # standard basis: D symmetric
    assert abs(D - D.T).max() < 1e-16
    # tied flat meshes: zero weighted gap
    np.testing.assert_array_equal(g, 0.0)


def test_sum_D_equals_clip_area_curved():
    itf = synth.cylinder(12, 9, seed=3)
    r = oracle.evaluate(itf)
    # total of D = sum over pairs of the clip polygon areas
    tot = 0.0
    for s, m in zip(r["pair_s"], r["pair_m"]):
        poly, st = oracle.pair_polygon(itf.slave.X[itf.slave.conn[s]], itf.master.X[itf.master.conn[m]],
                                       oracle.params(delta=itf.delta))
        x, y = poly[:, 0], poly[:, 1]
        tot += 0.5 * (np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))
    assert abs(r["D"].sum() - tot) < 1e-13
    np.testing.assert_allclose(np.asarray(r["M"].sum(1)).ravel(), np.asarray(r["D"].sum(1)).ravel(),
                               atol=1e-15)


def test_dual_basis_parallelogram_closed_form():
    C = np.array([[4, -2, 1, -2], [-2, 4, -2, 1], [1, -2, 4, -2], [-2, 1, -2, 4]], float)
    np.testing.assert_allclose(oracle.dual_matrix(flat_rect((0, 1), (0, 1))), C, atol=1e-13)
    par = np.array([[0, 0, 0], [2, 0.5, 0], [2.7, 2.0, 0], [0.7, 1.5, 0]], float)
    np.testing.assert_allclose(oracle.dual_matrix(par), C, atol=1e-12)
    # any rigid motion of the element leaves the coefficients unchanged
    Q, _ = np.linalg.qr(np.random.default_rng(1).normal(size=(3, 3)))
    np.testing.assert_allclose(oracle.dual_matrix(par @ Q.T + 3.0), C, atol=1e-12)


def test_dual_basis_biorthogonal_and_diagonal_D():
    # identical parallelogram elements: D_loc is diagonal with int N_j
    par = np.array([[0, 0, 0], [2, 0.5, 0], [2.7, 2.0, 0], [0.7, 1.5, 0]], float)
    nv, D, M, g, st = one_pair(par, par.copy(), oracle.params(dual=True))
    area = abs(np.cross(par[1] - par[0], par[3] - par[0])[2])
    np.testing.assert_allclose(D, np.diag([area / 4] * 4), atol=1e-14)
    # unjittered flat configuration: assembled D is diagonal, D_jj = sum_l M_jl
    itf = synth.flat_tied(8, 7, jitter=0.0)
    r = oracle.evaluate(itf, oracle.params(dual=True))
    Dd = r["D"].toarray()
    off = Dd - np.diag(np.diag(Dd))
    assert abs(off).max() < 1e-15
    np.testing.assert_allclose(np.diag(Dd), np.asarray(r["M"].sum(1)).ravel(), atol=1e-15)
