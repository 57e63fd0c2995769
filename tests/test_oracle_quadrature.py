"""Pins of the oracle's triangle rules and inverse bilinear map."""

from fractions import Fraction
from math import factorial

import numpy as np
import pytest

import oracle


def exact_monomial_ref_triangle(a, b):
    # integral of x^a y^b over the triangle (0,0), (1,0), (0,1)
    return Fraction(factorial(a) * factorial(b), factorial(a + b + 2))


@pytest.mark.parametrize("which,degree", [(3, 2), (7, 5)])
def test_rule_exact_to_degree(which, degree):
    l, w = oracle.rule(which)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(l.sum(1), 1.0, atol=1e-15)
    # points on the reference triangle: p = l0*(0,0) + l1*(1,0) + l2*(0,1)
    x, y = l[:, 1], l[:, 2]
    area = 0.5
    for a in range(degree + 1):
        for b in range(degree + 1 - a):
            q = area * np.sum(w * x ** a * y ** b)
            ex = float(exact_monomial_ref_triangle(a, b))
            assert abs(q - ex) < 1e-15, (a, b, q, ex)
    # and not exact one degree higher (it is the rule claimed, not more)
    errs = [abs(area * np.sum(w * x ** a * y ** (degree + 1 - a))
                - float(exact_monomial_ref_triangle(a, degree + 1 - a))) for a in range(degree + 2)]
    assert max(errs) > 1e-6


def test_fan_points_integrate_polygon_moments():
    # fan quadrature over a convex pentagon integrates x^a y^b (a+b<=5)
    # exactly; compare with the shoelace-type exact polygon moment via
    # Green's theorem evaluated with Fractions.
    P = [(Fraction(0), Fraction(0)), (Fraction(3), Fraction(0)), (Fraction(4), Fraction(2)),
         (Fraction(2), Fraction(4)), (Fraction(-1), Fraction(2))]

    def tri_moment(A, B, C, a, b):
        # exact integral of x^a y^b over triangle ABC via affine map from the
        # reference triangle and multinomial expansion
        (x0, y0), (x1, y1), (x2, y2) = A, B, C
        J = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)
        # x = x0 + s(x1-x0) + t(x2-x0); expand with polynomial dicts in (s,t)
        def poly_lin(c0, cs, ct):
            return {(0, 0): c0, (1, 0): cs, (0, 1): ct}

        def mul(p, q):
            r = {}
            for (i1, j1), c1 in p.items():
                for (i2, j2), c2 in q.items():
                    r[(i1 + i2, j1 + j2)] = r.get((i1 + i2, j1 + j2), 0) + c1 * c2
            return r
        X = poly_lin(x0, x1 - x0, x2 - x0)
        Y = poly_lin(y0, y1 - y0, y2 - y0)
        p = {(0, 0): Fraction(1)}
        for _ in range(a):
            p = mul(p, X)
        for _ in range(b):
            p = mul(p, Y)
        return abs(J) * sum(c * exact_monomial_ref_triangle(i, j) for (i, j), c in p.items())

    poly = np.array([[float(x), float(y)] for x, y in P])
    q, w = oracle.fan_points(poly, rule=7)
    for a in range(6):
        for b in range(6 - a):
            ex = sum(tri_moment(P[0], P[i], P[i + 1], a, b) for i in range(1, len(P) - 1))
            val = np.sum(w * q[:, 0] ** a * q[:, 1] ** b)
            assert abs(val - float(ex)) <= 1e-12 * max(1.0, abs(float(ex))), (a, b)


def test_inverse_bilinear_recovers_parameters():
    rng = np.random.default_rng(5)
    ref = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], float)
    for _ in range(50):
        quad = ref * rng.uniform(0.5, 2.0) + rng.normal(0, 0.2, (4, 2))
        xi = rng.uniform(-1, 1, 2)
        N = 0.25 * (1 + ref[:, 0] * xi[0]) * (1 + ref[:, 1] * xi[1])
        p = N @ quad
        got, st = oracle.inverse_bilinear(quad, p)
        assert st == 0
        np.testing.assert_allclose(got, xi, atol=1e-12)
    # nodes map to their reference coordinates
    quad = np.array([[0, 0], [2, 0.1], [2.2, 1.7], [-0.1, 1.2]], float)
    for k in range(4):
        got, st = oracle.inverse_bilinear(quad, quad[k])
        np.testing.assert_allclose(got, ref[k], atol=1e-13)
