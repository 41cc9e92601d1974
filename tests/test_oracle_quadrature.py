"""Pin: the 7-point rule integrates every monomial of degree <= 5 exactly (and
not degree 6), on the reference triangle and on a mapped triangle."""
import math

import numpy as np
import pytest

from oracle import quadrature


def exact_ref(a, b):
    # int over {x,y >= 0, x + y <= 1} of x^a y^b = a! b! / (a + b + 2)!
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


def test_weights_sum_to_one():
    _, w = quadrature.seven_point()
    assert abs(w.sum() - 1.0) < 1e-15


@pytest.mark.parametrize("deg", range(6))
def test_monomials_exact(deg):
    tri = np.array([[[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]])
    pts, w, area = quadrature.points(tri)
    assert abs(area[0] - 0.5) < 1e-16
    for a in range(deg + 1):
        b = deg - a
        val = np.sum(w[0] * pts[0, :, 0] ** a * pts[0, :, 1] ** b)
        assert abs(val - exact_ref(a, b)) < 1e-15


def test_degree6_not_exact():
    tri = np.array([[[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]])
    pts, w, _ = quadrature.points(tri)
    errs = [abs(np.sum(w[0] * pts[0, :, 0] ** a * pts[0, :, 1] ** (6 - a)) - exact_ref(a, 6 - a))
            for a in range(7)]
    assert max(errs) > 1e-8


def test_mapped_triangle_area_and_moment():
    tri = np.array([[[0.1, 0.2, 0.0], [0.4, 0.25, 0.0], [0.2, 0.7, 0.0]]])
    pts, w, area = quadrature.points(tri)
    e1, e2 = tri[0, 1] - tri[0, 0], tri[0, 2] - tri[0, 0]
    assert abs(area[0] - 0.5 * abs(e1[0] * e2[1] - e1[1] * e2[0])) < 1e-16
    # first moment equals area * centroid
    c = tri[0].mean(axis=0)
    np.testing.assert_allclose((w[0][:, None] * pts[0]).sum(axis=0), area[0] * c, rtol=0, atol=1e-16)
