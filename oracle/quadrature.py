"""Seven-point degree-5 triangle rule (Radon 1948; Dunavant 1985, degree 5).

Points are barycentric; weights sum to one and are multiplied by the triangle
area by the caller.  Used for every surface integral of the Galerkin EFIE of
eq. (1) (testing and source integrals; on 64 sub-triangles of the observer
triangle for overlapping triangles of different coding states, see efie),
the excitation and the radiation integrals.
"""
import math

import numpy as np


def seven_point():
    s15 = math.sqrt(15.0)
    a1 = (6.0 - s15) / 21.0
    b1 = 1.0 - 2.0 * a1
    a2 = (6.0 + s15) / 21.0
    b2 = 1.0 - 2.0 * a2
    w0 = 9.0 / 40.0
    w1 = (155.0 - s15) / 1200.0
    w2 = (155.0 + s15) / 1200.0
    bary = np.array([
        [1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0],
        [b1, a1, a1], [a1, b1, a1], [a1, a1, b1],
        [b2, a2, a2], [a2, b2, a2], [a2, a2, b2],
    ])
    w = np.array([w0, w1, w1, w1, w2, w2, w2])
    return bary, w


def points(tri_xyz: np.ndarray):
    """Quadrature points [T,7,3] and area-weighted weights [T,7] of triangles [T,3,3]."""
    bary, w = seven_point()
    pts = np.einsum("qa,tad->tqd", bary, tri_xyz)
    e1 = tri_xyz[:, 1] - tri_xyz[:, 0]
    e2 = tri_xyz[:, 2] - tri_xyz[:, 0]
    area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
    return pts, area[:, None] * w[None, :], area
