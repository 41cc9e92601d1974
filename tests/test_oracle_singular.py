"""Pin: closed-form potential integrals vs independent polar-coordinate quadrature.

The triangle integral over T is written as the signed sum of the three
sub-triangles (p, a, b) spanned by the projected observation point p and each
edge.  In polar coordinates about p the radial integral is elementary and the
angular one is done by adaptive scipy quadrature, with the ray/edge-line
intersection computed directly: no edge-sum formula is involved.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle.singular import potential_integrals, potential_integrals_paired


def polar_reference(r, tri):
    a0, a1, a2 = tri
    n = np.cross(a1 - a0, a2 - a0)
    n /= np.linalg.norm(n)
    d = float(np.dot(n, r - a0))
    p = r - d * n
    # orthonormal frame in the plane
    e1 = (a1 - a0) / np.linalg.norm(a1 - a0)
    e2 = np.cross(n, e1)
    S = 0.0
    V = np.zeros(3)
    ad = abs(d)
    for a, b in ((a0, a1), (a1, a2), (a2, a0)):
        A = np.array([np.dot(a - p, e1), np.dot(a - p, e2)])
        B = np.array([np.dot(b - p, e1), np.dot(b - p, e2)])
        cross = A[0] * B[1] - A[1] * B[0]
        if abs(cross) < 1e-14 * np.linalg.norm(A - B) ** 2:
            continue  # degenerate sub-triangle (p on the edge line)
        ta = math.atan2(A[1], A[0])
        tb = math.atan2(B[1], B[0])
        dth = tb - ta
        if dth > math.pi:
            dth -= 2 * math.pi
        if dth < -math.pi:
            dth += 2 * math.pi

        def smax(th):
            # ray p + s (cos th, sin th) meets line A + t (B - A)
            u = np.array([math.cos(th), math.sin(th)])
            D = B - A
            M = np.array([[u[0], -D[0]], [u[1], -D[1]]])
            s, _ = np.linalg.solve(M, A)
            return s

        def f_s(th):
            s = smax(th)
            return math.sqrt(s * s + d * d) - ad

        def f_v(th, comp):
            s = smax(th)
            if ad == 0.0:
                rad = 0.5 * s * s
            else:
                q = math.sqrt(s * s + d * d)
                rad = 0.5 * (s * q - d * d * math.log((s + q) / ad))
            u = math.cos(th) * e1 + math.sin(th) * e2
            return rad * u[comp]

        opts = dict(epsabs=1e-15, epsrel=1e-13, limit=200)
        S += integrate.quad(f_s, ta, ta + dth, **opts)[0]
        for c in range(3):
            V[c] += integrate.quad(lambda t: f_v(t, c), ta, ta + dth, **opts)[0]
    V = V - d * S * n
    return S, V


TRI = np.array([[0.0, 0.0, 0.0], [2.0e-3, 0.3e-3, 0.0], [0.5e-3, 1.7e-3, 0.0]])
CENT = TRI.mean(axis=0)
POINTS = {
    "centroid": CENT,
    "inside": np.array([0.6e-3, 0.5e-3, 0.0]),
    "outside": np.array([3.0e-3, 2.5e-3, 0.0]),
    "on_edge": 0.5 * (TRI[0] + TRI[1]),
    "edge_line_beyond": TRI[0] + 1.7 * (TRI[1] - TRI[0]),
    "vertex_near": TRI[2] + np.array([1e-7, -2e-7, 0.0]),
    "vertex": TRI[1].copy(),
    "above_inside": CENT + np.array([0.0, 0.0, 0.4e-3]),
    "above_outside": np.array([-1.0e-3, 2.0e-3, 0.7e-3]),
    "far": np.array([0.03, -0.02, 0.0]),
}


@pytest.mark.parametrize("name", sorted(POINTS))
def test_against_polar_quadrature(name):
    r = POINTS[name]
    S, V = potential_integrals_paired(r[None], TRI[None])
    Sr, Vr = polar_reference(r, TRI)
    scale = 2.0e-3  # triangle size: S ~ size, V ~ size^2
    assert abs(S[0] - Sr) <= 1e-10 * scale
    assert np.max(np.abs(V[0] - Vr)) <= 1e-10 * scale * scale


def test_far_point_limit():
    # far away, int 1/R -> area/|r - c|
    r = np.array([5.0, 3.0, 1.0])
    S, _ = potential_integrals_paired(r[None], TRI[None])
    area = 0.5 * np.linalg.norm(np.cross(TRI[1] - TRI[0], TRI[2] - TRI[0]))
    # next term of the multipole expansion is O((size/R)^2) ~ 1e-7
    assert abs(S[0] - area / np.linalg.norm(r - CENT)) < 1e-6 * S[0]


def test_overlapping_state_meshes(unit1):
    """Quadrature points of the 9 mm mesh against triangles of the 6 mm mesh of
    the same macro unit (coexistent meshes), including points on edge lines."""
    from oracle import quadrature
    off = unit1.tri_off
    big = unit1.vert[unit1.tri[off[1]:off[2]]]
    small = unit1.vert[unit1.tri[off[0]:off[1]]]
    pts, _, _ = quadrature.points(big)
    pts = pts.reshape(-1, 3)
    rng = np.random.default_rng(5)
    sel = rng.choice(len(pts), 12, replace=False)
    # make sure at least one point lies exactly on an edge line of the small mesh
    on_line = [i for i in range(len(pts)) if abs(abs(pts[i, 0]) - 1.5e-3) < 1e-18]
    sel = np.concatenate([sel, on_line[:3]])
    tq = [3, 17, 30]
    S, V = potential_integrals(pts[sel], small[tq])
    for a, i in enumerate(sel):
        for b, q in enumerate(tq):
            Sr, Vr = polar_reference(pts[i], small[q])
            assert abs(S[a, b] - Sr) <= 1e-10 * 1.5e-3
            assert np.max(np.abs(V[a, b] - Vr)) <= 1e-10 * 1.5e-3 ** 2
    assert np.all(np.isfinite(S)) and np.all(np.isfinite(V))
