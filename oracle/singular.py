"""Closed-form potential integrals of a flat triangle (singularity extraction).

For an observation point r and a triangle T with unit normal n, the static
kernel 1/R (R = |r' - r|) is integrated exactly:

    S(r)   = int_T 1/R dS'
    V(r)   = int_T (r' - r)/R dS'

by the edge-sum formulas of Wilton et al. (1984) and Graglia (1993).  These
integrals are used to remove the 1/R singularity of the Green's function from
the Galerkin EFIE entries of eq. (1) when the two triangles are close.

For each edge i (vertices a -> b, counter-clockwise about n):
  l_hat = (b - a)/|b - a|,  u_hat = l_hat x n  (outward in-plane normal),
  d     = n . (r - a)       (height of r above the plane),
  rho   = r - d n           (projection),
  t0    = (a - rho) . u_hat (signed in-plane distance to the edge line),
  l-    = (a - rho) . l_hat,  l+ = (b - rho) . l_hat,
  R0^2  = t0^2 + d^2,  R(+-) = sqrt(l(+-)^2 + R0^2),
  f     = ln((R+ + l+)/(R- + l-)),
  S     = sum_i [ t0 f - |d| (atan(t0 l+/(R0^2 + |d| R+)) - atan(t0 l-/(R0^2 + |d| R-))) ],
  V_par = 1/2 sum_i u_hat [ R0^2 f + l+ R+ - l- R- ],
  V     = V_par - d n S.

The logarithm is evaluated in the cancellation-free forms
  both l >= 0:   ln((R+ + l+)/(R- + l-))
  both l <= 0:   ln((R- - l-)/(R+ - l+))
  l- < 0 < l+:   ln((R+ + l+)(R- - l-)/R0^2)
and every term carrying f is dropped when R0 <= 1e-12 |b - a| (its limit is 0:
the point lies on the edge line).
"""
import numpy as np

GUARD_REL = 1e-12


def potential_integrals_paired(r: np.ndarray, tri_xyz: np.ndarray):
    """S [K] and V [K,3] for point r[i] against triangle tri_xyz[i] (paired)."""
    r = np.asarray(r, dtype=np.float64)
    tri_xyz = np.asarray(tri_xyz, dtype=np.float64)
    a0, a1, a2 = tri_xyz[:, 0], tri_xyz[:, 1], tri_xyz[:, 2]
    nrm = np.cross(a1 - a0, a2 - a0)
    n = nrm / np.linalg.norm(nrm, axis=1, keepdims=True)  # [K,3]

    d = np.einsum("kc,kc->k", n, r - a0)
    rho = r - d[:, None] * n
    ad = np.abs(d)

    S = np.zeros(d.shape)
    Vp = np.zeros(d.shape + (3,))
    verts = (a0, a1, a2)
    for i in range(3):
        a = verts[i]
        b = verts[(i + 1) % 3]
        elen = np.linalg.norm(b - a, axis=1)
        lh = (b - a) / elen[:, None]
        uh = np.cross(lh, n)
        am = a - rho
        bm = b - rho
        t0 = np.einsum("kc,kc->k", am, uh)
        lm = np.einsum("kc,kc->k", am, lh)
        lp = np.einsum("kc,kc->k", bm, lh)
        R0sq = t0 * t0 + d * d
        Rm = np.sqrt(lm * lm + R0sq)
        Rp = np.sqrt(lp * lp + R0sq)

        ok = np.sqrt(R0sq) > GUARD_REL * elen
        with np.errstate(divide="ignore", invalid="ignore"):
            f_pos = np.log((Rp + lp) / (Rm + lm))
            f_neg = np.log((Rm - lm) / (Rp - lp))
            f_mid = np.log((Rp + lp) * (Rm - lm) / R0sq)
        f = np.where(lm >= 0.0, f_pos, np.where(lp <= 0.0, f_neg, f_mid))
        f = np.where(ok, f, 0.0)

        term = t0 * f
        has_d = ad > 0.0
        with np.errstate(divide="ignore", invalid="ignore"):
            at = np.arctan(t0 * lp / (R0sq + ad * Rp)) - np.arctan(t0 * lm / (R0sq + ad * Rm))
        term = term - np.where(has_d, ad * at, 0.0)
        S += term
        Vp += 0.5 * (R0sq * f + lp * Rp - lm * Rm)[:, None] * uh

    V = Vp - (d * S)[:, None] * n
    return S, V


def potential_integrals(r: np.ndarray, tri_xyz: np.ndarray):
    """S [M,Q] and V [M,Q,3] for every point of r [M,3] against every triangle [Q,3,3]."""
    r = np.asarray(r, dtype=np.float64)
    tri_xyz = np.asarray(tri_xyz, dtype=np.float64)
    M, Q = len(r), len(tri_xyz)
    rr = np.repeat(r, Q, axis=0)
    tt = np.tile(tri_xyz, (M, 1, 1))
    S, V = potential_integrals_paired(rr, tt)
    return S.reshape(M, Q), V.reshape(M, Q, 3)
