"""Plane-wave excitation vector U of eq. (1): U_m = int f_m . E_inc dS (7-point rule).

E_inc(r) = E0 e_hat exp(-j k k_hat . r), with propagation direction
k_hat = -(sin t cos p, sin t sin p, cos t) (arriving from direction (t, p)) and
theta polarisation e_hat = (cos t cos p, cos t sin p, -sin t); at normal
incidence this is an x-polarised wave travelling towards -z.
"""
import math

import numpy as np

from . import quadrature


def incidence_vectors(theta: float, phi: float):
    st, ct = math.sin(theta), math.cos(theta)
    sp, cp = math.sin(phi), math.cos(phi)
    khat = -np.array([st * cp, st * sp, ct])
    ehat = np.array([ct * cp, ct * sp, -st])
    return khat, ehat


def plane_wave(mesh, k: float, theta: float = 0.0, phi: float = 0.0, e0: float = 1.0,
               khat=None, ehat=None) -> np.ndarray:
    if khat is None:
        khat, ehat = incidence_vectors(theta, phi)
    pts, w, area = quadrature.points(mesh.tri_xyz)
    U = np.zeros(mesh.n, dtype=np.complex128)
    for a, sgn in ((0, 1.0), (1, -1.0)):
        t = mesh.rwg_tri[:, a]
        v = mesh.tri_xyz[t, mesh.rwg_free[:, a]]  # free vertex [N,3]
        r = pts[t]  # [N,7,3]
        phase = np.exp(-1j * k * (r @ khat))  # [N,7]
        proj = (r - v[:, None, :]) @ ehat  # [N,7]
        c = sgn * mesh.rwg_len / (2.0 * area[t])
        U += c * np.sum(w[t] * proj * phase, axis=1)
    return e0 * U
