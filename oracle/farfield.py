"""Radiation vectors, bistatic RCS and radiated power from RWG currents.

For a current J = sum_n I_n f_n the far field is
  E(r) ~ -j k eta exp(-j k r)/(4 pi r) [N - (N . r_hat) r_hat],
  N(r_hat) = sum_n I_n int f_n(r') exp(j k r_hat . r') dS'   (7-point rule),
so the bistatic RCS is
  sigma = (k^2 eta^2 / 4 pi) |N - (N . r_hat) r_hat|^2 / |E0|^2     [m^2]
and the radiated power is (k^2 eta / 32 pi^2) * integral over the sphere of
|N_perp|^2.  D(r_hat) = sum_n I_n int div f_n exp(j k r_hat . r') dS' is the
charge transform used by the discrete power identity.
"""
import math

import numpy as np

from . import quadrature
from .constants import ETA0


def directions(thph: np.ndarray) -> np.ndarray:
    th, ph = thph[:, 0], thph[:, 1]
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)


def rwg_transforms(mesh, k: float, rhat: np.ndarray):
    """F[n, dir, 3] = int f_n exp(j k r_hat.r) dS and Dv[n, dir] = int div f_n exp(...) dS."""
    pts, w, area = quadrature.points(mesh.tri_xyz)
    F = np.zeros((mesh.n, len(rhat), 3), dtype=np.complex128)
    Dv = np.zeros((mesh.n, len(rhat)), dtype=np.complex128)
    for a, sgn in ((0, 1.0), (1, -1.0)):
        t = mesh.rwg_tri[:, a]
        v = mesh.tri_xyz[t, mesh.rwg_free[:, a]]
        r = pts[t]  # [N,7,3]
        ph = np.exp(1j * k * np.einsum("nqc,dc->nqd", r, rhat))  # [N,7,D]
        wt = w[t]  # [N,7]
        c = sgn * mesh.rwg_len / (2.0 * area[t])
        F += c[:, None, None] * np.einsum("nq,nqd,nqc->ndc", wt, ph, r - v[:, None, :])
        Dv += (2.0 * c)[:, None] * np.einsum("nq,nqd->nd", wt, ph)
    return F, Dv


def radiation_vector(mesh, I, k: float, rhat: np.ndarray) -> np.ndarray:
    F, _ = rwg_transforms(mesh, k, rhat)
    return np.einsum("n,ndc->dc", I, F)


def rcs(mesh, I, k: float, thph: np.ndarray, e0: float = 1.0) -> np.ndarray:
    rhat = directions(thph)
    N = radiation_vector(mesh, I, k, rhat)
    Nperp = N - np.sum(N * rhat, axis=1, keepdims=True) * rhat
    return (k * k * ETA0 * ETA0 / (4.0 * math.pi)) * np.sum(np.abs(Nperp) ** 2, axis=1) / abs(e0) ** 2


def sphere_rule(n_theta: int, n_phi: int):
    """Directions [n,3] and weights [n] (sum 4 pi): Gauss-Legendre in cos(theta) x uniform phi."""
    x, wx = np.polynomial.legendre.leggauss(n_theta)
    ph = 2.0 * math.pi * np.arange(n_phi) / n_phi
    th = np.arccos(x)
    T, P = np.meshgrid(th, ph, indexing="ij")
    rhat = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=-1).reshape(-1, 3)
    w = (wx[:, None] * np.full(n_phi, 2.0 * math.pi / n_phi)[None, :]).reshape(-1)
    return rhat, w


def radiated_power(mesh, I, k: float, n_theta: int = 48, n_phi: int = 96):
    """(physical, discrete) radiated power.

    physical = (k^2 eta/32 pi^2) sum_w |N_perp|^2
    discrete = (k^2 eta/32 pi^2) sum_w (|N|^2 - |D|^2/k^2), which equals
    Re(I^H Z I)/2 exactly (up to the sphere rule) for the 7-point Galerkin Z.
    """
    rhat, w = sphere_rule(n_theta, n_phi)
    F, Dv = rwg_transforms(mesh, k, rhat)
    N = np.einsum("n,ndc->dc", I, F)
    D = I @ Dv
    Nperp = N - np.sum(N * rhat, axis=1, keepdims=True) * rhat
    c = k * k * ETA0 / (32.0 * math.pi ** 2)
    phys = c * np.sum(w * np.sum(np.abs(Nperp) ** 2, axis=1))
    disc = c * np.sum(w * (np.sum(np.abs(N) ** 2, axis=1) - np.abs(D) ** 2 / (k * k)))
    return phys, disc
