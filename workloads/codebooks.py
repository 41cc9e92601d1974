"""Seeded codebooks, vectors and direction sets (data only, no method arithmetic).

A codebook assigns each unit of an L x L array one coding state; it is stored
row-major as uint8 [L*L] with unit u = iy*L + ix.  The families below stand in
for the random codebooks of Sec. IV-B (i.i.d. Bernoulli per unit) and the
steering codebooks of Table 2 (stripe / checkerboard layouts).
"""
from __future__ import annotations

import numpy as np


def bernoulli(L: int, seed: int, p: float = 0.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if p == 0.5:
        s = rng.integers(0, 2, (L, L))
    else:
        s = (rng.random((L, L)) < p).astype(np.int64)
    return s.astype(np.uint8).reshape(-1)


def uniform(L: int, n_states: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_states, (L, L)).astype(np.uint8).reshape(-1)


def checkerboard(L: int, block: int = 4) -> np.ndarray:
    iy, ix = np.mgrid[0:L, 0:L]
    return (((ix // block) + (iy // block)) % 2).astype(np.uint8).reshape(-1)


def stripes(L: int, seed: int) -> np.ndarray:
    """Linear phase-gradient stripes along x with a seeded period in [2, 8]."""
    rng = np.random.default_rng(seed)
    P = int(rng.integers(2, 9))
    iy, ix = np.mgrid[0:L, 0:L]
    return ((2 * (ix % P)) // P).astype(np.uint8).reshape(-1)


def family(c: int, L: int, base_seed: int) -> np.ndarray:
    """Codebook c of the batched family: Bernoulli, checkerboard, stripes in turn."""
    f = c % 3
    if f == 0:
        return bernoulli(L, base_seed + c)
    if f == 1:
        return checkerboard(L, 4)
    return stripes(L, base_seed + c)


def mirror_x(states: np.ndarray, L: int) -> np.ndarray:
    """Codebook mirrored ix -> L-1-ix."""
    return states.reshape(L, L)[:, ::-1].reshape(-1).copy()


def symmetrize_x(states: np.ndarray, L: int) -> np.ndarray:
    """Codebook made symmetric under ix -> L-1-ix (left half copied to the right)."""
    s = states.reshape(L, L).copy()
    s[:, L - L // 2:] = s[:, : L // 2][:, ::-1]
    return s.reshape(-1)


def random_complex(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def phi0_cut(step_deg: float = 1.0) -> np.ndarray:
    """Directions (theta, phi) in radians of a phi = 0 cut from -180 to <180 deg.

    Negative theta stands for phi = 180 deg.
    """
    th = np.deg2rad(np.arange(-180.0, 180.0, step_deg))
    return np.stack([th, np.zeros_like(th)], axis=1)


def cone16(half_angle_deg: float = 30.0) -> np.ndarray:
    """16 directions in a cone about +z: 8 at half the half-angle, 8 at the rim."""
    a = np.deg2rad(half_angle_deg)
    d = []
    for i in range(8):
        d.append((a / 2, np.deg2rad(45.0 * i)))
    for i in range(8):
        d.append((a, np.deg2rad(22.5 + 45.0 * i)))
    return np.asarray(d)
