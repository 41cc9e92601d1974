"""Shared helpers of the GPU parity tests (CPU oracle side + device setup)."""
import functools

import numpy as np

from oracle import efie, excitation, farfield, retrieval, solve
from oracle.constants import wavenumber
from workloads import codebooks as cb
from workloads.mesh import macro_unit

FREQ = 10.0e9
K = wavenumber(FREQ)
SIDES1 = (0.006, 0.009)
SIDES2 = (0.005, 0.007, 0.009, 0.011)


@functools.lru_cache(None)
def unit(bits: int):
    return macro_unit(SIDES1 if bits == 1 else SIDES2)


@functools.lru_cache(None)
def oracle_blocks(bits: int, D: int):
    return efie.displacement_blocks(unit(bits), D, D, K, extract=1)


@functools.lru_cache(None)
def oracle_direct(bits: int, L: int, seed: int):
    states = cb.bernoulli(L, seed) if bits == 1 else cb.uniform(L, 4, seed)
    Z = efie.direct_system(unit(bits), states, L, K, extract=1)
    return states, Z


def oracle_rhs(bits, states, L, theta=0.0, phi=0.0):
    mesh, _ = efie.active_array_mesh(unit(bits), states, L)
    return excitation.plane_wave(mesh, K, theta, phi)


def oracle_rcs(bits, states, L, I, dirs):
    mesh, _ = efie.active_array_mesh(unit(bits), states, L)
    return farfield.rcs(mesh, I, K, dirs)


def rel_max(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))
