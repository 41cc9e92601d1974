"""The synthetic workloads, as plain data.

Units are PEC square patches at 15 mm period and 10 GHz (the frequency and
period of the plain 6x6 case are inherited by the larger cases, which do not
restate them).  Sizes, precisions and seeds follow the workload list of the
project; nothing here performs electromagnetic arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import codebooks as cb
from .mesh import macro_unit

FREQ_HZ = 10.0e9
PERIOD = (0.015, 0.015)
SIDES_1BIT = (0.006, 0.009)
SIDES_2BIT = (0.005, 0.007, 0.009, 0.011)


@dataclass
class Workload:
    name: str
    sides: tuple
    L: int
    near_radius: int  # Chebyshev radius of the dense blocks (>= L-1: all dense)
    near_dtype: str  # "c128" | "c64"
    far_dtype: str  # "c128" | "c64" | "bf16x2" | "f16x2" | "none"
    aca_tol: float
    max_rank: int
    gmres_tol: float
    refine_tol: float  # 0: no outer refinement
    codebooks: list = field(default_factory=list)  # list of uint8 [L_b*L_b]
    sizes: list = field(default_factory=list)  # L_b per codebook
    angles_deg: tuple = (0.0,)
    ncell: int = 4
    freq_hz: float = FREQ_HZ
    period: tuple = PERIOD

    def unit(self):
        return macro_unit(self.sides, self.ncell, self.period)


def plain_6x6() -> Workload:
    """1-bit 6x6, complex128 everywhere, all 121 displacement blocks dense."""
    return Workload("plain-1bit-6x6-c128", SIDES_1BIT, 6, 5, "c128", "none",
                    0.0, 0, 1e-8, 0.0, [cb.bernoulli(6, 0)], [6])


def twobit_32x32() -> Workload:
    """2-bit 32x32: dense c64 near (|dx|,|dy|<=2), ACA c64 far at tol 1e-4."""
    return Workload("2bit-32x32-c64-aca", SIDES_2BIT, 32, 2, "c64", "c64",
                    1e-4, 40, 1e-4, 0.0, [cb.uniform(32, 4, 1)], [32])


def batched_1bit(n_per_size: int = 128) -> Workload:
    """1-bit codebooks of three array sizes sharing one store sized for 64x64."""
    books, sizes = [], []
    for L in (32, 48, 64):
        for c in range(n_per_size):
            books.append(cb.family(c, L, 2000))
            sizes.append(L)
    return Workload("batched-1bit-32/48/64", SIDES_1BIT, 64, 2, "c64", "bf16x2",
                    1e-4, 12, 1e-4, 1e-6, books, sizes, (0.0, 20.0, 40.0, 60.0))


def large_128x128(n_books: int = 16) -> Workload:
    books = [cb.bernoulli(128, 4000 + i) for i in range(n_books)]
    return Workload("large-1bit-128x128", SIDES_1BIT, 128, 2, "c64", "f16x2",
                    1e-4, 12, 1e-4, 1e-5, books, [128] * n_books)


def small_1bit(L: int, seed: int = 0, near_radius: int | None = None) -> Workload:
    """A small 1-bit case for tests (all dense unless near_radius is given)."""
    nr = L - 1 if near_radius is None else near_radius
    return Workload(f"1bit-{L}x{L}", SIDES_1BIT, L, nr, "c128", "c128",
                    1e-4, 40, 1e-10, 0.0, [cb.bernoulli(L, seed)], [L])


def displacement_count(L: int) -> int:
    return (2 * L - 1) ** 2


def far_pair_count(L: int, near_radius: int) -> int:
    """Number of ordered unit pairs (i, j) of an L x L array with Chebyshev
    distance > near_radius."""
    d = np.arange(-(L - 1), L)
    w = L - np.abs(d)  # pairs per component displacement
    tot = np.outer(w, w)
    near = (np.abs(d)[:, None] <= near_radius) & (np.abs(d)[None, :] <= near_radius)
    return int(tot[~near].sum())


def near_pair_count(L: int, near_radius: int) -> int:
    return L ** 4 - far_pair_count(L, near_radius)


# Solver settings of the batched workload (1,536 right-hand sides), shared by
# the benchmark and its full-size test: complex64 inner GMRES(20) to 1e-3 with
# block-Jacobi, complex128 refinement residual to 1e-6; the reference solution
# that the RCS error is measured against is the same system refined to 1e-10.
BATCHED_SOLVE = {"restart": 20, "inner_tol": 1e-3, "refine_tol": 1e-6, "max_refine": 20, "max_iter": 3000,
                 "ref_refine_tol": 1e-10}
# Headline solve of the 2-bit 32x32 workload: block ILU(0) radius 1, GMRES(60)
# to 5e-5 on the compressed complex64 store.
TWOBIT_SOLVE = {"restart": 60, "tol": 5e-5, "ilu_radius": 1, "max_iter": 6000}
