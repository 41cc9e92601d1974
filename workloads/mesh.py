"""Unit-cell geometry and RWG connectivity tables (data only).

Every coding state of a unit is a zero-thickness square PEC patch in the plane
z = 0, centred in its cell and meshed as an ncell x ncell grid of squares, each
split into two triangles.  The diagonal of every square runs through the square
corner nearest the patch centre, which keeps the mesh symmetric under the
eight symmetries of the square (so mirror tests hold to rounding).

An RWG function lives on every interior edge (Sec. II-A: Rao-Wilton-Glisson
bases on triangle pairs sharing an edge).  The table emitted here is pure
connectivity: (T+, T-, edge vertex 0, edge vertex 1) with T+ the lower
triangle id; interior edges are ordered by (lower vertex id, higher vertex id).

The macro unit of Sec. III-A is the union of all coding states of a unit: the
states' meshes are concatenated in state order, so that the basis functions of
state s occupy the contiguous range [state_off[s], state_off[s+1]).

This module computes no electromagnetic quantity; both the CPU oracle and the
GPU library consume its arrays.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class PatchMesh:
    side: float
    ncell: int
    vert: np.ndarray  # [nv, 3] float64, metres, unit-local
    tri: np.ndarray  # [nt, 3] int32, counter-clockwise about +z
    rwg: np.ndarray  # [nr, 4] int32: tri_plus, tri_minus, edge_v0, edge_v1


def patch_mesh(side: float, ncell: int = 4) -> PatchMesh:
    """Mesh of a square patch of the given side (m) centred at the origin."""
    if ncell < 1:
        raise ValueError("ncell must be >= 1")
    h = side / ncell
    nv1 = ncell + 1
    vert = np.zeros((nv1 * nv1, 3))
    for j in range(nv1):
        for i in range(nv1):
            # (i - ncell/2) * h is exactly antisymmetric about the centre
            vert[j * nv1 + i, 0] = (i - ncell / 2.0) * h
            vert[j * nv1 + i, 1] = (j - ncell / 2.0) * h

    def vid(i, j):
        return j * nv1 + i

    c2 = ncell  # twice the centre index, to stay in integers
    tris = []
    for cj in range(ncell):
        for ci in range(ncell):
            v00, v10 = vid(ci, cj), vid(ci + 1, cj)
            v01, v11 = vid(ci, cj + 1), vid(ci + 1, cj + 1)
            left = 2 * ci < c2  # square lies left of the centre column
            below = 2 * cj < c2
            # nearest corner to the centre: v11 (left, below), v00 (right, above),
            # v01 (right, below), v10 (left, above)
            if left == below:
                tris.append((v00, v10, v11))
                tris.append((v00, v11, v01))
            else:
                tris.append((v00, v10, v01))
                tris.append((v10, v11, v01))
    tri = np.asarray(tris, dtype=np.int32)

    edge_tris: dict[tuple[int, int], list[int]] = {}
    for t, (a, b, c) in enumerate(tri):
        for p, q in ((a, b), (b, c), (c, a)):
            key = (min(p, q), max(p, q))
            edge_tris.setdefault(key, []).append(t)
    rwg = []
    for key in sorted(edge_tris):
        ts = edge_tris[key]
        if len(ts) == 2:
            rwg.append((min(ts), max(ts), key[0], key[1]))
        elif len(ts) != 1:
            raise RuntimeError("non-manifold edge")
    return PatchMesh(side, ncell, vert, tri, np.asarray(rwg, dtype=np.int32))


@dataclass
class MacroUnit:
    """Concatenation of the coding states of one unit (coexistent meshes)."""

    sides: tuple
    ncell: int
    period: tuple  # (px, py) metres
    vert: np.ndarray
    tri: np.ndarray
    rwg: np.ndarray
    state_off: np.ndarray  # [n_states+1] RWG offsets
    tri_off: np.ndarray  # [n_states+1] triangle offsets
    vert_off: np.ndarray  # [n_states+1] vertex offsets
    states: list = field(default_factory=list)  # the PatchMesh of each state

    @property
    def n_states(self) -> int:
        return len(self.sides)

    @property
    def n(self) -> int:
        return int(self.state_off[-1])

    @property
    def n_a(self) -> int:
        sizes = np.diff(self.state_off)
        if not np.all(sizes == sizes[0]):
            raise ValueError("states differ in basis count")
        return int(sizes[0])


def macro_unit(sides, ncell: int = 4, period=(0.015, 0.015)) -> MacroUnit:
    meshes = [patch_mesh(s, ncell) for s in sides]
    vert, tri, rwg = [], [], []
    soff, toff, voff = [0], [0], [0]
    for m in meshes:
        vbase, tbase = voff[-1], toff[-1]
        vert.append(m.vert)
        tri.append(m.tri + vbase)
        r = m.rwg.copy()
        r[:, 0:2] += tbase
        r[:, 2:4] += vbase
        rwg.append(r)
        soff.append(soff[-1] + len(m.rwg))
        toff.append(toff[-1] + len(m.tri))
        voff.append(voff[-1] + len(m.vert))
    return MacroUnit(
        tuple(sides),
        ncell,
        (float(period[0]), float(period[1])),
        np.concatenate(vert),
        np.concatenate(tri).astype(np.int32),
        np.concatenate(rwg).astype(np.int32),
        np.asarray(soff, dtype=np.int32),
        np.asarray(toff, dtype=np.int32),
        np.asarray(voff, dtype=np.int32),
        meshes,
    )


def unit_centre(u: int, L: int, period) -> np.ndarray:
    """Centre of unit u = iy*L + ix (row-major, Sec. III-C lattice)."""
    iy, ix = divmod(u, L)
    return np.array([ix * period[0], iy * period[1], 0.0])
