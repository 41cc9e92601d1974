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


# ----------------------------------------------------------------------------
# connected geometries: a ground plane under the coding patches
#
# Sec. III-B (basis extension of periodic boundaries): a ground plane is a
# connected patch array.  Its RWG bases on the edges between two cells bridge
# two units and are ascribed to one of them, here the unit on the +x (+y)
# side of the edge: every unit owns the bridging bases of its -x and -y cell
# edges, whose second triangle lies in the neighbouring cell.  The unit is
# then rigorously periodic.  At the array's -x (-y) boundary those bases
# would reach outside the structure: they are the extended bases, present in
# the macro unit and masked out by D_k for the edge units.


@dataclass
class ConnectedUnit:
    """Extended macro unit: the coding patches at z = height over one cell of
    a ground plane at z = 0, with the bridging bases of the -x and -y cell
    edges.

    Basis order: the states' patch bases in state order ([state_off[s],
    state_off[s+1])), then the n_common ground bases: cell-interior ones,
    then the -x bridges (by y), then the -y bridges (by x).  ext[c] for
    ground basis c is 0 (interior), 1 (-x bridge) or 2 (-y bridge).
    tri_cell[t] is the lattice offset of the cell triangle t lies in: (0, 0),
    or (-1, 0) / (0, -1) for the neighbour halves of the bridges.
    """

    patches: MacroUnit
    height: float
    ground: PatchMesh
    period: tuple
    vert: np.ndarray
    tri: np.ndarray
    rwg: np.ndarray
    tri_cell: np.ndarray
    state_off: np.ndarray
    ext: np.ndarray

    @property
    def n_states(self) -> int:
        return self.patches.n_states

    @property
    def n_a(self) -> int:
        return self.patches.n_a

    @property
    def n_common(self) -> int:
        return len(self.ext)

    @property
    def n(self) -> int:
        return len(self.rwg)


def _boundary_edges(pm: PatchMesh):
    """Edges of a patch mesh with one triangle: {(v0, v1): triangle}."""
    cnt: dict[tuple[int, int], list[int]] = {}
    for t, (a, b, c) in enumerate(pm.tri):
        for p, q in ((a, b), (b, c), (c, a)):
            cnt.setdefault((min(p, q), max(p, q)), []).append(t)
    return {e: ts[0] for e, ts in cnt.items() if len(ts) == 1}


def connected_unit(sides, height: float = 0.0015, ncell: int = 4, ground_ncell: int = 4,
                   period: float = 0.015) -> ConnectedUnit:
    patches = macro_unit(sides, ncell, (period, period))
    ground = patch_mesh(period, ground_ncell)
    half = period / 2.0
    tol = 1e-9 * period
    bnd = _boundary_edges(ground)

    def side_edges(axis, value):
        out = []
        for (a, b), t in bnd.items():
            if abs(ground.vert[a, axis] - value) < tol and abs(ground.vert[b, axis] - value) < tol:
                lo = min(ground.vert[a, 1 - axis], ground.vert[b, 1 - axis])
                out.append((lo, a, b, t))
        return sorted(out)

    pv = patches.vert.copy()
    pv[:, 2] = height
    nv_p, nt_p = len(pv), len(patches.tri)
    vert = [pv, ground.vert]
    tri = [patches.tri, ground.tri + nv_p]
    rwg = [patches.rwg]
    g = ground.rwg.copy()
    g[:, 0:2] += nt_p
    g[:, 2:4] += nv_p
    rwg.append(g)
    ext = [np.zeros(len(ground.rwg), dtype=np.int32)]
    tri_cell = [np.zeros((nt_p + len(ground.tri), 2), dtype=np.int32)]
    extra_v, extra_t, bridges, cells = [], [], [], []
    nv_next = nv_p + len(ground.vert)
    nt_next = nt_p + len(ground.tri)
    for axis, flag in ((0, 1), (1, 2)):
        shift = np.zeros(3)
        shift[axis] = -period
        minus = side_edges(axis, -half)  # this cell's -x (-y) edges
        plus = {round(lo / tol): (a, b, t) for lo, a, b, t in side_edges(axis, +half)}
        for lo, a, b, t in minus:
            pa, pb, pt = plus[round(lo / tol)]
            free = [v for v in ground.tri[pt] if v not in (pa, pb)][0]
            extra_v.append(ground.vert[free] + shift)  # the neighbour's triangle, translated
            extra_t.append((a + nv_p, b + nv_p, nv_next))
            nv_next += 1
            c = np.zeros(2, dtype=np.int32)
            c[axis] = -1
            cells.append(c)
            bridges.append((t + nt_p, nt_next, min(a, b) + nv_p, max(a, b) + nv_p))
            nt_next += 1
            ext.append(np.array([flag], dtype=np.int32))
    vert.append(np.asarray(extra_v).reshape(-1, 3))
    tri.append(np.asarray(extra_t, dtype=np.int32).reshape(-1, 3))
    tri_cell.append(np.asarray(cells, dtype=np.int32).reshape(-1, 2))
    rwg.append(np.asarray(bridges, dtype=np.int32).reshape(-1, 4))
    return ConnectedUnit(patches, float(height), ground, (float(period), float(period)),
                         np.concatenate(vert), np.concatenate(tri).astype(np.int32),
                         np.concatenate(rwg).astype(np.int32), np.concatenate(tri_cell),
                         patches.state_off.copy(), np.concatenate(ext))


def connected_array_structure(cu: ConnectedUnit, states, Lx: int, Ly: int):
    """The physical structure of a codebook on an Lx x Ly array, built on its
    own (no macro unit): the active patch of every unit at z = height, and the
    ground plane of the whole array as one plate meshed cell by cell (vertices
    merged by position) with an RWG on every interior edge of the plate.

    Returns (vert, tri, rwg, tri_cell): rwg rows {T+, T-, v0, v1} with T+ the
    lower triangle id, tri_cell the lattice cell (ix, iy) of every triangle.
    Patch RWGs come first, unit by unit; then the plate's, by edge.
    """
    px = cu.period[0]
    vert, tri, rwg, cell = [], [], [], []
    nv = nt = 0
    for u in range(Lx * Ly):
        iy, ix = divmod(u, Lx)
        pm = cu.patches.states[int(states[u])]
        v = pm.vert + np.array([ix * px, iy * px, cu.height])
        vert.append(v)
        tri.append(pm.tri + nv)
        r = pm.rwg.copy()
        r[:, 0:2] += nt
        r[:, 2:4] += nv
        rwg.append(r)
        cell.append(np.tile([ix, iy], (len(pm.tri), 1)))
        nv += len(v)
        nt += len(pm.tri)
    # the plate: merge the cells' ground vertices by position
    h = px / cu.ground.ncell
    key_of, gvert, gtri, gcell = {}, [], [], []
    for iy in range(Ly):
        for ix in range(Lx):
            ids = []
            for p in cu.ground.vert + np.array([ix * px, iy * px, 0.0]):
                key = (int(round(p[0] / h * 2)), int(round(p[1] / h * 2)))
                if key not in key_of:
                    key_of[key] = len(gvert)
                    gvert.append(p)
                ids.append(key_of[key])
            ids = np.asarray(ids)
            for t in cu.ground.tri:
                gtri.append(ids[t])
                gcell.append((ix, iy))
    gtri = np.asarray(gtri)
    edges: dict[tuple[int, int], list[int]] = {}
    for t, (a, b, c) in enumerate(gtri):
        for p, q in ((a, b), (b, c), (c, a)):
            edges.setdefault((min(p, q), max(p, q)), []).append(t)
    grwg = [(min(ts) + nt, max(ts) + nt, e[0] + nv, e[1] + nv) for e, ts in sorted(edges.items()) if len(ts) == 2]
    vert.append(np.asarray(gvert))
    tri.append(gtri + nv)
    rwg.append(np.asarray(grwg, dtype=np.int64).reshape(-1, 4))
    cell.append(np.asarray(gcell))
    return (np.concatenate(vert), np.concatenate(tri).astype(np.int64), np.concatenate(rwg).astype(np.int64),
            np.concatenate(cell).astype(np.int64))
