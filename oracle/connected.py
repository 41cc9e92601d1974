"""Connected geometries: the basis extension of periodic boundaries (Sec. III-B).

Test infrastructure: only the tests, the smoke check and the bench's CPU
baseline use this package; the GPU library never does.

A ground plane under the coding patches is a connected patch array.  Each
unit owns the bridging RWG bases of its -x and -y cell edges (their second
triangle lies in the neighbouring cell), which makes every unit identical
and the array rigorously periodic, so the displacement blocks Z(d) of the
extended macro unit serve every codebook exactly as for isolated patches.
The units on the array's -x (-y) boundary carry bridging bases that reach
outside the structure (the extended bases): D_k masks them with zeros, eq. (6).

Active bases of unit u = iy Lx + ix under codebook k (the columns of P_k):
  - its state's patch bases [state_off[s_u], state_off[s_u + 1]);
  - every ground basis with ext = 0 (cell interior);
  - the -x bridges (ext = 1) unless ix = 0, the -y bridges (ext = 2) unless
    iy = 0.
The reduced vector is ordered by unit, then by macro index.

Singularity extraction follows the physical cell of each triangle (a
bridge's neighbour half is in the neighbour's cell), the same rule as for
the direct system on the physical structure.

Excitation and RCS integrate every active basis over its own triangles where
they lie, so a bridge belongs to the unit that owns it and its outer half
needs no special case; the masked bases carry no current.
"""
from __future__ import annotations

import numpy as np

from .efie import RwgMesh, concat, efie_matrix, rwg_mesh
from .excitation import plane_wave
from .farfield import rcs as farfield_rcs
from .retrieval import slot


def macro_mesh(cu, cell=(0, 0)) -> RwgMesh:
    """The extended macro unit placed at lattice cell (ix, iy)."""
    p = cu.period[0]
    ix, iy = cell
    return rwg_mesh(cu.vert, cu.tri, cu.rwg, (ix * p, iy * p, 0.0), (ix, iy), cu.tri_cell, cu.state_off)


def displacement_blocks(cu, Dx: int, Dy: int, k: float, extract: int = 1) -> np.ndarray:
    """Z(d) [n][n] of the extended macro unit for |dx| <= Dx, |dy| <= Dy
    (observer unit at d from the source unit), in slot order."""
    out = np.zeros(((2 * Dx + 1) * (2 * Dy + 1), cu.n, cu.n), dtype=np.complex128)
    src = macro_mesh(cu, (0, 0))
    for dy in range(-Dy, Dy + 1):
        for dx in range(-Dx, Dx + 1):
            out[slot(dx, dy, Dx, Dy)] = efie_matrix(macro_mesh(cu, (dx, dy)), src, k, extract)
    return out


def active_sets(cu, states, Lx: int, Ly: int) -> list:
    """Macro indices of the active bases of every unit (D_k with the masks of
    the extended bases)."""
    n_st = int(cu.state_off[-1])
    out = []
    for u in range(Lx * Ly):
        iy, ix = divmod(u, Lx)
        s = int(states[u])
        idx = list(range(int(cu.state_off[s]), int(cu.state_off[s + 1])))
        for c, e in enumerate(cu.ext):
            if e == 0 or (e == 1 and ix > 0) or (e == 2 and iy > 0):
                idx.append(n_st + c)
        out.append(np.asarray(idx, dtype=np.int64))
    return out


def retrieved_matvec(blocks: np.ndarray, Dx: int, Dy: int, active: list, Lx: int, Ly: int,
                     x: np.ndarray) -> np.ndarray:
    """y = P_k^T Z P_k x in reduced coordinates (unit by unit, active bases in
    macro order): every unit pair (i, j) adds Z(i - j)[A_i, A_j] x_j to y_i."""
    offs = np.cumsum([0] + [len(a) for a in active])
    y = np.zeros(offs[-1], dtype=np.complex128)
    for i in range(Lx * Ly):
        iy, ix = divmod(i, Lx)
        for j in range(Lx * Ly):
            jy, jx = divmod(j, Lx)
            Zd = blocks[slot(ix - jx, iy - jy, Dx, Dy)]
            y[offs[i]:offs[i + 1]] += Zd[np.ix_(active[i], active[j])] @ x[offs[j]:offs[j + 1]]
    return y


def direct_system(cu, states, Lx: int, Ly: int, k: float, extract: int = 1):
    """Z_k on the physical structure (active patches plus the whole ground
    plate, no macro unit), with the structure's own RWG numbering.  Returns
    (Z, mesh, (vert, tri, rwg, tri_cell))."""
    from workloads.mesh import connected_array_structure
    vert, tri, rwg, cell = connected_array_structure(cu, states, Lx, Ly)
    mesh = rwg_mesh(vert, tri, rwg, (0.0, 0.0, 0.0), (0, 0), cell)
    return efie_matrix(mesh, mesh, k, extract), mesh, (vert, tri, rwg, cell)


def array_mesh(cu, Lx: int, Ly: int) -> RwgMesh:
    """The extended macro units of every cell, concatenated in unit order
    (macro index u n + m)."""
    return concat([macro_mesh(cu, (u % Lx, u // Lx)) for u in range(Lx * Ly)])


def retrieved_system(blocks: np.ndarray, Dx: int, Dy: int, active: list, Lx: int, Ly: int) -> np.ndarray:
    """P_k^T Z P_k as a dense matrix in reduced coordinates (eq. (6) with the
    masks of the extended bases)."""
    offs = np.cumsum([0] + [len(a) for a in active])
    Z = np.zeros((offs[-1], offs[-1]), dtype=np.complex128)
    for i in range(Lx * Ly):
        iy, ix = divmod(i, Lx)
        for j in range(Lx * Ly):
            jy, jx = divmod(j, Lx)
            Zd = blocks[slot(ix - jx, iy - jy, Dx, Dy)]
            Z[offs[i]:offs[i + 1], offs[j]:offs[j + 1]] = Zd[np.ix_(active[i], active[j])]
    return Z


def excitation(cu, active: list, Lx: int, Ly: int, k: float, theta: float = 0.0, phi: float = 0.0,
               e0: float = 1.0) -> np.ndarray:
    """P_k^T U: the plane-wave excitation of every unit's active bases, each
    integrated over its own triangles where they lie (a bridge's outer half in
    the neighbouring cell), in reduced order."""
    out = []
    for u, idx in enumerate(active):
        U = plane_wave(macro_mesh(cu, (u % Lx, u // Lx)), k, theta, phi, e0)
        out.append(U[idx])
    return np.concatenate(out)


def rcs(cu, active: list, Lx: int, Ly: int, I: np.ndarray, k: float, thph: np.ndarray,
        e0: float = 1.0) -> np.ndarray:
    """Bistatic RCS of the reduced current I: P_k I placed on the macro bases
    of the array (masked and inactive bases carry no current)."""
    n = cu.n
    Imac = np.zeros(Lx * Ly * n, dtype=np.complex128)
    offs = np.cumsum([0] + [len(a) for a in active])
    for u, idx in enumerate(active):
        Imac[u * n + idx] = I[offs[u]:offs[u + 1]]
    return farfield_rcs(array_mesh(cu, Lx, Ly), Imac, k, thph, e0)
