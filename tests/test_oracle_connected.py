"""Pins of the basis extension of periodic boundaries (Sec. III-B): coding
patches over a ground plane that is one connected plate.

The extended macro unit (the unit's patches, its ground cell, and the
bridging bases of its -x and -y cell edges whose second triangle lies in the
neighbouring cell) is the same in every unit, so displacement blocks Z(d)
serve the whole array; D_k masks the bridging bases of the -x and -y edge
units, which would reach outside the structure.  The pins:

* counts: the active bases of a codebook are as many as the RWGs of the
  physical structure (patches plus the interior edges of the whole plate,
  built on its own from the cells' meshes with merged vertices);
* the R3M identity: the product retrieved from Z(d) with the masks equals the
  product with the system matrix computed directly on the physical structure
  (bases matched by geometry: the same edge and triangles, up to the sign of
  the orientation), to 1e-12, on 1x1 to 3x3 and 3x2 arrays and four codebooks;
* a negative control: without the masks the counts disagree.
"""
import numpy as np
import pytest

from oracle import connected
from workloads import codebooks as cb
from workloads.mesh import connected_unit


@pytest.fixture(scope="module")
def cu():
    return connected_unit((0.006, 0.009))


@pytest.fixture(scope="module")
def blocks(cu, k10):
    return connected.displacement_blocks(cu, 2, 2, k10, extract=1)


def signature(tri_xyz, rwg_tri, rwg_edge_xyz):
    """Per basis: edge midpoint, and the centroids of T+ and T-."""
    mid = rwg_edge_xyz.mean(axis=1)
    cp = tri_xyz[rwg_tri[:, 0]].mean(axis=1)
    cm = tri_xyz[rwg_tri[:, 1]].mean(axis=1)
    return mid, cp, cm


def macro_placed(cu, active, Lx):
    """Signatures of the active bases of every unit, in reduced order."""
    p = cu.period[0]
    mids, cps, cms = [], [], []
    for u, idx in enumerate(active):
        iy, ix = divmod(u, Lx)
        mesh = connected.macro_mesh(cu, (ix, iy))
        off = np.array([ix * p, iy * p, 0.0])
        edge = cu.vert[cu.rwg[idx][:, 2:4]] + off
        m, a, b = signature(mesh.tri_xyz, mesh.rwg_tri[idx], edge)
        mids.append(m)
        cps.append(a)
        cms.append(b)
    return np.concatenate(mids), np.concatenate(cps), np.concatenate(cms)


def match(cu, active, Lx, structure, mesh):
    """perm[r] = physical basis of reduced entry r, sign[r] = +-1."""
    vert, tri, rwg, cell = structure
    pm, pp, pmm = signature(mesh.tri_xyz, mesh.rwg_tri, vert[rwg[:, 2:4]])
    mm, mp, mmm = macro_placed(cu, active, Lx)
    scale = cu.period[0]
    key = {tuple(np.round(v / scale * 1e6).astype(np.int64)): i for i, v in enumerate(pm)}
    perm = np.array([key[tuple(np.round(v / scale * 1e6).astype(np.int64))] for v in mm])
    same = np.all(np.abs(pp[perm] - mp) < 1e-9 * scale, axis=1) & np.all(np.abs(pmm[perm] - mmm) < 1e-9 * scale, axis=1)
    swap = np.all(np.abs(pp[perm] - mmm) < 1e-9 * scale, axis=1) & np.all(np.abs(pmm[perm] - mp) < 1e-9 * scale, axis=1)
    assert np.all(same | swap), "a basis matches no physical RWG"
    return perm, np.where(same, 1.0, -1.0)


def books(Lx, Ly):
    rng = np.random.default_rng(41 + 10 * Lx + Ly)
    return {
        "all0": np.zeros(Lx * Ly, np.uint8),
        "all1": np.ones(Lx * Ly, np.uint8),
        "checker": ((np.arange(Lx * Ly) % Lx + np.arange(Lx * Ly) // Lx) % 2).astype(np.uint8),
        "random": rng.integers(0, 2, Lx * Ly).astype(np.uint8),
    }


def test_unit_tables(cu):
    # 40 interior ground bases of a 4 x 4 cell, 4 bridges per edge
    assert cu.n_common == 48 and list(cu.ext).count(1) == 4 and list(cu.ext).count(2) == 4
    assert cu.n == 2 * 40 + 48
    # every bridge's second triangle is the neighbour's copy: in its cell
    # frame it lies on the far side of the cell edge
    p = cu.period[0]
    n_st = int(cu.state_off[-1])
    for c, e in enumerate(cu.ext):
        if e == 0:
            continue
        tp, tm = cu.rwg[n_st + c, 0:2]
        axis = e - 1
        assert np.all(cu.vert[cu.tri[tm], axis] <= -p / 2 + 1e-12)
        assert np.all(cu.vert[cu.tri[tp], axis] >= -p / 2 - 1e-12)
        assert tuple(cu.tri_cell[tm]) == ((-1, 0) if e == 1 else (0, -1))


@pytest.mark.parametrize("Lx,Ly", [(1, 1), (2, 2), (3, 3), (3, 2)])
@pytest.mark.parametrize("name", ["all0", "all1", "checker", "random"])
def test_r3m_identity_connected(cu, k10, blocks, Lx, Ly, name):
    states = books(Lx, Ly)[name]
    active = connected.active_sets(cu, states, Lx, Ly)
    Zd, mesh, structure = connected.direct_system(cu, states, Lx, Ly, k10)
    n_act = sum(len(a) for a in active)
    assert n_act == Zd.shape[0], (n_act, Zd.shape)
    perm, sign = match(cu, active, Lx, structure, mesh)
    assert len(set(perm.tolist())) == n_act
    x = cb.random_complex(n_act, 5 + Lx + 3 * Ly)
    y = connected.retrieved_matvec(blocks, 2, 2, active, Lx, Ly, x)
    # the same product on the physical bases: Z_direct acting on the matched entries
    xp = np.zeros(n_act, np.complex128)
    xp[perm] = sign * x
    y_ref = sign * (Zd @ xp)[perm]
    err = np.abs(y - y_ref).max() / np.abs(y_ref).max()
    assert err <= 1e-12, err


def test_masks_are_needed(cu):
    """Without the masks the edge units would carry bases the structure lacks."""
    Lx = Ly = 2
    states = np.zeros(4, np.uint8)
    active = connected.active_sets(cu, states, Lx, Ly)
    from workloads.mesh import connected_array_structure
    n_phys = len(connected_array_structure(cu, states, Lx, Ly)[2])
    unmasked = Lx * Ly * (cu.n_a + cu.n_common)
    assert sum(len(a) for a in active) == n_phys and unmasked == n_phys + 2 * Lx * 4


@pytest.mark.parametrize("Lx,Ly,name,theta_deg", [(2, 2, "checker", 0.0), (3, 2, "random", 30.0)])
def test_solve_and_rcs_match_physical_structure(cu, k10, blocks, Lx, Ly, name, theta_deg):
    """The retrieved pipeline on connected units (excitation P_k^T U with every
    basis integrated over its own triangles, the masked system, the RCS of
    P_k I) against the same pipeline run directly on the physical structure:
    the excitations agree entry by entry on the matched bases, the RCS to
    1e-10 (relative L2 over a 10-degree phi = 0 cut)."""
    import math

    from oracle import excitation, farfield, solve
    states = books(Lx, Ly)[name]
    th = math.radians(theta_deg)
    active = connected.active_sets(cu, states, Lx, Ly)
    Ur = connected.excitation(cu, active, Lx, Ly, k10, th, 0.0)
    Ir = solve.lu_solve(connected.retrieved_system(blocks, 2, 2, active, Lx, Ly), Ur)
    dirs = cb.phi0_cut(10.0)
    sr = connected.rcs(cu, active, Lx, Ly, Ir, k10, dirs)
    Zd, mesh, structure = connected.direct_system(cu, states, Lx, Ly, k10)
    Ud = excitation.plane_wave(mesh, k10, th, 0.0)
    sd = farfield.rcs(mesh, solve.lu_solve(Zd, Ud), k10, dirs)
    perm, sign = match(cu, active, Lx, structure, mesh)
    assert np.abs(Ur - sign * Ud[perm]).max() <= 1e-13 * np.abs(Ud).max()
    err = np.linalg.norm(sr - sd) / np.linalg.norm(sd)
    print(f"connected {Lx}x{Ly} {name} theta {theta_deg}: RCS retrieved vs physical {err:.1e}")
    assert err <= 1e-10
