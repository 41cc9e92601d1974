"""Galerkin EFIE matrix on RWG bases, evaluated directly (FP64).

Eq. (1) of the paper, Z I = U, for PEC surfaces (Sec. II-A: EFIE, RWG bases,
Galerkin testing).  With the exp(+j w t) convention, Green's function
G(R) = exp(-j k R)/(4 pi R) and RWG functions f_m,

    Z_mn = j k eta  int_Tm int_Tn [ f_m . f_n - (1/k^2) div f_m  div' f_n ] G dS' dS .

An RWG function on triangles T+ / T- with free vertices v+ / v- and edge
length l is f = +(l/2A+)(r - v+) on T+, -(l/2A-)(r - v-) on T-; its
divergence is +l/A+ on T+, -l/A- on T-.

Both surface integrals use the 7-point rule.  For triangle pairs whose units
are within a Chebyshev radius `extract` of each other, G is split into
1/(4 pi R) (integrated in closed form over the source triangle, see
``singular``) plus the smooth remainder (exp(-j k R) - 1)/(4 pi R), whose
limit at R = 0 is -j k/(4 pi).

Overlapping coexistent meshes (Sec. III-A: the patches of different coding
states of one macro unit lie in one plane and overlap) make the closed-form
inner integral, seen as a function of the observation point, lose its
smoothness along the source triangle's edges, which then cross the interior
of the observer triangle.  For pairs of triangles of different coding states
in the same cell the outer integral therefore uses the composite rule: the
observer triangle split by three levels of midpoint subdivision into 64
congruent triangles, the 7-point rule on each (448 points).  Triangles of
the same state share whole edges (the usual case of the plain rule), and
one-hot retrieval never reads the cross-state entries; the relaxed codebook
of the differentiation path does.

The functions here take explicit geometry (triangles with unit coordinates),
so the same code builds both the direct active-only system Z_k of a codebook
(explicit retrieval, Sec. III-A) and the macro-unit displacement blocks Z(d).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import quadrature
from .constants import ETA0
from .singular import potential_integrals_paired


@dataclass
class RwgMesh:
    """Triangles with absolute coordinates plus an RWG table.

    tri_xyz : [T,3,3] vertex coordinates of every triangle
    tri_unit: [T,2]   integer (ix, iy) of the unit each triangle belongs to
    rwg_tri : [N,2]   (T+, T-) triangle ids
    rwg_free: [N,2]   local index (0..2) of the free vertex in T+ and in T-
    rwg_len : [N]     edge length
    tri_state: [T] or None  coding state whose patch holds the triangle, -1
              for triangles of bases shared by every state (None: no
              coexistent states, e.g. a physical array)
    """

    tri_xyz: np.ndarray
    tri_unit: np.ndarray
    rwg_tri: np.ndarray
    rwg_free: np.ndarray
    rwg_len: np.ndarray
    tri_state: np.ndarray | None = None

    @property
    def n(self) -> int:
        return len(self.rwg_len)


def rwg_mesh(vert, tri, rwg, offset=(0.0, 0.0, 0.0), unit=(0, 0), tri_cell=None, state_off=None) -> RwgMesh:
    """Build an RwgMesh from a connectivity table, translated by `offset`.

    Every triangle is in cell `unit`, shifted by tri_cell[t] when given (the
    neighbour-cell halves of bridging bases, Sec. III-B).  state_off (RWG
    ranges of the coding states of a macro unit, bases after the last range
    shared) gives each triangle the state of the bases it carries."""
    vert = np.asarray(vert, dtype=np.float64) + np.asarray(offset, dtype=np.float64)
    tri = np.asarray(tri)
    rwg = np.asarray(rwg)
    tri_xyz = vert[tri]
    free = np.zeros((len(rwg), 2), dtype=np.int64)
    for m, (tp, tm, e0, e1) in enumerate(rwg):
        for s, t in enumerate((tp, tm)):
            loc = [i for i in range(3) if tri[t, i] not in (e0, e1)]
            if len(loc) != 1:
                raise ValueError("RWG edge not on its triangle")
            free[m, s] = loc[0]
    elen = np.linalg.norm(vert[rwg[:, 2]] - vert[rwg[:, 3]], axis=1)
    tri_unit = np.tile(np.asarray(unit, dtype=np.int64), (len(tri), 1))
    if tri_cell is not None:
        tri_unit = tri_unit + np.asarray(tri_cell, dtype=np.int64)
    tri_state = None
    if state_off is not None:
        tri_state = np.full(len(tri), -1, dtype=np.int64)
        for s in range(len(state_off) - 1):
            for m in range(int(state_off[s]), int(state_off[s + 1])):
                for t in rwg[m, 0:2]:
                    if tri_state[t] not in (-1, s):
                        raise ValueError("triangle carries bases of two coding states")
                    tri_state[t] = s
    return RwgMesh(tri_xyz, tri_unit, rwg[:, 0:2].astype(np.int64), free, elen, tri_state)


def concat(meshes) -> RwgMesh:
    tri_off = np.cumsum([0] + [len(m.tri_xyz) for m in meshes])
    return RwgMesh(
        np.concatenate([m.tri_xyz for m in meshes]),
        np.concatenate([m.tri_unit for m in meshes]),
        np.concatenate([m.rwg_tri + tri_off[i] for i, m in enumerate(meshes)]),
        np.concatenate([m.rwg_free for m in meshes]),
        np.concatenate([m.rwg_len for m in meshes]),
        None if any(m.tri_state is None for m in meshes) else np.concatenate([m.tri_state for m in meshes]),
    )


def _smooth_remainder(kR, k):
    """(exp(-j k R) - 1)/(4 pi R) written without cancellation; -j k/(4 pi) at R = 0."""
    # exp(-jx) - 1 = -2 sin^2(x/2) - j sin x ;  divide by R = x/k
    s_half = np.sin(0.5 * kR)
    re = -k * s_half * np.sinc(kR / (2.0 * math.pi))
    im = -k * np.sinc(kR / math.pi)
    return (re + 1j * im) / (4.0 * math.pi)


def triangle_pair_integrals(obs: RwgMesh, src: RwgMesh, k: float, extract: int,
                            obs_sel=None, src_sel=None, src_chunk: int = 2048):
    """T[p,q,a,b] = int_p int_q [ (r - v_a).(r' - v_b)/4 - 1/k^2 ] G dS' dS.

    v_a is vertex a of observer triangle p, v_b vertex b of source triangle q.
    obs_sel / src_sel restrict the triangles (index arrays).
    """
    P_idx = np.arange(len(obs.tri_xyz)) if obs_sel is None else np.asarray(obs_sel)
    Q_idx = np.arange(len(src.tri_xyz)) if src_sel is None else np.asarray(src_sel)
    if len(Q_idx) > src_chunk:
        parts = [triangle_pair_integrals(obs, src, k, extract, P_idx, Q_idx[c:c + src_chunk], src_chunk)
                 for c in range(0, len(Q_idx), src_chunk)]
        return np.concatenate(parts, axis=1)
    to = obs.tri_xyz[P_idx]
    ts = src.tri_xyz[Q_idx]
    po, wo, _ = quadrature.points(to)  # [P,7,3], [P,7]
    ps, ws, _ = quadrature.points(ts)
    rho_o = po[:, :, None, :] - to[:, None, :, :]  # [P,7,3(vertex),3]
    rho_s = ps[:, :, None, :] - ts[:, None, :, :]  # [Q,7,3,3]

    uo = obs.tri_unit[P_idx]
    us = src.tri_unit[Q_idx]
    cheb = np.max(np.abs(uo[:, None, :] - us[None, :, :]), axis=2)  # [P,Q]
    ext = cheb <= extract

    # regular (or smooth-remainder) part, 7 x 7 points
    diff = po[:, None, :, None, :] - ps[None, :, None, :, :]  # [P,Q,7,7,3]
    R = np.sqrt(np.sum(diff * diff, axis=-1))
    kR = k * R
    with np.errstate(divide="ignore", invalid="ignore"):
        G_full = np.exp(-1j * kR) / (4.0 * math.pi * R)
    G = np.where(ext[:, :, None, None], _smooth_remainder(kR, k), G_full)
    Wg = G * wo[:, None, :, None] * ws[None, :, None, :]
    # A[p,q,a,b] = sum_ij Wg[p,q,i,j] (rho_o[p,i,a,:] . rho_s[q,j,b,:]), as two matmuls
    P, Q = Wg.shape[0], Wg.shape[1]
    X = np.matmul(Wg.transpose(1, 0, 2, 3).reshape(Q, P * 7, 7),
                  rho_s.reshape(Q, 7, 9).astype(np.complex128))  # [Q, P*7, (b,k)]
    X = X.reshape(Q, P, 7, 3, 3).transpose(1, 0, 3, 2, 4).reshape(P, Q * 3, 21)
    A = np.matmul(X, rho_o.transpose(0, 1, 3, 2).reshape(P, 21, 3).astype(np.complex128))
    A = A.reshape(P, Q, 3, 3).transpose(0, 1, 3, 2)  # [p,q,a,b]
    B = Wg.sum(axis=(2, 3))

    # closed-form 1/(4 pi R) part on the extracted pairs
    pp, qq = np.nonzero(ext)
    if len(pp):
        pts = po[pp].reshape(-1, 3)  # [E*7,3]
        tq = np.repeat(ts[qq], 7, axis=0)
        S, V = potential_integrals_paired(pts, tq)
        S = S.reshape(len(pp), 7)
        V = V.reshape(len(pp), 7, 3)
        # int_q (r' - v_b)/R dS' = V + (r - v_b) S
        inner = V[:, :, None, :] + (po[pp][:, :, None, :] - ts[qq][:, None, :, :]) * S[..., None, None]
        w = wo[pp] / (4.0 * math.pi)
        A[pp, qq] += np.einsum("ei,eiak,eibk->eab", w, rho_o[pp], inner, optimize=True)
        B[pp, qq] += np.einsum("ei,ei->e", w, S)

    T = A / 4.0 - B[:, :, None, None] / (k * k)
    # overlapping triangles of different coding states: the composite outer rule
    if obs.tri_state is not None and src.tri_state is not None:
        so = obs.tri_state[P_idx][:, None]
        ss = src.tri_state[Q_idx][None, :]
        pp, qq = np.nonzero(ext & (cheb == 0) & (so >= 0) & (ss >= 0) & (so != ss))
        for c in range(0, len(pp), 128):
            T[pp[c:c + 128], qq[c:c + 128]] = _overlap_pair_integrals(to[pp[c:c + 128]], ts[qq[c:c + 128]], k)
    return T


def _composite_rule(level: int):
    """Barycentric points [7 * 4^level, 3] and weights (summing to one) of the
    7-point rule on the 4^level triangles of `level` midpoint subdivisions."""
    bary, w = quadrature.seven_point()
    tris = [np.eye(3)]  # corners of each sub-triangle, in barycentric coordinates
    for _ in range(level):
        nxt = []
        for c in tris:
            m01, m12, m20 = (c[0] + c[1]) / 2, (c[1] + c[2]) / 2, (c[2] + c[0]) / 2
            nxt += [np.array([c[0], m01, m20]), np.array([m01, c[1], m12]),
                    np.array([m20, m12, c[2]]), np.array([m12, m20, m01])]
        tris = nxt
    pts = np.concatenate([bary @ c for c in tris])
    return pts, np.tile(w, len(tris)) / len(tris)


OVERLAP_LEVEL = 3


def _overlap_pair_integrals(tp: np.ndarray, tq: np.ndarray, k: float) -> np.ndarray:
    """T[e,a,b] (as triangle_pair_integrals) for paired triangles tp[e], tq[e]
    with the composite outer rule on tp; the inner integral over tq is the
    closed-form 1/(4 pi R) part plus the 7-point smooth remainder."""
    bary, wb = _composite_rule(OVERLAP_LEVEL)
    area = 0.5 * np.linalg.norm(np.cross(tp[:, 1] - tp[:, 0], tp[:, 2] - tp[:, 0]), axis=1)
    po = np.einsum("ia,ead->eid", bary, tp)  # [E,M,3]
    wo = area[:, None] * wb[None, :]  # [E,M]
    rho_o = po[:, :, None, :] - tp[:, None, :, :]  # [E,M,3(a),3]
    ps, ws, _ = quadrature.points(tq)  # [E,7,3], [E,7]
    rho_s = ps[:, :, None, :] - tq[:, None, :, :]  # [E,7,3(b),3]
    E, M = po.shape[0], po.shape[1]
    d = po[:, :, None, :] - ps[:, None, :, :]
    R = np.sqrt(np.sum(d * d, axis=-1))  # [E,M,7]
    Wg = _smooth_remainder(k * R, k) * wo[:, :, None] * ws[:, None, :]
    # inner[e,i,b,:] = int_q (r' - v_b) g dS' at outer point i: the 7-point sum
    # of the smooth remainder plus the closed-form 1/(4 pi R) part
    inner = np.matmul(Wg, rho_s.reshape(E, 7, 9).astype(np.complex128)).reshape(E, M, 3, 3)
    B = Wg.sum(axis=(1, 2))
    S, V = potential_integrals_paired(po.reshape(-1, 3), np.repeat(tq, M, axis=0))
    S = S.reshape(E, M)
    V = V.reshape(E, M, 3)
    w = wo / (4.0 * math.pi)
    inner = inner + w[:, :, None, None] * (V[:, :, None, :] + (po[:, :, None, :] - tq[:, None, :, :]) * S[..., None, None])
    B = B + np.sum(w * S, axis=1)
    # A[e,a,b] = sum_i rho_o[e,i,a,:] . inner[e,i,b,:]
    A = np.matmul(rho_o.transpose(0, 2, 1, 3).reshape(E, 3, M * 3),
                  inner.transpose(0, 1, 3, 2).reshape(E, M * 3, 3))
    return A / 4.0 - B[:, None, None] / (k * k)


def efie_matrix(obs: RwgMesh, src: RwgMesh, k: float, extract: int = 1,
                obs_rwg=None, chunk: int = 64) -> np.ndarray:
    """Z[m, n] for observer RWGs of `obs` (optionally a subset) and all RWGs of `src`."""
    m_idx = np.arange(obs.n) if obs_rwg is None else np.asarray(obs_rwg)
    Z = np.zeros((len(m_idx), src.n), dtype=np.complex128)
    area_o = quadrature.points(obs.tri_xyz)[2]
    area_s = quadrature.points(src.tri_xyz)[2]
    obs_tris = np.unique(obs.rwg_tri[m_idx].reshape(-1))
    sign = (1.0, -1.0)
    for c0 in range(0, len(obs_tris), chunk):
        tsel = obs_tris[c0:c0 + chunk]
        T = triangle_pair_integrals(obs, src, k, extract, obs_sel=tsel)  # [P,Qall,3,3]
        local = {int(t): i for i, t in enumerate(tsel)}
        for row, m in enumerate(m_idx):
            for a in range(2):
                p = int(obs.rwg_tri[m, a])
                if p not in local:
                    continue
                pa = local[p]
                alpha = obs.rwg_free[m, a]
                cm = sign[a] * obs.rwg_len[m] / area_o[p]
                for b in range(2):
                    q = src.rwg_tri[:, b]
                    beta = src.rwg_free[:, b]
                    cn = sign[b] * src.rwg_len / area_s[q]
                    Z[row] += cm * cn * T[pa, q, alpha, beta]
    return 1j * k * ETA0 * Z


# ----------------------------------------------------------------------------
# arrays of units


def active_array_mesh(unit, states, L: int) -> tuple[RwgMesh, np.ndarray]:
    """Mesh of only the active patches of a codebook (no macro unit).

    Returns the mesh and the unit index of every RWG.  Unit u = iy*L + ix sits
    at (ix*px, iy*py, 0); its RWGs are those of state states[u] in state order.
    """
    px, py = unit.period
    meshes, owner = [], []
    for u in range(L * L):
        iy, ix = divmod(u, L)
        pm = unit.states[int(states[u])]
        meshes.append(rwg_mesh(pm.vert, pm.tri, pm.rwg, (ix * px, iy * py, 0.0), (ix, iy)))
        owner.append(np.full(len(pm.rwg), u))
    return concat(meshes), np.concatenate(owner)


def macro_mesh(unit, cell=(0, 0)) -> RwgMesh:
    """The macro unit (union of all states) placed at lattice cell (ix, iy)."""
    px, py = unit.period
    ix, iy = cell
    return rwg_mesh(unit.vert, unit.tri, unit.rwg, (ix * px, iy * py, 0.0), (ix, iy), state_off=unit.state_off)


def direct_system(unit, states, L, k, extract=1, obs_units=None):
    """Explicitly retrieved system matrix Z_k on the active bases (Sec. III-A).

    If obs_units is given, only the rows of those observer units are returned
    (rows ordered by unit, then by RWG within the unit's active state).
    """
    mesh, owner = active_array_mesh(unit, states, L)
    rows = None
    if obs_units is not None:
        rows = np.concatenate([np.nonzero(owner == u)[0] for u in obs_units])
    return efie_matrix(mesh, mesh, k, extract, obs_rwg=rows)


def displacement_block(unit, dx: int, dy: int, k: float, extract: int = 1) -> np.ndarray:
    """Macro block Z(d) [n][n]: observer macro unit at lattice offset d = (dx, dy)
    from the source macro unit (rows = observer, cols = source)."""
    obs = macro_mesh(unit, (dx, dy))
    src = macro_mesh(unit, (0, 0))
    return efie_matrix(obs, src, k, extract)


def displacement_blocks(unit, Dx: int, Dy: int, k: float, extract: int = 1) -> np.ndarray:
    """All blocks for |dx| <= Dx, |dy| <= Dy, slot b = (dy+Dy)(2Dx+1) + (dx+Dx)."""
    out = np.zeros(((2 * Dx + 1) * (2 * Dy + 1), unit.n, unit.n), dtype=np.complex128)
    for dy in range(-Dy, Dy + 1):
        for dx in range(-Dx, Dx + 1):
            out[(dy + Dy) * (2 * Dx + 1) + (dx + Dx)] = displacement_block(unit, dx, dy, k, extract)
    return out
