"""Relaxed (blended) retrieval for codebook differentiation.

Test infrastructure: the CPU FP64 definition that the GPU relaxed matvec is
checked against; nothing on the product path imports it.

A relaxed codebook gives every unit u real state weights w[u][s] (e.g. a
softmax of logits) instead of one state.  The slicing matrix P_k of eq. (3)
(one unit vector per active basis) becomes the non-square blend
    P(w) = blockdiag_u [w[u][0] I; w[u][1] I; ...; w[u][S-1] I]   (n x n_a per unit)
so column (u, r) carries weight w[u][s] on macro row (u, off[s] + r) for every
state s, and
    Z_k(w) = P(w)^T Z P(w),     U_k(w) = P(w)^T U,     I = P(w) I_k(w).
For one-hot weights P(w) = P_k and this is eq. (3).  (A diagonal relaxation
of eq. (6)'s mask D_k would leave D I = Z^-1 U independent of the weights, so
the blend acts on the non-square P instead.)  The adjoint of a solve with
Z_k(w) uses the transposed operator Z_k(w)^T = P(w)^T Z^T P(w).

Two forms are written out: the matrix form from the assembled global matrix,
and a loop over unit pairs, y_i = sum_j sum_{s,s'} w[i][s] w[j][s']
Z(i - j)[A(s), A(s')] x_j, which shares no code with the first.
"""
from __future__ import annotations

import numpy as np

from .retrieval import macro_matrix, slot


def blend_matrix(weights: np.ndarray, state_off, L: int) -> np.ndarray:
    """P(w): [L*L*n] x [L*L*n_a]; weights [L*L][S]."""
    off = np.asarray(state_off, dtype=np.int64)
    S = len(off) - 1
    n_a = int(off[1] - off[0])
    n = int(off[-1])
    w = np.asarray(weights, dtype=np.float64).reshape(L * L, S)
    P = np.zeros((L * L * n, L * L * n_a))
    for u in range(L * L):
        for s in range(S):
            for r in range(n_a):
                P[u * n + off[s] + r, u * n_a + r] = w[u, s]
    return P


def relaxed_matvec(blocks: np.ndarray, Dx: int, Dy: int, state_off, weights: np.ndarray, L: int,
                   x: np.ndarray, transpose: bool = False) -> np.ndarray:
    """y = P(w)^T Z P(w) x (or with Z^T), matrix form (small L only)."""
    Z = macro_matrix(blocks, Dx, Dy, L)
    if transpose:
        Z = Z.T
    P = blend_matrix(weights, state_off, L)
    return P.T @ (Z @ (P @ np.asarray(x)))


def relaxed_matvec_pairs(blocks: np.ndarray, Dx: int, Dy: int, state_off, weights: np.ndarray, L: int,
                         x: np.ndarray, transpose: bool = False) -> np.ndarray:
    """The same product as a loop over unit pairs and state pairs.  With
    transpose the (i, j) block is Z(j - i)^T, the transpose of Z's (j, i)."""
    off = np.asarray(state_off, dtype=np.int64)
    S = len(off) - 1
    n_a = int(off[1] - off[0])
    w = np.asarray(weights, dtype=np.float64).reshape(L * L, S)
    xr = np.asarray(x).reshape(L * L, n_a)
    y = np.zeros((L * L, n_a), dtype=np.result_type(blocks.dtype, xr.dtype))
    for i in range(L * L):
        iy, ix = divmod(i, L)
        for j in range(L * L):
            jy, jx = divmod(j, L)
            blk = blocks[slot(jx - ix, jy - iy, Dx, Dy)].T if transpose else blocks[slot(ix - jx, iy - jy, Dx, Dy)]
            for s in range(S):
                for t in range(S):
                    sub = blk[off[s]:off[s] + n_a, off[t]:off[t] + n_a]
                    y[i] += w[i, s] * w[j, t] * (sub @ xr[j])
    return y.reshape(-1)


# ------------------------------------------------------------ objective
#
# The differentiation workload: incident plane wave, blended current
# I~ = P(w) I_k(w) on the macro array (every state's patch of every unit,
# the coexistent meshes of Sec. III-A), objective J(w) = mean bistatic RCS
# over a direction set.  Its gradient follows from one adjoint solve with
# Z_k(w)^T: with G = dJ/dI~ (Wirtinger derivative, I~* held fixed),
#   Z_k(w)^T lam = P(w)^T G,   lam~ = P(w) lam,
#   dJ/dw[u][s] = 2 Re sum_r [ (G - Z^T lam~)[u][s][r] I[u][r]
#                              + lam[u][r] (U - Z I~)[u][s][r] ],
# where [u][s][r] is macro row off[s] + r of unit u (derivation: dI~ = dP I +
# P dI, dI = Z_k^-1 (dP^T U - dP^T Z I~ - P^T Z dP I)).


def macro_array_mesh(unit, L: int):
    """Every state's patch of every unit, macro order [unit][n] (n in state order)."""
    from .efie import concat, macro_mesh
    return concat([macro_mesh(unit, (u % L, u // L)) for u in range(L * L)])


def relaxed_objective(unit, blocks: np.ndarray, D: int, weights: np.ndarray, L: int, k: float, thph: np.ndarray,
                      theta: float = 0.0, phi: float = 0.0, e0: float = 1.0, with_grad: bool = False):
    """J(w) = mean_d sigma_d of the blended current, by dense LU (small L);
    with_grad also returns dJ/dw [L*L][S] by the adjoint formula above."""
    from . import excitation, farfield
    from .constants import ETA0
    mesh = macro_array_mesh(unit, L)
    Umac = excitation.plane_wave(mesh, k, theta, phi, e0)
    Z = macro_matrix(blocks, D, D, L)
    P = blend_matrix(weights, unit.state_off, L)
    A = P.T @ Z @ P
    I = np.linalg.solve(A, P.T @ Umac)
    It = P @ I
    sigma = farfield.rcs(mesh, It, k, thph, e0)
    J = float(sigma.mean())
    if not with_grad:
        return J, sigma, I
    rhat = farfield.directions(thph)
    F, _ = farfield.rwg_transforms(mesh, k, rhat)  # [N][dir][3]
    N = np.einsum("n,ndc->dc", It, F)
    Np = N - np.sum(N * rhat, axis=1, keepdims=True) * rhat
    scale = k * k * ETA0 ** 2 / (4.0 * np.pi) / abs(e0) ** 2
    G = scale / len(thph) * np.einsum("dc,ndc->n", np.conj(Np), F)
    lam = np.linalg.solve(A.T, P.T @ G)
    Q = Z.T @ (P @ lam)
    R = Umac - Z @ It
    off = np.asarray(unit.state_off)
    S = len(off) - 1
    n_a = int(off[1] - off[0])
    n = int(off[-1])
    grad = np.zeros((L * L, S))
    for u in range(L * L):
        Iu, lu = I[u * n_a:(u + 1) * n_a], lam[u * n_a:(u + 1) * n_a]
        for s in range(S):
            rows = slice(u * n + off[s], u * n + off[s] + n_a)
            grad[u, s] = 2.0 * np.real(np.sum((G[rows] - Q[rows]) * Iu) + np.sum(lu * R[rows]))
    return J, sigma, I, grad
