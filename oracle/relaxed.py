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
