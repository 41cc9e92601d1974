"""Implicit retrieval of the codebook system from the macro-unit global matrix.

Sec. III-A: with every coding unit replaced by the macro unit, the array is
rigorously periodic and the global matrix Z (N macro bases) serves every
codebook.  For codebook k with slicing matrix P_k (N x N_k, one unit vector per
active basis):
    Z_k = P_k^T Z P_k                                     eq. (3)
    I = P_k I_k,  U = P_k U_k,  I_k = P_k^T I,  U_k = P_k^T U   eq. (4)
    D_k (.) (Z (D_k (.) I)) = D_k (.) U,  D_k = diag(P_k P_k^T)  eq. (6)

Periodicity makes the (unit i, unit j) block of Z depend only on the lattice
displacement d = i - j, so Z is stored as blocks Z(d) [n][n] (the finest 1x1
pattern of Sec. III-C, eq. (7): pattern = offset between two single units).
Block slot of d = (dx, dy): (dy + Dy)(2Dx + 1) + (dx + Dx).

Bases of unit u = iy*L + ix are ordered by state; state s occupies
[off[s], off[s+1]).  The reduced vector of a codebook is [unit][n_a] in unit
order, which is the column order of P_k.
"""
from __future__ import annotations

import numpy as np


def slot(dx: int, dy: int, Dx: int, Dy: int) -> int:
    return (dy + Dy) * (2 * Dx + 1) + (dx + Dx)


def active_index(states, state_off, L: int) -> np.ndarray:
    """Macro indices of the active bases, in P_k column order."""
    n = int(state_off[-1])
    idx = []
    for u in range(L * L):
        s = int(states[u])
        idx.append(u * n + np.arange(state_off[s], state_off[s + 1]))
    return np.concatenate(idx)


def slicing_matrix(states, state_off, L: int) -> np.ndarray:
    """P_k of eq. (3): N x N_k with a single 1 per column."""
    n = int(state_off[-1])
    idx = active_index(states, state_off, L)
    P = np.zeros((L * L * n, len(idx)))
    P[idx, np.arange(len(idx))] = 1.0
    return P


def indexing_vector(states, state_off, L: int) -> np.ndarray:
    """D_k of eq. (6): the diagonal of P_k P_k^T."""
    n = int(state_off[-1])
    D = np.zeros(L * L * n)
    D[active_index(states, state_off, L)] = 1.0
    return D


def macro_matrix(blocks: np.ndarray, Dx: int, Dy: int, L: int) -> np.ndarray:
    """Assemble the full global matrix Z (N x N) from displacement blocks (small L only)."""
    n = blocks.shape[1]
    Z = np.zeros((L * L * n, L * L * n), dtype=blocks.dtype)
    for i in range(L * L):
        iy, ix = divmod(i, L)
        for j in range(L * L):
            jy, jx = divmod(j, L)
            Z[i * n:(i + 1) * n, j * n:(j + 1) * n] = blocks[slot(ix - jx, iy - jy, Dx, Dy)]
    return Z


def hadamard_matvec(Zmacro: np.ndarray, D: np.ndarray, x_macro: np.ndarray) -> np.ndarray:
    """Left side of eq. (6) applied to a macro vector: D (.) (Z (D (.) x))."""
    return D * (Zmacro @ (D * x_macro))


def retrieved_matvec(blocks: np.ndarray, Dx: int, Dy: int, state_off, states, L: int,
                     x: np.ndarray) -> np.ndarray:
    """y_k = P_k^T Z P_k x_k in reduced coordinates, from displacement blocks.

    For each displacement d, every unit pair (i, j = i - d) inside the array
    contributes Z(d)[A(s_i), A(s_j)] x[j] to y[i].
    """
    states = np.asarray(states).astype(np.int64)
    off = np.asarray(state_off).astype(np.int64)
    n_a = int(off[1] - off[0])
    xr = np.asarray(x).reshape(L * L, n_a)
    y = np.zeros((L * L, n_a), dtype=np.result_type(blocks.dtype, xr.dtype))
    iy, ix = np.divmod(np.arange(L * L), L)
    ar = np.arange(n_a)
    for dy in range(-(L - 1), L):
        for dx in range(-(L - 1), L):
            jx, jy = ix - dx, iy - dy
            ok = (jx >= 0) & (jx < L) & (jy >= 0) & (jy < L)
            if not ok.any():
                continue
            I = np.nonzero(ok)[0]
            J = jy[ok] * L + jx[ok]
            Zd = blocks[slot(dx, dy, Dx, Dy)]
            rows = off[states[I]][:, None] + ar[None, :]  # [p, n_a]
            cols = off[states[J]][:, None] + ar[None, :]
            sub = Zd[rows[:, :, None], cols[:, None, :]]  # [p, n_a, n_a]
            y[I] += np.einsum("pab,pb->pa", sub, xr[J])
    return y.reshape(-1)


def lowrank_blocks(U: np.ndarray, V: np.ndarray, ranks: np.ndarray) -> np.ndarray:
    """Dense U V^H per block from factors [nb][n][r_max] with per-block ranks."""
    out = np.zeros((U.shape[0], U.shape[1], V.shape[1]), dtype=np.complex128)
    for b in range(U.shape[0]):
        r = int(ranks[b])
        out[b] = U[b, :, :r] @ np.conj(V[b, :, :r]).T
    return out
