"""Near-field block incomplete-LU preconditioner of a retrieved codebook system
(TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use this module).

Sec. III-D preconditions the retrieved system with an incomplete LU of its
near field, factored per codebook after retrieval: the inverse of a retrieved
matrix is not the retrieval of an inverse, so no factor can be shared across
codebooks.  The paper does not fix the pattern, the fill level or the unit
order.  The readings taken here:

  * blocks are whole units (n_a x n_a); the pattern holds the unit pairs at
    Chebyshev lattice distance <= r (r = 1: the unit and its 8 neighbours);
  * no fill outside the pattern (block ILU(0)); pivot blocks inverted exactly;
  * multicolour unit order: unit (ix, iy) has colour
    (iy mod (r + 1)) (r + 1) + (ix mod (r + 1)), units are taken by colour,
    then by index.  Two units of one colour are never in each other's
    pattern, so the order inside a colour changes nothing, and each colour is
    one parallel step of the factorisation and of both triangular solves.

With P the unit order, the factorisation is A ~ L U with L unit block-lower
and U block-upper in that order, and (L U)_ij = A_ij on every pattern pair
(the defining property of ILU(0)).  The preconditioner is M^-1 v = U^-1 L^-1 v.
"""
from __future__ import annotations

import numpy as np


def colour(ix: int, iy: int, r: int) -> int:
    return (iy % (r + 1)) * (r + 1) + (ix % (r + 1))


def unit_order(Lx: int, Ly: int, r: int) -> list:
    """Units (u = iy Lx + ix) by colour, then by index."""
    return sorted(range(Lx * Ly), key=lambda u: (colour(u % Lx, u // Lx, r), u))


def pattern(u: int, Lx: int, Ly: int, r: int) -> list:
    """Units at Chebyshev distance <= r from unit u (u itself included)."""
    iy, ix = divmod(u, Lx)
    return [(iy + dy) * Lx + ix + dx for dy in range(-r, r + 1) for dx in range(-r, r + 1)
            if 0 <= ix + dx < Lx and 0 <= iy + dy < Ly]


def block_ilu0(A: np.ndarray, Lx: int, Ly: int, n_a: int, r: int, order=None) -> dict:
    """Block ILU(0) of the retrieved matrix A ([unit][n_a] ordering) on the
    radius-r pattern, in multicolour order unless `order` (a permutation of
    the units) is given (row by row: each earlier pattern block of a row is
    turned into its multiplier, then removed from the rest of the row where
    the pattern allows).

    Returns {"L": {(i, k): L_ik}, "U": {(i, j): U_ij}, "Dinv": {i: U_ii^-1},
    "order", "pos", "r", "Lx", "Ly", "n_a"} with unit indices i, j, k."""
    U_n = Lx * Ly
    order = unit_order(Lx, Ly, r) if order is None else list(order)
    pos = {u: p for p, u in enumerate(order)}

    def blk(i, j):
        return np.array(A[i * n_a:(i + 1) * n_a, j * n_a:(j + 1) * n_a], dtype=np.complex128)

    row = {i: {j: blk(i, j) for j in pattern(i, Lx, Ly, r)} for i in range(U_n)}
    Dinv = {}
    for i in order:
        earlier = sorted((k for k in row[i] if pos[k] < pos[i]), key=lambda k: pos[k])
        for k in earlier:
            row[i][k] = row[i][k] @ Dinv[k]                # multiplier L_ik
            for j in row[i]:
                if pos[j] > pos[k] and j in row[k]:         # pattern pair (k, j) of the later part of row k
                    row[i][j] = row[i][j] - row[i][k] @ row[k][j]
        Dinv[i] = np.linalg.inv(row[i][i])
    Lf = {(i, k): row[i][k] for i in range(U_n) for k in row[i] if pos[k] < pos[i]}
    Uf = {(i, j): row[i][j] for i in range(U_n) for j in row[i] if pos[j] >= pos[i]}
    return {"L": Lf, "U": Uf, "Dinv": Dinv, "order": order, "pos": pos, "r": r, "Lx": Lx, "Ly": Ly, "n_a": n_a}


def ilu_apply(f: dict, v: np.ndarray) -> np.ndarray:
    """M^-1 v: forward substitution with the unit lower factor, then backward
    substitution with the upper one, unit by unit in the factor's order."""
    n_a, order, pos = f["n_a"], f["order"], f["pos"]
    v = np.asarray(v, dtype=np.complex128).reshape(-1, n_a)
    z = np.zeros_like(v)
    for i in order:
        t = v[i].copy()
        for (ii, k), Lik in f["L"].items():
            if ii == i:
                t -= Lik @ z[k]
        z[i] = t
    x = np.zeros_like(v)
    for i in reversed(order):
        t = z[i].copy()
        for (ii, j), Uij in f["U"].items():
            if ii == i and j != i:
                t -= Uij @ x[j]
        x[i] = f["Dinv"][i] @ t
    return x.reshape(-1)


def dense_factors(f: dict):
    """The factors as dense matrices in unit ordering: L (identity diagonal
    blocks) and U (pivot blocks U_ii on the diagonal), M = L U."""
    n_a, U_n = f["n_a"], f["Lx"] * f["Ly"]
    L = np.eye(U_n * n_a, dtype=np.complex128)
    U = np.zeros((U_n * n_a, U_n * n_a), dtype=np.complex128)
    for (i, k), b in f["L"].items():
        L[i * n_a:(i + 1) * n_a, k * n_a:(k + 1) * n_a] = b
    for (i, j), b in f["U"].items():
        U[i * n_a:(i + 1) * n_a, j * n_a:(j + 1) * n_a] = b
    return L, U


def slot_blocks(f: dict) -> np.ndarray:
    """Factors per unit and neighbour offset: out[u][(ey + r)(2r + 1) + ex + r]
    is L_uj (j earlier), U_uj (j later) or, at e = 0, U_uu^-1, for the unit j
    at offset e = (ex, ey) from u; zero where j lies outside the array."""
    r, Lx, Ly, n_a = f["r"], f["Lx"], f["Ly"], f["n_a"]
    S = 2 * r + 1
    out = np.zeros((Lx * Ly, S * S, n_a, n_a), dtype=np.complex128)
    for u in range(Lx * Ly):
        iy, ix = divmod(u, Lx)
        for ey in range(-r, r + 1):
            for ex in range(-r, r + 1):
                jx, jy = ix + ex, iy + ey
                if not (0 <= jx < Lx and 0 <= jy < Ly):
                    continue
                j = jy * Lx + jx
                s = (ey + r) * S + ex + r
                out[u, s] = f["Dinv"][u] if j == u else (f["L"][(u, j)] if (u, j) in f["L"] else f["U"][(u, j)])
    return out
