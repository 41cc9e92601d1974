"""Solvers for the retrieved system Z_k I_k = U_k.

The paper solves the retrieved system with an MVP-based Krylov method
(Sec. III-A: direct LU cannot reuse the global matrix across codebooks;
Sec. IV uses BiCGStab).  The oracle keeps two plain solvers:
  * dense LU (numpy.linalg.solve), the reference solution;
  * restarted GMRES(m): zero initial guess, Arnoldi with modified Gram-Schmidt,
    complex Givens rotations on the Hessenberg matrix, stopping when the
    relative residual ||b - A x|| / ||b|| (recomputed explicitly at every
    restart and at exit) reaches tol.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def lu_solve(Z: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.linalg.solve(Z, b)


def givens(a: complex, b: complex):
    """c (real), s (complex), r with [[c, s], [-conj(s), c]] @ [a, b] = [r, 0]."""
    if b == 0:
        return 1.0, 0.0j, a
    if a == 0:
        return 0.0, 1.0 + 0.0j, b
    nu = np.hypot(abs(a), abs(b))
    ph = a / abs(a)
    return abs(a) / nu, ph * np.conj(b) / nu, ph * nu


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    rel_residual: float
    converged: bool
    history: list = field(default_factory=list)  # implicit residual estimates
    basis_orth_err: float = 0.0


def block_jacobi(Zk: np.ndarray, block: int):
    """Right preconditioner M^{-1} from the inverses of the diagonal unit blocks
    of the retrieved matrix (the diagonal-block case of the near-field
    preconditioner built after retrieval, Sec. III-D)."""
    nb = Zk.shape[0] // block
    inv = [np.linalg.inv(Zk[i * block:(i + 1) * block, i * block:(i + 1) * block]) for i in range(nb)]

    def apply(v):
        v = np.asarray(v).reshape(nb, block)
        return np.concatenate([inv[i] @ v[i] for i in range(nb)])
    return apply


def gmres(matvec, b: np.ndarray, tol: float = 1e-8, restart: int = 100,
          max_iter: int = 1000, precond=None) -> GmresResult:
    """Right-preconditioned when precond (x -> M^{-1} x) is given: the Krylov
    space is built for A M^{-1} and the iterate is x = M^{-1} u."""
    if precond is not None:
        res = gmres(lambda v: matvec(precond(v)), b, tol, restart, max_iter, None)
        # the unpreconditioned solution and its true residual
        res.x = precond_solution(res, precond)
        r = b - matvec(res.x)
        res.rel_residual = float(np.linalg.norm(r) / np.linalg.norm(b))
        return res
    b = np.asarray(b, dtype=np.complex128)
    n = len(b)
    bnorm = np.linalg.norm(b)
    x = np.zeros(n, dtype=np.complex128)
    if bnorm == 0:
        return GmresResult(x, 0, 0.0, True)
    hist = []
    it = 0
    orth = 0.0
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol or it >= max_iter:
            return GmresResult(x, it, beta / bnorm, beta / bnorm <= tol, hist, orth)
        m = min(restart, max_iter - it)
        V = np.zeros((n, m + 1), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[:, 0] = r / beta
        j_end = 0
        for j in range(m):
            w = matvec(V[:, j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[:, j + 1] = w / H[j + 1, j]
            for i in range(j):
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * hi + sn[i] * hi1
                H[i + 1, j] = -np.conj(sn[i]) * hi + cs[i] * hi1
            cs[j], sn[j], H[j, j] = givens(H[j, j], H[j + 1, j])
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or H[j, j] == 0:
                break
        Vm = V[:, : j_end + 1]
        orth = max(orth, np.abs(Vm.conj().T @ Vm - np.eye(j_end + 1)).max())
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + V[:, :j_end] @ y


def precond_solution(res: GmresResult, precond) -> np.ndarray:
    return precond(res.x)
