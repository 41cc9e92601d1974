"""Low-rank compression of far displacement blocks: Z(d) ~ U V^H.

Admissible (far) blocks of the H-matrix are replaced by low-rank factors
built with adaptive cross approximation (Sec. II-B, ACA).  Because every far
block here is small (n <= 160) and is filled densely anyway, the oracle uses
the fully pivoted variant on the filled block:

  R_0 = Z
  repeat:  (i*, j*) = argmax |R|          (ties: lowest row-major index)
           u_k = R[:, j*],  v_k = conj(R[i*, :] / R[i*, j*])
           R  <- R - u_k v_k^H
  until ||R||_F <= tol ||Z||_F or rank == max_rank.

The stopping test uses the exact residual, so the achieved relative Frobenius
error is known and reported.  Factors are not unique; only products and errors
are comparable.
"""
import numpy as np


def aca_full(Z: np.ndarray, tol: float, max_rank: int):
    Z = np.asarray(Z, dtype=np.complex128)
    R = Z.copy()
    zn = np.linalg.norm(Z)
    us, vs = [], []
    err = np.linalg.norm(R) / zn if zn > 0 else 0.0
    while err > tol and len(us) < max_rank:
        flat = np.argmax(np.abs(R))
        i, j = divmod(int(flat), R.shape[1])
        piv = R[i, j]
        if piv == 0:
            break
        u = R[:, j].copy()
        v = np.conj(R[i, :] / piv)
        R -= np.outer(u, np.conj(v))
        us.append(u)
        vs.append(v)
        err = np.linalg.norm(R) / zn
    n, m = Z.shape
    U = np.array(us).T if us else np.zeros((n, 0), dtype=np.complex128)
    V = np.array(vs).T if vs else np.zeros((m, 0), dtype=np.complex128)
    return U, V, err


def svd_best_error(Z: np.ndarray, rank: int) -> float:
    """Eckart-Young: smallest relative Frobenius error of any rank-`rank` matrix."""
    s = np.linalg.svd(Z, compute_uv=False)
    return float(np.sqrt(np.sum(s[rank:] ** 2)) / np.sqrt(np.sum(s ** 2)))
