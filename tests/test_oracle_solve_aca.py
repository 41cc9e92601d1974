"""Pins of the oracle's GMRES and ACA.

GMRES: Arnoldi basis orthonormal to 1e-12, the implicit (Givens) residual is
non-increasing within a cycle and matches the explicit residual, and the
solution matches dense LU.  ACA: exact once the rank cap reaches n, achieved
error <= tol, and never better than the SVD optimum of the same rank
(Eckart-Young).
"""
import numpy as np
import pytest

from oracle import aca, efie, solve
from workloads import codebooks as cb


@pytest.fixture(scope="module")
def system(unit1, k10):
    states = cb.bernoulli(2, 12)
    Z = efie.direct_system(unit1, states, 2, k10, 1)
    b = cb.random_complex(Z.shape[0], 13)
    return Z, b


def test_gmres_matches_lu(system):
    Z, b = system
    res = solve.gmres(lambda v: Z @ v, b, tol=1e-12, restart=200, max_iter=400)
    assert res.converged
    x = solve.lu_solve(Z, b)
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x) * 1e2
    assert np.linalg.norm(b - Z @ res.x) <= 1e-12 * np.linalg.norm(b)
    h = np.array(res.history)
    assert np.all(np.diff(h) <= 1e-15)


def test_gmres_basis_orthonormal(system):
    """Before the residual becomes tiny, MGS keeps the Arnoldi basis orthonormal
    to rounding (it loses orthogonality only as the Krylov space saturates)."""
    Z, b = system
    res = solve.gmres(lambda v: Z @ v, b, tol=1e-14, restart=20, max_iter=20)
    assert res.basis_orth_err < 1e-12


def test_gmres_restart_and_cap(system):
    Z, b = system
    res = solve.gmres(lambda v: Z @ v, b, tol=1e-10, restart=10, max_iter=2000)
    assert res.converged and res.rel_residual <= 1e-10
    capped = solve.gmres(lambda v: Z @ v, b, tol=1e-14, restart=5, max_iter=3)
    assert not capped.converged and capped.iters == 3


def test_givens():
    for a, b in [(1 + 2j, 3 - 1j), (0.0, 2j), (1.5, 0.0)]:
        c, s, r = solve.givens(a, b)
        assert abs(c * a + s * b - r) < 1e-15 * abs(r)
        assert abs(-np.conj(s) * a + c * b) < 1e-15 * abs(r)
        assert abs(c * c + abs(s) ** 2 - 1) < 1e-15


@pytest.fixture(scope="module")
def far_block(unit1, k10):
    return efie.displacement_block(unit1, 4, 2, k10, 1)


def test_aca_exact_at_full_rank(far_block):
    U, V, err = aca.aca_full(far_block, 0.0, far_block.shape[0])
    assert np.linalg.norm(far_block - U @ V.conj().T) <= 1e-13 * np.linalg.norm(far_block)


@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-6])
def test_aca_tolerance_and_eckart_young(far_block, tol):
    U, V, err = aca.aca_full(far_block, tol, 80)
    r = U.shape[1]
    true = np.linalg.norm(far_block - U @ V.conj().T) / np.linalg.norm(far_block)
    assert abs(true - err) <= 1e-10
    assert err <= tol
    assert err >= aca.svd_best_error(far_block, r) * (1 - 1e-9)
    # a rank-capped run reports the error it achieved
    U2, V2, err2 = aca.aca_full(far_block, tol, max(1, r - 1))
    if r > 1:
        assert err2 > tol


def test_block_jacobi_gmres(unit1, k10):
    """Right block-Jacobi preconditioning (diagonal unit blocks of the
    retrieved matrix): same solution as LU, fewer iterations."""
    states = cb.bernoulli(3, 12)
    Z = efie.direct_system(unit1, states, 3, k10, 1)
    b = cb.random_complex(Z.shape[0], 2)
    M = solve.block_jacobi(Z, unit1.n_a)
    res_p = solve.gmres(lambda v: Z @ v, b, tol=1e-10, restart=100, max_iter=1000, precond=M)
    res = solve.gmres(lambda v: Z @ v, b, tol=1e-10, restart=100, max_iter=1000)
    x = solve.lu_solve(Z, b)
    assert res_p.converged and res_p.rel_residual <= 1e-9
    assert np.linalg.norm(res_p.x - x) <= 1e-7 * np.linalg.norm(x)
    assert res_p.iters < res.iters
    # M^{-1} applied to the diagonal blocks gives the identity
    e = np.zeros(Z.shape[0], complex)
    e[5] = 1.0
    blk = Z[:40, :40]
    assert np.allclose(M(np.concatenate([blk @ e[:40], np.zeros(Z.shape[0] - 40)]))[:40], e[:40], atol=1e-12)
