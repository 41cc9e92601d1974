"""Pins of the retrieval identities of Sec. III-A.

* eq. (3) / explicit slicing: P_k^T Z P_k equals Z(active, active);
* eq. (6): D_k (.) (Z (D_k (.) x)) equals P_k (Z_k x_k);
* the block-Toeplitz reduced matvec built from macro displacement blocks Z(d)
  equals the product with the system matrix computed *directly* on the active
  patches only (no macro unit) -- the R3M identity;
* special cases: a 1x1 array is the single patch; a uniform codebook is a plain
  periodic array;
* the inverse of the retrieved matrix is not the retrieval of the inverse.
"""
import numpy as np
import pytest

from oracle import efie, retrieval
from workloads import codebooks as cb


@pytest.fixture(scope="module")
def blocks3(unit1, k10):
    return efie.displacement_blocks(unit1, 2, 2, k10, extract=1)


def books(L):
    return {
        "all0": np.zeros(L * L, np.uint8),
        "all1": np.ones(L * L, np.uint8),
        "checker": cb.checkerboard(L, 1),
        "random": cb.bernoulli(L, 7),
    }


@pytest.mark.parametrize("L", [1, 2, 3])
@pytest.mark.parametrize("name", ["all0", "all1", "checker", "random"])
def test_r3m_identity(unit1, k10, blocks3, L, name):
    states = books(L)[name]
    Dx = 2
    # blocks for |d| <= L-1 are a sub-window of the 5x5 set
    sub = np.zeros(((2 * (L - 1) + 1) ** 2, unit1.n, unit1.n), np.complex128)
    for dy in range(-(L - 1), L):
        for dx in range(-(L - 1), L):
            sub[retrieval.slot(dx, dy, L - 1, L - 1)] = blocks3[retrieval.slot(dx, dy, Dx, Dx)]
    x = cb.random_complex(L * L * unit1.n_a, 11)
    y = retrieval.retrieved_matvec(sub, L - 1, L - 1, unit1.state_off, states, L, x)
    Zk = efie.direct_system(unit1, states, L, k10, extract=1)
    yref = Zk @ x
    assert np.abs(y - yref).max() <= 1e-12 * np.abs(yref).max()


def test_eq3_eq6_forms(unit1, k10, blocks3):
    L = 3
    states = cb.bernoulli(L, 3)
    Zm = retrieval.macro_matrix(blocks3, 2, 2, L)
    P = retrieval.slicing_matrix(states, unit1.state_off, L)
    D = retrieval.indexing_vector(states, unit1.state_off, L)
    idx = retrieval.active_index(states, unit1.state_off, L)
    Zk3 = P.T @ Zm @ P  # eq. (3)
    Zslice = Zm[np.ix_(idx, idx)]  # explicit retrieval
    assert np.array_equal(Zk3, Zslice)
    assert np.array_equal(np.diag(P @ P.T), D)
    xk = cb.random_complex(len(idx), 5)
    lhs6 = retrieval.hadamard_matvec(Zm, D, P @ xk)  # eq. (6) on a macro vector
    assert np.allclose(lhs6, P @ (Zk3 @ xk), rtol=0, atol=1e-14 * np.abs(lhs6).max())
    y = retrieval.retrieved_matvec(blocks3, 2, 2, unit1.state_off, states, L, xk)
    assert np.abs(y - Zk3 @ xk).max() <= 1e-14 * np.abs(y).max()
    # I = P_k I_k and I_k = P_k^T I (eq. (4))
    assert np.array_equal(P.T @ (P @ xk), xk)


def test_one_unit_is_single_patch(unit1, k10):
    from oracle.efie import rwg_mesh, efie_matrix
    for s in (0, 1):
        pm = unit1.states[s]
        Zp = efie_matrix(rwg_mesh(pm.vert, pm.tri, pm.rwg), rwg_mesh(pm.vert, pm.tri, pm.rwg), k10, 1)
        Z0 = efie.displacement_block(unit1, 0, 0, k10, 1)
        a = slice(unit1.state_off[s], unit1.state_off[s + 1])
        assert np.abs(Z0[a, a] - Zp).max() <= 1e-15 * np.abs(Zp).max()


def test_uniform_codebook_is_periodic_array(unit1, k10, blocks3):
    """All units in state 1: the retrieved matrix is the block-Toeplitz matrix of
    identical 9 mm patches; check its Toeplitz structure against the direct Z_k."""
    L = 3
    states = np.ones(L * L, np.uint8)
    Zk = efie.direct_system(unit1, states, L, k10, 1)
    na = unit1.n_a
    # block (i, j) depends only on i - j
    B = lambda i, j: Zk[i * na:(i + 1) * na, j * na:(j + 1) * na]
    assert np.abs(B(4, 3) - B(5, 4)).max() <= 1e-12 * np.abs(Zk).max()
    assert np.abs(B(8, 0) - blocks3[retrieval.slot(2, 2, 2, 2)][na:, na:]).max() <= 1e-12 * np.abs(Zk).max()


def test_inverse_of_retrieval_differs(unit1, k10, blocks3):
    """The inversion of the retrieved matrix differs from the retrieval of the
    inversion (Sec. III-D): a preconditioner must be built after retrieval."""
    L = 2
    sub = np.zeros((9, unit1.n, unit1.n), np.complex128)
    for dy in range(-1, 2):
        for dx in range(-1, 2):
            sub[retrieval.slot(dx, dy, 1, 1)] = blocks3[retrieval.slot(dx, dy, 2, 2)]
    Zm = retrieval.macro_matrix(sub, 1, 1, L)
    states = np.array([0, 1, 1, 0], np.uint8)
    idx = retrieval.active_index(states, unit1.state_off, L)
    a = np.linalg.inv(Zm[np.ix_(idx, idx)])
    b = np.linalg.inv(Zm)[np.ix_(idx, idx)]
    assert np.linalg.norm(a - b) > 1e-2 * np.linalg.norm(a)
