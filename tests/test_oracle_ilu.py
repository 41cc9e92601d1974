"""Pins of the near-field block ILU(0) oracle (preconditioner of Sec. III-D).

  * a pattern that covers every unit pair drops nothing: the factors are a
    complete block LU, so L U reproduces A and M^-1 (A x) = x (a wrong sign,
    index or operand order anywhere in the elimination breaks this);
  * on a partial pattern, (L U)_ij = A_ij on every pattern pair (the
    defining property of ILU(0)) while fill outside it is dropped;
  * the triangular solves equal a dense solve with L U;
  * radius 0 is block-Jacobi (the solver oracle's own block inverses);
  * reordering units inside a colour leaves every factor unchanged, the
    property the parallel colour steps rely on;
  * on a retrieved EFIE near field the preconditioner beats block-Jacobi in
    GMRES iterations (a behaviour check of the paper's claim, not a pin).
"""
import numpy as np
import pytest

from oracle import efie, ilu, retrieval, solve
from oracle.constants import wavenumber
from workloads import codebooks as cb
from workloads.mesh import macro_unit

K = wavenumber(10.0e9)


def random_system(Lx, Ly, n_a, seed):
    rng = np.random.default_rng(seed)
    N = Lx * Ly * n_a
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    return A + 2.0 * N ** 0.5 * np.eye(N)


def retrieved_near(L, r, states, seed_unit=(0.006, 0.009)):
    """Retrieved blocks Z(p_i - p_j)[A(s_i), A(s_j)] of an L x L codebook for
    unit pairs at Chebyshev distance <= r (zero elsewhere), and n_a."""
    unit = macro_unit(seed_unit)
    blocks = efie.displacement_blocks(unit, r, r, K, extract=1)
    off = np.asarray(unit.state_off)
    n_a = int(off[1] - off[0])
    A = np.zeros((L * L * n_a, L * L * n_a), dtype=np.complex128)
    for i in range(L * L):
        iy, ix = divmod(i, L)
        for j in ilu.pattern(i, L, L, r):
            jy, jx = divmod(j, L)
            Zd = blocks[retrieval.slot(ix - jx, iy - jy, r, r)]
            si, sj = int(states[i]), int(states[j])
            A[i * n_a:(i + 1) * n_a, j * n_a:(j + 1) * n_a] = Zd[off[si]:off[si + 1], off[sj]:off[sj + 1]]
    return A, n_a


@pytest.mark.parametrize("Lx,Ly,r", [(3, 3, 2), (2, 3, 2), (4, 1, 3)])
def test_full_pattern_is_complete_lu(Lx, Ly, r):
    n_a = 3
    A = random_system(Lx, Ly, n_a, 7)
    f = ilu.block_ilu0(A, Lx, Ly, n_a, r)
    Lm, Um = ilu.dense_factors(f)
    assert np.abs(Lm @ Um - A).max() <= 1e-12 * np.abs(A).max()
    x = np.random.default_rng(1).standard_normal(len(A)) + 0j
    assert np.abs(ilu.ilu_apply(f, A @ x) - x).max() <= 1e-11 * np.abs(x).max()


def test_partial_pattern_matches_on_pattern_and_drops_fill():
    Lx, Ly, n_a, r = 4, 4, 3, 1
    A = random_system(Lx, Ly, n_a, 11)
    f = ilu.block_ilu0(A, Lx, Ly, n_a, r)
    Lm, Um = ilu.dense_factors(f)
    M = Lm @ Um
    on, off = 0.0, 0.0
    for i in range(Lx * Ly):
        near = set(ilu.pattern(i, Lx, Ly, r))
        for j in range(Lx * Ly):
            d = np.abs(M[i * n_a:(i + 1) * n_a, j * n_a:(j + 1) * n_a] - A[i * n_a:(i + 1) * n_a, j * n_a:(j + 1) * n_a])
            if j in near:
                on = max(on, d.max())
            else:
                off = max(off, d.max())
    assert on <= 1e-12 * np.abs(A).max()
    assert off > 1e-3 * np.abs(A).max()  # an incomplete factorisation, not an LU


def test_triangular_solves_equal_dense_solve():
    Lx, Ly, n_a, r = 5, 3, 2, 1
    A = random_system(Lx, Ly, n_a, 3)
    f = ilu.block_ilu0(A, Lx, Ly, n_a, r)
    Lm, Um = ilu.dense_factors(f)
    v = np.random.default_rng(5).standard_normal(len(A)) + 1j * np.random.default_rng(6).standard_normal(len(A))
    ref = np.linalg.solve(Lm @ Um, v)
    assert np.abs(ilu.ilu_apply(f, v) - ref).max() <= 1e-11 * np.abs(ref).max()


def test_radius_zero_is_block_jacobi():
    Lx, Ly, n_a = 3, 2, 4
    A = random_system(Lx, Ly, n_a, 9)
    f = ilu.block_ilu0(A, Lx, Ly, n_a, 0)
    v = np.random.default_rng(2).standard_normal(len(A)) + 0j
    ref = solve.block_jacobi(A, n_a)(v)
    assert np.abs(ilu.ilu_apply(f, v) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("r", [1, 2])
def test_order_inside_a_colour_does_not_matter(r):
    Lx, Ly, n_a = 5, 4, 2
    A = random_system(Lx, Ly, n_a, 4)
    f = ilu.block_ilu0(A, Lx, Ly, n_a, r)
    # same colours, units of every colour reversed
    col = lambda u: ilu.colour(u % Lx, u // Lx, r)
    order = sorted(range(Lx * Ly), key=lambda u: (col(u), -u))
    g = ilu.block_ilu0(A, Lx, Ly, n_a, r, order=order)
    a, b = ilu.slot_blocks(f), ilu.slot_blocks(g)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    # a different colour order does change them (the reading matters)
    nat = ilu.block_ilu0(A, Lx, Ly, n_a, r, order=range(Lx * Ly))
    assert np.abs(ilu.slot_blocks(nat) - a).max() > 1e-6 * np.abs(a).max()


def test_neighbours_never_share_a_colour():
    for r in (1, 2, 3):
        Lx, Ly = 9, 7
        for u in range(Lx * Ly):
            for j in ilu.pattern(u, Lx, Ly, r):
                if j != u:
                    assert ilu.colour(u % Lx, u // Lx, r) != ilu.colour(j % Lx, j // Lx, r)


def test_ilu_reduces_gmres_iterations_on_retrieved_near_field():
    L, r = 4, 1
    states = cb.bernoulli(L, 5)
    Anear, n_a = retrieved_near(L, 1, states)
    f = ilu.block_ilu0(Anear, L, L, n_a, r)
    Lm, Um = ilu.dense_factors(f)
    M = Lm @ Um
    for i in range(L * L):  # the factors reproduce the retrieved near field
        for j in ilu.pattern(i, L, L, r):
            blk = np.s_[i * n_a:(i + 1) * n_a, j * n_a:(j + 1) * n_a]
            assert np.abs(M[blk] - Anear[blk]).max() <= 1e-10 * np.abs(Anear).max()
    # the full retrieved system of the same codebook
    unit = macro_unit((0.006, 0.009))
    Zk = efie.direct_system(unit, states, L, K, 1)
    b = cb.random_complex(len(Zk), 8)
    it_bj = solve.gmres(lambda v: Zk @ v, b, 1e-8, 60, 400, solve.block_jacobi(Zk, n_a)).iters
    res = solve.gmres(lambda v: Zk @ v, b, 1e-8, 60, 400, lambda v: ilu.ilu_apply(f, v))
    assert res.converged and res.rel_residual <= 1e-8
    assert res.iters < it_bj
