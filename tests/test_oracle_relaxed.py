"""Pins of the relaxed (blended) retrieval oracle.

  * one-hot weights reduce to eq. (3): the retrieval oracle's block-loop
    product (itself pinned to the direct active-only system);
  * the matrix form equals the unit-pair loop form (independent code) for
    random weights, with and without the transpose;
  * the transposed operator is the transpose: y^T (A x) = (A^T y)^T x for
    the pair-loop forms (catches a transpose that is not Z(-d)^T);
  * weights scale linearly in each unit's blend (a weight applied on one side
    only would scale quadratically or not at all).
"""
import numpy as np

from oracle import efie, relaxed, retrieval
from oracle.constants import wavenumber
from workloads import codebooks as cb
from workloads.mesh import macro_unit

K = wavenumber(10.0e9)


def setup(L=2):
    unit = macro_unit((0.006, 0.009))
    blocks = efie.displacement_blocks(unit, L - 1, L - 1, K, extract=1)
    return unit, blocks


def test_one_hot_is_eq3():
    L = 2
    unit, blocks = setup(L)
    states = cb.bernoulli(L, 3)
    w = np.zeros((L * L, 2))
    w[np.arange(L * L), states] = 1.0
    x = cb.random_complex(L * L * 40, 4)
    ref = retrieval.retrieved_matvec(blocks, L - 1, L - 1, unit.state_off, states, L, x)
    got = relaxed.relaxed_matvec(blocks, L - 1, L - 1, unit.state_off, w, L, x)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_matrix_form_equals_pair_loops():
    L = 2
    unit, blocks = setup(L)
    rng = np.random.default_rng(5)
    w = rng.random((L * L, 2))
    x = cb.random_complex(L * L * 40, 6)
    for tr in (False, True):
        a = relaxed.relaxed_matvec(blocks, L - 1, L - 1, unit.state_off, w, L, x, transpose=tr)
        b = relaxed.relaxed_matvec_pairs(blocks, L - 1, L - 1, unit.state_off, w, L, x, transpose=tr)
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_transpose_identity_pairs():
    L = 2
    unit, blocks = setup(L)
    rng = np.random.default_rng(7)
    w = rng.random((L * L, 2))
    x = cb.random_complex(L * L * 40, 8)
    y = cb.random_complex(L * L * 40, 9)
    ax = relaxed.relaxed_matvec_pairs(blocks, L - 1, L - 1, unit.state_off, w, L, x)
    aty = relaxed.relaxed_matvec_pairs(blocks, L - 1, L - 1, unit.state_off, w, L, y, transpose=True)
    lhs, rhs = y @ ax, aty @ x
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the non-transposed operator is not symmetric here (cross-state entries),
    # so the test would fail if the transpose were dropped
    ay = relaxed.relaxed_matvec_pairs(blocks, L - 1, L - 1, unit.state_off, w, L, y)
    assert abs(ay @ x - lhs) > 1e-8 * abs(lhs)


def test_blend_scales_per_unit():
    L = 2
    unit, blocks = setup(L)
    rng = np.random.default_rng(11)
    w = rng.random((L * L, 2))
    x = cb.random_complex(L * L * 40, 12)
    y0 = relaxed.relaxed_matvec(blocks, L - 1, L - 1, unit.state_off, w, L, x)
    w2 = w.copy()
    w2[0] *= 2.0  # unit 0's blend doubled: its row block doubles, its column block doubles
    y2 = relaxed.relaxed_matvec(blocks, L - 1, L - 1, unit.state_off, w2, L, x)
    Z = retrieval.macro_matrix(blocks, L - 1, L - 1, L)
    P = relaxed.blend_matrix(w, unit.state_off, L)
    A = P.T @ Z @ P
    Au = A.copy()
    Au[:40, :] *= 2.0
    Au[:, :40] *= 2.0
    assert np.abs(y2 - Au @ x).max() <= 1e-12 * np.abs(y2).max()
    assert np.abs(y2 - y0).max() > 1e-3 * np.abs(y0).max()


def test_adjoint_gradient_matches_finite_differences():
    """The adjoint gradient of J(w) = mean RCS over a 30-degree cone (2-bit,
    2 x 2 array) against central differences of J itself (forward solves
    only): every component within 1e-6 of the largest."""
    from workloads.mesh import macro_unit as mu
    unit = mu((0.005, 0.007, 0.009, 0.011))
    L = 2
    blocks = efie.displacement_blocks(unit, L - 1, L - 1, K, extract=1)
    rng = np.random.default_rng(13)
    logits = rng.standard_normal((L * L, 4))
    w = np.exp(logits) / np.exp(logits).sum(axis=1, keepdims=True)
    thph = cb.cone16(30.0)
    J, _, _, grad = relaxed.relaxed_objective(unit, blocks, L - 1, w, L, K, thph, with_grad=True)
    h = 1e-6
    fd = np.zeros_like(grad)
    for u in range(L * L):
        for s in range(4):
            wp, wm = w.copy(), w.copy()
            wp[u, s] += h
            wm[u, s] -= h
            Jp = relaxed.relaxed_objective(unit, blocks, L - 1, wp, L, K, thph)[0]
            Jm = relaxed.relaxed_objective(unit, blocks, L - 1, wm, L, K, thph)[0]
            fd[u, s] = (Jp - Jm) / (2 * h)
    assert np.abs(grad - fd).max() <= 1e-6 * np.abs(fd).max()
    assert np.abs(fd).max() > 0
