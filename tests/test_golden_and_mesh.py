"""Paper-printed bookkeeping (Table 1) and the mesh tables of the workloads."""
import os

import numpy as np
import pytest

from workloads import codebooks as cb
from workloads.configs import far_pair_count, near_pair_count
from workloads.mesh import macro_unit, patch_mesh

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_table1_unknowns_are_units_times_macro_bases():
    rows = np.loadtxt(os.path.join(GOLD, "table1_r3m_unknowns.txt"), dtype=np.int64)
    for L, unknowns in rows:
        assert L * L * 1056 == unknowns


def test_patch_mesh_counts_and_euler():
    m = patch_mesh(0.006, 4)
    assert m.vert.shape == (25, 3) and m.tri.shape == (32, 3) and m.rwg.shape == (40, 4)
    edges = {tuple(sorted(e)) for t in m.tri for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
    assert len(m.vert) - len(edges) + len(m.tri) == 1
    for nc, nr in ((8, 176), (16, 736)):
        assert len(patch_mesh(0.009, nc).rwg) == nr


def test_patch_mesh_ccw_and_d4_symmetric():
    m = patch_mesh(0.009, 4)
    v = m.vert
    e1 = v[m.tri[:, 1]] - v[m.tri[:, 0]]
    e2 = v[m.tri[:, 2]] - v[m.tri[:, 0]]
    assert np.all(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0] > 0)
    # the set of triangles maps to itself under x -> -x and x <-> y
    key = lambda tris: {tuple(sorted(map(tuple, np.round(v[t], 12).tolist()))) for t in tris}
    base = key(m.tri)
    for M in (np.diag([-1.0, 1.0, 1.0]), np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1.0]])):
        vm = v @ M.T
        img = {tuple(sorted(map(tuple, np.round(vm[t], 12).tolist()))) for t in m.tri}
        assert img == base


def test_macro_unit_layout():
    mu = macro_unit((0.005, 0.007, 0.009, 0.011))
    assert mu.n == 160 and mu.n_a == 40
    assert list(mu.state_off) == [0, 40, 80, 120, 160]
    assert 32 * 32 * mu.n == 163840


def test_pair_counts():
    assert far_pair_count(32, 2) == 1024860 and near_pair_count(32, 2) == 23716
    assert near_pair_count(6, 5) == 1296


def test_codebook_families():
    assert cb.bernoulli(6, 0).shape == (36,)
    s = cb.stripes(32, 5)
    assert set(np.unique(s)) <= {0, 1}
    c = cb.checkerboard(8, 4).reshape(8, 8)
    assert c[0, 0] == 0 and c[0, 4] == 1 and c[4, 4] == 0
