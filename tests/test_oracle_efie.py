"""Pins of the direct EFIE/RWG matrix (eq. (1), Sec. II-A).

* reciprocity: Z symmetric (Galerkin with a symmetric kernel), Z(-d) = Z(d)^T;
* discrete power balance: Re(I^H Z I)/2 equals the far-field integral of the
  same currents (this fixes Re Z, both of its terms, their signs and every
  constant, independently of the singular 1/R treatment);
* the singular treatment agrees with plain quadrature when triangles are far;
* physical-optics limit of a two-wavelength plate;
* mesh-refinement convergence.
"""
import math

import numpy as np
import pytest

from oracle import efie, excitation, farfield, solve
from oracle.constants import ETA0, wavenumber
from workloads import codebooks as cb
from workloads.mesh import macro_unit, patch_mesh


def test_direct_symmetry_2x2(unit1, k10):
    states = np.array([0, 1, 1, 0], dtype=np.uint8)
    Z = efie.direct_system(unit1, states, 2, k10, extract=1)
    assert np.all(np.isfinite(Z))
    scale = np.abs(Z).max()
    mesh, owner = efie.active_array_mesh(unit1, states, 2)
    # entries between different, non-extracted-neighbour units: symmetric to rounding
    # (2x2 has only neighbours, so use extract=0 to get plain quadrature off-diagonal)
    Z0 = efie.direct_system(unit1, states, 2, k10, extract=0)
    offd = owner[:, None] != owner[None, :]
    assert np.abs((Z0 - Z0.T)[offd]).max() <= 1e-13 * scale
    # extracted pairs: symmetric to the quadrature level (reported number)
    rel = np.abs(Z - Z.T).max() / scale
    assert rel < 1e-3


def test_block_reciprocity(unit1, k10):
    for d in [(3, 0), (2, -3)]:
        Zp = efie.displacement_block(unit1, d[0], d[1], k10, extract=1)
        Zm = efie.displacement_block(unit1, -d[0], -d[1], k10, extract=1)
        assert np.abs(Zp - Zm.T).max() <= 1e-12 * np.abs(Zp).max()


def test_extraction_matches_plain_quadrature_far(unit1, k10):
    Z1 = efie.displacement_block(unit1, 3, 1, k10, extract=3)
    Z0 = efie.displacement_block(unit1, 3, 1, k10, extract=0)
    assert np.linalg.norm(Z1 - Z0) <= 1e-8 * np.linalg.norm(Z0)


def test_self_block_finite_and_cross_state(unit2, k10):
    Z = efie.displacement_block(unit2, 0, 0, k10, extract=1)
    assert np.all(np.isfinite(Z))
    # same-state diagonal sub-blocks are symmetric to quadrature level
    for s in range(4):
        a = slice(40 * s, 40 * s + 40)
        assert np.abs(Z[a, a] - Z[a, a].T).max() < 1e-3 * np.abs(Z[a, a]).max()


@pytest.mark.parametrize("states", [[0, 1, 1, 0], [1, 1, 1, 1]])
def test_discrete_power_balance(unit1, k10, states):
    states = np.asarray(states, dtype=np.uint8)
    Z = efie.direct_system(unit1, states, 2, k10, extract=1)
    mesh, _ = efie.active_array_mesh(unit1, states, 2)
    rng = np.random.default_rng(1)
    I = rng.standard_normal(mesh.n) + 1j * rng.standard_normal(mesh.n)
    # entrywise Re Z is the symmetric smooth double sum; (Im Z is symmetric only
    # to the quadrature level on extracted pairs, so it is left out of the form)
    p_mom = 0.5 * np.real(np.vdot(I, np.real(Z) @ I))
    phys, disc = farfield.radiated_power(mesh, I, k10, 40, 80)
    assert abs(p_mom - disc) <= 1e-10 * abs(p_mom)
    # the physical (transverse) form differs only by the discrete
    # integration-by-parts error of the 7-point rule
    assert abs(phys - disc) <= 2e-2 * abs(disc)


def test_optical_theorem(unit1, k10):
    """Extinction = scattering for a lossless PEC array: half the real part of
    the forward radiation vector projected on the incident polarisation equals
    the radiated power of the induced current."""
    states = np.array([1, 0, 0, 1], dtype=np.uint8)
    Z = efie.direct_system(unit1, states, 2, k10, extract=1)
    mesh, _ = efie.active_array_mesh(unit1, states, 2)
    th = 0.3
    khat, ehat = excitation.incidence_vectors(th, 0.0)
    U = excitation.plane_wave(mesh, k10, th, 0.0)
    I = solve.lu_solve(Z, U)
    fwd = farfield.radiation_vector(mesh, I, k10, khat[None, :])[0]
    p_ext = 0.5 * np.real(np.dot(ehat, fwd))
    phys, disc = farfield.radiated_power(mesh, I, k10, 40, 80)
    # exact up to the quadrature-level asymmetry of Im Z and the discrete
    # integration by parts of the transverse projection
    assert abs(p_ext - disc) <= 5e-3 * abs(disc)
    assert abs(p_ext - phys) <= 2e-2 * abs(disc)


def plate_rcs(side, ncell, k):
    pm = patch_mesh(side, ncell)
    mesh = efie.rwg_mesh(pm.vert, pm.tri, pm.rwg)
    Z = efie.efie_matrix(mesh, mesh, k, extract=0)
    U = excitation.plane_wave(mesh, k)
    I = solve.lu_solve(Z, U)
    return farfield.rcs(mesh, I, k, np.array([[0.0, 0.0]]))[0]


@pytest.mark.slow
def test_physical_optics_plate(k10):
    """A 2-wavelength square PEC plate at normal incidence: monostatic RCS
    within 1.5 dB of the physical-optics value 4 pi A^2 / lambda^2."""
    lam = 2 * math.pi / k10
    side = 2 * lam
    sig = plate_rcs(side, 16, k10)
    po = 4 * math.pi * side ** 4 / lam ** 2
    assert abs(10 * math.log10(sig / po)) < 1.5


def test_mesh_refinement_converges(k10):
    """RCS of a single 9 mm patch: successive refinements 4 -> 8 -> 16 cells
    per side change the result by shrinking amounts, at a steady rate."""
    th = np.deg2rad(np.array([[0.0, 0.0], [30.0, 0.0], [60.0, 0.0]]))
    vals = []
    for nc in (4, 8, 16):
        pm = patch_mesh(0.009, nc)
        mesh = efie.rwg_mesh(pm.vert, pm.tri, pm.rwg)
        Z = efie.efie_matrix(mesh, mesh, k10, extract=0)
        I = solve.lu_solve(Z, excitation.plane_wave(mesh, k10))
        vals.append(farfield.rcs(mesh, I, k10, th))
    d1 = np.linalg.norm(vals[1] - vals[0]) / np.linalg.norm(vals[2])
    d2 = np.linalg.norm(vals[2] - vals[1]) / np.linalg.norm(vals[2])
    # observed order of convergence (first order for RWG with edge singularities)
    rate = np.log2(d1 / d2)
    assert 0.7 < rate < 2.5
