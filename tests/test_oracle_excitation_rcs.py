"""Pins of the excitation (eq. (1) right-hand side) and the far-field/RCS code.

* normal incidence: U_m has the closed form E0 (l/2) x . [(c+ - v+) + (v- - c-)]
  (the integrand is linear, so the 7-point rule is exact);
* I^T U(k_i, e) = E0 e . N(-k_i) for any current I;
* mirror symmetry of the RCS cut for a mirror-symmetric codebook;
* bistatic reciprocity of the scattering amplitude.
"""
import math

import numpy as np

from oracle import efie, excitation, farfield, solve
from workloads import codebooks as cb


def test_normal_incidence_closed_form(unit1, k10):
    states = cb.bernoulli(2, 1)
    mesh, _ = efie.active_array_mesh(unit1, states, 2)
    U = excitation.plane_wave(mesh, k10, 0.0, 0.0, e0=2.0)
    ref = np.zeros(mesh.n)
    for m in range(mesh.n):
        tp, tm = mesh.rwg_tri[m]
        vp = mesh.tri_xyz[tp, mesh.rwg_free[m, 0]]
        vm = mesh.tri_xyz[tm, mesh.rwg_free[m, 1]]
        cp = mesh.tri_xyz[tp].mean(axis=0)
        cm = mesh.tri_xyz[tm].mean(axis=0)
        ref[m] = 2.0 * 0.5 * mesh.rwg_len[m] * ((cp - vp) + (vm - cm))[0]
    assert np.abs(U - ref).max() <= 1e-14 * np.abs(ref).max()


def test_excitation_is_radiation_transform(unit1, k10):
    states = cb.bernoulli(2, 2)
    mesh, _ = efie.active_array_mesh(unit1, states, 2)
    I = cb.random_complex(mesh.n, 3)
    for th, ph in [(0.4, 0.0), (1.0, 0.7)]:
        khat, ehat = excitation.incidence_vectors(th, ph)
        U = excitation.plane_wave(mesh, k10, th, ph)
        N = farfield.radiation_vector(mesh, I, k10, -khat[None, :])[0]
        assert abs(I @ U - ehat @ N) <= 1e-13 * abs(ehat @ N)


def test_mirror_symmetry(unit1, k10):
    L = 3
    states = cb.symmetrize_x(cb.bernoulli(L, 9), L)
    assert np.array_equal(states, cb.mirror_x(states, L))
    Zk = efie.direct_system(unit1, states, L, k10, 1)
    mesh, _ = efie.active_array_mesh(unit1, states, L)
    I = solve.lu_solve(Zk, excitation.plane_wave(mesh, k10))
    cut = cb.phi0_cut(5.0)
    sig = farfield.rcs(mesh, I, k10, cut)
    th = np.rad2deg(cut[:, 0]).round().astype(int)
    pos = {t: s for t, s in zip(th, sig)}
    for t in range(5, 180, 5):
        assert abs(pos[t] - pos[-t]) <= 1e-12 * max(sig)


def test_mirror_pair_codebooks(unit1, k10):
    """A codebook and its mirror image give mirrored RCS cuts."""
    L = 2
    s1 = np.array([0, 1, 1, 1], np.uint8)
    s2 = cb.mirror_x(s1, L)
    cut = cb.phi0_cut(15.0)
    out = []
    for s in (s1, s2):
        Zk = efie.direct_system(unit1, s, L, k10, 1)
        mesh, _ = efie.active_array_mesh(unit1, s, L)
        I = solve.lu_solve(Zk, excitation.plane_wave(mesh, k10))
        out.append(farfield.rcs(mesh, I, k10, cut))
    th = np.rad2deg(cut[:, 0]).round().astype(int)
    d1 = dict(zip(th, out[0]))
    d2 = dict(zip(th, out[1]))
    for t in range(-165, 180, 15):
        assert abs(d1[t] - d2[-t]) <= 1e-12 * max(out[0])


def test_bistatic_reciprocity(unit1, k10):
    """Amplitude (incidence a, observe b) = (incidence from -b, observe -a)."""
    states = cb.bernoulli(2, 4)
    Zk = efie.direct_system(unit1, states, 2, k10, 1)
    Zs = 0.5 * (Zk + Zk.T)  # reciprocity holds exactly for the symmetric part
    mesh, _ = efie.active_array_mesh(unit1, states, 2)
    ka, ea = excitation.incidence_vectors(0.35, 0.0)  # travels along ka
    rb = farfield.directions(np.array([[1.1, 0.4]]))[0]
    eb = np.array([math.cos(1.1) * math.cos(0.4), math.cos(1.1) * math.sin(0.4), -math.sin(1.1)])
    Ia = np.linalg.solve(Zs, excitation.plane_wave(mesh, k10, khat=ka, ehat=ea))
    amp_ab = eb @ farfield.radiation_vector(mesh, Ia, k10, rb[None])[0]
    Ib = np.linalg.solve(Zs, excitation.plane_wave(mesh, k10, khat=-rb, ehat=eb))
    amp_ba = ea @ farfield.radiation_vector(mesh, Ib, k10, -ka[None])[0]
    assert abs(amp_ab - amp_ba) <= 1e-12 * abs(amp_ab)
    # with the raw Z: equal to the quadrature-level asymmetry
    Ia = np.linalg.solve(Zk, excitation.plane_wave(mesh, k10, khat=ka, ehat=ea))
    Ib = np.linalg.solve(Zk, excitation.plane_wave(mesh, k10, khat=-rb, ehat=eb))
    a1 = eb @ farfield.radiation_vector(mesh, Ia, k10, rb[None])[0]
    a2 = ea @ farfield.radiation_vector(mesh, Ib, k10, -ka[None])[0]
    assert abs(a1 - a2) <= 1e-2 * abs(a1)
