"""Pins of the CASSCF oracle (oracle/casscf.py) against what the definition
and the mathematics fix, independent of the oracle's own optimiser:
finite differences of the energy, a closed form without two-electron
integrals, stationarity and positive curvature at the optimum, invariance
under the starting orbitals, the canonical form, and full-order MBE = FCI in
the CASSCF orbitals (orbital invariance of FCI)."""
from dataclasses import replace

import numpy as np
import pytest
import scipy.linalg as sl

import synth
from oracle import casscf, fci, mbe


def _small():
    # 7 orbitals, 3a+3b, one frozen orbital, [Pi] = {2, 3}: core {1},
    # active {2, 3}, virtual {4, 5, 6}
    return synth.small_problem(7, 3, 3, [2, 3], nfrozen=1, nvec=6, seed=11, vec_std=0.15, offdiag_std=0.2)


def test_gradient_matches_finite_differences():
    P = synth.small_problem(6, 3, 3, [1, 2, 3], nfrozen=0, nvec=6, seed=5)
    pairs = casscf.rotation_pairs(P)
    rng = np.random.default_rng(1)
    x = 0.1 * rng.standard_normal(len(pairs))
    U0 = np.eye(P.norb)
    e, g = casscf.energy_and_gradient(P, U0, pairs, x)
    h = 1e-5
    for k in range(len(pairs)):
        xp, xm = x.copy(), x.copy()
        xp[k] += h
        xm[k] -= h
        fd = (casscf.energy_and_gradient(P, U0, pairs, xp)[0] - casscf.energy_and_gradient(P, U0, pairs, xm)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-8, (k, fd, g[k])
    # the local form 2 (F_qp - F_pq) at K = 0 against finite differences too
    e0, gl = casscf.local_gradient(P)
    for k in range(len(pairs)):
        d = np.zeros(len(pairs))
        d[k] = h
        fd = (casscf.energy_and_gradient(P, U0, pairs, d)[0] - casscf.energy_and_gradient(P, U0, pairs, -d)[0]) / (2 * h)
        assert abs(fd - gl[k]) < 1e-8


def test_no_two_electron_integrals_gives_aufbau():
    """With (pq|rs) = 0 every state is a Slater determinant of orbitals, and
    rotations can bring the lowest eigenvectors of h into the occupied core
    and active spaces: E_CASSCF = the aufbau sum of eigh(h)."""
    P = synth.small_problem(6, 3, 3, [2, 3], nfrozen=0, nvec=4, seed=3, offdiag_std=0.3)
    P = replace(P, eri=np.zeros_like(P.eri))
    e, _, _ = casscf.casscf(P)
    w = np.linalg.eigvalsh(P.h)
    assert abs(e - 2.0 * w[:3].sum()) < 1e-9, (e, 2.0 * w[:3].sum())
    assert e < fci.casci_energy(P, ()) - 1e-3    # the start was not optimal


def test_optimum_is_a_stationary_minimum():
    P = _small()
    e, U, Pc = casscf.casscf(P)
    e_c, g = casscf.local_gradient(Pc)
    assert np.abs(g).max() < 1e-6
    assert abs(e_c - e) < 1e-10          # canonicalisation only rotates inside the spaces
    assert e < fci.casci_energy(P, ()) - 1e-4
    pairs = casscf.rotation_pairs(P)
    rng = np.random.default_rng(7)
    for _ in range(6):
        d = rng.standard_normal(len(pairs))
        d *= 1e-3 / np.linalg.norm(d)
        K = casscf.kappa_matrix(P.norb, pairs, d)
        e2 = fci.casci_energy(casscf.transform(P, U @ sl.expm(K)), ())
        assert e2 > e - 1e-12


def test_full_active_space_is_fci():
    """No core or virtual orbitals: nothing to rotate, E_CASSCF = FCI."""
    P = synth.small_problem(5, 2, 2, [0, 1, 2, 3, 4], nfrozen=0, nvec=5, seed=2)
    assert casscf.rotation_pairs(P) == []
    e, U, Pc = casscf.casscf(P)
    H = fci.hamiltonian_matrix(P, fci.cas_space(P, ()))
    assert abs(e - np.linalg.eigvalsh(H)[0]) < 1e-12
    # the canonical orbitals are the natural orbitals; the energy is unchanged
    assert np.abs(U.T @ U - np.eye(5)).max() < 1e-12
    assert abs(casscf.reference_state(Pc)[0] - e) < 1e-12


def test_independent_of_the_starting_orbitals():
    """A small random rotation of the input orbitals (all non-frozen ones
    mixed) reaches the same minimum and the same canonical Hamiltonian."""
    P = _small()
    e, U, Pc = casscf.casscf(P)
    n = P.norb
    rng = np.random.default_rng(4)
    A = rng.standard_normal((n, n)) * 0.03
    A = A - A.T
    A[0, :] = A[:, 0] = 0.0              # frozen orbital kept
    R = sl.expm(A)
    P2 = casscf.transform(P, R)
    e2, U2, Pc2 = casscf.casscf(P2)
    assert abs(e2 - e) < 1e-10
    # the same orbitals in the original basis, up to the sign of each (the
    # sign rule refers to the basis a run starts from)
    W = R @ U2
    sg = np.sign(np.sum(W * U, axis=0))
    assert np.abs(W * sg - U).max() < 1e-6
    Pc2 = casscf.transform(Pc2, np.diag(sg))
    assert np.abs(Pc2.h - Pc.h).max() < 1e-6
    assert np.abs(Pc2.eri - Pc.eri).max() < 1e-6


def test_canonical_form():
    P = _small()
    _, U, Pc = casscf.casscf(P)
    _, C, A, V = casscf.spaces(P)
    assert np.abs(U.T @ U - np.eye(P.norb)).max() < 1e-12
    _, g1, _ = casscf.reference_state(Pc)
    f = casscf.fock(Pc, g1)
    for B in (C, V):
        fb = f[np.ix_(B, B)]
        assert np.abs(fb - np.diag(np.diag(fb))).max() < 1e-7
        assert np.all(np.diff(np.diag(fb)) >= -1e-10)
    ga = g1[np.ix_(A, A)]
    assert np.abs(ga - np.diag(np.diag(ga))).max() < 1e-7
    assert np.all(np.diff(np.diag(ga)) <= 1e-10)
    for j in range(P.norb):
        i = int(np.argmax(np.abs(U[:, j])))
        assert U[i, j] > 0


def test_full_order_mbe_in_casscf_orbitals_is_fci():
    """FCI is invariant under rotations of the non-frozen orbitals, so the
    full-order expansion in the CASSCF orbitals gives the FCI energy of the
    original problem."""
    P = _small()
    _, _, Pc = casscf.casscf(P)
    res = mbe.run(Pc, energy=lambda S: fci.casci_energy(Pc, S))
    assert abs(res.total - fci.fci_energy(P)) < 1e-9


def test_spin_targeted_reference_state():
    """With the reference state chosen by total spin (the plain problem's
    lowest M_s = 0 state of CAS(2e,2o) is a triplet component): the gradient
    of that state's energy equals finite differences, its optimum is
    stationary, and it lies above the optimum of the lowest state."""
    P = synth.config_plain(0)
    pairs = casscf.rotation_pairs(P)
    U0 = np.eye(P.norb)
    rng = np.random.default_rng(3)
    x = 0.05 * rng.standard_normal(len(pairs))
    e, g = casscf.energy_and_gradient(P, U0, pairs, x, spin=0.0)
    h = 1e-5
    for k in rng.choice(len(pairs), 6, replace=False):
        xp, xm = x.copy(), x.copy()
        xp[k] += h
        xm[k] -= h
        fd = (casscf.energy_and_gradient(P, U0, pairs, xp, spin=0.0)[0] -
              casscf.energy_and_gradient(P, U0, pairs, xm, spin=0.0)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-8
    es, _, Ps = casscf.casscf(P, spin=0.0)
    assert np.abs(casscf.local_gradient(Ps, spin=0.0)[1]).max() < 1e-8
    el, _, _ = casscf.casscf(P)
    assert es > el + 1e-3
