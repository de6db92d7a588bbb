"""Pins of the RHF oracle (oracle/hf.py) against what fixes Hartree-Fock
independently of its own Fock formula (on these synthetic problems the
minimum need not be aufbau: a virtual orbital energy can lie below an
occupied one): a one-body Hamiltonian gives the
aufbau sum of eigenvalues; the energy is stationary and a minimum under
occupied-virtual rotations (finite differences); it equals the diagonal
element of the aufbau determinant in the CASCI oracle's Slater-Condon
Hamiltonian of the transformed problem and lies above FCI; two electrons in
two orbitals reach the minimum of a one-angle brute-force scan; the
half-filled Hubbard chain's hopping eigenvectors are already its RHF
orbitals."""
from dataclasses import replace

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import cc, fci, hf


def _energy_of(P, C):
    no = P.nalpha
    D = C[:, :no] @ C[:, :no].T
    return hf.energy(P, D)


def test_one_body():
    P = synth.small_problem(7, 3, 3, [2, 3], nvec=4, seed=2, offdiag_std=0.2)
    P = replace(P, eri=np.zeros_like(P.eri))
    e, C, _ = hf.rhf(P)
    w = np.linalg.eigvalsh(P.h)
    assert abs(e - 2.0 * w[:3].sum()) < 1e-12


@pytest.mark.parametrize("seed", [0, 3])
def test_stationary_minimum(seed):
    P = synth.small_problem(8, 3, 3, [2, 3], nvec=6, seed=seed, vec_std=0.15, offdiag_std=0.1)
    e, C, _ = hf.rhf(P)
    rng = np.random.default_rng(seed)
    for _ in range(4):
        K = np.zeros((8, 8))
        K[3:, :3] = rng.standard_normal((5, 3))
        K = K - K.T
        s = 1e-5
        ep = _energy_of(P, C @ scipy.linalg.expm(s * K))
        em = _energy_of(P, C @ scipy.linalg.expm(-s * K))
        assert abs(ep - em) / (2 * s) < 1e-7          # gradient zero
        assert ep + em - 2 * e > 0.0                   # positive curvature


def test_energy_is_the_aufbau_determinant_and_above_fci():
    P = synth.small_problem(7, 3, 3, [2, 3], nvec=6, seed=5, vec_std=0.15)
    e, Q, C = hf.hf_problem(P)
    sp = fci.cas_space(Q, tuple(Q.expansion_space()))
    from oracle import base
    i0 = base.reference_index(Q, sp)
    H = fci.hamiltonian_matrix(Q, sp)
    assert abs(H[i0, i0] - e) < 1e-11
    assert e > fci.fci_energy(P) + 1e-4
    assert abs(fci.fci_energy(Q) - fci.fci_energy(P)) < 1e-10   # FCI does not depend on the orbitals
    fa, fb = cc.fock_matrix(Q, list(range(3)), list(range(3)))
    assert np.abs(fa - np.diag(np.diag(fa))).max() < 1e-9        # canonical: the Fock operator is diagonal
    d = np.diag(fa)
    assert np.all(np.diff(d[:3]) > 0) and np.all(np.diff(d[3:]) > 0)   # ascending in each block


def test_two_electrons_two_orbitals_brute_force():
    rng = np.random.default_rng(4)
    h = np.array([[-1.0, 0.2], [0.2, -0.3]])
    V = 0.4 * rng.standard_normal((3, 2, 2))
    V = 0.5 * (V + V.transpose(0, 2, 1))
    eri = np.einsum("kpq,krs->pqrs", V, V)
    P = synth.Problem("h2like", h, eri, 1, 1, 0, [0, 1])
    e, C, _ = hf.rhf(P)
    th = np.linspace(0.0, np.pi, 200001)
    best = min(_energy_of(P, np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])) for t in th[::1000])
    # refine around the coarse minimum
    t0 = th[::1000][int(np.argmin([_energy_of(P, np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]]))
                                    for t in th[::1000]]))]
    fine = np.linspace(t0 - 0.02, t0 + 0.02, 40001)
    best = min(best, min(_energy_of(P, np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])) for t in fine))
    assert e <= best + 1e-12 and best - e < 1e-9


def test_hubbard_orbitals_are_already_rhf():
    P = synth.config_hubbard(4.0, nsite=8)
    e, C, _ = hf.rhf(P)
    assert np.abs(np.abs(C) - np.eye(8)).max() < 1e-9
    assert abs(e - _energy_of(P, np.eye(8))) < 1e-12
