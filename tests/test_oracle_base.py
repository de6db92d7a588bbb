"""Pins of the base-model oracle (oracle/base.py) against what perturbation
theory and the expansion fix: the second-order energy is the lambda^2
coefficient of the lowest eigenvalue of H0 + lambda (H - H0) (finite
differences of exact eigenvalues), a one-body Hamiltonian has the textbook
second-order sum, and the full-order expansion of eps - eps_base plus the
base energy of the whole space is FCI."""
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import base, fci, mbe


def _h0_and_h(P, S):
    sp = fci.cas_space(P, S)
    H = fci.hamiltonian_matrix(P, sp)
    i0 = base.reference_index(P, sp)
    nb = len(sp.blist)
    occ = lambda m: [p for p in range(64) if (m >> p) & 1]  # noqa: E731
    fa, fb = base.fock_diagonal(P, occ(int(sp.alist[i0 // nb])), occ(int(sp.blist[i0 % nb])))
    e0 = np.array([sum(fa[p] for p in occ(int(sp.alist[d // nb]))) + sum(fb[p] for p in occ(int(sp.blist[d % nb])))
                   for d in range(sp.dim)])
    return np.diag(e0), H, i0


@pytest.mark.parametrize("S", [(), (0, 9), (1, 2, 7)])
def test_second_order_is_the_lambda_squared_coefficient(S):
    P = synth.config_hubbard(2.0)
    H0, H, i0 = _h0_and_h(P, S)
    assert np.argmin(np.diag(H0)) == i0          # Phi is the lowest state of H0

    def E(lam):
        return np.linalg.eigvalsh(H0 + lam * (H - H0))[0]
    d = 2e-3

    def second(dd):
        return (E(dd) - 2.0 * E(0.0) + E(-dd)) / (2.0 * dd * dd)
    e2 = (4.0 * second(d / 2) - second(d)) / 3.0   # Richardson: the d^2 error removed
    assert abs(base.base_energy(P, S) - (H[i0, i0] + e2)) < 1e-7


def test_one_body_closed_form():
    """(pq|rs) = 0: E_base = sum of occupied h_pp - sum_sigma sum_{i occ, a
    virt} h_ai^2 / (h_aa - h_ii)."""
    P = synth.small_problem(6, 3, 3, [2, 3], nfrozen=0, nvec=4, seed=2, offdiag_std=0.05)
    P = replace(P, eri=np.zeros_like(P.eri))
    for S in [(), (0, 4), (0, 1, 4, 5)]:
        A = sorted(set(P.ref) | set(S))
        occ = [p for p in A if p < 3]
        vir = [p for p in A if p >= 3]
        core = [p for p in range(3) if p not in A]
        h = P.h
        ref = 2.0 * sum(h[p, p] for p in core + occ)
        e2 = 2.0 * sum(h[a, i] ** 2 / (h[a, a] - h[i, i]) for i in occ for a in vir)
        assert abs(base.base_energy(P, S) - (ref - e2)) < 1e-12


def test_full_order_expansion_with_base_is_fci():
    """The base energies cancel at full order: E_base(whole space) plus the
    expansion of eps - eps_base equals FCI."""
    P = synth.config_hubbard(2.0, nsite=8)
    X = base.full_space_tuple(P)
    res = mbe.run(P, energy=lambda S: fci.casci_energy(P, S) - base.base_energy(P, S))
    assert abs(base.base_energy(P, X) + res.total - fci.fci_energy(P)) < 1e-9
