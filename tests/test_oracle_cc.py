"""Pins of the coupled-cluster base oracle (oracle/cc.py) against what the
theory fixes, none of them the oracle's own formulas:

* CCSD is exact for two electrons and for a one-body Hamiltonian (the
  textbook sum of orbital energies), and for non-interacting electron pairs
  it is the sum of the pair energies (the disconnected T2 T2 products);
* the CCSD energy does not change under rotations among the occupied and
  among the virtual active orbitals;
* order by order in the Moller-Plesset partition H(lam) = H0 + lam (H - H0)
  (finite differences of exact eigenvalues): FCI - CCSD starts at lam^4, and
  its lam^4 coefficient is that of (T), so FCI - CCSD(T) has none;
* (T) refuses orbitals in which the Fock operator of Phi is not diagonal.

The fifth-order singles-triples part of (T) (the y term) enters only at
lam^5 and is fixed by its definition alone (parity unpinned for that term).
"""
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import cc, fci

ATOL = 1e-10


def test_two_electrons_is_exact():
    P = synth.small_problem(6, 1, 1, [0, 1], nvec=4, seed=5)
    for S in [(), (2,), (2, 3, 4, 5)]:
        assert abs(cc.base_energy(P, S) - fci.casci_energy(P, S)) < ATOL
    P = synth.small_problem(5, 2, 0, [0, 1, 2], nvec=4, seed=6)     # two alpha electrons
    for S in [(), (3, 4)]:
        assert abs(cc.base_energy(P, S) - fci.casci_energy(P, S)) < ATOL


def test_one_body_hamiltonian_is_exact():
    """(pq|rs) = 0: E = 2 sum core h_cc + the lowest n_alpha and n_beta
    eigenvalues of h on the active orbitals, for non-canonical h."""
    P = synth.small_problem(7, 3, 2, [2, 3], nfrozen=0, nvec=4, seed=2, offdiag_std=0.2)
    P = replace(P, eri=np.zeros_like(P.eri))
    for S in [(), (0, 5), (1, 4, 5, 6)]:
        A = sorted(set(P.ref) | set(S))
        core = [p for p in range(P.nbeta) if p not in A]
        na = P.nalpha - len(core)
        nb = P.nbeta - len(core)
        w = np.linalg.eigvalsh(P.h[np.ix_(A, A)])
        ref = 2.0 * sum(P.h[c, c] for c in core) + w[:na].sum() + w[:nb].sum()
        assert abs(cc.base_energy(P, S) - ref) < ATOL


def _pairs_problem():
    """Two non-interacting two-electron blocks {0, 2, 4} and {1, 3, 5}
    (2 alpha + 2 beta electrons in all, Phi occupying 0 and 1)."""
    rng = np.random.default_rng(7)
    n = 6
    h = np.zeros((n, n))
    eri = np.zeros((n, n, n, n))
    for blk in ([0, 2, 4], [1, 3, 5]):
        hb = np.diag([-1.0, 0.2, 0.6]) + 0.1 * rng.standard_normal((3, 3))
        h[np.ix_(blk, blk)] = 0.5 * (hb + hb.T)
        V = 0.3 * rng.standard_normal((4, 3, 3))
        V = 0.5 * (V + V.transpose(0, 2, 1))
        eb = np.einsum("kpq,krs->pqrs", V, V)
        eri[np.ix_(blk, blk, blk, blk)] = eb
    P = synth.Problem("pairs", h, eri, 2, 2, 0, [0, 1])
    return P


def test_noninteracting_pairs_are_additive():
    P = _pairs_problem()
    S = (2, 3, 4, 5)
    e = cc.base_energy(P, S)
    assert abs(e - fci.casci_energy(P, S)) < ATOL
    # and that is the sum of the two one-pair problems
    parts = 0.0
    for blk in ([0, 2, 4], [1, 3, 5]):
        Pb = synth.Problem("pair", P.h[np.ix_(blk, blk)], P.eri[np.ix_(blk, blk, blk, blk)], 1, 1, 0, [0])
        parts += fci.casci_energy(Pb, (1, 2))
    assert abs(e - parts) < ATOL


def test_invariance_under_occupied_and_virtual_rotations():
    P = synth.small_problem(7, 3, 3, [2, 3], nvec=5, seed=4, offdiag_std=0.1)
    S = (0, 4, 6)                 # active orbitals 0, 2 (occupied) and 3, 4, 6 (virtual)
    A = sorted(set(P.ref) | set(S))
    occ = [p for p in A if p < P.nalpha]
    vir = [p for p in A if p >= P.nalpha]
    rng = np.random.default_rng(11)
    U = np.eye(P.norb)
    for blk in (occ, vir):
        Q, _ = np.linalg.qr(rng.standard_normal((len(blk), len(blk))))
        U[np.ix_(blk, blk)] = Q
    h = U.T @ P.h @ U
    eri = np.einsum("pqrs,pa,qb,rc,sd->abcd", P.eri, U, U, U, U, optimize=True)
    Pr = replace(P, h=h, eri=eri)
    assert abs(cc.base_energy(Pr, S) - cc.base_energy(P, S)) < ATOL
    assert abs(fci.casci_energy(Pr, S) - fci.casci_energy(P, S)) < ATOL


def _mp_problem(P, lam):
    """H0 + lam (H - H0) with H0 = sum_p f_p n_p (f the Fock diagonal of the
    aufbau determinant, canonical orbitals): one-body (1 - lam) diag(f) +
    lam h, two-body lam (pq|rs); its Fock operator stays diag(f)."""
    fa, fb = cc.fock_matrix(P, list(range(P.nalpha)), list(range(P.nbeta)))
    F = np.diag(np.diag(fa))
    return replace(P, h=(1.0 - lam) * F + lam * P.h, eri=lam * P.eri)


@pytest.mark.parametrize("S", [(0, 5), (1, 2, 6)])
def test_ccsd_t_is_exact_through_fourth_order(S):
    P = synth.config_hubbard(4.0, nsite=8)
    lam = 0.05

    def parts(lm):
        Q = _mp_problem(P, lm)
        e, t, cs = cc.ccsd(Q, S, tol=1e-14)
        return fci.casci_energy(Q, S), e, cc.triples_correction(Q, S, t, cs)

    r = {}
    for lm in (lam, lam / 2):
        ef, ec, et = parts(lm)
        r[lm] = ((ef - ec) / lm ** 4, (ef - ec - et) / lm ** 4, et / lm ** 4)
    # Richardson: the lam^4 coefficients (linear terms in lam removed)
    c_ccsd = 2 * r[lam / 2][0] - r[lam][0]
    c_full = 2 * r[lam / 2][1] - r[lam][1]
    c_t = 2 * r[lam / 2][2] - r[lam][2]
    print(S, c_ccsd, c_full, c_t)
    assert abs(c_t) > 1e-3                       # (T) has a lam^4 term here
    assert abs(c_ccsd - c_t) < 0.02 * abs(c_t)   # FCI - CCSD starts with exactly that term
    assert abs(c_full) < 0.02 * abs(c_t)         # and FCI - CCSD(T) has none


def test_triples_need_canonical_orbitals():
    P = synth.small_problem(7, 3, 3, [2, 3], nvec=5, seed=4, offdiag_std=0.1)
    e, t, cs = cc.ccsd(P, (0, 4))
    with pytest.raises(ValueError, match="canonical"):
        cc.triples_correction(P, (0, 4), t, cs)
