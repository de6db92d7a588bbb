"""ORACLE (test infrastructure): CASCI energies of a given spatial symmetry.

The paper's energies are those of states of a given symmetry (the 1A1 state
of H2O, Sec. 4.1.1; the X 1Sigma_g+ state of N2 and the states of C2, Sec.
4.1.2-4.1.3).  For an Abelian point group whose irreps are labelled 0..7, so
that the product of two irreps is the XOR of their labels, every determinant
has the irrep given by the XOR of the labels of its occupied spin-orbitals
(doubly occupied orbitals cancel), and a Hamiltonian that respects the
labels couples only determinants of one irrep.  The energy of a tuple for
target irrep G is then, by definition, the lowest eigenvalue of H restricted
to the determinants of its CAS whose irrep is G (an error if there is none).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla

from . import fci


def det_irrep(labels, ma: int, mb: int) -> int:
    g = 0
    for m in (ma, mb):
        p = 0
        while m:
            if m & 1:
                g ^= int(labels[p])
            m >>= 1
            p += 1
    return g


def irrep_indices(problem, sp: fci.CasSpace, labels, target: int):
    nb = len(sp.blist)
    return [i * nb + j for i, a in enumerate(sp.alist) for j, b in enumerate(sp.blist)
            if det_irrep(labels, int(a), int(b)) == target]


def respects(problem, labels, tol: float = 1e-12) -> bool:
    lab = np.asarray(labels)
    h_ok = np.abs(problem.h[lab[:, None] != lab[None, :]]).max(initial=0.0) <= tol
    x = lab[:, None, None, None] ^ lab[None, :, None, None] ^ lab[None, None, :, None] ^ lab[None, None, None, :]
    return bool(h_ok and np.abs(problem.eri[x != 0]).max(initial=0.0) <= tol)


def casci_energy_irrep(problem, tup, labels, target: int) -> float:
    sp = fci.cas_space(problem, tup)
    idx = irrep_indices(problem, sp, labels, target)
    if not idx:
        raise ValueError("no determinant of the target irrep in the CAS")
    if sp.dim <= fci.DENSE_MAX:
        H = fci.hamiltonian_matrix(problem, sp)
        return float(np.linalg.eigvalsh(H[np.ix_(idx, idx)])[0])
    idx = np.asarray(idx)

    def mv(x):
        full = np.zeros(sp.dim)
        full[idx] = np.asarray(x).reshape(-1)
        return fci.matvec(problem, sp, full)[idx]
    op = sla.LinearOperator((len(idx), len(idx)), matvec=mv, dtype=np.float64)
    v0 = np.random.default_rng(20190507).standard_normal(len(idx))
    w = sla.eigsh(op, k=1, which="SA", v0=v0, tol=1e-14, ncv=min(len(idx) - 1, 40), maxiter=100000,
                  return_eigenvectors=False)
    return float(w[0])
