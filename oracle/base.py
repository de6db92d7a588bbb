"""ORACLE (test infrastructure): base-model energies of tuples.

The paper expands the difference between the CASCI energies and those of a
cheaper base model (MBE-FCI-b, Sec. 4.2.1 and Table 3: a CCSD(T) base; Sec. 1
on coupled-cluster base models): each tuple contributes
eps(S) - eps_base(S) to Eq. 3, and the total is the base model's energy of
the whole space plus the expansion.  The base model here is second-order
Rayleigh-Schroedinger perturbation theory on the tuple's reference
determinant:

* Phi(S): the determinant of the tuple's CAS whose alpha (beta) electrons
  occupy the active orbitals of index below n_alpha (n_beta), the core
  doubly occupied (the aufbau occupation by index);
* H0 = sum over spin-orbitals of f_p n_p, with f_p the diagonal of the Fock
  operator of Phi: f_p = h_pp + sum over occupied spin-orbitals q of
  (pp|qq) - delta_spin (pq|qp);
* eps_base(S) = <Phi|H|Phi> - sum_{D != Phi} |<D|H|Phi>|^2 / (E0(D) - E0(Phi)),
  E0(D) the sum of f_p over the spin-orbitals occupied in D, D over the
  determinants of the CAS (only single and double excitations couple).

It is computed here by brute force over the CAS determinants (the column
H e_Phi from the Slater-Condon rules); the HIP library evaluates the
equivalent closed-form sums over excitations.
"""
from __future__ import annotations

import numpy as np

from . import fci


def _occ_lists(mask: int):
    out, p = [], 0
    while mask:
        if mask & 1:
            out.append(p)
        mask >>= 1
        p += 1
    return out


def reference_index(problem, sp: fci.CasSpace) -> int:
    """Index of Phi(S) in the CAS determinant list (ia * len(blist) + ib)."""
    ma = sum(1 << p for p in list(sp.core) + [p for p in sp.active if p < problem.nalpha])
    mb = sum(1 << p for p in list(sp.core) + [p for p in sp.active if p < problem.nbeta])
    ia = int(np.nonzero(sp.alist == np.uint64(ma))[0][0])
    ib = int(np.nonzero(sp.blist == np.uint64(mb))[0][0])
    return ia * len(sp.blist) + ib


def fock_diagonal(problem, occ_a, occ_b):
    """f_p (alpha, beta) of the determinant with the given occupied orbitals."""
    h, eri = problem.h, problem.eri
    n = problem.norb
    fa, fb = np.empty(n), np.empty(n)
    for p in range(n):
        coul = sum(eri[p, p, q, q] for q in occ_a) + sum(eri[p, p, q, q] for q in occ_b)
        fa[p] = h[p, p] + coul - sum(eri[p, q, q, p] for q in occ_a)
        fb[p] = h[p, p] + coul - sum(eri[p, q, q, p] for q in occ_b)
    return fa, fb


def base_energy(problem, tup) -> float:
    """eps_base(S) (total energy, constant and core included)."""
    sp = fci.cas_space(problem, tup)
    i0 = reference_index(problem, sp)
    e = np.zeros(sp.dim)
    e[i0] = 1.0
    col = fci.matvec(problem, sp, e)
    nb = len(sp.blist)
    ma, mb = int(sp.alist[i0 // nb]), int(sp.blist[i0 % nb])
    fa, fb = fock_diagonal(problem, _occ_lists(ma), _occ_lists(mb))

    def e0(ia, ib):
        return sum(fa[p] for p in _occ_lists(int(sp.alist[ia]))) + sum(fb[p] for p in _occ_lists(int(sp.blist[ib])))

    E0 = e0(i0 // nb, i0 % nb)
    e2 = 0.0
    for d in np.nonzero(col)[0]:
        if d == i0:
            continue
        den = e0(d // nb, d % nb) - E0
        if not den > 0.0:
            raise ValueError("base model: reference determinant not the lowest of H0")
        e2 -= col[d] ** 2 / den
    return float(col[i0] + e2)


def full_space_tuple(problem):
    """The tuple of every expansion orbital (the whole space of the MBE)."""
    return tuple(problem.expansion_space())
