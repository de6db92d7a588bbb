"""ORACLE (test infrastructure): the energy of one CASCI problem.

Sec. 2 of the paper defines the order-n term epsilon of a tuple of expansion
orbitals as the energy of a CASCI calculation in the composite space of the
reference space [Pi] and the tuple; orbitals outside that space are either
doubly occupied (frozen) or empty.  Here that energy is computed from its plain
definition: the lowest eigenvalue of the full Hamiltonian restricted to the
determinants whose core orbitals are doubly occupied, whose virtual orbitals
outside the active space are empty, and whose active orbitals hold the
remaining electrons in every possible way.  Matrix elements come from the
Slater-Condon rules in ``sc.c`` applied to full-orbital-space bit strings, so
no frozen-core effective Hamiltonian is ever formed here.

Spaces (the paper's partition, Sec. 2, generalised as in its case (b)):
  * occupied alpha orbitals: 0..nalpha-1; doubly occupied: 0..nbeta-1 (aufbau
    by index); singly occupied orbitals must belong to [Pi];
  * frozen core F = 0..nfrozen-1 (never correlated, Sec. 3);
  * expansion space X = all orbitals outside F and [Pi];
  * for a tuple S of X: active A = [Pi] u S, core C = F u (docc \\ A).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as sla

from . import native

DENSE_MAX = 1500          # dense eigensolver up to this many determinants


@dataclass
class CasSpace:
    active: list           # active orbitals A (ascending)
    core: list             # doubly occupied frozen orbitals C (ascending)
    na: int                # active alpha electrons
    nb: int                # active beta electrons
    alist: np.ndarray      # alpha strings, full-space bit masks, ascending
    blist: np.ndarray      # beta strings, full-space bit masks, ascending

    @property
    def dim(self) -> int:
        return len(self.alist) * len(self.blist)

    @property
    def act_mask(self) -> int:
        return sum(1 << p for p in self.active)


def strings(orbs, nel, fixed=()):
    """Every one-spin string with the `fixed` orbitals occupied plus `nel` of
    `orbs`, as full-space bit masks sorted ascending."""
    base = 0
    for p in fixed:
        base |= 1 << p
    out = []
    for comb in itertools.combinations(sorted(orbs), nel):
        m = base
        for p in comb:
            m |= 1 << p
        out.append(m)
    return np.array(sorted(out), dtype=np.uint64)


def cas_space(problem, tup) -> CasSpace:
    """Active space, core and electron counts for tuple `tup` (Sec. 2)."""
    n = problem.norb
    if n > 64:
        raise ValueError("oracle supports at most 64 orbitals")
    tup = tuple(tup)
    X = set(problem.expansion_space())
    if not set(tup) <= X or len(set(tup)) != len(tup):
        raise ValueError(f"tuple {tup} is not a set of expansion orbitals")
    A = sorted(set(problem.ref) | set(tup))
    docc = set(range(problem.nbeta))
    occa = set(range(problem.nalpha))
    C = sorted(set(range(problem.nfrozen)) | (docc - set(A)))
    if (occa - docc) - set(A):
        raise ValueError("singly occupied orbitals must lie in the reference space")
    if not set(C) <= docc:
        raise ValueError("frozen orbitals must be doubly occupied")
    na = problem.nalpha - len(C)
    nb = problem.nbeta - len(C)
    if not (0 <= nb <= len(A) and 0 <= na <= len(A)):
        raise ValueError("electron count outside the active space")
    return CasSpace(A, C, na, nb, strings(A, na, C), strings(A, nb, C))


def hamiltonian_matrix(problem, sp: CasSpace) -> np.ndarray:
    """Dense H (E_const on the diagonal) over the CAS determinants, index
    ia * len(blist) + ib."""
    L = native.lib()
    h = np.ascontiguousarray(problem.h, dtype=np.float64)
    eri = np.ascontiguousarray(problem.eri, dtype=np.float64)
    H = np.empty((sp.dim, sp.dim))
    L.sc_hmat(problem.norb, native.ptr(h), native.ptr(eri), float(problem.e_const),
              len(sp.alist), native.ptr(sp.alist), len(sp.blist), native.ptr(sp.blist),
              native.ptr(H))
    return H


def matvec(problem, sp: CasSpace, x: np.ndarray) -> np.ndarray:
    """Matrix-free y = H x over the CAS determinants."""
    L = native.lib()
    h = np.ascontiguousarray(problem.h, dtype=np.float64)
    eri = np.ascontiguousarray(problem.eri, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    L.sc_matvec(problem.norb, native.ptr(h), native.ptr(eri), float(problem.e_const),
                len(sp.alist), native.ptr(sp.alist), len(sp.blist), native.ptr(sp.blist),
                sp.act_mask, native.ptr(x), native.ptr(y))
    return y


def lowest_eigenpair(problem, sp: CasSpace, want_vector: bool = False, dense_max: int = DENSE_MAX):
    """Lowest eigenvalue (and normalised eigenvector) of H over the CAS."""
    if sp.dim <= dense_max:
        H = hamiltonian_matrix(problem, sp)
        if want_vector:
            w, v = np.linalg.eigh(H)
            return float(w[0]), v[:, 0].copy()
        return float(np.linalg.eigvalsh(H)[0]), None
    h = np.ascontiguousarray(problem.h, dtype=np.float64)
    eri = np.ascontiguousarray(problem.eri, dtype=np.float64)
    L = native.lib()
    na, nb = len(sp.alist), len(sp.blist)
    mask = sp.act_mask

    def mv(x):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
        y = np.empty_like(x)
        L.sc_matvec(problem.norb, native.ptr(h), native.ptr(eri), float(problem.e_const),
                    na, native.ptr(sp.alist), nb, native.ptr(sp.blist), mask,
                    native.ptr(x), native.ptr(y))
        return y

    op = sla.LinearOperator((sp.dim, sp.dim), matvec=mv, dtype=np.float64)
    v0 = np.random.default_rng(20190507).standard_normal(sp.dim)
    w, v = sla.eigsh(op, k=1, which="SA", v0=v0, tol=1e-14, ncv=min(sp.dim - 1, 40),
                     maxiter=100000)
    vec = v[:, 0] / np.linalg.norm(v[:, 0])
    return float(w[0]), (vec if want_vector else None)


def casci_energy(problem, tup, want_vector: bool = False, dense_max: int = DENSE_MAX):
    """epsilon(tup): lowest eigenvalue of H over the CAS of [Pi] u tup (total
    energy, frozen-core and constant contributions included)."""
    sp = cas_space(problem, tup)
    e, v = lowest_eigenpair(problem, sp, want_vector, dense_max)
    return (e, v, sp) if want_vector else e


def fci_energy(problem, dense_max: int = DENSE_MAX) -> float:
    """FCI energy inside the non-frozen orbitals: the CASCI of all of X."""
    return casci_energy(problem, tuple(problem.expansion_space()), dense_max=dense_max)
