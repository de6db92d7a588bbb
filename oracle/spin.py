"""ORACLE (test infrastructure): total spin of CAS vectors, and the lowest
CASCI state of a given total spin.

The paper's energies are those of particular states (its test molecules'
singlet ground states, Sec. 4), not simply the lowest eigenvalue of a fixed
(n_alpha, n_beta) sector.  Here a state's total spin comes from its plain
definition,

    S^2 = S_- S_+ + S_z (S_z + 1),   S_+ = sum_p a+_{p alpha} a_{p beta},
    S_- = S_+^dagger,

so <c|S^2|c> = |S_+ c|^2 + S_z (S_z + 1) |c|^2, with S_+ applied to
full-orbital-space determinants (alpha creators left of beta creators, each
in ascending orbital order, the ordering of the oracle's Slater-Condon
rules).  The spin-targeted CASCI energy of a tuple is the lowest eigenvalue
of H over its CAS whose eigenvector has <S^2> = S(S+1), S defaulting to the
sector's own S_z = (n_alpha - n_beta) / 2 (for closed shells: the lowest
singlet); eigenpairs are found by dense diagonalisation or, above the dense
limit, by ARPACK for the lowest few, more if none of them has that spin.

Nothing here is shared with the HIP library, which reaches the same states
through a level shift (H + lambda S_- S_+) inside its sigma kernels.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla

from . import fci, native


def _popc(x: int) -> int:
    return bin(x).count("1")


def s_plus(sp: fci.CasSpace, c: np.ndarray) -> dict:
    """S_+ c as a dict {(alpha mask, beta mask): coefficient} over the
    determinants with one more alpha and one fewer beta electron."""
    out = {}
    nb_list = len(sp.blist)
    for ia, a in enumerate(sp.alist):
        a = int(a)
        na_tot = _popc(a)
        for ib, b in enumerate(sp.blist):
            x = c[ia * nb_list + ib]
            if x == 0.0:
                continue
            b = int(b)
            for p in range(64):
                bit = 1 << p
                if bit > b:
                    break
                if not (b & bit) or (a & bit):
                    continue
                # a_{p beta}: the alpha block and the beta creators below p
                # stand to its left
                s = na_tot + _popc(b & (bit - 1))
                # a+_{p alpha}: the alpha creators below p stand to its left
                s += _popc(a & (bit - 1))
                key = (a | bit, b & ~bit)
                out[key] = out.get(key, 0.0) + (-x if s & 1 else x)
    return out


def s_minus_s_plus(sp: fci.CasSpace, c: np.ndarray) -> np.ndarray:
    """S_- S_+ c over the CAS determinants (S_- applied to the S_+ image,
    projected back; S_- maps into the original sector exactly)."""
    up = s_plus(sp, c)
    aidx = {int(a): i for i, a in enumerate(sp.alist)}
    bidx = {int(b): i for i, b in enumerate(sp.blist)}
    nb_list = len(sp.blist)
    y = np.zeros(sp.dim)
    for (a, b), x in up.items():
        if x == 0.0:
            continue
        na_tot = _popc(a)
        for p in range(64):
            bit = 1 << p
            if bit > a:
                break
            if not (a & bit) or (b & bit):
                continue
            # S_- = sum_p a+_{p beta} a_{p alpha}: first a_{p alpha} (alpha
            # creators below p to its left), then a+_{p beta} (the remaining
            # alpha block and the beta creators below p to its left)
            s = _popc(a & (bit - 1))
            s += (na_tot - 1) + _popc(b & (bit - 1))
            a2, b2 = a & ~bit, b | bit
            ia, ib = aidx.get(a2), bidx.get(b2)
            if ia is None or ib is None:
                raise AssertionError("S_- left the CAS")
            y[ia * nb_list + ib] += -x if s & 1 else x
    return y


def sz(sp: fci.CasSpace) -> float:
    return 0.5 * (_popc(int(sp.alist[0])) - _popc(int(sp.blist[0])))


def s2_expectation(sp: fci.CasSpace, c: np.ndarray) -> float:
    """<c|S^2|c> / <c|c>."""
    n2 = float(np.dot(c, c))
    up = s_plus(sp, c)
    m = sz(sp)
    return (sum(v * v for v in up.values()) + m * (m + 1.0) * n2) / n2


def lowest_with_spin(problem, sp: fci.CasSpace, S=None, want_vector: bool = False,
                     dense_max: int = fci.DENSE_MAX, tol: float = 1e-6):
    """Lowest eigenvalue of H over the CAS among eigenvectors of total spin S
    (default: the sector's S_z).  Returns (energy, vector or None, S)."""
    if S is None:
        S = abs(sz(sp))
    target = S * (S + 1.0)
    if sp.dim <= dense_max:
        w, v = np.linalg.eigh(fci.hamiltonian_matrix(problem, sp))
        for i in range(len(w)):
            if abs(s2_expectation(sp, v[:, i]) - target) < tol:
                return float(w[i]), (v[:, i].copy() if want_vector else None), S
        raise ValueError(f"no eigenstate of spin {S} in this CAS")
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
    k = 8
    while True:
        k = min(k, sp.dim - 2)
        w, v = sla.eigsh(op, k=k, which="SA", v0=v0, tol=1e-14, ncv=min(sp.dim - 1, max(2 * k + 1, 40)),
                         maxiter=100000)
        order = np.argsort(w)
        for i in order:
            vec = v[:, i] / np.linalg.norm(v[:, i])
            if abs(s2_expectation(sp, vec) - target) < tol:
                return float(w[i]), (vec if want_vector else None), S
        if k >= sp.dim - 2 or k >= 64:
            raise ValueError(f"no eigenstate of spin {S} among the {k} lowest")
        k *= 2


def casci_energy_spin(problem, tup, S=None) -> float:
    """Spin-targeted epsilon(tup): the lowest CASCI state of spin S (default
    the sector's S_z, i.e. the lowest singlet for closed shells)."""
    sp = fci.cas_space(problem, tup)
    return lowest_with_spin(problem, sp, S)[0]
