"""ORACLE (test infrastructure): density matrices and MBE gradients.

For a normalised CASCI ground state c of tuple S (full orbital space, frozen
core included):
    gamma_pq      = <c| E_pq |c>
    Gamma_pqrs    = <c| E_pq E_rs |c> - delta_qr gamma_ps
                  = sum_{u,v} <c| a+_{pu} a+_{rv} a_{sv} a_{qu} |c>,
so that eps(S) = E_const + sum h_pq gamma_pq + 1/2 sum (pq|rs) Gamma_pqrs and,
by the Hellmann-Feynman theorem for a non-degenerate lowest eigenvalue,
d eps(S)/d h_pq = gamma_pq and d eps(S)/d (pq|rs) = 1/2 Gamma_pqrs when every
array entry is treated as an independent variable.

The summed MBE energy E = sum_S d_eps(S) is linear in the tuple energies
(Eq. 3: d_eps = (I + L)^-1 eps with L_ST = 1 iff T is a proper subtuple of S,
both computed), so dE/d eps(S) = w_S with w = (I + L^T)^-1 1, an integer
vector, and dE = sum_S w_S d eps(S).  The tuple set is held fixed.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import fci, native


def rdm12(problem, sp: fci.CasSpace, vec: np.ndarray):
    """Full-space gamma (n, n) and Gamma (n, n, n, n) of `vec` over the CAS."""
    n = problem.norb
    L = native.lib()
    c = np.ascontiguousarray(vec, dtype=np.float64)
    g1 = np.empty((n, n))
    g2 = np.empty((n, n, n, n))
    L.sc_rdm12(n, len(sp.alist), native.ptr(sp.alist), len(sp.blist), native.ptr(sp.blist),
               native.ptr(c), native.ptr(g1), native.ptr(g2))
    return g1, g2


def energy_from_rdms(problem, g1, g2) -> float:
    return float(problem.e_const + np.sum(problem.h * g1) + 0.5 * np.sum(problem.eri * g2))


def adjoint_weights(result) -> dict:
    """w_S for every computed tuple S: w_S = 1 - sum_{U computed, U proper
    superset of S} w_U, evaluated from the highest order down (integers)."""
    orders = result.orders
    present = set(result.all_tuples())
    acc = {S: 0 for S in present}
    w = {}
    for o in reversed(orders):
        for U in o.tuples:
            w[U] = 1 - acc[U]
            for m in range(len(U)):
                for T in itertools.combinations(U, m):
                    if T in present:
                        acc[T] += w[U]
    return w


def mbe_gradient(problem, result, dense_max: int = fci.DENSE_MAX):
    """(dE/dh, dE/d(pq|rs)) of the summed MBE energy with the tuple set of
    `result` held fixed: sum_S w_S (gamma(S), 1/2 Gamma(S))."""
    n = problem.norb
    gh = np.zeros((n, n))
    ge = np.zeros((n, n, n, n))
    w = adjoint_weights(result)
    for S, wS in w.items():
        if wS == 0:
            continue
        e, v, sp = fci.casci_energy(problem, S, want_vector=True, dense_max=dense_max)
        g1, g2 = rdm12(problem, sp, v)
        gh += wS * g1
        ge += 0.5 * wS * g2
    return gh, ge
