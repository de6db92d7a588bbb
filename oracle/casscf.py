"""ORACLE (test infrastructure): CASSCF orbitals of the reference space.

The paper's best expansion references are CASSCF orbitals (Sec. 2, the
expansion reference of Fig. 2; Sec. 4.1.3 and Sec. 4.2.2): the orbitals are
chosen to minimise the CASCI energy of the reference space [Pi], and the MBE
is then carried out in that orbital basis.  Definitions used here:

* spaces: frozen orbitals (0 .. nfrozen-1, never rotated), core C (doubly
  occupied outside [Pi]), active A = [Pi], virtual V (the rest);
* orbitals phi'_j = sum_i phi_i U_ij, U = U_0 expm(K), K antisymmetric with
  K_pq = kappa, K_qp = -kappa for the non-redundant pairs (C, A), (C, V),
  (A, V) (rotations inside a space leave the CASCI energy unchanged);
* h' = U^T h U, (ij|kl)' = sum U_pi U_qj U_rk U_sl (pq|rs);
* E(U) = the lowest CASCI eigenvalue of [Pi] with h', (..|..)' (the state of
  epsilon(()) of the MBE), or with ``spin`` = S the lowest one of total spin
  S (oracle/spin.py), the state a spin-targeted expansion takes;
* gradient: with the full-space density matrices gamma, Gamma of that state
  in the basis U and the generalised Fock matrix
      F_pq = sum_r gamma_pr h'_qr + sum_rst Gamma_prst (qr|st)',
  a rotation dK at U changes E by 2 sum_ij dK_ij F_ji, so dE/dkappa_pq of the
  local rotation U expm(K) at K = 0 is 2 (F_qp - F_pq);
* the CASSCF orbitals minimise E over kappa; the oracle takes a plain BFGS
  minimisation (scipy) in the fixed frame U_0 expm(K(kappa)), whose exact
  gradient is the chain rule through the Frechet derivative of expm, and
  then solves g(kappa) = 0 from that minimum by Newton's method (energies
  stop resolving BFGS's line search near |g| = 1e-8);
* canonical orbitals: in the optimised basis, the core and virtual blocks are
  rotated to the eigenvectors of the Fock matrix
      f_pq = h'_pq + sum_rs gamma_rs [ (pq|rs)' - 1/2 (pr|sq)' ]
  (ascending eigenvalues, kept at the space's own orbital positions), the
  active block to the natural orbitals (eigenvectors of gamma_AA, descending
  occupation), and every column of U is signed so that its entry of largest
  magnitude is positive.  These orbitals are unique when the eigenvalues in
  each block are distinct.

Nothing here is shared with the HIP library.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import scipy.linalg as sl
import scipy.optimize as so

from . import fci, rdm, spin as spin_mod


def spaces(problem):
    """(frozen, core, active, virtual) orbital lists."""
    n = problem.norb
    F = list(range(problem.nfrozen))
    A = sorted(problem.ref)
    docc = set(range(problem.nbeta))
    C = sorted(docc - set(A) - set(F))
    V = sorted(set(range(n)) - set(F) - set(A) - docc)
    return F, C, A, V


def rotation_pairs(problem):
    """Non-redundant rotation pairs (p, q): core-active, core-virtual,
    active-virtual."""
    _, C, A, V = spaces(problem)
    return [(p, q) for p in C for q in A] + [(p, q) for p in C for q in V] + [(p, q) for p in A for q in V]


def transform(problem, U):
    """The problem with its integrals in the orbitals phi'_j = sum_i phi_i U_ij."""
    h = U.T @ problem.h @ U
    e = problem.eri
    e = np.tensordot(e, U, axes=([0], [0]))          # (q r s, i)
    e = np.tensordot(e, U, axes=([0], [0]))          # (r s, i, j)
    e = np.tensordot(e, U, axes=([0], [0]))          # (s, i, j, k)
    e = np.tensordot(e, U, axes=([0], [0]))          # (i, j, k, l)
    return replace(problem, h=np.ascontiguousarray(h), eri=np.ascontiguousarray(e))


def reference_state(problem, spin=None):
    """Energy and full-space gamma, Gamma of the reference-space CASCI (its
    lowest state, or with spin = S its lowest state of total spin S)."""
    if spin is None:
        e, v, sp = fci.casci_energy(problem, (), want_vector=True)
    else:
        sp = fci.cas_space(problem, ())
        e, v, _ = spin_mod.lowest_with_spin(problem, sp, spin, want_vector=True)
    g1, g2 = rdm.rdm12(problem, sp, v)
    return e, g1, g2


def generalised_fock(problem, g1, g2):
    """F_pq = sum_r gamma_pr h_qr + sum_rst Gamma_prst (qr|st)."""
    return g1 @ problem.h.T + np.einsum("prst,qrst->pq", g2, problem.eri)


def fock(problem, g1):
    """f_pq = h_pq + sum_rs gamma_rs [(pq|rs) - 1/2 (pr|sq)]."""
    return problem.h + np.einsum("rs,pqrs->pq", g1, problem.eri) - 0.5 * np.einsum("rs,prsq->pq", g1, problem.eri)


def local_gradient(problem, pairs=None, spin=None):
    """Energy and dE/dkappa_pq of a local rotation expm(K) at K = 0, one entry
    per pair: 2 (F_qp - F_pq)."""
    pairs = rotation_pairs(problem) if pairs is None else pairs
    e, g1, g2 = reference_state(problem, spin)
    F = generalised_fock(problem, g1, g2)
    return e, np.array([2.0 * (F[q, p] - F[p, q]) for p, q in pairs])


def kappa_matrix(n, pairs, kappa):
    K = np.zeros((n, n))
    for (p, q), k in zip(pairs, kappa):
        K[p, q] = k
        K[q, p] = -k
    return K


def energy_and_gradient(problem, U0, pairs, kappa, spin=None):
    """E(U0 expm(K(kappa))) and its exact gradient with respect to kappa: the
    energy changes by sum_ab M_ab dU_ab with M = 2 U F^T (F the generalised
    Fock matrix in the basis U), and dU = U0 L(K, dK) with L the Frechet
    derivative of expm."""
    n = problem.norb
    K = kappa_matrix(n, pairs, kappa)
    U = U0 @ sl.expm(K)
    pu = transform(problem, U)
    e, g1, g2 = reference_state(pu, spin)
    F = generalised_fock(pu, g1, g2)
    M = 2.0 * U @ F.T
    grad = np.empty(len(pairs))
    for k, (p, q) in enumerate(pairs):
        dK = np.zeros((n, n))
        dK[p, q], dK[q, p] = 1.0, -1.0
        L = sl.expm_frechet(K, dK, compute_expm=False)
        grad[k] = np.sum(M * (U0 @ L))
    return e, grad


def optimise(problem, U0=None, g_tol=1e-9, max_iter=2000, spin=None):
    """CASSCF orbitals (not yet canonical): U minimising E, and E."""
    n = problem.norb
    U0 = np.eye(n) if U0 is None else U0
    pairs = rotation_pairs(problem)
    if not pairs:
        return U0, reference_state(transform(problem, U0), spin)[0]
    res = so.minimize(lambda x: energy_and_gradient(problem, U0, pairs, x, spin), np.zeros(len(pairs)), jac=True,
                      method="BFGS", options={"gtol": g_tol, "maxiter": max_iter})
    x = res.x
    # BFGS stops where energy differences no longer resolve its line search
    # (|g| of about 1e-8); the stationarity condition g(kappa) = 0 is smooth
    # and is solved further from that minimum by Newton's method, the
    # Jacobian of the exact gradient by central differences
    grad = lambda y: energy_and_gradient(problem, U0, pairs, y, spin)[1]  # noqa: E731
    for _ in range(8):
        g = grad(x)
        if np.abs(g).max() <= g_tol:
            break
        hstep = 1e-6
        J = np.empty((len(x), len(x)))
        for k in range(len(x)):
            d = np.zeros(len(x))
            d[k] = hstep
            J[:, k] = (grad(x + d) - grad(x - d)) / (2.0 * hstep)
        x = x - np.linalg.solve(0.5 * (J + J.T), g)
    U = U0 @ sl.expm(kappa_matrix(n, pairs, x))
    return U, float(energy_and_gradient(problem, U0, pairs, x, spin)[0])


def canonicalise(problem, U, spin=None):
    """The canonical CASSCF orbitals from optimised orbitals U (see the module
    docstring)."""
    _, C, A, V = spaces(problem)
    pu = transform(problem, U)
    _, g1, _ = reference_state(pu, spin)
    f = fock(pu, g1)
    R = np.eye(problem.norb)
    for block, mat, descending in ((C, f, False), (V, f, False), (A, g1, True)):
        if not block:
            continue
        w, v = np.linalg.eigh(mat[np.ix_(block, block)])
        order = np.argsort(-w if descending else w, kind="stable")
        R[np.ix_(block, block)] = v[:, order]
    Uc = U @ R
    for j in range(Uc.shape[1]):
        i = int(np.argmax(np.abs(Uc[:, j])))
        if Uc[i, j] < 0.0:
            Uc[:, j] = -Uc[:, j]
    return Uc


def casscf(problem, U0=None, g_tol=1e-9, spin=None):
    """(E_CASSCF, canonical U, the problem in the canonical CASSCF orbitals)."""
    U, e = optimise(problem, U0, g_tol, spin=spin)
    Uc = canonicalise(problem, U, spin)
    return e, Uc, transform(problem, Uc)
