"""ORACLE (test infrastructure): restricted closed-shell Hartree-Fock orbitals.

The paper's expansions are formulated in the molecular orbitals of a preceding
Hartree-Fock calculation (Sec. 1; Sec. 2, where the HF determinant is the
simplest expansion reference), and its CCSD(T) base model (Sec. 4.2.1) is
built on that determinant.  Here, for a closed-shell problem given in an
orthonormal orbital basis: the n_occ = n_alpha = n_beta orbitals C_occ that
minimise

    E(C) = e_const + sum_pq D_pq (h_pq + f_pq),   D = C_occ C_occ^T,
    f(D)_pq = h_pq + sum_rs D_rs (2 (pq|rs) - (pr|sq)),

found by energy descent over the occupied-virtual orbital rotations (the
plain Roothaan iteration oscillates on these synthetic problems), finished by
Newton steps, until the orbital gradient 4 f_ai is below 1e-10.  Canonical form: the Fock operator
diagonalised in the occupied and in the virtual block, each ascending
(occupied orbitals first), each orbital signed so that its largest entry is
positive; the problem in them has h' = C^T h C and
(pq|rs)' = sum C_ap C_bq C_cr C_ds (ab|cd).
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import scipy.linalg


def fock(problem, D):
    eri = problem.eri
    return problem.h + 2.0 * np.einsum("pqrs,rs->pq", eri, D) - np.einsum("prsq,rs->pq", eri, D)


def energy(problem, D):
    return float(problem.e_const + np.sum(D * (problem.h + fock(problem, D))))


def _eigh_signed(F):
    w, C = np.linalg.eigh(F)
    for j in range(C.shape[1]):
        k = int(np.argmax(np.abs(C[:, j])))
        if C[k, j] < 0.0:
            C[:, j] = -C[:, j]
    return w, C


def _occ_virt_fock(problem, C):
    no = problem.nalpha
    D = C[:, :no] @ C[:, :no].T
    return D, C.T @ fock(problem, D) @ C


def _rotate(C, x, no):
    n = C.shape[0]
    K = np.zeros((n, n))
    K[no:, :no] = x.reshape(n - no, no)
    return C @ scipy.linalg.expm(K - K.T)


def _hessian(problem, C, s: float = 1e-4):
    """Orbital Hessian by central differences of the gradient 4 f_ai."""
    no = problem.nalpha
    npar = (problem.norb - no) * no
    H = np.zeros((npar, npar))
    for k in range(npar):
        x = np.zeros(npar)
        x[k] = s
        gp = 4.0 * _occ_virt_fock(problem, _rotate(C, x, no))[1][no:, :no]
        gm = 4.0 * _occ_virt_fock(problem, _rotate(C, -x, no))[1][no:, :no]
        H[:, k] = (gp - gm).ravel() / (2.0 * s)
    return 0.5 * (H + H.T)


def rhf(problem, tol: float = 1e-10, max_iter: int = 3000):
    """(E_HF, C, eps): canonical RHF orbitals as the columns of C (occupied
    first), eps the Fock diagonal in them.  Energy descent over the
    occupied-virtual rotations C <- C exp(K), K_ai = -K_ia = kappa_ai: the
    gradient at kappa = 0 is 4 f_ai in the current orbitals; steps from
    limited-memory BFGS (8 pairs, in the frame of the current orbitals)
    preconditioned by 4 (f_aa - f_ii) floored at 0.05, at most 0.5 per
    element, halved until the energy does not rise; once the gradient is
    below 1e-5, Newton steps on the Hessian from central differences of the
    gradient (at most six; quasi-Newton converges slowly there).  Stops when
    the largest gradient element is below tol."""
    if problem.nalpha != problem.nbeta:
        raise ValueError("RHF needs a closed-shell problem")
    n, no = problem.norb, problem.nalpha
    _, C = _eigh_signed(problem.h)
    D, Fm = _occ_virt_fock(problem, C)
    E = energy(problem, D)
    S, Y = [], []
    g_old = None
    step_old = None
    newton = 0
    for _ in range(max_iter):
        g = 4.0 * Fm[no:, :no]
        if np.abs(g).max() < tol:
            break
        if np.abs(g).max() < 1e-5 and newton < 6:
            # Newton step on the Hessian from central differences of the gradient
            H = _hessian(problem, C)
            try:
                L = np.linalg.cholesky(H)
                x = -scipy.linalg.cho_solve((L, True), g.ravel())
                C = _rotate(C, x, no)
                D, Fm = _occ_virt_fock(problem, C)
                E = energy(problem, D)
                newton += 1
                S, Y, g_old = [], [], None
                continue
            except np.linalg.LinAlgError:
                newton = 6                        # not positive definite: keep descending
        if g_old is not None:
            y = (g - g_old).ravel()
            s_ = step_old.ravel()
            if s_ @ y > 1e-16:
                S.append(s_)
                Y.append(y)
                S, Y = S[-8:], Y[-8:]
        hd = np.maximum(4.0 * (np.diag(Fm)[no:, None] - np.diag(Fm)[None, :no]), 0.05).ravel()
        q = g.ravel().copy()
        al = []
        for s_, y in zip(reversed(S), reversed(Y)):
            a = (s_ @ q) / (s_ @ y)
            al.append(a)
            q -= a * y
        r = q / hd
        for (s_, y), a in zip(zip(S, Y), reversed(al)):
            b = (y @ r) / (s_ @ y)
            r += (a - b) * s_
        step = -r.reshape(n - no, no)
        if np.sum(step * g) >= 0.0:              # not a descent direction: preconditioned gradient
            step = -(g.ravel() / hd).reshape(n - no, no)
            S, Y = [], []
        step = np.clip(step, -0.5, 0.5)
        alpha = 1.0
        while True:
            K = np.zeros((n, n))
            K[no:, :no] = alpha * step
            K = K - K.T
            Cn = C @ scipy.linalg.expm(K)
            Dn, Fn = _occ_virt_fock(problem, Cn)
            En = energy(problem, Dn)
            # (close to the minimum the energy cannot resolve the step: the
            # quasi-Newton step is taken as it is)
            if En <= E + 1e-13 * max(1.0, abs(E)) or alpha < 1e-6 or np.abs(g).max() < 1e-5:
                break
            alpha *= 0.5
        g_old = g
        step_old = alpha * step
        C, D, Fm, E = Cn, Dn, Fn, En
    else:
        raise RuntimeError("RHF did not converge")
    # canonical: the Fock operator diagonalised in the occupied and in the
    # virtual block, each ascending
    for blk in (slice(0, no), slice(no, n)):
        w, V = np.linalg.eigh(Fm[blk, blk])
        C[:, blk] = C[:, blk] @ V
    for j in range(n):
        k = int(np.argmax(np.abs(C[:, j])))
        if C[k, j] < 0.0:
            C[:, j] = -C[:, j]
    D, Fm = _occ_virt_fock(problem, C)
    return energy(problem, D), C, np.diag(Fm).copy()


def transform(problem, C):
    """The problem with its integrals in the orbitals C (columns)."""
    h = C.T @ problem.h @ C
    eri = np.einsum("pqrs,pa,qb,rc,sd->abcd", problem.eri, C, C, C, C, optimize=True)
    return replace(problem, h=h, eri=np.ascontiguousarray(eri))


def hf_problem(problem):
    """(E_HF, the problem in canonical RHF orbitals, C)."""
    e, C, _ = rhf(problem)
    return e, transform(problem, C), C
