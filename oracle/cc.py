"""ORACLE (test infrastructure): coupled-cluster base energies of tuples.

The paper's MBE-FCI-b expands eps(S) - eps_base(S) with a CCSD(T) base
(Sec. 4.2.1 and Table 3; Sec. 1 on coupled-cluster base models).  Both parts
are taken here from their definitions, on the determinants of the tuple's CAS
and its reference determinant Phi(S) (oracle/base.py: the core doubly
occupied, the active orbitals of index below n_alpha (n_beta) holding the
alpha (beta) electrons):

* CCSD.  T = T1 + T2 = sum_mu t_mu tau_mu over the spin-orbital single and
  double excitation operators tau_mu that move electrons from occupied to
  virtual active spin-orbitals of Phi; |mu> = tau_mu |Phi>.  The amplitudes
  solve <mu| exp(-T) H exp(T) |Phi> = 0 for every mu, and
  E_CCSD = <Phi| H exp(T) |Phi>.
* (T), for canonical orbitals (the Fock operator of Phi diagonal on the
  active orbitals; anything else raises).  Over the triply excited
  determinants mu, with D_mu = E0(Phi) - E0(mu) (E0: the sum of the Fock
  diagonal over occupied spin-orbitals),
      x = P_T H T2 |Phi>          (D x the connected triples amplitudes),
      y = P_T T1 P_D H |Phi>      (D y the disconnected ones),
      E_(T) = sum_mu x_mu (x_mu + y_mu) / D_mu,
  P_T and P_D the projectors on the triply and doubly excited determinants.

Operators are sparse matrices on the determinant basis with the phase
convention of the CASCI oracle (alpha creators to the left of beta creators,
each in ascending order); exp(+-T) is a finite Taylor series (T only
excites, so it is nilpotent).  The amplitude equations are solved by a
Jacobi iteration on the residual with the diagonal shifts H_mumu - H_PhiPhi,
accelerated by DIIS, until the largest residual is below 1e-12; the solver
only finds the root, the definition above is what is computed.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sps

from . import base, fci


def _parity(mask: int, p: int) -> int:
    return bin(mask & ((1 << p) - 1)).count("1") & 1


def _apply(ops, ia: int, ib: int):
    """Apply a product of creators/annihilators, rightmost first.  ops: list
    of (spin, orbital, create) in the written order.  Returns (sign, ia, ib)
    or None."""
    sign = 1
    for spin, p, create in reversed(ops):
        bit = 1 << p
        if spin == 0:
            if create == bool(ia & bit):
                return None
            if _parity(ia, p):
                sign = -sign
            ia ^= bit
        else:
            if create == bool(ib & bit):
                return None
            if (bin(ia).count("1") + _parity(ib, p)) & 1:
                sign = -sign
            ib ^= bit
    return sign, ia, ib


class CCSpace:
    """The CAS of a tuple with Phi, its excitations and their operators."""

    def __init__(self, problem, tup):
        self.problem = problem
        self.sp = sp = fci.cas_space(problem, tup)
        self.nb = len(sp.blist)
        self.index = {(int(a), int(b)): i * self.nb + j
                      for i, a in enumerate(sp.alist) for j, b in enumerate(sp.blist)}
        self.i0 = base.reference_index(problem, sp)
        self.phi = (int(sp.alist[self.i0 // self.nb]), int(sp.blist[self.i0 % self.nb]))
        act = sp.active
        occ = [[p for p in act if p < problem.nalpha], [p for p in act if p < problem.nbeta]]
        vir = [[p for p in act if p >= problem.nalpha], [p for p in act if p >= problem.nbeta]]
        self.occ, self.vir = occ, vir
        ex = []      # (rank, ops) with ops in written order (creators left)
        for s in (0, 1):
            for i in occ[s]:
                for a in vir[s]:
                    ex.append((1, [(s, a, True), (s, i, False)]))
        for s in (0, 1):
            for i, j in itertools.combinations(occ[s], 2):
                for a, b in itertools.combinations(vir[s], 2):
                    ex.append((2, [(s, a, True), (s, b, True), (s, j, False), (s, i, False)]))
        for i in occ[0]:
            for a in vir[0]:
                for j in occ[1]:
                    for b in vir[1]:
                        ex.append((2, [(0, a, True), (0, i, False), (1, b, True), (1, j, False)]))
        self.rank = np.array([r for r, _ in ex], dtype=int)
        self.ops = [self._matrix(o) for _, o in ex]
        # |mu> = tau_mu |Phi>: one entry each
        self.bra = sps.vstack([m[:, self.i0].T for m in self.ops]).tocsr() if ex else None
        dets = [(int(a), int(b)) for a in sp.alist for b in sp.blist]
        pa, pb = self.phi
        self.level = np.array([(bin(a ^ pa).count("1") + bin(b ^ pb).count("1")) // 2 for a, b in dets])
        self.H = fci.hamiltonian_matrix(problem, sp) if sp.dim <= 3000 else None

    def _matrix(self, ops):
        rows, cols, vals = [], [], []
        for (ia, ib), d in self.index.items():
            r = _apply(ops, ia, ib)
            if r is None:
                continue
            s, ja, jb = r
            rows.append(self.index[(ja, jb)])
            cols.append(d)
            vals.append(float(s))
        dim = self.sp.dim
        return sps.csr_matrix((vals, (rows, cols)), shape=(dim, dim))

    def hop(self, v):
        return self.H @ v if self.H is not None else fci.matvec(self.problem, self.sp, v)

    def t_matrix(self, t, ranks=(1, 2)):
        dim = self.sp.dim
        T = sps.csr_matrix((dim, dim))
        for c, m, r in zip(t, self.ops, self.rank):
            if r in ranks and c != 0.0:
                T = T + c * m
        return T

    @staticmethod
    def expm_apply(T, v, sign=1.0):
        """exp(sign T) v by its finite Taylor series."""
        out, term, k = v.copy(), v.copy(), 0
        while True:
            k += 1
            term = sign * (T @ term) / k
            if not np.any(term):
                return out
            out += term
            if k > 64:
                raise RuntimeError("exp(T): series did not terminate")

    def phi_vector(self):
        e = np.zeros(self.sp.dim)
        e[self.i0] = 1.0
        return e


def _residual(cs: CCSpace, t):
    T = cs.t_matrix(t)
    phi = cs.phi_vector()
    w = cs.hop(cs.expm_apply(T, phi))
    energy = float(w[cs.i0])
    hbar = cs.expm_apply(T, w, -1.0)
    return cs.bra @ hbar, energy


def ccsd(problem, tup, tol: float = 1e-12, max_iter: int = 500):
    """(E_CCSD, t, CCSpace) of the tuple's CAS."""
    cs = CCSpace(problem, tup)
    nt = len(cs.ops)
    if nt == 0:
        return float(cs.hop(cs.phi_vector())[cs.i0]), np.zeros(0), cs
    d = cs.bra.indices                          # the determinant of each |mu> (one entry per row)
    if cs.H is not None:
        hdiag, h00 = cs.H[d, d], cs.H[cs.i0, cs.i0]
    else:
        unit = lambda i: np.eye(1, cs.sp.dim, i).ravel()  # noqa: E731
        hdiag = np.array([cs.hop(unit(i))[i] for i in d])
        h00 = cs.hop(cs.phi_vector())[cs.i0]
    shift = hdiag - h00
    if not np.all(shift > 0.0):
        raise ValueError("coupled-cluster base: an excited determinant lies below Phi on the diagonal")
    t = np.zeros(nt)
    hist_t, hist_r = [], []
    for _ in range(max_iter):
        r, e = _residual(cs, t)
        if np.abs(r).max() < tol:
            return e, t, cs
        tn = t - r / shift
        hist_t.append(tn)
        hist_r.append(tn - t)
        hist_t, hist_r = hist_t[-8:], hist_r[-8:]
        m = len(hist_t)
        B = -np.ones((m + 1, m + 1))
        B[m, m] = 0.0
        for i in range(m):
            for j in range(m):
                B[i, j] = hist_r[i] @ hist_r[j]
        rhs = np.zeros(m + 1)
        rhs[m] = -1.0
        try:
            c = np.linalg.solve(B, rhs)[:m]
            t = sum(ci * ti for ci, ti in zip(c, hist_t))
        except np.linalg.LinAlgError:
            t = tn
    raise RuntimeError("CCSD amplitude equations did not converge")


def fock_matrix(problem, occ_a, occ_b):
    """Spin-orbital Fock matrices (alpha, beta) of the determinant with the
    given occupied orbitals: f_pq = h_pq + sum_k occupied (pq|kk) - same spin
    (pk|kq)."""
    h, eri = problem.h, problem.eri
    J = sum(eri[:, :, k, k] for k in occ_a) + sum(eri[:, :, k, k] for k in occ_b)
    Ka = sum(eri[:, k, k, :] for k in occ_a) if occ_a else 0.0
    Kb = sum(eri[:, k, k, :] for k in occ_b) if occ_b else 0.0
    return h + J - Ka, h + J - Kb


def triples_correction(problem, tup, t, cs: CCSpace, canon_tol: float = 1e-10):
    """E_(T) from the CCSD amplitudes t."""
    pa, pb = cs.phi
    occ = lambda m: [p for p in range(problem.norb) if (m >> p) & 1]  # noqa: E731
    fa, fb = fock_matrix(problem, occ(pa), occ(pb))
    act = cs.sp.active
    for f in (fa, fb):
        sub = f[np.ix_(act, act)]
        if np.abs(sub - np.diag(np.diag(sub))).max() > canon_tol:
            raise ValueError("(T) needs canonical orbitals: the Fock operator of Phi is not diagonal")
    trip = cs.level == 3
    if not trip.any():
        return 0.0
    phi = cs.phi_vector()
    x = cs.hop(cs.t_matrix(t, ranks=(2,)) @ phi)
    hphi = cs.hop(phi)
    hphi[cs.level != 2] = 0.0
    y = cs.t_matrix(t, ranks=(1,)) @ hphi
    da, db = np.diag(fa), np.diag(fb)
    e0 = np.array([sum(da[p] for p in occ(int(a))) + sum(db[p] for p in occ(int(b)))
                   for a in cs.sp.alist for b in cs.sp.blist])
    D = e0[cs.i0] - e0
    return float(np.sum(x[trip] * (x[trip] + y[trip]) / D[trip]))


def base_energy(problem, tup, triples: bool = False) -> float:
    """CCSD (triples=False) or CCSD(T) energy of the tuple's CAS (total energy,
    constant and core included)."""
    e, t, cs = ccsd(problem, tup)
    if triples:
        e += triples_correction(problem, tup, t, cs)
    return e
