"""Seeded synthetic Hamiltonians for the MBE-FCI hot path.

This module only *draws inputs*: a one-electron matrix h (n x n, symmetric),
two-electron integrals (pq|rs) in chemists' notation (n^4, 8-fold symmetric),
electron counts, the frozen-core count, the reference space [Pi] and the MBE
options.  It holds none of the method's arithmetic and serves both the CPU
oracle and the HIP path.

Conventions (the paper works on molecules whose integrals are not available, so
these stand in for them; the workload shapes follow the paper's systems):

* "N(0, s)": s is the standard deviation.  Random numbers come from
  ``numpy.random.default_rng(seed)`` (PCG64) in a fixed order: the strictly
  upper-triangular off-diagonal elements of h (row-major), then, for each
  Cholesky-like vector L = 0..N_L-1, the upper triangle including the diagonal
  of a symmetric B^L (row-major), mirrored.
* (pq|rs) = sum_L B^L_pq B^L_rs, which is 8-fold symmetric and positive
  semidefinite as a (pq),(rs) matrix.
* Orbital indices are 0-based; occupied orbitals are the lowest indices
  (aufbau by index); a reference space "HOMO/LUMO" is chosen by index.
* E_const = 0 everywhere.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "random_hamiltonian", "config_plain", "config_sweep",
    "config_hubbard", "config_large", "small_problem", "hubbard_site", "config_weak",
]


@dataclass
class Problem:
    """One MBE-FCI problem: integrals, electrons, spaces and options."""
    name: str
    h: np.ndarray            # (n, n) float64, symmetric
    eri: np.ndarray          # (n, n, n, n) float64, (pq|rs) chemists' notation
    nalpha: int              # total alpha electrons (frozen core included)
    nbeta: int               # total beta electrons (frozen core included)
    nfrozen: int             # orbitals 0..nfrozen-1 are frozen doubly occupied
    ref: list                # reference-space orbitals [Pi] (sorted)
    a: float = 0.0           # screening parameter; <= 0 disables screening
    max_order: int = 0       # <= 0 means full order |X|
    e_const: float = 0.0
    meta: dict = field(default_factory=dict)
    # degenerate orbital pairs (x, y) of the expansion space whose components
    # enter a tuple only together (pi-pruning); empty: no pruning
    pi_pairs: list = field(default_factory=list)

    @property
    def norb(self) -> int:
        return int(self.h.shape[0])

    def expansion_space(self) -> list:
        """Orbitals that are neither frozen nor in the reference space."""
        ref = set(self.ref)
        return [p for p in range(self.nfrozen, self.norb) if p not in ref]


def _sym_normal(rng, n, std):
    """Symmetric n x n matrix: upper triangle incl. diagonal, row-major, mirrored."""
    b = np.zeros((n, n))
    iu = np.triu_indices(n)
    b[iu] = rng.normal(0.0, std, size=len(iu[0]))
    b = b + b.T - np.diag(np.diag(b))
    return b


def random_hamiltonian(diag, offdiag_std, nvec, vec_std, seed):
    """h = diag + symmetric N(0, offdiag_std); (pq|rs) = sum_L B^L_pq B^L_rs."""
    diag = np.asarray(diag, dtype=np.float64)
    n = diag.size
    rng = np.random.default_rng(seed)
    h = np.diag(diag).astype(np.float64)
    iu = np.triu_indices(n, k=1)
    off = rng.normal(0.0, offdiag_std, size=len(iu[0]))
    h[iu] = off
    h[(iu[1], iu[0])] = off
    B = np.empty((nvec, n, n))
    for L in range(nvec):
        B[L] = _sym_normal(rng, n, vec_std)
    pi, qi = _pair_indices(n)
    Bp = B[:, pi, qi]                        # (nvec, npair), pairs p >= q
    Ep = Bp.T @ Bp
    Ep = 0.5 * (Ep + Ep.T)                   # bitwise (PQ) <-> (QP) symmetric
    return h, unpack_pairs(Ep, n)


def _pair_indices(n):
    """Pairs (p, q), p >= q, in the order P = p(p+1)/2 + q."""
    pi, qi = [], []
    for p in range(n):
        for q in range(p + 1):
            pi.append(p)
            qi.append(q)
    return np.array(pi), np.array(qi)


def unpack_pairs(Ep, n):
    """Expand a symmetric pair matrix E[P, Q] (P = p(p+1)/2+q, p >= q) into the
    full n^4 array with exact 8-fold permutational symmetry."""
    idx = np.empty((n, n), dtype=np.int64)
    for p in range(n):
        for q in range(p + 1):
            idx[p, q] = idx[q, p] = p * (p + 1) // 2 + q
    eri = Ep[idx[:, :, None, None], idx[None, None, :, :]]
    return np.ascontiguousarray(eri)


def config_plain(seed: int = 0) -> Problem:
    """Plain MBE-FCI: 10 orbitals, 4a+4b, h_pp = -1 + 0.3p, off-diag N(0,0.05),
    20 vectors N(0,0.1); reference CAS(2e,2o) HOMO/LUMO = {3,4}; full order, no
    screening.  Full-order sum must equal full FCI (dim 44100)."""
    n = 10
    h, eri = random_hamiltonian(-1.0 + 0.3 * np.arange(n), 0.05, 20, 0.1, seed)
    return Problem("plain-n10-4a4b", h, eri, 4, 4, 0, [3, 4], a=0.0, max_order=0,
                   meta={"seed": seed})


SWEEP_VEC_STD = math.sqrt(0.2 / 60.0)


def config_sweep(seed: int = 0, a: float = 5.0, max_order: int = 5,
                 vec_std: float = SWEEP_VEC_STD) -> Problem:
    """Batched order sweep: 24 orbitals, orbital 0 frozen, 5a+5b correlated
    electrons (6a+6b in total), water-like orbital energies over [-1.3, 2.5]:
    occupied 0..5 linspace(-1.3,-0.5), virtual 6..23 linspace(0.2,2.5);
    off-diag N(0,0.05); 60 vectors N(0, sqrt(0.2/60)), i.e. the same
    per-integral scale sum_L std^2 = 0.2 as the plain configuration (20 vectors
    of std 0.1).  Reference CAS(6e,6o) = {3..8}; expansion over the 17 other
    non-frozen orbitals; orders 1..5, a = 5.0."""
    n = 24
    diag = np.concatenate([np.linspace(-1.3, -0.5, 6), np.linspace(0.2, 2.5, 18)])
    h, eri = random_hamiltonian(diag, 0.05, 60, vec_std, seed)
    return Problem("sweep-n24-cas66", h, eri, 6, 6, 1, [3, 4, 5, 6, 7, 8], a=a,
                   max_order=max_order, meta={"seed": seed})


def hubbard_site(nsite: int, U: float, t: float = 1.0):
    """Open-chain Hubbard model in the site basis: h_ij = -t for |i-j| = 1,
    (ii|ii) = U."""
    h = np.zeros((nsite, nsite))
    for i in range(nsite - 1):
        h[i, i + 1] = h[i + 1, i] = -t
    eri = np.zeros((nsite,) * 4)
    for i in range(nsite):
        eri[i, i, i, i] = U
    return h, eri


def hubbard_mo_basis(nsite: int, t: float = 1.0):
    """U = 0 hopping eigenvectors of the open chain:
    phi_k(j) = sqrt(2/(L+1)) sin(pi j k/(L+1)), j,k = 1..L, ordered by
    eps_k = -2t cos(pi k/(L+1)) ascending (k = 1 lowest).  Columns are MOs."""
    L = nsite
    j = np.arange(1, L + 1)[:, None]
    k = np.arange(1, L + 1)[None, :]
    return math.sqrt(2.0 / (L + 1)) * np.sin(np.pi * j * k / (L + 1))


def config_hubbard(U: float = 4.0, nsite: int = 10, a: float = 0.0, t: float = 1.0) -> Problem:
    """Strong correlation: open 1D Hubbard chain at half filling, rotated to the
    U = 0 hopping-eigenvector MO basis; reference CAS(2e,2o) = HOMO/LUMO."""
    hs, eris = hubbard_site(nsite, U, t)
    C = hubbard_mo_basis(nsite, t)
    h = C.T @ hs @ C
    h = 0.5 * (h + h.T)
    pi, qi = _pair_indices(nsite)
    Bp = C[:, pi] * C[:, qi]                 # (site, npair): phi_pj phi_qj
    Ep = U * (Bp.T @ Bp)
    Ep = 0.5 * (Ep + Ep.T)
    eri = unpack_pairs(Ep, nsite)
    ne = nsite // 2
    return Problem(f"hubbard-{nsite}-U{U:g}", h, np.ascontiguousarray(eri), ne, ne, 0,
                   [ne - 1, ne], a=a, max_order=0, meta={"U": U, "t": t, "nsite": nsite})


def hubbard_irreps(nsite: int):
    """Irrep labels of the hopping eigenvectors of the open chain under the
    reflection j -> L + 1 - j: the k-th one (k = 1..L) has parity
    (-1)^(k + 1), label (k - 1) % 2 (0 even, 1 odd)."""
    return [c % 2 for c in range(nsite)]


def symmetric_problem(n: int, nalpha: int, nbeta: int, ref, labels, nvec: int = 8, seed: int = 0,
                      vec_std: float = 0.1, offdiag_std: float = 0.05, nfrozen: int = 0, a: float = 0.0) -> Problem:
    """Seeded problem whose Hamiltonian respects Abelian irrep labels (0..7,
    the product of two irreps is the XOR of their labels): h_pq = 0 unless
    labels p and q agree, and (pq|rs) = sum_L B^L_pq B^L_rs with B^L_pq = 0
    unless labels[p] ^ labels[q] equals the irrep L mod (max label + 1) of
    vector L; orbital energies -1.0 + 0.3 p on the diagonal."""
    rng = np.random.default_rng(seed)
    lab = np.asarray(labels)
    nirr = int(lab.max()) + 1
    same = lab[:, None] == lab[None, :]
    h = np.diag(-1.0 + 0.3 * np.arange(n))
    off = rng.normal(0.0, offdiag_std, size=(n, n))
    off = np.triu(off, 1)
    off = (off + off.T) * same
    h = h + off
    eri = np.zeros((n, n, n, n))
    for L in range(nvec):
        B = _sym_normal(rng, n, vec_std) * ((lab[:, None] ^ lab[None, :]) == (L % nirr))
        eri += np.einsum("pq,rs->pqrs", B, B)
    eri = 0.5 * (eri + eri.transpose(2, 3, 0, 1))
    return Problem(f"sym-n{n}-{nalpha}a{nbeta}b-s{seed}", h, eri, nalpha, nbeta, nfrozen, sorted(ref), a=a,
                   meta={"seed": seed, "irreps": [int(x) for x in lab]})


def config_large(seed: int = 0, a: float = 5.0, max_order: int = 4) -> Problem:
    """Large batched run: 60 orbitals, 6a+6b, orbital energies linspace(-1.5,4.0),
    off-diag N(0,0.05), 150 vectors N(0,0.05); reference CAS(8e,8o) = {2..9};
    orders 1..4 with a = 5.0."""
    n = 60
    h, eri = random_hamiltonian(np.linspace(-1.5, 4.0, n), 0.05, 150, 0.05, seed)
    return Problem("large-n60-cas88", h, eri, 6, 6, 0, list(range(2, 10)), a=a,
                   max_order=max_order, meta={"seed": seed})


def small_problem(n: int, nalpha: int, nbeta: int, ref, nfrozen: int = 0, nvec: int = 8,
                  seed: int = 0, a: float = 0.0, max_order: int = 0,
                  vec_std: float = 0.1, offdiag_std: float = 0.05, e_const: float = 0.0) -> Problem:
    """Small seeded problem with the same recipe as the plain configuration."""
    h, eri = random_hamiltonian(-1.0 + 0.3 * np.arange(n), offdiag_std, nvec, vec_std, seed)
    return Problem(f"small-n{n}-{nalpha}a{nbeta}b-s{seed}", h, eri, nalpha, nbeta, nfrozen,
                   sorted(ref), a=a, max_order=max_order, e_const=e_const, meta={"seed": seed})


def config_weak(seed: int = 1) -> Problem:
    """Weakly coupled 9-orbital problem (3a+3b, [Pi] = {2, 3}, off-diagonal h
    N(0, 0.005), 6 vectors N(0, 0.01)) on which the screening of a = 5.0 removes
    tuples from order 4 on; orders 1..5."""
    return small_problem(9, 3, 3, [2, 3], nvec=6, seed=seed, a=5.0, vec_std=0.01, offdiag_std=0.005,
                         max_order=5)
