"""Brute-force second quantisation in the full Fock space (test helper).

Builds the Hamiltonian H = E_const + sum h_pq a+_{pu} a_{qu}
+ 1/2 sum (pq|rs) a+_{pu} a+_{rv} a_{sv} a_{qu} as a sparse matrix product of
Jordan-Wigner mode operators made from Kronecker products of 2x2 matrices.
Mode m = p for (p, alpha) and m = n + p for (p, beta); basis index
b = sum_m occ_m 2^m, so |b> = prod_{m in b, ascending} a+_m |vac>, which puts
every alpha creator left of every beta creator.  Nothing here uses
Slater-Condon rules, so it checks them independently.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def mode_annihilators(M):
    I2 = sp.identity(2, format="csr")
    Z = sp.csr_matrix(np.diag([1.0, -1.0]))
    lower = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))   # |1> -> |0>
    ops = []
    for m in range(M):
        # kron factors from the highest mode (most significant bit) down to mode 0
        A = sp.identity(1, format="csr")
        for j in range(M - 1, -1, -1):
            f = I2 if j > m else (lower if j == m else Z)
            A = sp.kron(A, f, format="csr")
        ops.append(A)
    return ops


def fock_hamiltonian(h, eri, e_const=0.0):
    n = h.shape[0]
    M = 2 * n
    a = mode_annihilators(M)
    ad = [x.T.tocsr() for x in a]
    dim = 2 ** M
    H = e_const * sp.identity(dim, format="csr")
    for u in range(2):
        for p in range(n):
            for q in range(n):
                if h[p, q] != 0.0:
                    H = H + h[p, q] * (ad[u * n + p] @ a[u * n + q])
    for u in range(2):
        for v in range(2):
            for p in range(n):
                for q in range(n):
                    for r in range(n):
                        for s in range(n):
                            g = eri[p, q, r, s]
                            if g == 0.0:
                                continue
                            H = H + 0.5 * g * (ad[u * n + p] @ ad[v * n + r] @ a[v * n + s] @ a[u * n + q])
    return H.tocsr()


def det_index(alpha_mask, beta_mask, n):
    return int(alpha_mask) | (int(beta_mask) << n)
