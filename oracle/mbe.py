"""ORACLE (test infrastructure): the many-body expansion of Eq. 1-3.

Eq. 3 of the paper: with every tuple a superset of the reference space [Pi],
the increment of a tuple S of expansion orbitals is its CASCI energy minus the
reference-space energy and minus the increments of all its proper subtuples,

    d_eps(S) = eps(S) - sum_{T proper subset of S} d_eps(T),   d_eps({}) = eps([Pi]),

and the MBE energy is the sum of all increments, order by order (Eq. 1,
E = E^(0) + E^(1) + ...).  Without screening and at full order the sum equals
the CASCI energy of all expansion orbitals (the FCI energy); every tuple
energy here is a total energy, so frozen-core constants cancel order by order.

Screening (parity unpinned -- the paper only names a threshold a, with a = 5.0
"aggressive" and a = 2.5 tighter; the protocol itself is defined in Part I,
which is not available).  Reading used on both sides:
  * tau_k = 1e-10 * a**(k-1) for increments of order k;
  * an order-(k+1) candidate S is generated iff at least one of its k-subtuples
    T was computed at order k and |d_eps(T)| >= tau_k (subtuples never
    computed count as negligible);
  * order 1 is never screened; a <= 0 disables screening;
  * screened or never-generated tuples contribute zero (they are left out of
    the sums of Eq. 3, as the paper says screened contributions are not
    accounted for).

Summation order (fixed so that two implementations agree bitwise on the same
epsilons): subtuples T in (|T|, lexicographic) order, accumulated from 0.0,
then d_eps(S) = eps(S) - acc.  Order sums accumulate in tuple-list order,
tuple lists are lexicographic (itertools.combinations order).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

from . import fci


def screen_threshold(a: float, k: int) -> float:
    """tau_k for increments of order k (reading; parity unpinned)."""
    return 1.0e-10 * a ** (k - 1)


@dataclass
class Order:
    k: int
    tuples: list
    eps: list
    dinc: list
    order_sum: float


@dataclass
class MBEResult:
    orders: list = field(default_factory=list)

    @property
    def total(self) -> float:
        s = 0.0
        for o in self.orders:
            s += o.order_sum
        return s

    def all_tuples(self):
        for o in self.orders:
            yield from o.tuples

    def dinc_map(self):
        d = {}
        for o in self.orders:
            d.update(zip(o.tuples, o.dinc))
        return d


def children(parents, dinc, X, tau):
    """Order-(k+1) candidates from the order-k tuples `parents`: every
    T u {x}, x in X \\ T, for each T with |d_eps(T)| >= tau; sorted, unique."""
    out = set()
    for T in parents:
        if abs(dinc[T]) >= tau:
            for x in X:
                if x not in T:
                    out.add(tuple(sorted(T + (x,))))
    return sorted(out)


def candidates(problem, k, prev_order, dinc):
    """Tuples to compute at order k (k >= 1)."""
    X = problem.expansion_space()
    if k == 1:
        return [(x,) for x in X]
    if problem.a <= 0.0:
        return list(itertools.combinations(X, k))
    return children(prev_order.tuples, dinc, X, screen_threshold(problem.a, k - 1))


def increment(S, eps_S, dinc):
    """Eq. 3 for one tuple, subtuples in (|T|, lexicographic) order."""
    acc = 0.0
    for m in range(len(S)):
        for T in itertools.combinations(S, m):
            v = dinc.get(T)
            if v is not None:
                acc += v
    return eps_S - acc


def assemble(k, tuples, eps, dinc):
    """Increments and the order sum of one order given its tuple energies;
    updates `dinc` in place."""
    out = []
    for S, e in zip(tuples, eps):
        d = increment(S, e, dinc)
        out.append(d)
    for S, d in zip(tuples, out):
        dinc[S] = d
    s = 0.0
    for d in out:
        s += d
    return Order(k, list(tuples), list(eps), out, s)


def run(problem, energy=None, max_order=None) -> MBEResult:
    """The whole expansion: order 0 ([Pi] alone), then orders 1.. until the
    maximum order, |X|, or no candidates.  `energy(tuple) -> eps` defaults to
    the oracle's CASCI energy; any table of energies may be fed instead (the
    assembler and the screening do not depend on how eps was obtained)."""
    if energy is None:
        def energy(S):
            return fci.casci_energy(problem, S)
    X = problem.expansion_space()
    kmax = max_order if max_order is not None else problem.max_order
    if kmax is None or kmax <= 0:
        kmax = len(X)
    kmax = min(kmax, len(X))
    dinc = {}
    res = MBEResult()
    e0 = energy(())
    res.orders.append(assemble(0, [()], [e0], dinc))
    for k in range(1, kmax + 1):
        cand = candidates(problem, k, res.orders[-1], dinc)
        if not cand:
            break
        eps = [energy(S) for S in cand]
        res.orders.append(assemble(k, cand, eps, dinc))
    return res


def moebius_increment(S, eps):
    """Closed form of Eq. 3 without screening: sum_{T subset S} (-1)^{|S|-|T|} eps(T)."""
    acc = 0.0
    for m in range(len(S) + 1):
        for T in itertools.combinations(S, m):
            acc += (-1) ** (len(S) - m) * eps[T]
    return acc
