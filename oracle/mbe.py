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

Pi-pruning (Sec. 3: increments are computed only for tuples that hold both
components of a degenerate pair of pi orbitals, or neither; the counts of
Table 2, 6, 21, 56, 120, 216, 336 for 6 sigma orbitals and 6 pairs, pin it).
Reading for the candidates under screening: an order-k tuple is computed iff
it is pi-complete and either adds one unpaired orbital to a computed order-(k-1)
tuple T with |d_eps(T)| >= tau_{k-1}, or adds one whole pair to a computed
order-(k-2) tuple T with |d_eps(T)| >= tau_{k-2} (the empty tuple always
counts).  Without screening this gives every pi-complete tuple.  An order with
no candidates ends the expansion unless the order before it had tuples (a pair
added two orders back may still follow).

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


def pi_complete(S, pairs):
    s = set(S)
    return all((x in s) == (y in s) for x, y in pairs)


def pi_children(orders, dinc, X, pairs, a, k):
    """Order-k candidates under pi-pruning (reading in the module docstring);
    orders[j] is the computed order j."""
    paired = {x for pr in pairs for x in pr}
    out = set()
    if k - 1 >= 1:
        tau = screen_threshold(a, k - 1)
        for T in orders[k - 1].tuples:
            if abs(dinc[T]) >= tau:
                for x in X:
                    if x not in paired and x not in T:
                        out.add(tuple(sorted(T + (x,))))
    if k - 2 >= 0:
        tau2 = screen_threshold(a, k - 2)
        for T in orders[k - 2].tuples:
            if k - 2 == 0 or abs(dinc[T]) >= tau2:
                for x, y in pairs:
                    if x not in T and y not in T:
                        out.add(tuple(sorted(T + (x, y))))
    return sorted(out)


def candidates(problem, k, prev_order, dinc, orders=None):
    """Tuples to compute at order k (k >= 1)."""
    X = problem.expansion_space()
    pairs = [tuple(p) for p in getattr(problem, "pi_pairs", [])]
    if k == 1 or problem.a <= 0.0:
        allk = [(x,) for x in X] if k == 1 else list(itertools.combinations(X, k))
        return [S for S in allk if pi_complete(S, pairs)] if pairs else allk
    if pairs:
        return pi_children(orders, dinc, X, pairs, problem.a, k)
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
    pairs = getattr(problem, "pi_pairs", [])
    for k in range(1, kmax + 1):
        cand = candidates(problem, k, res.orders[-1], dinc, res.orders)
        if not cand:
            if pairs and res.orders[-1].tuples:
                res.orders.append(Order(k, [], [], [], 0.0))
                continue
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
