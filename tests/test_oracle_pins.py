"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, a brute-force Fock-space construction, library eigensolvers on
special cases, invariances, the paper's tuple counts and the MBE identity."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import fci, mbe, rdm
from tests.fockspace import det_index, fock_hamiltonian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _space(n, na, nb, core=(), active=None):
    active = list(range(n)) if active is None else list(active)
    return fci.CasSpace(active, list(core), na, nb,
                        fci.strings(active, na, core), fci.strings(active, nb, core))


def _prob(h, eri, na, nb, e_const=0.0, ref=None, nfrozen=0):
    n = h.shape[0]
    return synth.Problem("t", h, eri, na, nb, nfrozen, list(range(n)) if ref is None else ref,
                         e_const=e_const)


@pytest.mark.parametrize("na,nb", [(2, 2), (2, 1), (3, 1), (1, 0), (3, 3)])
def test_slater_condon_equals_fock_space(na, nb):
    """Every matrix element, sign included, equals the brute-force second-
    quantised operator product (Jordan-Wigner), for a random 4-orbital
    Hamiltonian with a constant."""
    n = 4
    h, eri = synth.random_hamiltonian(np.linspace(-1, 0.5, n), 0.2, 5, 0.3, seed=11)
    P = _prob(h, eri, na, nb, e_const=0.7)
    sp = _space(n, na, nb)
    H = fci.hamiltonian_matrix(P, sp)
    F = fock_hamiltonian(h, eri, 0.7).toarray()
    idx = [det_index(a, b, n) for a in sp.alist for b in sp.blist]
    np.testing.assert_allclose(H, F[np.ix_(idx, idx)], rtol=0, atol=1e-12)


def test_projected_cas_equals_fock_submatrix():
    """A CAS with one core and one empty orbital is the sub-block of the Fock
    space Hamiltonian on determinants with the core filled and the virtual empty."""
    n = 5
    h, eri = synth.random_hamiltonian(np.linspace(-1.2, 0.8, n), 0.1, 4, 0.25, seed=3)
    P = _prob(h, eri, 3, 2)
    sp = _space(n, 2, 1, core=[0], active=[1, 2, 3])
    H = fci.hamiltonian_matrix(P, sp)
    F = fock_hamiltonian(h, eri).toarray()
    idx = [det_index(a, b, n) for a in sp.alist for b in sp.blist]
    np.testing.assert_allclose(H, F[np.ix_(idx, idx)], rtol=0, atol=1e-12)
    x = np.random.default_rng(0).standard_normal(sp.dim)
    np.testing.assert_allclose(fci.matvec(P, sp, x), H @ x, rtol=0, atol=1e-12)


def test_two_electrons_two_orbitals_closed_form():
    """Minimal-basis two-electron problem with h_12 = (11|12) = (22|12) = 0:
    closed-shell singlet pair 1/2(E11+E22) -/+ sqrt(1/4(E22-E11)^2 + K^2),
    triplet h11+h22+J-K and open-shell singlet h11+h22+J+K."""
    h11, h22, J11, J22, J12, K12 = -1.3, -0.4, 0.7, 0.6, 0.45, 0.18
    h = np.diag([h11, h22])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0], eri[1, 1, 1, 1] = J11, J22
    eri[0, 0, 1, 1] = eri[1, 1, 0, 0] = J12
    for p, q, r, s in itertools.permutations([0, 1, 0, 1]):
        if (p, q, r, s) in {(0, 1, 0, 1), (1, 0, 1, 0), (0, 1, 1, 0), (1, 0, 0, 1)}:
            eri[p, q, r, s] = K12
    P = _prob(h, eri, 1, 1)
    w = np.linalg.eigvalsh(fci.hamiltonian_matrix(P, _space(2, 1, 1)))
    E11, E22 = 2 * h11 + J11, 2 * h22 + J22
    rt = math.sqrt(0.25 * (E22 - E11) ** 2 + K12 ** 2)
    ref = sorted([0.5 * (E11 + E22) - rt, 0.5 * (E11 + E22) + rt,
                  h11 + h22 + J12 - K12, h11 + h22 + J12 + K12])
    np.testing.assert_allclose(w, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("U,E0", [(2.0, -1.236067977500), (4.0, -0.828427124746), (8.0, -0.472135955000)])
def test_hubbard_dimer(U, E0):
    """Two-site Hubbard model, one electron of each spin: E0 = (U - sqrt(U^2+16t^2))/2."""
    h, eri = synth.hubbard_site(2, U, 1.0)
    P = _prob(h, eri, 1, 1)
    e = fci.lowest_eigenpair(P, _space(2, 1, 1))[0]
    assert abs(e - 0.5 * (U - math.sqrt(U * U + 16.0))) < 1e-13
    assert abs(e - E0) < 1e-11


def test_u0_chain_closed_form_and_zero_increments():
    """U = 0 chain in its hopping eigenbasis: E = 2 sum_{k<=N/2} eps_k, and every
    increment beyond order 0 vanishes (each CASCI is the same determinant)."""
    P = synth.config_hubbard(U=0.0, nsite=8)
    eps_k = -2.0 * np.cos(np.pi * np.arange(1, 9) / 9.0)
    e_exact = 2.0 * np.sort(eps_k)[:4].sum()
    assert abs(fci.fci_energy(P) - e_exact) < 1e-11
    res = mbe.run(P)
    assert abs(res.total - e_exact) < 1e-11
    for o in res.orders[1:]:
        assert max(abs(d) for d in o.dinc) < 1e-12


def test_u0_chain_ten_sites_value():
    """Ten-site U = 0 chain at half filling: 2 sum_{k=1..5} -2cos(pi k/11)."""
    eps_k = -2.0 * np.cos(np.pi * np.arange(1, 11) / 11.0)
    assert abs(2.0 * np.sort(eps_k)[:5].sum() - (-12.053348366665)) < 1e-11
    P = synth.config_hubbard(U=0.0, nsite=10)
    # the CASCI of the reference space alone already is the exact energy
    assert abs(fci.casci_energy(P, ()) - 2.0 * np.sort(eps_k)[:5].sum()) < 1e-11


def test_one_electron_is_eigh_of_h():
    n = 6
    h, eri = synth.random_hamiltonian(np.linspace(-1, 1, n), 0.2, 4, 0.3, seed=5)
    P = _prob(h, eri, 1, 0, e_const=0.25)
    e = fci.lowest_eigenpair(P, _space(n, 1, 0))[0]
    assert abs(e - (0.25 + np.linalg.eigvalsh(h)[0])) < 1e-13


def test_no_two_electron_integrals_whole_pipeline():
    """With (pq|rs) = 0 every CASCI energy is 2 sum_C h_cc plus the lowest
    active-electron eigenvalues of h restricted to A; checked for every tuple
    of a screened expansion with a frozen core."""
    n = 8
    h, _ = synth.random_hamiltonian(-1.0 + 0.3 * np.arange(n), 0.08, 1, 0.1, seed=2)
    eri = np.zeros((n, n, n, n))
    P = synth.Problem("eri0", h, eri, 3, 3, 1, [2, 3], a=5.0, max_order=4, e_const=0.3)
    res = mbe.run(P)
    for o in res.orders:
        for S, e in zip(o.tuples, o.eps):
            sp = fci.cas_space(P, S)
            w = np.linalg.eigvalsh(h[np.ix_(sp.active, sp.active)])
            ref = 0.3 + 2 * sum(h[c, c] for c in sp.core) + w[:sp.na].sum() + w[:sp.nb].sum()
            assert abs(e - ref) < 1e-12, S
    assert len(res.orders) >= 3


def _rotate(h, eri, Q):
    h2 = Q.T @ h @ Q
    e2 = np.einsum("pqrs,pa,qb,rc,sd->abcd", eri, Q, Q, Q, Q, optimize=True)
    return 0.5 * (h2 + h2.T), e2


def test_fci_rotation_invariance():
    n = 6
    h, eri = synth.random_hamiltonian(np.linspace(-1, 1, n), 0.1, 6, 0.2, seed=9)
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((n, n)))
    h2, e2 = _rotate(h, eri, Q)
    e_a = fci.lowest_eigenpair(_prob(h, eri, 3, 2), _space(n, 3, 2))[0]
    e_b = fci.lowest_eigenpair(_prob(h2, e2, 3, 2), _space(n, 3, 2))[0]
    assert abs(e_a - e_b) < 1e-11


def test_casci_invariant_under_active_and_core_rotations():
    """CASCI is unchanged by rotations inside A and inside C separately, and
    changes under a rotation mixing A with the virtual space."""
    P = synth.small_problem(8, 3, 3, [2, 3], nfrozen=1, nvec=6, seed=4)
    S = (1, 5)
    sp = fci.cas_space(P, S)
    e0 = fci.casci_energy(P, S)
    n = P.norb
    Q = np.eye(n)
    rng = np.random.default_rng(2)
    A = sp.active
    QA, _ = np.linalg.qr(rng.standard_normal((len(A), len(A))))
    Q[np.ix_(A, A)] = QA
    h2, e2 = _rotate(P.h, P.eri, Q)
    P2 = synth.Problem("rot", h2, e2, P.nalpha, P.nbeta, P.nfrozen, P.ref)
    assert abs(fci.casci_energy(P2, S) - e0) < 1e-11
    C = sp.core
    Q = np.eye(n)
    QC, _ = np.linalg.qr(rng.standard_normal((len(C), len(C))))
    Q[np.ix_(C, C)] = QC
    h3, e3 = _rotate(P.h, P.eri, Q)
    P3 = synth.Problem("rot", h3, e3, P.nalpha, P.nbeta, P.nfrozen, P.ref)
    assert abs(fci.casci_energy(P3, S) - e0) < 1e-11
    Q = np.eye(n)
    c, s = math.cos(0.3), math.sin(0.3)
    Q[np.ix_([5, 7], [5, 7])] = [[c, -s], [s, c]]
    h4, e4 = _rotate(P.h, P.eri, Q)
    P4 = synth.Problem("rot", h4, e4, P.nalpha, P.nbeta, P.nfrozen, P.ref)
    assert abs(fci.casci_energy(P4, S) - e0) > 1e-6


def test_hubbard_site_and_mo_basis_agree():
    Pm = synth.config_hubbard(U=4.0, nsite=6)
    hs, es = synth.hubbard_site(6, 4.0)
    e_site = fci.lowest_eigenpair(_prob(hs, es, 3, 3), _space(6, 3, 3))[0]
    assert abs(fci.fci_energy(Pm) - e_site) < 1e-11


def test_spin_flip_and_multiplets():
    n = 5
    h, eri = synth.random_hamiltonian(np.linspace(-1, 1, n), 0.1, 5, 0.25, seed=7)
    P = _prob(h, eri, 3, 1)
    w31 = np.linalg.eigvalsh(fci.hamiltonian_matrix(P, _space(n, 3, 1)))
    w13 = np.linalg.eigvalsh(fci.hamiltonian_matrix(P, _space(n, 1, 3)))
    w22 = np.linalg.eigvalsh(fci.hamiltonian_matrix(P, _space(n, 2, 2)))
    np.testing.assert_allclose(w31, w13, atol=1e-12)
    # every M_s = 1 level reappears in the M_s = 0 sector
    for x in w31:
        assert np.min(np.abs(w22 - x)) < 1e-10


def test_lanczos_equals_dense():
    P = synth.small_problem(8, 4, 3, [3, 4], nvec=6, seed=8)
    sp = fci.cas_space(P, (0, 1, 2, 5, 6, 7))
    assert sp.dim > 1000
    e_d = fci.lowest_eigenpair(P, sp, dense_max=10 ** 9)[0]
    e_l = fci.lowest_eigenpair(P, sp, dense_max=10)[0]
    assert abs(e_d - e_l) < 1e-11


# ---------------------------------------------------------------- MBE ------

def test_mbe_full_order_equals_fci_for_any_reference():
    """Eq. 3 without screening sums to the FCI energy whatever the reference
    space (the paper's cases (a) and (d) give the same result)."""
    P = synth.small_problem(7, 3, 3, [2, 3], nvec=6, seed=6)
    e_fci = fci.fci_energy(P)
    for ref in ([2, 3], [0, 1, 2], [0, 1, 2, 3, 4], [3]):
        Q = synth.Problem("r", P.h, P.eri, 3, 3, 0, ref)
        res = mbe.run(Q)
        assert abs(res.total - e_fci) < 1e-10, ref


def test_mbe_recursion_equals_moebius_form():
    P = synth.small_problem(7, 3, 3, [2, 3], nvec=6, seed=12)
    res = mbe.run(P, max_order=3)
    eps = {}
    for o in res.orders:
        eps.update(zip(o.tuples, o.eps))
    d = res.dinc_map()
    for S in eps:
        assert abs(d[S] - mbe.moebius_increment(S, eps)) < 1e-12


def test_paper_tuple_counts():
    """Counts printed in the paper (fixture cites the passages)."""
    with open(os.path.join(GOLDEN, "paper_counts.json")) as f:
        G = json.load(f)
    for case in G["fig2_cases"]:
        P = synth.Problem(case["name"], np.zeros((10, 10)), np.zeros((10,) * 4),
                          case["nalpha"], case["nbeta"], case["nfrozen"], case["ref"])
        X = P.expansion_space()
        counts, labels = {}, {}
        for k in range(1, len(X) + 1):
            cand = mbe.candidates(P, k, None, {}) if k == 1 else list(itertools.combinations(X, k))
            counts[str(k)] = len(cand)
            labels[k] = {tuple([fci.cas_space(P, S).na + fci.cas_space(P, S).nb,
                                len(fci.cas_space(P, S).active)]) for S in cand}
        for k, c in case["printed_counts"].items():
            assert counts[k] == c, (case["name"], k)
        assert max(int(k) for k in counts) == max(int(k) for k in case["printed_counts"])
        assert labels[1] == {tuple(case["order1_casci"])}, case["name"]
        if "order2_casci" in case:
            assert labels[2] == {tuple(case["order2_casci"])}, case["name"]
        assert labels[len(X)] == {tuple(case["final_casci"])}, case["name"]
    # Table 2, standard expansion: orders 1-4 are unscreened, C(18, k)
    t2 = G["table2_standard_orders_1_4"]
    X = list(range(18))
    assert [math.comb(len(X), k) for k in range(1, 5)] == t2["counts"]

    def energy(S):
        # every increment equals (2-1)^|S| = 1, far above every threshold
        return float(2 ** len(S))
    Pn = synth.Problem("t2", np.zeros((18, 18)), np.zeros((18,) * 4), 0, 0, 0, [], a=5.0)
    res = mbe.run(Pn, energy=energy, max_order=4)
    assert [len(o.tuples) for o in res.orders[1:]] == t2["counts"]


def test_screening_rule_on_handmade_table():
    """Child generation: a candidate exists iff one parent is significant;
    thresholds compare with >=; screened tuples drop out of Eq. 3."""
    Pn = synth.Problem("s", np.zeros((4, 4)), np.zeros((4,) * 4), 0, 0, 0, [], a=5.0)
    table = {(): 0.0, (0,): 1e-10, (1,): 0.5e-10, (2,): -0.99e-10, (3,): -3e-9}
    res1 = mbe.run(Pn, energy=lambda S: table[S], max_order=1)
    d = res1.dinc_map()
    assert d[(0,)] == 1e-10
    # order-1 threshold tau_1 = 1e-10: (0,) and (3,) are significant (>=), (1,), (2,) not
    ch = mbe.children(res1.orders[1].tuples, d, [0, 1, 2, 3], mbe.screen_threshold(5.0, 1))
    assert ch == [(0, 1), (0, 2), (0, 3), (1, 3), (2, 3)]
    assert mbe.screen_threshold(5.0, 3) == pytest.approx(2.5e-9)
    # a missing subtuple contributes nothing to Eq. 3
    dd = {(): 1.0, (0,): 0.25, (1,): 0.5}
    assert mbe.increment((0, 1), 2.0, dd) == 2.0 - (1.0 + 0.25 + 0.5)
    dd2 = {(): 1.0, (0,): 0.25}
    assert mbe.increment((0, 1), 2.0, dd2) == 2.0 - 1.25


def test_no_screening_counts_are_binomial():
    P = synth.config_plain()
    X = P.expansion_space()
    assert len(X) == 8
    dummy = {}
    for k in range(1, 9):
        c = mbe.candidates(P, k, None, dummy)
        assert len(c) == math.comb(8, k)
        assert c == sorted(c)


# ---------------------------------------------------------------- RDMs -----

def test_rdm_traces_and_energy():
    P = synth.small_problem(6, 3, 2, [2, 3], nfrozen=1, nvec=6, seed=3)
    for S in [(), (1,), (4, 5), (1, 4, 5)]:
        e, v, sp = fci.casci_energy(P, S, want_vector=True)
        g1, g2 = rdm.rdm12(P, sp, v)
        N = P.nalpha + P.nbeta
        assert abs(np.trace(g1) - N) < 1e-11
        assert abs(np.einsum("pprr->", g2) - N * (N - 1)) < 1e-10
        np.testing.assert_allclose(g1, g1.T, atol=1e-12)
        w = np.linalg.eigvalsh(g1)
        assert w.min() > -1e-12 and w.max() < 2 + 1e-12
        assert abs(rdm.energy_from_rdms(P, g1, g2) - e) < 1e-11
        for c in sp.core:
            assert abs(g1[c, c] - 2.0) < 1e-12


def test_adjoint_weights_full_order_are_unit_at_top():
    P = synth.small_problem(6, 2, 2, [1, 2], nvec=4, seed=5)
    res = mbe.run(P)
    w = rdm.adjoint_weights(res)
    X = tuple(P.expansion_space())
    for S, wS in w.items():
        assert wS == (1 if S == X else 0)


def _orbit_fd(P, res_fixed, which, idx, step=1e-5):
    """Central difference of the MBE energy along one symmetry orbit of h or
    (pq|rs), with the tuple set of `res_fixed` held fixed."""
    tuples = [list(o.tuples) for o in res_fixed.orders]

    def energy_at(sign):
        h = P.h.copy()
        eri = P.eri.copy()
        if which == "h":
            p, q = idx
            for a, b in {(p, q), (q, p)}:
                h[a, b] += sign * step
        else:
            p, q, r, s = idx
            orbit = {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                     (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}
            for o in orbit:
                eri[o] += sign * step
        Q = synth.Problem("fd", h, eri, P.nalpha, P.nbeta, P.nfrozen, P.ref, e_const=P.e_const)
        dinc = {}
        tot = 0.0
        for k, tl in enumerate(tuples):
            o = mbe.assemble(k, tl, [fci.casci_energy(Q, S) for S in tl], dinc)
            tot += o.order_sum
        return tot

    return (energy_at(+1) - energy_at(-1)) / (2 * step)


def test_mbe_gradient_matches_finite_differences():
    P = synth.small_problem(6, 3, 3, [2, 3], nvec=5, seed=21)
    res = mbe.run(P, max_order=2)
    gh, ge = rdm.mbe_gradient(P, res)
    rng = np.random.default_rng(0)
    for _ in range(4):
        p, q = sorted(rng.integers(0, 6, size=2))
        fd = _orbit_fd(P, res, "h", (p, q))
        an = gh[p, q] + (gh[q, p] if p != q else 0.0)
        assert abs(fd - an) < 1e-7, (p, q, fd, an)
    for _ in range(4):
        p, q, r, s = rng.integers(0, 6, size=4)
        orbit = {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                 (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}
        fd = _orbit_fd(P, res, "eri", (p, q, r, s))
        an = sum(ge[o] for o in orbit)
        assert abs(fd - an) < 1e-7, ((p, q, r, s), fd, an)


def test_full_order_gradient_is_fci_rdm():
    P = synth.small_problem(6, 2, 2, [1, 2], nvec=4, seed=5)
    res = mbe.run(P)
    gh, ge = rdm.mbe_gradient(P, res)
    e, v, sp = fci.casci_energy(P, tuple(P.expansion_space()), want_vector=True)
    g1, g2 = rdm.rdm12(P, sp, v)
    np.testing.assert_allclose(gh, g1, atol=1e-10)
    np.testing.assert_allclose(ge, 0.5 * g2, atol=1e-10)


def _fock_vector(sp, vec, n):
    """The CAS vector (index ia * len(blist) + ib, creators ordered over the
    full orbital space) as a Fock-space vector of tests.fockspace."""
    out = np.zeros(2 ** (2 * n))
    for ia, a in enumerate(sp.alist):
        for ib, b in enumerate(sp.blist):
            out[det_index(a, b, n)] = vec[ia * len(sp.blist) + ib]
    return out


@pytest.mark.parametrize("case", ["closed", "open", "core"])
def test_rdm_elements_equal_fock_space_operators(case):
    """Every element of the oracle's gamma and Gamma equals the Jordan-Wigner
    construction gamma_pq = <c|E_pq|c>, Gamma_pqrs = <c|E_pq E_rs|c> -
    delta_qr gamma_ps with E_pq = sum_spin a+_p a_q (no Slater-Condon rule, no
    symmetry assumed): closed shell, open shell, and a CAS with a doubly
    occupied core orbital and an empty virtual.  A p <-> q transposition of
    Gamma would fail this test (checked on the same vector)."""
    from tests.fockspace import mode_annihilators
    if case == "closed":
        n, na, nb, core, active = 4, 2, 2, [], [0, 1, 2, 3]
    elif case == "open":
        n, na, nb, core, active = 4, 3, 1, [], [0, 1, 2, 3]
    else:
        n, na, nb, core, active = 5, 2, 1, [1], [0, 2, 3]
    h, eri = synth.random_hamiltonian(np.linspace(-1.1, 0.9, n), 0.15, 4, 0.3, seed=17)
    P = _prob(h, eri, na + len(core), nb + len(core))
    sp = _space(n, na, nb, core=core, active=active)
    H = fci.hamiltonian_matrix(P, sp)
    w, v = np.linalg.eigh(H)
    vec = v[:, 0]
    g1, g2 = rdm.rdm12(P, sp, vec)
    a = mode_annihilators(2 * n)
    ad = [x.T.tocsr() for x in a]
    E = [[(ad[p] @ a[q] + ad[n + p] @ a[n + q]).tocsr() for q in range(n)] for p in range(n)]
    c = _fock_vector(sp, vec, n)
    Ec = [[E[p][q] @ c for q in range(n)] for p in range(n)]
    r1 = np.array([[c @ Ec[p][q] for q in range(n)] for p in range(n)])
    r2 = np.zeros((n, n, n, n))
    for p in range(n):
        for q in range(n):
            left = E[q][p] @ c          # <c|E_pq = (E_qp |c>)^T
            for r in range(n):
                for s in range(n):
                    r2[p, q, r, s] = left @ Ec[r][s] - (r1[p, s] if q == r else 0.0)
    np.testing.assert_allclose(g1, r1, rtol=0, atol=1e-12)
    np.testing.assert_allclose(g2, r2, rtol=0, atol=1e-12)
    # sensitivity: the transposed convention differs from the operator form
    assert np.abs(g2.transpose(1, 0, 2, 3) - r2).max() > 1e-3
    # and the energy of the CAS follows from these elements
    assert abs(rdm.energy_from_rdms(P, r1, r2) - w[0]) < 1e-11


def _n2_like(a):
    """N2-like spaces of Table 2: 28 orbitals, 2 frozen, CAS(10,8) reference,
    18 expansion orbitals of which 6 sigma and 6 degenerate pi pairs."""
    pairs = [(12, 13), (14, 15), (18, 19), (20, 21), (24, 25), (26, 27)]
    return synth.Problem("n2-like", np.zeros((28, 28)), np.zeros((1,)), 7, 7, 2, list(range(2, 10)), a=a,
                         max_order=6, pi_pairs=pairs)


@pytest.mark.parametrize("a", [0.0, 5.0])
def test_pi_pruned_counts_table2(a):
    """Pi-pruning counts of Table 2 (6, 21, 56, 120, 216, 336 for orders 1-6),
    by the oracle's planner without screening and with screening whose
    increments all exceed the thresholds (then the child rule must reach
    every pi-complete tuple); the unpruned order 1 is the standard 18."""
    with open(os.path.join(GOLDEN, "paper_counts.json")) as f:
        t2 = json.load(f)["table2_pi_pruned_orders_1_6"]
    P = _n2_like(a)
    assert len(P.expansion_space()) == t2["standard_order1"] == 18
    res = mbe.run(P, energy=lambda S: float(2 ** len(S)))
    assert [len(o.tuples) for o in res.orders[1:]] == t2["counts"]
    for o in res.orders[1:]:
        assert all(mbe.pi_complete(S, P.pi_pairs) for S in o.tuples)


def test_pi_pruning_screening_rule_on_handmade_table():
    """Children under pi-pruning: unpaired orbitals join significant
    order-(k-1) parents, whole pairs join significant order-(k-2) parents (the
    empty tuple always)."""
    P = synth.Problem("pi", np.zeros((5, 5)), np.zeros((1,)), 0, 0, 0, [], a=5.0, pi_pairs=[(1, 2)])
    X = P.expansion_space()
    assert X == [0, 1, 2, 3, 4]
    orders = [mbe.Order(0, [()], [0.0], [0.0], 0.0)]
    dinc = {(): 0.0}
    o1 = mbe.candidates(P, 1, orders[0], dinc, orders)
    assert o1 == [(0,), (3,), (4,)]
    dinc.update({(0,): 1.0, (3,): 1e-12, (4,): 1.0})
    orders.append(mbe.Order(1, o1, [0.0] * 3, [1.0, 1e-12, 1.0], 0.0))
    o2 = mbe.candidates(P, 2, orders[1], dinc, orders)
    # (3,) is negligible: (0,3), (3,4) come from (0,), (4,); the pair from {}
    assert o2 == [(0, 3), (0, 4), (1, 2), (3, 4)]
    dinc.update({(0, 3): 1e-12, (0, 4): 1e-12, (1, 2): 1.0, (3, 4): 1e-12})
    orders.append(mbe.Order(2, o2, [0.0] * 4, [1e-12, 1e-12, 1.0, 1e-12], 0.0))
    o3 = mbe.candidates(P, 3, orders[2], dinc, orders)
    # from (1,2) + unpaired; pairs onto significant order-1 tuples (0,), (4,)
    assert o3 == [(0, 1, 2), (1, 2, 3), (1, 2, 4)]


# --------------------------------------------------------------- total spin --
def _fock_spin_ops(n):
    """S_+, S_z and S^2 in the full Fock space from Jordan-Wigner mode
    operators (mode p: p alpha, mode n + p: p beta)."""
    from tests.fockspace import mode_annihilators
    a = mode_annihilators(2 * n)
    ad = [x.T.tocsr() for x in a]
    Sp = sum(ad[p] @ a[n + p] for p in range(n))
    Sz = 0.5 * sum(ad[p] @ a[p] - ad[n + p] @ a[n + p] for p in range(n))
    S2 = Sp.T @ Sp + Sz @ Sz + Sz
    return Sp.tocsr(), S2.tocsr()


@pytest.mark.parametrize("na,nb,core", [(2, 2, ()), (3, 1, ()), (2, 1, (0,)), (3, 2, (0,))])
def test_s2_matches_fock_space(na, nb, core):
    """<S^2> and S_- S_+ c of the oracle's spin module equal the brute-force
    Jordan-Wigner S^2 on random CAS vectors (closed and open shells, with a
    doubly occupied core orbital)."""
    from oracle import spin
    n = 5
    act = [p for p in range(n) if p not in core]
    sp = _space(n, na, nb, core=core, active=act)
    _, S2 = _fock_spin_ops(n)
    idx = [det_index(a, b, n) for a in sp.alist for b in sp.blist]
    rng = np.random.default_rng(3)
    for _ in range(3):
        c = rng.standard_normal(sp.dim)
        full = np.zeros(2 ** (2 * n))
        full[idx] = c
        ref = float(full @ (S2 @ full)) / float(c @ c)
        assert abs(spin.s2_expectation(sp, c) - ref) < 1e-11
        m = spin.sz(sp)
        y = spin.s_minus_s_plus(sp, c)
        yref = (S2 @ full)[idx] - m * (m + 1.0) * c
        np.testing.assert_allclose(y, yref, rtol=0, atol=1e-11)


def test_spin_targeted_closed_form_and_multiplets():
    """Two electrons in two orbitals: the lowest singlet is the lower of the
    closed-shell pair energy 1/2(E11+E22) - sqrt(1/4(E22-E11)^2 + K^2) and the
    open-shell singlet h11+h22+J+K, even when the triplet lies below both; the
    triplet's energy is h11+h22+J-K, found as S = 1
    in the M_s = 0 sector and as the only state of the M_s = 1 sector; every
    eigenvector of H has <S^2> = S(S+1)."""
    from oracle import spin
    h11, h22, J11, J22, J12, K12 = -1.3, -1.25, 0.9, 0.85, 0.45, 0.18
    h = np.diag([h11, h22])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0], eri[1, 1, 1, 1] = J11, J22
    eri[0, 0, 1, 1] = eri[1, 1, 0, 0] = J12
    for p, q, r, s in [(0, 1, 0, 1), (1, 0, 1, 0), (0, 1, 1, 0), (1, 0, 0, 1)]:
        eri[p, q, r, s] = K12
    P = _prob(h, eri, 1, 1)
    sp0 = _space(2, 1, 1)
    E11, E22 = 2 * h11 + J11, 2 * h22 + J22
    sing = min(0.5 * (E11 + E22) - math.sqrt(0.25 * (E22 - E11) ** 2 + K12 ** 2), h11 + h22 + J12 + K12)
    trip = h11 + h22 + J12 - K12
    assert trip < sing   # the case the targeting is for
    assert abs(fci.lowest_eigenpair(P, sp0)[0] - trip) < 1e-13
    assert abs(spin.lowest_with_spin(P, sp0)[0] - sing) < 1e-13
    assert abs(spin.lowest_with_spin(P, sp0, S=1)[0] - trip) < 1e-13
    P1 = _prob(h, eri, 2, 0)
    assert abs(spin.lowest_with_spin(P1, _space(2, 2, 0))[0] - trip) < 1e-13
    w, v = np.linalg.eigh(fci.hamiltonian_matrix(P, sp0))
    for i in range(len(w)):
        s2 = spin.s2_expectation(sp0, v[:, i])
        assert min(abs(s2 - S * (S + 1)) for S in (0, 1)) < 1e-10


def test_spin_multiplets_agree_across_sectors():
    """The lowest triplet of a 6-orbital, 4-electron CAS found in the M_s = 0
    sector (S = 1 targeted) equals the lowest state of the M_s = 1 sector
    with S = 1 (the multiplet's components are degenerate); likewise S = 0 in
    the M_s = 0 sector lies at or above the lowest M_s = 0 eigenvalue, and
    every eigenvector's <S^2> is S(S+1) for an integer S."""
    from oracle import spin
    P0 = synth.small_problem(6, 2, 2, list(range(6)), nvec=6, seed=7, vec_std=0.3)
    P1 = synth.Problem("t1", P0.h, P0.eri, 3, 1, 0, list(range(6)))
    sp0, sp1 = fci.cas_space(P0, ()), fci.cas_space(P1, ())
    t0 = spin.lowest_with_spin(P0, sp0, S=1)[0]
    t1 = spin.lowest_with_spin(P1, sp1)[0]
    assert abs(t0 - t1) < 1e-10
    s0 = spin.lowest_with_spin(P0, sp0)[0]
    assert s0 >= fci.lowest_eigenpair(P0, sp0)[0] - 1e-12
    w, v = np.linalg.eigh(fci.hamiltonian_matrix(P0, sp0))
    for i in range(len(w)):
        s2 = spin.s2_expectation(sp0, v[:, i])
        S = 0.5 * (math.sqrt(1.0 + 4.0 * s2) - 1.0)
        assert abs(S - round(S)) < 1e-8
