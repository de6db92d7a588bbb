"""Spatial-symmetry targeting (options.sym_shift / irrep with orbital irrep
labels) against the oracle (oracle/sym.py: the lowest eigenvalue on the
determinants of the target irrep).  lambda = 2 E_h exceeds the distance of
every target irrep's lowest state to the lowest state of the CAS in these
problems (at most 1.2 E_h), so the shifted lowest state is the target's.
Tolerance 1e-10 as in the other parity tests."""
import itertools

import numpy as np
import pytest

import synth
from oracle import fci, mbe, sym

torch = pytest.importorskip("torch")
import paper_1905_02786_amd as M  # noqa: E402

pytestmark = pytest.mark.gpu
LAM = 2.0


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return M.workspace(2 << 30)


LAB4 = [0, 1, 2, 3, 0, 1, 2, 3]
PROBLEMS = {
    "hubbard8": (lambda: synth.config_hubbard(4.0, nsite=8), synth.hubbard_irreps(8), (0, 1)),
    "sym4": (lambda: synth.symmetric_problem(8, 3, 3, [2, 3], LAB4, seed=1), LAB4, (0, 1, 2, 3)),
}


def _ctx(P, lab, g):
    ctx = M.Context.from_problem(P, device=0, sym_shift=LAM, irrep=g)
    ctx.set_orbital_irreps(lab)
    return ctx


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_irrep_energies_match_oracle(ws, name):
    make, lab, targets = PROBLEMS[name]
    P = make()
    X = P.expansion_space()
    worst = 0.0
    for g in targets:
        ctx = _ctx(P, lab, g)
        for k in (0, 1, 2):
            tl = list(itertools.combinations(X, k)) if k else [()]
            ok = []
            for S in tl:
                try:
                    ok.append((S, sym.casci_energy_irrep(P, S, lab, g)))
                except ValueError:
                    pass
            if len(ok) < len(tl):   # a tuple without the irrep makes the whole call an error
                with pytest.raises(M.MBEFCIError, match="target irrep"):
                    ctx.solve_tuples(k, tl, ws)
            if not ok:
                continue
            e, st = ctx.solve_tuples(k, [S for S, _ in ok], ws)
            assert (st == 0).all()
            worst = max(worst, float(np.abs(e - np.array([r for _, r in ok])).max()))
    print(f"{name}: max |dE| {worst:.1e}", flush=True)
    assert worst <= 1e-10


@pytest.mark.parametrize("g", [0, 1])
def test_irrep_expansion_matches_oracle(ws, g):
    """Full-order MBE of the 8-site chain for each reflection irrep: every
    increment against the oracle's, the total equal to the irrep's FCI."""
    P = synth.config_hubbard(4.0, nsite=8)
    lab = synth.hubbard_irreps(8)
    res = _ctx(P, lab, g).run(ws)
    ref = mbe.run(P, energy=lambda S: sym.casci_energy_irrep(P, S, lab, g))
    for o, ro in zip(res.orders, ref.orders):
        assert [tuple(int(x) for x in t) for t in o.tuples] == [tuple(t) for t in ro.tuples] or o.k == 0
        assert np.abs(o.eps - np.asarray(ro.eps)).max() <= 1e-10
        assert np.abs(o.dinc - np.asarray(ro.dinc)).max() <= 1e-9
    e_fci = sym.casci_energy_irrep(P, tuple(P.expansion_space()), lab, g)
    assert abs(res.total - e_fci) <= 1e-9
    if g == 0:   # the chain's ground state is even: the plain expansion agrees
        assert abs(res.total - fci.fci_energy(P)) <= 1e-9


def test_symmetry_errors(ws):
    P = synth.config_hubbard(4.0, nsite=8)
    ctx = M.Context.from_problem(P, device=0, sym_shift=LAM, irrep=1)
    with pytest.raises(M.MBEFCIError, match="labels"):
        ctx.solve_tuples(0, [()], ws)             # labels not set
    Q = synth.small_problem(8, 4, 4, [3, 4], nvec=4, seed=3)
    ctx = _ctx(Q, synth.hubbard_irreps(8), 1)
    with pytest.raises(M.MBEFCIError, match="respect"):
        ctx.solve_tuples(0, [()], ws)             # a Hamiltonian without the symmetry


def _irrep_vector(P, S, lab, g):
    """The oracle's lowest irrep-g eigenvector, embedded in the CAS."""
    sp = fci.cas_space(P, S)
    idx = sym.irrep_indices(P, sp, lab, g)
    H = fci.hamiltonian_matrix(P, sp)
    w, V = np.linalg.eigh(H[np.ix_(idx, idx)])
    v = np.zeros(sp.dim)
    v[idx] = V[:, 0]
    return w[0], v, sp


def test_irrep_density_matrices_and_gradient(ws):
    """The density matrices of a symmetry-targeted tuple state, and the
    full-order gradient of the odd-irrep expansion, against the oracle's
    density matrices of the irrep eigenvector (the shift does not depend on
    the integrals, so dE/dh = gamma and dE/d(pq|rs) = Gamma / 2 of that
    state)."""
    from oracle import rdm as ordm
    P = synth.config_hubbard(4.0, nsite=8)
    lab = synth.hubbard_irreps(8)
    ctx = M.Context.from_problem(P, device=0, sym_shift=LAM, irrep=1, r_tol=1e-10, e_tol=1e-13)
    ctx.set_orbital_irreps(lab)
    S = (1, 6)
    e, g1, g2 = ctx.tuple_rdm(len(S), S, ws)
    e_ref, v, sp = _irrep_vector(P, S, lab, 1)
    r1, r2 = ordm.rdm12(P, sp, v)
    assert abs(e - e_ref) <= 1e-10
    assert np.abs(g1 - r1).max() <= 1e-7 and np.abs(g2 - r2).max() <= 1e-7
    res, handle = ctx.run(ws, keep=True)
    gh, ge = ctx.backward(handle, ws)
    e_ref, v, sp = _irrep_vector(P, tuple(P.expansion_space()), lab, 1)
    r1, r2 = ordm.rdm12(P, sp, v)
    assert abs(res.total - e_ref) <= 1e-9
    assert np.abs(gh - r1).max() <= 1e-7
    assert np.abs(ge - 0.5 * r2).max() <= 1e-7


def test_spin_and_symmetry_together(ws):
    """Both shifts: the lowest singlet of the odd irrep (the lowest odd state
    of the chain's tuples is often a triplet component) against the oracle's
    lowest eigenvector of the irrep block with <S^2> = 0."""
    from oracle import spin
    P = synth.config_hubbard(4.0, nsite=8)
    lab = synth.hubbard_irreps(8)
    # the odd singlet lies up to 1.49 E_h above the lowest odd state here, so
    # lambda_sym = 3 keeps the shifted even states clear of it
    ctx = M.Context.from_problem(P, device=0, sym_shift=3.0, irrep=1, spin_shift=1.0)
    ctx.set_orbital_irreps(lab)
    X = P.expansion_space()
    worst, differs = 0.0, 0
    for k in (0, 1, 2):
        tl = list(itertools.combinations(X, k)) if k else [()]
        ref = []
        for S in tl:
            sp = fci.cas_space(P, S)
            idx = sym.irrep_indices(P, sp, lab, 1)
            H = fci.hamiltonian_matrix(P, sp)
            w, V = np.linalg.eigh(H[np.ix_(idx, idx)])
            for c in range(len(w)):
                v = np.zeros(sp.dim)
                v[idx] = V[:, c]
                if abs(spin.s2_expectation(sp, v)) < 1e-8:
                    ref.append(w[c])
                    differs += c > 0
                    break
        e, st = ctx.solve_tuples(k, tl, ws)
        assert (st == 0).all()
        worst = max(worst, float(np.abs(e - np.array(ref)).max()))
    print(f"max |dE| {worst:.1e}; tuples whose odd singlet is not the odd ground state: {differs}")
    assert differs > 0
    assert worst <= 1e-10
